/*
 * sfem.h -- C ABI of the MI355X (gfx950) library for matrix-free, sum-factorized
 * high-order hexahedral Q_p operators and the Jacobi-preconditioned CG that drives
 * the Poisson and Helmholtz solves of a projection step.
 *
 * The operations follow the method's statement of the problem:
 *   - mesh + order -> setup that stores the geometric factors at quadrature
 *     points (Section 3.1, after eq. tensorGradient: setup O(p^d), the Jacobian
 *     kept at quadrature points);
 *   - operator action of the mass, diffusion and Helmholtz operators
 *     (eq. vectorMass, eq. vectorDiffusion, eq. localStiffnessMapped, the
 *     Helmholtz combination A = c M + L of Section 5.2 and eq. proj-helmholtz),
 *     evaluated by sum factorization (eq. sumFactorized, eq. B1D, eq. D1D,
 *     eq. tensorGradient, L^K = G^T W G);
 *   - the exact diagonal of the assembled operator (Jacobi preconditioner);
 *   - Jacobi-PCG to a relative residual tolerance (Section 5, Section 5.3,
 *     the residual convention of Section 7.1), optionally with an FP32 inner
 *     solve inside FP64 iterative refinement;
 *   - the collocated (GLL-integrated, diagonal) mass matrix as the preconditioner
 *     of mass solves (Section 5.1), and the pure-Neumann Poisson problem closed by
 *     the mean-zero condition (eq. meanZero), whose CG orthogonalizes every
 *     preconditioner application against the constants (Section 5.3);
 *   - the adjoint gradient of an objective with respect to a per-quadrature-point
 *     coefficient nu (K depends linearly on nu through the factor W of Section 3.1).
 *
 * Conventions shared by every call:
 *   - Array arguments are DEVICE pointers owned by the caller, on the context's
 *     device, contiguous, unless stated otherwise.  The library never keeps or frees
 *     a caller pointer after a call returns; what it needs later it copies.
 *   - All device work is enqueued on the context's stream (sfem_create /
 *     sfem_set_stream).  apply, diagonal, load, grad_nu, qpoint_coords and
 *     set_coeffs are asynchronous with respect to the host.  setup synchronizes
 *     (it validates the mesh on the host); pcg synchronizes at its convergence
 *     checks and at exit.
 *   - No exception crosses the ABI.  Every call returns an sfem_status: 0 on
 *     success, negative on error (sfem_last_error(ctx) describes it), and the
 *     positive SFEM_NOCONV warning from pcg.  On error the output arrays are
 *     unspecified.  A context is not thread-safe; distinct contexts are independent.
 *   - Element geometry: trilinear hexahedra, vertex v = i + 2j + 4k at reference
 *     corner (2i-1, 2j-1, 2k-1).  Element DoFs: local l = i + n (j + n k), n = p + 1,
 *     i along xi_1 (GLL nodes).  Quadrature: Gauss-Legendre, q points per direction,
 *     point index a + q (b + q c); only q = p + 2 is built.
 *   - Essential (Dirichlet) DoFs: the operator is the constrained one,
 *     A_c = P A P + (I - P) with P zeroing essential DoFs, so (A_c x)_i = x_i and
 *     diag_i = 1 on them.  For homogeneous data the caller passes b_i = 0 there.
 *   - Batched vectors are [nbatch][ndof] (member-major).  Per-quadrature-point
 *     fields are [nfield][nelem][q^3] in the caller's element order.
 */
#ifndef SFEM_H
#define SFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFEM_ABI_VERSION 10
#define SFEM_MAX_P 8

typedef struct sfem_ctx sfem_ctx;

typedef enum {
  SFEM_OK = 0,
  SFEM_NOCONV = 1,         /* warning: maxit reached; x holds the last iterate, info is filled */
  SFEM_E_ARG = -1,         /* invalid argument (null pointer, bad size, bad enum, aliasing) */
  SFEM_E_MESH = -2,        /* invalid mesh: det J <= 0 at a quadrature point, bad DoF map */
  SFEM_E_HIP = -3,         /* a HIP runtime call or kernel launch failed */
  SFEM_E_NOMEM = -4,       /* device or host allocation failed */
  SFEM_E_UNSUPPORTED = -5, /* (p, q) not instantiated (p in 1..8, q = p + 2 only) */
  SFEM_E_NAN = -6,         /* non-finite value met in a solve */
  SFEM_E_BREAKDOWN = -7,   /* CG breakdown: p^T A p <= 0 (operator not SPD) */
  SFEM_E_STATE = -8        /* call out of order (e.g. apply before setup) */
} sfem_status;

typedef enum { SFEM_F64 = 0, SFEM_F32 = 1 } sfem_prec;

/* Operator kinds.  MASS: y = M x.  DIFFUSION: y = K(nu) x.  HELMHOLTZ:
 * y = alpha M x + beta K(nu) x with alpha, beta, nu from sfem_set_coeffs. */
typedef enum { SFEM_MASS = 0, SFEM_DIFFUSION = 1, SFEM_HELMHOLTZ = 2 } sfem_op;

/* Library ABI version (SFEM_ABI_VERSION). */
int sfem_abi_version(void);

/* Create a context on HIP device `device` whose work goes to `stream` (a
 * hipStream_t; NULL = the default stream).  *out receives a library-owned handle,
 * released by sfem_destroy.  On failure *out is NULL and sfem_last_error(NULL)
 * holds the message. */
sfem_status sfem_create(int device, void *stream, sfem_ctx **out);

/* Release every device and host resource of the context.  NULL is a no-op.
 * Waits for the context's stream to finish. */
void sfem_destroy(sfem_ctx *ctx);

/* Change the stream later calls enqueue on. */
sfem_status sfem_set_stream(sfem_ctx *ctx, void *stream);

/* Message of the last error on ctx (ctx = NULL: of the last failed sfem_create in
 * this process).  The string is owned by the library, valid until the next call. */
const char *sfem_last_error(const sfem_ctx *ctx);

/* Mesh + order setup (Section 3.1: geometric factors stored at quadrature points).
 *   p          polynomial order, 1..SFEM_MAX_P;  q: Gauss points per direction (= p + 2)
 *   nelem      number of hexahedra (>= 0)
 *   elem_xyz   [nelem][8][3] float64 vertex coordinates (device)
 *   elem_dofs  [nelem][(p+1)^3] int32 global DoF of each local node (device);
 *              values in [0, ndof), no DoF twice in one element, every DoF used
 *   ndof       number of global DoFs (< 2^30)
 *   ess_mask   [ndof] uint8, nonzero = essential DoF (device), or NULL (none)
 * Computes per quadrature point w|J| and w|J| J^{-1} J^{-T} (FP64), classifies the
 * DoFs (owned by one element, or shared and summed by an assembly pass without
 * atomics), and resets the coefficients to alpha = 1, beta = 1, nu = 1.  Returns SFEM_E_MESH if some
 * det J <= 0 or the map is invalid.  May be called again to replace the mesh. */
sfem_status sfem_setup(sfem_ctx *ctx, int p, int q, int64_t nelem, const double *elem_xyz,
                       const int32_t *elem_dofs, int64_t ndof, const uint8_t *ess_mask);

/* Physical coordinates of every quadrature point: xq[3][nelem * q^3] (device,
 * float64), element order of the caller. */
sfem_status sfem_qpoint_coords(sfem_ctx *ctx, double *xq);

/* Helmholtz coefficients A = alpha M + beta K(nu) (Section 5.2, eq. proj-helmholtz).
 *   nu_q       [nbatch_nu][nelem * q^3] float64 per-quadrature-point viscosity
 *              (device, copied), or NULL for nu = 1
 *   nbatch_nu  number of nu fields (>= 1); with more than one field, a batched
 *              apply / solve must use nbatch == nbatch_nu and member m uses field m
 * Recomputes the folded quadrature data and the operator diagonals. */
sfem_status sfem_set_coeffs(sfem_ctx *ctx, double alpha, double beta, const double *nu_q,
                            int nbatch_nu);

/* y = A x for nbatch vectors.  x, y: [nbatch][ndof] of float64 (SFEM_F64) or
 * float32 (SFEM_F32), device, not aliased.  FP32 uses float32 copies of the 1D
 * tables and the quadrature data rounded from FP64. */
sfem_status sfem_apply(sfem_ctx *ctx, int op, int prec, int nbatch, const void *x, void *y);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): y = A x exactly as sfem_apply (same
 * kernels, same results), except that the E-vector of the shared-node contributions lives
 * in a fixed library scratch array of SFEM_APPLY_NOALLOC_MAX_BYTES on each GPU instead of
 * context memory.  The call allocates and frees nothing (no hipMalloc, hipFree or
 * allocating library routine); the context must be set up (sfem_setup, sfem_set_coeffs)
 * beforehand.  Needs nbatch * nentries * (8 for SFEM_F64, 4 for SFEM_F32) bytes of scratch
 * (nentries from sfem_get_info); larger calls return SFEM_E_ARG without launching.  Every
 * context on one GPU shares that GPU's scratch, which keeps the last call's contents: each
 * call writes every scratch entry it reads before reading it, so nothing needs clearing,
 * but calls that overlap in time on one GPU (other streams, other host threads) race and
 * must be ordered by the caller.  The scratch is held until the process ends. */
#define SFEM_APPLY_NOALLOC_MAX_BYTES (64ull << 20)
sfem_status sfem_apply_noalloc(sfem_ctx *ctx, int op, int prec, int nbatch, const void *x, void *y);

/* Low-order-refined preconditioner (Section 5.2).  A_LOR = a M_LOR + b K_LOR is the
 * trilinear (Q1) discretization of the operator kind op (MASS: a = 1, b = 0; DIFFUSION:
 * 0, 1; HELMHOLTZ: alpha, beta of sfem_set_coeffs) on the refined mesh that splits every
 * element into the p^3 sub-hexahedra between its GLL points (each the trilinear element
 * through its 8 corner nodes, 2 x 2 x 2 Gauss points); nu enters as its mean over each
 * element's quadrature points; essential DoFs are constrained as in the operator.  A_LOR
 * has the operator's unknowns, is spectrally equivalent to it with h- and p-independent
 * constants, and has at most 27 nonzeros per row on a structured mesh.  Its solver is a
 * smoothed-aggregation algebraic multigrid V-cycle (strength threshold 0.02, three-pass
 * aggregation, Jacobi-smoothed prolongator, Galerkin coarse operators down to <= 200 rows,
 * dense pseudo-inverse there, one damped-Jacobi sweep before and one after each coarse
 * correction): the setup runs on the host (the mesh copy kept by sfem_setup; up to 16
 * host threads, SFEM_HOST_THREADS in the environment sets their number, the result does
 * not depend on it), every step of the V-cycle on the GPU.  sfem_pcg with precond = SFEM_PRECOND_LOR builds it on first
 * use; sfem_set_coeffs discards it.  One nu field only (SFEM_E_ARG otherwise).
 *   sfem_lor_setup   build it now; info (host, may be NULL) gets the level sizes
 *   sfem_lor_apply   y = A_LOR x  (device [ndof] float64)
 *   sfem_lor_vcycle  x = one V-cycle for A_LOR x = b from x = 0 (device [ndof] float64),
 *                    computed in FP64 (prec = SFEM_F64) or with FP32 copies of the
 *                    hierarchy's matrices and FP32 vectors (SFEM_F32: b is rounded to
 *                    float32 on entry, the result widened to float64; the FP32 copies are
 *                    made on first use and kept with the hierarchy)
 * Synchronous (setup); apply and vcycle are asynchronous on the context stream. */
#define SFEM_LOR_MAX_LEVELS 12
typedef struct {
  int levels;                          /* multigrid levels (the finest is A_LOR) */
  int64_t rows[SFEM_LOR_MAX_LEVELS];   /* rows per level */
  int64_t nnz[SFEM_LOR_MAX_LEVELS];    /* nonzeros per level */
  double setup_ms;                     /* host setup time of the hierarchy */
  int32_t sliced[SFEM_LOR_MAX_LEVELS]; /* device storage per level: bit 0 the operator, bit 1
                                          the prolongator, bit 2 the restriction in sliced
                                          ELL (64-row slices), else CSR (the coarsest
                                          level: a dense inverse); bit 3: slices of the
                                          operator whose rows share their column offsets
                                          store those once instead of column indices */
} sfem_lor_info;
sfem_status sfem_lor_setup(sfem_ctx *ctx, int op, sfem_lor_info *info);
sfem_status sfem_lor_apply(sfem_ctx *ctx, int op, const double *x, double *y);
sfem_status sfem_lor_vcycle(sfem_ctx *ctx, int op, int prec, const double *b, double *x);

/* Exact diagonal of the constrained assembled operator (1 on essential DoFs).
 * diag: [nfield][ndof] with nfield = 1 for MASS (and when nu is NULL), otherwise
 * the number of nu fields; float64 or float32 per prec (device). */
sfem_status sfem_diagonal(sfem_ctx *ctx, int op, int prec, void *diag);

/* Load vector b_i = sum_e sum_q w|J| f_q phi_i for nbatch sources,
 * f_q: [nbatch][nelem * q^3] float64, b: [nbatch][ndof] float64 (device);
 * essential entries of b are set to 0. */
sfem_status sfem_load(sfem_ctx *ctx, int nbatch, const double *f_q, double *b);

/* Collocated mass diagonal (Section 5.1): the mass matrix integrated with the GLL rule
 * at the element nodes is diagonal, entry g = sum over the elements and their nodes
 * l -> g of w_l |J(xi_l)| (tensor GLL weight, Jacobian determinant at the node);
 * spectrally equivalent to the Gauss-integrated mass with h- and p-independent
 * constants.  diag: [ndof] float64 (device); essential entries are 1. */
sfem_status sfem_collocated_mass(sfem_ctx *ctx, double *diag);

typedef enum {
  SFEM_PRECOND_JACOBI = 0,          /* exact diagonal of the (constrained) operator */
  SFEM_PRECOND_COLLOCATED_MASS = 1, /* collocated mass diagonal (for mass solves, Section 5.1) */
  SFEM_PRECOND_LOR = 2,             /* one multigrid V-cycle on the low-order-refined operator
                                       (Section 5.2, see sfem_lor_setup); FP64 CG (mode 0) */
  SFEM_PRECOND_LOR32 = 3            /* the same V-cycle in FP32 arithmetic (sfem_lor_vcycle with
                                       SFEM_F32) inside FP64 CG (mode 0): half the bytes per
                                       cycle; the CG, its residuals and scalars stay FP64 */
} sfem_precond;

typedef struct {
  double rtol;       /* stop when ||r||_2 <= rtol ||b||_2, per batch member */
  int maxit;         /* iteration cap (mode 1: cap on the total inner iterations) */
  int mode;          /* 0: FP64 Jacobi-PCG; 1: FP32 inner Jacobi-PCG inside FP64 iterative refinement */
  double inner_rtol; /* mode 1: relative tolerance of an inner solve (e.g. 1e-5); once the
                        reduction still needed, need = rtol ||b|| / ||r||, is >= inner_rtol / 10,
                        the inner solve asks for need / 2 instead and ends the refinement */
  int max_outer;     /* mode 1: cap on refinement steps */
  int check_every;   /* iterations between host convergence checks (>= 1) */
  int x0_zero;       /* nonzero: ignore x on entry and start from x = 0 */
  int precond;       /* sfem_precond: diagonal preconditioner */
  int nullspace;     /* nonzero: pure-Neumann problem (op = SFEM_DIFFUSION, no essential
                        DoFs): b is made orthogonal to the constants, every preconditioner
                        application is orthogonalized against them (Section 5.3), and x is
                        returned with int x = 0 (eq. meanZero); modes 0 and 1 (in mode 1
                        the inner FP32 solves are orthogonalized the same way), with or
                        without an initial guess (its constant part does not matter) */
} sfem_pcg_opts;

typedef struct {
  int iters;           /* CG iterations (mode 1: total inner iterations) */
  int outer;           /* mode 1: refinement steps; mode 0: 0 */
  double rel_res;      /* last recursive (mode 0) or true (mode 1) ||r|| / ||b|| */
  double true_rel_res; /* ||b - A_c x|| / ||b|| recomputed in FP64 at exit */
  int status;          /* per-member sfem_status */
} sfem_pcg_info;

/* Solve A x = b for nbatch right-hand sides by diagonally preconditioned CG
 * (opts->precond: the exact operator diagonal or the collocated mass).  b: [nbatch][ndof] float64; x: [nbatch][ndof]
 * float64, initial guess on entry (unless opts->x0_zero), solution on exit.
 * info: host array of nbatch entries (may be NULL).  Returns SFEM_OK when every
 * member converged, SFEM_NOCONV if some did not (x = last iterate), or an error. */
sfem_status sfem_pcg(sfem_ctx *ctx, int op, int nbatch, const double *b, double *x,
                     const sfem_pcg_opts *opts, sfem_pcg_info *info);

/* Adjoint gradient integrand for a per-quadrature-point nu:
 *   g_q = -beta * w|J| (J^{-T} grad lam) . (J^{-T} grad u)
 * so that dJ/dnu_q = g_q when A(nu) u = b and A lam = dJ/du.
 * u, lam: [nbatch][ndof] float64; g: [nbatch][nelem * q^3] float64 (device). */
sfem_status sfem_grad_nu(sfem_ctx *ctx, int nbatch, const double *u, const double *lam, double *g);

/* Taylor-Hood pressure space for the Stokes blocks (Section 3: velocity (Q_p)^3, pressure
 * Q_{p-1}, nodal GLL bases; p >= 2): the order-(p-1) element->DoF map of the same elements
 * as sfem_setup, pres_dofs [nelem][p^3] int32 (device, local l = i + p (j + p k)), with
 * npres pressure DoFs; the pressure space has no essential DoFs.  Also stores the
 * coupling factors w |J| J^{-T} at the quadrature points.  Once per sfem_setup.
 * Errors: SFEM_E_UNSUPPORTED for p < 2, SFEM_E_MESH for an invalid map, SFEM_E_STATE
 * before sfem_setup or when called twice. */
sfem_status sfem_setup_pressure(sfem_ctx *ctx, const int32_t *pres_dofs, int64_t npres);

/* Constrained Stokes block operator of one implicit stage (eq. unsteadyStokesDiscrete,
 * with the coefficients of sfem_set_coeffs, one nu field: H = alpha M + beta K(nu) on each
 * velocity component):
 *   y_u = P H P u + (I - P) u + P G p,    y_p = -D P u,
 * G and D the gradient and divergence blocks (eq. gradient, eq. divergence), P zeroing
 * the essential velocity DoFs.  u, y_u: [3][ndof] float64 (component-major); p, y_p:
 * [npres] float64 (device).  Asynchronous on the context stream.  Errors: SFEM_E_STATE
 * before sfem_setup_pressure, SFEM_E_ARG for NULL or aliased arrays or several nu
 * fields. */
sfem_status sfem_stokes_apply(sfem_ctx *ctx, const double *u, const double *p, double *yu,
                              double *yp);

/* Convection term of the Navier-Stokes problem (eq. nonlinear) on the velocity space:
 *   y_{c,i} = sum_e sum_q w|J| phi_i ((u . grad) u)_c,
 * u, y: [3][ndof] float64 (device, component-major).  u is taken with its boundary values;
 * rows of essential DoFs are set to 0 (the term is a right-hand side of the constrained
 * solves).  Uses the coupling factors w |J| J^{-T} (computed on first use).
 * Asynchronous on the context stream.  Errors: SFEM_E_ARG for NULL or aliased arrays. */
sfem_status sfem_convection(sfem_ctx *ctx, const double *u, double *y);

/* Equal-order weak vector operators of the projection step (Section 4.2, the pressure
 * Poisson right-hand side of eq. pres-poisson and the pressure gradient of
 * eq. proj-helmholtz), every field in the scalar space of the context:
 *   SFEM_WEAK_GRADIENT    y_{c,i} = sum_e sum_q w|J| phi_i (grad x)_c
 *                         x: [ndof], y: [3][ndof]
 *   SFEM_WEAK_CURL        y_{c,i} = sum_e sum_q w|J| phi_i (curl x)_c
 *                         x, y: [3][ndof]
 *   SFEM_WEAK_DIVERGENCE  y_i = sum_e sum_q w|J| grad phi_i . x
 *                         x: [3][ndof], y: [ndof]
 * (float64, device, component-major; grad = J^{-T} grad_ref at the Gauss points.)  x is
 * taken with all its values; rows of essential DoFs are set to 0 (a context without
 * essential DoFs gives every row).  Uses the coupling factors w |J| J^{-T} (computed on
 * first use).  Asynchronous on the context stream.  Errors: SFEM_E_ARG for a bad kind or
 * NULL or aliased arrays. */
#define SFEM_WEAK_GRADIENT 1
#define SFEM_WEAK_CURL 2
#define SFEM_WEAK_DIVERGENCE 3
sfem_status sfem_weak_op(sfem_ctx *ctx, int kind, const double *x, double *y);

/* Nodal combination of the projection step (eq. projKnown, the extrapolations of
 * Section 4.2 and the nodal fields B^{-1} y of the collocated mass B, Section 5.1):
 *   y[m][i] = (sum_{j < nterm} coef[j] xs[j][m][i]) / scale[i],   0 where mask[i] != 0,
 * for nb members of length n.  coef: host array [nterm] (1 <= nterm <= 8); xs: host array
 * of nterm device pointers to [nb][n] float64; scale: device [n] float64 or NULL (no
 * division); mask: device [n] uint8 or NULL; y: device [nb][n] float64, which may be one
 * of the xs[j].  Asynchronous on the context stream.  Errors: SFEM_E_ARG for a bad nterm,
 * sizes or NULL arrays. */
sfem_status sfem_lincomb(sfem_ctx *ctx, int nterm, const double *coef, const double *const *xs,
                         const double *scale, const uint8_t *mask, int64_t n, int nb, double *y);

/* ---- Projection time stepping (Section 4.2) ------------------------------------------
 *
 * BDF-k / EXT-k weights for a constant step (k = 1, 2, 3): b[0..k] with
 * sum_j b_j g(t_{n+1-j}) = dt g'(t_{n+1}) for every polynomial g of degree <= k, and
 * a[0..k-1] (a_j of u^{n+1-j}, j = 1..k) with sum_j a_j g(t_{n+1-j}) = g(t_{n+1}) for
 * degree <= k - 1; solved from these exactness conditions.  b, a: host arrays of k + 1 and
 * k doubles.  A host computation (no device call).  Errors: SFEM_E_ARG for k outside 1..3
 * or NULL arrays. */
sfem_status sfem_bdf_ext_weights(int k, double *b, double *a);

typedef struct sfem_flow sfem_flow; /* opaque, library-owned */

typedef struct {
  double dt;          /* time step (> 0), constant */
  double nu;          /* kinematic viscosity (>= 0), constant */
  double rtol;        /* relative residual tolerance of the pressure and velocity solves */
  int order;          /* BDF/EXT order 1..3; the first steps ramp up 1, 2, .. to it */
  int pressure_mode;  /* pressure Poisson: 0 FP64 Jacobi-PCG, 1 FP32 inner solves in FP64 refinement */
  int check_every;    /* iterations between host convergence checks of the solves (>= 1) */
  int maxit;          /* iteration cap of each solve (>= 1) */
  int pressure_precond; /* pressure Poisson preconditioner: SFEM_PRECOND_JACOBI,
                           SFEM_PRECOND_LOR or SFEM_PRECOND_LOR32 (Section 5.2; FP64 CG,
                           pressure_mode ignored) */
  int velocity_mode;  /* Helmholtz velocity solve (Jacobi-preconditioned, three members): 0 FP64
                         PCG, 1 FP32 inner solves in FP64 refinement */
} sfem_flow_opts;

typedef struct {
  int order;                  /* BDF/EXT order of the step just taken */
  sfem_pcg_info pressure;     /* the pressure Poisson solve */
  sfem_pcg_info velocity[3];  /* the Helmholtz solve of each velocity component */
} sfem_flow_info;

/* Velocity-correction projection stepper (Section 4.2: eq. projKnown, eq. projLinear,
 * eq. pres-poisson with eq. presPoissonBC and eq. meanZero, eq. proj-helmholtz) for
 * equal-order velocity and pressure (each velocity component and the pressure in the
 * continuous Q_p space of the mesh), no-slip walls on the essential DoFs given by ess_mask,
 * constant nu and dt.  Mesh arguments as for sfem_setup (device arrays, copied; ess_mask
 * must not be NULL).  The stepper holds two set-up contexts on the mesh (with and without
 * the walls), the collocated GLL mass B (Section 5.1), the step history and its work
 * vectors (about 25 ndof doubles).  *out receives the handle; on failure it is NULL and
 * sfem_flow_last_error(NULL) holds the message. */
sfem_status sfem_flow_create(int device, void *stream, int p, int64_t nelem, const double *elem_xyz,
                             const int32_t *elem_dofs, int64_t ndof, const uint8_t *ess_mask,
                             const sfem_flow_opts *opts, sfem_flow **out);
void sfem_flow_destroy(sfem_flow *flow);
const char *sfem_flow_last_error(const sfem_flow *flow);
sfem_status sfem_flow_set_stream(sfem_flow *flow, void *stream);

/* One step of order k = min(steps taken + 1, order) from u = u^n [3][ndof] (device, float64,
 * component-major, 0 on the walls) with the nodal forcing f = f^{n+1} [3][ndof] (device) or
 * NULL:
 *   N^n = -B^{-1} C(u^n) (the convection term, rows of wall DoFs 0);
 *   F* = sum_j a_j N^{n+1-j} - sum_j (b_j / dt) u^{n+1-j} + f^{n+1};
 *   u* = sum_j a_j u^{n+1-j};  L* = -nu B^{-1} curl_w(B^{-1} curl_w u*);
 *   K p = div_w(F* + L*) with int p = 0, by the orthogonalized pure-Neumann CG
 *   (pressure_precond, pressure_mode), from the previous step's pressure (an EXT
 *   extrapolation of the previous pressures took more iterations on the 32^3 p = 4 runs);
 *   (b_0/dt) M u + nu K u = M F* - grad_w p on the free rows, u = 0 on the walls, by
 *   three-member Jacobi-PCG (velocity_mode) from u*.
 * Writes u_out = u^{n+1} [3][ndof] and p_out = p^{n+1} [ndof] (device, not aliasing u) and
 * shifts the history; info (host, may be NULL) gets the order and the solves' outcomes.
 * Returns SFEM_NOCONV (the step is taken) if a solve reached maxit, negative on error.
 * Synchronizes with the host at the solves' convergence checks. */
sfem_status sfem_flow_step(sfem_flow *flow, const double *u, const double *f, double *u_out,
                           double *p_out, sfem_flow_info *info);

typedef struct {
  int p, q;
  int64_t nelem, ndof;
  int compact;            /* 1: only element-surface nodes pass through the E-vector */
  int nfields;            /* nu fields set by sfem_set_coeffs (1 when nu is NULL) */
  int64_t device_bytes;   /* device memory held by the context */
  int64_t nassembled;     /* DoFs shared by several elements, plus essential DoFs */
  int64_t nentries;       /* E-vector entries per batch member (shared-node contributions) */
} sfem_ctx_info;

/* Sizes and counters of a set-up context (host struct). */
sfem_status sfem_get_info(const sfem_ctx *ctx, sfem_ctx_info *out);

#ifdef __cplusplus
}
#endif
#endif /* SFEM_H */
