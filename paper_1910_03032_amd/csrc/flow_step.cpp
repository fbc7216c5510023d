// Velocity-correction projection steps (Section 4.2) behind the C ABI: the BDF-k/EXT-k
// weights, and a stepper that owns two contexts on one mesh (the velocity space with the
// no-slip walls as essential DoFs, and the same space without essential DoFs for the
// weak vector operators, the mass and the pure-Neumann pressure problem), the step
// history and its work vectors, and orders the library's kernels and solves.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "sfem.h"

namespace {

// Solve the dense n x n system M z = r (row-major, n <= 4) by Gaussian elimination with
// partial pivoting; false if M is singular.
bool dense_solve(int n, double *M, double *r, double *z) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int i = c + 1; i < n; ++i)
      if (std::fabs(M[i * n + c]) > std::fabs(M[piv * n + c])) piv = i;
    if (M[piv * n + c] == 0.0) return false;
    if (piv != c) {
      for (int j = 0; j < n; ++j) std::swap(M[c * n + j], M[piv * n + j]);
      std::swap(r[c], r[piv]);
    }
    for (int i = c + 1; i < n; ++i) {
      const double f = M[i * n + c] / M[c * n + c];
      for (int j = c; j < n; ++j) M[i * n + j] -= f * M[c * n + j];
      r[i] -= f * r[c];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double v = r[i];
    for (int j = i + 1; j < n; ++j) v -= M[i * n + j] * z[j];
    z[i] = v / M[i * n + i];
  }
  return true;
}

}  // namespace

struct sfem_flow {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  sfem_ctx *vel = nullptr;   // essential DoFs = walls: convection, Helmholtz solve
  sfem_ctx *free = nullptr;  // no essential DoFs: weak operators, mass, pressure solve
  int64_t n = 0;
  sfem_flow_opts o{};
  double alpha_set = -1.0;   // b_0 / dt of the velocity context's coefficients
  int nstep = 0;
  int nhist = 0;             // history entries held (<= order)
  std::vector<void *> bufs;  // every device allocation
  double *us[3] = {}, *ns[3] = {};  // newest first, [3][n] each
  double *F = nullptr, *ustar = nullptr, *t3 = nullptr, *w = nullptr, *L = nullptr, *R = nullptr;
  double *r = nullptr, *pprev = nullptr, *B = nullptr;
  uint8_t *mask = nullptr;
};

namespace {

sfem_status ffail(sfem_flow *f, sfem_status st, const std::string &msg) {
  if (f) f->err = msg;
  return st;
}

// Run a library call on one of the stepper's contexts; on failure copy its message.
sfem_status chk(sfem_flow *f, sfem_ctx *c, sfem_status st, const char *what) {
  if (st < 0) return ffail(f, st, std::string(what) + ": " + sfem_last_error(c));
  return SFEM_OK;
}

#define FCHK(f, c, call)                                        \
  do {                                                          \
    sfem_status st_ = chk((f), (c), (call), #call);             \
    if (st_ != SFEM_OK) return st_;                             \
  } while (0)

#define FHIP(f, expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ffail((f), SFEM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DevGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

void release(sfem_flow *f) {
  for (void *p : f->bufs) (void)hipFree(p);
  f->bufs.clear();
  sfem_destroy(f->vel);
  sfem_destroy(f->free);
  f->vel = f->free = nullptr;
}

template <typename T>
sfem_status falloc(sfem_flow *f, T **out, int64_t count) {
  void *p = nullptr;
  if (hipMalloc(&p, (size_t)count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return ffail(f, SFEM_E_NOMEM, "projection stepper: device allocation failed");
  }
  f->bufs.push_back(p);
  *out = (T *)p;
  return SFEM_OK;
}

}  // namespace

extern "C" {

sfem_status sfem_bdf_ext_weights(int k, double *b, double *a) {
  if (k < 1 || k > 3 || !b || !a) return SFEM_E_ARG;
  // node t_{n+1-j} at s_j = -j steps from t_{n+1}
  double M[16], r[4], z[4];
  // BDF: sum_j b_j s_j^m = d/ds s^m at 0 (1 for m = 1, else 0), m = 0..k
  for (int m = 0; m <= k; ++m) {
    for (int j = 0; j <= k; ++j) M[m * (k + 1) + j] = std::pow(-(double)j, m);
    r[m] = (m == 1) ? 1.0 : 0.0;
  }
  if (!dense_solve(k + 1, M, r, z)) return SFEM_E_ARG;
  for (int j = 0; j <= k; ++j) b[j] = z[j];
  // EXT: sum_{j=1..k} a_j s_j^m = s^m at 0 (1 for m = 0, else 0), m = 0..k-1
  for (int m = 0; m < k; ++m) {
    for (int j = 1; j <= k; ++j) M[m * k + (j - 1)] = std::pow(-(double)j, m);
    r[m] = (m == 0) ? 1.0 : 0.0;
  }
  if (!dense_solve(k, M, r, z)) return SFEM_E_ARG;
  for (int j = 0; j < k; ++j) a[j] = z[j];
  return SFEM_OK;
}

static std::string g_flow_create_error;

sfem_status sfem_flow_create(int device, void *stream, int p, int64_t nelem, const double *elem_xyz,
                             const int32_t *elem_dofs, int64_t ndof, const uint8_t *ess_mask,
                             const sfem_flow_opts *opts, sfem_flow **out) {
  if (!out) return SFEM_E_ARG;
  *out = nullptr;
  auto bad = [](sfem_status st, const std::string &m) {
    g_flow_create_error = m;
    return st;
  };
  if (!opts) return bad(SFEM_E_ARG, "opts must not be NULL");
  if (!(opts->dt > 0.0) || !(opts->nu >= 0.0) || !std::isfinite(opts->dt) || !std::isfinite(opts->nu))
    return bad(SFEM_E_ARG, "dt > 0 and nu >= 0 (finite) are required");
  if (opts->order < 1 || opts->order > 3) return bad(SFEM_E_ARG, "order must be 1, 2 or 3");
  if (!(opts->rtol > 0.0) || (opts->pressure_mode != 0 && opts->pressure_mode != 1) ||
      (opts->velocity_mode != 0 && opts->velocity_mode != 1) || opts->check_every < 1 || opts->maxit < 1 ||
      (opts->pressure_precond != SFEM_PRECOND_JACOBI && opts->pressure_precond != SFEM_PRECOND_LOR &&
       opts->pressure_precond != SFEM_PRECOND_LOR32))
    return bad(SFEM_E_ARG, "rtol > 0, pressure_mode and velocity_mode 0 or 1, check_every >= 1, "
                           "maxit >= 1 and a Jacobi or LOR pressure preconditioner are required");
  if (!ess_mask) return bad(SFEM_E_ARG, "ess_mask (the no-slip walls) must not be NULL");
  sfem_flow *f = new (std::nothrow) sfem_flow();
  if (!f) return bad(SFEM_E_NOMEM, "host allocation failed");
  f->device = device;
  f->stream = (hipStream_t)stream;
  f->o = *opts;
  f->n = ndof;
  DevGuard g(device);
  auto fail_create = [&](sfem_status st, const std::string &m) {
    g_flow_create_error = m;
    release(f);
    delete f;
    return st;
  };
  sfem_status st = sfem_create(device, stream, &f->vel);
  if (st != SFEM_OK) return fail_create(st, std::string("velocity context: ") + sfem_last_error(nullptr));
  st = sfem_create(device, stream, &f->free);
  if (st != SFEM_OK) return fail_create(st, std::string("pressure context: ") + sfem_last_error(nullptr));
  const int q = p + 2;
  st = sfem_setup(f->vel, p, q, nelem, elem_xyz, elem_dofs, ndof, ess_mask);
  if (st != SFEM_OK) return fail_create(st, std::string("velocity setup: ") + sfem_last_error(f->vel));
  st = sfem_setup(f->free, p, q, nelem, elem_xyz, elem_dofs, ndof, nullptr);
  if (st != SFEM_OK) return fail_create(st, std::string("pressure setup: ") + sfem_last_error(f->free));
  const int64_t n = ndof;
  sfem_status sa = SFEM_OK;
  for (int j = 0; j < 3 && sa == SFEM_OK; ++j) {
    sa = falloc(f, &f->us[j], 3 * n);
    if (sa == SFEM_OK) sa = falloc(f, &f->ns[j], 3 * n);
  }
  double **v3[] = {&f->F, &f->ustar, &f->t3, &f->w, &f->L, &f->R};
  for (double **d : v3)
    if (sa == SFEM_OK) sa = falloc(f, d, 3 * n);
  double **v1[] = {&f->r, &f->pprev, &f->B};
  for (double **d : v1)
    if (sa == SFEM_OK) sa = falloc(f, d, n);
  if (sa == SFEM_OK) sa = falloc(f, &f->mask, n > 0 ? n : 1);
  if (sa != SFEM_OK) return fail_create(sa, f->err);
  if (n > 0) {
    if (hipMemcpyAsync(f->mask, ess_mask, (size_t)n, hipMemcpyDeviceToDevice, f->stream) != hipSuccess)
      return fail_create(SFEM_E_HIP, "copying the wall mask failed");
    st = sfem_collocated_mass(f->free, f->B);
    if (st != SFEM_OK) return fail_create(st, std::string("collocated mass: ") + sfem_last_error(f->free));
  }
  *out = f;
  return SFEM_OK;
}

void sfem_flow_destroy(sfem_flow *f) {
  if (!f) return;
  {
    DevGuard g(f->device);
    (void)hipStreamSynchronize(f->stream);
    release(f);
  }
  delete f;
}

const char *sfem_flow_last_error(const sfem_flow *f) {
  return f ? f->err.c_str() : g_flow_create_error.c_str();
}

sfem_status sfem_flow_set_stream(sfem_flow *f, void *stream) {
  if (!f) return SFEM_E_ARG;
  f->stream = (hipStream_t)stream;
  sfem_set_stream(f->vel, stream);
  sfem_set_stream(f->free, stream);
  return SFEM_OK;
}

sfem_status sfem_flow_step(sfem_flow *f, const double *u, const double *frc, double *u_out,
                           double *p_out, sfem_flow_info *info) {
  if (!f) return SFEM_E_ARG;
  const int64_t n = f->n;
  if (n == 0) return SFEM_OK;
  if (!u || !u_out || !p_out) return ffail(f, SFEM_E_ARG, "u, u_out and p_out must not be NULL");
  if (u == u_out || (const double *)p_out == u) return ffail(f, SFEM_E_ARG, "outputs must not alias u");
  DevGuard g(f->device);
  hipStream_t s = f->stream;
  const double dt = f->o.dt, nu = f->o.nu;
  const int k = f->nstep + 1 < f->o.order ? f->nstep + 1 : f->o.order;
  double b[4], a[3];
  if (sfem_bdf_ext_weights(k, b, a) != SFEM_OK) return ffail(f, SFEM_E_ARG, "BDF/EXT weights");
  // history: the oldest slot becomes the newest (u^n and N^n = -B^{-1} C(u^n))
  double *u_new = f->us[2], *n_new = f->ns[2];
  for (int j = 2; j > 0; --j) {
    f->us[j] = f->us[j - 1];
    f->ns[j] = f->ns[j - 1];
  }
  f->us[0] = u_new;
  f->ns[0] = n_new;
  f->nhist = f->nhist + 1 < 3 ? f->nhist + 1 : 3;
  FHIP(f, hipMemcpyAsync(u_new, u, (size_t)3 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  FCHK(f, f->vel, sfem_convection(f->vel, u_new, f->t3));
  {
    const double c[1] = {-1.0};
    const double *xs[1] = {f->t3};
    FCHK(f, f->free, sfem_lincomb(f->free, 1, c, xs, f->B, nullptr, n, 3, n_new));
  }
  // F* = sum_j a_j N^{n+1-j} - (b_j / dt) u^{n+1-j} (+ f^{n+1})      (eq. projKnown)
  {
    double c[8];
    const double *xs[8];
    int t = 0;
    for (int j = 0; j < k; ++j) {
      c[t] = a[j];
      xs[t++] = f->ns[j];
    }
    for (int j = 0; j < k; ++j) {
      c[t] = -b[j + 1] / dt;
      xs[t++] = f->us[j];
    }
    if (frc) {
      c[t] = 1.0;
      xs[t++] = frc;
    }
    FCHK(f, f->free, sfem_lincomb(f->free, t, c, xs, nullptr, nullptr, n, 3, f->F));
  }
  // u* = sum_j a_j u^{n+1-j}
  {
    const double *xs[3] = {f->us[0], f->us[1], f->us[2]};
    FCHK(f, f->free, sfem_lincomb(f->free, k, a, xs, nullptr, nullptr, n, 3, f->ustar));
  }
  // L* = -nu B^{-1} curl_w(B^{-1} curl_w u*)                          (eq. projLinear)
  FCHK(f, f->free, sfem_weak_op(f->free, SFEM_WEAK_CURL, f->ustar, f->t3));
  {
    const double c[1] = {1.0};
    const double *xs[1] = {f->t3};
    FCHK(f, f->free, sfem_lincomb(f->free, 1, c, xs, f->B, nullptr, n, 3, f->w));
  }
  FCHK(f, f->free, sfem_weak_op(f->free, SFEM_WEAK_CURL, f->w, f->t3));
  {
    const double c[1] = {-nu};
    const double *xs[1] = {f->t3};
    FCHK(f, f->free, sfem_lincomb(f->free, 1, c, xs, f->B, nullptr, n, 3, f->L));
  }
  // pressure Poisson K p = div_w(F* + L*), int p = 0   (eq. pres-poisson, eq. meanZero)
  {
    const double c[2] = {1.0, 1.0};
    const double *xs[2] = {f->F, f->L};
    FCHK(f, f->free, sfem_lincomb(f->free, 2, c, xs, nullptr, nullptr, n, 3, f->t3));
  }
  FCHK(f, f->free, sfem_weak_op(f->free, SFEM_WEAK_DIVERGENCE, f->t3, f->r));
  sfem_pcg_opts po{};
  po.rtol = f->o.rtol;
  po.maxit = f->o.maxit;
  po.mode = f->o.pressure_mode;
  po.inner_rtol = 1e-5;
  po.max_outer = 30;
  po.check_every = f->o.check_every;
  po.precond = f->o.pressure_precond;
  if (po.precond != SFEM_PRECOND_JACOBI) po.mode = 0;  // the LOR V-cycle runs with FP64 CG
  po.nullspace = 1;
  po.x0_zero = f->nstep == 0 ? 1 : 0;  // later steps start from the previous pressure
  if (!po.x0_zero)
    FHIP(f, hipMemcpyAsync(p_out, f->pprev, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  sfem_pcg_info pinfo{};
  sfem_status stp = sfem_pcg(f->free, SFEM_DIFFUSION, 1, f->r, p_out, &po, &pinfo);
  if (stp < 0) return chk(f, f->free, stp, "pressure solve");
  FHIP(f, hipMemcpyAsync(f->pprev, p_out, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  // Helmholtz (b_0/dt) M u + nu K u = M F* - grad_w p, u = 0 on the walls (eq. proj-helmholtz)
  FCHK(f, f->free, sfem_apply(f->free, SFEM_MASS, SFEM_F64, 3, f->F, f->R));
  FCHK(f, f->free, sfem_weak_op(f->free, SFEM_WEAK_GRADIENT, p_out, f->t3));
  {
    const double c[2] = {1.0, -1.0};
    const double *xs[2] = {f->R, f->t3};
    FCHK(f, f->free, sfem_lincomb(f->free, 2, c, xs, nullptr, f->mask, n, 3, f->R));
  }
  const double alpha = b[0] / dt;
  if (alpha != f->alpha_set) {
    FCHK(f, f->vel, sfem_set_coeffs(f->vel, alpha, nu, nullptr, 1));
    f->alpha_set = alpha;
  }
  // start from the extrapolated velocity
  FHIP(f, hipMemcpyAsync(u_out, f->ustar, (size_t)3 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  sfem_pcg_opts vo = po;
  vo.mode = f->o.velocity_mode;
  vo.precond = SFEM_PRECOND_JACOBI;
  vo.nullspace = 0;
  vo.x0_zero = 0;
  sfem_pcg_info vinfo[3] = {};
  sfem_status stv = sfem_pcg(f->vel, SFEM_HELMHOLTZ, 3, f->R, u_out, &vo, vinfo);
  if (stv < 0) return chk(f, f->vel, stv, "velocity solve");
  if (info) {
    info->order = k;
    info->pressure = pinfo;
    for (int c = 0; c < 3; ++c) info->velocity[c] = vinfo[c];
  }
  ++f->nstep;
  if (stp == SFEM_NOCONV || stv == SFEM_NOCONV)
    return ffail(f, SFEM_NOCONV, "projection step: a solve reached its iteration cap");
  return SFEM_OK;
}

}  // extern "C"
