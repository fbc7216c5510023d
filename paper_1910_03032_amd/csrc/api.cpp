// C ABI of the sfem library: context, mesh setup (map validation, sole/shared DoF
// classification, assembly lists, geometric factors), operator apply / diagonal / load /
// adjoint gradient dispatch, and the Jacobi-PCG and FP32-inner iterative-refinement
// drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "internal.h"
#include "flow.h"
#include "lor.h"

using namespace sfem;

// Scratch of the allocation-free apply (sfem_apply_noalloc): the E-vector of the
// shared-node contributions.  Each GPU the library runs on holds its own copy of this
// array until the process ends.  In host code its name is only a stand-in: the device
// address comes from hipGetSymbolAddress, resolved once per device (resolve_scratch).
static __device__ __align__(256) char scratch[SFEM_APPLY_NOALLOC_MAX_BYTES];

namespace {

std::string g_create_error;  // message of the last failed sfem_create

// Device address of `scratch` per device, resolved at the first sfem_create on that
// device (with the device current).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxDevices] = {};
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

hipError_t resolve_scratch(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();
    g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
    g_scratch_err[device] = e;
    g_scratch_done[device] = true;
  }
  *out = g_scratch_ptr[device];
  return g_scratch_err[device];
}

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct sfem_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  void *scratch = nullptr;             // this device's `scratch` array (device address)
  hipError_t scratch_err = hipSuccess;  // outcome of resolving it

  // ---- mesh
  bool ready = false;
  int p = 0, q = 0;
  int64_t nelem = 0, ndof = 0;
  Rules1D rules;
  int32_t *d_map = nullptr;        // [nelem][n^3] flagged (sole / essential bits)
  double *d_xyz = nullptr;         // [nelem][8][3]
  double *d_qd = nullptr;          // [nelem][7][q^3]
  float *d_qd32 = nullptr;
  // assembly of the shared and essential DoFs
  int compact = 0;                 // E-vector over surface nodes only
  int64_t epe = 0;                 // E-vector entries per element (surface nodes or n^3)
  int64_t na = 0;                  // number of DoFs the assembly kernel writes
  int32_t *d_alist = nullptr;      // [na] those DoFs, ascending
  int32_t *d_aoff = nullptr;       // [na + 1] CSR offsets of their E-vector entries
  int32_t *d_pos = nullptr;        // DoF-ordered E-vector: [nelem][epe] entry of each node
  int32_t *d_slot = nullptr;       // element-ordered E-vector: entries of the contributions
  int64_t nentries = 0;            // E-vector entries per member
  int64_t n_ess = 0;               // essential DoFs
  // geometry-only vectors, computed on first use
  double *d_cm = nullptr;          // collocated mass diagonal (essential rows 1)
  double *d_cminv = nullptr;       // its inverse, FP64 and FP32
  float *d_cminv32 = nullptr;
  double *d_m1 = nullptr;          // M 1 (the integral of a DoF vector is m1^T x)
  double m1sum = 0.0;              // 1^T M 1 = |Omega| (no essential DoFs)
  AsmPlan plan{};                  // the three arrays above, for the assembly kernel
  // Taylor-Hood pressure space (order p - 1) and the Stokes coupling factors
  bool pres_ready = false;
  int64_t npres = 0;
  int32_t *d_pmap = nullptr;       // [nelem][p^3] flagged pressure map
  int pcompact = 0;
  int64_t pnentries = 0;           // pressure E-vector entries (element-ordered)
  AsmPlan pplan{};
  double *d_cq = nullptr;          // [nelem][9 q^3] coupling factors w |J| J^{-T}, slice-pair order

  // ---- coefficients
  double alpha = 1.0, beta = 1.0;
  int nfield = 1;
  bool has_nu = false;
  double *d_fold64 = nullptr;  // [nfield][nelem][7 q^3], slice-pair order (k_setup.hip: fold_kernel)
  float *d_fold32 = nullptr;
  double *d_nu64 = nullptr;    // [nfield][nelem][q^3]
  float *d_nu32 = nullptr;

  // ---- diagonals per operator kind: [nf][ndof]
  bool diag_ok[3] = {false, false, false};
  double *d_diag[3] = {nullptr, nullptr, nullptr};
  double *d_dinv[3] = {nullptr, nullptr, nullptr};
  float *d_diag32[3] = {nullptr, nullptr, nullptr};
  float *d_dinv32[3] = {nullptr, nullptr, nullptr};

  // ---- host copies of the mesh (the LOR assembly) and the LOR multigrid per operator kind
  std::vector<double> h_xyz;
  std::vector<int32_t> h_dofs;     // unflagged element->DoF map
  std::vector<uint8_t> h_ess;
  bool lor_ok[3] = {false, false, false};
  Amg lor[3];
  double *lor_work = nullptr;      // [5][ndof] vectors of the LOR-preconditioned CG
  double *lor_scal = nullptr;      // device scalars: [kLorScalarSlots] doubles, then 2 PcgScalars
  float *lor_work32 = nullptr;     // [2][ndof] FP32 residual and V-cycle output

  // ---- E-vector of the apply and solver workspace (grown on demand)
  DevBuf evec;
  DevBuf ws;
  void *h_pinned = nullptr;
  size_t h_pinned_bytes = 0;

  std::vector<DevBuf> owned;  // every device allocation of the mesh/coeff state
  int64_t bytes = 0;
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

sfem_status fail(sfem_ctx *c, sfem_status st, const std::string &msg) {
  if (c) c->err = msg;
  return st;
}

// Runs the body of an entry point whose host-side work allocates (mesh plan, LOR
// assembly and multigrid set-up): a failed host allocation becomes SFEM_E_NOMEM instead
// of an exception crossing the C boundary.
template <class F>
sfem_status guarded(sfem_ctx *c, F &&body) {
  try {
    return body();
  } catch (const std::bad_alloc &) {
    return fail(c, SFEM_E_NOMEM, "host allocation failed");
  } catch (const std::length_error &) {
    return fail(c, SFEM_E_NOMEM, "host allocation failed (size beyond the allocator's limit)");
  }
}

#define HIPCHK(c, expr)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail((c), SFEM_E_HIP, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
sfem_status dalloc(sfem_ctx *c, T **out, int64_t count) {
  *out = nullptr;
  if (count <= 0) return SFEM_OK;
  void *p = nullptr;
  const size_t bytes = (size_t)count * sizeof(T);
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, SFEM_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  c->owned.push_back({p, bytes});
  c->bytes += (int64_t)bytes;
  *out = (T *)p;
  return SFEM_OK;
}

void dfree(sfem_ctx *c, void *p) {
  if (!p) return;
  for (size_t i = 0; i < c->owned.size(); ++i) {
    if (c->owned[i].p == p) {
      c->bytes -= (int64_t)c->owned[i].bytes;
      (void)hipFree(p);
      c->owned.erase(c->owned.begin() + i);
      return;
    }
  }
}

void free_lor(sfem_ctx *c) {
  for (int o = 0; o < 3; ++o) {
    amg_free(c->lor[o]);
    c->lor_ok[o] = false;
  }
}

void free_coeffs(sfem_ctx *c) {
  free_lor(c);
  dfree(c, c->d_fold64);
  dfree(c, c->d_fold32);
  dfree(c, c->d_nu64);
  dfree(c, c->d_nu32);
  c->d_fold64 = nullptr;
  c->d_fold32 = nullptr;
  c->d_nu64 = nullptr;
  c->d_nu32 = nullptr;
  for (int o = 0; o < 3; ++o) {
    dfree(c, c->d_diag[o]);
    dfree(c, c->d_dinv[o]);
    dfree(c, c->d_diag32[o]);
    dfree(c, c->d_dinv32[o]);
    c->d_diag[o] = c->d_dinv[o] = nullptr;
    c->d_diag32[o] = c->d_dinv32[o] = nullptr;
    c->diag_ok[o] = false;
  }
}

void free_all(sfem_ctx *c) {
  free_lor(c);
  c->lor_work = nullptr;
  c->lor_scal = nullptr;
  c->lor_work32 = nullptr;
  for (auto &b : c->owned) (void)hipFree(b.p);
  c->owned.clear();
  c->bytes = 0;
  c->d_map = nullptr;
  c->d_xyz = nullptr;
  c->d_qd = nullptr;
  c->d_qd32 = nullptr;
  c->d_alist = nullptr;
  c->d_aoff = nullptr;
  c->d_pos = nullptr;
  c->d_slot = nullptr;
  c->nentries = 0;
  c->n_ess = 0;
  c->d_cm = c->d_cminv = c->d_m1 = nullptr;
  c->d_cminv32 = nullptr;
  c->m1sum = 0.0;
  c->plan = AsmPlan{};
  c->na = 0;
  c->pres_ready = false;
  c->npres = 0;
  c->d_pmap = nullptr;
  c->pcompact = 0;
  c->pnentries = 0;
  c->pplan = AsmPlan{};
  c->d_cq = nullptr;
  c->d_fold64 = nullptr;
  c->d_fold32 = nullptr;
  c->d_nu64 = nullptr;
  c->d_nu32 = nullptr;
  for (int o = 0; o < 3; ++o) {
    c->d_diag[o] = c->d_dinv[o] = nullptr;
    c->d_diag32[o] = c->d_dinv32[o] = nullptr;
    c->diag_ok[o] = false;
  }
  if (c->ws.p) (void)hipFree(c->ws.p);
  c->ws = DevBuf{};
  if (c->evec.p) (void)hipFree(c->evec.p);
  c->evec = DevBuf{};
  c->ready = false;
}

int64_t q3_of(const sfem_ctx *c) { return (int64_t)c->q * c->q * c->q; }

// Number of coefficient fields an operator kind uses.
int nfields_of(const sfem_ctx *c, int op) { return op == SFEM_MASS ? 1 : c->nfield; }

sfem_status fold_coeffs(sfem_ctx *c, const double *nu_user, int nfield, double alpha,
                        double beta) {
  free_coeffs(c);
  c->alpha = alpha;
  c->beta = beta;
  c->nfield = nfield;
  c->has_nu = nu_user != nullptr;
  const int64_t nq = c->nelem * q3_of(c);
  sfem_status st;
  if ((st = dalloc(c, &c->d_fold64, nq * kQdSlots * nfield)) != SFEM_OK) return st;
  if ((st = dalloc(c, &c->d_fold32, nq * kQdSlots * nfield)) != SFEM_OK) return st;
  if ((st = dalloc(c, &c->d_nu64, nq * nfield)) != SFEM_OK) return st;
  if ((st = dalloc(c, &c->d_nu32, nq * nfield)) != SFEM_OK) return st;
  HIPCHK(c, launch_fold(c->q, c->d_qd, nu_user, c->nelem, nfield, alpha, beta, c->d_fold64,
                        c->d_fold32, c->d_nu64, c->d_nu32, c->stream));
  return SFEM_OK;
}

sfem_status ensure_evec(sfem_ctx *c, size_t bytes) {
  if (c->evec.bytes >= bytes) return SFEM_OK;
  if (c->evec.p) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    (void)hipFree(c->evec.p);
    c->evec = DevBuf{};
  }
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, SFEM_E_NOMEM, "E-vector allocation of " + std::to_string(bytes) + " bytes failed");
  }
  c->evec.p = p;
  c->evec.bytes = bytes;
  return SFEM_OK;
}

// Compute (lazily) the diagonal of operator kind op for every field.
sfem_status ensure_diag(sfem_ctx *c, int op) {
  if (c->diag_ok[op]) return SFEM_OK;
  const int nf = nfields_of(c, op);
  const int64_t n = c->ndof * nf;
  sfem_status st;
  if (!c->d_diag[op]) {
    if ((st = dalloc(c, &c->d_diag[op], n)) != SFEM_OK) return st;
    if ((st = dalloc(c, &c->d_dinv[op], n)) != SFEM_OK) return st;
    if ((st = dalloc(c, &c->d_diag32[op], n)) != SFEM_OK) return st;
    if ((st = dalloc(c, &c->d_dinv32[op], n)) != SFEM_OK) return st;
  }
  if ((st = ensure_evec(c, (size_t)c->nentries * sizeof(double))) != SFEM_OK) return st;
  double a = 1.0, b = 0.0;
  if (op == SFEM_DIFFUSION) {
    a = 0.0;
    b = 1.0;
  } else if (op == SFEM_HELMHOLTZ) {
    a = c->alpha;
    b = c->beta;
  }
  for (int f = 0; f < nf; ++f) {
    DiagArgs da;
    da.p = c->p;
    da.map = c->d_map;
    da.qd = c->d_qd;
    da.nu = (op != SFEM_MASS && c->has_nu) ? c->d_nu64 + (int64_t)f * c->nelem * q3_of(c) : nullptr;
    da.alpha = a;
    da.beta = b;
    da.nelem = c->nelem;
    da.diag = c->d_diag[op] + (int64_t)f * c->ndof;
    da.evec = (double *)c->evec.p;
    da.pos = c->d_pos;
    da.compact = c->compact;
    HIPCHK(c, launch_diag(da, c->stream));
    HIPCHK(c, launch_assemble<double>(c->plan, (const double *)c->evec.p, 0, nullptr, da.diag, c->ndof,
                                      1, kEssOne, nullptr, 0, c->stream));
  }
  HIPCHK(c, VecOps<double>::recip(c->d_diag[op], c->d_dinv[op], n, c->stream));
  HIPCHK(c, VecOps<float>::recip(c->d_diag[op], c->d_dinv32[op], n, c->stream));
  HIPCHK(c, launch_cast_f32(c->d_diag[op], c->d_diag32[op], n, c->stream));
  c->diag_ok[op] = true;
  return SFEM_OK;
}

// Collocated mass diagonal and its inverses (geometry only; computed once per setup).
sfem_status ensure_cmass(sfem_ctx *c) {
  if (c->d_cm) return SFEM_OK;
  const int64_t n = c->ndof;
  sfem_status st;
  double *cm = nullptr, *cminv = nullptr;
  float *cminv32 = nullptr;
  if ((st = dalloc(c, &cm, n)) != SFEM_OK) return st;
  if ((st = dalloc(c, &cminv, n)) != SFEM_OK) return st;
  if ((st = dalloc(c, &cminv32, n)) != SFEM_OK) return st;
  if ((st = ensure_evec(c, (size_t)c->nentries * sizeof(double))) != SFEM_OK) return st;
  HIPCHK(c, launch_colloc_mass(c->p, c->rules.gll_x.data(), c->rules.gll_w.data(), c->d_xyz, c->d_map,
                               c->d_pos, c->compact, c->nelem, cm, (double *)c->evec.p, c->stream));
  HIPCHK(c, launch_assemble<double>(c->plan, (const double *)c->evec.p, 0, nullptr, cm, n, 1, kEssOne,
                                    nullptr, 0, c->stream));
  HIPCHK(c, VecOps<double>::recip(cm, cminv, n, c->stream));
  HIPCHK(c, VecOps<float>::recip(cm, cminv32, n, c->stream));
  c->d_cm = cm;
  c->d_cminv = cminv;
  c->d_cminv32 = cminv32;
  return SFEM_OK;
}

// (assemble = false: the element kernel only; y holds the sole DoFs and evec the shared
// nodes' contributions, for a caller that adds more before assembling)
sfem_status do_apply(sfem_ctx *c, int op, bool f32, int nbatch, const void *x, void *y,
                     double *part = nullptr, void *evec = nullptr, bool assemble = true);

// m1 = M 1 and 1^T M 1 (geometry only), for the mean-zero condition int x = m1^T x.
sfem_status ensure_m1(sfem_ctx *c, double *tmp_ones, double *tmp_part, double *tmp_out) {
  if (c->d_m1) return SFEM_OK;
  const int64_t n = c->ndof;
  sfem_status st;
  double *m1 = nullptr;
  if ((st = dalloc(c, &m1, n)) != SFEM_OK) return st;
  HIPCHK(c, VecOps<double>::fill(tmp_ones, 1.0, n, c->stream));
  if ((st = do_apply(c, SFEM_MASS, false, 1, tmp_ones, m1, nullptr)) != SFEM_OK) return st;
  const int nblk = vec_nblk(n);
  HIPCHK(c, VecOps<double>::dot(m1, nullptr, 0, tmp_part, nblk, n, 1, c->stream));
  HIPCHK(c, launch_reduce1(tmp_part, nblk, 1, tmp_out, c->stream));
  HIPCHK(c, hipMemcpyAsync(&c->m1sum, tmp_out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->d_m1 = m1;
  return SFEM_OK;
}

sfem_status check_op_batch(sfem_ctx *c, int op, int nbatch) {
  if (op < 0 || op > 2) return fail(c, SFEM_E_ARG, "op must be SFEM_MASS, SFEM_DIFFUSION or SFEM_HELMHOLTZ");
  if (nbatch < 0) return fail(c, SFEM_E_ARG, "nbatch must be >= 0");
  if (op != SFEM_MASS && c->nfield > 1 && nbatch != c->nfield && nbatch != 0)
    return fail(c, SFEM_E_ARG, "with " + std::to_string(c->nfield) +
                                   " nu fields, nbatch must equal the number of fields");
  return SFEM_OK;
}

// Per-block dot partials of one apply of nb members, per member: the element kernel's
// blocks (one per group of (element, member) pairs), then the assembly's (which fold the
// element partials in, so that the apply's sum is the sum of the assembly partials alone
// when there is an assembly phase).
int apply_nparts_elem(const sfem_ctx *c, bool f32, int nb) {
  const int e = f32 ? apply_group_elems_f32(c->p) : apply_group_elems_f64(c->p);
  return (int)((c->nelem * nb + e - 1) / e);
}
int apply_nparts(const sfem_ctx *c, bool f32, int nb) {
  return apply_nparts_elem(c, f32, nb) + (c->na > 0 ? assemble_nblk_dot(c->na) : 0);
}
// Offset and count of the partials that sum to the apply's x . y.
int apply_final_off(const sfem_ctx *c, bool f32, int nb) {
  return c->na > 0 ? apply_nparts_elem(c, f32, nb) : 0;
}
int apply_final_count(const sfem_ctx *c, bool f32, int nb) {
  return c->na > 0 ? assemble_nblk_dot(c->na) : apply_nparts_elem(c, f32, nb);
}

// Enqueue y = A x on the context stream (no argument checks).  With part != null the
// two launches also leave the per-block partial sums of x . y in part[m][0..nparts).
// evec: E-vector storage of at least nbatch * nentries values given by the caller, or
// null for the context's own (grown on demand).
sfem_status do_apply(sfem_ctx *c, int op, bool f32, int nbatch, const void *x, void *y,
                     double *part, void *evec, bool assemble) {
  if (nbatch == 0 || c->ndof == 0) return SFEM_OK;
  const int64_t estride = c->nentries;
  const size_t esz = f32 ? sizeof(float) : sizeof(double);
  sfem_status st;
  if (!evec) {
    if ((st = ensure_evec(c, (size_t)estride * nbatch * esz)) != SFEM_OK) return st;
    evec = c->evec.p;
  }
  const int nparts = apply_nparts(c, f32, nbatch);
  const int nblk_e = apply_nparts_elem(c, f32, nbatch);
  ApplyArgs a;
  a.p = c->p;
  a.op = op;
  a.map = c->d_map;
  a.ndof = c->ndof;
  a.nbatch = nbatch;
  a.nelem = c->nelem;
  a.x = x;
  a.y = y;
  a.evec = evec;
  a.estride = estride;
  a.pos = c->d_pos;
  a.compact = c->compact;
  a.part = part;
  a.part_mstride = nparts;
  a.nu = nullptr;
  a.qd_mstride = 0;
  a.nu_mstride = 0;
  const int64_t nq = c->nelem * q3_of(c);
  const bool per_member = c->nfield > 1;
  if (op == SFEM_HELMHOLTZ) {
    a.qd = f32 ? (const void *)c->d_fold32 : (const void *)c->d_fold64;
    a.qd_mstride = per_member ? nq * kQdSlots : 0;
  } else {
    a.qd = f32 ? (const void *)c->d_qd32 : (const void *)c->d_qd;
    if (op == SFEM_DIFFUSION) {  // nu = 1 is stored when no field was given
      a.nu = f32 ? (const void *)c->d_nu32 : (const void *)c->d_nu64;
      a.nu_mstride = per_member ? nq : 0;
    }
  }
  hipError_t e = f32 ? launch_apply_f32(a, c->stream) : launch_apply_f64(a, c->stream);
  if (e != hipSuccess) return fail(c, SFEM_E_HIP, std::string("apply launch: ") + hipGetErrorString(e));
  if (!assemble) return SFEM_OK;
  double *pa = part ? part + nblk_e : nullptr;
  if (f32)
    e = launch_assemble<float>(c->plan, (const float *)evec, estride, (const float *)x, (float *)y,
                               c->ndof, nbatch, kEssCopyX, pa, nparts, c->stream, part, nblk_e);
  else
    e = launch_assemble<double>(c->plan, (const double *)evec, estride, (const double *)x,
                                (double *)y, c->ndof, nbatch, kEssCopyX, pa, nparts, c->stream, part,
                                nblk_e);
  if (e != hipSuccess) return fail(c, SFEM_E_HIP, std::string("assembly launch: ") + hipGetErrorString(e));
  return SFEM_OK;
}

sfem_status ensure_ws(sfem_ctx *c, size_t bytes) {
  if (c->ws.bytes >= bytes) return SFEM_OK;
  if (c->ws.p) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    (void)hipFree(c->ws.p);
    c->ws = DevBuf{};
  }
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, SFEM_E_NOMEM, "solver workspace allocation of " + std::to_string(bytes) + " bytes failed");
  }
  c->ws.p = p;
  c->ws.bytes = bytes;
  return SFEM_OK;
}

sfem_status ensure_pinned(sfem_ctx *c, size_t bytes) {
  if (c->h_pinned_bytes >= bytes) return SFEM_OK;
  if (c->h_pinned) (void)hipHostFree(c->h_pinned);
  c->h_pinned = nullptr;
  c->h_pinned_bytes = 0;
  HIPCHK(c, hipHostMalloc(&c->h_pinned, bytes, hipHostMallocDefault));
  c->h_pinned_bytes = bytes;
  return SFEM_OK;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Carve a workspace into named pieces.
struct Carver {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(int64_t count) {
    T *p = (T *)(base + off);
    off = align_up(off + (size_t)count * sizeof(T));
    return p;
  }
};

template <typename T>
struct PcgWork {
  T *r, *p, *w;
  double *part;   // vector-kernel partials [nb][5][nblk]
  double *dpart;  // p^T A p partials of the apply [nb][nparts]
  PcgScalars *sc;  // [2][nb]: the current and the next iteration's scalars
  int nblk, nparts;
};

template <typename T>
size_t pcg_work_bytes(const sfem_ctx *c, int64_t n, int nb) {
  const int nblk = vec_nblk(n);
  return 3 * align_up((size_t)n * nb * sizeof(T)) + align_up((size_t)nb * 5 * nblk * sizeof(double)) +
         align_up((size_t)nb * apply_nparts(c, sizeof(T) == 4, nb) * sizeof(double)) +
         align_up((size_t)2 * nb * sizeof(PcgScalars));
}

template <typename T>
PcgWork<T> carve_pcg(const sfem_ctx *c, Carver &cv, int64_t n, int nb) {
  PcgWork<T> w;
  w.nblk = vec_nblk(n);
  w.nparts = apply_nparts(c, sizeof(T) == 4, nb);
  w.r = cv.take<T>(n * nb);
  w.p = cv.take<T>(n * nb);
  w.w = cv.take<T>(n * nb);
  w.part = cv.take<double>((int64_t)nb * 5 * w.nblk);
  w.dpart = cv.take<double>((int64_t)nb * w.nparts);
  w.sc = cv.take<PcgScalars>(2 * (int64_t)nb);
  return w;
}

// Jacobi-PCG on the context stream.  On return hs[] holds the final scalars.
template <typename T>
sfem_status run_pcg(sfem_ctx *c, int op, int nb, const T *b, T *x, bool x0_zero, double rtol,
                    int maxit, int check_every, const T *dinv, int64_t dms, PcgWork<T> &w,
                    PcgScalars *hs, int nullspace = 0) {
  const int64_t n = c->ndof;
  const bool f32 = sizeof(T) == 4;
  hipStream_t s = c->stream;
  sfem_status st;
  if (x0_zero) {
    HIPCHK(c, VecOps<T>::start(b, nullptr, x, w.r, dinv, dms, w.p, w.part, w.nblk, n, nb, s));
  } else {
    if ((st = do_apply(c, op, f32, nb, x, w.w)) != SFEM_OK) return st;
    HIPCHK(c, VecOps<T>::start(b, w.w, nullptr, w.r, dinv, dms, w.p, w.part, w.nblk, n, nb, s));
  }
  HIPCHK(c, launch_pcg_init(w.part, w.nblk, nb, rtol, w.sc, s, nullspace, n));
  if (nullspace) HIPCHK(c, launch_zshift<T>(w.p, w.sc, n, nb, s));
  int cur = 0;  // slot of the current scalars in w.sc
  auto all_done = [&]() -> sfem_status {
    HIPCHK(c, hipMemcpyAsync(hs, w.sc + (int64_t)cur * nb, sizeof(PcgScalars) * nb,
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return SFEM_OK;
  };
  if ((st = all_done()) != SFEM_OK) return st;
  for (int m = 0; m < nb; ++m)  // b = 0: the solution is x = 0
    if (hs[m].bb == 0.0 && !x0_zero) HIPCHK(c, VecOps<T>::fill(x + (int64_t)m * n, T(0), n, s));
  auto any_active = [&]() {
    for (int m = 0; m < nb; ++m)
      if (hs[m].active) return true;
    return false;
  };
  if (!any_active()) return SFEM_OK;
  for (int it = 0; it < maxit; ++it) {
    if ((st = do_apply(c, op, f32, nb, w.p, w.w, w.dpart)) != SFEM_OK) return st;
    const double *dp = w.dpart + apply_final_off(c, f32, nb);
    const int dcount = apply_final_count(c, f32, nb);
    PcgScalars *sc = w.sc + (int64_t)cur * nb, *sc_next = w.sc + (int64_t)(1 - cur) * nb;
    HIPCHK(c, VecOps<T>::update(x, w.p, w.r, w.w, dinv, dms, sc, dp, w.nparts, dcount, w.part,
                                w.nblk, n, nb, s));
    HIPCHK(c, VecOps<T>::newdir(w.r, dinv, dms, w.p, sc, sc_next, dp, w.nparts, dcount, w.part,
                                w.nblk, nullspace, n, nb, s));
    cur = 1 - cur;
    if ((it + 1) % check_every == 0 || it + 1 == maxit) {
      if ((st = all_done()) != SFEM_OK) return st;
      if (!any_active()) break;
    }
  }
  return SFEM_OK;
}

// ---- LOR preconditioner (Section 5.2) --------------------------------------------------

// Multigrid parameters: strength threshold, coarsest size, level cap, Jacobi sweeps.
constexpr double kLorTheta = 0.02;
constexpr int64_t kLorCoarse = 200;
constexpr int kLorMaxLevels = 12;
constexpr int kLorSweeps = 1;
// device scalar doubles of the LOR solves ahead of the CG scalars (the null-space mean)
constexpr int64_t kLorScalarSlots = 8;
static_assert(sizeof(PcgScalars) % sizeof(double) == 0, "PcgScalars packs into doubles");

// Build (once per operator kind and coefficients) A_LOR of op and its multigrid hierarchy.
sfem_status ensure_lor_f64(sfem_ctx *c, int op) {
  if (c->lor_ok[op]) return SFEM_OK;
  if (op != SFEM_MASS && c->nfield > 1)
    return fail(c, SFEM_E_ARG, "the LOR preconditioner takes one nu field");
  double a = 1.0, b = 0.0;
  if (op == SFEM_DIFFUSION) {
    a = 0.0;
    b = 1.0;
  } else if (op == SFEM_HELMHOLTZ) {
    a = c->alpha;
    b = c->beta;
  }
  // nu enters as its mean over each element's quadrature points
  std::vector<double> nu_e;
  if (op != SFEM_MASS && c->has_nu && c->nelem > 0) {
    const int64_t q3 = q3_of(c);
    std::vector<double> nu((size_t)(c->nelem * q3));
    HIPCHK(c, hipMemcpyAsync(nu.data(), c->d_nu64, nu.size() * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    nu_e.assign((size_t)c->nelem, 0.0);
    for (int64_t e = 0; e < c->nelem; ++e) {
      double sum = 0.0;
      for (int64_t k = 0; k < q3; ++k) sum += nu[(size_t)(e * q3 + k)];
      nu_e[(size_t)e] = sum / (double)q3;
    }
  }
  HostCsr A;
  lor_assemble(c->p, c->rules.gll_x.data(), c->nelem, c->h_xyz.data(), c->h_dofs.data(), c->ndof,
               c->h_ess.data(), a, b, nu_e.empty() ? nullptr : nu_e.data(), A);
  const std::string e = amg_setup(A, kLorTheta, kLorCoarse, kLorMaxLevels, kLorSweeps, c->lor[op]);
  if (!e.empty()) {
    amg_free(c->lor[op]);
    return fail(c, SFEM_E_NOMEM, e);
  }
  if (!c->lor_work) {
    sfem_status st;
    if ((st = dalloc(c, &c->lor_work, 5 * c->ndof)) != SFEM_OK) return st;
    if ((st = dalloc(c, &c->lor_scal, kLorScalarSlots + 2 * (int64_t)(sizeof(PcgScalars) / sizeof(double)))) != SFEM_OK) return st;
  }
  c->lor_ok[op] = true;
  return SFEM_OK;
}

// The hierarchy of op with (f32) its FP32 copy and FP32 work vectors.
sfem_status ensure_lor(sfem_ctx *c, int op, bool f32 = false) {
  sfem_status st;
  if ((st = ensure_lor_f64(c, op)) != SFEM_OK) return st;
  if (!f32) return SFEM_OK;
  const std::string e = amg_make_f32(c->lor[op], c->stream);
  if (!e.empty()) return fail(c, SFEM_E_NOMEM, e);
  if (!c->lor_work32 && (st = dalloc(c, &c->lor_work32, 2 * c->ndof)) != SFEM_OK) return st;
  return SFEM_OK;
}

// z = V-cycle(r) of op's hierarchy in FP64 or (f32) in FP32 arithmetic (r and z FP64).
hipError_t lor_vcycle(sfem_ctx *c, int op, bool f32, const double *r, double *z) {
  if (!f32) return amg_vcycle<double>(c->lor[op], r, z, c->stream);
  const int64_t n = c->ndof;
  float *r32 = c->lor_work32, *z32 = r32 + n;
  hipError_t e;
  if ((e = launch_convert<double, float>(r, r32, n, c->stream)) != hipSuccess) return e;
  if ((e = amg_vcycle<float>(c->lor[op], r32, z32, c->stream)) != hipSuccess) return e;
  return launch_convert<float, double>(z32, z, n, c->stream);
}

sfem_status lor_precond(sfem_ctx *c, int op, bool f32, const double *r, double *z, int nullspace,
                        double *part) {
  HIPCHK(c, lor_vcycle(c, op, f32, r, z));
  if (nullspace) {
    const int64_t n = c->ndof;
    const int nblk = vec_nblk(n);
    HIPCHK(c, VecOps<double>::dot(z, nullptr, 0, part, nblk, n, 1, c->stream));
    HIPCHK(c, launch_reduce1(part, nblk, 1, c->lor_scal, c->stream));
    HIPCHK(c, launch_shift(z, c->lor_scal, 1.0 / (double)n, n, 1, c->stream));
  }
  return SFEM_OK;
}

// CG for one member preconditioned by the LOR multigrid V-cycle.  The scalars stay on the
// device (step length, direction and stopping test formed by the kernels from partial
// sums); after each iteration they are copied to pinned host memory behind an event, and
// the host reads the previous iteration's copy once the next iteration is queued, so the
// GPU never waits for the host.  When that copy shows the solve stopped, the iteration
// queued after it changes nothing (alpha = 0 once inactive).  dpart: the apply's partials;
// part: [5][vec_nblk(n)] partials.  On return hs holds the final scalars.
sfem_status run_pcg_lor(sfem_ctx *c, int op, bool f32, const double *b, double *x, bool x0_zero,
                        double rtol, int maxit, int nullspace, double *dpart, double *part,
                        PcgScalars &hs) {
  const int64_t n = c->ndof;
  hipStream_t s = c->stream;
  double *r = c->lor_work, *z = r + n, *pv = z + n, *w = pv + n;
  PcgScalars *sc = reinterpret_cast<PcgScalars *>(c->lor_scal + kLorScalarSlots);  // [2]
  PcgScalars *h = reinterpret_cast<PcgScalars *>(c->h_pinned);                       // [2]
  const int nblk = vec_nblk(n);
  sfem_status st;
  hs = PcgScalars{};
  if (x0_zero) {
    HIPCHK(c, VecOps<double>::fill(x, 0.0, n, s));
    HIPCHK(c, hipMemcpyAsync(r, b, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    if ((st = do_apply(c, op, false, 1, x, w)) != SFEM_OK) return st;
    HIPCHK(c, launch_axpby(n, 1.0, b, -1.0, w, r, s));  // r = b - A x
  }
  if ((st = lor_precond(c, op, f32, r, z, nullspace, part)) != SFEM_OK) return st;
  HIPCHK(c, hipMemcpyAsync(pv, z, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(c, launch_gpcg_dots<double>(r, z, b, 0, part, nblk, n, s));
  HIPCHK(c, launch_pcg_init(part, nblk, 1, rtol, sc, s));
  HIPCHK(c, hipMemcpyAsync(h, sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  hs = h[0];
  if (hs.bb == 0.0) {  // b = 0: the solution is x = 0
    HIPCHK(c, VecOps<double>::fill(x, 0.0, n, s));
    return SFEM_OK;
  }
  if (!hs.active) return SFEM_OK;
  const double *dp = dpart + apply_final_off(c, false, 1);
  const int dcount = apply_final_count(c, false, 1);
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (hipEvent_t &e : ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      for (hipEvent_t &d : ev)
        if (d) (void)hipEventDestroy(d);
      return fail(c, SFEM_E_HIP, "LOR CG: event creation failed");
    }
  // in the loop the V-cycle's FP32 input comes from the update and its output is read by
  // the dots and the new direction as it is; the null-space shift is folded into those
  float *r32 = f32 ? c->lor_work32 : nullptr, *z32 = f32 ? c->lor_work32 + n : nullptr;
  auto body = [&]() -> sfem_status {
    int cur = 0, last = -1;
    for (int it = 0; it < maxit; ++it) {
      if ((st = do_apply(c, op, false, 1, pv, w, dpart)) != SFEM_OK) return st;
      HIPCHK(c, launch_gpcg_update(x, pv, r, w, r32, sc + cur, dp, dcount, n, s));
      if (f32) {
        HIPCHK(c, amg_vcycle<float>(c->lor[op], r32, z32, s));
        HIPCHK(c, launch_gpcg_dots<float>(r, z32, nullptr, nullspace, part, nblk, n, s));
        HIPCHK(c, launch_gpcg_newdir<float>(z32, pv, sc + cur, sc + 1 - cur, dp, dcount, part, nblk, nullspace,
                                            n, s));
      } else {
        HIPCHK(c, amg_vcycle<double>(c->lor[op], r, z, s));
        HIPCHK(c, launch_gpcg_dots<double>(r, z, nullptr, nullspace, part, nblk, n, s));
        HIPCHK(c, launch_gpcg_newdir<double>(z, pv, sc + cur, sc + 1 - cur, dp, dcount, part, nblk, nullspace,
                                             n, s));
      }
      cur = 1 - cur;
      HIPCHK(c, hipMemcpyAsync(h + (it & 1), sc + cur, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipEventRecord(ev[it & 1], s));
      last = it;
      if (it > 0) {
        HIPCHK(c, hipEventSynchronize(ev[(it - 1) & 1]));
        if (!h[(it - 1) & 1].active) break;
      }
    }
    HIPCHK(c, hipEventSynchronize(ev[last & 1]));
    hs = h[last & 1];
    return SFEM_OK;
  };
  st = body();
  for (hipEvent_t &e : ev) (void)hipEventDestroy(e);
  return st;
}

sfem_status require_ready(sfem_ctx *c) {
  if (!c) return SFEM_E_ARG;
  if (!c->ready) return fail(c, SFEM_E_STATE, "sfem_setup has not succeeded on this context");
  return SFEM_OK;
}

}  // namespace

// ===================================================================================
extern "C" {

int sfem_abi_version(void) { return SFEM_ABI_VERSION; }

sfem_status sfem_create(int device, void *stream, sfem_ctx **out) {
  if (!out) {
    g_create_error = "out must not be NULL";
    return SFEM_E_ARG;
  }
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    g_create_error = "no HIP device available";
    return SFEM_E_HIP;
  }
  if (device < 0 || device >= ndev) {
    g_create_error = "device index out of range";
    return SFEM_E_ARG;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    g_create_error = "hipGetDeviceProperties failed";
    return SFEM_E_HIP;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_create_error = std::string("device is ") + prop.gcnArchName + ", the library is built for gfx950";
    return SFEM_E_UNSUPPORTED;
  }
  sfem_ctx *c = new (std::nothrow) sfem_ctx();
  if (!c) {
    g_create_error = "host allocation failed";
    return SFEM_E_NOMEM;
  }
  c->device = device;
  c->stream = (hipStream_t)stream;
  {
    DeviceGuard g(device);
    c->scratch_err = resolve_scratch(device, &c->scratch);
  }
  *out = c;
  return SFEM_OK;
}

void sfem_destroy(sfem_ctx *c) {
  if (!c) return;
  {
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
  }
  delete c;
}

sfem_status sfem_set_stream(sfem_ctx *c, void *stream) {
  if (!c) return SFEM_E_ARG;
  c->stream = (hipStream_t)stream;
  return SFEM_OK;
}

const char *sfem_last_error(const sfem_ctx *c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

static sfem_status sfem_setup_body(sfem_ctx *c, int p, int q, int64_t nelem, const double *elem_xyz,
                       const int32_t *elem_dofs, int64_t ndof, const uint8_t *ess_mask) {
  if (!c) return SFEM_E_ARG;
  DeviceGuard g(c->device);
  if (p < 1 || p > SFEM_MAX_P || q != p + 2)
    return fail(c, SFEM_E_UNSUPPORTED, "supported orders: p = 1..8 with q = p + 2");
  if (nelem < 0 || ndof < 0 || ndof > kDofMask)
    return fail(c, SFEM_E_ARG, "nelem must be >= 0 and 0 <= ndof < 2^30");
  if (nelem > 0 && (!elem_xyz || !elem_dofs))
    return fail(c, SFEM_E_ARG, "elem_xyz and elem_dofs must not be NULL");
  if (nelem == 0 && ndof > 0)
    return fail(c, SFEM_E_MESH, "DoFs without elements: every DoF must belong to an element");
  const int n = p + 1;
  const int64_t n3 = (int64_t)n * n * n;
  if (nelem > (int64_t)INT32_MAX / 8 || nelem * n3 >= (int64_t)INT32_MAX)
    return fail(c, SFEM_E_ARG, "mesh too large");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  free_all(c);

  // ---- host copies
  std::vector<double> xyz((size_t)nelem * 24);
  std::vector<int32_t> dofs((size_t)(nelem * n3));
  std::vector<uint8_t> ess((size_t)ndof, 0);
  if (nelem > 0) {
    HIPCHK(c, hipMemcpyAsync(xyz.data(), elem_xyz, xyz.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(dofs.data(), elem_dofs, dofs.size() * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  }
  if (ess_mask && ndof > 0)
    HIPCHK(c, hipMemcpyAsync(ess.data(), ess_mask, (size_t)ndof, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));

  // ---- validate the map, encode it, and build the assembly plan (host)
  HostPlan hp;
  {
    std::string err;
    // E-vector layout: DoF-ordered up to p = 4, element-ordered above (at high order the
    // scattered entry writes cost the element kernel more than the assembly saves)
    const int rc = build_host_plan(p, nelem, dofs.data(), ndof, ess.data(), hp, err, evec_dof_ordered(p));
    if (rc != 0) return fail(c, (sfem_status)rc, err);
  }
  const bool compact = hp.compact;
  const int64_t epe = hp.epe;
  const int64_t na = hp.na;
  const std::vector<int32_t> &imap = hp.imap;
  const std::vector<int32_t> &alist = hp.alist;
  const std::vector<int32_t> &aoff = hp.aoff;
  const std::vector<int32_t> &pos = hp.pos;
  const std::vector<int32_t> &slots = hp.slots;
  if (hp.nentries >= (int64_t)kDofMask) return fail(c, SFEM_E_ARG, "mesh too large");

  // ---- rules
  if (!make_rules(p, q, c->rules)) return fail(c, SFEM_E_HIP, "1D rule construction failed");
  c->h_xyz = xyz;
  c->h_dofs = dofs;
  c->h_ess = ess;
  c->p = p;
  c->q = q;
  c->nelem = nelem;
  c->ndof = ndof;
  c->compact = compact ? 1 : 0;
  c->epe = epe;
  c->na = na;

  // ---- upload + geometric factors
  sfem_status st;
  const int64_t q3 = (int64_t)q * q * q;
  if ((st = dalloc(c, &c->d_map, nelem * n3)) != SFEM_OK) return st;
  if ((st = dalloc(c, &c->d_xyz, nelem * 24)) != SFEM_OK) return st;
  if ((st = dalloc(c, &c->d_qd, nelem * q3 * kQdSlots)) != SFEM_OK) return st;
  if ((st = dalloc(c, &c->d_qd32, nelem * q3 * kQdSlots)) != SFEM_OK) return st;
  if ((st = dalloc(c, &c->d_alist, na)) != SFEM_OK) return st;
  if ((st = dalloc(c, &c->d_aoff, na + 1)) != SFEM_OK) return st;
  if ((st = dalloc(c, &c->d_pos, (int64_t)pos.size())) != SFEM_OK) return st;
  if ((st = dalloc(c, &c->d_slot, (int64_t)slots.size())) != SFEM_OK) return st;
  int *d_bad = nullptr;
  if ((st = dalloc(c, &d_bad, 1)) != SFEM_OK) return st;
  if (na > 0) {
    HIPCHK(c, hipMemcpyAsync(c->d_alist, alist.data(), alist.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_aoff, aoff.data(), aoff.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  }
  if (!pos.empty())
    HIPCHK(c, hipMemcpyAsync(c->d_pos, pos.data(), pos.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  if (!slots.empty())
    HIPCHK(c, hipMemcpyAsync(c->d_slot, slots.data(), slots.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  c->plan.alist = c->d_alist;
  c->plan.aoff = c->d_aoff;
  c->plan.slot = c->d_slot;
  c->nentries = hp.nentries;
  c->n_ess = 0;
  for (int64_t gd = 0; gd < ndof; ++gd) c->n_ess += ess[(size_t)gd] ? 1 : 0;
  c->plan.na = na;
  if (nelem > 0) {
    HIPCHK(c, hipMemcpyAsync(c->d_map, imap.data(), imap.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_xyz, xyz.data(), xyz.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  }
  int h_bad = 0;
  if (d_bad) {
    HIPCHK(c, VecOps<float>::fill((float *)d_bad, 0.0f, 1, c->stream));
    HIPCHK(c, launch_qdata_setup(q, c->rules.gauss_x.data(), c->rules.gauss_w.data(), c->d_xyz,
                                 nelem, c->d_qd, d_bad, c->stream));
    HIPCHK(c, launch_cast_f32(c->d_qd, c->d_qd32, nelem * q3 * kQdSlots, c->stream));
    HIPCHK(c, hipMemcpyAsync(&h_bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  dfree(c, d_bad);
  if (h_bad) {
    free_all(c);
    return fail(c, SFEM_E_MESH, "det J <= 0 (or not finite) at some quadrature point: inverted or degenerate element");
  }
  if ((st = fold_coeffs(c, nullptr, 1, 1.0, 1.0)) != SFEM_OK) return st;
  c->ready = true;
  return SFEM_OK;
}

sfem_status sfem_setup(sfem_ctx *c, int p, int q, int64_t nelem, const double *elem_xyz,
                       const int32_t *elem_dofs, int64_t ndof, const uint8_t *ess_mask) {
  if (!c) return SFEM_E_ARG;
  return guarded(c, [&] { return sfem_setup_body(c, p, q, nelem, elem_xyz, elem_dofs, ndof, ess_mask); });
}

sfem_status sfem_qpoint_coords(sfem_ctx *c, double *xq) {
  sfem_status st = require_ready(c);
  if (st != SFEM_OK) return st;
  if (c->nelem > 0 && !xq) return fail(c, SFEM_E_ARG, "xq must not be NULL");
  DeviceGuard g(c->device);
  HIPCHK(c, launch_qpoint_coords(c->q, c->rules.gauss_x.data(), c->rules.gauss_w.data(), c->d_xyz,
                                 c->nelem, xq, c->stream));
  return SFEM_OK;
}

static sfem_status sfem_set_coeffs_body(sfem_ctx *c, double alpha, double beta, const double *nu_q, int nbatch_nu) {
  sfem_status st = require_ready(c);
  if (st != SFEM_OK) return st;
  if (nbatch_nu < 1) return fail(c, SFEM_E_ARG, "nbatch_nu must be >= 1");
  if (!nu_q && nbatch_nu != 1) return fail(c, SFEM_E_ARG, "nbatch_nu must be 1 when nu_q is NULL");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(c, SFEM_E_ARG, "alpha and beta must be finite");
  DeviceGuard g(c->device);
  return fold_coeffs(c, nu_q, nbatch_nu, alpha, beta);
}

sfem_status sfem_set_coeffs(sfem_ctx *c, double alpha, double beta, const double *nu_q, int nbatch_nu) {
  if (!c) return SFEM_E_ARG;
  return guarded(c, [&] { return sfem_set_coeffs_body(c, alpha, beta, nu_q, nbatch_nu); });
}

sfem_status sfem_apply(sfem_ctx *c, int op, int prec, int nbatch, const void *x, void *y) {
  sfem_status st = require_ready(c);
  if (st != SFEM_OK) return st;
  if ((st = check_op_batch(c, op, nbatch)) != SFEM_OK) return st;
  if (prec != SFEM_F64 && prec != SFEM_F32) return fail(c, SFEM_E_ARG, "prec must be SFEM_F64 or SFEM_F32");
  if (nbatch > 0 && c->ndof > 0) {
    if (!x || !y) return fail(c, SFEM_E_ARG, "x and y must not be NULL");
    if (x == y) return fail(c, SFEM_E_ARG, "x and y must not alias");
  }
  DeviceGuard g(c->device);
  return do_apply(c, op, prec == SFEM_F32, nbatch, x, y);
}

sfem_status sfem_apply_noalloc(sfem_ctx *c, int op, int prec, int nbatch, const void *x, void *y) {
  sfem_status st = require_ready(c);
  if (st != SFEM_OK) return st;
  if ((st = check_op_batch(c, op, nbatch)) != SFEM_OK) return st;
  if (prec != SFEM_F64 && prec != SFEM_F32) return fail(c, SFEM_E_ARG, "prec must be SFEM_F64 or SFEM_F32");
  if (nbatch == 0 || c->ndof == 0) return SFEM_OK;
  if (!x || !y) return fail(c, SFEM_E_ARG, "x and y must not be NULL");
  if (x == y) return fail(c, SFEM_E_ARG, "x and y must not alias");
  const size_t esz = prec == SFEM_F32 ? sizeof(float) : sizeof(double);
  const double need = (double)c->nentries * (double)nbatch * (double)esz;
  if (need > (double)SFEM_APPLY_NOALLOC_MAX_BYTES)
    return fail(c, SFEM_E_ARG,
                "sfem_apply_noalloc: the E-vector of this apply needs " + std::to_string((int64_t)need) +
                    " bytes, more than the " + std::to_string((int64_t)SFEM_APPLY_NOALLOC_MAX_BYTES) +
                    "-byte scratch (use sfem_apply or fewer members)");
  if (c->scratch_err != hipSuccess || !c->scratch)
    return fail(c, SFEM_E_HIP, std::string("scratch address of this device: ") +
                                   hipGetErrorString(c->scratch_err));
  DeviceGuard g(c->device);
  return do_apply(c, op, prec == SFEM_F32, nbatch, x, y, nullptr, c->scratch);
}

static sfem_status sfem_lor_setup_body(sfem_ctx *c, int op, sfem_lor_info *info) {
  sfem_status st = require_ready(c);
  if (st != SFEM_OK) return st;
  if ((st = check_op_batch(c, op, 0)) != SFEM_OK) return st;
  DeviceGuard g(c->device);
  if ((st = ensure_lor(c, op)) != SFEM_OK) return st;
  if (info) {
    const Amg &a = c->lor[op];
    *info = sfem_lor_info{};
    info->levels = (int)a.rows.size();
    for (int l = 0; l < info->levels && l < SFEM_LOR_MAX_LEVELS; ++l) {
      info->rows[l] = a.rows[(size_t)l];
      info->nnz[l] = a.nnzs[(size_t)l];
      info->sliced[l] = a.sliced[(size_t)l];
    }
    info->setup_ms = a.setup_ms;
  }
  return SFEM_OK;
}

sfem_status sfem_lor_setup(sfem_ctx *c, int op, sfem_lor_info *info) {
  if (!c) return SFEM_E_ARG;
  return guarded(c, [&] { return sfem_lor_setup_body(c, op, info); });
}

static sfem_status sfem_lor_apply_body(sfem_ctx *c, int op, const double *x, double *y) {
  sfem_status st = require_ready(c);
  if (st != SFEM_OK) return st;
  if ((st = check_op_batch(c, op, 0)) != SFEM_OK) return st;
  if (c->ndof == 0) return SFEM_OK;
  if (!x || !y || x == y) return fail(c, SFEM_E_ARG, "x and y must be distinct non-NULL arrays");
  DeviceGuard g(c->device);
  if ((st = ensure_lor(c, op)) != SFEM_OK) return st;
  HIPCHK(c, amg_apply_fine(c->lor[op], x, y, c->stream));
  return SFEM_OK;
}

sfem_status sfem_lor_apply(sfem_ctx *c, int op, const double *x, double *y) {
  if (!c) return SFEM_E_ARG;
  return guarded(c, [&] { return sfem_lor_apply_body(c, op, x, y); });
}

static sfem_status sfem_lor_vcycle_body(sfem_ctx *c, int op, int prec, const double *b, double *x) {
  sfem_status st = require_ready(c);
  if (st != SFEM_OK) return st;
  if ((st = check_op_batch(c, op, 0)) != SFEM_OK) return st;
  if (prec != SFEM_F64 && prec != SFEM_F32) return fail(c, SFEM_E_ARG, "prec must be SFEM_F64 or SFEM_F32");
  if (c->ndof == 0) return SFEM_OK;
  if (!b || !x || b == x) return fail(c, SFEM_E_ARG, "b and x must be distinct non-NULL arrays");
  DeviceGuard g(c->device);
  const bool f32 = prec == SFEM_F32;
  if ((st = ensure_lor(c, op, f32)) != SFEM_OK) return st;
  HIPCHK(c, lor_vcycle(c, op, f32, b, x));
  return SFEM_OK;
}

sfem_status sfem_lor_vcycle(sfem_ctx *c, int op, int prec, const double *b, double *x) {
  if (!c) return SFEM_E_ARG;
  return guarded(c, [&] { return sfem_lor_vcycle_body(c, op, prec, b, x); });
}

sfem_status sfem_diagonal(sfem_ctx *c, int op, int prec, void *diag) {
  sfem_status st = require_ready(c);
  if (st != SFEM_OK) return st;
  if ((st = check_op_batch(c, op, 0)) != SFEM_OK) return st;
  if (prec != SFEM_F64 && prec != SFEM_F32) return fail(c, SFEM_E_ARG, "prec must be SFEM_F64 or SFEM_F32");
  if (c->ndof > 0 && !diag) return fail(c, SFEM_E_ARG, "diag must not be NULL");
  DeviceGuard g(c->device);
  if ((st = ensure_diag(c, op)) != SFEM_OK) return st;
  const int64_t n = c->ndof * nfields_of(c, op);
  if (n == 0) return SFEM_OK;
  if (prec == SFEM_F64)
    HIPCHK(c, hipMemcpyAsync(diag, c->d_diag[op], n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  else
    HIPCHK(c, hipMemcpyAsync(diag, c->d_diag32[op], n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  return SFEM_OK;
}

sfem_status sfem_load(sfem_ctx *c, int nbatch, const double *f_q, double *b) {
  sfem_status st = require_ready(c);
  if (st != SFEM_OK) return st;
  if (nbatch < 0) return fail(c, SFEM_E_ARG, "nbatch must be >= 0");
  if (nbatch == 0 || c->ndof == 0) return SFEM_OK;
  if (!f_q || !b) return fail(c, SFEM_E_ARG, "f_q and b must not be NULL");
  DeviceGuard g(c->device);
  const int64_t estride = c->nentries;
  if ((st = ensure_evec(c, (size_t)estride * nbatch * sizeof(double))) != SFEM_OK) return st;
  LoadArgs a;
  a.p = c->p;
  a.map = c->d_map;
  a.qd = c->d_qd;
  a.ndof = c->ndof;
  a.nei = c->nelem;
  a.nbatch = nbatch;
  a.f = f_q;
  a.b = b;
  a.evec = (double *)c->evec.p;
  a.estride = estride;
  a.pos = c->d_pos;
  a.compact = c->compact;
  HIPCHK(c, launch_load(a, c->stream));
  HIPCHK(c, launch_assemble<double>(c->plan, (const double *)c->evec.p, estride, nullptr, b, c->ndof,
                                    nbatch, kEssZero, nullptr, 0, c->stream));
  return SFEM_OK;
}

sfem_status sfem_collocated_mass(sfem_ctx *c, double *diag) {
  sfem_status st = require_ready(c);
  if (st != SFEM_OK) return st;
  if (c->ndof == 0) return SFEM_OK;
  if (!diag) return fail(c, SFEM_E_ARG, "diag must not be NULL");
  DeviceGuard g(c->device);
  if ((st = ensure_cmass(c)) != SFEM_OK) return st;
  HIPCHK(c, hipMemcpyAsync(diag, c->d_cm, (size_t)c->ndof * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
  return SFEM_OK;
}

sfem_status sfem_grad_nu(sfem_ctx *c, int nbatch, const double *u, const double *lam, double *gq) {
  sfem_status st = require_ready(c);
  if (st != SFEM_OK) return st;
  if (nbatch < 0) return fail(c, SFEM_E_ARG, "nbatch must be >= 0");
  if (nbatch == 0 || c->nelem == 0) return SFEM_OK;
  if (!u || !lam || !gq) return fail(c, SFEM_E_ARG, "u, lam and g must not be NULL");
  DeviceGuard g(c->device);
  GradArgs a;
  a.p = c->p;
  a.map = c->d_map;
  a.qd = c->d_qd;
  a.beta = c->beta;
  a.ndof = c->ndof;
  a.nei = c->nelem;
  a.nbatch = nbatch;
  a.u = u;
  a.lam = lam;
  a.g = gq;
  HIPCHK(c, launch_grad(a, c->stream));
  return SFEM_OK;
}

static sfem_status sfem_pcg_body(sfem_ctx *c, int op, int nbatch, const double *b, double *x,
                     const sfem_pcg_opts *opts, sfem_pcg_info *info) {
  sfem_status st = require_ready(c);
  if (st != SFEM_OK) return st;
  if ((st = check_op_batch(c, op, nbatch)) != SFEM_OK) return st;
  if (!opts) return fail(c, SFEM_E_ARG, "opts must not be NULL");
  if (!(opts->rtol >= 0.0) || opts->maxit < 0 || opts->check_every < 1 ||
      (opts->mode != 0 && opts->mode != 1))
    return fail(c, SFEM_E_ARG, "invalid options (rtol >= 0, maxit >= 0, check_every >= 1, mode 0/1)");
  if (opts->mode == 1 && (!(opts->inner_rtol > 0.0) || opts->max_outer < 1))
    return fail(c, SFEM_E_ARG, "mode 1 needs inner_rtol > 0 and max_outer >= 1");
  if (opts->precond != SFEM_PRECOND_JACOBI && opts->precond != SFEM_PRECOND_COLLOCATED_MASS &&
      opts->precond != SFEM_PRECOND_LOR && opts->precond != SFEM_PRECOND_LOR32)
    return fail(c, SFEM_E_ARG,
                "precond must be SFEM_PRECOND_JACOBI, SFEM_PRECOND_COLLOCATED_MASS, SFEM_PRECOND_LOR or "
                "SFEM_PRECOND_LOR32");
  const bool lor = opts->precond == SFEM_PRECOND_LOR || opts->precond == SFEM_PRECOND_LOR32;
  const bool lor32 = opts->precond == SFEM_PRECOND_LOR32;
  if (lor && opts->mode != 0)
    return fail(c, SFEM_E_ARG, "the LOR preconditioner runs with FP64 CG (mode 0)");
  const int ns = opts->nullspace ? 1 : 0;
  if (ns && (op != SFEM_DIFFUSION || c->n_ess != 0))
    return fail(c, SFEM_E_ARG, "nullspace solves need op = SFEM_DIFFUSION and no essential DoFs");
  const int nb = nbatch;
  const int64_t n = c->ndof;
  if (nb == 0) return SFEM_OK;
  if (n == 0) {
    if (info)
      for (int m = 0; m < nb; ++m) info[m] = sfem_pcg_info{0, 0, 0.0, 0.0, SFEM_OK};
    return SFEM_OK;
  }
  if (!b || !x) return fail(c, SFEM_E_ARG, "b and x must not be NULL");
  if ((const void *)b == (const void *)x) return fail(c, SFEM_E_ARG, "b and x must not alias");
  DeviceGuard g(c->device);
  const bool cmass = opts->precond == SFEM_PRECOND_COLLOCATED_MASS;
  if (lor) {
    if ((st = ensure_lor(c, op, lor32)) != SFEM_OK) return st;
  }
  if ((st = cmass ? ensure_cmass(c) : ensure_diag(c, op)) != SFEM_OK) return st;
  const int64_t dms = (!cmass && nfields_of(c, op) > 1) ? n : 0;
  const double *dinv64 = cmass ? c->d_cminv : c->d_dinv[op];
  const float *dinv32 = cmass ? c->d_cminv32 : c->d_dinv32[op];
  hipStream_t s = c->stream;
  const int nblk = vec_nblk(n);
  std::vector<int> iters(nb, 0), status(nb, 0);
  std::vector<double> rel(nb, 0.0), trel(nb, 0.0);
  int outer = 0;

  if (opts->mode == 0) {
    const size_t bytes = pcg_work_bytes<double>(c, n, nb) + align_up((size_t)nb * sizeof(double)) +
                         (ns ? align_up((size_t)n * nb * sizeof(double)) : 0);
    if ((st = ensure_ws(c, bytes)) != SFEM_OK) return st;
    // (the LOR CG keeps two scalar copies in flight)
    if ((st = ensure_pinned(c, std::max(sizeof(PcgScalars), sizeof(double)) * std::max(nb, 2))) != SFEM_OK)
      return st;
    Carver cv{(char *)c->ws.p};
    PcgWork<double> w = carve_pcg<double>(c, cv, n, nb);
    double *d_out = cv.take<double>(nb);
    const double *bs = b;  // the right-hand side actually solved for
    if (ns) {
      // the pure-Neumann right-hand side is made orthogonal to the constants: b - mean(b) 1
      double *bc = cv.take<double>(n * nb);
      if ((st = ensure_m1(c, w.r, w.part, d_out)) != SFEM_OK) return st;
      HIPCHK(c, VecOps<double>::dot(b, nullptr, 0, w.part, nblk, n, nb, s));
      HIPCHK(c, launch_reduce1(w.part, nblk, nb, d_out, s));
      HIPCHK(c, hipMemcpyAsync(bc, b, (size_t)n * nb * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(c, launch_shift(bc, d_out, 1.0 / (double)n, n, nb, s));
      bs = bc;
    }
    PcgScalars *hs = (PcgScalars *)c->h_pinned;
    std::vector<PcgScalars> fin(nb);
    if (lor) {
      // members one after another, each preconditioned by the LOR multigrid V-cycle
      for (int m = 0; m < nb; ++m)
        if ((st = run_pcg_lor(c, op, lor32, bs + (int64_t)m * n, x + (int64_t)m * n,
                              opts->x0_zero != 0, opts->rtol, opts->maxit, ns, w.dpart, w.part,
                              fin[m])) != SFEM_OK)
          return st;
    } else {
      if ((st = run_pcg<double>(c, op, nb, bs, x, opts->x0_zero != 0, opts->rtol, opts->maxit,
                                opts->check_every, dinv64, dms, w, hs, ns)) != SFEM_OK)
        return st;
      fin.assign(hs, hs + nb);
    }
    if (ns) {
      // mean-zero condition: x <- x - (m1^T x / 1^T m1) 1
      HIPCHK(c, VecOps<double>::dot(x, c->d_m1, 0, w.part, nblk, n, nb, s));
      HIPCHK(c, launch_reduce1(w.part, nblk, nb, d_out, s));
      HIPCHK(c, launch_shift(x, d_out, 1.0 / c->m1sum, n, nb, s));
    }
    // true residual ||b - A x|| in FP64
    if ((st = do_apply(c, op, false, nb, x, w.w)) != SFEM_OK) return st;
    HIPCHK(c, launch_sub_norm(bs, w.w, nullptr, w.part, nblk, n, nb, s));
    HIPCHK(c, launch_reduce1(w.part, nblk, nb, d_out, s));
    std::vector<double> tr(nb);
    HIPCHK(c, hipMemcpyAsync(tr.data(), d_out, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int m = 0; m < nb; ++m) {
      iters[m] = fin[m].iters;
      const double bb = fin[m].bb;
      rel[m] = bb > 0 ? std::sqrt(fin[m].rr / bb) : 0.0;
      trel[m] = bb > 0 ? std::sqrt(tr[m] / bb) : 0.0;
      status[m] = fin[m].status;
      if (status[m] == 0 && fin[m].active) status[m] = SFEM_NOCONV;
    }
  } else {
    // FP64 iterative refinement around an FP32 Jacobi-PCG
    const size_t bytes = pcg_work_bytes<float>(c, n, nb) + 2 * align_up((size_t)n * nb * sizeof(double)) +
                         2 * align_up((size_t)n * nb * sizeof(float)) +
                         align_up((size_t)nb * 3 * sizeof(double)) +
                         align_up((size_t)nb * nblk * sizeof(double)) +
                         (ns ? align_up((size_t)n * nb * sizeof(double)) : 0);
    if ((st = ensure_ws(c, bytes)) != SFEM_OK) return st;
    if ((st = ensure_pinned(c, std::max(sizeof(PcgScalars), 3 * sizeof(double)) * nb)) != SFEM_OK) return st;
    Carver cv{(char *)c->ws.p};
    PcgWork<float> w = carve_pcg<float>(c, cv, n, nb);
    double *r64 = cv.take<double>(n * nb);
    double *w64 = cv.take<double>(n * nb);
    float *r32 = cv.take<float>(n * nb);
    float *d32 = cv.take<float>(n * nb);
    double *ir = cv.take<double>((int64_t)nb * 3);
    double *part = cv.take<double>((int64_t)nb * nblk);
    std::vector<double> hir(3 * nb);
    std::vector<int> conv(nb, 0);
    int total_inner = 0;
    const double *bs = b;  // the right-hand side actually solved for
    if (ns) {
      // pure Neumann: b - mean(b) 1 as in mode 0; the inner solves orthogonalize their
      // preconditioner against the constants, the mean-zero shift comes at the end
      double *bc = cv.take<double>(n * nb);
      if ((st = ensure_m1(c, r64, part, ir)) != SFEM_OK) return st;
      HIPCHK(c, VecOps<double>::dot(b, nullptr, 0, part, nblk, n, nb, s));
      HIPCHK(c, launch_reduce1(part, nblk, nb, ir, s));
      HIPCHK(c, hipMemcpyAsync(bc, b, (size_t)n * nb * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(c, launch_shift(bc, ir, 1.0 / (double)n, n, nb, s));
      bs = bc;
    }
    // ||b||^2
    HIPCHK(c, launch_sub_norm(bs, nullptr, nullptr, part, nblk, n, nb, s));
    HIPCHK(c, launch_ir_norm(part, nblk, nb, 1, opts->rtol, ir, s));
    if (opts->x0_zero) HIPCHK(c, VecOps<double>::fill(x, 0.0, n * nb, s));
    for (;;) {
      // outer residual in FP64 with the FP64 operator
      if ((st = do_apply(c, op, false, nb, x, w64)) != SFEM_OK) return st;
      HIPCHK(c, launch_sub_norm(bs, w64, r64, part, nblk, n, nb, s));
      HIPCHK(c, launch_ir_norm(part, nblk, nb, 0, opts->rtol, ir, s));
      HIPCHK(c, hipMemcpyAsync(hir.data(), ir, 3 * nb * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      bool all = true;
      for (int m = 0; m < nb; ++m) {
        const double rn2 = hir[3 * m], bb = hir[3 * m + 1];
        if (!std::isfinite(rn2) || !std::isfinite(bb)) {
          status[m] = SFEM_E_NAN;
          conv[m] = 1;
        }
        rel[m] = trel[m] = bb > 0 ? std::sqrt(rn2 / bb) : 0.0;
        if (!conv[m] && hir[3 * m + 2] == 0.0) conv[m] = 1;
        all = all && conv[m];
      }
      if (all || outer >= opts->max_outer || total_inner >= opts->maxit) break;
      if (ns) {
        // keep the inner right-hand side orthogonal to the constants (w64 is free here)
        HIPCHK(c, VecOps<double>::dot(r64, nullptr, 0, part, nblk, n, nb, s));
        HIPCHK(c, launch_reduce1(part, nblk, nb, w64, s));
        HIPCHK(c, launch_shift(r64, w64, 1.0 / (double)n, n, nb, s));
      }
      HIPCHK(c, launch_ir_cast(r64, ir, r32, n, nb, s));
      // Inner tolerance: a refinement step reduces the residual by the inner solve's
      // tolerance, normally inner_rtol; once the reduction still needed to reach rtol,
      // need = rtol ||b|| / ||r|| (the smallest over the unconverged members), is within
      // reach of one FP32 solve (need >= inner_rtol / 10), the step asks for need / 2
      // and finishes the refinement.
      double need = 0.0;
      for (int m = 0; m < nb; ++m) {
        if (conv[m]) continue;
        const double rn = std::sqrt(hir[3 * m]), bn = std::sqrt(hir[3 * m + 1]);
        const double f = rn > 0 ? opts->rtol * bn / rn : 1.0;
        need = (need == 0.0) ? f : std::min(need, f);
      }
      const double itol = need >= 0.1 * opts->inner_rtol ? 0.5 * need : opts->inner_rtol;
      PcgScalars *hs = (PcgScalars *)c->h_pinned;
      if ((st = run_pcg<float>(c, op, nb, r32, d32, true, itol,
                               opts->maxit - total_inner, opts->check_every, dinv32, dms,
                               w, hs, ns)) != SFEM_OK)
        return st;
      int mx = 0;
      for (int m = 0; m < nb; ++m) {
        iters[m] += hs[m].iters;
        mx = std::max(mx, hs[m].iters);
        if (hs[m].status != 0 && status[m] == 0) status[m] = hs[m].status;
      }
      total_inner += std::max(mx, 1);
      HIPCHK(c, launch_ir_accum(x, d32, ir, n, nb, s));
      ++outer;
    }
    for (int m = 0; m < nb; ++m)
      if (status[m] == 0 && !conv[m]) status[m] = SFEM_NOCONV;
    if (ns) {
      // mean-zero condition: x <- x - (m1^T x / 1^T m1) 1 (the residual does not change)
      HIPCHK(c, VecOps<double>::dot(x, c->d_m1, 0, part, nblk, n, nb, s));
      HIPCHK(c, launch_reduce1(part, nblk, nb, ir, s));
      HIPCHK(c, launch_shift(x, ir, 1.0 / c->m1sum, n, nb, s));
    }
  }
  sfem_status ret = SFEM_OK;
  for (int m = 0; m < nb; ++m) {
    if (info) info[m] = sfem_pcg_info{iters[m], outer, rel[m], trel[m], status[m]};
    if (status[m] < 0 && (ret >= 0 || status[m] < ret)) ret = (sfem_status)status[m];
    if (status[m] == SFEM_NOCONV && ret == SFEM_OK) ret = SFEM_NOCONV;
  }
  if (ret < 0) fail(c, ret, ret == SFEM_E_BREAKDOWN ? "CG breakdown: p^T A p <= 0" : "non-finite value in the solve");
  return ret;
}

sfem_status sfem_pcg(sfem_ctx *c, int op, int nbatch, const double *b, double *x,
                     const sfem_pcg_opts *opts, sfem_pcg_info *info) {
  if (!c) return SFEM_E_ARG;
  return guarded(c, [&] { return sfem_pcg_body(c, op, nbatch, b, x, opts, info); });
}

// Coupling factors w |J| J^{-T} at the quadrature points (Stokes blocks, convection),
// computed on first use.
sfem_status ensure_cq(sfem_ctx *c) {
  if (c->d_cq || c->nelem == 0) return SFEM_OK;
  sfem_status st;
  const int64_t q3 = (int64_t)c->q * c->q * c->q;
  if ((st = dalloc(c, &c->d_cq, c->nelem * 9 * q3)) != SFEM_OK) return st;
  HIPCHK(c, launch_coupling_setup(c->q, c->rules.gauss_x.data(), c->rules.gauss_w.data(), c->d_xyz,
                                  c->nelem, c->d_cq, c->stream));
  return SFEM_OK;
}

static sfem_status sfem_setup_pressure_body(sfem_ctx *c, const int32_t *pres_dofs, int64_t npres) {
  sfem_status st;
  if ((st = require_ready(c)) != SFEM_OK) return st;
  DeviceGuard g(c->device);
  if (c->p < 2) return fail(c, SFEM_E_UNSUPPORTED, "the Taylor-Hood pressure space needs p >= 2");
  if (c->pres_ready) return fail(c, SFEM_E_STATE, "the pressure space is already set up");
  if (npres < 0 || npres > kDofMask) return fail(c, SFEM_E_ARG, "0 <= npres < 2^30 is required");
  if (c->nelem > 0 && !pres_dofs) return fail(c, SFEM_E_ARG, "pres_dofs must not be NULL");
  if (c->nelem == 0 && npres > 0)
    return fail(c, SFEM_E_MESH, "pressure DoFs without elements");
  const int pp = c->p - 1;
  const int64_t n3p = (int64_t)(pp + 1) * (pp + 1) * (pp + 1);
  std::vector<int32_t> dofs((size_t)(c->nelem * n3p));
  if (c->nelem > 0) {
    HIPCHK(c, hipMemcpyAsync(dofs.data(), pres_dofs, dofs.size() * sizeof(int32_t),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  HostPlan hp;
  {
    std::string err;
    std::vector<uint8_t> none((size_t)npres, 0);
    // the pressure space has no essential DoFs; its E-vector is element-ordered
    const int rc = build_host_plan(pp, c->nelem, dofs.data(), npres, none.data(), hp, err, false);
    if (rc != 0) return fail(c, (sfem_status)rc, "pressure map: " + err);
  }
  if (hp.nentries >= (int64_t)kDofMask) return fail(c, SFEM_E_ARG, "mesh too large");
  const int64_t q3 = (int64_t)c->q * c->q * c->q;
  if ((st = dalloc(c, &c->d_pmap, c->nelem * n3p)) != SFEM_OK) return st;
  int32_t *d_alist = nullptr, *d_aoff = nullptr, *d_slot = nullptr;
  if ((st = dalloc(c, &d_alist, hp.na)) != SFEM_OK) return st;
  if ((st = dalloc(c, &d_aoff, hp.na + 1)) != SFEM_OK) return st;
  if ((st = dalloc(c, &d_slot, (int64_t)hp.slots.size())) != SFEM_OK) return st;
  if (c->nelem > 0)
    HIPCHK(c, hipMemcpyAsync(c->d_pmap, hp.imap.data(), hp.imap.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, c->stream));
  if (hp.na > 0) {
    HIPCHK(c, hipMemcpyAsync(d_alist, hp.alist.data(), hp.alist.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d_aoff, hp.aoff.data(), hp.aoff.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, c->stream));
  }
  if (!hp.slots.empty())
    HIPCHK(c, hipMemcpyAsync(d_slot, hp.slots.data(), hp.slots.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, c->stream));
  if ((st = ensure_cq(c)) != SFEM_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->pplan.alist = d_alist;
  c->pplan.aoff = d_aoff;
  c->pplan.slot = d_slot;
  c->pplan.na = hp.na;
  c->pcompact = hp.compact ? 1 : 0;
  c->pnentries = hp.nentries;
  c->npres = npres;
  c->pres_ready = true;
  return SFEM_OK;
}

sfem_status sfem_setup_pressure(sfem_ctx *c, const int32_t *pres_dofs, int64_t npres) {
  if (!c) return SFEM_E_ARG;
  return guarded(c, [&] { return sfem_setup_pressure_body(c, pres_dofs, npres); });
}

sfem_status sfem_stokes_apply(sfem_ctx *c, const double *u, const double *pres, double *yu,
                              double *yp) {
  sfem_status st;
  if ((st = require_ready(c)) != SFEM_OK) return st;
  if (!c->pres_ready) return fail(c, SFEM_E_STATE, "sfem_setup_pressure has not succeeded");
  if (c->nfield != 1)
    return fail(c, SFEM_E_ARG, "the Stokes operator takes one nu field (sfem_set_coeffs with nbatch_nu = 1)");
  const int64_t nv = c->ndof, np = c->npres;
  if (nv == 0 && np == 0) return SFEM_OK;
  if (!u || !pres || !yu || !yp) return fail(c, SFEM_E_ARG, "u, pres, yu and yp must not be NULL");
  if ((const void *)u == (const void *)yu || (const void *)pres == (const void *)yp)
    return fail(c, SFEM_E_ARG, "outputs must not alias inputs");
  DeviceGuard g(c->device);
  // workspace: the pressure E-vector
  if ((st = ensure_ws(c, align_up((size_t)c->pnentries * sizeof(double)) + 256)) != SFEM_OK) return st;
  double *Yp = (double *)c->ws.p;
  // y_u = H u + P G p (essential rows copy u), y_p = -D P u.  With the DoF-ordered
  // E-vector the coupling kernel adds G p into the Helmholtz element kernel's output (sole
  // DoFs of y_u, E-vector entries) and one assembly follows; with the element-ordered one
  // H u is assembled first and G p goes through an E-vector of its own and an additive
  // assembly.
  const bool one_asm = evec_dof_ordered(c->p);
  if ((st = ensure_evec(c, (size_t)c->nentries * 3 * sizeof(double))) != SFEM_OK) return st;
  if ((st = do_apply(c, SFEM_HELMHOLTZ, false, 3, u, yu, nullptr, c->evec.p, !one_asm)) != SFEM_OK)
    return st;
  StokesArgs a{};
  a.p = c->p;
  a.nelem = c->nelem;
  a.vmap = c->d_map;
  a.vpos = c->d_pos;
  a.vcompact = c->compact;
  a.pmap = c->d_pmap;
  a.pcompact = c->pcompact;
  a.cq = c->d_cq;
  a.u = u;
  a.pres = pres;
  a.nv = nv;
  a.Yv = (double *)c->evec.p;
  a.vestride = c->nentries;
  a.yv = yu;
  a.Yp = Yp;
  a.yp = yp;
  HIPCHK(c, launch_stokes(a, c->stream));
  HIPCHK(c, launch_assemble<double>(c->plan, (const double *)c->evec.p, c->nentries, one_asm ? u : nullptr,
                                    yu, nv, 3, one_asm ? kEssCopyX : kEssAdd, nullptr, 0, c->stream));
  HIPCHK(c, launch_assemble<double>(c->pplan, Yp, 0, nullptr, yp, np, 1, kEssZero, nullptr, 0,
                                    c->stream));
  return SFEM_OK;
}

sfem_status sfem_convection(sfem_ctx *c, const double *u, double *y) {
  sfem_status st;
  if ((st = require_ready(c)) != SFEM_OK) return st;
  const int64_t nv = c->ndof;
  if (nv == 0) return SFEM_OK;
  if (!u || !y) return fail(c, SFEM_E_ARG, "u and y must not be NULL");
  if ((const void *)u == (const void *)y) return fail(c, SFEM_E_ARG, "y must not alias u");
  DeviceGuard g(c->device);
  if ((st = ensure_cq(c)) != SFEM_OK) return st;
  if ((st = ensure_evec(c, (size_t)c->nentries * 3 * sizeof(double))) != SFEM_OK) return st;
  ConvArgs a{};
  a.p = c->p;
  a.nelem = c->nelem;
  a.vmap = c->d_map;
  a.vpos = c->d_pos;
  a.vcompact = c->compact;
  a.cq = c->d_cq;
  a.u = u;
  a.nv = nv;
  a.Yv = (double *)c->evec.p;
  a.vestride = c->nentries;
  a.yv = y;
  HIPCHK(c, launch_convection(a, c->stream));
  HIPCHK(c, launch_assemble<double>(c->plan, (const double *)c->evec.p, c->nentries, nullptr, y, nv, 3,
                                    kEssZero, nullptr, 0, c->stream));
  return SFEM_OK;
}

sfem_status sfem_weak_op(sfem_ctx *c, int kind, const double *x, double *y) {
  sfem_status st;
  if ((st = require_ready(c)) != SFEM_OK) return st;
  if (kind != SFEM_WEAK_GRADIENT && kind != SFEM_WEAK_CURL && kind != SFEM_WEAK_DIVERGENCE)
    return fail(c, SFEM_E_ARG, "kind must be SFEM_WEAK_GRADIENT, SFEM_WEAK_CURL or SFEM_WEAK_DIVERGENCE");
  const int64_t nv = c->ndof;
  if (nv == 0) return SFEM_OK;
  if (!x || !y) return fail(c, SFEM_E_ARG, "x and y must not be NULL");
  if ((const void *)x == (const void *)y) return fail(c, SFEM_E_ARG, "y must not alias x");
  DeviceGuard g(c->device);
  if ((st = ensure_cq(c)) != SFEM_OK) return st;
  if ((st = ensure_evec(c, (size_t)c->nentries * 3 * sizeof(double))) != SFEM_OK) return st;
  ConvArgs a{};
  a.kind = kind == SFEM_WEAK_GRADIENT ? kWeakGradient
                                      : (kind == SFEM_WEAK_CURL ? kWeakCurl : kWeakDivergence);
  a.p = c->p;
  a.nelem = c->nelem;
  a.vmap = c->d_map;
  a.vpos = c->d_pos;
  a.vcompact = c->compact;
  a.cq = c->d_cq;
  a.u = x;
  a.nv = nv;
  a.Yv = (double *)c->evec.p;
  a.vestride = c->nentries;
  a.yv = y;
  HIPCHK(c, launch_convection(a, c->stream));
  const int nout = kind == SFEM_WEAK_DIVERGENCE ? 1 : 3;
  HIPCHK(c, launch_assemble<double>(c->plan, (const double *)c->evec.p, c->nentries, nullptr, y, nv,
                                    nout, kEssZero, nullptr, 0, c->stream));
  return SFEM_OK;
}

sfem_status sfem_lincomb(sfem_ctx *c, int nterm, const double *coef, const double *const *xs,
                         const double *scale, const uint8_t *mask, int64_t n, int nb, double *y) {
  sfem_status st;
  if ((st = require_ready(c)) != SFEM_OK) return st;
  if (nterm < 1 || nterm > kMaxLinTerms) return fail(c, SFEM_E_ARG, "1 <= nterm <= 8 is required");
  if (n < 0 || nb < 0) return fail(c, SFEM_E_ARG, "n and nb must be >= 0");
  if (n == 0 || nb == 0) return SFEM_OK;
  if (!coef || !xs || !y) return fail(c, SFEM_E_ARG, "coef, xs and y must not be NULL");
  LinComb lc{};
  lc.nterm = nterm;
  for (int j = 0; j < nterm; ++j) {
    if (!xs[j]) return fail(c, SFEM_E_ARG, "xs[j] must not be NULL");
    lc.c[j] = coef[j];
    lc.x[j] = xs[j];
  }
  DeviceGuard g(c->device);
  HIPCHK(c, launch_lincomb(lc, scale, mask, y, n, nb, c->stream));
  return SFEM_OK;
}

sfem_status sfem_get_info(const sfem_ctx *c, sfem_ctx_info *out) {
  if (!c || !out) return SFEM_E_ARG;
  out->p = c->p;
  out->q = c->q;
  out->nelem = c->nelem;
  out->ndof = c->ndof;
  out->compact = c->compact;
  out->nassembled = c->na;
  out->nfields = c->nfield;
  out->device_bytes = c->bytes + (int64_t)c->ws.bytes + (int64_t)c->evec.bytes;
  out->nentries = c->nentries;
  return SFEM_OK;
}

}  // extern "C"
