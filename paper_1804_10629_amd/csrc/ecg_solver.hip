// Host driver and C ABI of the s-step enlarged CG solver.
//
// Method (Moufawad, arXiv 1804.10629, Section 3.1, algorithms "s-step
// SRE-CG" and "s-step SRE-CG2"; update by eqs (1)-(3)):
//   r = b - A x, rho_0 = ||r||
//   per s-step iteration: s blocks W_j (t columns), the first after a
//   (re)start from T(r), the others from A W_{j-1}; each A-orthonormalized
//   against W_{j-2}, W_{j-1} by CGS2 and against itself by A-CholQR;
//   alpha = V^t r, x += V alpha, r -= A V alpha, rho = ||r||.
//
// Representation used on the device: block j is stored unnormalized as
// U_j (the CGS2 output) and its product A U_j, together with R_j^{-1} from
// the Cholesky factor of U_j^t A U_j; W_j = U_j R_j^{-1} and
// A W_j = (A U_j) R_j^{-1} are never formed.  Every use of W_j folds R_j^{-1}
// into the small coefficient matrices of the block kernels, which saves one
// full read-and-write pass over two n x t blocks per basis block.  In exact
// arithmetic the iterates are those of the algorithm; the first CGS2 Gram
// of block j+1, (A W_p)^t A W_j, comes from the product kernel of block j.

#include "ecg_kernels.h"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <utility>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <queue>
#include <string>
#include <type_traits>
#include <vector>

#include "ecg.h"

using namespace ecg;

// Staging array of ecg_spmm_noalloc (two n x w blocks, 64 MiB), one copy per
// GPU.  Its name is a host-side stand-in in host code: kernels get the
// per-device address that resolve_noalloc_scratch records.
constexpr size_t kNoAllocDoubles = 2 * (size_t)ECG_SPMM_NOALLOC_MAX;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ECG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

const char* kclass_names[ECG_K_COUNT] = {"resid",     "tsplit", "cgs_gram", "cgs_update", "spmm",
                                         "xr_update", "gram",   "update",   "small",      "precond"};

struct Timed {
  int k;
  hipEvent_t a, b;
  double bytes, flops;
};

}  // namespace

struct ecg_ctx {
  int64_t n = 0, nnz = 0;
  int t = 0, s = 0, tpi = 16;
  int max_row = 0;            // most entries in a row
  ecg_opts o{};
  hipStream_t st = nullptr;
  int dev = 0;
  int sbytes = 8;   // bytes per basis element

  int32_t* rowptr = nullptr;
  int32_t* colind = nullptr;
  int32_t* dom = nullptr;
  // domain-contiguous row order (opts.permute_domains): perm[i] is the
  // caller's row of solver row i, emap[p] the caller's entry of solver
  // entry p; both NULL when the caller's order is kept
  int32_t* perm = nullptr;
  int32_t* emap = nullptr;
  // block Jacobi preconditioner M = L L^t (ecg_set_preconditioner), in the
  // solver's row order: strictly lower L and strictly upper L^t in CSR,
  // 1 / diag(L), and the rows of every level of the two triangular solves
  int prec = ECG_PREC_NONE;
  int32_t *pl_rp = nullptr, *pl_ci = nullptr, *pu_rp = nullptr, *pu_ci = nullptr;
  double *pl_v = nullptr, *pu_v = nullptr, *p_dinv = nullptr;
  int32_t *lev_f = nullptr, *lev_b = nullptr;
  std::vector<int> levp_f, levp_b;   // level offsets into lev_f / lev_b (host)
  int64_t pl_nnz = 0;
  double* vals = nullptr;
  float* vals32 = nullptr;
  double* b = nullptr;
  double* x = nullptr;        // last completed iterate
  double* r = nullptr;        // its recursive residual
  double* x2 = nullptr;       // the iterate being formed (swapped with x per iteration)
  double* r2 = nullptr;

  int nslot = 0;              // block slots (SRE-CG2: the block cap)
  int nalloc = 0;             // slots with allocated U / AU
  std::vector<void*> U, AU;
  void* Zp = nullptr;
  double* rinv = nullptr;     // [nslot][T2]
  double* beta = nullptr;     // [nslot][tpi]
  double* cnext = nullptr;    // [3][T2]
  double* dcoef = nullptr;    // [2][T2]
  double* ctab = nullptr;     // SRE-CG2: [nslot][T2] first-pass coefficients
  double* dtab = nullptr;     // SRE-CG2: [nslot][T2] second-pass coefficients
  double* pre_rinv = nullptr; // Pre-CholQR: Re^{-1}
  double* scratch = nullptr;  // op buffers (n * tpi doubles, lazily)
  double* scratch2 = nullptr;
  DevStatus* status = nullptr;
  DevStatus* h_status = nullptr;   // pinned

  double* partials = nullptr;
  double* groups = nullptr;
  int grid = 1024;
  int group_size = 32;

  // basis of the last completed iteration
  int last_nb = 0;
  int last_slots[kMaxS];

  ecg_stats stats{};
  std::vector<Timed> pending;
  std::vector<hipEvent_t> free_events;
  hipEvent_t ev_solve0 = nullptr, ev_solve1 = nullptr;

  RedCtl rc() const { return RedCtl{partials, groups, group_size}; }
  int T2() const { return tpi * tpi; }
  double blk_bytes() const { return (double)n * t * sbytes; }
  double csr_bytes(int vb) const { return (double)nnz * (vb + 4) + 4.0 * (n + 1); }

  hipEvent_t get_event() {
    if (!free_events.empty()) {
      hipEvent_t e = free_events.back();
      free_events.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  // start timing a launch of class k
  void tstart(Timed& tm, int k, double bytes, double flops) {
    tm.k = k;
    tm.bytes = bytes;
    tm.flops = flops;
    tm.a = tm.b = nullptr;
    if (!o.collect_stats) return;
    tm.a = get_event();
    tm.b = get_event();
    if (tm.a) (void)hipEventRecord(tm.a, st);
  }
  void tstop(Timed& tm) {
    stats.launches[tm.k] += 1;
    stats.bytes[tm.k] += tm.bytes;
    stats.flops[tm.k] += tm.flops;
    if (!o.collect_stats || !tm.a || !tm.b) return;
    (void)hipEventRecord(tm.b, st);
    pending.push_back(tm);
  }
  // after a stream synchronisation
  void flush_timing() {
    for (auto& tm : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, tm.a, tm.b) == hipSuccess) stats.ms[tm.k] += ms;
      free_events.push_back(tm.a);
      free_events.push_back(tm.b);
    }
    pending.clear();
  }
};

// ---------------------------------------------------------------------------

extern "C" {

void ecg_opts_default(ecg_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->variant = ECG_SRECG;
  o->orth = ECG_ACHOLQR;
  o->precision = ECG_FP64;
  o->device_ptrs = 0;
  o->inner_tol = 1e-4;
  o->max_restarts = 20;
  o->q_cap_blocks = 0;
  o->ws_cap_bytes = 0;
  o->hip_stream = nullptr;
  o->collect_stats = 0;
  o->grid = 0;
  o->progress_every = 0;
  o->permute_domains = 1;
}

const char* ecg_version(void) { return "ecg-mi355x 0.1.0 (gfx950)"; }

const char* ecg_strerror(int s) {
  switch (s) {
    case ECG_OK: return "converged";
    case ECG_MAXIT: return "iteration limit reached";
    case ECG_BREAKDOWN: return "breakdown: Gram matrix not positive definite";
    case ECG_STAGNATED: return "true residual stagnated above tolerance";
    case ECG_EINVAL: return "invalid argument";
    case ECG_ENOMEM: return "out of device memory";
    case ECG_EDEVICE: return "HIP device error";
    case ECG_ENOTSUP: return "not supported";
    default: return "unknown status";
  }
}

const char* ecg_last_error(void) { return g_last_error.c_str(); }

const char* ecg_kclass_name(int k) {
  if (k < 0 || k >= ECG_K_COUNT) return nullptr;
  return kclass_names[k];
}

}  // extern "C"

namespace {

int check_device() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    int count = 0;
    hipError_t e2 = hipGetDeviceCount(&count);
    return fail(ECG_EDEVICE, std::string("no usable HIP device (hipGetDevice: ") +
                                 hipGetErrorString(e) + ", hipGetDeviceCount: " +
                                 hipGetErrorString(e2) + ", count " + std::to_string(count) + ")");
  }
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(ECG_EDEVICE, std::string("device is ") + prop.gcnArchName + ", built for gfx950");
  return ECG_OK;
}

// Per-device addresses of `scratch`: ecg_setup resolves each device's own
// once, with that device current; ecg_spmm_noalloc uses only these.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// With device `dev` current: resolve (once) its address of `scratch`.
int resolve_noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(ECG_EDEVICE, "device index " + std::to_string(dev) + " beyond the " +
                                 std::to_string(kMaxDevices) + " the library tracks");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return ECG_OK;
  void* p = nullptr;
  HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return fail(ECG_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
  g_scratch_ptr[dev] = (double*)p;
  return ECG_OK;
}

double* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}

// Copy `count` elements of an input array to host memory (device_ptrs mode).
template <typename T>
int fetch(const T* src, int64_t count, bool dev, std::vector<T>& out, const T** view) {
  if (!dev) {
    *view = src;
    return ECG_OK;
  }
  out.resize((size_t)count);
  HIP_TRY(hipMemcpy(out.data(), src, sizeof(T) * count, hipMemcpyDeviceToHost));
  *view = out.data();
  return ECG_OK;
}

template <typename T>
int dalloc(T** p, size_t count, size_t& total) {
  size_t bytes = std::max<size_t>(sizeof(T) * count, 256);
  total += bytes;
  hipError_t e = hipMalloc((void**)p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(ECG_ENOMEM, std::string("hipMalloc of ") + std::to_string(bytes) + " bytes failed");
  }
  return ECG_OK;
}

int pick_tpi(int t) { return t <= 16 ? 16 : (t <= 32 ? 32 : 64); }

int rows_per_wg(int) { return 64; }

}  // namespace

extern "C" void ecg_destroy(ecg_ctx* c) {
  if (!c) return;
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  f(c->rowptr); f(c->colind); f(c->dom); f(c->vals); f(c->vals32);
  f(c->perm); f(c->emap);
  f(c->pl_rp); f(c->pl_ci); f(c->pl_v); f(c->pu_rp); f(c->pu_ci); f(c->pu_v); f(c->p_dinv);
  f(c->lev_f); f(c->lev_b);
  f(c->b); f(c->x); f(c->r); f(c->x2); f(c->r2);
  for (void* p : c->U) f(p);
  for (void* p : c->AU) f(p);
  f(c->Zp); f(c->rinv); f(c->beta); f(c->cnext); f(c->dcoef);
  f(c->ctab); f(c->dtab); f(c->pre_rinv);
  f(c->scratch); f(c->scratch2); f(c->status);
  f(c->partials); f(c->groups);
  if (c->h_status) (void)hipHostFree(c->h_status);
  for (auto& tm : c->pending) {
    (void)hipEventDestroy(tm.a);
    (void)hipEventDestroy(tm.b);
  }
  for (auto e : c->free_events) (void)hipEventDestroy(e);
  if (c->ev_solve0) (void)hipEventDestroy(c->ev_solve0);
  if (c->ev_solve1) (void)hipEventDestroy(c->ev_solve1);
  delete c;
}

extern "C" int ecg_partition_grid(int64_t nx, int64_t ny, int64_t nz, int32_t px, int32_t py,
                                  int32_t pz, int32_t* dom_dev, void* stream) {
  if (!dom_dev) return fail(ECG_EINVAL, "dom_dev is NULL");
  if (nx <= 0 || ny <= 0 || nz <= 0 || px <= 0 || py <= 0 || pz <= 0)
    return fail(ECG_EINVAL, "grid and part counts must be positive");
  if (px > nx || py > ny || pz > nz) return fail(ECG_EINVAL, "more parts than cells along an axis");
  if (nx * ny > (int64_t(1) << 31) || nx * ny * nz >= (int64_t(1) << 31))
    return fail(ECG_EINVAL, "grid too large for int32 row indices");
  int rc = check_device();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_partition(nx, ny, nz, px, py, pz, dom_dev, st));
  HIP_TRY(hipStreamSynchronize(st));
  return ECG_OK;
}

extern "C" int ecg_grid_morton_keys(int64_t nx, int64_t ny, int64_t nz, int64_t* keys) {
  if (!keys) return fail(ECG_EINVAL, "keys is NULL");
  if (nx <= 0 || ny <= 0 || nz <= 0) return fail(ECG_EINVAL, "grid sizes must be positive");
  constexpr int64_t kSide = int64_t(1) << 21;   // 3 x 21 bits fit an int64 key
  if (nx >= kSide || ny >= kSide || nz >= kSide) return fail(ECG_EINVAL, "grid side >= 2^21");
  if (nx * ny >= (int64_t(1) << 31) || nx * ny * nz >= (int64_t(1) << 31))
    return fail(ECG_EINVAL, "grid too large for int32 row indices");
  // spread the 21 low bits of v to every third bit
  auto spread = [](uint64_t v) {
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1u) << (3 * b);
    return r;
  };
  for (int64_t k = 0; k < nz; ++k) {
    const uint64_t kz = spread((uint64_t)k) << 2;
    for (int64_t j = 0; j < ny; ++j) {
      const uint64_t kyz = kz | (spread((uint64_t)j) << 1);
      int64_t* row = keys + nx * (j + ny * k);
      for (int64_t i = 0; i < nx; ++i) row[i] = (int64_t)(kyz | spread((uint64_t)i));
    }
  }
  return ECG_OK;
}

// Allocate and zero block pairs up to `want` slots (padding columns of a
// block stay zero from here on).  On failure the slots allocated so far
// stay usable and ECG_ENOMEM is returned.
static int grow_slots(ecg_ctx* c, int want) {
  const size_t bytes = (size_t)c->n * c->tpi * c->sbytes;
  for (int i = c->nalloc; i < want; ++i) {
    void *u = nullptr, *au = nullptr;
    if (hipMalloc(&u, bytes) != hipSuccess) return fail(ECG_ENOMEM, "block allocation failed");
    if (hipMalloc(&au, bytes) != hipSuccess) {
      (void)hipFree(u);
      return fail(ECG_ENOMEM, "block allocation failed");
    }
    c->U[i] = u;
    c->AU[i] = au;
    if (hipMemsetAsync(u, 0, bytes, c->st) != hipSuccess ||
        hipMemsetAsync(au, 0, bytes, c->st) != hipSuccess)
      return fail(ECG_EDEVICE, "block clear failed");
    c->nalloc = i + 1;
  }
  return ECG_OK;
}

extern "C" int ecg_setup(ecg_ctx** out, int64_t n, const int32_t* rowptr, const int32_t* colind,
                         const double* vals, const int32_t* partition, int32_t t, int32_t s,
                         const ecg_opts* opts) {
  if (!out) return fail(ECG_EINVAL, "out is NULL");
  *out = nullptr;
  ecg_opts o;
  if (opts) o = *opts;
  else ecg_opts_default(&o);
  if (o.reserved[0] != 0) return fail(ECG_EINVAL, "reserved option fields must be zero");
  if (!rowptr || !colind || !vals || !partition) return fail(ECG_EINVAL, "NULL array argument");
  if (n <= 0) return fail(ECG_EINVAL, "n must be positive");
  if (n >= (int64_t(1) << 31)) return fail(ECG_EINVAL, "n must be < 2^31");
  if (t < 1 || t > 64) return fail(ECG_EINVAL, "t must be in [1, 64]");
  if (t > n) return fail(ECG_EINVAL, "t must not exceed n");
  if (s < 1 || s > kMaxS) return fail(ECG_EINVAL, "s must be in [1, 16]");
  if (o.variant != ECG_SRECG && o.variant != ECG_SRECG2 && o.variant != ECG_MSDO)
    return fail(ECG_EINVAL, "bad variant");
  if (o.orth != ECG_ACHOLQR && o.orth != ECG_PRECHOLQR) return fail(ECG_EINVAL, "bad orth");
  if (o.precision != ECG_FP64 && o.precision != ECG_MIXED) return fail(ECG_EINVAL, "bad precision");
  if (o.device_ptrs != 0 && o.device_ptrs != 1) return fail(ECG_EINVAL, "bad device_ptrs");
  if (o.permute_domains != 0 && o.permute_domains != 1)
    return fail(ECG_EINVAL, "bad permute_domains");
  if (o.ca < 0 || o.ca > 2) return fail(ECG_EINVAL, "bad ca");
  if (o.row_key && o.permute_domains != 1)
    return fail(ECG_EINVAL, "row_key needs permute_domains = 1");
  if (!(o.inner_tol >= 0.0 && o.inner_tol < 1.0)) return fail(ECG_EINVAL, "inner_tol must be in [0, 1)");
  if (o.max_restarts < 0 || o.q_cap_blocks < 0 || o.ws_cap_bytes < 0 || o.grid < 0 ||
      o.progress_every < 0)
    return fail(ECG_EINVAL, "negative option");
  if (o.variant != ECG_SRECG && o.q_cap_blocks > 0 && o.q_cap_blocks < s)
    return fail(ECG_EINVAL, "q_cap_blocks must be 0 or at least s");
  const bool dev = o.device_ptrs == 1;
  if (dev) {
    int rc = check_device();
    if (rc) return rc;
  }

  // ---- validate on the host ----
  std::vector<int32_t> hrp, hci, hdom;
  std::vector<double> hv;
  const int32_t *rp = nullptr, *ci = nullptr, *pd = nullptr;
  const double* vv = nullptr;
  int rc = fetch(rowptr, n + 1, dev, hrp, &rp);
  if (rc) return rc;
  if (rp[0] != 0) return fail(ECG_EINVAL, "rowptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) return fail(ECG_EINVAL, "rowptr must be non-decreasing");
  const int64_t nnz = rp[n];
  if (nnz <= 0) return fail(ECG_EINVAL, "matrix has no nonzeros");
  rc = fetch(colind, nnz, dev, hci, &ci);
  if (rc) return rc;
  for (int64_t p = 0; p < nnz; ++p)
    if (ci[p] < 0 || ci[p] >= n) return fail(ECG_EINVAL, "column index out of range");
  rc = fetch(vals, nnz, dev, hv, &vv);
  if (rc) return rc;
  for (int64_t p = 0; p < nnz; ++p)
    if (!std::isfinite(vv[p])) return fail(ECG_EINVAL, "non-finite matrix value");
  rc = fetch(partition, n, dev, hdom, &pd);
  if (rc) return rc;
  std::vector<int64_t> dsize(t, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (pd[i] < 0 || pd[i] >= t) return fail(ECG_EINVAL, "partition value out of [0, t)");
    dsize[pd[i]]++;
  }
  for (int d = 0; d < t; ++d)
    if (dsize[d] == 0) return fail(ECG_EINVAL, "empty domain " + std::to_string(d));

  // Domain-contiguous order (the paper reorders the matrix by its Metis
  // domains, Section 4): solver row i is the caller's row perm[i], rows
  // sorted by domain, keeping the caller's order within a domain (or, with
  // row_key, sorted by key within a domain, ties in the caller's order);
  // column indices renumbered and sorted ascending within each row.
  const bool permute = o.permute_domains == 1;
  std::vector<int32_t> perm_h, emap_h, prp_h, pci_h, pdom_h;
  std::vector<double> pv_h;
  if (permute) {
    std::vector<int64_t> pos(t + 1, 0);
    for (int d = 0; d < t; ++d) pos[d + 1] = pos[d] + dsize[d];
    perm_h.resize(n);
    std::vector<int32_t> iperm(n);
    for (int64_t i = 0; i < n; ++i) perm_h[pos[pd[i]]++] = (int32_t)i;
    if (o.row_key) {
      std::vector<int64_t> hkey;
      const int64_t* key = nullptr;
      if ((rc = fetch(o.row_key, n, dev, hkey, &key))) return rc;
      // pos[d] is now the end of domain d's rows
      for (int d = 0; d < t; ++d)
        std::stable_sort(perm_h.begin() + (pos[d] - dsize[d]), perm_h.begin() + pos[d],
                         [key](int32_t a, int32_t b) { return key[a] < key[b]; });
    }
    for (int64_t j = 0; j < n; ++j) iperm[perm_h[j]] = (int32_t)j;
    prp_h.resize(n + 1);
    pci_h.resize(nnz);
    pv_h.resize(nnz);
    emap_h.resize(nnz);
    pdom_h.resize(n);
    std::vector<std::pair<int32_t, int32_t>> ent;
    int64_t k = 0;
    prp_h[0] = 0;
    for (int64_t j = 0; j < n; ++j) {
      const int32_t p = perm_h[j];
      ent.clear();
      for (int32_t e = rp[p]; e < rp[p + 1]; ++e) ent.emplace_back(iperm[ci[e]], e);
      std::sort(ent.begin(), ent.end());
      for (const auto& ce : ent) {
        pci_h[k] = ce.first;
        pv_h[k] = vv[ce.second];
        emap_h[k] = ce.second;
        ++k;
      }
      prp_h[j + 1] = (int32_t)k;
      pdom_h[j] = pd[p];
    }
  }

  rc = check_device();
  if (rc) return rc;
  {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if ((rc = resolve_noalloc_scratch(dev))) return rc;
  }

  ecg_ctx* c = new ecg_ctx();
  c->n = n;
  c->nnz = nnz;
  for (int64_t i = 0; i < n; ++i) c->max_row = std::max(c->max_row, (int)(rp[i + 1] - rp[i]));
  c->t = t;
  c->s = s;
  c->tpi = pick_tpi(t);
  c->o = o;
  c->st = (hipStream_t)o.hip_stream;
  c->sbytes = o.precision == ECG_MIXED ? 4 : 8;
  (void)hipGetDevice(&c->dev);
  const int tpi = c->tpi, T2 = tpi * tpi;
  const size_t blk = (size_t)n * tpi;

  // grid of the streaming kernels
  {
    int64_t steps = (n + rows_per_wg(tpi) - 1) / rows_per_wg(tpi);
    int g = o.grid > 0 ? o.grid : (int)std::min<int64_t>(steps, tpi == 64 ? 512 : 1024);
    c->grid = std::max(1, g);
  }
  const int max_grid = std::max(c->grid, 1024);
  const int max_partials = max_grid * kCSGroups;   // column-split kernels: per row group
  const int ngroups = (max_partials + c->group_size - 1) / c->group_size;
  const size_t L = 3 * (size_t)T2 + tpi;

  // ---- workspace size check ----
  const size_t esz = c->sbytes;
  const double fixed = blk * esz + (double)nnz * (4 + 8 + (o.precision ? 4 : 0)) +
                       4.0 * (n + 1) + 4.0 * n + 5.0 * 8 * n + (double)max_partials * L * 8 +
                       (double)ngroups * L * 8;
  const double per_slot = 2.0 * blk * esz + 8.0 * (3.0 * T2 + tpi);
  size_t freeb = 0, totalb = 0;
  HIP_TRY(hipMemGetInfo(&freeb, &totalb));
  double cap = o.ws_cap_bytes > 0 ? (double)o.ws_cap_bytes : 0.9 * (double)freeb;
  if (o.variant != ECG_SRECG) {
    // every block since the last restart is kept: one slot per block, at
    // least the s blocks of one iteration
    int64_t fit = (int64_t)((cap - fixed) / per_slot);
    int64_t want = o.q_cap_blocks > 0 ? o.q_cap_blocks : std::min<int64_t>(fit, 2048);
    if (want < s || want > fit) {
      delete c;
      return fail(ECG_ENOMEM, "SRE-CG2 workspace: " + std::to_string(want) + " blocks requested, " +
                                  std::to_string(fit) + " fit, at least s needed");
    }
    c->nslot = (int)want;
  } else {
    // s-step SRE-CG: blocks m-2 .. m of (s+2); CA SRE-CG: the s+1 kept
    // blocks and the s of the iteration being built
    c->nslot = o.ca ? 2 * s + 1 : s + 2;
  }
  double need = fixed + per_slot * c->nslot;
  if (need > cap) {
    delete c;
    return fail(ECG_ENOMEM, "workspace of " + std::to_string(need) + " bytes exceeds the cap of " +
                                std::to_string(cap));
  }

  size_t total = 0;
  auto cleanup = [&](int code) {
    ecg_destroy(c);
    return code;
  };
#define ALLOC(ptr, type, count)                       \
  do {                                                \
    int r_ = dalloc<type>(&(ptr), (count), total);    \
    if (r_) return cleanup(r_);                       \
  } while (0)
  ALLOC(c->rowptr, int32_t, n + 1);
  ALLOC(c->colind, int32_t, nnz);
  ALLOC(c->vals, double, nnz);
  ALLOC(c->dom, int32_t, n);
  ALLOC(c->b, double, n);
  ALLOC(c->x, double, n);
  ALLOC(c->r, double, n);
  ALLOC(c->x2, double, n);
  ALLOC(c->r2, double, n);
  if (o.precision == ECG_MIXED) ALLOC(c->vals32, float, nnz);
  if (permute) {
    ALLOC(c->perm, int32_t, n);
    ALLOC(c->emap, int32_t, nnz);
  }
  // SRE-CG2 keeps one block pair per block since the last restart; its
  // pairs are allocated when a solve first needs them (grow_slots)
  c->U.assign(c->nslot, nullptr);
  c->AU.assign(c->nslot, nullptr);
  {
    const int first = o.variant != ECG_SRECG ? std::min(c->nslot, s + 2) : c->nslot;
    if ((rc = grow_slots(c, first))) return cleanup(rc);
  }
  if (o.precision == ECG_MIXED) ALLOC(*(float**)&c->Zp, float, blk);
  else ALLOC(*(double**)&c->Zp, double, blk);
  ALLOC(c->rinv, double, (size_t)c->nslot * T2);
  ALLOC(c->beta, double, (size_t)c->nslot * tpi);
  ALLOC(c->cnext, double, 3 * (size_t)T2);
  ALLOC(c->dcoef, double, 2 * (size_t)T2);
  ALLOC(c->pre_rinv, double, (size_t)T2);
  // CGS coefficient tables: SRE-CG2 / MSDO-CG, and the preconditioned forms
  ALLOC(c->ctab, double, (size_t)std::max(c->nslot, 2) * T2);
  ALLOC(c->dtab, double, (size_t)std::max(c->nslot, 2) * T2);
  ALLOC(c->status, DevStatus, 1);
  ALLOC(c->partials, double, (size_t)max_partials * L);
  ALLOC(c->groups, double, (size_t)ngroups * L);
#undef ALLOC
  if (hipHostMalloc((void**)&c->h_status, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(ECG_ENOMEM, "pinned host allocation failed"));

  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  auto up = [&](void* dst, const void* src, size_t bytes) -> int {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, kind, c->st));
    return ECG_OK;
  };
  auto uph = [&](void* dst, const void* src, size_t bytes) -> int {
    HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return ECG_OK;
  };
  if (permute) {
    if ((rc = uph(c->rowptr, prp_h.data(), sizeof(int32_t) * (n + 1)))) return cleanup(rc);
    if ((rc = uph(c->colind, pci_h.data(), sizeof(int32_t) * nnz))) return cleanup(rc);
    if ((rc = uph(c->vals, pv_h.data(), sizeof(double) * nnz))) return cleanup(rc);
    if ((rc = uph(c->dom, pdom_h.data(), sizeof(int32_t) * n))) return cleanup(rc);
    if ((rc = uph(c->perm, perm_h.data(), sizeof(int32_t) * n))) return cleanup(rc);
    if ((rc = uph(c->emap, emap_h.data(), sizeof(int32_t) * nnz))) return cleanup(rc);
  } else {
    if ((rc = up(c->rowptr, rowptr, sizeof(int32_t) * (n + 1)))) return cleanup(rc);
    if ((rc = up(c->colind, colind, sizeof(int32_t) * nnz))) return cleanup(rc);
    if ((rc = up(c->vals, vals, sizeof(double) * nnz))) return cleanup(rc);
    if ((rc = up(c->dom, partition, sizeof(int32_t) * n))) return cleanup(rc);
  }
  if (o.precision == ECG_MIXED) {
    const double* vsrc = permute ? pv_h.data() : vv;
    std::vector<float> v32((size_t)nnz);
    for (int64_t p = 0; p < nnz; ++p) v32[p] = (float)vsrc[p];
    if (hipMemcpy(c->vals32, v32.data(), sizeof(float) * nnz, hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(ECG_EDEVICE, "upload of binary32 values failed"));
  }
  // zero everything the kernels read before writing (padding columns stay zero)
  if (hipMemsetAsync(c->Zp, 0, blk * esz, c->st) != hipSuccess ||
      hipMemsetAsync(c->rinv, 0, sizeof(double) * c->nslot * T2, c->st) != hipSuccess ||
      hipMemsetAsync(c->beta, 0, sizeof(double) * c->nslot * tpi, c->st) != hipSuccess ||
      hipMemsetAsync(c->cnext, 0, sizeof(double) * 3 * T2, c->st) != hipSuccess ||
      hipMemsetAsync(c->dcoef, 0, sizeof(double) * 2 * T2, c->st) != hipSuccess ||
      hipMemsetAsync(c->status, 0, sizeof(DevStatus), c->st) != hipSuccess)
    return cleanup(fail(ECG_EDEVICE, "workspace clear failed"));
  if (hipEventCreate(&c->ev_solve0) != hipSuccess || hipEventCreate(&c->ev_solve1) != hipSuccess)
    return cleanup(fail(ECG_EDEVICE, "event creation failed"));
  if (hipStreamSynchronize(c->st) != hipSuccess)
    return cleanup(fail(ECG_EDEVICE, "setup synchronisation failed"));
  *out = c;
  return ECG_OK;
}

// ---------------------------------------------------------------------------
// The solve
// ---------------------------------------------------------------------------

namespace {

// x/r contribution of the previous block carried by the next block's first
// CGS kernel (which reads that block and its A-image anyway).
struct Fold {
  const double* beta;
  const double* x_in;
  const double* r_in;
};

template <int TPI, typename S, typename SA>
struct Engine {
  ecg_ctx* c;

  template <typename A>
  void set_fold(A& a, const Fold* f) const {
    if (!f) return;
    a.fold_beta = f->beta;
    a.x_in = f->x_in;
    a.r_in = f->r_in;
    a.x_out = c->x2;
    a.r_out = c->r2;
    a.status = c->status;
  }
  const SA* avals() const {
    if constexpr (std::is_same<SA, float>::value) return c->vals32;
    else return c->vals;
  }
  S* U(int slot) const { return (S*)c->U[slot]; }
  S* AU(int slot) const { return (S*)c->AU[slot]; }
  double* rinv(int slot) const { return c->rinv + (size_t)slot * TPI * TPI; }
  double* beta(int slot) const { return c->beta + (size_t)slot * TPI; }

  TailArgs tail0(int m) const {
    TailArgs ta{};
    ta.t = c->t;
    ta.m = m;
    ta.cnext = c->cnext;
    ta.dcoef = c->dcoef;
    ta.status = c->status;
    return ta;
  }

  // totals of the partials of the last producer (G work-groups, L values)
  // and the small algebra `tail`
  int reduce(int G, int L, int tail, int ng, const TailArgs& ta) {
    Timed tm;
    c->tstart(tm, ECG_K_SMALL, 8.0 * G * L + 8.0 * ((G + c->group_size - 1) / c->group_size) * L,
              (double)G * L);
    HIP_TRY(launch_reduce(c->rc(), G, L, TPI, tail, ng, ta, c->st));
    c->tstop(tm);
    return ECG_OK;
  }

  int resid(int which) {
    TailArgs ta = tail0(0);
    ta.which = which;
    Timed tm;
    c->tstart(tm, ECG_K_RESID, c->csr_bytes(8) + 24.0 * c->n, 2.0 * c->nnz + 3.0 * c->n);
    const int g = (int)std::min<int64_t>((c->n + kThreads - 1) / kThreads, c->grid);
    HIP_TRY(launch_resid(c->rowptr, c->colind, c->vals, c->b, c->x, c->r, c->n, g, c->rc(), ta,
                         c->st));
    c->tstop(tm);
    return reduce(g, 1, TAIL_NORM, 0, ta);
  }

  // One launch of the generic update/Gram kernel, timed as class k.
  int ug(int k, int nu, int ng, bool ident0, bool write, const UGArgs<S>& a, double bytes,
         double flops) {
    Timed tm;
    c->tstart(tm, k, bytes, flops);
    HIP_TRY((launch_update_gram<TPI, S>(nu, ng, ident0, write, TAIL_NONE, a, c->grid, c->st)));
    c->tstop(tm);
    return ECG_OK;
  }

  // SRE-CG2 (Algorithm "s-step SRE-CG2"): CGS2 of block m against every
  // block since the last restart, slots 0 .. m-2 (block p in slot p-1), in
  // chunks of at most CH earlier blocks per launch.  Blocks m-1 and m-2 take
  // their first-pass coefficients from the product tail of block m-1, the
  // older ones from Gram chunks against A U_{m-1}.
  int cgs_all(int m, int slot, const Fold* fold) {
    constexpr int T2 = TPI * TPI;
    constexpr int CH = TPI == 64 ? 2 : 3;
    const double bb = c->blk_bytes();
    const double nt2 = (double)c->n * c->t * c->t;
    const int newest = m - 2;                     // slot of block m-1
    int rc;
    // (a) first-pass Grams G_p = (A U_p)^t A U_{m-1} for blocks p <= m-3
    for (int p0 = 0; p0 <= m - 4; p0 += CH) {
      const int len = std::min(CH, m - 3 - p0);
      UGArgs<S> g{};
      g.X[0] = AU(newest);
      for (int k = 0; k < len; ++k) g.P[k] = AU(p0 + k);
      g.n = c->n;
      g.rc = c->rc();
      if ((rc = ug(ECG_K_GRAM, 1, len, true, false, g, (1.0 + len) * bb, 2.0 * nt2 * len)))
        return rc;
      TailArgs ta = tail0(m);
      for (int k = 0; k < len; ++k) {
        ta.rinv_g[k] = rinv(p0 + k);
        ta.coef_out[k] = c->ctab + (size_t)(p0 + k) * T2;
      }
      ta.rinv_right = rinv(newest);
      if ((rc = reduce(gram_partials(TPI, c->grid), len * T2, TAIL_GRAM, len, ta))) return rc;
    }
    // (b) first update: Z' = A U_{m-1} C0 + U_{m-1} C1 + U_{m-2} C2 + sum_p U_p C_p
    {
      UGArgs<S> u{};
      u.X[0] = AU(newest);
      u.X[1] = U(newest);
      u.X[2] = U(newest - 1);
      u.C[0] = c->cnext;
      u.C[1] = c->cnext + T2;
      u.C[2] = c->cnext + 2 * T2;
      u.out = (S*)c->Zp;
      u.n = c->n;
      u.rc = c->rc();
      set_fold(u, fold);
      if ((rc = ug(ECG_K_UPDATE, 3, 0, false, true, u, 4.0 * bb + (fold ? 32.0 * c->n : 0.0),
                   6.0 * nt2)))
        return rc;
    }
    for (int p0 = 0; p0 <= m - 4; p0 += CH) {
      const int len = std::min(CH, m - 3 - p0);
      UGArgs<S> u{};
      u.X[0] = (const S*)c->Zp;
      for (int k = 0; k < len; ++k) {
        u.X[1 + k] = U(p0 + k);
        u.C[1 + k] = c->ctab + (size_t)(p0 + k) * T2;
      }
      u.out = (S*)c->Zp;
      u.n = c->n;
      u.rc = c->rc();
      if ((rc = ug(ECG_K_UPDATE, 1 + len, 0, true, true, u, (2.0 + len) * bb, 2.0 * nt2 * len)))
        return rc;
    }
    // (c), (d) second pass against every earlier block, into the slot
    if ((rc = pass_gram(m, (const S*)c->Zp, c->dtab))) return rc;
    return pass_update(m, (const S*)c->Zp, c->dtab, U(slot));
  }

  // One CGS pass, first half: coefficients tab[i] = -R_p^{-1} R_p^{-t}
  // (A U_p)^t X for the blocks p in slots sl[0 .. cnt-1].
  int pass_gram_slots(const int* sl, int cnt, const S* X, double* tab) {
    constexpr int T2 = TPI * TPI;
    constexpr int CH = TPI == 64 ? 2 : 3;
    const double bb = c->blk_bytes();
    const double nt2 = (double)c->n * c->t * c->t;
    int rc;
    for (int p0 = 0; p0 < cnt; p0 += CH) {
      const int len = std::min(CH, cnt - p0);
      UGArgs<S> g{};
      g.X[0] = X;
      for (int k = 0; k < len; ++k) g.P[k] = AU(sl[p0 + k]);
      g.n = c->n;
      g.rc = c->rc();
      if ((rc = ug(ECG_K_GRAM, 1, len, true, false, g, (1.0 + len) * bb, 2.0 * nt2 * len)))
        return rc;
      TailArgs ta = tail0(0);
      for (int k = 0; k < len; ++k) {
        ta.rinv_g[k] = rinv(sl[p0 + k]);
        ta.coef_out[k] = tab + (size_t)(p0 + k) * T2;
      }
      ta.rinv_right = nullptr;
      if ((rc = reduce(gram_partials(TPI, c->grid), len * T2, TAIL_GRAM, len, ta))) return rc;
    }
    return ECG_OK;
  }

  // Second half: out = X + sum_i U_{sl[i]} tab[i] (in place after the first
  // chunk; out may be X).
  int pass_update_slots(const int* sl, int cnt, const S* X, const double* tab, S* out) {
    constexpr int T2 = TPI * TPI;
    constexpr int CH = TPI == 64 ? 2 : 3;
    const double bb = c->blk_bytes();
    const double nt2 = (double)c->n * c->t * c->t;
    int rc;
    for (int p0 = 0; p0 < cnt; p0 += CH) {
      const int len = std::min(CH, cnt - p0);
      UGArgs<S> u{};
      u.X[0] = p0 == 0 ? X : out;
      for (int k = 0; k < len; ++k) {
        u.X[1 + k] = U(sl[p0 + k]);
        u.C[1 + k] = tab + (size_t)(p0 + k) * T2;
      }
      u.out = out;
      u.n = c->n;
      u.rc = c->rc();
      if ((rc = ug(ECG_K_UPDATE, 1 + len, 0, true, true, u, (2.0 + len) * bb, 2.0 * nt2 * len)))
        return rc;
    }
    return ECG_OK;
  }

  // The same against every block since the restart (block p in slot p - 1).
  int pass_gram(int m, const S* X, double* tab) {
    std::vector<int> sl(std::max(m - 1, 0));
    for (int p = 0; p < m - 1; ++p) sl[p] = p;
    return pass_gram_slots(sl.data(), m - 1, X, tab);
  }
  int pass_update(int m, const S* X, const double* tab, S* out) {
    std::vector<int> sl(std::max(m - 1, 0));
    for (int p = 0; p < m - 1; ++p) sl[p] = p;
    return pass_update_slots(sl.data(), m - 1, X, tab, out);
  }

  // Z <- M^{-1} Z = L^{-t} L^{-1} Z for the block Jacobi preconditioner:
  // level-scheduled triangular solves, in place.
  int apply_minv(S* Z) {
    Timed tm;
    const double lvl = (double)(c->levp_f.size() + c->levp_b.size());
    c->tstart(tm, ECG_K_PRECOND,
              4.0 * c->blk_bytes() + 2.0 * c->pl_nnz * 12.0 + 8.0 * c->n + 0.0 * lvl,
              4.0 * c->pl_nnz * c->t + 2.0 * c->n * c->t);
    for (size_t l = 0; l + 1 < c->levp_f.size(); ++l)
      HIP_TRY((launch_trsv_level<TPI, S>(c->lev_f + c->levp_f[l], c->levp_f[l + 1] - c->levp_f[l],
                                         c->pl_rp, c->pl_ci, c->pl_v, c->p_dinv, Z, c->st)));
    for (size_t l = 0; l + 1 < c->levp_b.size(); ++l)
      HIP_TRY((launch_trsv_level<TPI, S>(c->lev_b + c->levp_b[l], c->levp_b[l + 1] - c->levp_b[l],
                                         c->pu_rp, c->pu_ci, c->pu_v, c->p_dinv, Z, c->st)));
    c->tstop(tm);
    return ECG_OK;
  }

  // Split preconditioned s-step methods (Section 5): the first block after a
  // (re)start is M^{-1} T(r); later blocks start from M^{-1} A W_{m-1}
  // (A W_{m-1} = A U_{m-1} R_{m-1}^{-1} formed by scale_into), A-orthonormalized
  // by CGS2 against the previous two blocks
  // (SRE-CG) or every block since the restart (SRE-CG2), and MSDO-CG's first
  // block of an iteration is M^{-1} T(r_{k-1}) against every earlier block.
  int block_prec(int m, int slot, int p1, int p2, bool first) {
    const double bb = c->blk_bytes();
    int rc;
    const bool split = m == 1 || (c->o.variant == ECG_MSDO && first);
    S* Zp = (S*)c->Zp;
    if (split) {
      S* dst = m == 1 ? U(slot) : Zp;
      Timed tm;
      c->tstart(tm, ECG_K_TSPLIT, bb + 12.0 * c->n, 0.0);
      HIP_TRY((launch_tsplit<TPI, S>(c->r, c->dom, dst, c->n, c->grid, c->st)));
      c->tstop(tm);
      if ((rc = apply_minv(dst))) return rc;
      if (m == 1) return ECG_OK;
    } else {
      if ((rc = scale_into(AU(p1), rinv(p1), Zp))) return rc;   // A W_{m-1}
      if ((rc = apply_minv(Zp))) return rc;
    }
    std::vector<int> sl;
    if (c->o.variant == ECG_SRECG) {
      if (m >= 3) sl.push_back(p2);
      sl.push_back(p1);
    } else {
      for (int p = 0; p < m - 1; ++p) sl.push_back(p);
    }
    const int cnt = (int)sl.size();
    if ((rc = pass_gram_slots(sl.data(), cnt, Zp, c->ctab))) return rc;
    if ((rc = pass_update_slots(sl.data(), cnt, Zp, c->ctab, Zp))) return rc;
    if ((rc = pass_gram_slots(sl.data(), cnt, Zp, c->dtab))) return rc;
    return pass_update_slots(sl.data(), cnt, Zp, c->dtab, U(slot));
  }

  // s-step MSDO-CG (Section 3.2): the first block of an iteration after the
  // first is T(r_{k-1}), A-orthonormalised against every block since the
  // restart by two full CGS passes.
  int msdo_first(int m, int slot) {
    const double bb = c->blk_bytes();
    Timed tm;
    c->tstart(tm, ECG_K_TSPLIT, bb + 12.0 * c->n, 0.0);
    HIP_TRY((launch_tsplit<TPI, S>(c->r, c->dom, (S*)c->Zp, c->n, c->grid, c->st)));
    c->tstop(tm);
    int rc;
    if ((rc = pass_gram(m, (const S*)c->Zp, c->ctab))) return rc;
    if ((rc = pass_update(m, (const S*)c->Zp, c->ctab, (S*)c->Zp))) return rc;
    if ((rc = pass_gram(m, (const S*)c->Zp, c->dtab))) return rc;
    return pass_update(m, (const S*)c->Zp, c->dtab, U(slot));
  }

  // Pre-CholQR: Euclidean CholQR of the block before A-CholQR,
  // U <- U Re^{-1} with U^t U = Re^t Re.
  int pre_cholqr(int m, int slot) {
    constexpr int T2 = TPI * TPI;
    const double bb = c->blk_bytes();
    const double nt2 = (double)c->n * c->t * c->t;
    UGArgs<S> g{};
    g.X[0] = U(slot);
    g.P[0] = U(slot);
    g.n = c->n;
    g.rc = c->rc();
    int rc = ug(ECG_K_GRAM, 1, 1, true, false, g, bb, 2.0 * nt2);
    if (rc) return rc;
    TailArgs ta = tail0(m);
    ta.coef_out[0] = c->pre_rinv;
    if ((rc = reduce(gram_partials(TPI, c->grid), T2, TAIL_PRE, 1, ta))) return rc;
    UGArgs<S> u{};
    u.X[0] = U(slot);
    u.C[0] = c->pre_rinv;
    u.out = U(slot);
    u.n = c->n;
    u.rc = c->rc();
    return ug(ECG_K_UPDATE, 1, 0, false, true, u, 2.0 * bb, 2.0 * nt2);
  }

  // out = X R^{-1}: the A-image of an orthonormalized block from its stored
  // unnormalized A-image (keeps the raw blocks of the preconditioned and CA
  // forms at the scale of A W, not of a growing product of unnormalized
  // blocks)
  int scale_into(const S* X, const double* rinv_x, S* out) {
    const double bb = c->blk_bytes();
    const double nt2 = (double)c->n * c->t * c->t;
    UGArgs<S> u{};
    u.X[0] = X;
    u.C[0] = rinv_x;
    u.out = out;
    u.n = c->n;
    u.rc = c->rc();
    return ug(ECG_K_UPDATE, 1, 0, false, true, u, 2.0 * bb, 2.0 * nt2);
  }

  // Build block m (1-based since the last restart) into `slot`; p1, p2 are
  // the slots of blocks m-1 and m-2; `first`: the first block of an s-step
  // iteration.
  int block(int m, int slot, int p1, int p2, bool first, const Fold* fold) {
    const double bb = c->blk_bytes();
    const double nt2 = (double)c->n * c->t * c->t;
    if (c->prec != ECG_PREC_NONE) {
      int rc = block_prec(m, slot, p1, p2, first);
      if (rc) return rc;
    } else if (c->o.variant == ECG_MSDO && first && m >= 2) {
      int rc = msdo_first(m, slot);
      if (rc) return rc;
    } else if (c->o.variant != ECG_SRECG && m >= 4) {
      int rc = cgs_all(m, slot, fold);
      if (rc) return rc;
    } else if (m == 1) {
      Timed tm;
      c->tstart(tm, ECG_K_TSPLIT, bb + 12.0 * c->n, 0.0);
      HIP_TRY((launch_tsplit<TPI, S>(c->r, c->dom, U(slot), c->n, c->grid, c->st)));
      c->tstop(tm);
    } else {
      const int np = m >= 3 ? 2 : 1;
      UGArgs<S> ka{};
      ka.X[0] = AU(p1);
      ka.X[1] = U(p1);
      ka.X[2] = np == 2 ? U(p2) : nullptr;
      ka.C[0] = c->cnext;
      ka.C[1] = c->cnext + TPI * TPI;
      ka.C[2] = c->cnext + 2 * TPI * TPI;
      ka.P[0] = AU(p1);
      ka.P[1] = np == 2 ? AU(p2) : nullptr;
      ka.out = (S*)c->Zp;
      ka.n = c->n;
      ka.rc = c->rc();
      ka.tail = tail0(m);
      ka.tail.rinv_p1 = rinv(p1);
      ka.tail.rinv_p2 = np == 2 ? rinv(p2) : nullptr;
      set_fold(ka, fold);
      Timed tm;
      // update with np + 1 operands, np Grams (2 n t^2 flops each)
      c->tstart(tm, ECG_K_CGS_GRAM, (2.0 * np + 1.0) * bb + (fold ? 32.0 * c->n : 0.0),
                2.0 * nt2 * ((np + 1) + np) + (fold ? 4.0 * c->n * c->t : 0.0));
      HIP_TRY((launch_update_gram<TPI, S>(np + 1, np, false, true, TAIL_CGS, ka, c->grid, c->st)));
      c->tstop(tm);
      int rc = reduce(gram_partials(TPI, c->grid), np * TPI * TPI, TAIL_CGS, np, ka.tail);
      if (rc) return rc;

      UGArgs<S> kb{};
      kb.X[0] = (const S*)c->Zp;
      kb.X[1] = U(p1);
      kb.X[2] = np == 2 ? U(p2) : nullptr;
      kb.C[1] = c->dcoef;
      kb.C[2] = c->dcoef + TPI * TPI;
      kb.out = U(slot);
      kb.n = c->n;
      kb.rc = c->rc();
      kb.tail = tail0(m);
      Timed tm2;
      c->tstart(tm2, ECG_K_CGS_UPDATE, (np + 2.0) * bb, 2.0 * nt2 * np);
      HIP_TRY((launch_update_gram<TPI, S>(np + 1, 0, true, true, TAIL_NONE, kb, c->grid, c->st)));
      c->tstop(tm2);
    }
    return cholqr(m, slot, m >= 2 ? p1 : -1);
  }

  // A-orthonormalize the CGS2 output in `slot` against itself (Pre-CholQR
  // first when asked): the product A U with the Grams G, F, a = U^t r and,
  // with the previous block in slot p1 >= 0, E; the tail forms R^{-1}, beta
  // and the next block's first-pass coefficients.
  int cholqr(int m, int slot, int p1) {
    const double bb = c->blk_bytes();
    const double nt2 = (double)c->n * c->t * c->t;
    if (c->o.orth == ECG_PRECHOLQR) {
      int rc = pre_cholqr(m, slot);
      if (rc) return rc;
    }
    const bool prev = p1 >= 0;
    SpArgs<S, SA> sa{};
    sa.rowptr = c->rowptr;
    sa.colind = c->colind;
    sa.vals = avals();
    sa.Z = U(slot);
    sa.AZ = AU(slot);
    sa.AZprev = prev ? AU(p1) : nullptr;
    sa.rvec = c->r;
    sa.n = c->n;
    sa.max_row = c->max_row;
    sa.rc = c->rc();
    sa.tail = tail0(m);
    sa.tail.rinv_cur = rinv(slot);
    sa.tail.rinv_p1 = prev ? rinv(p1) : nullptr;
    sa.tail.beta = beta(slot);
    Timed tm;
    const int vb = std::is_same<SA, float>::value ? 4 : 8;
    // algorithmic flops: the product, the upper triangles of the symmetric
    // Grams G and F (n t (t + 1) each), E in full, a = Z^t r
    const double ntt1 = (double)c->n * c->t * (c->t + 1);
    c->tstart(tm, ECG_K_SPMM, c->csr_bytes(vb) + (prev ? 3.0 : 2.0) * bb + 8.0 * c->n,
              2.0 * c->nnz * c->t + 2.0 * ntt1 + (prev ? 2.0 * nt2 : 0.0) +
                  2.0 * c->n * c->t);
    HIP_TRY((launch_spmm<TPI, S, SA>(true, prev, TAIL_SPMM, sa, c->grid, c->st)));
    c->tstop(tm);
    return reduce(spmm_partials(TPI, c->grid, c->max_row), 3 * TPI * TPI + TPI, TAIL_SPMM, 0,
                  sa.tail);
  }

  // out = A X with no Grams (one step of the matrix powers of the CA forms)
  int power(const S* X, S* out) {
    SpArgs<S, SA> sa{};
    sa.rowptr = c->rowptr;
    sa.colind = c->colind;
    sa.vals = avals();
    sa.Z = X;
    sa.AZ = out;
    sa.n = c->n;
    sa.max_row = c->max_row;
    sa.rc = c->rc();
    Timed tm;
    const int vb = std::is_same<SA, float>::value ? 4 : 8;
    c->tstart(tm, ECG_K_SPMM, c->csr_bytes(vb) + 2.0 * c->blk_bytes(),
              2.0 * c->nnz * c->t);
    HIP_TRY((launch_spmm<TPI, S, SA>(false, false, TAIL_NONE, sa, c->grid, c->st)));
    c->tstop(tm);
    return ECG_OK;
  }

  // The CA-Arnoldi of Section 3.1 (ca = 2): the raw block W_j (T(r), or
  // A W_{j-1} = A U_{j-1} R_{j-1}^{-1}) and its raw powers A W_j, ..,
  // A^{s-1} W_j into slots[0 .. s-1], then each against q and the
  // iteration's earlier blocks (CGS2) and itself (A-CholQR) -- in exact
  // arithmetic the CGS2 of all s t columns against q and their A-CholQR.
  int ca_plain_blocks(int m0, const int* slots, const std::vector<int>& q, int last) {
    const double bb = c->blk_bytes();
    const bool prec = c->prec != ECG_PREC_NONE;
    int rc;
    if (m0 == 0 || c->o.variant == ECG_MSDO) {
      Timed tm;
      c->tstart(tm, ECG_K_TSPLIT, bb + 12.0 * c->n, 0.0);
      HIP_TRY((launch_tsplit<TPI, S>(c->r, c->dom, U(slots[0]), c->n, c->grid, c->st)));
      c->tstop(tm);
    } else if ((rc = scale_into(AU(last), rinv(last), U(slots[0])))) {
      return rc;
    }
    if (prec && (rc = apply_minv(U(slots[0])))) return rc;
    for (int i = 1; i < c->s; ++i) {
      if ((rc = power(U(slots[i - 1]), U(slots[i])))) return rc;
      if (prec && (rc = apply_minv(U(slots[i])))) return rc;
    }
    std::vector<int> sl = q;
    for (int i = 0; i < c->s; ++i) {
      if (i > 0) sl.push_back(slots[i - 1]);
      if ((rc = cgs2_slots(sl, U(slots[i]), U(slots[i])))) return rc;
      if ((rc = cholqr(m0 + 1 + i, slots[i], -1))) return rc;
    }
    return ECG_OK;
  }

  // CGS2 of X against the blocks in slots sl into `out` (X and out may be
  // the same block; with no blocks, a copy)
  int cgs2_slots(const std::vector<int>& sl, const S* X, S* out) {
    const int cnt = (int)sl.size();
    S* Zp = (S*)c->Zp;
    if (cnt == 0) {
      if (X != out)
        HIP_TRY(hipMemcpyAsync(out, X, (size_t)c->n * TPI * sizeof(S), hipMemcpyDeviceToDevice,
                               c->st));
      return ECG_OK;
    }
    int rc;
    if ((rc = pass_gram_slots(sl.data(), cnt, X, c->ctab))) return rc;
    if ((rc = pass_update_slots(sl.data(), cnt, X, c->ctab, Zp))) return rc;
    if ((rc = pass_gram_slots(sl.data(), cnt, Zp, c->dtab))) return rc;
    return pass_update_slots(sl.data(), cnt, Zp, c->dtab, out);
  }

  // The CA forms (Section 4, modified CA-Arnoldi A-orthonormalization):
  // blocks m0+1 .. m0+s of one iteration into slots[0 .. s-1]; q holds the
  // slots of the kept blocks (oldest first) and `last` the slot of the
  // previous iteration's last block.
  //   W_j: T(r) after a restart (every iteration for MSDO-CG), else
  //        A W_{j-1} = A U_{j-1} R_{j-1}^{-1}; against q (CGS2), then A-CholQR.
  //   powers: P_1 = A W_j from its stored A-image, P_i = A P_{i-1} (raw, in
  //        the slots of blocks j+i): the matrix powers of W_j.
  //   P_i: against q and W_j .. W_{j+i-1} (CGS2), then A-CholQR.  In exact
  //        arithmetic this is the CGS2 of [W_j, P_1, ..] against q followed
  //        by the A-CholQR of all s t columns at once, carried out block by
  //        block so that every small factorization stays t x t.
  // With a preconditioner every raw block is multiplied by M^{-1} (Section
  // 5): M^{-1} T(r), M^{-1} A W_{j-1}, P_i = M^{-1} A P_{i-1}.
  int ca_blocks(int m0, const int* slots, const std::vector<int>& q, int last) {
    const double bb = c->blk_bytes();
    const bool prec = c->prec != ECG_PREC_NONE;
    const int s = c->s;
    S* Zp = (S*)c->Zp;
    int rc;
    if (c->o.ca == 2) return ca_plain_blocks(m0, slots, q, last);
    if (m0 == 0 || c->o.variant == ECG_MSDO) {
      S* dst = q.empty() ? U(slots[0]) : Zp;
      Timed tm;
      c->tstart(tm, ECG_K_TSPLIT, bb + 12.0 * c->n, 0.0);
      HIP_TRY((launch_tsplit<TPI, S>(c->r, c->dom, dst, c->n, c->grid, c->st)));
      c->tstop(tm);
      if (prec && (rc = apply_minv(dst))) return rc;
      if (!q.empty() && (rc = cgs2_slots(q, Zp, U(slots[0])))) return rc;
    } else {
      if ((rc = scale_into(AU(last), rinv(last), Zp))) return rc;   // A W_{j-1}
      if (prec && (rc = apply_minv(Zp))) return rc;
      if ((rc = cgs2_slots(q, Zp, U(slots[0])))) return rc;
    }
    if ((rc = cholqr(m0 + 1, slots[0], -1))) return rc;
    // the raw powers of W_j (all formed before any is orthogonalized):
    // P_1 = A W_j = A U_j R_j^{-1}, P_i = A P_{i-1}
    for (int i = 1; i < s; ++i) {
      if (i == 1) {
        if ((rc = scale_into(AU(slots[0]), rinv(slots[0]), U(slots[1])))) return rc;
      } else if ((rc = power(U(slots[i - 1]), U(slots[i])))) {
        return rc;
      }
      if (prec && (rc = apply_minv(U(slots[i])))) return rc;
    }
    std::vector<int> sl = q;
    for (int i = 1; i < s; ++i) {
      sl.push_back(slots[i - 1]);
      if ((rc = cgs2_slots(sl, U(slots[i]), U(slots[i])))) return rc;
      if ((rc = cholqr(m0 + 1 + i, slots[i], -1))) return rc;
    }
    return ECG_OK;
  }

  // x2 = x_in + sum U beta, r2 = r_in - sum AU beta over the given blocks, and ||r2||
  int xr(const int* slots, int nb, const double* x_in, const double* r_in) {
    XRArgs<S> xa{};
    for (int i = 0; i < nb; ++i) {
      xa.U[i] = U(slots[i]);
      xa.AU[i] = AU(slots[i]);
      xa.beta[i] = beta(slots[i]);
    }
    xa.nb = nb;
    xa.x_in = x_in;
    xa.r_in = r_in;
    xa.x = c->x2;
    xa.r = c->r2;
    xa.n = c->n;
    xa.status_in = c->status;
    xa.rc = c->rc();
    xa.tail = tail0(0);
    Timed tm;
    c->tstart(tm, ECG_K_XR_UPDATE, 2.0 * nb * c->blk_bytes() + 32.0 * c->n,
              4.0 * nb * (double)c->n * c->t + 2.0 * c->n);
    const int g = (int)std::min<int64_t>((c->n + 63) / 64, c->grid);
    HIP_TRY((launch_xr<TPI, S>(xa, g, c->st)));
    c->tstop(tm);
    return reduce(g, 1, TAIL_NORM, 0, xa.tail);
  }

  int read_status(DevStatus* h) {
    HIP_TRY(hipMemcpyAsync(c->h_status, c->status, sizeof(DevStatus), hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    *h = *c->h_status;
    c->flush_timing();
    return ECG_OK;
  }

  int run(double tol, int maxit, double* hist, int cap, ecg_result* res) {
    int rc;
    int hl = 0;
    auto push = [&](double v) {
      if (hist && hl < cap) hist[hl] = v;
      ++hl;
    };
    const auto t_start = std::chrono::steady_clock::now();
    double rho0_log = 0.0;
    // opt-in progress line on stderr (long solves)
    auto progress = [&](const char* what, int k, int restarts, double rho) {
      if (c->o.progress_every <= 0 || rho0_log <= 0.0) return;
      const double ms = std::chrono::duration<double, std::milli>(
                            std::chrono::steady_clock::now() - t_start).count();
      std::fprintf(stderr, "ecg: %s iter %d restarts %d rho/rho0 %.3e  %.1f ms\n", what, k,
                   restarts, rho / rho0_log, ms);
      std::fflush(stderr);
    };
    DevStatus h{};
    HIP_TRY(hipMemsetAsync(c->status, 0, sizeof(DevStatus), c->st));
    if ((rc = resid(1))) return rc;
    if ((rc = read_status(&h))) return rc;
    const double rho0 = h.rho_true;
    res->rho0 = rho0;
    rho0_log = rho0;
    if (!std::isfinite(rho0)) return fail(ECG_EINVAL, "b or x0 contains a non-finite value");
    push(rho0);
    if (rho0 == 0.0) {
      res->relres = res->true_relres = 0.0;
      res->hist_len = std::min(hl, cap);
      return ECG_OK;
    }
    const double thr_final = tol * rho0;
    const double inner = c->o.precision == ECG_MIXED ? c->o.inner_tol : 0.0;
    double rho = rho0, rho_restart = rho0;
    int k = 0, restarts = 0, m = 0, nblocks = 0;
    int status = ECG_OK;
    int ns = c->nslot;
    const bool cg2 = c->o.variant != ECG_SRECG;   // every block since the restart is kept
    int slot_of[3] = {-1, -1, -1};   // slots of blocks m, m-1, m-2
    std::vector<int> since;          // CA forms: slots of the blocks since the restart
    while (true) {
      const double thr = std::max(inner * rho_restart, thr_final);
      while (rho > thr && k < maxit) {
        if (cg2 && m + c->s > c->nalloc && c->nalloc < ns) {
          // more block pairs: on allocation failure the blocks held so far
          // become the cap
          const int g = grow_slots(c, std::min(ns, m + c->s));
          if (g == ECG_ENOMEM) ns = c->nalloc;   // >= s from setup
          else if (g) return g;
        }
        if (cg2 && m > 0 && m + c->s > ns) {
          // every slot holds a block since the last restart: restart from x
          if ((rc = resid(1))) return rc;
          if ((rc = read_status(&h))) return rc;
          rho = h.rho_true;
          push(rho);
          ++restarts;
          progress("block-cap restart at", k, restarts, rho);
          rho_restart = rho;
          m = 0;
          slot_of[0] = slot_of[1] = slot_of[2] = -1;
          since.clear();
          continue;
        }
        int slots[kMaxS];
        if (c->o.ca) {
          // CA SRE-CG keeps the last s+1 blocks, the other forms all since
          // the restart
          const int kept = cg2 ? (int)since.size() : std::min((int)since.size(), c->s + 1);
          const std::vector<int> q(since.end() - kept, since.end());
          const int last = since.empty() ? -1 : since.back();
          const int m0 = m;
          for (int i = 0; i < c->s; ++i) {
            ++m;
            slots[i] = cg2 ? m - 1 : nblocks % ns;
            ++nblocks;
          }
          if ((rc = ca_blocks(m0, slots, q, last))) return rc;
          for (int i = 0; i < c->s; ++i) since.push_back(slots[i]);
          if (!cg2 && (int)since.size() > c->s + 1)
            since.erase(since.begin(), since.end() - (c->s + 1));
          if ((rc = xr(slots, c->s, c->x, c->r))) return rc;
        }
        for (int i = 0; i < (c->o.ca ? 0 : c->s); ++i) {
          ++m;
          const int slot = cg2 ? m - 1 : nblocks % ns;
          slot_of[2] = slot_of[1];
          slot_of[1] = slot_of[0];
          slot_of[0] = slot;
          // blocks after the first of an iteration carry the x/r
          // contribution of the block before them
          Fold f{};
          if (i >= 1 && c->prec == ECG_PREC_NONE) {
            f.beta = beta(slots[i - 1]);
            f.x_in = i == 1 ? c->x : c->x2;
            f.r_in = i == 1 ? c->r : c->r2;
          }
          const bool fold = i >= 1 && c->prec == ECG_PREC_NONE;
          if ((rc = block(m, slot, slot_of[1], slot_of[2], i == 0, fold ? &f : nullptr)))
            return rc;
          slots[i] = slot;
          ++nblocks;
        }
        // the last block's contribution (the earlier ones were carried by the
        // next block's first CGS kernel; with a preconditioner all s blocks
        // here); x2, r2 then hold the new iterate
        if (c->o.ca) {
          // x/r done above over the s blocks
        } else if (c->prec != ECG_PREC_NONE) {
          if ((rc = xr(slots, c->s, c->x, c->r))) return rc;
        } else if ((rc = xr(&slots[c->s - 1], 1, c->s == 1 ? c->x : c->x2,
                            c->s == 1 ? c->r : c->r2))) {
          return rc;
        }
        if ((rc = read_status(&h))) return rc;
        if (h.breakdown) {       // x, r stay the last completed iterate
          // a restart from x would repeat a breakdown in the first block (in
          // the CA forms: in the first iteration) since the last restart
          const int first = c->o.ca ? c->s : 1;
          if (h.breakdown_block > first && restarts < c->o.max_restarts) {
            // a rank-deficient block after the first one since the restart:
            // restart from the last completed iterate
            HIP_TRY(hipMemsetAsync(&c->status->breakdown, 0, 2 * sizeof(int), c->st));
            if ((rc = resid(1))) return rc;
            if ((rc = read_status(&h))) return rc;
            rho = h.rho_true;
            push(rho);
            ++restarts;
            progress("breakdown restart at", k, restarts, rho);
            rho_restart = rho;
            m = 0;
            slot_of[0] = slot_of[1] = slot_of[2] = -1;
            since.clear();
            continue;
          }
          status = ECG_BREAKDOWN;
          break;
        }
        std::swap(c->x, c->x2);
        std::swap(c->r, c->r2);
        rho = h.rho;
        ++k;
        push(rho);
        if (c->o.progress_every > 0 && k % c->o.progress_every == 0)
          progress("", k, restarts, rho);
        c->last_nb = c->s;
        for (int i = 0; i < c->s; ++i) c->last_slots[i] = slots[i];
      }
      if (status == ECG_BREAKDOWN) break;
      if (rho > thr) {
        status = ECG_MAXIT;
        break;
      }
      if ((rc = resid(1))) return rc;   // r <- b - A x (true residual)
      if ((rc = read_status(&h))) return rc;
      const double tau = h.rho_true;
      if (tau <= thr_final) {
        status = ECG_OK;
        rho = tau;
        break;
      }
      if (restarts >= c->o.max_restarts || k >= maxit) {
        status = k < maxit ? ECG_STAGNATED : ECG_MAXIT;
        rho = tau;
        break;
      }
      rho = tau;
      push(tau);
      ++restarts;
      progress("true-residual restart at", k, restarts, tau);
      rho_restart = tau;
      m = 0;
      slot_of[0] = slot_of[1] = slot_of[2] = -1;
      since.clear();
    }
    // final true residual (the residual kernel leaves r = b - A x)
    if ((rc = resid(1))) return rc;
    if ((rc = read_status(&h))) return rc;
    res->iters = k;
    res->restarts = restarts;
    res->blocks = nblocks;
    res->relres = rho / rho0;
    res->true_relres = h.rho_true / rho0;
    res->hist_len = std::min(hl, cap);
    progress("done at", k, restarts, h.rho_true);
    return status;
  }
};

template <int TPI>
int run_tpi(ecg_ctx* c, double tol, int maxit, double* hist, int cap, ecg_result* res) {
  if (c->o.precision == ECG_MIXED) {
    Engine<TPI, float, float> e{c};
    return e.run(tol, maxit, hist, cap, res);
  }
  Engine<TPI, double, double> e{c};
  return e.run(tol, maxit, hist, cap, res);
}

}  // namespace

namespace {
int solve_impl(ecg_ctx* c, const double* b, double* x, double tol, int32_t maxit,
               double* reshist, int32_t reshist_cap, ecg_result* res) {
  if (!c || !b || !x) return fail(ECG_EINVAL, "NULL argument");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(ECG_EINVAL, "tol must be positive and finite");
  if (maxit < 0) return fail(ECG_EINVAL, "maxit must be >= 0");
  if (reshist_cap < 0) return fail(ECG_EINVAL, "reshist_cap must be >= 0");
  std::memset(&c->stats, 0, sizeof(c->stats));
  c->last_nb = 0;
  const bool dev = c->o.device_ptrs == 1;
  const hipMemcpyKind in = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const hipMemcpyKind outk = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (c->perm) {
    // into the solver's row order (host arrays through the spare vectors)
    const double* bs = b;
    const double* xs = x;
    if (!dev) {
      HIP_TRY(hipMemcpyAsync(c->x2, b, sizeof(double) * c->n, in, c->st));
      HIP_TRY(hipMemcpyAsync(c->r2, x, sizeof(double) * c->n, in, c->st));
      bs = c->x2;
      xs = c->r2;
    }
    HIP_TRY(launch_pack(bs, 1, c->b, 1, c->n, c->perm, c->st));
    HIP_TRY(launch_pack(xs, 1, c->x, 1, c->n, c->perm, c->st));
  } else {
    HIP_TRY(hipMemcpyAsync(c->b, b, sizeof(double) * c->n, in, c->st));
    HIP_TRY(hipMemcpyAsync(c->x, x, sizeof(double) * c->n, in, c->st));
  }
  HIP_TRY(hipEventRecord(c->ev_solve0, c->st));
  int st;
  switch (c->tpi) {
    case 16: st = run_tpi<16>(c, tol, maxit, reshist, reshist_cap, res); break;
    case 32: st = run_tpi<32>(c, tol, maxit, reshist, reshist_cap, res); break;
    default: st = run_tpi<64>(c, tol, maxit, reshist, reshist_cap, res); break;
  }
  if (st < 0) {
    // a failed solve leaves no timings behind for the next one
    (void)hipStreamSynchronize(c->st);
    c->flush_timing();
    std::memset(&c->stats, 0, sizeof(c->stats));
    return st;
  }
  HIP_TRY(hipEventRecord(c->ev_solve1, c->st));
  if (c->perm) {
    // back to the caller's row order (x2 is free after the solve)
    if (dev) {
      HIP_TRY(launch_unpack(c->x, 1, x, 1, c->n, c->perm, c->st));
    } else {
      HIP_TRY(launch_unpack(c->x, 1, c->x2, 1, c->n, c->perm, c->st));
      HIP_TRY(hipMemcpyAsync(x, c->x2, sizeof(double) * c->n, outk, c->st));
    }
  } else {
    HIP_TRY(hipMemcpyAsync(x, c->x, sizeof(double) * c->n, outk, c->st));
  }
  HIP_TRY(hipStreamSynchronize(c->st));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, c->ev_solve0, c->ev_solve1));
  res->solve_ms = ms;
  return st;
}
}  // namespace

extern "C" int ecg_solve_ex(ecg_ctx* c, const double* b, double* x, double tol, int32_t maxit,
                            double* reshist, int32_t reshist_cap, ecg_result* res) {
  ecg_result tmp{};
  if (!res) res = &tmp;
  std::memset(res, 0, sizeof(*res));
  const int st = solve_impl(c, b, x, tol, maxit, reshist, reshist_cap, res);
  res->status = st;
  return st;
}

extern "C" int ecg_solve(ecg_ctx* c, const double* b, double* x, double tol, int32_t maxit,
                         int32_t* iters, double* reshist, int32_t* reshist_len,
                         double* true_relres) {
  ecg_result res{};
  int cap = 0;
  if (reshist) {
    // rho_0, one value per iteration, one per residual replacement and one
    // per block-cap restart (at most one per iteration)
    const int64_t want = c ? 2 * (int64_t)maxit + c->o.max_restarts + 2 : 0;
    cap = (int)std::min<int64_t>(want, INT32_MAX);
  }
  const int st = solve_impl(c, b, x, tol, maxit, reshist, cap, &res);
  if (iters) *iters = res.iters;
  if (reshist_len) *reshist_len = res.hist_len;
  if (true_relres) *true_relres = res.true_relres;
  return st;
}

extern "C" int ecg_sddmm(ecg_ctx* c, const double* lambda, const double* x, double* grad_vals) {
  if (!c || !lambda || !x || !grad_vals) return fail(ECG_EINVAL, "NULL argument");
  const bool dev = c->o.device_ptrs == 1;
  const double *dl = lambda, *dx = x;
  double* dg = grad_vals;
  double *tl = nullptr, *tx = nullptr, *tg = nullptr;
  if (!dev) {
    size_t tot = 0;
    if (dalloc(&tl, c->n, tot) || dalloc(&tx, c->n, tot) || dalloc(&tg, c->nnz, tot)) {
      if (tl) (void)hipFree(tl);
      if (tx) (void)hipFree(tx);
      if (tg) (void)hipFree(tg);
      return ECG_ENOMEM;
    }
    (void)hipMemcpyAsync(tl, lambda, sizeof(double) * c->n, hipMemcpyHostToDevice, c->st);
    (void)hipMemcpyAsync(tx, x, sizeof(double) * c->n, hipMemcpyHostToDevice, c->st);
    dl = tl;
    dx = tx;
    dg = tg;
  }
  hipError_t e = launch_sddmm(c->rowptr, c->colind, dl, dx, dg, c->n, c->perm, c->emap, c->st);
  if (e == hipSuccess && !dev)
    e = hipMemcpyAsync(grad_vals, tg, sizeof(double) * c->nnz, hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (tl) (void)hipFree(tl);
  if (tx) (void)hipFree(tx);
  if (tg) (void)hipFree(tg);
  if (e != hipSuccess) return fail(ECG_EDEVICE, std::string("sddmm: ") + hipGetErrorString(e));
  return ECG_OK;
}

namespace {
int ensure_scratch(ecg_ctx* c) {
  size_t tot = 0;
  if (!c->scratch) {
    int rc = dalloc(&c->scratch, (size_t)c->n * 64, tot);
    if (rc) return rc;
  }
  if (!c->scratch2) {
    int rc = dalloc(&c->scratch2, (size_t)c->n * 64, tot);
    if (rc) return rc;
  }
  return ECG_OK;
}

template <int TPI>
int spmm_op(ecg_ctx* c, double* Xp, double* Yp) {
  SpArgs<double, double> sa{};
  sa.rowptr = c->rowptr;
  sa.colind = c->colind;
  sa.vals = c->vals;
  sa.Z = Xp;
  sa.AZ = Yp;
  sa.n = c->n;
  sa.max_row = c->max_row;
  sa.rc = c->rc();
  const int g = (int)std::min<int64_t>((c->n + rows_per_wg(TPI) - 1) / rows_per_wg(TPI), 1024);
  HIP_TRY((launch_spmm<TPI, double, double>(false, false, TAIL_NONE, sa, g, c->st)));
  return ECG_OK;
}
}  // namespace

extern "C" int ecg_spmm(ecg_ctx* c, const double* X, double* Y, int32_t k) {
  if (!c || !X || !Y) return fail(ECG_EINVAL, "NULL argument");
  if (k < 1 || k > 64) return fail(ECG_EINVAL, "k must be in [1, 64]");
  int rc = ensure_scratch(c);
  if (rc) return rc;
  const bool dev = c->o.device_ptrs == 1;
  const int tpi = pick_tpi(k);
  double* Xin = c->scratch2;   // row-major n x k staging for host inputs
  if (dev) Xin = (double*)X;
  else HIP_TRY(hipMemcpyAsync(Xin, X, sizeof(double) * c->n * k, hipMemcpyHostToDevice, c->st));
  // pack to n x tpi in scratch, product into scratch2 (after the pack consumed it)
  HIP_TRY(launch_pack(Xin, k, c->scratch, tpi, c->n, c->perm, c->st));
  switch (tpi) {
    case 16: rc = spmm_op<16>(c, c->scratch, c->scratch2); break;
    case 32: rc = spmm_op<32>(c, c->scratch, c->scratch2); break;
    default: rc = spmm_op<64>(c, c->scratch, c->scratch2); break;
  }
  if (rc) return rc;
  if (dev) {
    HIP_TRY(launch_unpack(c->scratch2, tpi, Y, k, c->n, c->perm, c->st));
  } else {
    HIP_TRY(launch_unpack(c->scratch2, tpi, c->scratch, k, c->n, c->perm, c->st));
    HIP_TRY(hipMemcpyAsync(Y, c->scratch, sizeof(double) * c->n * k, hipMemcpyDeviceToHost, c->st));
  }
  HIP_TRY(hipStreamSynchronize(c->st));
  return ECG_OK;
}

extern "C" int ecg_spmm_noalloc(ecg_ctx* c, const double* X, double* Y, int32_t k) {
  if (!c || !X || !Y) return fail(ECG_EINVAL, "NULL argument");
  if (k < 1 || k > 64) return fail(ECG_EINVAL, "k must be in [1, 64]");
  const int tpi = pick_tpi(k);
  if (c->n * tpi > (int64_t)ECG_SPMM_NOALLOC_MAX)
    return fail(ECG_EINVAL, "ecg_spmm_noalloc: n x padded width = " + std::to_string(c->n) +
                                " x " + std::to_string(tpi) + " exceeds ECG_SPMM_NOALLOC_MAX (" +
                                std::to_string(ECG_SPMM_NOALLOC_MAX) + ")");
  double* base = noalloc_scratch(c->dev);
  if (!base) return fail(ECG_EDEVICE, "ecg_spmm_noalloc: no staging array for device " +
                                          std::to_string(c->dev));
  const bool dev = c->o.device_ptrs == 1;
  const size_t blk = (size_t)c->n * tpi;
  double* Xp = base;         // packed input, n x tpi (every entry written by the pack)
  double* Yp = base + blk;   // product, n x tpi (every entry written by the product)
  // host input: staged row-major n x k in Yp, which the product overwrites
  // only after the pack has consumed it (stream order)
  const double* Xin = X;
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(Yp, X, sizeof(double) * c->n * k, hipMemcpyHostToDevice, c->st));
    Xin = Yp;
  }
  HIP_TRY(launch_pack(Xin, k, Xp, tpi, c->n, c->perm, c->st));
  int rc;
  switch (tpi) {
    case 16: rc = spmm_op<16>(c, Xp, Yp); break;
    case 32: rc = spmm_op<32>(c, Xp, Yp); break;
    default: rc = spmm_op<64>(c, Xp, Yp); break;
  }
  if (rc) return rc;
  if (dev) {
    HIP_TRY(launch_unpack(Yp, tpi, Y, k, c->n, c->perm, c->st));
  } else {   // unpacked into Xp (free once the product has read it), then copied out
    HIP_TRY(launch_unpack(Yp, tpi, Xp, k, c->n, c->perm, c->st));
    HIP_TRY(hipMemcpyAsync(Y, Xp, sizeof(double) * c->n * k, hipMemcpyDeviceToHost, c->st));
  }
  HIP_TRY(hipStreamSynchronize(c->st));
  return ECG_OK;
}

extern "C" int ecg_tsplit(ecg_ctx* c, const double* r, double* Z) {
  if (!c || !r || !Z) return fail(ECG_EINVAL, "NULL argument");
  int rc = ensure_scratch(c);
  if (rc) return rc;
  const bool dev = c->o.device_ptrs == 1;
  double* rin = c->scratch2;
  if (dev) rin = (double*)r;
  else HIP_TRY(hipMemcpyAsync(rin, r, sizeof(double) * c->n, hipMemcpyHostToDevice, c->st));
  if (c->perm) {   // r in the solver's row order (x2 is free between solves)
    HIP_TRY(launch_pack(rin, 1, c->x2, 1, c->n, c->perm, c->st));
    rin = c->x2;
  }
  double* out = c->scratch;
  switch (c->tpi) {
    case 16: HIP_TRY((launch_tsplit<16, double>(rin, c->dom, out, c->n, 0, c->st))); break;
    case 32: HIP_TRY((launch_tsplit<32, double>(rin, c->dom, out, c->n, 0, c->st))); break;
    default: HIP_TRY((launch_tsplit<64, double>(rin, c->dom, out, c->n, 0, c->st))); break;
  }
  double* dst = dev ? Z : c->scratch2;
  HIP_TRY(launch_unpack(out, c->tpi, dst, c->t, c->n, c->perm, c->st));
  if (!dev)
    HIP_TRY(hipMemcpyAsync(Z, dst, sizeof(double) * c->n * c->t, hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  return ECG_OK;
}

extern "C" int ecg_get_basis(ecg_ctx* c, double* V, double* AV) {
  if (!c || !V || !AV) return fail(ECG_EINVAL, "NULL argument");
  if (c->last_nb <= 0) return fail(ECG_EINVAL, "no completed iteration");
  const bool dev = c->o.device_ptrs == 1;
  const int st = c->last_nb * c->t;
  size_t tot = 0;
  double* dv = nullptr;
  double* dav = nullptr;
  if (!dev) {
    if (dalloc(&dv, (size_t)c->n * st, tot) || dalloc(&dav, (size_t)c->n * st, tot)) {
      if (dv) (void)hipFree(dv);
      return ECG_ENOMEM;
    }
  } else {
    dv = V;
    dav = AV;
  }
  hipError_t e = hipSuccess;
  for (int i = 0; i < c->last_nb && e == hipSuccess; ++i) {
    const int slot = c->last_slots[i];
    const double* ri = c->rinv + (size_t)slot * c->T2();
    const bool mixed = c->o.precision == ECG_MIXED;
#define EXP(TPI)                                                                                \
  if (mixed) {                                                                                  \
    e = launch_basis_export<TPI, float>((const float*)c->U[slot], ri, dv, c->n, c->t, st,       \
                                        i * c->t, c->perm, c->st);                                       \
    if (e == hipSuccess)                                                                        \
      e = launch_basis_export<TPI, float>((const float*)c->AU[slot], ri, dav, c->n, c->t, st,   \
                                          i * c->t, c->perm, c->st);                                     \
  } else {                                                                                      \
    e = launch_basis_export<TPI, double>((const double*)c->U[slot], ri, dv, c->n, c->t, st,     \
                                         i * c->t, c->perm, c->st);                                      \
    if (e == hipSuccess)                                                                        \
      e = launch_basis_export<TPI, double>((const double*)c->AU[slot], ri, dav, c->n, c->t, st, \
                                           i * c->t, c->perm, c->st);                                    \
  }
    if (c->tpi == 16) { EXP(16) }
    else if (c->tpi == 32) { EXP(32) }
    else { EXP(64) }
#undef EXP
  }
  if (e == hipSuccess && !dev) {
    e = hipMemcpyAsync(V, dv, sizeof(double) * c->n * st, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(AV, dav, sizeof(double) * c->n * st, hipMemcpyDeviceToHost, c->st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (!dev) {
    (void)hipFree(dv);
    (void)hipFree(dav);
  }
  if (e != hipSuccess) return fail(ECG_EDEVICE, std::string("get_basis: ") + hipGetErrorString(e));
  return ECG_OK;
}

namespace {

void free_prec(ecg_ctx* c) {
  auto f = [](auto*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
  };
  f(c->pl_rp); f(c->pl_ci); f(c->pl_v); f(c->pu_rp); f(c->pu_ci); f(c->pu_v); f(c->p_dinv);
  f(c->lev_f); f(c->lev_b);
  c->levp_f.clear();
  c->levp_b.clear();
  c->pl_nnz = 0;
  c->prec = ECG_PREC_NONE;
}

// Rows grouped by level (level[i] from 0): rows of level l are
// out[off[l] .. off[l+1]), increasing within a level.
void bucket_levels(const std::vector<int>& level, std::vector<int32_t>& out, std::vector<int>& off) {
  const int64_t n = (int64_t)level.size();
  int nl = 0;
  for (int v : level) nl = std::max(nl, v + 1);
  off.assign(nl + 1, 0);
  for (int v : level) off[v + 1]++;
  for (int l = 0; l < nl; ++l) off[l + 1] += off[l];
  std::vector<int> pos(off.begin(), off.end() - 1);
  out.resize(n);
  for (int64_t i = 0; i < n; ++i) out[pos[level[i]]++] = (int32_t)i;
}

}  // namespace

extern "C" int ecg_set_preconditioner(ecg_ctx* c, int32_t kind, const int32_t* blocks) {
  if (!c) return fail(ECG_EINVAL, "NULL context");
  if (kind != ECG_PREC_NONE && kind != ECG_PREC_BJ_IC0 && kind != ECG_PREC_BJ_CHOL)
    return fail(ECG_EINVAL, "bad kind");
  free_prec(c);
  if (kind == ECG_PREC_NONE) return ECG_OK;
  if (!blocks) return fail(ECG_EINVAL, "blocks is NULL");
  const int64_t n = c->n, nnz = c->nnz;
  const bool dev = c->o.device_ptrs == 1;
  // the solver's matrix, domains and row order on the host
  std::vector<int32_t> rp(n + 1), ci(nnz), dom(n), perm, bl(n);
  std::vector<double> av(nnz);
  HIP_TRY(hipMemcpy(rp.data(), c->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(ci.data(), c->colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(av.data(), c->vals, sizeof(double) * nnz, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(dom.data(), c->dom, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  if (c->perm) {
    perm.resize(n);
    HIP_TRY(hipMemcpy(perm.data(), c->perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  }
  std::vector<int32_t> bc;
  const int32_t* bv = blocks;
  if (dev) {
    bc.resize(n);
    HIP_TRY(hipMemcpy(bc.data(), blocks, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    bv = bc.data();
  }
  int32_t nb = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t b = bv[perm.empty() ? i : perm[i]];
    if (b < 0) return fail(ECG_EINVAL, "negative preconditioner block");
    bl[i] = b;
    nb = std::max(nb, b + 1);
  }
  // every block inside one domain (then T and M^{-1} commute, Section 5)
  std::vector<int32_t> bdom(nb, -1);
  for (int64_t i = 0; i < n; ++i) {
    if (bdom[bl[i]] < 0) bdom[bl[i]] = dom[i];
    else if (bdom[bl[i]] != dom[i])
      return fail(ECG_EINVAL, "preconditioner block " + std::to_string(bl[i]) +
                                  " spans more than one domain");
  }
  std::vector<int64_t> lp(n + 1, 0);
  std::vector<int32_t> lc;
  std::vector<double> lv, diag(n);
  lc.reserve((size_t)(nnz - n) / 2 + 16);
  lv.reserve((size_t)(nnz - n) / 2 + 16);
  std::vector<std::pair<int32_t, double>> row;
  if (kind == ECG_PREC_BJ_CHOL) {
    // complete Cholesky of the block diagonal part, row by row in the
    // solver's order (up-looking): row i of L solves L(0:i-1, 0:i-1) l =
    // A(0:i-1, i) over i's block by a sparse forward substitution; a
    // nonzero l_j spreads to the rows p of column j computed so far, which
    // is where the fill comes from
    constexpr int64_t kMaxFactor = int64_t(1) << 28;   // entries of L
    std::vector<std::vector<std::pair<int32_t, double>>> colL(n);
    std::vector<double> xa(n, 0.0);
    std::vector<int64_t> mark(n, -1);
    std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> heap;
    for (int64_t i = 0; i < n; ++i) {
      double aii = 0.0;
      for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t j = ci[e];
        if (j == i) {
          aii += av[e];
        } else if (j < i && bl[j] == bl[i]) {
          xa[j] += av[e];
          if (mark[j] != i) {
            mark[j] = i;
            heap.push(j);
          }
        }
      }
      double d = aii;
      while (!heap.empty()) {
        const int32_t j = heap.top();
        heap.pop();
        const double lij = xa[j] / diag[j];
        xa[j] = 0.0;
        lc.push_back(j);
        lv.push_back(lij);
        d -= lij * lij;
        for (const auto& pl : colL[j]) {
          xa[pl.first] -= pl.second * lij;
          if (mark[pl.first] != i) {
            mark[pl.first] = i;
            heap.push(pl.first);
          }
        }
      }
      if (!(d > 0.0) || !std::isfinite(d))
        return fail(ECG_EINVAL, "Cholesky pivot of row " + std::to_string(i) + " is not positive");
      diag[i] = std::sqrt(d);
      for (int64_t a = lp[i]; a < (int64_t)lc.size(); ++a) colL[lc[a]].emplace_back((int32_t)i, lv[a]);
      lp[i + 1] = (int64_t)lc.size();
      if ((int64_t)lc.size() > kMaxFactor)
        return fail(ECG_ENOMEM, "complete Cholesky factor beyond " + std::to_string(kMaxFactor) +
                                    " entries (blocks too large)");
    }
  }
  // IC(0) of the block diagonal part, row by row in the solver's order:
  // L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj over the pattern, L_ii =
  // sqrt(A_ii - sum L_ik^2)
  for (int64_t i = 0; kind == ECG_PREC_BJ_IC0 && i < n; ++i) {
    row.clear();
    double aii = 0.0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int32_t j = ci[e];
      if (j == i) aii += av[e];
      else if (j < i && bl[j] == bl[i]) row.emplace_back(j, av[e]);
    }
    std::sort(row.begin(), row.end());
    const int64_t base = (int64_t)lc.size();
    for (auto& jv : row) {
      const int32_t j = jv.first;
      double acc = jv.second;
      // sum over k < j in both row i (computed so far) and row j of L
      int64_t a = base, b = lp[j];
      const int64_t ae = (int64_t)lc.size(), be = lp[j + 1];
      while (a < ae && b < be) {
        if (lc[a] == lc[b]) acc -= lv[a++] * lv[b++];
        else if (lc[a] < lc[b]) ++a;
        else ++b;
      }
      lc.push_back(j);
      lv.push_back(acc / diag[j]);
    }
    double d = aii;
    for (int64_t a = base; a < (int64_t)lc.size(); ++a) d -= lv[a] * lv[a];
    if (!(d > 0.0) || !std::isfinite(d))
      return fail(ECG_EINVAL, "IC(0) pivot of row " + std::to_string(i) + " is not positive");
    diag[i] = std::sqrt(d);
    lp[i + 1] = (int64_t)lc.size();
  }
  const int64_t ln = (int64_t)lc.size();
  if (ln >= (int64_t(1) << 31)) return fail(ECG_EINVAL, "factor too large");
  // L^t (strictly upper) by rows
  std::vector<int32_t> up(n + 1, 0), uc(ln);
  std::vector<double> uv(ln);
  for (int64_t a = 0; a < ln; ++a) up[lc[a] + 1]++;
  for (int64_t i = 0; i < n; ++i) up[i + 1] += up[i];
  {
    std::vector<int32_t> pos(up.begin(), up.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t a = lp[i]; a < lp[i + 1]; ++a) {
        uc[pos[lc[a]]] = (int32_t)i;
        uv[pos[lc[a]]++] = lv[a];
      }
  }
  // levels: forward over L, backward over L^t
  std::vector<int> lf(n, 0), lb(n, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t a = lp[i]; a < lp[i + 1]; ++a) lf[i] = std::max(lf[i], lf[lc[a]] + 1);
  for (int64_t i = n - 1; i >= 0; --i)
    for (int32_t a = up[i]; a < up[i + 1]; ++a) lb[i] = std::max(lb[i], lb[uc[a]] + 1);
  std::vector<int32_t> rows_f, rows_b;
  bucket_levels(lf, rows_f, c->levp_f);
  bucket_levels(lb, rows_b, c->levp_b);
  std::vector<int32_t> lp32(n + 1);
  std::vector<double> dinv(n);
  for (int64_t i = 0; i <= n; ++i) lp32[i] = (int32_t)lp[i];
  for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0 / diag[i];
  size_t tot = 0;
  int rc = 0;
  auto upl = [&](auto** dst, const auto& vec) -> int {
    using T = typename std::remove_reference<decltype(vec)>::type::value_type;
    int r = dalloc(dst, vec.size(), tot);
    if (r) return r;
    HIP_TRY(hipMemcpy(*dst, vec.data(), sizeof(T) * vec.size(), hipMemcpyHostToDevice));
    return ECG_OK;
  };
  if ((rc = upl(&c->pl_rp, lp32)) || (rc = upl(&c->pl_ci, lc)) || (rc = upl(&c->pl_v, lv)) ||
      (rc = upl(&c->pu_rp, up)) || (rc = upl(&c->pu_ci, uc)) || (rc = upl(&c->pu_v, uv)) ||
      (rc = upl(&c->p_dinv, dinv)) || (rc = upl(&c->lev_f, rows_f)) ||
      (rc = upl(&c->lev_b, rows_b))) {
    free_prec(c);
    return rc;
  }
  c->pl_nnz = ln;
  c->prec = kind;
  return ECG_OK;
}

extern "C" int ecg_domain_order(ecg_ctx* c, int32_t* order) {
  if (!c || !order) return fail(ECG_EINVAL, "NULL argument");
  const bool dev = c->o.device_ptrs == 1;
  std::vector<int32_t> h;
  if (!c->perm) {
    h.resize(c->n);
    for (int64_t i = 0; i < c->n; ++i) h[i] = (int32_t)i;
    HIP_TRY(hipMemcpy(order, h.data(), sizeof(int32_t) * c->n,
                      dev ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
    return ECG_OK;
  }
  HIP_TRY(hipMemcpyAsync(order, c->perm, sizeof(int32_t) * c->n,
                         dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  return ECG_OK;
}

extern "C" int ecg_last_stats(ecg_ctx* c, ecg_stats* st) {
  if (!c || !st) return fail(ECG_EINVAL, "NULL argument");
  *st = c->stats;
  return ECG_OK;
}
