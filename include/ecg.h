/*
 * ecg.h -- C ABI of the s-step enlarged Conjugate Gradient solver for one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Moufawad, "Numerical Stability of s-step Enlarged Krylov Subspace
 * Conjugate Gradient methods" (arXiv 1804.10629).  The problem is A x = b
 * with A (n x n) symmetric positive definite (Section 3.1, the input lines
 * of the s-step algorithms).  The residual is split over t domains of the
 * graph of A by the operator T (Section 2); every s-step iteration builds
 * s*t A-orthonormal basis vectors V of the enlarged Krylov subspace and
 * updates alpha = V^t r, x += V alpha, r -= A V alpha (eqs (1)-(3) and the
 * algorithms "s-step SRE-CG" and "s-step SRE-CG2" of Section 3.1, "s-step
 * MSDO-CG" of Section 3.2).
 *
 * Conventions
 *   - Every function returning int returns an ecg status: 0 (ECG_OK),
 *     a positive solver outcome, or a negative error.  No C++ exception
 *     crosses this interface.
 *   - Matrices are CSR with 0-based int32 indices, rows of the caller's
 *     ordering; dense n x k blocks are row-major (k values per row,
 *     contiguous).
 *   - Array arguments are host pointers, unless the context was created
 *     with opts.device_ptrs = 1, in which case every array argument of
 *     calls on that context (setup included) is a device pointer on the
 *     current HIP device.  The caller keeps ownership of all its arrays;
 *     the library copies what it keeps.
 *   - All work is enqueued on opts.hip_stream (0 = the null stream) and the
 *     calls return after it has completed.  A context is not re-entrant:
 *     calls on one context must not overlap.  Distinct contexts are
 *     independent.
 */
#ifndef ECG_H
#define ECG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define ECG_OK          0  /* converged: true residual <= tol * ||b - A x0|| */
#define ECG_MAXIT       1  /* iteration budget spent; x is the last iterate */
#define ECG_BREAKDOWN   2  /* a Cholesky pivot of a basis Gram matrix was <= 0
                              or not finite in the first block after a
                              (re)start (later blocks restart the solve from
                              the last completed iterate, at most
                              opts.max_restarts times); x is the last
                              completed iterate */
#define ECG_STAGNATED   3  /* the recursive residual met tol but the true
                              residual did not, after opts.max_restarts
                              residual replacements */
#define ECG_EINVAL     -1  /* invalid argument (message: ecg_last_error) */
#define ECG_ENOMEM     -2  /* device allocation failed */
#define ECG_EDEVICE    -3  /* HIP runtime error or no usable gfx950 device */
#define ECG_ENOTSUP    -4  /* valid request the library does not support */

/* ---- options ----------------------------------------------------------- */
enum ecg_variant   { ECG_SRECG = 0,   /* s-step SRE-CG: each block against the
                                         previous two (Section 3.1) */
                     ECG_SRECG2 = 1,  /* s-step SRE-CG2: against every block
                                         since the last (re)start */
                     ECG_MSDO = 2     /* s-step MSDO-CG (Section 3.2): as
                                         SRE-CG2, but the first block of every
                                         iteration is T(r_{k-1}) */ };
enum ecg_orth      { ECG_ACHOLQR = 0, ECG_PRECHOLQR = 1 };
enum ecg_precond   { ECG_PREC_NONE = 0,   /* no preconditioner */
                     ECG_PREC_BJ_IC0 = 1, /* block Jacobi, IC(0) blocks (Section 5) */
                     ECG_PREC_BJ_CHOL = 2 /* block Jacobi, complete Cholesky blocks
                                             (Section 5); the factor's fill grows
                                             with the blocks: at most 2^28 entries */ };
enum ecg_precision { ECG_FP64 = 0,    /* everything in binary64 */
                     ECG_MIXED = 1    /* binary32 basis blocks and matrix values
                                         for the basis product; Gram matrices,
                                         Cholesky factors, alpha, x and r in
                                         binary64; residual replacement in
                                         binary64 whenever the recursive
                                         residual has dropped by inner_tol */ };

typedef struct ecg_opts {
  int32_t variant;        /* enum ecg_variant (default ECG_SRECG) */
  int32_t orth;           /* enum ecg_orth (default ECG_ACHOLQR) */
  int32_t precision;      /* enum ecg_precision (default ECG_FP64) */
  int32_t device_ptrs;    /* 0: host arrays, 1: device arrays (default 0) */
  double  inner_tol;      /* ECG_MIXED: restart from the true residual when the
                             recursive residual is <= inner_tol times the one
                             at the last restart (default 1e-4; ignored in
                             ECG_FP64) */
  int32_t max_restarts;   /* bound on residual replacements (default 20) */
  int32_t q_cap_blocks;   /* ECG_SRECG2, ECG_MSDO: blocks kept since the last
                             restart; when another s would exceed it the
                             solve restarts from x.  0 = as many as
                             ws_cap_bytes allows, at most 2048; otherwise at
                             least s (default 0) */
  int64_t ws_cap_bytes;   /* device workspace cap; 0 = 90% of free memory */
  void*   hip_stream;     /* hipStream_t to run on; NULL = null stream */
  int32_t collect_stats;  /* 1: time every kernel with HIP events (ecg_last_stats) */
  int32_t grid;           /* work-groups per streaming kernel; 0 = automatic */
  int32_t progress_every; /* > 0: print the iteration count, rho_k / rho_0 and
                             the elapsed host time to stderr after every this
                             many s-step iterations and at every restart
                             (default 0: silent) */
  int32_t permute_domains; /* 1: the solver numbers the rows domain by domain
                             (the caller's order within a domain) so that
                             each domain's rows, and the neighbours a sparse
                             row reaches inside its domain, are contiguous in
                             device memory; every array argument and result
                             stays in the caller's order.  0: the caller's
                             order (default 1) */
  int32_t ca;             /* 1: build each iteration's basis with the modified
                             CA-Arnoldi A-orthonormalization (Section 4):
                             CA SRE-CG, CA SRE-CG2 or CA MSDO-CG by
                             `variant`; the first block of an iteration is
                             A-orthonormalized against the kept blocks and
                             itself, then its monomial powers A W, ..,
                             A^{s-1} W are formed and A-orthonormalized
                             against the kept blocks and each other.
                             2: the CA-Arnoldi A-orthonormalization of
                             Section 3.1: the powers of the raw first block,
                             all A-orthonormalized together.  CA SRE-CG keeps
                             the last s+1 blocks; a breakdown in the first
                             iteration after a (re)start ends the solve.
                             0: the s-step construction (default 0) */
  int32_t reserved[1];    /* must be zero */
  const int64_t* row_key; /* with permute_domains = 1: n keys (host or device
                             array as the other arrays of ecg_setup); the
                             rows of each domain are then stored by ascending
                             key (ties in the caller's order) instead of in
                             the caller's order.  A locality order (for grid
                             problems the Morton order, ecg_grid_morton_keys)
                             keeps the rows a sparse row reaches close in
                             device memory, so that the basis product finds
                             them in L2.  NULL: the caller's order within a
                             domain (default NULL) */
} ecg_opts;

/* Fill *o with the defaults above. */
void ecg_opts_default(ecg_opts* o);

/* ---- results and statistics -------------------------------------------- */
typedef struct ecg_result {
  int32_t status;         /* same value as the ecg_solve return */
  int32_t iters;          /* s-step iterations executed, restarts included */
  int32_t hist_len;       /* entries written to reshist */
  int32_t restarts;       /* residual replacements performed */
  int32_t blocks;         /* t-column basis blocks built */
  int32_t reserved;
  double  rho0;           /* ||b - A x0||_2 */
  double  relres;         /* last recursive residual norm / rho0 */
  double  true_relres;    /* ||b - A x||_2 / rho0 at exit, in binary64 */
  double  solve_ms;       /* device time of the solve (HIP events) */
} ecg_result;

/* Kernel classes timed when opts.collect_stats = 1. */
enum ecg_kclass {
  ECG_K_RESID = 0,   /* r = b - A x and ||r|| */
  ECG_K_TSPLIT,      /* T(r) */
  ECG_K_CGS_GRAM,    /* first CGS2 update fused with the second Gram */
  ECG_K_CGS_UPDATE,  /* second CGS2 update */
  ECG_K_SPMM,        /* A Z with the A-CholQR Gram and the next block's Grams */
  ECG_K_XR_UPDATE,   /* x += V alpha, r -= A V alpha, ||r|| */
  ECG_K_GRAM,        /* stand-alone Gram (SRE-CG2, Pre-CholQR) */
  ECG_K_UPDATE,      /* stand-alone block update (SRE-CG2, Pre-CholQR) */
  ECG_K_SMALL,       /* sums of work-group partials and the t x t algebra
                        (Cholesky, R^{-1}, coefficient matrices) */
  ECG_K_PRECOND,     /* M^{-1} of the preconditioner (both triangular solves) */
  ECG_K_COUNT
};

typedef struct ecg_stats {
  int64_t launches[ECG_K_COUNT];
  double  ms[ECG_K_COUNT];       /* summed device time */
  double  bytes[ECG_K_COUNT];    /* summed algorithmic HBM bytes */
  double  flops[ECG_K_COUNT];    /* summed algorithmic floating-point operations */
} ecg_stats;

/* ---- library ----------------------------------------------------------- */
const char* ecg_version(void);
const char* ecg_strerror(int status);
/* Message of the last error raised on the calling thread ("" if none). */
const char* ecg_last_error(void);
/* Name of a kernel class, or NULL. */
const char* ecg_kclass_name(int k);

typedef struct ecg_ctx ecg_ctx;

/*
 * Geometric domain decomposition of an nx x ny x nz grid (rows numbered
 * i + nx*(j + ny*k)) into px*py*pz boxes: row -> floor(i*px/nx) +
 * px*(floor(j*py/ny) + py*floor(k*pz/nz)).  The paper decomposes the graph
 * of A into t domains with Metis (Section 4); this is the box
 * decomposition used in its place for grid problems.  dom_dev: device
 * array of nx*ny*nz int32 written by a GPU kernel on `stream`.  Errors:
 * ECG_EINVAL (non-positive sizes, a part count larger than its axis,
 * nx*ny*nz >= 2^31, NULL pointer), ECG_EDEVICE.
 */
int ecg_partition_grid(int64_t nx, int64_t ny, int64_t nz, int32_t px, int32_t py,
                       int32_t pz, int32_t* dom_dev, void* stream);

/*
 * Morton (Z-order) keys of an nx x ny x nz grid, rows numbered as for
 * ecg_partition_grid: keys[i] interleaves the bits of the cell's
 * coordinates (bit b of x, y, z at bits 3b, 3b+1, 3b+2).  A row order for
 * ecg_opts.row_key.  keys: host array of nx*ny*nz int64, written on the
 * host.  Errors: ECG_EINVAL (non-positive sizes, nx*ny*nz >= 2^31, a side
 * >= 2^21, NULL pointer).
 */
int ecg_grid_morton_keys(int64_t nx, int64_t ny, int64_t nz, int64_t* keys);

/*
 * Create a solver for the n x n SPD matrix (rowptr, colind, vals) with the
 * t domains partition[i] in [0, t) and s blocks per iteration.  This is the
 * set-up of the s-step algorithms (Section 3.1: A symmetric positive
 * definite; the t domains are the subdomains of the graph of A that the
 * split operator T of Section 2 uses; Section 4 orders the matrix by them).
 * Copies everything to device memory (with opts.permute_domains, in the
 * domain-contiguous row order) and allocates the workspace: (s+2) pairs of
 * n x t blocks (basis W and its A-image) for ECG_SRECG, one pair per kept
 * block (q_cap_blocks; allocated when first needed) for ECG_SRECG2 and
 * ECG_MSDO, plus scratch.
 * Errors: ECG_EINVAL (out == NULL; n <= 0; t < 1; t > 64; t > n; s < 1;
 * rowptr not starting at 0 or decreasing; nnz >= 2^31; a column index out
 * of [0, n); a partition value out of [0, t); an empty domain; a
 * non-finite value; nonzero reserved fields; ECG_SRECG2 or ECG_MSDO with
 * q_cap_blocks in [1, s); permute_domains not 0 or 1), ECG_ENOMEM (the
 * workspace does not fit ws_cap_bytes or device memory), ECG_EDEVICE.
 * Symmetry and definiteness are not checked here; an indefinite matrix is
 * reported by ecg_solve as ECG_BREAKDOWN.  On error *out is NULL.
 */
int ecg_setup(ecg_ctx** out, int64_t n, const int32_t* rowptr, const int32_t* colind,
              const double* vals, const int32_t* partition, int32_t t, int32_t s,
              const ecg_opts* opts);

/*
 * Solve A x = b (Section 3.1: the s-step algorithms take A, b, x0, the
 * tolerance, s and the iteration bound k_max and return x).  x holds x0 on
 * entry and the solution on exit.  The iteration stops when the recursive
 * residual norm rho_k <= tol * rho_0 (rho_0 = ||b - A x0||; the stopping test
 * of the s-step algorithms), then checks the true residual b - A x and, if
 * that is above tol * rho_0, restarts from x with r = b - A x (at most
 * opts.max_restarts times).  maxit bounds the s-step iterations executed
 * (restarts included).
 *   iters (may be NULL): s-step iterations executed.
 *   reshist (may be NULL): caller buffer of at least
 *     2 * maxit + opts.max_restarts + 2 doubles; receives rho_0, then rho_k
 *     after every iteration and the true residual norm at every restart.
 *   reshist_len (may be NULL): number of values written to reshist.
 *   true_relres (may be NULL): ||b - A x||_2 / rho_0 at exit, in binary64.
 * Returns ECG_OK, ECG_MAXIT, ECG_BREAKDOWN (x = last completed iterate) or
 * ECG_STAGNATED, or ECG_EINVAL (NULL c/b/x; tol <= 0 or not finite;
 * maxit < 0; a non-finite entry in b or x0), ECG_EDEVICE.  Synchronous on
 * opts.hip_stream.
 */
int ecg_solve(ecg_ctx* c, const double* b, double* x, double tol, int32_t maxit,
              int32_t* iters, double* reshist, int32_t* reshist_len, double* true_relres);

/*
 * ecg_solve with every count of the solve: reshist (may be NULL) receives at
 * most reshist_cap values of the history above; res (may be NULL) receives
 * the counts and norms of ecg_result (res->status = the return value, also
 * on errors).  Errors as ecg_solve, plus ECG_EINVAL for reshist_cap < 0.
 */
int ecg_solve_ex(ecg_ctx* c, const double* b, double* x, double tol, int32_t maxit,
                 double* reshist, int32_t reshist_cap, ecg_result* res);

/*
 * Gradient of a loss through x = A^{-1} b with respect to the stored
 * nonzeros: grad_vals[p] = -lambda[row(p)] * x[col(p)] for every stored
 * entry p, in the caller's CSR order, where lambda solves A lambda = dL/dx
 * (the adjoint; A is symmetric).  Arrays: lambda and x of length n,
 * grad_vals of length nnz.  Errors: ECG_EINVAL (NULL argument),
 * ECG_EDEVICE.
 */
int ecg_sddmm(ecg_ctx* c, const double* lambda, const double* x, double* grad_vals);

/*
 * y = A X for a row-major n x k block X (1 <= k <= 64), binary64, with the
 * solver's sparse-times-block kernel.  Errors: ECG_EINVAL, ECG_EDEVICE.
 */
int ecg_spmm(ecg_ctx* c, const double* X, double* Y, int32_t k);

/*
 * ecg_spmm for callers that cannot allocate device memory (serving loops,
 * harnesses that forbid hipMalloc, code around a HIP graph capture): the same
 * kernels and result, but the two staging blocks (X packed to the padded
 * width w = 16, 32 or 64 for k <= 16, <= 32, <= 64, in the solver's row
 * order, and its product) live in a fixed 64 MiB device array of the
 * library, one per GPU, held until the process ends.  The call makes no
 * hipMalloc / hipFree and allocates nothing else on the device; X and Y are
 * host or device pointers as opts.device_ptrs says, exactly as for ecg_spmm
 * (host arrays are copied with hipMemcpyAsync, which stages pageable memory
 * through the HIP runtime's own buffers: a caller that must avoid even that
 * passes device pointers).  Like every call here it returns after its work
 * on opts.hip_stream has completed, so it is not itself recorded into a
 * graph: it synchronizes that stream.
 * Limit: n * w <= ECG_SPMM_NOALLOC_MAX (both staging blocks fit the array);
 * larger inputs return ECG_EINVAL before any work.  Every call on a GPU uses
 * that GPU's one array, and each call writes all of it that it reads, so
 * nothing carries over between calls; calls that overlap in time on one GPU
 * (two host threads, or contexts on different streams) race on it.
 * Errors: ECG_EINVAL, ECG_EDEVICE.
 */
#define ECG_SPMM_NOALLOC_MAX 4194304
int ecg_spmm_noalloc(ecg_ctx* c, const double* X, double* Y, int32_t k);

/*
 * Z = T(r): the n x t row-major block whose column d holds r on the rows
 * of domain d and zero elsewhere (Section 2).  Errors: ECG_EINVAL,
 * ECG_EDEVICE.
 */
int ecg_tsplit(ecg_ctx* c, const double* r, double* Z);

/*
 * The basis of the last completed s-step iteration of the last solve:
 * V = [W_j .. W_{j+s-1}] and A V, each n x (s*t) row-major, binary64
 * (block-major, then domain order).  Errors: ECG_EINVAL (no completed
 * iteration), ECG_EDEVICE.
 */
int ecg_get_basis(ecg_ctx* c, double* V, double* AV);

/*
 * Split preconditioning of the s-step methods (Section 5: the system
 * L^{-1} A L^{-t} (L^t x) = L^{-1} b with M = L L^t, solved by
 * A-orthonormalizing V = L^{-t} V-hat; the first block after a restart is
 * M^{-1} T(r), every later one starts from M^{-1} A W_{j-1}).
 * kind = ECG_PREC_BJ_IC0: the block Jacobi preconditioner whose diagonal
 * blocks A(B, B), B = {i : blocks[i] = b}, are factorised by incomplete
 * Cholesky with zero fill-in (the paper's experiments use 64 blocks, each of
 * the t domains a union of blocks); blocks (n int32 values >= 0, host or
 * device array as the context's other arrays, caller's row order) must
 * place every block inside one domain.  kind = ECG_PREC_BJ_CHOL: the same
 * blocks factorised by complete Cholesky (the fill-in kept; for large 2D or
 * 3D blocks the factor grows quickly: beyond 2^28 entries ECG_ENOMEM).  The
 * factorisation runs on the host; the two triangular solves of every
 * application run on the device, level by level.  kind = ECG_PREC_NONE
 * (blocks ignored) removes it.  Applies to every later ecg_solve on the
 * context (all variants, the CA forms and both precision forms).
 * Errors: ECG_EINVAL (bad kind; NULL blocks; a negative value; a block
 * spanning two domains; a pivot <= 0: the matrix is then not suitable for
 * the factorisation), ECG_ENOMEM, ECG_EDEVICE; on error no preconditioner
 * is set.
 */
int ecg_set_preconditioner(ecg_ctx* c, int32_t kind, const int32_t* blocks);

/*
 * The solver's row order: order[i] (n int32 values, host or device array as
 * the context's other arrays) is the caller's row that the solver stores as
 * row i -- the rows of domain 0 in the caller's order (by ascending
 * opts.row_key when given), then those of domain 1, and so on
 * (opts.permute_domains = 1), or i itself (0).
 * Errors: ECG_EINVAL (NULL argument), ECG_EDEVICE.
 */
int ecg_domain_order(ecg_ctx* c, int32_t* order);

/* Per-kernel-class statistics of the last ecg_solve (zeros unless
 * opts.collect_stats = 1). */
int ecg_last_stats(ecg_ctx* c, ecg_stats* st);

/* Release a context and all its device memory.  NULL is a no-op. */
void ecg_destroy(ecg_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* ECG_H */
