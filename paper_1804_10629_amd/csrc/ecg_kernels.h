// Internal declarations shared by the HIP kernels and the host driver.
// Not part of the public interface (include/ecg.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace ecg {

// A basis block of width t is stored row-major with TPI >= t columns
// (TPI in {16, 32, 64}); columns t..TPI-1 are kept at zero.
constexpr int kThreads = 256;     // threads per work-group of the block kernels
constexpr int kMaxS = 16;         // largest s supported by the x/r update

// 64-column blocks use the matrix-core block update with kCSGroups
// work-groups (one Gram partial each) per unit of the grid, and the 64-column
// product kernels (see launch_spmm).
#ifndef ECG_CS_MIN_TPI
#define ECG_CS_MIN_TPI 64
#endif
constexpr int kCSGroups = 2;
constexpr bool uses_cs(int tpi) { return tpi >= ECG_CS_MIN_TPI; }
// Gram partials written by a launch of `grid` work-groups.
constexpr int gram_partials(int tpi, int grid) { return uses_cs(tpi) ? grid * kCSGroups : grid; }
// Gram partials written by the product kernel with Grams (launch_spmm), and
// the compute units of the current device.
int spmm_partials(int tpi, int grid, int max_row);
int device_cus();

// Deterministic reduction over work-groups: every work-group of a streaming
// kernel writes its partial vector; k_reduce_groups then sums groups of
// `group_size` partials in index order and k_final sums the group sums in
// index order and runs the small dense algebra (the tail).
struct RedCtl {
  double* partials;      // [grid][L]
  double* groups;        // [ngroups][L]
  int group_size;
};

// Device-side scalars the host reads back once per s-step iteration.
struct DevStatus {
  double rho;            // ||r|| after the last x/r update
  double rho_true;       // ||b - A x|| from the last residual kernel
  int breakdown;         // 1 once a Cholesky pivot failed
  int breakdown_block;   // block index (since restart) of the failure
};

// Arguments of the small-algebra tails run by the last work-group.
struct TailArgs {
  int t;                       // active columns (<= TPI)
  int m;                       // block index since the last restart (1-based)
  double* rinv_cur;            // R^{-1} of the block just built (write), TPI x TPI
  const double* rinv_p1;       // R^{-1} of block m-1 (nullable)
  const double* rinv_p2;       // R^{-1} of block m-2 (nullable)
  double* cnext;               // [3][TPI*TPI] coefficients of the next first CGS pass
  double* dcoef;               // [2][TPI*TPI] coefficients of the second CGS pass
  double* beta;                // [TPI] x/r coefficients of the block just built
  DevStatus* status;
  double* sums_out;            // copy of the reduced sums (nullable)
  int which;                   // TAIL_NORM: 0 -> status.rho, 1 -> status.rho_true
  // TAIL_GRAM: for the Grams G_g of one chunk (g < ng),
  //   coef_out[g] = -R_g^{-1} R_g^{-t} G_g (R_right^{-1} if rinv_right)
  const double* rinv_g[3];
  double* coef_out[3];
  const double* rinv_right;
  // TAIL_PRE: Cholesky of the Euclidean Gram; R^{-1} to coef_out[0]
};

enum TailKind {
  TAIL_NONE = 0,
  TAIL_SPMM = 1,   // A-CholQR of the new block + next first-pass coefficients
  TAIL_CGS = 2,    // second-pass coefficients against the previous two blocks
  TAIL_NORM = 3,   // a residual norm
  TAIL_PRE = 4,    // Euclidean CholQR factor (Pre-CholQR)
  TAIL_GRAM = 5    // coefficients for one chunk of earlier blocks (SRE-CG2)
};

template <typename S>
struct UGArgs {
  const S* X[4];        // update operands; X[0] enters with the identity when ident0
  const double* C[4];   // TPI x TPI coefficient matrices (device)
  const S* P[3];        // left operands of the Grams H_g = P_g^t out
  S* out;               // written when write_out
  int64_t n;
  RedCtl rc;
  TailArgs tail;
  // Optional x/r contribution of the previous block, whose A-image and
  // block are X[0] and X[1]: x_out = x_in + X[1] beta, r_out = r_in - X[0] beta
  // (fold_beta == nullptr: none; skipped after a breakdown).
  const double* fold_beta;
  const double* x_in;
  double* x_out;
  const double* r_in;
  double* r_out;
  const DevStatus* status;
};

template <typename S, typename SA>
struct SpArgs {
  const int32_t* rowptr;
  const int32_t* colind;
  const SA* vals;
  const S* Z;           // input block (row-major, TPI columns)
  S* AZ;                // output block
  const S* AZprev;      // A-image of the previous block (E Gram), nullable
  const double* rvec;   // residual for a = Z^t r, nullable
  int64_t n;
  int max_row;          // most entries in a row of the matrix
  RedCtl rc;
  TailArgs tail;
};

template <typename S>
struct XRArgs {
  const S* U[kMaxS];
  const S* AU[kMaxS];
  const double* beta[kMaxS];   // [TPI] each
  int nb;
  const double* x_in;          // x_out = x_in + sum U_i beta_i (may alias)
  const double* r_in;          // r_out = r_in - sum AU_i beta_i (may alias)
  double* x;                   // x_out
  double* r;                   // r_out
  int64_t n;
  const DevStatus* status_in;  // skip everything after a breakdown
  RedCtl rc;
  TailArgs tail;
};

// Launchers (defined in ecg_kernels.hip).  All return hipError_t of the launch.
// Sum the partials of a kernel that ran with G work-groups (L values each)
// and run the tail `tail` (TAIL_SPMM, TAIL_CGS with ng Grams, TAIL_NORM).
hipError_t launch_reduce(const RedCtl& rc, int G, int L, int tpi, int tail, int ng,
                         const TailArgs& ta, hipStream_t st);

hipError_t launch_partition(int64_t nx, int64_t ny, int64_t nz, int px, int py, int pz,
                            int32_t* dom, hipStream_t st);

hipError_t launch_resid(const int32_t* rowptr, const int32_t* colind, const double* vals,
                        const double* b, const double* x, double* r, int64_t n, int grid,
                        RedCtl rc, TailArgs tail, hipStream_t st);

template <int TPI, typename S>
hipError_t launch_tsplit(const double* r, const int32_t* dom, S* Z, int64_t n, int grid,
                         hipStream_t st);

// One level (count rows) of the level-scheduled triangular solve, in place
// on the n x TPI block X (k_trsv_level).
template <int TPI, typename S>
hipError_t launch_trsv_level(const int32_t* lrows, int count, const int32_t* rp, const int32_t* ci,
                             const double* v, const double* dinv, S* X, hipStream_t st);

template <int TPI, typename S>
hipError_t launch_update_gram(int nu, int ng, bool ident0, bool write_out, int tail,
                              const UGArgs<S>& a, int grid, hipStream_t st);

template <int TPI, typename S, typename SA>
hipError_t launch_spmm(bool grams, bool has_prev, int tail, const SpArgs<S, SA>& a, int grid,
                       hipStream_t st);

template <int TPI, typename S>
hipError_t launch_xr(const XRArgs<S>& a, int grid, hipStream_t st);

// Optional row maps (nullable): perm[i] is the caller's row of solver row i,
// emap[p] the caller's entry of solver entry p.
template <int TPI, typename S>
hipError_t launch_basis_export(const S* U, const double* rinv, double* V, int64_t n, int t,
                               int ldv, int col0, const int32_t* perm, hipStream_t st);

hipError_t launch_sddmm(const int32_t* rowptr, const int32_t* colind, const double* lam,
                        const double* x, double* grad, int64_t n, const int32_t* perm,
                        const int32_t* emap, hipStream_t st);

// pack: row i of Xp = row perm[i] of X; unpack: row i of Xp to row perm[i] of X
hipError_t launch_pack(const double* X, int k, double* Xp, int TPI, int64_t n,
                       const int32_t* perm, hipStream_t st);
hipError_t launch_unpack(const double* Xp, int TPI, double* X, int k, int64_t n,
                         const int32_t* perm, hipStream_t st);

}  // namespace ecg
