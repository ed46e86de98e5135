// HIP kernels of the s-step enlarged CG solver (gfx950 / CDNA4).
//
// Storage: an n x t basis block is row-major with TPI columns (TPI in
// {16, 32, 64}, padding columns zero).  In the block kernels a row is
// handled by the 16 lanes of one DPP row of a wave64: lane l holds the
// columns (l % 16) + 16 e, e < TPI/16, of row  base + 4 q + l / 16.  That is
// exactly the operand layout of v_mfma_f64_16x16x4f64 with the four rows of
// a quad as the contraction index (A[i][k] and B[k][j] in lane i + 16 k,
// resp. j + 16 k), so tall-skinny Gram products P^t Q = sum_rows P[r]^t Q[r]
// feed loaded registers straight into MFMA.  The 16 x 16 result D comes
// back with D[4 v + l / 16][l % 16] in element v of lane l.
// Block updates out[r] = sum_b X_b[r] C_b (C_b small, t x t) run on the
// matrix cores (k_update_gram_mf), except the 16-column binary64 updates
// without Grams, which stream on the FP64 VALU (k_update_gram): X_b[r][k]
// broadcast across its DPP row (row_newbcast), C_b read from LDS.  The
// product kernels gather the rows of the block that A's pattern selects and
// fold the Grams of A-CholQR and of the next block's first CGS pass into
// their epilogue.
//
// Reductions never use floating-point atomics: every work-group writes its
// partial, and two small kernels after the producer (k_reduce_groups, then
// k_final in one work-group) sum them in a fixed index order and run the
// small dense algebra (Cholesky of the t x t Gram, R^{-1}, the next block's
// CGS coefficients) on the device, so results are bitwise reproducible run
// to run and no host round trip is needed between blocks.

#include "ecg_kernels.h"

#include <algorithm>
#include <type_traits>
#include <utility>

namespace ecg {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (N > 0) {
    static_for<N - 1>(f);
    f(std::integral_constant<int, N - 1>{});
  }
}

// acc + x[16 * (lane / 16) + N] * c: a double-precision FMA whose first
// operand is broadcast from lane N of each 16-lane DPP row (row_newbcast,
// the form of DPP the FP64 ALU supports).  DPP reads its source two wait
// states after the last VALU write, which the compiler cannot see inside
// inline assembly; FIRST adds them before the first read of a new x.
template <int N, bool FIRST>
__device__ __forceinline__ double fmac_bcast(double acc, double x, double c) {
  if constexpr (FIRST) {
    asm("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "+v"(acc)
        : "v"(x), "v"(c), "n"(N));
  } else {
    asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "+v"(acc)
        : "v"(x), "v"(c), "n"(N));
  }
  return acc;
}

// Value of lane (16 * (lane / 16) + N) of a 64-bit register (DPP row_newbcast).
template <int N>
__device__ __forceinline__ double bcast64(double v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x150 + N, 0xF, 0xF, true);
}

// Value of lane (16 * (lane / 16) + N) of a 32-bit register.
template <int N>
__device__ __forceinline__ int bcast32(int v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x150 + N, 0xF, 0xF, true);
}

// Sum over the 16 lanes of each DPP row, result in every lane of the row:
// pairs (quad_perm 1,0,3,2), quads (2,3,0,1), half rows (row_half_mirror),
// rows (row_mirror); no LDS traffic.
__device__ __forceinline__ double row_sum16(double v) {
  v += __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false);
  return v;
}

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename S>
__device__ __forceinline__ double ld(const S* p) { return static_cast<double>(*p); }

// A value the optimiser cannot see through.  Masks built from row bounds go
// through it, so that `loaded * mask` stays an arithmetic use of the load:
// written as a select, the compiler sinks the load into a branch and waits
// on all outstanding loads before it, which serialises the memory pipeline.
template <typename T>
__device__ __forceinline__ T opaque(T v) {
  asm("" : "+v"(v));
  return v;
}

// Tuning knobs (compile-time): row quads per lane of the block-update
// kernels at TPI = 16 / 32, prefetch of the next step's operands, which
// block updates run on the matrix cores, rows per step of the product and
// x/r kernels.  The defaults are the measured fastest; every kernel they
// select between is also used by default for some block width.
#ifndef ECG_UG_RPL16
#define ECG_UG_RPL16 4
#endif
#ifndef ECG_UG_RPL32
#define ECG_UG_RPL32 2
#endif
#ifndef ECG_UG_PREFETCH
#define ECG_UG_PREFETCH 0
#endif
#ifndef ECG_XCD_MAP
#define ECG_XCD_MAP 1
#endif
// Occupancy the streaming kernels are scheduled for (waves per SIMD).  The
// launches give each CU a few work-groups of four waves, so the compiler is
// told not to trade memory-level parallelism (loads kept in flight) for an
// occupancy the grid never reaches.
#ifndef ECG_WAVES_PER_EU
#define ECG_WAVES_PER_EU 2
#endif
#define ECG_STREAM __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(ECG_WAVES_PER_EU, ECG_WAVES_PER_EU)))
#ifndef ECG_SP_WPE
#define ECG_SP_WPE ECG_WAVES_PER_EU
#endif
#define ECG_SPMM_ATTR __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(ECG_SP_WPE, ECG_SP_WPE)))
#ifndef ECG_SP_NT
#define ECG_SP_NT 1            // streaming (non-temporal) access to A, r, A Z_prev and A Z
#endif

// Loads and stores of data used once (CSR arrays, streamed blocks): with
// ECG_SP_NT they carry the non-temporal hint so that they do not displace
// the gathered block from the caches.
template <typename T>
__device__ __forceinline__ T ld_s(const T* p) {
  if constexpr (ECG_SP_NT != 0) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename T>
__device__ __forceinline__ void st_s(T* p, T v) {
  if constexpr (ECG_SP_NT != 0) __builtin_nontemporal_store(v, p);
  else *p = v;
}

#ifndef ECG_F32_RPL_MUL
#define ECG_F32_RPL_MUL 2      // row-quad multiplier of the update kernels for binary32 blocks
#endif
#ifndef ECG_UG_CGROUP
#define ECG_UG_CGROUP 4        // coefficient rows read from LDS per group (divides 16)
#endif
#ifndef ECG_MF32
#define ECG_MF32 1             // 32-column block updates on the matrix cores as well
#endif
#ifndef ECG_MF16F
#define ECG_MF16F 1            // 16-column binary32 block updates on the matrix cores
#endif
#ifndef ECG_MF16D
#define ECG_MF16D 1            // 16-column binary64 launches with Grams on the matrix cores
#endif
#ifndef ECG_MF_PF
#define ECG_MF_PF 1            // matrix-core update: load the next step during this one
#endif
#ifndef ECG_MF_WPE
#define ECG_MF_WPE 2
#endif
#ifndef ECG_XR_WIDE
#define ECG_XR_WIDE 1          // 16-byte-load x/r update for one 16-column block
#endif
#ifndef ECG_XR_RQ
#define ECG_XR_RQ 4            // row sets per step of that kernel
#endif
#ifndef ECG_SPW32_RQ
#define ECG_SPW32_RQ 2         // row quads per step of that kernel
#endif
#ifndef ECG_SPWF_RQ
#define ECG_SPWF_RQ 1          // 16-row sets per step of the binary32 wide-gather kernel
#endif


template <int TPI, typename S = double>
struct Cfg {
  static constexpr int EPL = TPI / 16;                              // columns per lane
  // binary32 operands take half the registers: more row quads in flight
  static constexpr int RPL = (TPI == 16 ? ECG_UG_RPL16 : (TPI == 32 ? ECG_UG_RPL32 : 1)) *
                             (sizeof(S) == 4 ? ECG_F32_RPL_MUL : 1);
  static constexpr int WROWS = 4 * RPL;                             // rows per wave step
  static constexpr int NWAVE = kThreads / 64;
  static constexpr int WGROWS = WROWS * NWAVE;                      // rows per WG step
  static constexpr int T2 = TPI * TPI;
};

// Row steps of a work-group.  Work-groups are dispatched to the 8 XCDs of the
// device in round-robin order and each XCD has its own L2, so each XCD gets
// a contiguous range of steps (its work-groups sweep that range together):
// the neighbours a sparse row reaches (+-1, +-nx, +-nx*ny rows on a grid)
// were then fetched by the same XCD shortly before.
struct Steps {
  int64_t first, end, stride;
};

__device__ __forceinline__ Steps my_steps(int64_t nsteps) {
  const int G = gridDim.x;
  if (ECG_XCD_MAP && G % 8 == 0 && G >= 64) {
    const int xcd = blockIdx.x % 8, local = blockIdx.x / 8, per = G / 8;
    const int64_t sx = (nsteps + 7) / 8;
    const int64_t b = xcd * sx;
    return Steps{b + local, min(nsteps, b + sx), per};
  }
  return Steps{blockIdx.x, nsteps, G};
}

// ---------------------------------------------------------------------------
// Work-group and grid reductions
// ---------------------------------------------------------------------------

// Sum of v over the work-group in a fixed order; result valid in all threads.
__device__ double wg_sum(double v, double* lds_scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if (lane == 0) lds_scratch[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += lds_scratch[w];
  __syncthreads();
  return s;
}

// Write this work-group's partial (LDS, L doubles) to rc.partials[blockIdx].
// The totals are formed after the kernel by k_reduce_groups and k_final, so
// no work-group waits for another and no device-scope fence is needed
// inside the streaming kernels.
__device__ void write_partial(const double* red, int L, const RedCtl& rc) {
  double* mine = rc.partials + (size_t)blockIdx.x * L;
  for (int i = threadIdx.x; i < L; i += blockDim.x) mine[i] = red[i];
}

// ---------------------------------------------------------------------------
// Small dense algebra on t x t matrices, run by one wave after the totals
// are formed.  Matrices are row-major with leading dimension TPI, zero in
// the padding.  Lane c holds column c of the matrix being formed in
// registers (lanes c >= TPI are idle); the other operand of a product is
// read from LDS or global memory, every lane reading the same element
// (a broadcast).  Lanes exchange data only through LDS, ordered by wsync():
// the wave's LDS accesses complete in program order, so a fence at wave
// scope that keeps the compiler from reordering them is enough.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lanes c < TPI take part; the caller returns the others.
template <int TPI>
__device__ __forceinline__ void col_load(const double* M, int c, double (&x)[TPI]) {
#pragma unroll
  for (int i = 0; i < TPI; ++i) x[i] = M[i * TPI + c];
}

template <int TPI>
__device__ __forceinline__ void col_store(double* M, int c, const double (&x)[TPI], double sc) {
#pragma unroll
  for (int i = 0; i < TPI; ++i) M[i * TPI + c] = sc * x[i];
}

// Copy a TPI x TPI matrix (global) into LDS.
template <int TPI>
__device__ __forceinline__ void mat_to_lds(const double* src, double* dst, int c) {
#pragma unroll
  for (int i = 0; i < TPI; ++i) dst[i * TPI + c] = src[i * TPI + c];
}

// y = op(A) x for lane c's column x, A in LDS; op(A) = A^t if TRANS.
// Outer loop over k: the TPI accumulators are independent, so the FMAs of
// one step issue back to back.
template <int TPI, bool TRANS>
__device__ __forceinline__ void col_mul(const double* A, const double (&x)[TPI], double (&y)[TPI]) {
  // column k+1 of op(A) is read while column k's FMAs run (two columns in
  // registers at a time)
  double cur[TPI], nxt[TPI];
#pragma unroll
  for (int i = 0; i < TPI; ++i) {
    y[i] = 0.0;
    cur[i] = TRANS ? A[i] : A[i * TPI];
  }
#pragma unroll
  for (int k = 0; k < TPI; ++k) {
    if (k + 1 < TPI) {
#pragma unroll
      for (int i = 0; i < TPI; ++i) nxt[i] = TRANS ? A[(k + 1) * TPI + i] : A[i * TPI + k + 1];
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < TPI; ++i) y[i] = __builtin_fma(cur[i], x[k], y[i]);
    if (k + 1 < TPI) {
#pragma unroll
      for (int i = 0; i < TPI; ++i) cur[i] = nxt[i];
    }
  }
}

// Lane-uniform value of lane L's register (v_readlane).
template <int L>
__device__ __forceinline__ double lane_value(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), L);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), L);
  return __hiloint2double(hi, lo);
}

// Upper Cholesky G = R^t R of the leading t x t block, lane c holding
// column c of G on entry and of R on return (zero below the diagonal and
// in the padding).  Pivots and rows of R are read across lanes with
// v_readlane.  A pivot <= 0 or not finite sets *bad and is replaced by 1
// so that the factorisation runs to the end.
template <int TPI>
__device__ void w_chol(double (&g)[TPI], int t, int* bad) {
  const int c = threadIdx.x & 63;
  static_for<TPI>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    if (j >= t) {            // uniform: padding rows of R are zero
      g[j] = 0.0;
      return;
    }
    double d2 = lane_value<j>(g[j]);
    if (!(d2 > 0.0) || !isfinite(d2)) {
      *bad = 1;
      d2 = 1.0;
    }
    const double d = sqrt(d2);
    const double rj = c > j ? g[j] / d : (c == j ? d : 0.0);
    const double rjc = c < t ? rj : 0.0;
    // trailing update of the rows below j: G[i][c] -= R[j][i] R[j][c],
    // R[j][i] broadcast from lane i by the FMA's DPP operand
    const double nrjc = -rjc;
    static_for<TPI - j - 1>([&](auto ic) {
      constexpr int i = j + 1 + decltype(ic)::value;
      g[i] = ic == 0 ? fmac_bcast<i, true>(g[i], rjc, nrjc) : fmac_bcast<i, false>(g[i], rjc, nrjc);
    });
    g[j] = rjc;              // R[j][c]; zero for j > c
  });
}

// Lane c: column c of R^{-1} (R upper triangular in LDS, t x t leading
// block) by back substitution in column (axpy) order; zero in the padding.
template <int TPI>
__device__ void w_trinv(const double* R, int t, double (&x)[TPI]) {
  const int c = threadIdx.x & 63;
  // reciprocals of the pivots first: independent divisions, not a chain
  double rd[TPI];
#pragma unroll
  for (int k = 0; k < TPI; ++k) rd[k] = k < t ? 1.0 / R[k * TPI + k] : 0.0;
#pragma unroll
  for (int i = 0; i < TPI; ++i) x[i] = (i == c) ? 1.0 : 0.0;
#pragma unroll
  for (int k = TPI - 1; k >= 0; --k) {
    if (k >= t) {
      x[k] = 0.0;
      continue;
    }
    asm volatile("" ::: "memory");
    x[k] = c < t ? x[k] * rd[k] : 0.0;
#pragma unroll
    for (int i = 0; i < k; ++i) x[i] = __builtin_fma(-R[i * TPI + k], x[k], x[i]);
  }
}

// Tail after the product A U_m with the Grams G = U^t AU, F = AU^t AU,
// E = AU_{m-1}^t AU and a = U^t r (layout of `sums`: G | F | E | a).
// Produces R_m^{-1}, the x/r coefficients beta_m = R^{-1} R^{-t} a, and the
// coefficients of the next block's first CGS pass:
//   C0 = R_m^{-1}, C1 = -R_m^{-1} H_m, C2 = -R_{m-1}^{-1} H_{m-1}
// with H_m = R_m^{-t} F R_m^{-1}, H_{m-1} = R_{m-1}^{-t} E R_m^{-1}.
// LDS: sums (3 TPI^2 + TPI) and tmp (2 TPI + TPI^2).
template <int TPI>
__device__ void tail_spmm(double* sums, double* tmp, const TailArgs& ta) {
  constexpr int T2 = TPI * TPI;
  const int c = threadIdx.x & 63, t = ta.t;
  double* G = sums;
  double* F = sums + T2;
  double* E = sums + 2 * T2;
  const double* a = sums + 3 * T2;
  double* Rp = tmp + 2 * TPI;
  const bool prev = ta.m >= 2 && ta.rinv_p1 != nullptr;
  // R_{m-1}^{-1} is read from global memory while the factorisation runs
  double rp[TPI];
  if (prev) col_load<TPI>(ta.rinv_p1, c, rp);
  int bad = 0;
  double x[TPI], y[TPI], h[TPI];
  col_load<TPI>(G, c, x);
  wsync();
  w_chol<TPI>(x, t, &bad);
  col_store<TPI>(G, c, x, 1.0);               // G <- R
  wsync();
  w_trinv<TPI>(G, t, y);                      // y: column c of R^{-1}
  if (prev) col_store<TPI>(Rp, c, rp, 1.0);
  wsync();
  col_store<TPI>(G, c, y, 1.0);               // G <- R^{-1}
  col_store<TPI>(ta.rinv_cur, c, y, 1.0);
  col_store<TPI>(ta.cnext, c, y, 1.0);        // C0
  // beta = R^{-1} (R^{-t} a): lane c forms (R^{-t} a)_c from its column
  double al = 0.0;
#pragma unroll
  for (int k = 0; k < TPI; ++k) al = __builtin_fma(y[k], a[k], al);
  tmp[TPI + c] = al;
  wsync();
  double b = 0.0;
#pragma unroll
  for (int k = 0; k < TPI; ++k) b = __builtin_fma(G[c * TPI + k], tmp[TPI + k], b);
  ta.beta[c] = b;
  // C1 = -R^{-1} R^{-t} F R^{-1}
  col_mul<TPI, false>(F, y, x);               // x = F R^{-1} e_c
  col_mul<TPI, true>(G, x, h);                // h = H_m e_c
  col_mul<TPI, false>(G, h, x);
  col_store<TPI>(ta.cnext + T2, c, x, -1.0);
  if (prev) {
    // C2 = -R_{m-1}^{-1} R_{m-1}^{-t} E R_m^{-1}
    col_mul<TPI, false>(E, y, x);             // x = E R_m^{-1} e_c
    col_mul<TPI, true>(Rp, x, h);
    col_mul<TPI, false>(Rp, h, x);
    col_store<TPI>(ta.cnext + 2 * T2, c, x, -1.0);
  }
  if (bad && c == 0 && ta.status->breakdown == 0) {   // the first failing block is kept
    ta.status->breakdown = 1;
    ta.status->breakdown_block = ta.m;
  }
}

// Tail after the first CGS update: sums hold H2'_g = AU_g^t Z' (g < ng);
// D_g = -R_g^{-1} R_g^{-t} H2'_g, where g = 0 is block m-1 and g = 1 block m-2.
// LDS scratch: TPI^2.
template <int TPI>
__device__ void tail_cgs(double* sums, double* tmp, int ng, const TailArgs& ta) {
  constexpr int T2 = TPI * TPI;
  const int c = threadIdx.x & 63;
  double rg[2][TPI];                          // both R^{-1} in flight at once
  for (int g = 0; g < ng; ++g) col_load<TPI>(g == 0 ? ta.rinv_p1 : ta.rinv_p2, c, rg[g]);
  for (int g = 0; g < ng; ++g) {
    col_store<TPI>(tmp, c, rg[g], 1.0);
    double x[TPI], y[TPI];
    col_load<TPI>(sums + g * T2, c, x);
    wsync();
    col_mul<TPI, true>(tmp, x, y);
    col_mul<TPI, false>(tmp, y, x);
    col_store<TPI>(ta.dcoef + g * T2, c, x, -1.0);
    wsync();
  }
}

// Tail for one chunk of earlier blocks (SRE-CG2, MSDO-CG): sums hold G_g
// (g < ng); coef_out[g] = -R_g^{-1} R_g^{-t} G_g [R_right^{-1}].
// LDS scratch: TPI^2.
template <int TPI>
__device__ void tail_gram(double* sums, double* tmp, int ng, const TailArgs& ta) {
  constexpr int T2 = TPI * TPI;
  const int c = threadIdx.x & 63;
  double rr[TPI];
  if (ta.rinv_right) col_load<TPI>(ta.rinv_right, c, rr);
  for (int g = 0; g < ng; ++g) {
    mat_to_lds<TPI>(ta.rinv_g[g], tmp, c);
    double x[TPI], y[TPI];
    if (ta.rinv_right) col_mul<TPI, false>(sums + g * T2, rr, x);   // G_g R_right^{-1} e_c
    else col_load<TPI>(sums + g * T2, c, x);
    wsync();
    col_mul<TPI, true>(tmp, x, y);
    col_mul<TPI, false>(tmp, y, x);
    col_store<TPI>(ta.coef_out[g], c, x, -1.0);
    wsync();
  }
}

// Tail of Pre-CholQR: the Euclidean Gram Z^t Z = Re^t Re; Re^{-1} to
// coef_out[0] (breakdown as for A-CholQR).  LDS scratch: TPI.
template <int TPI>
__device__ void tail_pre(double* sums, double* tmp, const TailArgs& ta) {
  const int c = threadIdx.x & 63;
  int bad = 0;
  double x[TPI], y[TPI];
  col_load<TPI>(sums, c, x);
  wsync();
  w_chol<TPI>(x, ta.t, &bad);
  col_store<TPI>(sums, c, x, 1.0);
  wsync();
  w_trinv<TPI>(sums, ta.t, y);
  col_store<TPI>(ta.coef_out[0], c, y, 1.0);
  if (bad && c == 0 && ta.status->breakdown == 0) {
    ta.status->breakdown = 1;
    ta.status->breakdown_block = ta.m;
  }
}

// ---------------------------------------------------------------------------
// The same tails run by the whole work-group on LDS-resident matrices, for
// 32 and 64 stored columns (a lane would need 3 x TPI doubles of registers
// for the one-wave form).
// ---------------------------------------------------------------------------

// In-place upper Cholesky G = R^t R of the leading t x t block (upper
// triangle of G used).  Breakdown iff a pivot is <= 0 or not finite.
// On return the block holds R with zeros below the diagonal and in the
// padding.
template <int TPI>
__device__ void b_chol(double* G, int t, int* bad) {
  // Right-looking, one barrier per pivot: step j updates the trailing upper
  // triangle with the unscaled row j over the pivot (G[i][c] -= G[j][i]
  // G[j][c] / G[j][j]); the rows are scaled by their pivots' square roots
  // in one pass at the end.  Every thread derives the same pivot value.
  const int tid = threadIdx.x;
  for (int j = 0; j < t; ++j) {
    double piv = G[j * TPI + j];
    const bool okp = piv > 0.0 && isfinite(piv);
    if (!okp) piv = 1.0;
    if (!okp && tid == 0) *bad = 1;
    const double inv = 1.0 / piv;
    const int w = t - j - 1;
    for (int idx = tid; idx < w * w; idx += blockDim.x) {
      const int i = j + 1 + idx / w, c = j + 1 + idx % w;
      if (i <= c) G[i * TPI + c] -= G[j * TPI + i] * G[j * TPI + c] * inv;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < TPI * TPI; idx += blockDim.x) {
    const int i = idx / TPI, c = idx % TPI;
    double v = 0.0;
    if (i < t && c < t && i <= c) {
      double piv = G[i * TPI + i];
      if (!(piv > 0.0 && isfinite(piv))) piv = 1.0;
      const double d = sqrt(piv);
      v = (i == c) ? d : G[idx] / d;
    }
    G[idx] = v;
  }
  __syncthreads();
}

// In-place inverse of the upper triangular leading t x t block.
template <int TPI>
__device__ void b_trinv(double* R, int t, double* tmp) {
  const int tid = threadIdx.x;
  for (int j = 0; j < t; ++j) {
    // column j of the inverse: X[i][j] = -X[j][j] * sum_{k=i}^{j-1} X[i][k] R[k][j]
    for (int i = tid; i < j; i += blockDim.x) {
      double acc = 0.0;
      for (int k = i; k < j; ++k) acc += R[i * TPI + k] * R[k * TPI + j];
      tmp[i] = acc;
    }
    __syncthreads();
    const double inv = 1.0 / R[j * TPI + j];
    for (int i = tid; i < j; i += blockDim.x) R[i * TPI + j] = -tmp[i] * inv;
    if (tid == 0) R[j * TPI + j] = inv;
    __syncthreads();
  }
}

// R <- R^{-1}: at 32 columns lane c of wave 0 forms column c by back
// substitution (w_trinv, no barriers) into tmp, then the work-group copies
// it back; at 64 columns (a column per lane would need 128 registers more)
// the barrier-per-column form b_trinv.
template <int TPI>
__device__ void b_inverse(double* R, int t, double* tmp) {
  if constexpr (TPI == 32) {
    if (threadIdx.x < TPI) {
      double x[TPI];
      w_trinv<TPI>(R, t, x);
      const int c = threadIdx.x;
#pragma unroll
      for (int i = 0; i < TPI; ++i) tmp[i * TPI + c] = x[i];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < TPI * TPI; idx += blockDim.x) R[idx] = tmp[idx];
    __syncthreads();
  } else {
    b_trinv<TPI>(R, t, tmp);
  }
}

// C = op(A) B on the leading t x t blocks (op = transpose if ta); the
// padding of C is zero.  Operands normally live in LDS; any of them may be
// in global memory.
template <int TPI>
__device__ void b_mm(const double* A, bool ta, const double* B, double* C, int t,
                         double scale) {
  for (int idx = threadIdx.x; idx < TPI * TPI; idx += blockDim.x) {
    const int i = idx / TPI, c = idx % TPI;
    double acc = 0.0;
    if (i < t && c < t) {
      for (int k = 0; k < t; ++k) acc += (ta ? A[k * TPI + i] : A[i * TPI + k]) * B[k * TPI + c];
    }
    C[idx] = scale * acc;
  }
  __syncthreads();
}

template <int TPI>
__device__ void b_copy(const double* src, double* dst) {
  for (int idx = threadIdx.x; idx < TPI * TPI; idx += blockDim.x) dst[idx] = src[idx];
  __syncthreads();
}

// Tail after the product A U_m with the Grams G = U^t AU, F = AU^t AU,
// E = AU_{m-1}^t AU and a = U^t r (layout of `sums`: G | F | E | a).
// Produces R_m^{-1}, the x/r coefficients beta_m = R^{-1} R^{-t} a, and the
// coefficients of the next block's first CGS pass:
//   C0 = R_m^{-1}, C1 = -R_m^{-1} H_m, C2 = -R_{m-1}^{-1} H_{m-1}
// with H_m = R_m^{-t} F R_m^{-1}, H_{m-1} = R_{m-1}^{-t} E R_m^{-1}.
template <int TPI>
__device__ void btail_spmm(double* sums, double* tmp, const TailArgs& ta) {
  constexpr int T2 = TPI * TPI;
  __shared__ int s_bad;
  const int t = ta.t, tid = threadIdx.x;
  double* G = sums;
  double* F = sums + T2;
  double* E = sums + 2 * T2;
  double* a = sums + 3 * T2;
  if (tid == 0) s_bad = 0;
  // F is symmetric: the product kernels may form only its upper triangle
  for (int idx = tid; idx < T2; idx += blockDim.x) {
    const int i = idx / TPI, c = idx % TPI;
    if (i > c) F[idx] = F[c * TPI + i];
  }
  __syncthreads();
  b_chol<TPI>(G, t, &s_bad);
  b_inverse<TPI>(G, t, tmp);         // G now holds R^{-1}
  for (int idx = tid; idx < T2; idx += blockDim.x) {
    ta.rinv_cur[idx] = G[idx];
    ta.cnext[idx] = G[idx];                      // C0
  }
  // alpha = R^{-t} a ; beta = R^{-1} alpha
  for (int i = tid; i < TPI; i += blockDim.x) {
    double acc = 0.0;
    if (i < t)
      for (int k = 0; k <= i; ++k) acc += G[k * TPI + i] * a[k];
    tmp[i] = acc;
  }
  __syncthreads();
  for (int i = tid; i < TPI; i += blockDim.x) {
    double acc = 0.0;
    if (i < t)
      for (int k = i; k < t; ++k) acc += G[i * TPI + k] * tmp[k];
    ta.beta[i] = acc;
  }
  __syncthreads();
  // H_m = R^{-t} F R^{-1}; C1 = -R^{-1} H_m
  b_mm<TPI>(F, false, G, tmp, t, 1.0);       // tmp = F R^{-1}
  b_mm<TPI>(G, true, tmp, F, t, 1.0);        // F <- H_m
  b_mm<TPI>(G, false, F, ta.cnext + T2, t, -1.0);
  if (ta.m >= 2 && ta.rinv_p1 != nullptr) {
    b_mm<TPI>(E, false, G, tmp, t, 1.0);     // tmp = E R_m^{-1}
    b_copy<TPI>(ta.rinv_p1, E);                // E <- R_{m-1}^{-1}
    b_mm<TPI>(E, true, tmp, F, t, 1.0);      // F <- H_{m-1}
    b_mm<TPI>(E, false, F, ta.cnext + 2 * T2, t, -1.0);
  }
  if (tid == 0 && s_bad && ta.status->breakdown == 0) {
    ta.status->breakdown = 1;
    ta.status->breakdown_block = ta.m;
  }
}

// Tail after the first CGS update: sums hold H2'_g = AU_g^t Z' (g < ng);
// D_g = -R_g^{-1} R_g^{-t} H2'_g, where g = 0 is block m-1 and g = 1 block m-2.
template <int TPI>
__device__ void btail_cgs(double* sums, double* tmp, int ng, const TailArgs& ta) {
  constexpr int T2 = TPI * TPI;
  double* Rs = tmp;
  double* T = tmp + T2;
  for (int g = 0; g < ng; ++g) {
    b_copy<TPI>(g == 0 ? ta.rinv_p1 : ta.rinv_p2, Rs);
    b_mm<TPI>(Rs, true, sums + g * T2, T, ta.t, 1.0);
    b_mm<TPI>(Rs, false, T, ta.dcoef + g * T2, ta.t, -1.0);
  }
}

// Tail for one chunk of earlier blocks (SRE-CG2): sums hold G_g (g < ng);
// coef_out[g] = -R_g^{-1} (R_g^{-t} G_g [R_right^{-1}]).
template <int TPI>
__device__ void btail_gram(double* sums, double* tmp, int ng, const TailArgs& ta) {
  constexpr int T2 = TPI * TPI;
  double* Rs = tmp;
  double* T = tmp + T2;
  for (int g = 0; g < ng; ++g) {
    b_copy<TPI>(ta.rinv_g[g], Rs);
    b_mm<TPI>(Rs, true, sums + g * T2, T, ta.t, 1.0);      // T = R_g^{-t} G_g
    if (ta.rinv_right) {
      // G_g <- T R_right^{-1} (the right factor is read from global memory)
      b_mm<TPI>(T, false, ta.rinv_right, sums + g * T2, ta.t, 1.0);
      b_mm<TPI>(Rs, false, sums + g * T2, ta.coef_out[g], ta.t, -1.0);
    } else {
      b_mm<TPI>(Rs, false, T, ta.coef_out[g], ta.t, -1.0);
    }
  }
}

// Tail of Pre-CholQR: the Euclidean Gram Z^t Z = Re^t Re; Re^{-1} to
// coef_out[0] (breakdown as for A-CholQR).
template <int TPI>
__device__ void btail_pre(double* sums, double* tmp, const TailArgs& ta) {
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  b_chol<TPI>(sums, ta.t, &s_bad);
  b_inverse<TPI>(sums, ta.t, tmp);
  for (int idx = threadIdx.x; idx < TPI * TPI; idx += blockDim.x) ta.coef_out[0][idx] = sums[idx];
  if (threadIdx.x == 0 && s_bad && ta.status->breakdown == 0) {
    ta.status->breakdown = 1;
    ta.status->breakdown_block = ta.m;
  }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

__global__ void k_partition(int64_t nx, int64_t ny, int64_t nz, int px, int py, int pz,
                            int32_t* dom) {
  const int64_t n = nx * ny * nz;
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = row % nx, j = (row / nx) % ny, k = row / (nx * ny);
    const int64_t di = i * px / nx, dj = j * py / ny, dk = k * pz / nz;
    dom[row] = (int32_t)(di + px * (dj + py * dk));
  }
}

// r = b - A x ; sums: ||r||^2
__global__ ECG_STREAM void k_resid(const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ colind,
                                                    const double* __restrict__ vals,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ r, int64_t n,
                                                    RedCtl rc, TailArgs ta) {
  __shared__ double red[8];
  double rr = 0.0;
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int p = rowptr[row]; p < rowptr[row + 1]; ++p) acc += vals[p] * x[colind[p]];
    const double v = b[row] - acc;
    r[row] = v;
    rr += v * v;
  }
  const double s = wg_sum(rr, red);
  if (threadIdx.x == 0) red[0] = s;
  __syncthreads();
  write_partial(red, 1, rc);
  (void)ta;
}

template <int TPI, typename S>
__global__ __launch_bounds__(kThreads) void k_tsplit(const double* __restrict__ r,
                                                     const int32_t* __restrict__ dom,
                                                     S* __restrict__ Z, int64_t n) {
  const int64_t total = n * TPI;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = idx / TPI;
    const int c = (int)(idx % TPI);
    Z[idx] = (c == dom[row]) ? static_cast<S>(r[row]) : static_cast<S>(0);
  }
}

// One level of a sparse triangular solve with an n x TPI block, in place:
// X[i] = (X[i] - sum_j T[i][j] X[j]) * dinv[i] for the rows i of the level
// (T strictly lower for L y = x, strictly upper for L^t z = y; every j is
// in an earlier level).  A thread per (row, column); a row's TPI threads
// read its entries as one broadcast and its neighbours' rows coalesced.
// Arithmetic in binary64, the block stored as S.
template <int TPI, typename S>
__global__ __launch_bounds__(kThreads) void k_trsv_level(const int32_t* __restrict__ lrows,
                                                         int count,
                                                         const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const double* __restrict__ v,
                                                         const double* __restrict__ dinv,
                                                         S* __restrict__ X) {
  const int64_t total = (int64_t)count * TPI;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = lrows[idx / TPI];
    const int c = (int)(idx % TPI);
    double acc = static_cast<double>(X[row * TPI + c]);
    for (int e = rp[row]; e < rp[row + 1]; ++e)
      acc -= v[e] * static_cast<double>(X[(int64_t)ci[e] * TPI + c]);
    X[row * TPI + c] = static_cast<S>(acc * dinv[row]);
  }
}

// out[r] = (ident0 ? X0[r] : 0) + sum_b X_b[r] C_b ; H_g = sum_r P_g[r]^t out[r].
// P0X tells that P[0] is the same block as the first coefficient operand
// (the first CGS pass of block m uses A U_{m-1} both ways); it is loaded once.
template <int TPI, typename S, int NU, int NG, bool IDENT0, bool WRITE, int TAIL, bool P0X>
__global__ ECG_STREAM void k_update_gram(UGArgs<S> a) {
  using C = Cfg<TPI, S>;
  constexpr int EPL = C::EPL, RPL = C::RPL, T2 = C::T2;
  constexpr int NCOEF = NU - (IDENT0 ? 1 : 0);
  constexpr int NX = NU;                         // loaded update operands (incl. X0)
  constexpr int NP = NG - (P0X ? 1 : 0);         // separately loaded Gram operands
  constexpr int NLD = NX + NP;
  constexpr int BODY = NCOEF * T2;
  constexpr int TAILSZ = NG * T2;
  constexpr int LDSN = (BODY > TAILSZ ? BODY : TAILSZ) > 1 ? (BODY > TAILSZ ? BODY : TAILSZ) : 1;
  __shared__ double lds[LDSN];
  __shared__ double fbeta[TPI];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, rq = lane >> 4;

  for (int b = 0; b < NCOEF; ++b) {
    const double* src = a.C[b + (IDENT0 ? 1 : 0)];
    for (int idx = tid; idx < T2; idx += blockDim.x) lds[b * T2 + idx] = src[idx];
  }
  // fold of the previous block's x/r contribution (uniform)
  const bool fold = !IDENT0 && NU >= 2 && a.fold_beta != nullptr && a.status->breakdown == 0;
  if (fold)
    for (int idx = tid; idx < TPI; idx += blockDim.x) fbeta[idx] = a.fold_beta[idx];
  __syncthreads();

  d4 acc[NG > 0 ? NG : 1][EPL][EPL];
  for (int g = 0; g < (NG > 0 ? NG : 1); ++g)
    for (int i = 0; i < EPL; ++i)
      for (int j = 0; j < EPL; ++j) acc[g][i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const S* src[NLD];
  for (int b = 0; b < NX; ++b) src[b] = a.X[b];
  for (int g = 0; g < NP; ++g) src[NX + g] = a.P[g + (P0X ? 1 : 0)];

  const int64_t n = a.n;
  // x_in and r_in are null when the launch carries no fold: the loads then
  // read the first operand instead, and go unused
  constexpr bool FOLDK = !IDENT0 && NU >= 2;
  const double* xsrc = fold ? a.x_in : reinterpret_cast<const double*>(src[0]);
  const double* rsrc = fold ? a.r_in : reinterpret_cast<const double*>(src[0]);
  // without a fold, row rc reads the first 8 bytes of its own row of X[0]
  // (loaded anyway): no extra traffic
  const int64_t xstride = fold ? 1 : (int64_t)(TPI * sizeof(S) / 8);
  // operands of one wave step: [operand][q][e], zero on rows >= n; for the
  // fold, x and r of row 4 (m % RPL) + rq (one row per lane, lanes with
  // m >= RPL repeating them), so one instruction covers the step's rows
  auto load_step = [&](int64_t step, double (&v)[NLD][RPL][EPL], double& vx, double& vr) {
    const int64_t row0 = step * C::WGROWS + wave * C::WROWS + rq;
    for (int q = 0; q < RPL; ++q) {
      const int64_t row = row0 + 4 * q;
      const int64_t rc = row < n ? row : n - 1;
      const double okf = opaque(row < n ? 1.0 : 0.0);
      for (int b = 0; b < NLD; ++b)
        for (int e = 0; e < EPL; ++e) v[b][q][e] = ld(src[b] + rc * TPI + m + 16 * e) * okf;
    }
    if constexpr (FOLDK) {
      const int64_t row = row0 + 4 * (m % RPL);
      const int64_t rc = row < n ? row : n - 1;
      vx = xsrc[rc * xstride];
      vr = rsrc[rc * xstride];
    }
  };

  constexpr bool PF = ECG_UG_PREFETCH != 0;
  double cur[NLD][RPL][EPL], nxt[PF ? NLD : 1][RPL][EPL];
  double fx = 0.0, fr = 0.0, nfx = 0.0, nfr = 0.0;
  const Steps sp = my_steps((n + C::WGROWS - 1) / C::WGROWS);
  int64_t step = sp.first;
  bool have = step < sp.end;
  if (have) load_step(step, cur, fx, fr);
  while (have) {
    const int64_t nstep = step + sp.stride;
    const bool have_next = nstep < sp.end;
    if constexpr (PF) {
      if (have_next) load_step(nstep, nxt, nfx, nfr);
    }

    if constexpr (!IDENT0 && NU >= 2) {
      if (fold) {
        const int64_t row0f = step * C::WGROWS + wave * C::WROWS + rq;
        double dxm = 0.0, drm = 0.0;   // sums of row 4 (m % RPL) + rq
        for (int q = 0; q < RPL; ++q) {
          double dx = 0.0, dr = 0.0;
          for (int e = 0; e < EPL; ++e) {
            const double bv = fbeta[m + 16 * e];
            dx = __builtin_fma(cur[1][q][e], bv, dx);
            dr = __builtin_fma(cur[0][q][e], bv, dr);
          }
          dx = row_sum16(dx);
          dr = row_sum16(dr);
          dxm = (m % RPL) == q ? dx : dxm;
          drm = (m % RPL) == q ? dr : drm;
        }
        const int64_t row = row0f + 4 * (m % RPL);
        if (m < RPL && row < n) {
          a.x_out[row] = fx + dxm;
          a.r_out[row] = fr - drm;
        }
      }
    }
    double o[RPL][EPL];
    for (int q = 0; q < RPL; ++q)
      for (int e = 0; e < EPL; ++e) o[q][e] = IDENT0 ? cur[0][q][e] : 0.0;
    // Coefficient rows come from LDS (ds_read) in groups of CG: the empty
    // asm with a memory clobber keeps the compiler from hoisting the
    // loop-invariant reads out of the row loop, which would need all
    // NCOEF * TPI * EPL values in registers.
    constexpr int CG = ECG_UG_CGROUP;
    static_for<NCOEF>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      constexpr int xb = b + (IDENT0 ? 1 : 0);
      static_for<EPL>([&](auto ec) {
        constexpr int e2 = decltype(ec)::value;
        static_for<16 / CG>([&](auto gc) {
          constexpr int g0 = CG * decltype(gc)::value;
          asm volatile("" ::: "memory");
          double cv[CG][EPL];
          for (int u = 0; u < CG; ++u)
            for (int e = 0; e < EPL; ++e)
              cv[u][e] = lds[b * T2 + (16 * e2 + g0 + u) * TPI + m + 16 * e];
          static_for<CG>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            constexpr int nn = g0 + u;
            for (int q = 0; q < RPL; ++q)
              for (int e = 0; e < EPL; ++e)
                o[q][e] = (nn == 0 && e == 0)
                              ? fmac_bcast<nn, true>(o[q][e], cur[xb][q][e2], cv[u][e])
                              : fmac_bcast<nn, false>(o[q][e], cur[xb][q][e2], cv[u][e]);
          });
        });
      });
    });
    const int64_t row0 = step * C::WGROWS + wave * C::WROWS + rq;
    if constexpr (WRITE) {
      for (int q = 0; q < RPL; ++q) {
        const int64_t row = row0 + 4 * q;
        if (row < n)
          for (int e = 0; e < EPL; ++e) a.out[row * TPI + m + 16 * e] = static_cast<S>(o[q][e]);
      }
    }
    if constexpr (NG > 0) {
      static_for<NG>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        constexpr int slot = (P0X && g == 0) ? 0 : NX + g - (P0X ? 1 : 0);
        for (int q = 0; q < RPL; ++q)
          for (int i = 0; i < EPL; ++i)
            for (int j = 0; j < EPL; ++j)
              acc[g][i][j] = mfma16(cur[slot][q][i], o[q][j], acc[g][i][j]);
      });
    }
    if constexpr (PF) {
      if (have_next) {
        for (int b = 0; b < NLD; ++b)
          for (int q = 0; q < RPL; ++q)
            for (int e = 0; e < EPL; ++e) cur[b][q][e] = nxt[b][q][e];
        fx = nfx;
        fr = nfr;
      }
    } else {
      if (have_next) load_step(nstep, cur, fx, fr);
    }
    step = nstep;
    have = have_next;
  }

  if constexpr (NG > 0) {
    __syncthreads();   // coefficient LDS no longer needed
    constexpr int L = NG * T2;
    for (int w = 0; w < C::NWAVE; ++w) {
      if (wave == w) {
        for (int g = 0; g < NG; ++g)
          for (int i = 0; i < EPL; ++i)
            for (int j = 0; j < EPL; ++j)
              for (int v = 0; v < 4; ++v) {
                const int idx = g * T2 + (16 * i + 4 * v + rq) * TPI + 16 * j + m;
                lds[idx] = (w == 0 ? 0.0 : lds[idx]) + acc[g][i][j][v];
              }
      }
      __syncthreads();
    }
    write_partial(lds, L, a.rc);
  }
}

// Wide-gather product kernel for 16-column binary64 blocks.  The gathers
// dominate the kernel's vector-memory instructions and its address unit is
// the busy resource, so rows are gathered 16 bytes per lane: 8 lanes per
// row (lane l: row l / 8 of an 8-row set, columns 2 (l % 8) and
// 2 (l % 8) + 1), a (column, value) pair per lane (entry l % 8 of the row's
// chunk), half the gather instructions of the 16-lanes-per-row form.  The
// Gram epilogue needs 16 lanes per row (the MFMA operand layout): A Z is
// moved there with ds_bpermute, Z and A Z_prev are loaded in it directly.
// Pipeline: row pointers two steps ahead, the chunk one step ahead, loaded
// values processed only in the step that uses them.
__device__ __forceinline__ double bperm64(int src_lane, double v) {
  const int lo = __builtin_amdgcn_ds_bpermute(src_lane * 4, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src_lane * 4, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Value of lane 8 * (lane / 8) + N (N < 8) of a 64-bit register: row
// broadcasts of lanes N and N + 8, chosen by the lane's half row.
template <int N>
__device__ __forceinline__ double bcast8_64(double v, bool upper) {
  const double a = bcast64<N>(v), b = bcast64<N + 8>(v);
  return upper ? b : a;
}
template <int N>
__device__ __forceinline__ int bcast8_32(int v, bool upper) {
  const int a = bcast32<N>(v), b = bcast32<N + 8>(v);
  return upper ? b : a;
}

template <bool GRAMS, bool HAS_PREV>
__global__ ECG_SPMM_ATTR void k_spmm_wide(SpArgs<double, double> a) {
  constexpr int TPI = 16, T2 = TPI * TPI, L = 3 * T2 + TPI;
  constexpr int RQ = 2;                          // 8-row sets per wave step
  constexpr int WROWS = 8 * RQ, NWAVE = kThreads / 64, WGROWS = WROWS * NWAVE;
  constexpr int LDSN = GRAMS ? L : 1;
  __shared__ double lds[LDSN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ri = lane >> 3, pp = lane & 7;       // gather layout
  const int m = lane & 15, rq = lane >> 4;       // MFMA layout
  const bool upper = (lane & 8) != 0;

  d4 accG = d4{0.0, 0.0, 0.0, 0.0}, accF = accG, accE = accG;
  double av = 0.0;
  const int64_t n = a.n;
  const int nnz_last = a.rowptr[n] - 1;
  const Steps sp = my_steps((n + WGROWS - 1) / WGROWS);

  struct RowPtr {
    int p0[RQ], p1[RQ];
  };
  struct Head {              // raw chunk: entry pp of each row set's row
    int col[RQ];
    double val[RQ];
  };
  auto row_of = [&](int64_t step, int q) { return step * WGROWS + wave * WROWS + ri + 8 * q; };
  auto load_rowptr = [&](int64_t step, RowPtr& rp) {
    for (int q = 0; q < RQ; ++q) {
      const int64_t row = row_of(step, q);
      const int64_t rc = row < n ? row : n - 1;
      rp.p0[q] = ld_s(a.rowptr + rc);
      rp.p1[q] = ld_s(a.rowptr + rc + 1);
    }
  };
  auto load_chunk = [&](const RowPtr& rp, int c, Head& h) {
    for (int q = 0; q < RQ; ++q) {
      const int idc = min(rp.p0[q] + c + pp, nnz_last);
      h.col[q] = ld_s(a.colind + idc);
      h.val[q] = ld_s(a.vals + idc);
    }
  };
  // sum of chunk c of the step's rows into y (two columns per lane)
  auto gather = [&](const RowPtr& rp, int c, const Head& h, double (&y)[RQ][2]) {
    int offw[RQ];
    double valb[RQ];
    for (int q = 0; q < RQ; ++q) {
      const bool ok = rp.p0[q] + c + pp < rp.p1[q];
      offw[q] = ok ? h.col[q] : 0;
      valb[q] = h.val[q] * opaque(ok ? 1.0 : 0.0);
    }
    static_for<8>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      for (int q = 0; q < RQ; ++q) {
        const int col = bcast8_32<j>(offw[q], upper);
        const double vj = bcast8_64<j>(valb[q], upper);
        const double2 z = *reinterpret_cast<const double2*>(a.Z + (int64_t)col * TPI + 2 * pp);
        y[q][0] = __builtin_fma(vj, z.x, y[q][0]);
        y[q][1] = __builtin_fma(vj, z.y, y[q][1]);
      }
    });
  };

  RowPtr rp_cur, rp_nxt;
  Head h_cur;
  int64_t step = sp.first;
  if (step < sp.end) {
    load_rowptr(step, rp_cur);
    load_chunk(rp_cur, 0, h_cur);
    // past the work-group's last step the current one is loaded again
    // (cache hits; unused)
    load_rowptr(step + sp.stride < sp.end ? step + sp.stride : step, rp_nxt);
  }
  for (; step < sp.end; step += sp.stride) {
    // next step's chunk and the row pointers after it: issued before this
    // step's gathers, processed only when used (no wait here)
    Head h_nxt;
    RowPtr rp_nn;
    load_chunk(rp_nxt, 0, h_nxt);
    load_rowptr(step + 2 * sp.stride < sp.end ? step + 2 * sp.stride : step, rp_nn);
    // Gram operands in the MFMA layout (lane: row rq + 4 k, column m)
    double z[4], pz[4], rv[4], okm[4];
    if constexpr (GRAMS) {
      for (int k = 0; k < 4; ++k) {
        const int64_t row = step * WGROWS + wave * WROWS + rq + 4 * k;
        const int64_t rc = row < n ? row : n - 1;
        okm[k] = opaque(row < n ? 1.0 : 0.0);
        rv[k] = ld_s(a.rvec + rc);
        z[k] = a.Z[rc * TPI + m];
        pz[k] = HAS_PREV ? ld_s(a.AZprev + rc * TPI + m) : 0.0;
      }
    }
    double y[RQ][2];
    for (int q = 0; q < RQ; ++q) y[q][0] = y[q][1] = 0.0;
    gather(rp_cur, 0, h_cur, y);
    int len = 0;
    for (int q = 0; q < RQ; ++q) len = max(len, rp_cur.p1[q] - rp_cur.p0[q]);
    for (int c = 8; c < len; c += 8) {   // rows longer than one chunk
      Head h;
      load_chunk(rp_cur, c, h);
      gather(rp_cur, c, h, y);
    }
    for (int q = 0; q < RQ; ++q) {
      const int64_t row = row_of(step, q);
      if (row < n) {
        double2 v;
        v.x = y[q][0];
        v.y = y[q][1];
        *reinterpret_cast<double2*>(a.AZ + row * TPI + 2 * pp) = v;
      }
    }
    if constexpr (GRAMS) {
      // A Z into the MFMA layout: row 4 k + rq of the step (row set k / 2,
      // row (4 k + rq) % 8 of it), column m (lane 8 ((4 k + rq) % 8) + m / 2,
      // element m % 2)
      for (int k = 0; k < 4; ++k) {
        const int q = k >> 1;
        const int src = 8 * (4 * (k & 1) + rq) + (m >> 1);
        const double e0 = bperm64(src, y[q][0]), e1 = bperm64(src, y[q][1]);
        const double yk = ((m & 1) ? e1 : e0) * okm[k];
        av = __builtin_fma(z[k] * okm[k], rv[k], av);
        accG = mfma16(z[k], yk, accG);
        accF = mfma16(yk, yk, accF);
        if constexpr (HAS_PREV) accE = mfma16(pz[k], yk, accE);
      }
    }
    h_cur = h_nxt;
    rp_cur = rp_nxt;
    rp_nxt = rp_nn;
  }
  if constexpr (GRAMS) {
    av += __shfl_xor(av, 16, 64);
    av += __shfl_xor(av, 32, 64);
    for (int w = 0; w < NWAVE; ++w) {
      if (wave == w) {
        for (int v = 0; v < 4; ++v) {
          const int idx = (4 * v + rq) * TPI + m;
          const bool first = (w == 0);
          lds[idx] = (first ? 0.0 : lds[idx]) + accG[v];
          lds[T2 + idx] = (first ? 0.0 : lds[T2 + idx]) + accF[v];
          lds[2 * T2 + idx] = (first ? 0.0 : lds[2 * T2 + idx]) + accE[v];
        }
        if (rq == 0) lds[3 * T2 + m] = (w == 0 ? 0.0 : lds[3 * T2 + m]) + av;
      }
      __syncthreads();
    }
    write_partial(lds, L, a.rc);
  }
}

// The wide-gather form for 32-column binary64 blocks: a row (256 bytes) is
// gathered by the 16 lanes of a DPP row with one 16-byte load each
// (columns 2 (l % 16), 2 (l % 16) + 1), half the load instructions of two
// 8-byte loads per lane; the chunk's (column, value) pairs are broadcast
// within the DPP row (lanes l % 16 and l % 16 + 8 hold entry l % 8).  The
// Gram epilogue takes columns l % 16 and l % 16 + 16 per lane (the MFMA
// layout): A Z is moved there with ds_bpermute within the row's lanes.
template <bool GRAMS, bool HAS_PREV>
__global__ ECG_SPMM_ATTR void k_spmm_w32(SpArgs<double, double> a) {
  constexpr int TPI = 32, EPL = 2, T2 = TPI * TPI, L = 3 * T2 + TPI;
  constexpr int RQ = ECG_SPW32_RQ;               // row quads per wave step
  constexpr int WROWS = 4 * RQ, NWAVE = kThreads / 64, WGROWS = WROWS * NWAVE;
  constexpr int LDSN = GRAMS ? L : 1;
  __shared__ double lds[LDSN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, rq = lane >> 4;

  d4 accG[EPL][EPL], accF[EPL][EPL], accE[EPL][EPL];
  double av[EPL];
  for (int i = 0; i < EPL; ++i) {
    av[i] = 0.0;
    for (int j = 0; j < EPL; ++j) {
      accG[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      accF[i][j] = accG[i][j];
      accE[i][j] = accG[i][j];
    }
  }
  const int64_t n = a.n;
  const int nnz_last = a.rowptr[n] - 1;
  const Steps sp = my_steps((n + WGROWS - 1) / WGROWS);

  struct RowPtr {
    int p0[RQ], p1[RQ];
  };
  struct Head {              // raw chunk: entry l % 8 of each row quad's row
    int col[RQ];
    double val[RQ];
  };
  auto row_of = [&](int64_t step, int q) { return step * WGROWS + wave * WROWS + rq + 4 * q; };
  auto load_rowptr = [&](int64_t step, RowPtr& rp) {
    for (int q = 0; q < RQ; ++q) {
      const int64_t row = row_of(step, q);
      const int64_t rc = row < n ? row : n - 1;
      rp.p0[q] = ld_s(a.rowptr + rc);
      rp.p1[q] = ld_s(a.rowptr + rc + 1);
    }
  };
  auto load_chunk = [&](const RowPtr& rp, int c, Head& h) {
    for (int q = 0; q < RQ; ++q) {
      const int idc = min(rp.p0[q] + c + (m & 7), nnz_last);
      h.col[q] = ld_s(a.colind + idc);
      h.val[q] = ld_s(a.vals + idc);
    }
  };
  auto gather = [&](const RowPtr& rp, int c, const Head& h, double (&y)[RQ][2]) {
    int offw[RQ];
    double valb[RQ];
    for (int q = 0; q < RQ; ++q) {
      const bool ok = rp.p0[q] + c + (m & 7) < rp.p1[q];
      offw[q] = ok ? h.col[q] : 0;
      valb[q] = h.val[q] * opaque(ok ? 1.0 : 0.0);
    }
    static_for<8>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      for (int q = 0; q < RQ; ++q) {
        const int col = bcast32<j>(offw[q]);
        const double vj = bcast64<j>(valb[q]);
        const double2 z = *reinterpret_cast<const double2*>(a.Z + (int64_t)col * TPI + 2 * m);
        y[q][0] = __builtin_fma(vj, z.x, y[q][0]);
        y[q][1] = __builtin_fma(vj, z.y, y[q][1]);
      }
    });
  };

  RowPtr rp_cur, rp_nxt;
  Head h_cur;
  int64_t step = sp.first;
  if (step < sp.end) {
    load_rowptr(step, rp_cur);
    load_chunk(rp_cur, 0, h_cur);
    // past the work-group's last step the current one is loaded again
    // (cache hits; unused)
    load_rowptr(step + sp.stride < sp.end ? step + sp.stride : step, rp_nxt);
  }
  for (; step < sp.end; step += sp.stride) {
    Head h_nxt;
    RowPtr rp_nn;
    load_chunk(rp_nxt, 0, h_nxt);
    load_rowptr(step + 2 * sp.stride < sp.end ? step + 2 * sp.stride : step, rp_nn);
    double z[RQ][EPL], pz[RQ][EPL], rv[RQ], okm[RQ];
    if constexpr (GRAMS) {
      for (int q = 0; q < RQ; ++q) {
        const int64_t row = row_of(step, q);
        const int64_t rc = row < n ? row : n - 1;
        okm[q] = opaque(row < n ? 1.0 : 0.0);
        rv[q] = ld_s(a.rvec + rc);
        for (int e = 0; e < EPL; ++e) {
          z[q][e] = a.Z[rc * TPI + m + 16 * e];
          pz[q][e] = HAS_PREV ? ld_s(a.AZprev + rc * TPI + m + 16 * e) : 0.0;
        }
      }
    }
    double y[RQ][2];
    for (int q = 0; q < RQ; ++q) y[q][0] = y[q][1] = 0.0;
    gather(rp_cur, 0, h_cur, y);
    int len = 0;
    for (int q = 0; q < RQ; ++q) len = max(len, rp_cur.p1[q] - rp_cur.p0[q]);
    for (int c = 8; c < len; c += 8) {   // rows longer than one chunk
      Head h;
      load_chunk(rp_cur, c, h);
      gather(rp_cur, c, h, y);
    }
    for (int q = 0; q < RQ; ++q) {
      const int64_t row = row_of(step, q);
      if (row < n) {
        double2 v;
        v.x = y[q][0];
        v.y = y[q][1];
        *reinterpret_cast<double2*>(a.AZ + row * TPI + 2 * m) = v;
      }
    }
    if constexpr (GRAMS) {
      for (int q = 0; q < RQ; ++q) {
        // A Z at column m + 16 e of this lane's row: lane (m >> 1) + 8 e of
        // the same DPP row, element m & 1
        double yk[EPL];
        for (int e = 0; e < EPL; ++e) {
          const int src = 16 * rq + (m >> 1) + 8 * e;
          const double e0 = bperm64(src, y[q][0]), e1 = bperm64(src, y[q][1]);
          yk[e] = ((m & 1) ? e1 : e0) * okm[q];
        }
        for (int i = 0; i < EPL; ++i) {
          av[i] = __builtin_fma(z[q][i] * okm[q], rv[q], av[i]);
          for (int j = 0; j < EPL; ++j) {
            accG[i][j] = mfma16(z[q][i], yk[j], accG[i][j]);
            accF[i][j] = mfma16(yk[i], yk[j], accF[i][j]);
            if constexpr (HAS_PREV) accE[i][j] = mfma16(pz[q][i], yk[j], accE[i][j]);
          }
        }
      }
    }
    h_cur = h_nxt;
    rp_cur = rp_nxt;
    rp_nxt = rp_nn;
  }
  if constexpr (GRAMS) {
    for (int i = 0; i < EPL; ++i) {
      av[i] += __shfl_xor(av[i], 16, 64);
      av[i] += __shfl_xor(av[i], 32, 64);
    }
    for (int w = 0; w < NWAVE; ++w) {
      if (wave == w) {
        for (int i = 0; i < EPL; ++i)
          for (int j = 0; j < EPL; ++j)
            for (int v = 0; v < 4; ++v) {
              const int idx = (16 * i + 4 * v + rq) * TPI + 16 * j + m;
              const bool first = (w == 0);
              lds[idx] = (first ? 0.0 : lds[idx]) + accG[i][j][v];
              lds[T2 + idx] = (first ? 0.0 : lds[T2 + idx]) + accF[i][j][v];
              lds[2 * T2 + idx] = (first ? 0.0 : lds[2 * T2 + idx]) + accE[i][j][v];
            }
        if (rq == 0)
          for (int i = 0; i < EPL; ++i) {
            const int idx = 3 * T2 + 16 * i + m;
            lds[idx] = (w == 0 ? 0.0 : lds[idx]) + av[i];
          }
      }
      __syncthreads();
    }
    write_partial(lds, L, a.rc);
  }
}

// The wide-gather form for 32-column binary32 blocks: a row (128 bytes) is
// gathered by 8 lanes with one 16-byte load each (columns 4 (l % 8) ..
// 4 (l % 8) + 3), 8 rows per wave instruction, RQ such row sets per step;
// lane l holds entry l % 8 of its row's chunk, broadcast within the half
// DPP row.  Products are accumulated in binary64 and rounded once.  For the
// Grams the wave's rounded A Z tile goes through LDS (its own region,
// ordered within the wave) into the MFMA layout.
template <bool GRAMS, bool HAS_PREV>
__global__ ECG_SPMM_ATTR void k_spmm_w32f(SpArgs<float, float> a) {
  constexpr int TPI = 32, EPL = 2, T2 = TPI * TPI, L = 3 * T2 + TPI;
  constexpr int RQ = 2;                          // 8-row sets per wave step
  constexpr int WROWS = 8 * RQ, NWAVE = kThreads / 64, WGROWS = WROWS * NWAVE;
  constexpr int LDSN = GRAMS ? L : 1;
  constexpr int TLD = TPI + 1;                   // padded rows of the A Z tile (floats)
  __shared__ double lds[LDSN];
  __shared__ float azt[GRAMS ? NWAVE * WROWS * TLD : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ri = lane >> 3, pp = lane & 7;       // gather layout
  const int m = lane & 15, rq = lane >> 4;       // MFMA layout
  const bool upper = (lane & 8) != 0;
  float* tile = azt + (GRAMS ? wave * WROWS * TLD : 0);

  d4 accG[EPL][EPL], accF[EPL][EPL], accE[EPL][EPL];
  double av[EPL];
  for (int i = 0; i < EPL; ++i) {
    av[i] = 0.0;
    for (int j = 0; j < EPL; ++j) {
      accG[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      accF[i][j] = accG[i][j];
      accE[i][j] = accG[i][j];
    }
  }
  const int64_t n = a.n;
  const int nnz_last = a.rowptr[n] - 1;
  const Steps sp = my_steps((n + WGROWS - 1) / WGROWS);

  struct RowPtr {
    int p0[RQ], p1[RQ];
  };
  struct Head {
    int col[RQ];
    float val[RQ];
  };
  auto row_of = [&](int64_t step, int q) { return step * WGROWS + wave * WROWS + ri + 8 * q; };
  auto load_rowptr = [&](int64_t step, RowPtr& rp) {
    for (int q = 0; q < RQ; ++q) {
      const int64_t row = row_of(step, q);
      const int64_t rc = row < n ? row : n - 1;
      rp.p0[q] = ld_s(a.rowptr + rc);
      rp.p1[q] = ld_s(a.rowptr + rc + 1);
    }
  };
  auto load_chunk = [&](const RowPtr& rp, int c, Head& h) {
    for (int q = 0; q < RQ; ++q) {
      const int idc = min(rp.p0[q] + c + pp, nnz_last);
      h.col[q] = ld_s(a.colind + idc);
      h.val[q] = ld_s(a.vals + idc);
    }
  };
  auto gather = [&](const RowPtr& rp, int c, const Head& h, double (&y)[RQ][4]) {
    int offw[RQ], valw[RQ];
    for (int q = 0; q < RQ; ++q) {
      const bool ok = rp.p0[q] + c + pp < rp.p1[q];
      offw[q] = ok ? h.col[q] : 0;
      valw[q] = __builtin_bit_cast(int, h.val[q] * opaque(ok ? 1.0f : 0.0f));
    }
    static_for<8>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      for (int q = 0; q < RQ; ++q) {
        const int col = bcast8_32<j>(offw[q], upper);
        const double vj = static_cast<double>(__builtin_bit_cast(float, bcast8_32<j>(valw[q], upper)));
        const float4 z = *reinterpret_cast<const float4*>(a.Z + (int64_t)col * TPI + 4 * pp);
        y[q][0] = __builtin_fma(vj, static_cast<double>(z.x), y[q][0]);
        y[q][1] = __builtin_fma(vj, static_cast<double>(z.y), y[q][1]);
        y[q][2] = __builtin_fma(vj, static_cast<double>(z.z), y[q][2]);
        y[q][3] = __builtin_fma(vj, static_cast<double>(z.w), y[q][3]);
      }
    });
  };

  RowPtr rp_cur, rp_nxt;
  Head h_cur;
  int64_t step = sp.first;
  if (step < sp.end) {
    load_rowptr(step, rp_cur);
    load_chunk(rp_cur, 0, h_cur);
    // past the work-group's last step the current one is loaded again
    // (cache hits; unused)
    load_rowptr(step + sp.stride < sp.end ? step + sp.stride : step, rp_nxt);
  }
  for (; step < sp.end; step += sp.stride) {
    Head h_nxt;
    RowPtr rp_nn;
    load_chunk(rp_nxt, 0, h_nxt);
    load_rowptr(step + 2 * sp.stride < sp.end ? step + 2 * sp.stride : step, rp_nn);
    // Gram operands in the MFMA layout: row 4 k + rq of the step, column m + 16 e
    double z[4][EPL], pz[4][EPL], rv[4], okm[4];
    if constexpr (GRAMS) {
      for (int k = 0; k < 4; ++k) {
        const int64_t row = step * WGROWS + wave * WROWS + rq + 4 * k;
        const int64_t rc = row < n ? row : n - 1;
        okm[k] = opaque(row < n ? 1.0 : 0.0);
        rv[k] = ld_s(a.rvec + rc);
        for (int e = 0; e < EPL; ++e) {
          z[k][e] = static_cast<double>(a.Z[rc * TPI + m + 16 * e]);
          pz[k][e] = HAS_PREV ? static_cast<double>(ld_s(a.AZprev + rc * TPI + m + 16 * e)) : 0.0;
        }
      }
    }
    double y[RQ][4];
    for (int q = 0; q < RQ; ++q) y[q][0] = y[q][1] = y[q][2] = y[q][3] = 0.0;
    gather(rp_cur, 0, h_cur, y);
    int len = 0;
    for (int q = 0; q < RQ; ++q) len = max(len, rp_cur.p1[q] - rp_cur.p0[q]);
    for (int c = 8; c < len; c += 8) {   // rows longer than one chunk
      Head h;
      load_chunk(rp_cur, c, h);
      gather(rp_cur, c, h, y);
    }
    float4 yf[RQ];
    for (int q = 0; q < RQ; ++q) {
      yf[q].x = static_cast<float>(y[q][0]);
      yf[q].y = static_cast<float>(y[q][1]);
      yf[q].z = static_cast<float>(y[q][2]);
      yf[q].w = static_cast<float>(y[q][3]);
      const int64_t row = row_of(step, q);
      if (row < n) *reinterpret_cast<float4*>(a.AZ + row * TPI + 4 * pp) = yf[q];
    }
    if constexpr (GRAMS) {
      // the stored (rounded) A Z: tile row 8 q + ri, then read back in the
      // MFMA layout (row 4 k + rq, columns m and m + 16)
      wsync();   // the previous step's tile reads are done
      for (int q = 0; q < RQ; ++q) {
        float* t = tile + (8 * q + ri) * TLD + 4 * pp;
        t[0] = yf[q].x;
        t[1] = yf[q].y;
        t[2] = yf[q].z;
        t[3] = yf[q].w;
      }
      wsync();
      for (int k = 0; k < 4; ++k) {
        double yk[EPL];
        for (int e = 0; e < EPL; ++e)
          yk[e] = static_cast<double>(tile[(4 * k + rq) * TLD + m + 16 * e]) * okm[k];
        for (int i = 0; i < EPL; ++i) {
          av[i] = __builtin_fma(z[k][i] * okm[k], rv[k], av[i]);
          for (int j = 0; j < EPL; ++j) {
            accG[i][j] = mfma16(z[k][i], yk[j], accG[i][j]);
            accF[i][j] = mfma16(yk[i], yk[j], accF[i][j]);
            if constexpr (HAS_PREV) accE[i][j] = mfma16(pz[k][i], yk[j], accE[i][j]);
          }
        }
      }
    }
    h_cur = h_nxt;
    rp_cur = rp_nxt;
    rp_nxt = rp_nn;
  }
  if constexpr (GRAMS) {
    for (int i = 0; i < EPL; ++i) {
      av[i] += __shfl_xor(av[i], 16, 64);
      av[i] += __shfl_xor(av[i], 32, 64);
    }
    for (int w = 0; w < NWAVE; ++w) {
      if (wave == w) {
        for (int i = 0; i < EPL; ++i)
          for (int j = 0; j < EPL; ++j)
            for (int v = 0; v < 4; ++v) {
              const int idx = (16 * i + 4 * v + rq) * TPI + 16 * j + m;
              const bool first = (w == 0);
              lds[idx] = (first ? 0.0 : lds[idx]) + accG[i][j][v];
              lds[T2 + idx] = (first ? 0.0 : lds[T2 + idx]) + accF[i][j][v];
              lds[2 * T2 + idx] = (first ? 0.0 : lds[2 * T2 + idx]) + accE[i][j][v];
            }
        if (rq == 0)
          for (int i = 0; i < EPL; ++i) {
            const int idx = 3 * T2 + 16 * i + m;
            lds[idx] = (w == 0 ? 0.0 : lds[idx]) + av[i];
          }
      }
      __syncthreads();
    }
    write_partial(lds, L, a.rc);
  }
}

// The wide-gather form for 16-column binary32 blocks: a row is 64 bytes, so
// 4 lanes per row gather 16 bytes each (columns 4 (l % 4) .. 4 (l % 4) + 3)
// and each lane holds two entries (l % 4 and l % 4 + 4) of its row's chunk,
// broadcast within the quad with quad_perm.  RQ sets of 16 rows per step.
template <int N>
__device__ __forceinline__ int qbcast32(int v) {
  return __builtin_amdgcn_update_dpp(v, v, N | (N << 2) | (N << 4) | (N << 6), 0xF, 0xF, false);
}

template <bool GRAMS, bool HAS_PREV>
__global__ ECG_SPMM_ATTR void k_spmm_widef(SpArgs<float, float> a) {
  constexpr int TPI = 16, T2 = TPI * TPI, L = 3 * T2 + TPI;
  constexpr int RQ = ECG_SPWF_RQ;                // 16-row sets per wave step
  constexpr int WROWS = 16 * RQ, NWAVE = kThreads / 64, WGROWS = WROWS * NWAVE;
  constexpr int LDSN = GRAMS ? L : 1;
  __shared__ double lds[LDSN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ri = lane >> 2, pp = lane & 3;       // gather layout
  const int m = lane & 15, rq = lane >> 4;       // MFMA layout

  d4 accG = d4{0.0, 0.0, 0.0, 0.0}, accF = accG, accE = accG;
  double av = 0.0;
  const int64_t n = a.n;
  const int nnz_last = a.rowptr[n] - 1;
  const Steps sp = my_steps((n + WGROWS - 1) / WGROWS);

  struct RowPtr {
    int p0[RQ], p1[RQ];
  };
  struct Head {              // raw chunk: entries pp and pp + 4 of the row
    int col[RQ][2];
    float val[RQ][2];
  };
  auto row_of = [&](int64_t step, int q) { return step * WGROWS + wave * WROWS + ri + 16 * q; };
  auto load_rowptr = [&](int64_t step, RowPtr& rp) {
    for (int q = 0; q < RQ; ++q) {
      const int64_t row = row_of(step, q);
      const int64_t rc = row < n ? row : n - 1;
      rp.p0[q] = ld_s(a.rowptr + rc);
      rp.p1[q] = ld_s(a.rowptr + rc + 1);
    }
  };
  auto load_chunk = [&](const RowPtr& rp, int c, Head& h) {
    for (int q = 0; q < RQ; ++q)
      for (int u = 0; u < 2; ++u) {
        const int idc = min(rp.p0[q] + c + pp + 4 * u, nnz_last);
        h.col[q][u] = ld_s(a.colind + idc);
        h.val[q][u] = ld_s(a.vals + idc);
      }
  };
  // products of binary32 values accumulated in binary64, rounded once
  auto gather = [&](const RowPtr& rp, int c, const Head& h, double (&y)[RQ][4]) {
    int offw[RQ][2];
    float valb[RQ][2];
    for (int q = 0; q < RQ; ++q)
      for (int u = 0; u < 2; ++u) {
        const bool ok = rp.p0[q] + c + pp + 4 * u < rp.p1[q];
        offw[q][u] = ok ? h.col[q][u] : 0;
        valb[q][u] = h.val[q][u] * opaque(ok ? 1.0f : 0.0f);
      }
    static_for<8>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      for (int q = 0; q < RQ; ++q) {
        const int col = qbcast32<j % 4>(offw[q][j / 4]);
        const float vj = __builtin_bit_cast(float, qbcast32<j % 4>(__builtin_bit_cast(int, valb[q][j / 4])));
        const float4 z = *reinterpret_cast<const float4*>(a.Z + (int64_t)col * TPI + 4 * pp);
        const double vd = vj;
        y[q][0] = __builtin_fma(vd, (double)z.x, y[q][0]);
        y[q][1] = __builtin_fma(vd, (double)z.y, y[q][1]);
        y[q][2] = __builtin_fma(vd, (double)z.z, y[q][2]);
        y[q][3] = __builtin_fma(vd, (double)z.w, y[q][3]);
      }
    });
  };

  RowPtr rp_cur, rp_nxt;
  Head h_cur;
  int64_t step = sp.first;
  if (step < sp.end) {
    load_rowptr(step, rp_cur);
    load_chunk(rp_cur, 0, h_cur);
    load_rowptr(step + sp.stride < sp.end ? step + sp.stride : step, rp_nxt);
  }
  for (; step < sp.end; step += sp.stride) {
    Head h_nxt;
    RowPtr rp_nn;
    load_chunk(rp_nxt, 0, h_nxt);
    load_rowptr(step + 2 * sp.stride < sp.end ? step + 2 * sp.stride : step, rp_nn);
    constexpr int NK = 4 * RQ;                   // 4-row groups of the step
    double z[NK], pz[NK], rv[NK], okm[NK];
    if constexpr (GRAMS) {
      for (int k = 0; k < NK; ++k) {
        const int64_t row = step * WGROWS + wave * WROWS + rq + 4 * k;
        const int64_t rc = row < n ? row : n - 1;
        okm[k] = opaque(row < n ? 1.0 : 0.0);
        rv[k] = ld_s(a.rvec + rc);
        z[k] = static_cast<double>(a.Z[rc * TPI + m]);
        pz[k] = HAS_PREV ? static_cast<double>(ld_s(a.AZprev + rc * TPI + m)) : 0.0;
      }
    }
    double yd[RQ][4];
    for (int q = 0; q < RQ; ++q) yd[q][0] = yd[q][1] = yd[q][2] = yd[q][3] = 0.0;
    gather(rp_cur, 0, h_cur, yd);
    int len = 0;
    for (int q = 0; q < RQ; ++q) len = max(len, rp_cur.p1[q] - rp_cur.p0[q]);
    for (int c = 8; c < len; c += 8) {
      Head h;
      load_chunk(rp_cur, c, h);
      gather(rp_cur, c, h, yd);
    }
    float y[RQ][4];                              // the stored values
    for (int q = 0; q < RQ; ++q)
      for (int u = 0; u < 4; ++u) y[q][u] = static_cast<float>(yd[q][u]);
    for (int q = 0; q < RQ; ++q) {
      const int64_t row = row_of(step, q);
      if (row < n) {
        float4 v;
        v.x = y[q][0];
        v.y = y[q][1];
        v.z = y[q][2];
        v.w = y[q][3];
        *reinterpret_cast<float4*>(a.AZ + row * TPI + 4 * pp) = v;
      }
    }
    if constexpr (GRAMS) {
      // A Z into the MFMA layout: step row 4 k + rq is row (4 k + rq) % 16 of
      // set (4 k + rq) / 16; column m is element m % 4 of lane 4 row + m / 4
      for (int k = 0; k < NK; ++k) {
        const int r = 4 * k + rq;
        const int q = r >> 4;          // uniform in k for rq < 4: (4 k) / 16
        const int src = 4 * (r & 15) + (m >> 2);
        float e[4];
        for (int u = 0; u < 4; ++u)
          e[u] = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src * 4, __builtin_bit_cast(int, y[k >> 2][u])));
        (void)q;
        const float ev = (m & 2) ? ((m & 1) ? e[3] : e[2]) : ((m & 1) ? e[1] : e[0]);
        const double yk = static_cast<double>(ev) * okm[k];
        av = __builtin_fma(z[k] * okm[k], rv[k], av);
        accG = mfma16(z[k], yk, accG);
        accF = mfma16(yk, yk, accF);
        if constexpr (HAS_PREV) accE = mfma16(pz[k], yk, accE);
      }
    }
    h_cur = h_nxt;
    rp_cur = rp_nxt;
    rp_nxt = rp_nn;
  }
  if constexpr (GRAMS) {
    av += __shfl_xor(av, 16, 64);
    av += __shfl_xor(av, 32, 64);
    for (int w = 0; w < NWAVE; ++w) {
      if (wave == w) {
        for (int v = 0; v < 4; ++v) {
          const int idx = (4 * v + rq) * TPI + m;
          const bool first = (w == 0);
          lds[idx] = (first ? 0.0 : lds[idx]) + accG[v];
          lds[T2 + idx] = (first ? 0.0 : lds[T2 + idx]) + accF[v];
          lds[2 * T2 + idx] = (first ? 0.0 : lds[2 * T2 + idx]) + accE[v];
        }
        if (rq == 0) lds[3 * T2 + m] = (w == 0 ? 0.0 : lds[3 * T2 + m]) + av;
      }
      __syncthreads();
    }
    write_partial(lds, L, a.rc);
  }
}

// Block update and Grams on the matrix cores (32 and 64 columns; at 16
// columns binary32 blocks and the binary64 launches with Grams, while the
// binary64 pure updates keep the VALU kernel above, measured faster).  A
// row group of W = TPI / 16 waves takes 16 rows per step; wave w of it owns
// output columns 16 w .. 16 w + 15 (a work-group of four waves holds 4 / W
// row groups).  The update out = sum_b X_b C_b is a 16 x TPI by TPI x 16
// product per wave and operand: MFMA f64 16x16x4 with the rows as M, the
// input columns as K (four per instruction) and the wave's output columns
// as N.  The B operands (this wave's slice of each coefficient matrix) stay
// in registers for the whole launch; the A operands (row l % 16, column
// 4 kk + l / 16 of X_b) come from an LDS tile the row group's waves fill
// with their column slices.  The result lands in the natural layout (lane:
// row 4 v + l / 16, column l % 16), which is the B operand of the Gram
// products H_g = P_g^t out (K = rows) and the layout of the coalesced store.
template <int TPI, typename S, int NU, int NG, bool IDENT0, bool WRITE, bool P0X>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(ECG_MF_WPE, ECG_MF_WPE)))
void k_update_gram_mf(UGArgs<S> a) {
  constexpr int T2 = TPI * TPI, LD = TPI + 1;   // LD: padded tile rows
  constexpr int W = TPI / 16, RG = 4 / W, KQ = TPI / 4, NV = 4 / W;
  constexpr int NCOEF = NU - (IDENT0 ? 1 : 0);
  constexpr int NX = NU;
  constexpr int NP = NG - (P0X ? 1 : 0);
  constexpr int NLD = NX + NP;
  static_assert(RG * NLD * 16 * LD >= (RG - 1) * NG * T2, "Gram exchange fits the tiles");
  __shared__ double tile[RG][NLD][16 * LD];
  __shared__ double fbeta[TPI];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cb = wave % W, rg = wave / W;
  const int m = lane & 15, rq = lane >> 4;
  double(*const tl)[16 * LD] = tile[rg];

  // B operands: cf[b][kk] = C[4 kk + l / 16][16 cb + l % 16]
  double cf[NCOEF > 0 ? NCOEF : 1][KQ];
  for (int b = 0; b < NCOEF; ++b) {
    const double* cm = a.C[b + (IDENT0 ? 1 : 0)];
    for (int kk = 0; kk < KQ; ++kk) cf[b][kk] = cm[(4 * kk + rq) * TPI + 16 * cb + m];
  }
  const bool fold = !IDENT0 && NU >= 2 && a.fold_beta != nullptr && a.status->breakdown == 0;
  if (fold)
    for (int idx = tid; idx < TPI; idx += blockDim.x) fbeta[idx] = a.fold_beta[idx];

  d4 acc[NG > 0 ? NG : 1][W];
  for (int g = 0; g < (NG > 0 ? NG : 1); ++g)
    for (int e = 0; e < W; ++e) acc[g][e] = d4{0.0, 0.0, 0.0, 0.0};

  const S* src[NLD];
  for (int b = 0; b < NX; ++b) src[b] = a.X[b];
  for (int g = 0; g < NP; ++g) src[NX + g] = a.P[g + (P0X ? 1 : 0)];

  const int64_t n = a.n;
  const Steps sp = my_steps((n + 16 * RG - 1) / (16 * RG));
  constexpr bool FOLDK = !IDENT0 && NU >= 2;
  // this wave's column slice of every operand (natural layout) and, for the
  // fold, x_in and r_in of the rows; with PF the next step's are loaded
  // while this step's products run
  // (measured: faster at 32 columns for binary32 blocks and for the
  // binary64 kernels with Grams, slower for the binary64 pure updates, no
  // gain at 64 columns; at 16 columns only binary32 blocks take this kernel)
  constexpr bool PF = ECG_MF_PF && ((TPI == 32 && (sizeof(S) == 4 || NG > 0)) || TPI == 16);
  // x and r: the fold's rows are shared out over the row group's W waves,
  // NV = 4 / W row quads each; lane l of wave cb takes row 4 vq + l / 16 with
  // vq = cb + W (l % NV), so one instruction covers the wave's rows (lanes
  // l % 16 >= NV repeat them)
  struct Ld {
    double c[NLD][4];
    double xo, ro;
  };
  // x_in and r_in are null when the launch carries no fold: the loads then
  // read the first operand instead, and go unused
  const double* xsrc = fold ? a.x_in : reinterpret_cast<const double*>(src[0]);
  const double* rsrc = fold ? a.r_in : reinterpret_cast<const double*>(src[0]);
  // without a fold, row rc reads the first 8 bytes of its own row of X[0]
  // (loaded anyway): no extra traffic
  const int64_t xstride = fold ? 1 : (int64_t)(TPI * sizeof(S) / 8);
  auto load_step = [&](int64_t st, Ld& d) {
    const int64_t r0 = st * (16 * RG) + 16 * rg + rq;
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 4 * v;
      const int64_t rc = row < n ? row : n - 1;
      const double okf = opaque(row < n ? 1.0 : 0.0);
      for (int b = 0; b < NLD; ++b) d.c[b][v] = ld(src[b] + rc * TPI + 16 * cb + m) * okf;
    }
    if constexpr (FOLDK) {
      const int64_t row = r0 + 4 * (cb + W * (m % NV));
      const int64_t rc = row < n ? row : n - 1;
      d.xo = xsrc[rc * xstride];
      d.ro = rsrc[rc * xstride];
    }
  };
  // a one-wave row group (16 columns) orders its own LDS accesses; wider
  // row groups synchronise the work-group
  auto rg_sync = [&]() {
    if constexpr (W == 1) wsync();
    else __syncthreads();
  };
  if constexpr (W == 1) __syncthreads();   // fbeta
  Ld nx;
  if (PF && sp.first < sp.end) load_step(sp.first, nx);
  for (int64_t step = sp.first; step < sp.end; step += sp.stride) {
    const int64_t row0 = step * (16 * RG) + 16 * rg + rq;
    Ld ldc;
    if constexpr (PF) {
      ldc = nx;
      // past the work-group's last step the current one is loaded again
      // (cache hits; unused)
      load_step(step + sp.stride < sp.end ? step + sp.stride : step, nx);
    } else {
      load_step(step, ldc);
    }
    const double(&cur)[NLD][4] = ldc.c;
    rg_sync();   // the previous step's tile readers are done (and fbeta is set)
    for (int b = 0; b < NLD; ++b)
      for (int v = 0; v < 4; ++v) tl[b][(4 * v + rq) * LD + 16 * cb + m] = cur[b][v];
    rg_sync();

    d4 o;
    for (int v = 0; v < 4; ++v) o[v] = IDENT0 ? cur[0][v] : 0.0;
    static_for<NCOEF>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      constexpr int xb = b + (IDENT0 ? 1 : 0);
      for (int kk = 0; kk < KQ; ++kk) o = mfma16(tl[xb][m * LD + 4 * kk + rq], cf[b][kk], o);
    });

    if constexpr (WRITE) {
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + 4 * v;
        if (row < n) a.out[row * TPI + 16 * cb + m] = static_cast<S>(o[v]);
      }
    }
    if constexpr (NG > 0) {
      static_for<NG>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        constexpr int slot = (P0X && g == 0) ? 0 : NX + g - (P0X ? 1 : 0);
        for (int e = 0; e < W; ++e)
          for (int v = 0; v < 4; ++v) {
            const double pv = tl[slot][(4 * v + rq) * LD + 16 * e + m];
            acc[g][e] = mfma16(pv, o[v], acc[g][e]);
          }
      });
    }
    if constexpr (!IDENT0 && NU >= 2) {
      // x/r contribution of the previous block (X[1] = U, X[0] = A U): wave
      // cb of the row group reads the full rows 4 vq + rq, vq = cb + W k,
      // from the tiles (all waves share the work)
      if (fold) {
        double dxm = 0.0, drm = 0.0;   // sums of row 4 (cb + W (m % NV)) + rq
        for (int k = 0; k < NV; ++k) {
          const int v = cb + W * k;
          double dx = 0.0, dr = 0.0;
          for (int e = 0; e < W; ++e) {
            const double bv = fbeta[16 * e + m];
            dx = __builtin_fma(tl[1][(4 * v + rq) * LD + 16 * e + m], bv, dx);
            dr = __builtin_fma(tl[0][(4 * v + rq) * LD + 16 * e + m], bv, dr);
          }
          dx = row_sum16(dx);
          dr = row_sum16(dr);
          dxm = (m % NV) == k ? dx : dxm;
          drm = (m % NV) == k ? dr : drm;
        }
        const int64_t row = row0 + 4 * (cb + W * (m % NV));
        if (m < NV && row < n) {
          a.x_out[row] = ldc.xo + dxm;
          a.r_out[row] = ldc.ro - drm;
        }
      }
    }
  }
  if constexpr (NG > 0) {
    // H_g[16 e + 4 v + rq][16 cb + m]; one partial per work-group.  With
    // two row groups, the second one's sums pass through LDS and the first
    // adds them to its own (a fixed order).
    double* mine = a.rc.partials + (size_t)blockIdx.x * (NG * T2);
    if constexpr (RG == 1) {
      for (int g = 0; g < NG; ++g)
        for (int e = 0; e < W; ++e)
          for (int v = 0; v < 4; ++v)
            mine[g * T2 + (16 * e + 4 * v + rq) * TPI + 16 * cb + m] = acc[g][e][v];
    } else {
      // row groups 1 .. RG-1 park their sums in LDS; row group 0 adds them
      // in row-group order
      double* xch = &tile[0][0][0];
      __syncthreads();
      if (rg > 0)
        for (int g = 0; g < NG; ++g)
          for (int e = 0; e < W; ++e)
            for (int v = 0; v < 4; ++v)
              xch[(rg - 1) * NG * T2 + g * T2 + (16 * e + 4 * v + rq) * TPI + 16 * cb + m] =
                  acc[g][e][v];
      __syncthreads();
      if (rg == 0)
        for (int g = 0; g < NG; ++g)
          for (int e = 0; e < W; ++e)
            for (int v = 0; v < 4; ++v) {
              const int idx = g * T2 + (16 * e + 4 * v + rq) * TPI + 16 * cb + m;
              double sum = acc[g][e][v];
              for (int r = 1; r < RG; ++r) sum += xch[(r - 1) * NG * T2 + idx];
              mine[idx] = sum;
            }
    }
  }
}

// ---------------------------------------------------------------------------
// Product kernel for 64-column blocks: A Z, with the Grams G = Z^t (A Z)
// (A-CholQR), F = (A Z)^t (A Z), E = (A Z_prev)^t (A Z) (the next block's
// first CGS pass) and a = Z^t r fused in.  At 64 columns the Grams are 27
// times the arithmetic of the product (three 64 x 64 Grams per row against
// seven 64-wide FMAs), so the kernel is built around the matrix cores:
//
//   * gather: a work-group takes R = 16 rows per step, a wave 4 of them.  A
//     wave forms one row at a time across its 64 lanes (lane = column), so
//     the (column, value) pairs of a row are wave-uniform: lanes 8 q + j
//     load entry j of row q in one instruction, v_readlane hands them to
//     the scalar unit, and each neighbour row is one coalesced load with a
//     scalar base.  The rows of Z, A Z and A Z_prev of the step are parked
//     in LDS tiles (row stride 80 doubles: the four rows of an MFMA operand
//     fall on alternating halves of the banks).
//   * Grams: G and F are symmetric, so only their 16 x 16 tiles on or above
//     the diagonal are formed (10 of 16 each; the tail mirrors F), E in
//     full: 36 tiles of MFMA f64 16x16x4 (K = the step's rows), 9 per wave,
//     assigned so that every wave has the same count (20 tiles, 5 per wave,
//     without E).  Tiles of a wave are compile-time (one instantiation of
//     the loop per wave).
//   * two LDS buffers: the next step's gather fills one while slower waves
//     still read the other, so one barrier per step suffices.
// ---------------------------------------------------------------------------

constexpr int kP64R = 16;      // rows per work-group step
constexpr int kP64LD = 80;     // LDS tile row stride (doubles)
#ifndef ECG_P64_CH
#define ECG_P64_CH 7
#endif
constexpr int kP64CH = ECG_P64_CH;   // entries of a row gathered per chunk (<= 8)

// tile code: mat * 16 + a * 4 + b, tile (a, b) of mat 0 = G, 1 = F, 2 = E:
// the 16 x 16 block rows 16 a.., columns 16 b..
constexpr int kP64TileE[4][9] = {
    {0x03, 0x07, 0x0B, 0x0F, 0x13, 0x17, 0x1B, 0x1F, 0x23},
    {0x27, 0x2B, 0x2F, 0x02, 0x06, 0x0A, 0x12, 0x16, 0x1A},
    {0x22, 0x26, 0x2A, 0x2E, 0x01, 0x05, 0x11, 0x15, 0x21},
    {0x25, 0x29, 0x2D, 0x00, 0x10, 0x20, 0x24, 0x28, 0x2C}};
constexpr int kP64TileN[4][5] = {{0x03, 0x07, 0x0B, 0x0F, 0x13},
                                            {0x17, 0x1B, 0x1F, 0x02, 0x06},
                                            {0x0A, 0x12, 0x16, 0x1A, 0x01},
                                            {0x05, 0x11, 0x15, 0x00, 0x10}};

constexpr int p64_tile(int w, bool hp, int k) { return hp ? kP64TileE[w][k] : kP64TileN[w][k]; }

template <typename S, typename SA, bool GRAMS, bool HAS_PREV, int W>
__device__ __forceinline__ void p64_run(const SpArgs<S, SA>& a, double* tiles, double* asum) {
  constexpr int TPI = 64, T2 = TPI * TPI, R = kP64R, LD = kP64LD, CH = kP64CH;
  constexpr int NT = HAS_PREV ? 9 : 5;
  constexpr int TB = 3 * R * LD;      // doubles per buffer: Z, A Z, A Z_prev tiles
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, rq = lane >> 4;
  const int64_t n = a.n;
  const int nnz_last = a.rowptr[n] - 1;
  const Steps sp = my_steps((n + R - 1) / R);
  // lanes 8 q + j (q < 4, j < CH) hold entry j of the current chunk of row q
  const int q_l = (lane >> 3) & 3, j_l = lane & 7;

  // software pipeline: row pointers three steps ahead, the (column, value)
  // pairs of a row's first chunk two steps ahead, the gathered neighbour
  // rows and the own rows one step ahead (issued before the current step's
  // matrix-core phase)
  struct RowPtr { int p0, p1; };
  struct Head { int col; double val; };
  struct Rows { double zg[4][CH]; double zo[4], po[4], rv[4]; };
  auto load_rowptr = [&](int64_t st, RowPtr& rp) {
    const int64_t rl = st * R + 4 * W + q_l;
    const int64_t rlc = rl < n ? rl : n - 1;
    rp.p0 = ld_s(a.rowptr + rlc);
    rp.p1 = ld_s(a.rowptr + rlc + 1);
  };
  auto load_head = [&](const RowPtr& rp, int c, Head& h) {
    // entries past the row's end (or past CH) read a valid entry with the
    // value zero
    const int idx = rp.p0 + c + j_l;
    const int idc = min(idx, nnz_last);
    h.col = ld_s(a.colind + idc);
    h.val = static_cast<double>(ld_s(a.vals + idc)) *
            opaque(idx < rp.p1 && j_l < CH ? 1.0 : 0.0);
  };
  auto load_rows = [&](int64_t st, const Head& h, Rows& d) {
    static_for<4>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      static_for<CH>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        const int cj = __builtin_amdgcn_readlane(h.col, 8 * q + j);
        d.zg[q][j] = ld(a.Z + (int64_t)cj * TPI + lane);
      });
    });
    if constexpr (GRAMS) {
      for (int q = 0; q < 4; ++q) {
        const int64_t row = st * R + 4 * W + q;
        const int64_t rc = row < n ? row : n - 1;
        d.zo[q] = ld(a.Z + rc * TPI + lane);
        d.po[q] = HAS_PREV ? static_cast<double>(ld_s(a.AZprev + rc * TPI + lane)) : 0.0;
        d.rv[q] = ld_s(a.rvec + rc);
      }
    }
  };
  auto head_val = [&](const Head& h, int q, int j) {
    const uint64_t vb = __builtin_bit_cast(uint64_t, h.val);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)vb, 8 * q + j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(vb >> 32), 8 * q + j);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
  };

  d4 acc[NT];
  for (int k = 0; k < NT; ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};
  double av = 0.0;
  int buf = 0;

  RowPtr rp_cur{0, 0}, rp1{0, 0}, rp2{0, 0};
  Head h_cur{0, 0.0}, h1{0, 0.0};
  Rows d_cur;
  int64_t step = sp.first;
  const int64_t st = sp.stride;
  if (step < sp.end) {
    load_rowptr(step, rp_cur);
    if (step + st < sp.end) load_rowptr(step + st, rp1);
    if (step + 2 * st < sp.end) load_rowptr(step + 2 * st, rp2);
    load_head(rp_cur, 0, h_cur);
    if (step + st < sp.end) load_head(rp1, 0, h1);
    load_rows(step, h_cur, d_cur);
  }
  for (; step < sp.end; step += st) {
    const bool has1 = step + st < sp.end, has2 = step + 2 * st < sp.end,
               has3 = step + 3 * st < sp.end;
    const int64_t row0 = step * R + 4 * W;
    double y[4];
    static_for<4>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      double acc_y = 0.0;
      static_for<CH>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        acc_y = __builtin_fma(head_val(h_cur, q, j), d_cur.zg[q][j], acc_y);
      });
      y[q] = acc_y;
    });
    // rows longer than one chunk (none in 5- and 7-point stencils)
    int maxlen = 0;
    for (int q = 0; q < 4; ++q)
      maxlen = max(maxlen, __builtin_amdgcn_readlane(rp_cur.p1 - rp_cur.p0, 8 * q));
    for (int c = CH; c < maxlen; c += CH) {
      Head h;
      load_head(rp_cur, c, h);
      static_for<4>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        static_for<CH>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          const int cj = __builtin_amdgcn_readlane(h.col, 8 * q + j);
          y[q] = __builtin_fma(head_val(h, q, j), ld(a.Z + (int64_t)cj * TPI + lane), y[q]);
        });
      });
    }
    for (int q = 0; q < 4; ++q)
      if (row0 + q < n) st_s(a.AZ + (row0 + q) * TPI + lane, static_cast<S>(y[q]));
    if constexpr (GRAMS) {
      double* tb = tiles + buf * TB;
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * W + q;
        const double okf = row0 + q < n ? 1.0 : 0.0;
        // the stored (rounded) value of A Z enters the Grams
        tb[r * LD + lane] = d_cur.zo[q] * okf;
        tb[R * LD + r * LD + lane] = static_cast<double>(static_cast<S>(y[q])) * okf;
        if constexpr (HAS_PREV) tb[2 * R * LD + r * LD + lane] = d_cur.po[q] * okf;
        av = __builtin_fma(d_cur.zo[q] * okf, d_cur.rv[q], av);
      }
      __syncthreads();
    }
    // the next steps' loads go out before this step's matrix-core phase
    Rows d_nxt;
    Head h2{0, 0.0};
    RowPtr rp3{0, 0};
    if (has1) load_rows(step + st, h1, d_nxt);
    if (has2) load_head(rp2, 0, h2);
    if (has3) load_rowptr(step + 3 * st, rp3);
    if constexpr (GRAMS) {
      const double* X = tiles + buf * TB;
      const double* Y = X + R * LD;
      const double* P = X + 2 * R * LD;
      for (int kk = 0; kk < R / 4; ++kk) {
        const int ro = (4 * kk + rq) * LD + m;
        static_for<NT>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          constexpr int code = p64_tile(W, HAS_PREV, k);
          constexpr int mat = code >> 4, ta = (code >> 2) & 3, tbk = code & 3;
          const double* M = mat == 0 ? X : (mat == 1 ? Y : P);
          acc[k] = mfma16(M[ro + 16 * ta], Y[ro + 16 * tbk], acc[k]);
        });
      }
      buf ^= 1;
    }
    d_cur = d_nxt;
    h_cur = h1;
    h1 = h2;
    rp_cur = rp1;
    rp1 = rp2;
    rp2 = rp3;
  }
  if constexpr (GRAMS) {
    constexpr int L = 3 * T2 + TPI;
    double* mine = a.rc.partials + (size_t)blockIdx.x * L;
    static_for<NT>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int code = p64_tile(W, HAS_PREV, k);
      constexpr int mat = code >> 4, ta = (code >> 2) & 3, tbk = code & 3;
      for (int v = 0; v < 4; ++v)
        mine[mat * T2 + (16 * ta + 4 * v + rq) * TPI + 16 * tbk + m] = acc[k][v];
    });
    asum[W * 64 + lane] = av;
  }
}

template <typename S, typename SA, bool GRAMS, bool HAS_PREV>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_spmm64(SpArgs<S, SA> a) {
  constexpr int T2 = 64 * 64;
  __shared__ double tiles[GRAMS ? 2 * 3 * kP64R * kP64LD : 1];
  __shared__ double asum[GRAMS ? 4 * 64 : 1];
  const int wave = threadIdx.x >> 6;
  switch (wave) {
    case 0: p64_run<S, SA, GRAMS, HAS_PREV, 0>(a, tiles, asum); break;
    case 1: p64_run<S, SA, GRAMS, HAS_PREV, 1>(a, tiles, asum); break;
    case 2: p64_run<S, SA, GRAMS, HAS_PREV, 2>(a, tiles, asum); break;
    default: p64_run<S, SA, GRAMS, HAS_PREV, 3>(a, tiles, asum); break;
  }
  if constexpr (GRAMS) {
    constexpr int L = 3 * T2 + 64;
    double* mine = a.rc.partials + (size_t)blockIdx.x * L;
    // tiles below the diagonal of G and F are not formed: zero (the tail
    // mirrors F and reads only the upper triangle of G); E without a
    // previous block is zero
    for (int idx = threadIdx.x; idx < 3 * T2; idx += blockDim.x) {
      const int mat = idx / T2, e = idx % T2;
      const int br = (e / 64) / 16, bc = (e % 64) / 16;
      if ((mat < 2 && br > bc) || (mat == 2 && !HAS_PREV)) mine[idx] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      double s = 0.0;
      for (int w = 0; w < 4; ++w) s += asum[w * 64 + threadIdx.x];
      mine[3 * T2 + threadIdx.x] = s;
    }
  }
}

// Producer/consumer form of the 64-column product (16 waves per work-group,
// one work-group per CU).  Waves 0-11 (producers) gather: wave w forms rows
// 2 w, 2 w + 1 of each 24-row step as above, with the neighbour rows of a
// step requested two steps ahead (the (column, value) pairs three steps
// ahead, the row pointers four; two steps of requests stay within the 63
// vector-memory instructions a wave can have in flight), and park the
// step's Z, A Z and A Z_prev rows in an LDS slot.  Waves 12-15 (consumers)
// run the Gram tiles on the matrix cores, one step behind: iteration i
// produces step i into slot i % 2 while the consumers read step i - 1 from
// the other slot, so one barrier per iteration orders both and the matrix
// cores do not wait for a gather.  Each SIMD holds three producer waves and
// one consumer wave: their VALU / memory and MFMA instructions co-issue.
// The gather is latency-bound, so more producers mean more rows in flight
// (measured at 256^3: 8 producers and 16-row steps 11.75 ms, 12 and 24 rows
// 10.05 ms per launch; 16 producers would exceed 1024 threads).
#ifndef ECG_PC_R
#define ECG_PC_R 24
#endif
// Step order: 1 = each XCD sweeps its own contiguous eighth of the steps
// (its work-groups interleaved), 0 = all work-groups sweep the rows together
// with the XCDs side by side.  With 16-row steps and 256 work-groups the
// latter advances 4096 rows per round, the distance of a z-neighbour in a
// 64^3 domain, so every XCD met its neighbours in its own L2; 24-row steps
// break that (measured at 256^3: FETCH 38.4 GB per launch with 0, 33.4 GB
// with 1, against 21.9 GB for 16-row steps), and 1 does not depend on the
// geometry.
#ifndef ECG_PC_MAP
#define ECG_PC_MAP 1
#endif
#ifndef ECG_PC_PR
#define ECG_PC_PR 2
#endif
constexpr int kPCR = ECG_PC_R;                // rows per step of the producer/consumer form
constexpr int kP64PR = ECG_PC_PR;             // rows of a step per producer wave
constexpr int kP64NP = kPCR / kP64PR;         // producer waves
constexpr int kP64THREADS = 64 * (kP64NP + 4);

template <typename S, typename SA, bool HAS_PREV>
struct P64Prod {
  static constexpr int TPI = 64, R = kPCR, LD = kP64LD, CH = kP64CH, PR = kP64PR;
  struct RowPtr { int p0, p1; };
  struct Head { int col; double val; };
  struct Rows { double zg[PR][CH]; double zo[PR], po[PR], rv[PR]; };

  const SpArgs<S, SA>& a;
  int64_t n, first, stride;
  int N, nnz_last, lane, q_l, j_l, w;

  // Every load and store below is issued unconditionally (past the last
  // step the last step is read and its values stored again), so that the
  // compiler's count of outstanding memory operations stays exact across
  // the pipelined loop and its waits cover only what they must.
  __device__ int64_t step_of(int j) const { return first + (int64_t)min(j, N - 1) * stride; }
  __device__ void load_rowptr(int j, RowPtr& rp) const {
    const int64_t rl = step_of(j) * R + PR * w + q_l;
    const int64_t rlc = rl < n ? rl : n - 1;
    rp.p0 = ld_s(a.rowptr + rlc);
    rp.p1 = ld_s(a.rowptr + rlc + 1);
  }
  // entries past the row's end (or past CH) read a valid entry with the
  // value zero; rows have at most CH entries (checked by the launcher)
  __device__ void load_head(const RowPtr& rp, Head& h) const {
    const int idx = rp.p0 + j_l;
    const int idc = min(idx, nnz_last);
    h.col = ld_s(a.colind + idc);
    h.val = static_cast<double>(ld_s(a.vals + idc)) * opaque(idx < rp.p1 && j_l < CH ? 1.0 : 0.0);
  }
  __device__ void load_rows(int j, const Head& h, Rows& d) const {
    static_for<PR>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      static_for<CH>([&](auto jc) {
        constexpr int jj = decltype(jc)::value;
        const int cj = __builtin_amdgcn_readlane(h.col, 8 * q + jj);
        d.zg[q][jj] = ld(a.Z + (int64_t)cj * TPI + lane);
      });
    });
    for (int q = 0; q < PR; ++q) {
      const int64_t row = step_of(j) * R + PR * w + q;
      const int64_t rc = row < n ? row : n - 1;
      d.zo[q] = ld(a.Z + rc * TPI + lane);
      d.po[q] = HAS_PREV ? static_cast<double>(ld_s(a.AZprev + rc * TPI + lane)) : 0.0;
      d.rv[q] = ld_s(a.rvec + rc);
    }
  }
  __device__ static double head_val(double val, int q, int jj) {
    const uint64_t vb = __builtin_bit_cast(uint64_t, val);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)vb, 8 * q + jj);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(vb >> 32), 8 * q + jj);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
  }
  // A Z of step j from its gathered rows, stored; the step's tiles to LDS.
  // Rows past n (clamped to n - 1) compute row n - 1's value again and store
  // it there; they enter the tiles and a as zeros.  Past the last step
  // (j >= N) the tiles are written but not read and a is not accumulated.
  __device__ void produce(int j, const Head& h0, const Rows& d, double* tb, double& av) const {
    const int64_t row0 = step_of(j) * R + PR * w;
    const double live = j < N ? 1.0 : 0.0;
    static_for<PR>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      double y = 0.0;
      static_for<CH>([&](auto jc) {
        constexpr int jj = decltype(jc)::value;
        y = __builtin_fma(head_val(h0.val, q, jj), d.zg[q][jj], y);
      });
      const int64_t row = row0 + q;
      const int64_t rc = row < n ? row : n - 1;
      const double okf = row < n ? 1.0 : 0.0;
      st_s(a.AZ + rc * TPI + lane, static_cast<S>(y));
      const int r = PR * w + q;
      // the stored (rounded) value of A Z enters the Grams
      tb[r * LD + lane] = d.zo[q] * okf;
      tb[R * LD + r * LD + lane] = static_cast<double>(static_cast<S>(y)) * okf;
      if constexpr (HAS_PREV) tb[2 * R * LD + r * LD + lane] = d.po[q] * okf;
      av = __builtin_fma(d.zo[q] * (okf * live), d.rv[q], av);
    });
  }
};

template <typename S, typename SA, bool HAS_PREV, int W>
__device__ __forceinline__ void p64pc_consume(const double* tb, d4 (&acc)[HAS_PREV ? 9 : 5],
                                              int lane) {
  constexpr int R = kPCR, LD = kP64LD, NT = HAS_PREV ? 9 : 5;
  const int m = lane & 15, rq = lane >> 4;
  const double* X = tb;
  const double* Y = tb + R * LD;
  const double* P = tb + 2 * R * LD;
  // one K-step's operands live at a time (the nine MFMAs of a step cover
  // the next step's LDS reads)
#pragma unroll 1
  for (int kk = 0; kk < R / 4; ++kk) {
    const int ro = (4 * kk + rq) * LD + m;
    static_for<NT>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int code = p64_tile(W, HAS_PREV, k);
      constexpr int mat = code >> 4, ta = (code >> 2) & 3, tbk = code & 3;
      const double* M = mat == 0 ? X : (mat == 1 ? Y : P);
      acc[k] = mfma16(M[ro + 16 * ta], Y[ro + 16 * tbk], acc[k]);
    });
  }
}

template <typename S, typename SA, bool HAS_PREV, int W>
__device__ __forceinline__ void p64pc_consumer(const SpArgs<S, SA>& a, double* tiles, int N) {
  constexpr int T2 = 64 * 64, TPI = 64, NT = HAS_PREV ? 9 : 5;
  constexpr int TB = 3 * kPCR * kP64LD;
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, rq = lane >> 4;
  d4 acc[NT];
  for (int k = 0; k < NT; ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i <= N; i += 2) {
    if (i >= 1) p64pc_consume<S, SA, HAS_PREV, W>(tiles + TB, acc, lane);   // step i - 1
    __syncthreads();
    if (i + 1 > N) break;
    p64pc_consume<S, SA, HAS_PREV, W>(tiles, acc, lane);                    // step i
    __syncthreads();
  }
  constexpr int L = 3 * T2 + TPI;
  double* mine = a.rc.partials + (size_t)blockIdx.x * L;
  static_for<NT>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int code = p64_tile(W, HAS_PREV, k);
    constexpr int mat = code >> 4, ta = (code >> 2) & 3, tbk = code & 3;
    for (int v = 0; v < 4; ++v)
      mine[mat * T2 + (16 * ta + 4 * v + rq) * TPI + 16 * tbk + m] = acc[k][v];
  });
}

template <typename S, typename SA, bool HAS_PREV>
__device__ __forceinline__ void p64pc_producer(const SpArgs<S, SA>& a, double* tiles,
                                               double* asum, int N, const Steps& sp) {
  constexpr int TB = 3 * kPCR * kP64LD;
  using Pr = P64Prod<S, SA, HAS_PREV>;
  const int lane = threadIdx.x & 63;
  Pr pr{a, a.n, sp.first, sp.stride, N, a.rowptr[a.n] - 1, lane, (lane >> 3) % kP64PR,
        lane & 7, (int)(threadIdx.x >> 6)};
  double av = 0.0;
  if (N > 0) {
    typename Pr::RowPtr q[2], r0, r1;
    typename Pr::Head hh[2], h_cur[2];
    typename Pr::Rows rows[2];
    // prologue: rows of steps 0, 1; heads of steps 0, 1 (kept for the
    // values) and 2; row pointers of step 3
    pr.load_rowptr(0, r0);
    pr.load_rowptr(1, r1);
    pr.load_rowptr(2, q[0]);
    pr.load_head(r0, h_cur[0]);
    pr.load_head(r1, h_cur[1]);
    pr.load_head(q[0], hh[0]);
    pr.load_rowptr(3, q[1]);
    pr.load_rows(0, h_cur[0], rows[0]);
    pr.load_rows(1, h_cur[1], rows[1]);
    // iteration i (parity K): produce step i from rows[K] / h_cur[K]; then
    // request head i + 3 (row pointers q[1 - K]) into hh[1 - K], row
    // pointers i + 4 into q[K], and the rows of step i + 2 (head hh[K])
    // into rows[K].  Issued in that order, every wait is for the oldest
    // requests: the rows of step i + 1 stay in flight.
    auto iter = [&](int i, auto kc) {
      constexpr int K = decltype(kc)::value;
      pr.produce(i, h_cur[K], rows[K], tiles + K * TB, av);
      pr.load_head(q[1 - K], hh[1 - K]);
      pr.load_rowptr(i + 4, q[K]);
      h_cur[K] = hh[K];
      pr.load_rows(i + 2, hh[K], rows[K]);
    };
    for (int i = 0; i <= N; i += 2) {
      iter(i, std::integral_constant<int, 0>{});
      __syncthreads();
      if (i + 1 > N) break;
      iter(i + 1, std::integral_constant<int, 1>{});
      __syncthreads();
    }
  } else {
    __syncthreads();   // the consumers' single barrier
  }
  asum[(threadIdx.x >> 6) * 64 + lane] = av;
}

template <typename S, typename SA, bool HAS_PREV>
__global__ __launch_bounds__(kP64THREADS) __attribute__((amdgpu_waves_per_eu(kP64THREADS / 256, kP64THREADS / 256)))
void k_spmm64pc(SpArgs<S, SA> a) {
  constexpr int T2 = 64 * 64;
  __shared__ double tiles[2 * 3 * kPCR * kP64LD];
  __shared__ double asum[kP64NP * 64];
  const int wave = threadIdx.x >> 6;
  const int64_t nsteps = (a.n + kPCR - 1) / kPCR;
  const int G = gridDim.x;
#if ECG_PC_MAP == 1
  // each XCD sweeps its own contiguous eighth of the steps
  const int64_t x8 = blockIdx.x % 8;
  const Steps sp = (G % 8 == 0) ? Steps{x8 * nsteps / 8 + blockIdx.x / 8, (x8 + 1) * nsteps / 8,
                                        G / 8}
                                : Steps{blockIdx.x, nsteps, G};
#else
  // all work-groups sweep the rows together, the 1/8 of them on one XCD
  // taking adjacent steps (G / 8 steps per XCD and round)
  const Steps sp = (G % 8 == 0) ? Steps{(int64_t)(blockIdx.x % 8) * (G / 8) + blockIdx.x / 8,
                                        nsteps, G}
                                : Steps{blockIdx.x, nsteps, G};
#endif
  const int N = sp.first < sp.end ? (int)((sp.end - sp.first + sp.stride - 1) / sp.stride) : 0;
  switch (wave - kP64NP) {
    case 0: p64pc_consumer<S, SA, HAS_PREV, 0>(a, tiles, N); break;
    case 1: p64pc_consumer<S, SA, HAS_PREV, 1>(a, tiles, N); break;
    case 2: p64pc_consumer<S, SA, HAS_PREV, 2>(a, tiles, N); break;
    case 3: p64pc_consumer<S, SA, HAS_PREV, 3>(a, tiles, N); break;
    default: p64pc_producer<S, SA, HAS_PREV>(a, tiles, asum, N, sp); break;
  }
  constexpr int L = 3 * T2 + 64;
  double* mine = a.rc.partials + (size_t)blockIdx.x * L;
  // tiles below the diagonal of G and F are not formed: zero (the tail
  // mirrors F and reads only the upper triangle of G); E without a
  // previous block is zero
  for (int idx = threadIdx.x; idx < 3 * T2; idx += blockDim.x) {
    const int mat = idx / T2, e = idx % T2;
    const int br = (e / 64) / 16, bc = (e % 64) / 16;
    if ((mat < 2 && br > bc) || (mat == 2 && !HAS_PREV)) mine[idx] = 0.0;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int w = 0; w < kP64NP; ++w) s += asum[w * 64 + threadIdx.x];
    mine[3 * T2 + threadIdx.x] = s;
  }
}

// x += sum_i U_i beta_i ; r -= sum_i AU_i beta_i ; ||r||^2.  Blocks are
// taken four at a time so that eight loads per row are in flight.
template <int TPI, typename S, int NB4>
__global__ ECG_STREAM void k_xr(XRArgs<S> a) {
  // NB4 blocks per pass; a single block gets twice the row quads instead
  constexpr int EPL = TPI / 16, RPL = (TPI == 16 ? 4 : (TPI == 32 ? 2 : 1)) * (NB4 == 1 ? 2 : 1);
  constexpr int WROWS = 4 * RPL, NWAVE = kThreads / 64;
  constexpr int WGROWS = WROWS * NWAVE;
  __shared__ double bl[kMaxS * TPI];
  __shared__ double red[8];
  if (a.status_in->breakdown) return;     // uniform: the host stops after this iteration
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, rq = lane >> 4;
  for (int i = 0; i < kMaxS; ++i)
    for (int c = tid; c < TPI; c += blockDim.x) bl[i * TPI + c] = i < a.nb ? a.beta[i][c] : 0.0;
  __syncthreads();
  double rr = 0.0;
  const int64_t n = a.n;
  const Steps sp = my_steps((n + WGROWS - 1) / WGROWS);
  for (int64_t step = sp.first; step < sp.end; step += sp.stride) {
    const int64_t row0 = step * WGROWS + wave * WROWS + rq;
    int64_t rowc[RPL];
    bool ok[RPL];
    double xo[RPL], ro[RPL];
    for (int q = 0; q < RPL; ++q) {
      const int64_t row = row0 + 4 * q;
      ok[q] = row < n;
      rowc[q] = ok[q] ? row : n - 1;
      // issued with the block loads; only lane m = 0 of a row uses them
      xo[q] = a.x_in[rowc[q]];
      ro[q] = a.r_in[rowc[q]];
    }
    double dx[RPL], dr[RPL];
    for (int q = 0; q < RPL; ++q) {
      dx[q] = 0.0;
      dr[q] = 0.0;
    }
    for (int i0 = 0; i0 < a.nb; i0 += NB4) {
      double u[NB4][RPL][EPL], au[NB4][RPL][EPL];
      for (int j = 0; j < NB4; ++j) {
        const int i = min(i0 + j, a.nb - 1);   // past the end: beta is zero
        for (int q = 0; q < RPL; ++q)
          for (int e = 0; e < EPL; ++e) {
            u[j][q][e] = ld(a.U[i] + rowc[q] * TPI + m + 16 * e);
            au[j][q][e] = ld(a.AU[i] + rowc[q] * TPI + m + 16 * e);
          }
      }
      for (int j = 0; j < NB4; ++j)
        for (int e = 0; e < EPL; ++e) {
          const double bv = bl[(i0 + j) * TPI + m + 16 * e];
          for (int q = 0; q < RPL; ++q) {
            dx[q] = __builtin_fma(u[j][q][e], bv, dx[q]);
            dr[q] = __builtin_fma(au[j][q][e], bv, dr[q]);
          }
        }
    }
    for (int q = 0; q < RPL; ++q) {
      dx[q] = row_sum16(dx[q]);
      dr[q] = row_sum16(dr[q]);
      const double rn = ro[q] - dr[q];
      if (m == 0 && ok[q]) {
        a.x[rowc[q]] = xo[q] + dx[q];
        a.r[rowc[q]] = rn;
        rr += rn * rn;
      }
    }
  }
  const double s = wg_sum(rr, red);
  if (tid == 0) red[0] = s;
  __syncthreads();
  write_partial(red, 1, a.rc);
}

// One block at 16 columns (the x/r update that ends an s-step iteration):
// 16-byte loads, LPR = 16 / (values per 16 bytes) lanes per row, so a wave
// instruction covers 8 (binary64) or 16 (binary32) rows; RQ such row sets
// per step.  Row sums over a row's lanes by DPP; the row's first lane
// writes x and r.
template <typename S>
__global__ ECG_STREAM void k_xr_wide(XRArgs<S> a) {
  constexpr int TPI = 16, VPL = 16 / sizeof(S), LPR = TPI / VPL;
  constexpr int RSET = 64 / LPR, RQ = ECG_XR_RQ;
  constexpr int WROWS = RSET * RQ, NWAVE = kThreads / 64, WGROWS = WROWS * NWAVE;
  using V = typename std::conditional<sizeof(S) == 8, double2, float4>::type;
  __shared__ double bl[TPI];
  __shared__ double red[8];
  if (a.status_in->breakdown) return;     // uniform: the host stops after this iteration
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ri = lane / LPR, pp = lane % LPR;
  if (tid < TPI) bl[tid] = a.beta[0][tid];
  __syncthreads();
  double bv[VPL];
  for (int u = 0; u < VPL; ++u) bv[u] = bl[VPL * pp + u];
  double rr = 0.0;
  const int64_t n = a.n;
  const Steps sp = my_steps((n + WGROWS - 1) / WGROWS);
  for (int64_t step = sp.first; step < sp.end; step += sp.stride) {
    const int64_t row0 = step * WGROWS + wave * WROWS + ri;
    int64_t rowc[RQ];
    V u[RQ], au[RQ];
    double xo[RQ], ro[RQ];
    for (int q = 0; q < RQ; ++q) {
      const int64_t row = row0 + RSET * q;
      rowc[q] = row < n ? row : n - 1;
      u[q] = *reinterpret_cast<const V*>(a.U[0] + rowc[q] * TPI + VPL * pp);
      au[q] = *reinterpret_cast<const V*>(a.AU[0] + rowc[q] * TPI + VPL * pp);
      xo[q] = a.x_in[rowc[q]];
      ro[q] = a.r_in[rowc[q]];
    }
    for (int q = 0; q < RQ; ++q) {
      const S* uv = reinterpret_cast<const S*>(&u[q]);
      const S* av = reinterpret_cast<const S*>(&au[q]);
      double dx = 0.0, dr = 0.0;
      for (int e = 0; e < VPL; ++e) {
        dx = __builtin_fma(static_cast<double>(uv[e]), bv[e], dx);
        dr = __builtin_fma(static_cast<double>(av[e]), bv[e], dr);
      }
      // sums over the LPR lanes of the row (pairs, quads, then eights)
      dx += __builtin_amdgcn_update_dpp(dx, dx, 0xB1, 0xF, 0xF, false);
      dr += __builtin_amdgcn_update_dpp(dr, dr, 0xB1, 0xF, 0xF, false);
      dx += __builtin_amdgcn_update_dpp(dx, dx, 0x4E, 0xF, 0xF, false);
      dr += __builtin_amdgcn_update_dpp(dr, dr, 0x4E, 0xF, 0xF, false);
      if constexpr (LPR == 8) {
        dx += __builtin_amdgcn_update_dpp(dx, dx, 0x141, 0xF, 0xF, false);
        dr += __builtin_amdgcn_update_dpp(dr, dr, 0x141, 0xF, 0xF, false);
      }
      const int64_t row = row0 + RSET * q;
      const double rn = ro[q] - dr;
      if (pp == 0 && row < n) {
        a.x[row] = xo[q] + dx;
        a.r[row] = rn;
        rr += rn * rn;
      }
    }
  }
  const double s = wg_sum(rr, red);
  if (tid == 0) red[0] = s;
  __syncthreads();
  write_partial(red, 1, a.rc);
}

template <int TPI, typename S>
__global__ void k_basis_export(const S* __restrict__ U, const double* __restrict__ rinv,
                               double* __restrict__ V, int64_t n, int t, int ldv, int col0,
                               const int32_t* __restrict__ perm) {
  const int64_t total = n * t;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = idx / t;
    const int c = (int)(idx % t);
    double acc = 0.0;
    for (int k = 0; k <= c; ++k) acc += ld(U + row * TPI + k) * rinv[k * TPI + c];
    const int64_t orow = perm ? perm[row] : row;
    V[orow * ldv + col0 + c] = acc;
  }
}

// grad[p] = -lam[row(p)] x[col(p)] for every stored entry p of the caller's
// matrix.  The kernel walks the solver's (possibly domain-permuted) rows;
// with a permutation, perm maps solver rows to caller rows and emap solver
// entries to caller entries (lam, x and grad are in the caller's order).
__global__ void k_sddmm(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                        const double* __restrict__ lam, const double* __restrict__ x,
                        double* __restrict__ grad, int64_t n, const int32_t* __restrict__ perm,
                        const int32_t* __restrict__ emap) {
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x) {
    const double l = lam[perm ? perm[row] : row];
    for (int p = rowptr[row]; p < rowptr[row + 1]; ++p) {
      const int c = colind[p];
      grad[emap ? emap[p] : p] = -l * x[perm ? perm[c] : c];
    }
  }
}

// Row-major n x k block X to the n x TPI block Xp (padding columns zero);
// with perm, row i of Xp is row perm[i] of X.
__global__ void k_pack(const double* __restrict__ X, int k, double* __restrict__ Xp, int TPI,
                       int64_t n, const int32_t* __restrict__ perm) {
  const int64_t total = n * TPI;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = idx / TPI;
    const int c = (int)(idx % TPI);
    const int64_t src = perm ? perm[row] : row;
    Xp[idx] = c < k ? X[src * k + c] : 0.0;
  }
}

// The first k columns of the n x TPI block Xp to the n x k block X; with
// perm, row i of Xp goes to row perm[i] of X.
__global__ void k_unpack(const double* __restrict__ Xp, int TPI, double* __restrict__ X, int k,
                         int64_t n, const int32_t* __restrict__ perm) {
  const int64_t total = n * k;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = idx / k;
    const int c = (int)(idx % k);
    const int64_t dst = perm ? perm[row] : row;
    X[dst * k + c] = Xp[row * TPI + c];
  }
}

__global__ __launch_bounds__(kThreads) void k_reduce_groups(const double* __restrict__ partials,
                                                            int G, int L, int GS,
                                                            double* __restrict__ groups) {
  const int chunks = (L + kThreads - 1) / kThreads;
  const int g = blockIdx.x / chunks;
  const int e = (blockIdx.x % chunks) * kThreads + threadIdx.x;
  if (e >= L) return;
  const int w0 = g * GS, w1 = min(G, w0 + GS);
  const double* p = partials + (size_t)w0 * L + e;
  double acc = 0.0;
  int w = w0;
  for (; w + 8 <= w1; w += 8) {
    double v[8];
    for (int j = 0; j < 8; ++j) v[j] = p[(size_t)(w - w0 + j) * L];
    for (int j = 0; j < 8; ++j) acc += v[j];
  }
  for (; w < w1; ++w) acc += p[(size_t)(w - w0) * L];
  groups[(size_t)g * L + e] = acc;
}

// Totals over the group sums (index order), then the small dense algebra.
template <int TPI, int TAIL, int NG>
__global__ __launch_bounds__(kThreads) void k_final(const double* __restrict__ groups,
                                                    int ngroups, int L, TailArgs ta) {
  constexpr int T2 = TPI * TPI;
  constexpr int LSP = 3 * T2 + TPI;
  // one-wave tails (16 columns): the sums and 2 TPI of scratch; the
  // work-group tails: the sums and one or two t x t scratch matrices
  constexpr bool WAVE = TPI == 16;
  constexpr int LDSN = TAIL == TAIL_SPMM ? LSP + (WAVE ? 2 * TPI + T2 : T2)
                       : (TAIL == TAIL_CGS || TAIL == TAIL_GRAM ? (NG + (WAVE ? 1 : 2)) * T2
                       : (TAIL == TAIL_PRE ? T2 + (WAVE ? TPI : T2) : 8));
  __shared__ double lds[LDSN];
  // entries four at a time, group sums sixteen at a time: up to 64 loads in
  // flight per thread; each entry is still summed in group order
  constexpr int NE = 4, NQ = 16;
  for (int i0 = threadIdx.x; i0 < L; i0 += NE * blockDim.x) {
    double acc[NE];
    for (int u = 0; u < NE; ++u) acc[u] = 0.0;
    for (int q = 0; q < ngroups; q += NQ) {
      double v[NE][NQ];
      for (int u = 0; u < NE; ++u) {
        const int i = min(i0 + u * (int)blockDim.x, L - 1);
        for (int j = 0; j < NQ; ++j) v[u][j] = groups[(size_t)min(q + j, ngroups - 1) * L + i];
      }
      for (int u = 0; u < NE; ++u)
        for (int j = 0; j < NQ; ++j)
          if (q + j < ngroups) acc[u] += v[u][j];
    }
    for (int u = 0; u < NE; ++u) {
      const int i = i0 + u * (int)blockDim.x;
      if (i < L) lds[i] = acc[u];
    }
  }
  __syncthreads();
  if (ta.sums_out)
    for (int i = threadIdx.x; i < L; i += blockDim.x) ta.sums_out[i] = lds[i];
  if constexpr (TPI > 16 && TAIL != TAIL_NORM) {
    // whole work-group on LDS (the sums region is followed by scratch)
    if constexpr (TAIL == TAIL_SPMM) btail_spmm<TPI>(lds, lds + LSP, ta);
    else if constexpr (TAIL == TAIL_CGS) btail_cgs<TPI>(lds, lds + NG * T2, NG, ta);
    else if constexpr (TAIL == TAIL_GRAM) btail_gram<TPI>(lds, lds + NG * T2, NG, ta);
    else if constexpr (TAIL == TAIL_PRE) btail_pre<TPI>(lds, lds + T2, ta);
    return;
  }
  if constexpr (TAIL == TAIL_NORM) {
    if (threadIdx.x == 0) {
      if (ta.which == 0) ta.status->rho = sqrt(lds[0]);
      else ta.status->rho_true = sqrt(lds[0]);
    }
    return;
  }
  if (threadIdx.x >= TPI) return;   // the small algebra: lanes 0 .. TPI-1 of wave 0
  if constexpr (TAIL == TAIL_SPMM) {
    tail_spmm<TPI>(lds, lds + LSP, ta);
  } else if constexpr (TAIL == TAIL_CGS) {
    tail_cgs<TPI>(lds, lds + NG * T2, NG, ta);
  } else if constexpr (TAIL == TAIL_GRAM) {
    tail_gram<TPI>(lds, lds + NG * T2, NG, ta);
  } else if constexpr (TAIL == TAIL_PRE) {
    tail_pre<TPI>(lds, lds + T2, ta);
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
    else
      cus = 256;
  }
  return cus;
}

int spmm_partials(int tpi, int grid, int max_row) {
  if (uses_cs(tpi) && max_row <= kP64CH) return std::max(1, std::min(grid * kCSGroups, device_cus()));
  return gram_partials(tpi, grid);
}

static int simple_grid(int64_t work) {
  int64_t g = (work + kThreads - 1) / kThreads;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_reduce(const RedCtl& rc, int G, int L, int tpi, int tail, int ng,
                         const TailArgs& ta, hipStream_t st) {
  const int GS = rc.group_size;
  const int ngroups = (G + GS - 1) / GS;
  const int chunks = (L + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_reduce_groups, dim3(ngroups * chunks), dim3(kThreads), 0, st, rc.partials,
                     G, L, GS, rc.groups);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
#define ECG_FIN(TPIV, TL, NGV)                                                               \
  if (tpi == TPIV && tail == TL && ng == NGV) {                                              \
    hipLaunchKernelGGL((k_final<TPIV, TL, NGV>), dim3(1), dim3(kThreads), 0, st, rc.groups,  \
                       ngroups, L, ta);                                                      \
    return hipGetLastError();                                                                \
  }
  if (tail == TAIL_NORM) {   // scalar tail: independent of the block width
    hipLaunchKernelGGL((k_final<16, TAIL_NORM, 0>), dim3(1), dim3(kThreads), 0, st, rc.groups,
                       ngroups, L, ta);
    return hipGetLastError();
  }
  ECG_FIN(16, TAIL_SPMM, 0)
  ECG_FIN(32, TAIL_SPMM, 0)
  ECG_FIN(64, TAIL_SPMM, 0)
  ECG_FIN(16, TAIL_CGS, 1)
  ECG_FIN(32, TAIL_CGS, 1)
  ECG_FIN(64, TAIL_CGS, 1)
  ECG_FIN(16, TAIL_CGS, 2)
  ECG_FIN(32, TAIL_CGS, 2)
  ECG_FIN(64, TAIL_CGS, 2)
  ECG_FIN(16, TAIL_GRAM, 1)
  ECG_FIN(16, TAIL_GRAM, 2)
  ECG_FIN(16, TAIL_GRAM, 3)
  ECG_FIN(32, TAIL_GRAM, 1)
  ECG_FIN(32, TAIL_GRAM, 2)
  ECG_FIN(32, TAIL_GRAM, 3)
  ECG_FIN(64, TAIL_GRAM, 1)
  ECG_FIN(64, TAIL_GRAM, 2)
  ECG_FIN(16, TAIL_PRE, 1)
  ECG_FIN(32, TAIL_PRE, 1)
  ECG_FIN(64, TAIL_PRE, 1)
#undef ECG_FIN
  return hipErrorInvalidValue;
}

hipError_t launch_partition(int64_t nx, int64_t ny, int64_t nz, int px, int py, int pz,
                            int32_t* dom, hipStream_t st) {
  hipLaunchKernelGGL(k_partition, dim3(simple_grid(nx * ny * nz)), dim3(kThreads), 0, st, nx, ny,
                     nz, px, py, pz, dom);
  return hipGetLastError();
}

hipError_t launch_resid(const int32_t* rowptr, const int32_t* colind, const double* vals,
                        const double* b, const double* x, double* r, int64_t n, int grid,
                        RedCtl rc, TailArgs tail, hipStream_t st) {
  hipLaunchKernelGGL(k_resid, dim3(grid), dim3(kThreads), 0, st, rowptr, colind, vals, b, x, r,
                     n, rc, tail);
  return hipGetLastError();
}

template <int TPI, typename S>
hipError_t launch_tsplit(const double* r, const int32_t* dom, S* Z, int64_t n, int grid,
                         hipStream_t st) {
  (void)grid;
  hipLaunchKernelGGL((k_tsplit<TPI, S>), dim3(simple_grid(n * TPI)), dim3(kThreads), 0, st, r,
                     dom, Z, n);
  return hipGetLastError();
}

template <int TPI, typename S>
hipError_t launch_trsv_level(const int32_t* lrows, int count, const int32_t* rp, const int32_t* ci,
                             const double* v, const double* dinv, S* X, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t work = (int64_t)count * TPI;
  const int g = (int)std::min<int64_t>((work + kThreads - 1) / kThreads, 8192);
  hipLaunchKernelGGL((k_trsv_level<TPI, S>), dim3(g), dim3(kThreads), 0, st, lrows, count, rp, ci,
                     v, dinv, X);
  return hipGetLastError();
}

template <int TPI, typename S>
hipError_t launch_update_gram(int nu, int ng, bool ident0, bool write_out, int tail,
                              const UGArgs<S>& a, int grid, hipStream_t st) {
#define ECG_UG(NU, NG, ID, WR, TL, P0X)                                                   \
  if (nu == NU && ng == NG && ident0 == ID && write_out == WR && tail == TL &&             \
      (a.P[0] == a.X[0]) == P0X) {                                                         \
    if constexpr (uses_cs(TPI))   /* one Gram partial per work-group of 4 waves */         \
      hipLaunchKernelGGL((k_update_gram_mf<TPI, S, NU, NG, ID, WR, P0X>),                  \
                         dim3(grid * kCSGroups), dim3(kThreads), 0, st, a);                \
    else if constexpr ((TPI == 32 && ECG_MF32) ||                                         \
                       (TPI == 16 && ECG_MF16F && sizeof(S) == 4) ||                        \
                       (TPI == 16 && ECG_MF16D && sizeof(S) == 8 && NG > 0))                \
      hipLaunchKernelGGL((k_update_gram_mf<TPI, S, NU, NG, ID, WR, P0X>), dim3(grid),      \
                         dim3(kThreads), 0, st, a);                                        \
    else                                                                                   \
      hipLaunchKernelGGL((k_update_gram<TPI, S, NU, NG, ID, WR, TL, P0X>), dim3(grid),     \
                         dim3(kThreads), 0, st, a);                                        \
    return hipGetLastError();                                                              \
  }
  // first CGS pass of blocks m = 2 and m >= 3 (fused with the second Gram)
  ECG_UG(2, 1, false, true, TAIL_CGS, true)
  ECG_UG(3, 2, false, true, TAIL_CGS, true)
  // second CGS pass
  ECG_UG(2, 0, true, true, TAIL_NONE, false)
  ECG_UG(3, 0, true, true, TAIL_NONE, false)
  // SRE-CG2 chunks: first update chunk, in-place update chunks, Gram chunks
  ECG_UG(3, 0, false, true, TAIL_NONE, false)
  ECG_UG(2, 0, false, true, TAIL_NONE, false)
  ECG_UG(4, 0, true, true, TAIL_NONE, false)
  ECG_UG(1, 1, true, false, TAIL_NONE, false)
  ECG_UG(1, 2, true, false, TAIL_NONE, false)
  ECG_UG(1, 3, true, false, TAIL_NONE, false)
  // Pre-CholQR: Euclidean Gram of a block with itself, and the scaling
  ECG_UG(1, 1, true, false, TAIL_NONE, true)
  ECG_UG(1, 0, false, true, TAIL_NONE, false)
#undef ECG_UG
  return hipErrorInvalidValue;
}

// The product kernel for a block width and storage type: 16 columns
// k_spmm_wide (binary64) / k_spmm_widef (binary32), 32 columns k_spmm_w32 /
// k_spmm_w32f, 64 columns the producer/consumer k_spmm64pc (rows of at most
// kP64CH entries) or k_spmm64 (any rows, and the product without Grams).
template <int TPI, typename S, typename SA>
hipError_t launch_spmm(bool grams, bool has_prev, int tail, const SpArgs<S, SA>& a, int grid,
                       hipStream_t st) {
  static_assert(std::is_same<S, SA>::value, "block and matrix values share the storage type");
  if (grams && tail != TAIL_SPMM) return hipErrorInvalidValue;
  constexpr bool F64 = std::is_same<S, double>::value;
#define ECG_SP3(K)                                                                         \
  do {                                                                                     \
    if (!grams) hipLaunchKernelGGL((K<false, false>), dim3(grid), dim3(kThreads), 0, st, a); \
    else if (has_prev)                                                                     \
      hipLaunchKernelGGL((K<true, true>), dim3(grid), dim3(kThreads), 0, st, a);           \
    else hipLaunchKernelGGL((K<true, false>), dim3(grid), dim3(kThreads), 0, st, a);       \
  } while (0)
  if constexpr (TPI == 16 && F64) ECG_SP3(k_spmm_wide);
  else if constexpr (TPI == 16) ECG_SP3(k_spmm_widef);
  else if constexpr (TPI == 32 && F64) ECG_SP3(k_spmm_w32);
  else if constexpr (TPI == 32) ECG_SP3(k_spmm_w32f);
  else {
    // kCSGroups work-groups (one Gram partial each) per unit of `grid`, or
    // spmm_partials(TPI, grid, max_row) work-groups of the producer/consumer form
    if (!grams) {
      hipLaunchKernelGGL((k_spmm64<S, SA, false, false>), dim3(grid * kCSGroups), dim3(kThreads),
                         0, st, a);
    } else if (a.max_row <= kP64CH) {
      const dim3 g(spmm_partials(TPI, grid, a.max_row)), blk(kP64THREADS);
      if (has_prev) hipLaunchKernelGGL((k_spmm64pc<S, SA, true>), g, blk, 0, st, a);
      else hipLaunchKernelGGL((k_spmm64pc<S, SA, false>), g, blk, 0, st, a);
    } else if (has_prev) {
      hipLaunchKernelGGL((k_spmm64<S, SA, true, true>), dim3(grid * kCSGroups), dim3(kThreads),
                         0, st, a);
    } else {
      hipLaunchKernelGGL((k_spmm64<S, SA, true, false>), dim3(grid * kCSGroups), dim3(kThreads),
                         0, st, a);
    }
  }
#undef ECG_SP3
  return hipGetLastError();
}

template <int TPI, typename S>
hipError_t launch_xr(const XRArgs<S>& a, int grid, hipStream_t st) {
  if (ECG_XR_WIDE && TPI == 16 && a.nb == 1)
    hipLaunchKernelGGL((k_xr_wide<S>), dim3(grid), dim3(kThreads), 0, st, a);
  else if (a.nb == 1)
    hipLaunchKernelGGL((k_xr<TPI, S, 1>), dim3(grid), dim3(kThreads), 0, st, a);
  else
    hipLaunchKernelGGL((k_xr<TPI, S, 4>), dim3(grid), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

template <int TPI, typename S>
hipError_t launch_basis_export(const S* U, const double* rinv, double* V, int64_t n, int t,
                               int ldv, int col0, const int32_t* perm, hipStream_t st) {
  hipLaunchKernelGGL((k_basis_export<TPI, S>), dim3(simple_grid(n * t)), dim3(kThreads), 0, st,
                     U, rinv, V, n, t, ldv, col0, perm);
  return hipGetLastError();
}

hipError_t launch_sddmm(const int32_t* rowptr, const int32_t* colind, const double* lam,
                        const double* x, double* grad, int64_t n, const int32_t* perm,
                        const int32_t* emap, hipStream_t st) {
  hipLaunchKernelGGL(k_sddmm, dim3(simple_grid(n)), dim3(kThreads), 0, st, rowptr, colind, lam, x,
                     grad, n, perm, emap);
  return hipGetLastError();
}

hipError_t launch_pack(const double* X, int k, double* Xp, int TPI, int64_t n,
                       const int32_t* perm, hipStream_t st) {
  hipLaunchKernelGGL(k_pack, dim3(simple_grid(n * TPI)), dim3(kThreads), 0, st, X, k, Xp, TPI, n,
                     perm);
  return hipGetLastError();
}

hipError_t launch_unpack(const double* Xp, int TPI, double* X, int k, int64_t n,
                         const int32_t* perm, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack, dim3(simple_grid(n * k)), dim3(kThreads), 0, st, Xp, TPI, X, k, n,
                     perm);
  return hipGetLastError();
}

#define ECG_INST(TPI, S)                                                                   \
  template hipError_t launch_tsplit<TPI, S>(const double*, const int32_t*, S*, int64_t, int, \
                                            hipStream_t);                                  \
  template hipError_t launch_trsv_level<TPI, S>(const int32_t*, int, const int32_t*,         \
                                                const int32_t*, const double*, const double*, \
                                                S*, hipStream_t);                          \
  template hipError_t launch_update_gram<TPI, S>(int, int, bool, bool, int, const UGArgs<S>&, \
                                                 int, hipStream_t);                        \
  template hipError_t launch_xr<TPI, S>(const XRArgs<S>&, int, hipStream_t);               \
  template hipError_t launch_basis_export<TPI, S>(const S*, const double*, double*, int64_t, \
                                                  int, int, int, const int32_t*, hipStream_t);
ECG_INST(16, double)
ECG_INST(32, double)
ECG_INST(64, double)
ECG_INST(16, float)
ECG_INST(32, float)
ECG_INST(64, float)
#undef ECG_INST

#define ECG_INST_SP(TPI, S, SA)                                                            \
  template hipError_t launch_spmm<TPI, S, SA>(bool, bool, int, const SpArgs<S, SA>&, int,  \
                                              hipStream_t);
ECG_INST_SP(16, double, double)
ECG_INST_SP(32, double, double)
ECG_INST_SP(64, double, double)
ECG_INST_SP(16, float, float)
ECG_INST_SP(32, float, float)
ECG_INST_SP(64, float, float)
#undef ECG_INST_SP

}  // namespace ecg
