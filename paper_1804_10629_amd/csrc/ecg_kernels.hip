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
// The block update out[r] = sum_b X_b[r] C_b (C_b small, t x t) runs on the
// FP64 VALU, broadcasting X_b[r][k] across its DPP row (row_newbcast) and
// reading C_b from LDS.
//
// Reductions never use floating-point atomics: work-group partials are
// combined by a fixed-order two-level tree (RedCtl), so results are
// bitwise reproducible run to run.  The last work-group then runs the small
// dense algebra (Cholesky of the t x t Gram, R^{-1}, the next block's CGS
// coefficients) so no host round trip is needed between blocks.

#include "ecg_kernels.h"

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

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename S>
__device__ __forceinline__ double ld(const S* p) { return static_cast<double>(*p); }

template <int TPI>
struct Cfg {
  static constexpr int EPL = TPI / 16;                              // columns per lane
  static constexpr int RPL = TPI == 16 ? 4 : (TPI == 32 ? 2 : 1);   // row quads per lane
  static constexpr int WROWS = 4 * RPL;                             // rows per wave step
  static constexpr int NWAVE = kThreads / 64;
  static constexpr int WGROWS = WROWS * NWAVE;                      // rows per WG step
  static constexpr int T2 = TPI * TPI;
};

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

// See RedCtl.  `red` (LDS, L doubles) holds this work-group's partial on
// entry and, in the one work-group that returns true, the grid total.
__device__ bool grid_reduce(double* red, int L, const RedCtl& rc) {
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int G = gridDim.x, GS = rc.group_size;
  const int g = blockIdx.x / GS;
  const int ngroups = (G + GS - 1) / GS;
  const int gsize = min(GS, G - g * GS);
  double* mine = rc.partials + (size_t)blockIdx.x * L;
  for (int i = tid; i < L; i += blockDim.x) mine[i] = red[i];
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    unsigned prev = __hip_atomic_fetch_add(&rc.counters[g], 1u, __ATOMIC_ACQ_REL,
                                           __HIP_MEMORY_SCOPE_AGENT);
    s_last = (prev == (unsigned)(gsize - 1));
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  double* gsum = rc.groups + (size_t)g * L;
  const double* base = rc.partials + (size_t)g * GS * L;
  for (int i = tid; i < L; i += blockDim.x) {
    double acc = 0.0;
    for (int w = 0; w < gsize; ++w) acc += base[(size_t)w * L + i];
    gsum[i] = acc;
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    rc.counters[g] = 0u;
    unsigned prev = __hip_atomic_fetch_add(&rc.counters[ngroups], 1u, __ATOMIC_ACQ_REL,
                                           __HIP_MEMORY_SCOPE_AGENT);
    s_last = (prev == (unsigned)(ngroups - 1));
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  for (int i = tid; i < L; i += blockDim.x) {
    double acc = 0.0;
    for (int q = 0; q < ngroups; ++q) acc += rc.groups[(size_t)q * L + i];
    red[i] = acc;
  }
  if (tid == 0) rc.counters[ngroups] = 0u;
  __syncthreads();
  return true;
}

// ---------------------------------------------------------------------------
// Small dense algebra on t x t matrices in LDS (row-major, leading dim TPI),
// run by one work-group.
// ---------------------------------------------------------------------------

// In-place upper Cholesky G = R^t R of the leading t x t block (upper
// triangle of G used).  Breakdown iff a pivot is <= 0 or not finite.
// On return the block holds R with zeros below the diagonal and in the
// padding.
template <int TPI>
__device__ void chol_upper_inplace(double* G, int t, int* bad) {
  const int tid = threadIdx.x;
  for (int j = 0; j < t; ++j) {
    if (tid == 0) {
      const double piv = G[j * TPI + j];
      if (!(piv > 0.0) || !isfinite(piv)) {
        *bad = 1;
        G[j * TPI + j] = 1.0;
      } else {
        G[j * TPI + j] = sqrt(piv);
      }
    }
    __syncthreads();
    const double d = G[j * TPI + j];
    for (int c = j + 1 + tid; c < t; c += blockDim.x) G[j * TPI + c] /= d;
    __syncthreads();
    const int w = t - j - 1;
    for (int idx = tid; idx < w * w; idx += blockDim.x) {
      const int i = j + 1 + idx / w, c = j + 1 + idx % w;
      if (i <= c) G[i * TPI + c] -= G[j * TPI + i] * G[j * TPI + c];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < TPI * TPI; idx += blockDim.x) {
    const int i = idx / TPI, c = idx % TPI;
    if (i > c || i >= t || c >= t) G[idx] = 0.0;
  }
  __syncthreads();
}

// In-place inverse of the upper triangular leading t x t block.
template <int TPI>
__device__ void trinv_upper_inplace(double* R, int t, double* tmp) {
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

// C = op(A) B on the leading t x t blocks (op = transpose if ta); the
// padding of C is zero.  C may live in global memory; A, B in LDS.
template <int TPI>
__device__ void small_mm(const double* A, bool ta, const double* B, double* C, int t,
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
__device__ void copy_mat(const double* src, double* dst) {
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
__device__ void tail_spmm(double* sums, double* tmp, const TailArgs& ta) {
  constexpr int T2 = TPI * TPI;
  __shared__ int s_bad;
  const int t = ta.t, tid = threadIdx.x;
  double* G = sums;
  double* F = sums + T2;
  double* E = sums + 2 * T2;
  double* a = sums + 3 * T2;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  chol_upper_inplace<TPI>(G, t, &s_bad);
  trinv_upper_inplace<TPI>(G, t, tmp);           // G now holds R^{-1}
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
  small_mm<TPI>(F, false, G, tmp, t, 1.0);       // tmp = F R^{-1}
  small_mm<TPI>(G, true, tmp, F, t, 1.0);        // F <- H_m
  small_mm<TPI>(G, false, F, ta.cnext + T2, t, -1.0);
  if (ta.m >= 2 && ta.rinv_p1 != nullptr) {
    small_mm<TPI>(E, false, G, tmp, t, 1.0);     // tmp = E R_m^{-1}
    copy_mat<TPI>(ta.rinv_p1, E);                // E <- R_{m-1}^{-1}
    small_mm<TPI>(E, true, tmp, F, t, 1.0);      // F <- H_{m-1}
    small_mm<TPI>(E, false, F, ta.cnext + 2 * T2, t, -1.0);
  }
  if (tid == 0 && s_bad && ta.status->breakdown == 0) {
    ta.status->breakdown = 1;
    ta.status->breakdown_block = ta.m;
  }
}

// Tail after the first CGS update: sums hold H2'_g = AU_g^t Z' (g < ng);
// D_g = -R_g^{-1} R_g^{-t} H2'_g, where g = 0 is block m-1 and g = 1 block m-2.
template <int TPI>
__device__ void tail_cgs(double* sums, double* tmp, int ng, const TailArgs& ta) {
  constexpr int T2 = TPI * TPI;
  double* Rs = tmp;
  double* T = tmp + T2;
  for (int g = 0; g < ng; ++g) {
    copy_mat<TPI>(g == 0 ? ta.rinv_p1 : ta.rinv_p2, Rs);
    small_mm<TPI>(Rs, true, sums + g * T2, T, ta.t, 1.0);
    small_mm<TPI>(Rs, false, T, ta.dcoef + g * T2, ta.t, -1.0);
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
__global__ __launch_bounds__(kThreads) void k_resid(const int32_t* __restrict__ rowptr,
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
  if (grid_reduce(red, 1, rc) && threadIdx.x == 0) {
    if (ta.which == 0) ta.status->rho = sqrt(red[0]);
    else ta.status->rho_true = sqrt(red[0]);
  }
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

// out[r] = (ident0 ? X0[r] : 0) + sum_b X_b[r] C_b ; H_g = sum_r P_g[r]^t out[r]
template <int TPI, typename S, int NU, int NG, bool IDENT0, bool WRITE, int TAIL>
__global__ __launch_bounds__(kThreads) void k_update_gram(UGArgs<S> a) {
  using C = Cfg<TPI>;
  constexpr int EPL = C::EPL, RPL = C::RPL, T2 = C::T2;
  constexpr int NCOEF = NU - (IDENT0 ? 1 : 0);
  constexpr int BODY = NCOEF * T2;
  constexpr int TAILSZ = (TAIL == TAIL_CGS) ? (NG + 2) * T2 : NG * T2;
  constexpr int LDSN = (BODY > TAILSZ ? BODY : TAILSZ) > 1 ? (BODY > TAILSZ ? BODY : TAILSZ) : 1;
  __shared__ double lds[LDSN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, rq = lane >> 4;

  // coefficient matrices into LDS
  for (int b = 0; b < NCOEF; ++b) {
    const double* src = a.C[b + (IDENT0 ? 1 : 0)];
    for (int idx = tid; idx < T2; idx += blockDim.x) lds[b * T2 + idx] = src[idx];
  }
  __syncthreads();

  d4 acc[NG > 0 ? NG : 1][EPL][EPL];
  for (int g = 0; g < (NG > 0 ? NG : 1); ++g)
    for (int i = 0; i < EPL; ++i)
      for (int j = 0; j < EPL; ++j) acc[g][i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int64_t n = a.n;
  for (int64_t step = blockIdx.x; step * C::WGROWS < n; step += gridDim.x) {
    // keep the coefficient reads from LDS inside the loop (registers would
    // not hold them for TPI >= 32, and hoisting lowers occupancy)
    asm volatile("" ::: "memory");
    const int64_t row0 = step * C::WGROWS + wave * C::WROWS + rq;
    int64_t rowc[RPL];     // clamped rows: loads stay in bounds, values are masked
    bool ok[RPL];
    for (int q = 0; q < RPL; ++q) {
      const int64_t row = row0 + 4 * q;
      ok[q] = row < n;
      rowc[q] = ok[q] ? row : n - 1;
    }
    double xv[NCOEF > 0 ? NCOEF : 1][RPL][EPL];
    for (int b = 0; b < NCOEF; ++b) {
      const S* X = a.X[b + (IDENT0 ? 1 : 0)];
      for (int q = 0; q < RPL; ++q)
        for (int e = 0; e < EPL; ++e) {
          const double v = ld(X + rowc[q] * TPI + m + 16 * e);
          xv[b][q][e] = ok[q] ? v : 0.0;
        }
    }
    double o[RPL][EPL];
    for (int q = 0; q < RPL; ++q)
      for (int e = 0; e < EPL; ++e) {
        if constexpr (IDENT0) {
          const double v = ld(a.X[0] + rowc[q] * TPI + m + 16 * e);
          o[q][e] = ok[q] ? v : 0.0;
        } else {
          o[q][e] = 0.0;
        }
      }
    static_for<NCOEF>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      const double* Cs = lds + b * T2;
      static_for<EPL>([&](auto ec) {
        constexpr int e2 = decltype(ec)::value;
        static_for<16>([&](auto nc) {
          constexpr int nn = decltype(nc)::value;
          const int k = 16 * e2 + nn;
          double cv[EPL];
          for (int e = 0; e < EPL; ++e) cv[e] = Cs[k * TPI + m + 16 * e];
          for (int q = 0; q < RPL; ++q)
            for (int e = 0; e < EPL; ++e)
              o[q][e] = (nn == 0 && e == 0) ? fmac_bcast<nn, true>(o[q][e], xv[b][q][e2], cv[e])
                                            : fmac_bcast<nn, false>(o[q][e], xv[b][q][e2], cv[e]);
        });
      });
    });
    if constexpr (WRITE) {
      for (int q = 0; q < RPL; ++q)
        if (ok[q])
          for (int e = 0; e < EPL; ++e)
            a.out[rowc[q] * TPI + m + 16 * e] = static_cast<S>(o[q][e]);
    }
    if constexpr (NG > 0) {
      for (int g = 0; g < NG; ++g) {
        double pv[RPL][EPL];
        for (int q = 0; q < RPL; ++q)
          for (int e = 0; e < EPL; ++e) {
            const double v = ld(a.P[g] + rowc[q] * TPI + m + 16 * e);
            pv[q][e] = ok[q] ? v : 0.0;
          }
        for (int q = 0; q < RPL; ++q)
          for (int i = 0; i < EPL; ++i)
            for (int j = 0; j < EPL; ++j) acc[g][i][j] = mfma16(pv[q][i], o[q][j], acc[g][i][j]);
      }
    }
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
    if (grid_reduce(lds, L, a.rc)) {
      if (a.tail.sums_out)
        for (int i = tid; i < L; i += blockDim.x) a.tail.sums_out[i] = lds[i];
      if constexpr (TAIL == TAIL_CGS) tail_cgs<TPI>(lds, lds + L, NG, a.tail);
    }
  }
}

// AZ = A Z (row by row) with the Gram epilogue G = Z^t AZ, F = AZ^t AZ,
// E = AZprev^t AZ and a = Z^t r.
template <int TPI, typename S, typename SA, bool GRAMS, bool HAS_PREV, int TAIL>
__global__ __launch_bounds__(kThreads) void k_spmm(SpArgs<S, SA> a) {
  using C = Cfg<TPI>;
  constexpr int EPL = C::EPL, RPL = C::RPL, T2 = C::T2;
  constexpr int L = 3 * T2 + TPI;
  constexpr int LDSN = GRAMS ? (TAIL == TAIL_SPMM ? L + T2 : L) : 1;
  __shared__ double lds[LDSN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, rq = lane >> 4;

  d4 accG[EPL][EPL], accF[EPL][EPL], accE[EPL][EPL];
  double av[EPL];
  for (int i = 0; i < EPL; ++i) {
    av[i] = 0.0;
    for (int j = 0; j < EPL; ++j) {
      accG[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      accF[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      accE[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  }
  const int64_t n = a.n;
  for (int64_t step = blockIdx.x; step * C::WGROWS < n; step += gridDim.x) {
    const int64_t row0 = step * C::WGROWS + wave * C::WROWS + rq;
    double y[RPL][EPL];
    for (int q = 0; q < RPL; ++q) {
      const int64_t row = row0 + 4 * q;
      for (int e = 0; e < EPL; ++e) y[q][e] = 0.0;
      if (row < n) {
        const int p0 = a.rowptr[row], p1 = a.rowptr[row + 1];
        for (int p = p0; p < p1; ++p) {
          const int64_t col = a.colind[p];
          const double v = static_cast<double>(a.vals[p]);
          for (int e = 0; e < EPL; ++e)
            y[q][e] = __builtin_fma(v, ld(a.Z + col * TPI + m + 16 * e), y[q][e]);
        }
        for (int e = 0; e < EPL; ++e) a.AZ[row * TPI + m + 16 * e] = static_cast<S>(y[q][e]);
      }
    }
    if constexpr (GRAMS) {
      double z[RPL][EPL], pz[RPL][EPL], rv[RPL];
      for (int q = 0; q < RPL; ++q) {
        const int64_t row = row0 + 4 * q;
        rv[q] = (row < n && a.rvec) ? a.rvec[row] : 0.0;
        for (int e = 0; e < EPL; ++e) {
          // the stored (rounded) value of AZ enters the Grams
          y[q][e] = static_cast<double>(static_cast<S>(y[q][e]));
          z[q][e] = row < n ? ld(a.Z + row * TPI + m + 16 * e) : 0.0;
          pz[q][e] = (HAS_PREV && row < n) ? ld(a.AZprev + row * TPI + m + 16 * e) : 0.0;
        }
      }
      for (int q = 0; q < RPL; ++q) {
        for (int i = 0; i < EPL; ++i) {
          av[i] = __builtin_fma(z[q][i], rv[q], av[i]);
          for (int j = 0; j < EPL; ++j) {
            accG[i][j] = mfma16(z[q][i], y[q][j], accG[i][j]);
            accF[i][j] = mfma16(y[q][i], y[q][j], accF[i][j]);
            if constexpr (HAS_PREV) accE[i][j] = mfma16(pz[q][i], y[q][j], accE[i][j]);
          }
        }
      }
    }
  }
  if constexpr (GRAMS) {
    // a: reduce over the four row lanes of each column, then over waves
    for (int i = 0; i < EPL; ++i) {
      av[i] += __shfl_xor(av[i], 16, 64);
      av[i] += __shfl_xor(av[i], 32, 64);
    }
    for (int w = 0; w < C::NWAVE; ++w) {
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
    if (grid_reduce(lds, L, a.rc)) {
      if (a.tail.sums_out)
        for (int i = tid; i < L; i += blockDim.x) a.tail.sums_out[i] = lds[i];
      if constexpr (TAIL == TAIL_SPMM) tail_spmm<TPI>(lds, lds + L, a.tail);
    }
  }
}

// x += sum_i U_i beta_i ; r -= sum_i AU_i beta_i ; ||r||^2
template <int TPI, typename S>
__global__ __launch_bounds__(kThreads) void k_xr(XRArgs<S> a) {
  constexpr int EPL = TPI / 16, RPL = 4, WROWS = 4 * RPL, NWAVE = kThreads / 64;
  constexpr int WGROWS = WROWS * NWAVE;
  __shared__ double bl[kMaxS * TPI];
  __shared__ double red[8];
  if (a.status_in->breakdown) return;     // uniform: the host stops after this iteration
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, rq = lane >> 4;
  for (int i = 0; i < a.nb; ++i)
    for (int c = tid; c < TPI; c += blockDim.x) bl[i * TPI + c] = a.beta[i][c];
  __syncthreads();
  double rr = 0.0;
  const int64_t n = a.n;
  for (int64_t step = blockIdx.x; step * WGROWS < n; step += gridDim.x) {
    const int64_t row0 = step * WGROWS + wave * WROWS + rq;
    double dx[RPL], dr[RPL];
    for (int q = 0; q < RPL; ++q) {
      dx[q] = 0.0;
      dr[q] = 0.0;
    }
    for (int i = 0; i < a.nb; ++i) {
      for (int q = 0; q < RPL; ++q) {
        const int64_t row = row0 + 4 * q;
        if (row < n)
          for (int e = 0; e < EPL; ++e) {
            const double bv = bl[i * TPI + m + 16 * e];
            dx[q] = __builtin_fma(ld(a.U[i] + row * TPI + m + 16 * e), bv, dx[q]);
            dr[q] = __builtin_fma(ld(a.AU[i] + row * TPI + m + 16 * e), bv, dr[q]);
          }
      }
    }
    for (int q = 0; q < RPL; ++q) {
      for (int off = 8; off > 0; off >>= 1) {
        dx[q] += __shfl_xor(dx[q], off, 16);
        dr[q] += __shfl_xor(dr[q], off, 16);
      }
      const int64_t row = row0 + 4 * q;
      if (m == 0 && row < n) {
        a.x[row] += dx[q];
        const double rn = a.r[row] - dr[q];
        a.r[row] = rn;
        rr += rn * rn;
      }
    }
  }
  const double s = wg_sum(rr, red);
  if (tid == 0) red[0] = s;
  __syncthreads();
  if (grid_reduce(red, 1, a.rc) && tid == 0) a.tail.status->rho = sqrt(red[0]);
}

template <int TPI, typename S>
__global__ void k_basis_export(const S* __restrict__ U, const double* __restrict__ rinv,
                               double* __restrict__ V, int64_t n, int t, int ldv, int col0) {
  const int64_t total = n * t;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = idx / t;
    const int c = (int)(idx % t);
    double acc = 0.0;
    for (int k = 0; k <= c; ++k) acc += ld(U + row * TPI + k) * rinv[k * TPI + c];
    V[row * ldv + col0 + c] = acc;
  }
}

__global__ void k_sddmm(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                        const double* __restrict__ lam, const double* __restrict__ x,
                        double* __restrict__ grad, int64_t n) {
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x) {
    const double l = lam[row];
    for (int p = rowptr[row]; p < rowptr[row + 1]; ++p) grad[p] = -l * x[colind[p]];
  }
}

__global__ void k_pack(const double* __restrict__ X, int k, double* __restrict__ Xp, int TPI,
                       int64_t n) {
  const int64_t total = n * TPI;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = idx / TPI;
    const int c = (int)(idx % TPI);
    Xp[idx] = c < k ? X[row * k + c] : 0.0;
  }
}

__global__ void k_unpack(const double* __restrict__ Xp, int TPI, double* __restrict__ X, int k,
                         int64_t n) {
  const int64_t total = n * k;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = idx / k;
    const int c = (int)(idx % k);
    X[idx] = Xp[row * TPI + c];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static int simple_grid(int64_t work) {
  int64_t g = (work + kThreads - 1) / kThreads;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
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
hipError_t launch_update_gram(int nu, int ng, bool ident0, bool write_out, int tail,
                              const UGArgs<S>& a, int grid, hipStream_t st) {
#define ECG_UG(NU, NG, ID, WR, TL)                                                        \
  if (nu == NU && ng == NG && ident0 == ID && write_out == WR && tail == TL) {             \
    hipLaunchKernelGGL((k_update_gram<TPI, S, NU, NG, ID, WR, TL>), dim3(grid),           \
                       dim3(kThreads), 0, st, a);                                         \
    return hipGetLastError();                                                             \
  }
  // first CGS pass of blocks m = 2 and m >= 3 (fused with the second Gram)
  ECG_UG(2, 1, false, true, TAIL_CGS)
  ECG_UG(3, 2, false, true, TAIL_CGS)
  // second CGS pass
  ECG_UG(2, 0, true, true, TAIL_NONE)
  ECG_UG(3, 0, true, true, TAIL_NONE)
#undef ECG_UG
  return hipErrorInvalidValue;
}

template <int TPI, typename S, typename SA>
hipError_t launch_spmm(bool grams, bool has_prev, int tail, const SpArgs<S, SA>& a, int grid,
                       hipStream_t st) {
  if (!grams) {
    hipLaunchKernelGGL((k_spmm<TPI, S, SA, false, false, TAIL_NONE>), dim3(grid), dim3(kThreads),
                       0, st, a);
  } else if (tail != TAIL_SPMM) {
    return hipErrorInvalidValue;
  } else if (has_prev) {
    hipLaunchKernelGGL((k_spmm<TPI, S, SA, true, true, TAIL_SPMM>), dim3(grid), dim3(kThreads),
                       0, st, a);
  } else {
    hipLaunchKernelGGL((k_spmm<TPI, S, SA, true, false, TAIL_SPMM>), dim3(grid), dim3(kThreads),
                       0, st, a);
  }
  return hipGetLastError();
}

template <int TPI, typename S>
hipError_t launch_xr(const XRArgs<S>& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_xr<TPI, S>), dim3(grid), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

template <int TPI, typename S>
hipError_t launch_basis_export(const S* U, const double* rinv, double* V, int64_t n, int t,
                               int ldv, int col0, hipStream_t st) {
  hipLaunchKernelGGL((k_basis_export<TPI, S>), dim3(simple_grid(n * t)), dim3(kThreads), 0, st,
                     U, rinv, V, n, t, ldv, col0);
  return hipGetLastError();
}

hipError_t launch_sddmm(const int32_t* rowptr, const int32_t* colind, const double* lam,
                        const double* x, double* grad, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_sddmm, dim3(simple_grid(n)), dim3(kThreads), 0, st, rowptr, colind, lam, x,
                     grad, n);
  return hipGetLastError();
}

hipError_t launch_pack(const double* X, int k, double* Xp, int TPI, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_pack, dim3(simple_grid(n * TPI)), dim3(kThreads), 0, st, X, k, Xp, TPI, n);
  return hipGetLastError();
}

hipError_t launch_unpack(const double* Xp, int TPI, double* X, int k, int64_t n,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_unpack, dim3(simple_grid(n * k)), dim3(kThreads), 0, st, Xp, TPI, X, k,
                     n);
  return hipGetLastError();
}

#define ECG_INST(TPI, S)                                                                   \
  template hipError_t launch_tsplit<TPI, S>(const double*, const int32_t*, S*, int64_t, int, \
                                            hipStream_t);                                  \
  template hipError_t launch_update_gram<TPI, S>(int, int, bool, bool, int, const UGArgs<S>&, \
                                                 int, hipStream_t);                        \
  template hipError_t launch_xr<TPI, S>(const XRArgs<S>&, int, hipStream_t);               \
  template hipError_t launch_basis_export<TPI, S>(const S*, const double*, double*, int64_t, \
                                                  int, int, int, hipStream_t);
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
