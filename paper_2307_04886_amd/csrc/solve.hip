// V-cycle kernels (Alg. 2): multicolour Gauss-Seidel, residual, restriction
// by P^T, prolongation and correction, coarsest-level solve, norms.
//
// Matrices (A_l and P_l^T) are in the colour-sorted SELL-64 layout: slice s
// holds rows 64s..64s+63, entry t of row r at ptr[s] + 64 t + (r mod 64).
// Every row sum adds its terms sequentially in the CSR order of the original
// row, so each row is the same floating-point computation as in the method's
// definition.  Two row kernels exist:
//  - one lane per row (level 0: about 7 entries, streaming, coalesced across
//    the 64 consecutive rows of a slice), loads issued kChunkFine at a time;
//  - R lanes per row (Galerkin levels: 15-40 entries, latency-bound): the R
//    lanes load and multiply the row's entries in parallel and the first lane
//    of the group adds the products in entry order (wavefront shuffles).
#include "gmg_internal.hpp"

namespace gmg {

namespace {

constexpr int kChunkFine = 8;

// One lane per row: sum_t val[t] * x[col[t]] in entry order, skipping column
// `skip`; the row's loads are issued CH at a time before any is consumed.
template <int CH>
__device__ __forceinline__ double row_sum_seq(const SellView& A, int32_t r, const double* x, int32_t skip) {
  const int32_t base = A.ptr[r / kSlice] + (r & (kSlice - 1));
  const int32_t len = A.len[r];
  double acc = 0.0;
  for (int32_t t0 = 0; t0 < len; t0 += CH) {
    int32_t j[CH];
    double v[CH], xv[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const bool ok = t0 + u < len;
      j[u] = ok ? A.col[base + (t0 + u) * kSlice] : skip;
      v[u] = ok ? A.val[base + (t0 + u) * kSlice] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      xv[u] = 0.0;
      if (t0 + u < len && j[u] != skip) xv[u] = x[j[u]];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (t0 + u < len && j[u] != skip) acc = acc + v[u] * xv[u];
  }
  return acc;
}

__device__ __forceinline__ double row_sum1(const SellView& A, int32_t r, const double* x, int32_t skip) {
  return row_sum_seq<kChunkFine>(A, r, x, skip);
}

// R lanes per row (R divides 64; the lanes of a group are consecutive).  All
// lanes of the wavefront must call this (shuffles); `active` marks lanes whose
// group has a row.  maxlen bounds every row length (uniform).  The result is
// valid on the group's first lane.
template <int R>
__device__ __forceinline__ double row_sumR(const SellView& A, int32_t r, bool active, const double* x,
                                           int32_t skip, int32_t maxlen) {
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (R - 1);
  const int lane0 = lane - sub;
  int32_t base = 0, len = 0;
  if (active) {
    base = A.ptr[r / kSlice] + (r & (kSlice - 1));
    len = A.len[r];
  }
  double acc = 0.0;
  for (int32_t t0 = 0; t0 < maxlen; t0 += R * kLaneEntries) {
    int32_t j[kLaneEntries];
    double v[kLaneEntries], p[kLaneEntries];
    uint32_t mask = 0;
#pragma unroll
    for (int k = 0; k < kLaneEntries; ++k) {
      const int32_t t = t0 + sub + R * k;
      const bool ok = t < len;
      j[k] = ok ? A.col[base + t * kSlice] : skip;
      v[k] = ok ? A.val[base + t * kSlice] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kLaneEntries; ++k) {
      const bool ok = (t0 + sub + R * k < len) && j[k] != skip;
      p[k] = 0.0;
      if (ok) p[k] = v[k] * x[j[k]];
      mask |= ok ? (1u << k) : 0u;
    }
    uint32_t m[R];
#pragma unroll
    for (int s = 0; s < R; ++s) m[s] = __shfl(mask, lane0 + s, kWave);
#pragma unroll
    for (int k = 0; k < kLaneEntries; ++k)
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const double q = __shfl(p[k], lane0 + s, kWave);
        if ((m[s] >> k) & 1u) acc = acc + q;
      }
  }
  return acc;
}

__device__ __forceinline__ void prolong_row(const LevelView& L, const double* __restrict__ xc, double* x,
                                            int32_t i) {
  const int32_t c = L.q_cnt[i];
  double acc = 0.0;
  double v[3], u[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    v[t] = L.q_val[(int64_t)t * L.n + i];
    u[t] = xc[L.q_col[(int64_t)t * L.n + i]];
  }
#pragma unroll
  for (int t = 0; t < 3; ++t)
    if (t < c) acc = acc + v[t] * u[t];
  x[i] = x[i] + acc;
}

// One colour of a Gauss-Seidel sweep on level 0, rows [r0, r1):
//   x_r <- (b_r - sum_{j != r} A_rj x_j) / A_rr.
// Rows of one colour are not coupled, so they update in parallel.
__global__ void __launch_bounds__(kBlock) k_gs_color_fine(SellView A, const double* __restrict__ diag,
                                                          const double* __restrict__ b, double* x, int32_t r0,
                                                          int32_t r1) {
  const int32_t r = (r0 & ~(kSlice - 1)) + (int32_t)(blockIdx.x * kBlock + threadIdx.x);
  if (r < r0 || r >= r1) return;
  const double acc = row_sum1(A, r, x, r);
  x[r] = (b[r] - acc) / diag[r];
}

// The same update on a Galerkin level, R lanes per row.
template <int R>
__global__ void __launch_bounds__(kBlock) k_gs_color(SellView A, const double* __restrict__ diag,
                                                     const double* __restrict__ b, double* x, int32_t r0,
                                                     int32_t r1, int32_t maxlen) {
  const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / R;
  const int32_t r = r0 + (int32_t)g;
  const bool active = r < r1;
  const double acc = row_sumR<R>(A, r, active, x, r, maxlen);
  if (active && (threadIdx.x & (R - 1)) == 0) x[r] = (b[r] - acc) / diag[r];
}

// r = b - A x on level 0
__global__ void __launch_bounds__(kBlock) k_residual_fine(SellView A, const double* __restrict__ b,
                                                          const double* __restrict__ x, double* __restrict__ res,
                                                          int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  res[r] = b[r] - row_sum1(A, (int32_t)r, x, -1);
}

// r = b - A x on a Galerkin level, R lanes per row
template <int R>
__global__ void __launch_bounds__(kBlock) k_residual(SellView A, const double* __restrict__ b,
                                                     const double* __restrict__ x, double* __restrict__ res,
                                                     int64_t n, int32_t maxlen) {
  const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / R;
  const bool active = g < n;
  const double acc = row_sumR<R>(A, (int32_t)g, active, x, -1, maxlen);
  if (active && (threadIdx.x & (R - 1)) == 0) res[g] = b[g] - acc;
}

// Block-level sum in a fixed tree order.
__device__ inline double block_sum(double v) {
  __shared__ double ws[kBlock / kWave];
  v = wave_sum(v);
  if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / kWave; ++w) t += ws[w];
  __syncthreads();
  return t;
}

// r = b - A x on level 0, plus per-block partial sums of r^2 (fixed grid:
// deterministic).
__global__ void __launch_bounds__(kBlock) k_residual_norm(SellView A, const double* __restrict__ b,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ res, int64_t n,
                                                          double* partials) {
  double sq = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kBlock) {
    const double v = b[r] - row_sum1(A, (int32_t)r, x, -1);
    res[r] = v;
    sq += v * v;
  }
  double t = block_sum(sq);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kBlock) k_norm_partials(const double* v, int64_t n, double* partials) {
  double sq = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    sq += v[i] * v[i];
  double t = block_sum(sq);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kBlock) k_finish_norm(const double* partials, double* out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < kNormBlocks; i += kBlock) s += partials[i];
  double t = block_sum(s);
  if (threadIdx.x == 0) *out = sqrt(t);
}

// b_c[I] = sum over row I of P^T (ascending original fine index) of P[i,I] r_i
template <int R>
__global__ void __launch_bounds__(kBlock) k_restrict(SellView T, const double* __restrict__ r,
                                                     double* __restrict__ bc, int64_t nc, int32_t maxlen) {
  const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / R;
  const bool active = g < nc;
  const double acc = row_sumR<R>(T, (int32_t)g, active, r, -1, maxlen);
  if (active && (threadIdx.x & (R - 1)) == 0) bc[g] = acc;
}

// x_i <- x_i + sum_t P[i, t] x_c[col_t]
__global__ void __launch_bounds__(kBlock) k_prolong_correct(LevelView L, const double* __restrict__ xc,
                                                            double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.n) return;
  prolong_row(L, xc, x, (int32_t)i);
}

// x = A_c^-1 b, one wavefront per row of the dense inverse.
__global__ void __launch_bounds__(kBlock) k_dense_gemv(const double* __restrict__ M,
                                                       const double* __restrict__ b, double* __restrict__ x,
                                                       int64_t n) {
  const int64_t row = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= n) return;
  double s = 0.0;
  for (int64_t k = lane; k < n; k += kWave) s += M[row * n + k] * b[k];
  s = wave_sum(s);
  if (lane == 0) x[row] = s;
}

// The V-cycle below a level with few rows, in one workgroup: every phase
// (colour of a sweep, residual, restriction, coarsest solve, prolongation) is
// separated by a workgroup barrier instead of a kernel boundary, and the
// iterates x of the tail levels live in LDS when they fit.  Each phase
// performs exactly the operations of the corresponding multi-launch kernel.
constexpr int kChunkTail = 16;

__device__ __forceinline__ void tail_gs(const LevelView& L, double* X) {
  const int tid = threadIdx.x;
  for (int c = 0; c < L.ncolors; ++c) {
    for (int32_t r = L.cptr[c] + tid; r < L.cptr[c + 1]; r += kTailThreads) {
      const double acc = row_sum_seq<kChunkTail>(L.A, r, X, r);
      X[r] = (L.b[r] - acc) / L.diag[r];
    }
    __syncthreads();
  }
}

// The V-cycle below a level with few rows, in one workgroup: every phase
// (colour of a sweep, residual, restriction, coarsest solve, prolongation) is
// separated by a workgroup barrier instead of a kernel boundary, and the
// iterates x of the tail levels live in LDS when they fit.  One lane per row
// (a single compute unit has little shuffle throughput to spare); each phase
// performs exactly the operations of the corresponding multi-launch kernel.
__global__ void __launch_bounds__(kTailThreads) k_tail_vcycle(TailDesc d) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  double* X0 = d.lds_off[0] >= 0 ? lds + d.lds_off[0] : d.lv[0].x;
  if (d.lds_off[0] >= 0)
    for (int32_t i = tid; i < d.lv[0].n; i += kTailThreads) X0[i] = d.lv[0].x[i];
  __syncthreads();
  for (int l = 0; l + 1 < d.nlev; ++l) {
    const LevelView& L = d.lv[l];
    double* XL = d.lds_off[l] >= 0 ? lds + d.lds_off[l] : L.x;
    for (int s = 0; s < d.nu_pre; ++s) tail_gs(L, XL);
    for (int32_t r = tid; r < L.n; r += kTailThreads) L.r[r] = L.b[r] - row_sum_seq<kChunkTail>(L.A, r, XL, -1);
    __syncthreads();
    const LevelView& C = d.lv[l + 1];
    double* XC = d.lds_off[l + 1] >= 0 ? lds + d.lds_off[l + 1] : C.x;
    for (int32_t I = tid; I < C.n; I += kTailThreads) {
      C.b[I] = row_sum_seq<kChunkTail>(L.T, I, L.r, -1);
      XC[I] = 0.0;
    }
    __syncthreads();
  }
  {
    const LevelView& C = d.lv[d.nlev - 1];
    double* XC = d.lds_off[d.nlev - 1] >= 0 ? lds + d.lds_off[d.nlev - 1] : C.x;
    const int lane = tid & (kWave - 1), w = tid / kWave;
    for (int64_t row = w; row < C.n; row += kTailThreads / kWave) {
      double s = 0.0;
      for (int64_t k = lane; k < C.n; k += kWave) s += d.cinv[row * C.n + k] * C.b[k];
      s = wave_sum(s);
      if (lane == 0) XC[row] = s;
    }
    __syncthreads();
  }
  for (int l = d.nlev - 2; l >= 0; --l) {
    const LevelView& L = d.lv[l];
    double* XL = d.lds_off[l] >= 0 ? lds + d.lds_off[l] : L.x;
    const double* XC = d.lds_off[l + 1] >= 0 ? lds + d.lds_off[l + 1] : d.lv[l + 1].x;
    for (int32_t i = tid; i < L.n; i += kTailThreads) {
      const int32_t c = L.q_cnt[i];
      double acc = 0.0;
      for (int t = 0; t < c; ++t) acc = acc + L.q_val[(int64_t)t * L.n + i] * XC[L.q_col[(int64_t)t * L.n + i]];
      XL[i] = XL[i] + acc;
    }
    __syncthreads();
    for (int s = 0; s < d.nu_post; ++s) tail_gs(L, XL);
  }
  if (d.lds_off[0] >= 0)
    for (int32_t i = tid; i < d.lv[0].n; i += kTailThreads) d.lv[0].x[i] = X0[i];
}

__global__ void k_gather(const int32_t* perm, const double* src, double* dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

__global__ void k_scatter(const int32_t* perm, const double* src, double* dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[perm[i]] = src[i];
}

__global__ void k_check_finite(const double* v, int64_t n, int32_t* flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(v[i])) atomicOr(flag, F_INVALID);
}

template <template <int> class Launch, typename... Args>
void dispatch_lanes(int R, Args&&... args) {
  switch (R) {
    case 4: Launch<4>::run(args...); break;
    case 8: Launch<8>::run(args...); break;
    case 16: Launch<16>::run(args...); break;
    case 32: Launch<32>::run(args...); break;
    default: Launch<64>::run(args...); break;
  }
}

template <int R>
struct LaunchGS {
  static void run(const Level& lv, int32_t r0, int32_t r1, hipStream_t s) {
    const int64_t threads = (int64_t)(r1 - r0) * R;
    k_gs_color<R><<<blocks_for(threads), kBlock, 0, s>>>(lv.view.A, lv.diag, lv.b, lv.x, r0, r1, lv.view.maxa);
  }
};

template <int R>
struct LaunchResidual {
  static void run(const Level& lv, hipStream_t s) {
    k_residual<R><<<blocks_for(lv.n * R), kBlock, 0, s>>>(lv.view.A, lv.b, lv.x, lv.r, lv.n, lv.view.maxa);
  }
};

template <int R>
struct LaunchRestrict {
  static void run(const Level& lv, Level& nx, hipStream_t s) {
    k_restrict<R><<<blocks_for(nx.n * R), kBlock, 0, s>>>(lv.view.T, lv.r, nx.b, nx.n, lv.view.maxt);
  }
};

}  // namespace

void gs_sweep(const Level& lv, hipStream_t s, bool finest) {
  for (size_t c = 0; c + 1 < lv.color_ptr.size(); ++c) {
    int32_t r0 = lv.color_ptr[c], r1 = lv.color_ptr[c + 1];
    if (r1 <= r0) continue;
    if (finest) {
      KernelTimer::Scope t(KernelTimer::GS_FINEST, lv.color_bytes[c]);
      int32_t span = r1 - (r0 & ~(kSlice - 1));
      hipExtLaunchKernelGGL(k_gs_color_fine, dim3(blocks_for(span)), dim3(kBlock), 0, s, t.start, t.stop, 0,
                            lv.view.A, (const double*)lv.diag, (const double*)lv.b, lv.x, r0, r1);
    } else {
      dispatch_lanes<LaunchGS>(lv.view.ra, lv, r0, r1, s);
    }
  }
}

void residual(const Level& lv, hipStream_t s, bool finest) {
  if (finest)
    k_residual_fine<<<blocks_for(lv.n), kBlock, 0, s>>>(lv.view.A, lv.b, lv.x, lv.r, lv.n);
  else
    dispatch_lanes<LaunchResidual>(lv.view.ra, lv, s);
}

void restrict_to(const Level& lv, Level& nx, hipStream_t s) { dispatch_lanes<LaunchRestrict>(lv.view.rt, lv, nx, s); }

void prolong_correct(Level& lv, const Level& nx, hipStream_t s) {
  k_prolong_correct<<<blocks_for(lv.n), kBlock, 0, s>>>(lv.view, nx.x, lv.x);
}

void coarse_solve(Handle& h, Level& lv, hipStream_t s) {
  k_dense_gemv<<<blocks_for(lv.n, kBlock / kWave), kBlock, 0, s>>>(h.cinv, lv.b, lv.x, lv.n);
}

void tail_vcycle(Handle& h, hipStream_t s) {
  k_tail_vcycle<<<1, kTailThreads, (size_t)h.tail.lds_doubles * 8, s>>>(h.tail);
}

void permute_in(const int32_t* perm, const double* src, double* dst, int64_t n, hipStream_t s) {
  k_gather<<<blocks_for(n), kBlock, 0, s>>>(perm, src, dst, n);
}

void permute_out(const int32_t* perm, const double* src, double* dst, int64_t n, hipStream_t s) {
  k_scatter<<<blocks_for(n), kBlock, 0, s>>>(perm, src, dst, n);
}

void norm2_partials(const double* v, int64_t n, double* partials, hipStream_t s) {
  k_norm_partials<<<kNormBlocks, kBlock, 0, s>>>(v, n, partials);
}

void residual_norm(const Level& lv, double* partials, hipStream_t s) {
  KernelTimer::Scope t(KernelTimer::RESIDUAL_FINEST, lv.residual_bytes);
  hipExtLaunchKernelGGL(k_residual_norm, dim3(kNormBlocks), dim3(kBlock), 0, s, t.start, t.stop, 0, lv.view.A,
                        (const double*)lv.b, (const double*)lv.x, lv.r, (int64_t)lv.n, partials);
}

void finish_norm(const double* partials, double* out, hipStream_t s) {
  k_finish_norm<<<1, kBlock, 0, s>>>(partials, out);
}

void check_finite(const double* v, int64_t n, int32_t* flag, hipStream_t s) {
  k_check_finite<<<blocks_for(n), kBlock, 0, s>>>(v, n, flag);
}

}  // namespace gmg
