// V-cycle kernels (Alg. 2): multicolour Gauss-Seidel, residual, restriction
// by P^T, prolongation and correction, coarsest-level solve, norms.
//
// Every kernel is written once for the value type V of the level data: double
// for the solve of Alg. 1, float for the mixed-precision CG preconditioner.
// The coarsest level is always solved in double with the dense inverse.
#include <type_traits>

#include "rows.hpp"

namespace gmg {

namespace {

constexpr int kChunkFine = 8;

template <class V>
__device__ __forceinline__ void prolong_row(const LevelViewT<V>& L, const V* __restrict__ xc, V* x, int32_t i) {
  const int32_t c = L.q_cnt[i];
  V acc = V(0);
  V v[3], u[3];
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
template <class V>
__global__ void __launch_bounds__(kBlock) k_gs_color_fine(Sell<V> A, const V* __restrict__ diag,
                                                          const V* __restrict__ b, V* x, int32_t r0, int32_t r1) {
  const int32_t r = (r0 & ~(kSlice - 1)) + (int32_t)(blockIdx.x * kBlock + threadIdx.x);
  if (r < r0 || r >= r1) return;
  const V br = b[r], dr = diag[r];        // issued with the row's loads
  const V acc = row_sum_seq<kChunkFine>(A, r, x, r);
  x[r] = (br - acc) / dr;
}

// The same update on a Galerkin level, R lanes per row.
template <int R, class V>
__global__ void __launch_bounds__(kBlock) k_gs_color(Sell<V> A, const V* __restrict__ diag,
                                                     const V* __restrict__ b, V* x, int32_t r0, int32_t r1,
                                                     int32_t maxlen) {
  const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / R;
  const int32_t r = r0 + (int32_t)g;
  const bool active = r < r1;
  const int32_t rc = active ? r : r0;     // in range for every lane: the loads need no branch
  const V br = b[rc], dr = diag[rc];
  const V acc = row_sumR<R>(A, r, active, x, r, maxlen);
  if (active && (threadIdx.x & (R - 1)) == 0) x[r] = (br - acc) / dr;
}

// r = b - A x on level 0
template <class V>
__global__ void __launch_bounds__(kBlock) k_residual_fine(Sell<V> A, const V* __restrict__ b,
                                                          const V* __restrict__ x, V* __restrict__ res,
                                                          int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  res[r] = b[r] - row_sum_seq<kChunkFine>(A, (int32_t)r, x, -1);
}

// r = b - A x on a Galerkin level, R lanes per row
template <int R, class V>
__global__ void __launch_bounds__(kBlock) k_residual(Sell<V> A, const V* __restrict__ b, const V* __restrict__ x,
                                                     V* __restrict__ res, int64_t n, int32_t maxlen) {
  const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / R;
  const bool active = g < n;
  const V acc = row_sumR<R>(A, (int32_t)g, active, x, -1, maxlen);
  if (active && (threadIdx.x & (R - 1)) == 0) res[g] = b[g] - acc;
}

// r = b - A x on level 0 (double), plus per-block partial sums of r^2 (fixed
// grid: deterministic).
__global__ void __launch_bounds__(kBlock) k_residual_norm(SellView A, const double* __restrict__ b,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ res, int64_t n,
                                                          double* partials) {
  double sq = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kBlock) {
    const double v = b[r] - row_sum_seq<kChunkFine>(A, (int32_t)r, x, -1);
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

// b_c[I] = sum over row I of P^T (ascending original fine index) of P[i,I] r_i,
// and the coarse iterate starts from zero: x_c[I] = 0
template <int R, class V>
__global__ void __launch_bounds__(kBlock) k_restrict(Sell<V> T, const V* __restrict__ r, V* __restrict__ bc,
                                                     V* __restrict__ xc, int64_t nc, int32_t maxlen) {
  const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / R;
  const bool active = g < nc;
  const V acc = row_sumR<R>(T, (int32_t)g, active, r, -1, maxlen);
  if (active && (threadIdx.x & (R - 1)) == 0) {
    bc[g] = acc;
    xc[g] = V(0);
  }
}

// x_i <- x_i + sum_t P[i, t] x_c[col_t]
template <class V>
__global__ void __launch_bounds__(kBlock) k_prolong_correct(LevelViewT<V> L, const V* __restrict__ xc,
                                                            V* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.n) return;
  prolong_row(L, xc, x, (int32_t)i);
}

// x = A_c^-1 b in double (b widened from V, x rounded to V), one wavefront per
// row of the dense inverse.
template <class V>
__global__ void __launch_bounds__(kBlock) k_dense_gemv(const double* __restrict__ M, const V* __restrict__ b,
                                                       V* __restrict__ x, int64_t n) {
  const int64_t row = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= n) return;
  double s = 0.0;
  for (int64_t k = lane; k < n; k += kWave) s += M[row * n + k] * (double)b[k];
  s = wave_sum(s);
  if (lane == 0) x[row] = (V)s;
}

// The V-cycle below a level with few rows, in one workgroup: every phase
// (colour of a sweep, residual, restriction, coarsest solve, prolongation) is
// separated by a workgroup barrier instead of a kernel boundary, and the
// iterates x of the tail levels live in LDS when they fit.  One lane per row
// (a single compute unit has little shuffle throughput to spare); each phase
// performs exactly the operations of the corresponding multi-launch kernel.
constexpr int kChunkTail = 16;

template <class V>
__device__ __forceinline__ void tail_gs(const LevelViewT<V>& L, V* X, bool descending) {
  const int tid = threadIdx.x;
  for (int k = 0; k < L.ncolors; ++k) {
    const int c = descending ? L.ncolors - 1 - k : k;
    for (int32_t r = L.cptr[c] + tid; r < L.cptr[c + 1]; r += kTailThreads) {
      const V acc = row_sum_seq<kChunkTail>(L.A, r, X, r);
      X[r] = (L.b[r] - acc) / L.diag[r];
    }
    __syncthreads();
  }
}

template <class V>
__global__ void __launch_bounds__(kTailThreads) k_tail_vcycle(TailDescT<V> d) {
  extern __shared__ double lds_raw[];
  V* lds = reinterpret_cast<V*>(lds_raw);
  const int tid = threadIdx.x;
  V* X0 = d.lds_off[0] >= 0 ? lds + d.lds_off[0] : d.lv[0].x;
  if (d.lds_off[0] >= 0)
    for (int32_t i = tid; i < d.lv[0].n; i += kTailThreads) X0[i] = d.lv[0].x[i];
  __syncthreads();
  for (int l = 0; l + 1 < d.nlev; ++l) {
    const LevelViewT<V>& L = d.lv[l];
    V* XL = d.lds_off[l] >= 0 ? lds + d.lds_off[l] : L.x;
    for (int s = 0; s < d.nu_pre; ++s) tail_gs(L, XL, false);
    for (int32_t r = tid; r < L.n; r += kTailThreads) L.r[r] = L.b[r] - row_sum_seq<kChunkTail>(L.A, r, XL, -1);
    __syncthreads();
    const LevelViewT<V>& C = d.lv[l + 1];
    V* XC = d.lds_off[l + 1] >= 0 ? lds + d.lds_off[l + 1] : C.x;
    for (int32_t I = tid; I < C.n; I += kTailThreads) {
      C.b[I] = row_sum_seq<kChunkTail>(L.T, I, (const V*)L.r, -1);
      XC[I] = V(0);
    }
    __syncthreads();
  }
  {
    const LevelViewT<V>& C = d.lv[d.nlev - 1];
    V* XC = d.lds_off[d.nlev - 1] >= 0 ? lds + d.lds_off[d.nlev - 1] : C.x;
    const int lane = tid & (kWave - 1), w = tid / kWave;
    for (int64_t row = w; row < C.n; row += kTailThreads / kWave) {
      double s = 0.0;
      for (int64_t k = lane; k < C.n; k += kWave) s += d.cinv[row * C.n + k] * (double)C.b[k];
      s = wave_sum(s);
      if (lane == 0) XC[row] = (V)s;
    }
    __syncthreads();
  }
  for (int l = d.nlev - 2; l >= 0; --l) {
    const LevelViewT<V>& L = d.lv[l];
    V* XL = d.lds_off[l] >= 0 ? lds + d.lds_off[l] : L.x;
    const V* XC = d.lds_off[l + 1] >= 0 ? lds + d.lds_off[l + 1] : d.lv[l + 1].x;
    for (int32_t i = tid; i < L.n; i += kTailThreads) {
      const int32_t c = L.q_cnt[i];
      V acc = V(0);
      for (int t = 0; t < c; ++t) acc = acc + L.q_val[(int64_t)t * L.n + i] * XC[L.q_col[(int64_t)t * L.n + i]];
      XL[i] = XL[i] + acc;
    }
    __syncthreads();
    for (int s = 0; s < d.nu_post; ++s) tail_gs(L, XL, d.descending_post != 0);
  }
  if (d.lds_off[0] >= 0)
    for (int32_t i = tid; i < d.lv[0].n; i += kTailThreads) d.lv[0].x[i] = X0[i];
}

__global__ void k_gather(const int32_t* perm, const double* src, double* dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

template <class V>
__global__ void k_scatter(const int32_t* perm, const V* src, double* dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[perm[i]] = (double)src[i];
}

__global__ void k_to_f32(const double* src, float* dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

template <class V>
__global__ void k_zero(V* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = V(0);
}

__global__ void k_check_finite(const double* v, int64_t n, int32_t* flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(v[i])) atomicOr(flag, F_INVALID);
}

}  // namespace

template <class V>
void gs_sweep(const LevelViewT<V>& v, const Level& lv, hipStream_t s, bool finest, bool descending, bool timed) {
  const int C = (int)lv.color_ptr.size() - 1;
  for (int k = 0; k < C; ++k) {
    const int c = descending ? C - 1 - k : k;
    const int32_t r0 = lv.color_ptr[c], r1 = lv.color_ptr[c + 1];
    if (r1 <= r0) continue;
    if (finest) {
      KernelTimer::Scope t(timed ? (int)KernelTimer::GS_FINEST : -1, lv.color_bytes[c]);
      const int32_t span = r1 - (r0 & ~(kSlice - 1));
      hipExtLaunchKernelGGL(k_gs_color_fine<V>, dim3(blocks_for(span)), dim3(kBlock), 0, s, t.start, t.stop, 0,
                            v.A, (const V*)v.diag, (const V*)v.b, v.x, r0, r1);
    } else {
      KernelTimer::Scope t(timed ? (int)KernelTimer::GS_GALERKIN : -1, lv.color_bytes[c]);
      with_lanes(v.ra, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        const auto kern = k_gs_color<R, V>;
        hipExtLaunchKernelGGL(kern, dim3(blocks_for((int64_t)(r1 - r0) * R)), dim3(kBlock), 0, s, t.start, t.stop,
                              0, v.A, (const V*)v.diag, (const V*)v.b, v.x, r0, r1, v.maxa);
      });
    }
  }
}

template <class V>
void residual(const LevelViewT<V>& v, hipStream_t s, bool finest) {
  if (finest) {
    k_residual_fine<V><<<blocks_for(v.n), kBlock, 0, s>>>(v.A, v.b, v.x, v.r, v.n);
  } else {
    with_lanes(v.ra, [&](auto RC) {
      constexpr int R = decltype(RC)::value;
      k_residual<R, V><<<blocks_for((int64_t)v.n * R), kBlock, 0, s>>>(v.A, v.b, v.x, v.r, v.n, v.maxa);
    });
  }
}

template <class V>
void restrict_to(const LevelViewT<V>& v, const LevelViewT<V>& c, hipStream_t s) {
  with_lanes(v.rt, [&](auto RC) {
    constexpr int R = decltype(RC)::value;
    k_restrict<R, V><<<blocks_for((int64_t)c.n * R), kBlock, 0, s>>>(v.T, v.r, c.b, c.x, c.n, v.maxt);
  });
}

template <class V>
void prolong_correct(const LevelViewT<V>& v, const LevelViewT<V>& c, hipStream_t s) {
  k_prolong_correct<V><<<blocks_for(v.n), kBlock, 0, s>>>(v, c.x, v.x);
}

template <class V>
void coarse_solve(const double* cinv, const LevelViewT<V>& c, hipStream_t s) {
  k_dense_gemv<V><<<blocks_for(c.n, kBlock / kWave), kBlock, 0, s>>>(cinv, c.b, c.x, c.n);
}

template <class V>
void tail_vcycle(const TailDescT<V>& d, hipStream_t s) {
  k_tail_vcycle<V><<<1, kTailThreads, (size_t)d.lds_elems * sizeof(V), s>>>(d);
}

template <class V>
void fill_zero(V* p, int64_t n, hipStream_t s) {
  k_zero<V><<<blocks_for(n), kBlock, 0, s>>>(p, n);
}

void to_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  k_to_f32<<<blocks_for(n), kBlock, 0, s>>>(src, dst, n);
}

void permute_in(const int32_t* perm, const double* src, double* dst, int64_t n, hipStream_t s) {
  k_gather<<<blocks_for(n), kBlock, 0, s>>>(perm, src, dst, n);
}

template <class V>
void permute_out(const int32_t* perm, const V* src, double* dst, int64_t n, hipStream_t s) {
  k_scatter<V><<<blocks_for(n), kBlock, 0, s>>>(perm, src, dst, n);
}

void norm2_partials(const double* v, int64_t n, double* partials, hipStream_t s) {
  k_norm_partials<<<kNormBlocks, kBlock, 0, s>>>(v, n, partials);
}

void residual_norm(const Level& lv, const double* b, const double* x, double* res, double* partials,
                   hipStream_t s) {
  KernelTimer::Scope t(KernelTimer::RESIDUAL_FINEST, lv.residual_bytes);
  hipExtLaunchKernelGGL(k_residual_norm, dim3(kNormBlocks), dim3(kBlock), 0, s, t.start, t.stop, 0, lv.view.A, b,
                        x, res, (int64_t)lv.n, partials);
}

void finish_norm(const double* partials, double* out, hipStream_t s) {
  k_finish_norm<<<1, kBlock, 0, s>>>(partials, out);
}

void check_finite(const double* v, int64_t n, int32_t* flag, hipStream_t s) {
  k_check_finite<<<blocks_for(n), kBlock, 0, s>>>(v, n, flag);
}

#define GMG_INSTANTIATE(V)                                                                              \
  template void gs_sweep<V>(const LevelViewT<V>&, const Level&, hipStream_t, bool, bool, bool);       \
  template void residual<V>(const LevelViewT<V>&, hipStream_t, bool);                                  \
  template void restrict_to<V>(const LevelViewT<V>&, const LevelViewT<V>&, hipStream_t);               \
  template void prolong_correct<V>(const LevelViewT<V>&, const LevelViewT<V>&, hipStream_t);           \
  template void coarse_solve<V>(const double*, const LevelViewT<V>&, hipStream_t);                     \
  template void tail_vcycle<V>(const TailDescT<V>&, hipStream_t);                                      \
  template void fill_zero<V>(V*, int64_t, hipStream_t);                                                \
  template void permute_out<V>(const int32_t*, const V*, double*, int64_t, hipStream_t);
GMG_INSTANTIATE(double)
GMG_INSTANTIATE(float)
#undef GMG_INSTANTIATE

}  // namespace gmg
