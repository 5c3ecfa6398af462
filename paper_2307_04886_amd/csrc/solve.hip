// V-cycle kernels (Alg. 2): multicolour Gauss-Seidel, residual, restriction
// by P^T, prolongation and correction, coarsest-level solve, norms.
//
// Matrices are in the colour-sorted SELL-64 layout: slice s holds rows
// 64s..64s+63, entry t of row r at s_ptr[s] + 64 t + (r mod 64), so one
// wavefront streams one slice with fully coalesced loads.  Every row sum adds
// its terms sequentially in the CSR order of the original row.
#include "gmg_internal.hpp"

namespace gmg {

namespace {

// One colour of a Gauss-Seidel sweep, rows [r0, r1):
//   x_r <- (b_r - sum_{j != r} A_rj x_j) / A_rr.
// Rows of one colour are not coupled, so they update in parallel.
__global__ void __launch_bounds__(kBlock) k_gs_color(const int32_t* __restrict__ sptr,
                                                     const int32_t* __restrict__ scol,
                                                     const double* __restrict__ sval,
                                                     const int32_t* __restrict__ slen,
                                                     const double* __restrict__ diag,
                                                     const double* __restrict__ b, double* x, int32_t r0,
                                                     int32_t r1) {
  const int32_t r = (r0 & ~(kSlice - 1)) + (int32_t)(blockIdx.x * kBlock + threadIdx.x);
  if (r < r0 || r >= r1) return;
  const int32_t base = sptr[r / kSlice] + (r & (kSlice - 1));
  const int32_t len = slen[r];
  double acc = 0.0;
  for (int32_t t = 0; t < len; ++t) {
    const int32_t j = scol[base + t * kSlice];
    if (j != r) acc = acc + sval[base + t * kSlice] * x[j];
  }
  x[r] = (b[r] - acc) / diag[r];
}

// r = b - A x
__global__ void __launch_bounds__(kBlock) k_residual(const int32_t* __restrict__ sptr,
                                                     const int32_t* __restrict__ scol,
                                                     const double* __restrict__ sval,
                                                     const int32_t* __restrict__ slen,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ x, double* __restrict__ res,
                                                     int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int32_t base = sptr[r / kSlice] + (int32_t)(r & (kSlice - 1));
  const int32_t len = slen[r];
  double acc = 0.0;
  for (int32_t t = 0; t < len; ++t) acc = acc + sval[base + t * kSlice] * x[scol[base + t * kSlice]];
  res[r] = b[r] - acc;
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

// r = b - A x, plus per-block partial sums of r^2 (fixed grid: deterministic).
__global__ void __launch_bounds__(kBlock) k_residual_norm(const int32_t* __restrict__ sptr,
                                                          const int32_t* __restrict__ scol,
                                                          const double* __restrict__ sval,
                                                          const int32_t* __restrict__ slen,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ res, int64_t n,
                                                          double* partials) {
  double sq = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kBlock) {
    const int32_t base = sptr[r / kSlice] + (int32_t)(r & (kSlice - 1));
    const int32_t len = slen[r];
    double acc = 0.0;
    for (int32_t t = 0; t < len; ++t) acc = acc + sval[base + t * kSlice] * x[scol[base + t * kSlice]];
    const double v = b[r] - acc;
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
__global__ void __launch_bounds__(kBlock) k_restrict(const int32_t* __restrict__ trp,
                                                     const int32_t* __restrict__ tcol,
                                                     const double* __restrict__ tval,
                                                     const double* __restrict__ r, double* __restrict__ bc,
                                                     int64_t nc) {
  const int64_t I = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (I >= nc) return;
  double acc = 0.0;
  for (int32_t q = trp[I]; q < trp[I + 1]; ++q) acc = acc + tval[q] * r[tcol[q]];
  bc[I] = acc;
}

// x_i <- x_i + sum_t P[i, t] x_c[col_t]
__global__ void __launch_bounds__(kBlock) k_prolong_correct(const int32_t* __restrict__ qcol,
                                                            const double* __restrict__ qval,
                                                            const int32_t* __restrict__ qcnt,
                                                            const double* __restrict__ xc,
                                                            double* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t c = qcnt[i];
  double acc = 0.0;
  for (int t = 0; t < c; ++t) acc = acc + qval[t * n + i] * xc[qcol[t * n + i]];
  x[i] = x[i] + acc;
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

}  // namespace

void gs_sweep(const Level& lv, hipStream_t s) {
  for (size_t c = 0; c + 1 < lv.color_ptr.size(); ++c) {
    int32_t r0 = lv.color_ptr[c], r1 = lv.color_ptr[c + 1];
    if (r1 <= r0) continue;
    int32_t span = r1 - (r0 & ~(kSlice - 1));
    k_gs_color<<<blocks_for(span), kBlock, 0, s>>>(lv.s_ptr, lv.s_col, lv.s_val, lv.s_len, lv.diag, lv.b,
                                                   lv.x, r0, r1);
  }
}

void residual(const Level& lv, hipStream_t s) {
  k_residual<<<blocks_for(lv.n), kBlock, 0, s>>>(lv.s_ptr, lv.s_col, lv.s_val, lv.s_len, lv.b, lv.x, lv.r,
                                                 lv.n);
}

void restrict_to(const Level& lv, Level& nx, hipStream_t s) {
  k_restrict<<<blocks_for(nx.n), kBlock, 0, s>>>(lv.t_rp, lv.t_col, lv.t_val, lv.r, nx.b, nx.n);
}

void prolong_correct(Level& lv, const Level& nx, hipStream_t s) {
  k_prolong_correct<<<blocks_for(lv.n), kBlock, 0, s>>>(lv.q_col, lv.q_val, lv.q_cnt, nx.x, lv.x, lv.n);
}

void coarse_solve(Handle& h, Level& lv, hipStream_t s) {
  k_dense_gemv<<<blocks_for(lv.n, kBlock / kWave), kBlock, 0, s>>>(h.cinv, lv.b, lv.x, lv.n);
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
  k_residual_norm<<<kNormBlocks, kBlock, 0, s>>>(lv.s_ptr, lv.s_col, lv.s_val, lv.s_len, lv.b, lv.x, lv.r,
                                                 lv.n, partials);
}

void finish_norm(const double* partials, double* out, hipStream_t s) {
  k_finish_norm<<<1, kBlock, 0, s>>>(partials, out);
}

void check_finite(const double* v, int64_t n, int32_t* flag, hipStream_t s) {
  k_check_finite<<<blocks_for(n), kBlock, 0, s>>>(v, n, flag);
}

}  // namespace gmg
