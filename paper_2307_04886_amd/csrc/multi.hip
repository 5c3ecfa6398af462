// Batched right-hand sides: the V-cycle and the preconditioned CG of
// krylov.hip for kBatch right-hand sides at once on one hierarchy (the
// workload of many solves per hierarchy that a geometric hierarchy is built
// for, Sec. 2 and Sec. 5.5).  Vectors are interleaved, entry (i, q) at
// i * kBatch + q, so that the kBatch values a row update gathers from a
// neighbour are contiguous.  One lane per (row, right-hand side): the kBatch
// lanes of a row read the same matrix entries (one cache line serves them
// all) and each sums its own products in the row's entry order, so every
// right-hand side gets exactly the arithmetic of the single-vector kernels.
#include "rows.hpp"

namespace gmg {

namespace {

constexpr int K = kBatch;
constexpr int kChunkMulti = 8;

// sum_t val[t] * x[col[t] * K + q] in entry order, skipping column `skip`
// (branch-free loads as in row_sum_seq; every row has at least one entry).
template <class V>
__device__ __forceinline__ V row_sum_multi(const Sell<V>& A, int32_t r, const V* x, int32_t skip, int q) {
  const int32_t len = A.len[r];
  const int32_t base = A.ptr[r / kSlice] + (r & (kSlice - 1));
  V acc = V(0);
  int32_t t0 = 0;
  do {
    int32_t j[kChunkMulti];
    V v[kChunkMulti], xv[kChunkMulti];
#pragma unroll
    for (int u = 0; u < kChunkMulti; ++u) {
      const int32_t o = base + min(t0 + u, len - 1) * kSlice;
      j[u] = A.col[o];
      v[u] = A.val[o];
    }
#pragma unroll
    for (int u = 0; u < kChunkMulti; ++u) xv[u] = x[(int64_t)j[u] * K + q];
#pragma unroll
    for (int u = 0; u < kChunkMulti; ++u)
      if (t0 + u < len && j[u] != skip) acc = acc + v[u] * xv[u];
    t0 += kChunkMulti;
  } while (t0 < len);
  return acc;
}

// Element t of a colour class [r0, r1): row r0 + t / K, right-hand side t % K.
template <class V>
__device__ __forceinline__ void mgs_entry(const Sell<V>& A, const V* diag, const V* b, V* x, int32_t r0, int32_t r1,
                                          int64_t t) {
  const int32_t r = r0 + (int32_t)(t / K);
  const int q = (int)(t % K);
  if (r >= r1) return;
  const V br = b[(int64_t)r * K + q], dr = diag[r];
  const V acc = row_sum_multi(A, r, x, r, q);
  x[(int64_t)r * K + q] = (br - acc) / dr;
}

template <class V>
__device__ __forceinline__ void mresidual_entry(const Sell<V>& A, const V* b, const V* x, V* res, int64_t n,
                                                int64_t t) {
  if (t >= n * K) return;
  const int32_t r = (int32_t)(t / K);
  const int q = (int)(t % K);
  res[t] = b[t] - row_sum_multi(A, r, x, -1, q);
}

template <class V>
__device__ __forceinline__ void mrestrict_entry(const Sell<V>& T, const V* r, V* bc, V* xc, int64_t nc, int64_t t) {
  if (t >= nc * K) return;
  bc[t] = row_sum_multi(T, (int32_t)(t / K), r, -1, (int)(t % K));
  xc[t] = V(0);                                   // the coarse iterate starts from zero
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_mgs(Sell<V> A, const V* __restrict__ diag, const V* __restrict__ b,
                                                V* x, int32_t r0, int32_t r1) {
  mgs_entry(A, diag, b, x, r0, r1, (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_mresidual(Sell<V> A, const V* __restrict__ b, const V* __restrict__ x,
                                                      V* __restrict__ res, int64_t n) {
  mresidual_entry(A, b, x, res, n, (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_mrestrict(Sell<V> T, const V* __restrict__ r, V* __restrict__ bc,
                                                      V* __restrict__ xc, int64_t nc) {
  mrestrict_entry(T, r, bc, xc, nc, (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

template <class V>
__device__ __forceinline__ void mprolong_entry(const int32_t* q_col, const V* q_val, const int32_t* q_cnt, int32_t n,
                                               const V* xc, V* x, int64_t t) {
  const int32_t i = (int32_t)(t / K);
  const int q = (int)(t % K);
  const int32_t c = q_cnt[i];
  V acc = V(0);
  V v[3], u[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    v[s] = q_val[(int64_t)s * n + i];
    u[s] = xc[(int64_t)q_col[(int64_t)s * n + i] * K + q];
  }
#pragma unroll
  for (int s = 0; s < 3; ++s)
    if (s < c) acc = acc + v[s] * u[s];
  x[t] = x[t] + acc;
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_mprolong(LevelViewT<V> L, const V* __restrict__ xc, V* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (int64_t)L.n * K) return;
  mprolong_entry(L.q_col, L.q_val, L.q_cnt, L.n, xc, x, t);
}

// x = A_c^-1 b for the K right-hand sides, in double, as the single-vector
// coarse solve: entry (i, q) is the sum over k ascending of (A_c^-1 e_k)_i b_kq.
template <class V>
__device__ __forceinline__ void mgemv_entry(const double* M, const V* b, V* x, int64_t n, int64_t t) {
  const int64_t i = t / K;
  const int q = (int)(t % K);
  double acc = 0.0;
  const int64_t ld = inv_ld(n);
  // the loads of eight terms are issued before they are added (in ascending k)
  int64_t k = 0;
  for (; k + 8 <= n; k += 8) {
    double m[8], v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      m[u] = M[(k + u) * ld + i];
      v[u] = (double)b[(k + u) * K + q];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = acc + m[u] * v[u];
  }
  for (; k < n; ++k) acc = acc + M[k * ld + i] * (double)b[k * K + q];
  x[t] = (V)acc;
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_mgemv(const double* __restrict__ M, const V* __restrict__ b,
                                                  V* __restrict__ x, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n * K) return;
  mgemv_entry(M, b, x, n, t);
}

// The tail of the cycle in one workgroup (as k_tail_vcycle), one lane per
// (row, right-hand side); iterates in LDS where they fit.
template <class V>
__device__ __forceinline__ void mtail_gs(const LevelViewT<V>& L, V* X, bool descending) {
  for (int k = 0; k < L.ncolors; ++k) {
    const int c = descending ? L.ncolors - 1 - k : k;
    const int32_t r0 = L.cptr[c], r1 = L.cptr[c + 1];
    for (int64_t t = threadIdx.x; t < (int64_t)(r1 - r0) * K; t += kTailThreads) {
      const int32_t r = r0 + (int32_t)(t / K);
      const int q = (int)(t % K);
      const V acc = row_sum_multi(L.A, r, (const V*)X, r, q);
      X[(int64_t)r * K + q] = (L.b[(int64_t)r * K + q] - acc) / L.diag[r];
    }
    __syncthreads();
  }
}

template <class V>
__device__ __forceinline__ void mtail_run(const TailDescT<V>& d) {
  extern __shared__ double lds_raw[];
  V* lds = reinterpret_cast<V*>(lds_raw);
  const int tid = threadIdx.x;
  auto X = [&](int l) -> V* { return d.lds_off[l] >= 0 ? lds + d.lds_off[l] : d.lv[l].x; };
  if (d.lds_off[0] >= 0)
    for (int64_t i = tid; i < (int64_t)d.lv[0].n * K; i += kTailThreads) X(0)[i] = d.lv[0].x[i];
  __syncthreads();
  for (int l = 0; l + 1 < d.nlev; ++l) {
    const LevelViewT<V>& L = d.lv[l];
    V* XL = X(l);
    for (int s = 0; s < d.nu_pre; ++s) mtail_gs(L, XL, false);
    for (int64_t t = tid; t < (int64_t)L.n * K; t += kTailThreads)
      L.r[t] = L.b[t] - row_sum_multi(L.A, (int32_t)(t / K), (const V*)XL, -1, (int)(t % K));
    __syncthreads();
    const LevelViewT<V>& C = d.lv[l + 1];
    V* XC = X(l + 1);
    for (int64_t t = tid; t < (int64_t)C.n * K; t += kTailThreads) {
      C.b[t] = row_sum_multi(L.T, (int32_t)(t / K), (const V*)L.r, -1, (int)(t % K));
      XC[t] = V(0);
    }
    __syncthreads();
  }
  {
    const LevelViewT<V>& C = d.lv[d.nlev - 1];
    V* XC = X(d.nlev - 1);
    for (int64_t t = tid; t < (int64_t)C.n * K; t += kTailThreads) mgemv_entry(d.cinv, (const V*)C.b, XC, C.n, t);
    __syncthreads();
  }
  for (int l = d.nlev - 2; l >= 0; --l) {
    const LevelViewT<V>& L = d.lv[l];
    V* XL = X(l);
    const V* XC = X(l + 1);
    for (int64_t t = tid; t < (int64_t)L.n * K; t += kTailThreads)
      mprolong_entry(L.q_col, L.q_val, L.q_cnt, L.n, XC, XL, t);
    __syncthreads();
    for (int s = 0; s < d.nu_post; ++s) mtail_gs(L, XL, d.descending_post != 0);
  }
  if (d.lds_off[0] >= 0)
    for (int64_t i = tid; i < (int64_t)d.lv[0].n * K; i += kTailThreads) d.lv[0].x[i] = X(0)[i];
}

template <class V>
__global__ void __launch_bounds__(kTailThreads) k_mtail(TailDescT<V> d) {
  mtail_run(d);
}

// ------------------------------------------------------------ CG, K right-hand sides
// Per-block partial sums by right-hand side: with a grid stride that is a
// multiple of K, thread t always handles right-hand side t mod K; lanes of a
// wavefront with the same q are combined with shuffles, then the wavefronts
// of the block in a fixed order.
__device__ inline void block_sums_by_rhs(double v, double* out /* [K] */) {
  __shared__ double ws[kBlock / kWave][K];
  for (int o = kWave / 2; o >= K; o >>= 1) v += __shfl_xor(v, o, kWave);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane < K) ws[w][lane] = v;
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int i = 0; i < kBlock / kWave; ++i) s += ws[i][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// sum over blocks of part[b * K + q], for every q, in one block
__device__ inline void finish_by_rhs(const double* part, double* out /* [K] shared */) {
  __shared__ double acc[kBlock];
  double s = 0.0;
  const int q = threadIdx.x % K;
  for (int b = threadIdx.x / K; b < kNormBlocks; b += kBlock / K) s += part[(int64_t)b * K + q];
  acc[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0.0;
    for (int i = threadIdx.x; i < kBlock; i += K) t += acc[i];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

// The CG steps as bodies over a logical block lb of nb (the grid-stride
// kernels run nb = kNormBlocks blocks per hierarchy, so that the partial sums,
// and with them every reduction, are the same whether a launch serves one
// hierarchy or a group of them).
__device__ __forceinline__ void mkry_init_entry(double* p, double* r_old, int64_t nk, double* scal, int64_t i) {
  if (i < nk) {
    p[i] = 0.0;
    r_old[i] = 0.0;
  }
  if (i < K) {
    scal[KS_RHO * K + i] = 1.0;
    scal[KS_BETA * K + i] = 0.0;
    scal[KS_ALPHA * K + i] = 0.0;
  }
}

template <class V>
__device__ __forceinline__ void mkry_dots_block(const double* r, const double* r_old, const V* z, int64_t nk,
                                                double* part, int64_t lb, int64_t nb) {
  __shared__ double o1[K], o2[K];
  double a = 0.0, c = 0.0;
  for (int64_t i = lb * kBlock + threadIdx.x; i < nk; i += nb * kBlock) {
    const double zi = (double)z[i];
    a += r[i] * zi;
    c += r_old[i] * zi;
  }
  block_sums_by_rhs(a, o1);
  block_sums_by_rhs(c, o2);
  if (threadIdx.x < K) {
    part[lb * K + threadIdx.x] = o1[threadIdx.x];
    part[(kNormBlocks + lb) * K + threadIdx.x] = o2[threadIdx.x];
  }
}

__device__ __forceinline__ void mkry_beta_block(const double* part, double* scal) {
  __shared__ double rho_new[K], rz[K];
  finish_by_rhs(part, rho_new);
  finish_by_rhs(part + (int64_t)kNormBlocks * K, rz);
  if (threadIdx.x < K) {
    const double rho = scal[KS_RHO * K + threadIdx.x];
    scal[KS_BETA * K + threadIdx.x] = rho != 0.0 ? (rho_new[threadIdx.x] - rz[threadIdx.x]) / rho : 0.0;
    scal[KS_RHO * K + threadIdx.x] = rho_new[threadIdx.x];
  }
}

template <class V>
__device__ __forceinline__ void mkry_p_entry(const V* z, const double* scal, double* p, int64_t nk, int64_t i) {
  if (i >= nk) return;
  p[i] = (double)z[i] + scal[KS_BETA * K + i % K] * p[i];
}

__device__ __forceinline__ void mkry_spmv_block(const SellView& A, const double* p, double* qv, int64_t n,
                                                double* part, int64_t lb, int64_t nb) {
  __shared__ double o[K];
  double s = 0.0;
  for (int64_t t = lb * kBlock + threadIdx.x; t < n * K; t += nb * kBlock) {
    const double v = row_sum_multi(A, (int32_t)(t / K), p, -1, (int)(t % K));
    qv[t] = v;
    s += p[t] * v;
  }
  block_sums_by_rhs(s, o);
  if (threadIdx.x < K) part[(2 * kNormBlocks + lb) * K + threadIdx.x] = o[threadIdx.x];
}

// alpha = rho / p.q per right-hand side; rho = 0 (an exactly solved one) gives alpha = 0
__device__ __forceinline__ void mkry_alpha_block(const double* part, double* scal, int32_t* flags) {
  __shared__ double pq[K];
  finish_by_rhs(part + (int64_t)2 * kNormBlocks * K, pq);
  if (threadIdx.x < K) {
    const double rho = scal[KS_RHO * K + threadIdx.x];
    double a = 0.0;
    if (rho != 0.0) {
      if (!(pq[threadIdx.x] > 0.0) || !(rho > 0.0)) atomicOr(flags, F_NOT_SPD);
      else a = rho / pq[threadIdx.x];
    }
    scal[KS_ALPHA * K + threadIdx.x] = a;
  }
}

__device__ __forceinline__ void mkry_update_block(double* x, const double* p, const double* qv, double* r,
                                                  double* r_old, const double* scal, int64_t nk, double* part,
                                                  int64_t lb, int64_t nb) {
  __shared__ double o[K];
  double s = 0.0;
  for (int64_t i = lb * kBlock + threadIdx.x; i < nk; i += nb * kBlock) {
    const double alpha = scal[KS_ALPHA * K + i % K];
    x[i] = x[i] + alpha * p[i];
    const double ri = r[i];
    r_old[i] = ri;
    const double rn = ri - alpha * qv[i];
    r[i] = rn;
    s += rn * rn;
  }
  block_sums_by_rhs(s, o);
  if (threadIdx.x < K) part[lb * K + threadIdx.x] = o[threadIdx.x];
}

__device__ __forceinline__ void mkry_norm_block(const double* part, double* out /* [K] */) {
  __shared__ double s[K];
  finish_by_rhs(part, s);
  if (threadIdx.x < K) out[threadIdx.x] = sqrt(s[threadIdx.x]);
}

// r = b - A x (level 0, double) and partials of |r_q|^2
__device__ __forceinline__ void mresidual_norm_block(const SellView& A, const double* b, const double* x, double* res,
                                                     int64_t n, double* part, int64_t lb, int64_t nb) {
  __shared__ double o[K];
  double s = 0.0;
  for (int64_t t = lb * kBlock + threadIdx.x; t < n * K; t += nb * kBlock) {
    const double v = b[t] - row_sum_multi(A, (int32_t)(t / K), x, -1, (int)(t % K));
    res[t] = v;
    s += v * v;
  }
  block_sums_by_rhs(s, o);
  if (threadIdx.x < K) part[lb * K + threadIdx.x] = o[threadIdx.x];
}

__device__ __forceinline__ void mnorm_partials_block(const double* v, int64_t nk, double* part, int64_t lb,
                                                     int64_t nb) {
  __shared__ double o[K];
  double s = 0.0;
  for (int64_t i = lb * kBlock + threadIdx.x; i < nk; i += nb * kBlock) s += v[i] * v[i];
  block_sums_by_rhs(s, o);
  if (threadIdx.x < K) part[lb * K + threadIdx.x] = o[threadIdx.x];
}

__global__ void k_mkry_init(double* p, double* r_old, int64_t nk, double* scal) {
  mkry_init_entry(p, r_old, nk, scal, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_mkry_dots(const double* __restrict__ r, const double* __restrict__ r_old,
                                                      const V* __restrict__ z, int64_t nk, double* part) {
  mkry_dots_block(r, r_old, z, nk, part, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_mkry_beta(const double* part, double* scal) { mkry_beta_block(part, scal); }

template <class V>
__global__ void k_mkry_p(const V* __restrict__ z, const double* __restrict__ scal, double* __restrict__ p,
                         int64_t nk) {
  mkry_p_entry(z, scal, p, nk, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(kBlock) k_mkry_spmv(SellView A, const double* __restrict__ p, double* __restrict__ qv,
                                                      int64_t n, double* part) {
  mkry_spmv_block(A, p, qv, n, part, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_mkry_alpha(const double* part, double* scal, int32_t* flags) {
  mkry_alpha_block(part, scal, flags);
}

__global__ void __launch_bounds__(kBlock) k_mkry_update(double* __restrict__ x, const double* __restrict__ p,
                                                        const double* __restrict__ qv, double* __restrict__ r,
                                                        double* __restrict__ r_old, const double* __restrict__ scal,
                                                        int64_t nk, double* part) {
  mkry_update_block(x, p, qv, r, r_old, scal, nk, part, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_mkry_norm(const double* part, double* out /* [K] */) {
  mkry_norm_block(part, out);
}

__global__ void __launch_bounds__(kBlock) k_mresidual_norm(SellView A, const double* __restrict__ b,
                                                           const double* __restrict__ x, double* __restrict__ res,
                                                           int64_t n, double* part) {
  mresidual_norm_block(A, b, x, res, n, part, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_mnorm_partials(const double* v, int64_t nk, double* part) {
  mnorm_partials_block(v, nk, part, blockIdx.x, gridDim.x);
}

// dst[i * K + q] = src[q * n + perm[i]] for q < nq, 0 for the padding columns
__global__ void k_mgather(const int32_t* perm, const double* src, int64_t n, int nq, double* dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * K) return;
  const int64_t i = t / K;
  const int q = (int)(t % K);
  dst[t] = q < nq ? src[(int64_t)q * n + perm[i]] : 0.0;
}

__global__ void k_mscatter(const int32_t* perm, const double* src, int64_t n, int nq, double* dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * K) return;
  const int64_t i = t / K;
  const int q = (int)(t % K);
  if (q < nq) dst[(int64_t)q * n + perm[i]] = src[t];
}

template <class V>
__global__ void k_mscatter_v(const int32_t* perm, const V* src, int64_t n, int nq, double* dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * K) return;
  const int64_t i = t / K;
  const int q = (int)(t % K);
  if (q < nq) dst[(int64_t)q * n + perm[i]] = (double)src[t];
}

__global__ void k_mzero_columns(double* x, int64_t n, unsigned mask) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * K && ((mask >> (t % K)) & 1u)) x[t] = 0.0;
}

// ------------------------------------------------------------ grouped launches
// A workgroup of a row-parallel grouped step takes its job, tile and member
// from the tile map; element t of its job is tile * kBlock + threadIdx.x, as
// blockIdx.x * kBlock + threadIdx.x in the single-hierarchy kernel.
template <class V>
__global__ void __launch_bounds__(kBlock) k_gsweep(const GSweepJob<V>* __restrict__ jobs,
                                                   const GTile* __restrict__ tiles, const int32_t* __restrict__ active) {
  const GTile g = tiles[blockIdx.x];
  if (!active[g.member]) return;
  const GSweepJob<V> J = jobs[g.job];
  mgs_entry(J.A, J.diag, J.b, J.x, J.r0, J.r1, (int64_t)g.tile * kBlock + threadIdx.x);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_gresidual(const GResJob<V>* __restrict__ jobs,
                                                      const GTile* __restrict__ tiles,
                                                      const int32_t* __restrict__ active) {
  const GTile g = tiles[blockIdx.x];
  if (!active[g.member]) return;
  const GResJob<V> J = jobs[g.job];
  mresidual_entry(J.A, J.b, J.x, J.r, J.n, (int64_t)g.tile * kBlock + threadIdx.x);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_grestrict(const GRestJob<V>* __restrict__ jobs,
                                                      const GTile* __restrict__ tiles,
                                                      const int32_t* __restrict__ active) {
  const GTile g = tiles[blockIdx.x];
  if (!active[g.member]) return;
  const GRestJob<V> J = jobs[g.job];
  mrestrict_entry(J.T, J.r, J.bc, J.xc, J.nc, (int64_t)g.tile * kBlock + threadIdx.x);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_gprolong(const GProlJob<V>* __restrict__ jobs,
                                                     const GTile* __restrict__ tiles,
                                                     const int32_t* __restrict__ active) {
  const GTile g = tiles[blockIdx.x];
  if (!active[g.member]) return;
  const GProlJob<V> J = jobs[g.job];
  const int64_t t = (int64_t)g.tile * kBlock + threadIdx.x;
  if (t >= J.n * K) return;
  mprolong_entry(J.q_col, J.q_val, J.q_cnt, (int32_t)J.n, J.xc, J.x, t);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_ggemv(const GGemvJob<V>* __restrict__ jobs,
                                                  const GTile* __restrict__ tiles, const int32_t* __restrict__ active) {
  const GTile g = tiles[blockIdx.x];
  if (!active[g.member]) return;
  const GGemvJob<V> J = jobs[g.job];
  const int64_t t = (int64_t)g.tile * kBlock + threadIdx.x;
  if (t >= J.n * K) return;
  mgemv_entry(J.M, J.b, J.x, J.n, t);
}

template <class V>
__global__ void __launch_bounds__(kTailThreads) k_gtail(const TailDescT<V>* __restrict__ descs,
                                                        const int32_t* __restrict__ members,
                                                        const int32_t* __restrict__ active) {
  if (!active[members[blockIdx.x]]) return;
  mtail_run(descs[blockIdx.x]);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_gkry_init(const GKryJob<V>* __restrict__ jobs,
                                                      const GTile* __restrict__ tiles,
                                                      const int32_t* __restrict__ active) {
  const GTile g = tiles[blockIdx.x];
  if (!active[g.member]) return;
  const GKryJob<V>& J = jobs[g.job];
  mkry_init_entry(J.p, J.r_old, J.n * K, J.scal, (int64_t)g.tile * kBlock + threadIdx.x);
}

// the cycle's start (as bat_precondition): the float cycle reads r rounded to
// float; the iterate starts at zero
template <class V>
__global__ void __launch_bounds__(kBlock) k_gcycle_start(const GKryJob<V>* __restrict__ jobs,
                                                         const GTile* __restrict__ tiles,
                                                         const int32_t* __restrict__ active) {
  const GTile g = tiles[blockIdx.x];
  if (!active[g.member]) return;
  const GKryJob<V>& J = jobs[g.job];
  const int64_t i = (int64_t)g.tile * kBlock + threadIdx.x;
  if (i >= J.n * K) return;
  if constexpr (std::is_same<V, float>::value) J.cb[i] = (float)J.r[i];
  J.cx[i] = V(0);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_gkry_dots(const GKryJob<V>* __restrict__ jobs,
                                                      const int32_t* __restrict__ active) {
  const int32_t m = blockIdx.x / kNormBlocks;
  if (!active[m]) return;
  const GKryJob<V>& J = jobs[m];
  mkry_dots_block(J.r, J.r_old, (const V*)J.cx, J.n * K, J.part, blockIdx.x % kNormBlocks, kNormBlocks);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_gkry_beta(const GKryJob<V>* __restrict__ jobs,
                                                      const int32_t* __restrict__ active) {
  if (!active[blockIdx.x]) return;
  const GKryJob<V>& J = jobs[blockIdx.x];
  mkry_beta_block(J.part, J.scal);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_gkry_p(const GKryJob<V>* __restrict__ jobs, const GTile* __restrict__ tiles,
                                                   const int32_t* __restrict__ active) {
  const GTile g = tiles[blockIdx.x];
  if (!active[g.member]) return;
  const GKryJob<V>& J = jobs[g.job];
  mkry_p_entry((const V*)J.cx, J.scal, J.p, J.n * K, (int64_t)g.tile * kBlock + threadIdx.x);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_gkry_spmv(const GKryJob<V>* __restrict__ jobs,
                                                      const int32_t* __restrict__ active) {
  const int32_t m = blockIdx.x / kNormBlocks;
  if (!active[m]) return;
  const GKryJob<V>& J = jobs[m];
  mkry_spmv_block(J.A0, J.p, J.q, J.n, J.part, blockIdx.x % kNormBlocks, kNormBlocks);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_gkry_alpha(const GKryJob<V>* __restrict__ jobs,
                                                       const int32_t* __restrict__ active) {
  if (!active[blockIdx.x]) return;
  const GKryJob<V>& J = jobs[blockIdx.x];
  mkry_alpha_block(J.part, J.scal, J.flags);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_gkry_update(const GKryJob<V>* __restrict__ jobs,
                                                        const int32_t* __restrict__ active) {
  const int32_t m = blockIdx.x / kNormBlocks;
  if (!active[m]) return;
  const GKryJob<V>& J = jobs[m];
  mkry_update_block(J.x, J.p, J.q, J.r, J.r_old, J.scal, J.n * K, J.part, blockIdx.x % kNormBlocks, kNormBlocks);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_gkry_norm(const GKryJob<V>* __restrict__ jobs, int which,
                                                      const int32_t* __restrict__ active) {
  if (!active[blockIdx.x]) return;
  const GKryJob<V>& J = jobs[blockIdx.x];
  mkry_norm_block(J.part, J.scal + which * K);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_gresidual_norm(const GKryJob<V>* __restrict__ jobs,
                                                           const int32_t* __restrict__ active) {
  const int32_t m = blockIdx.x / kNormBlocks;
  if (!active[m]) return;
  const GKryJob<V>& J = jobs[m];
  mresidual_norm_block(J.A0, J.b, J.x, J.r, J.n, J.part, blockIdx.x % kNormBlocks, kNormBlocks);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_gnorm_partials_b(const GKryJob<V>* __restrict__ jobs,
                                                             const int32_t* __restrict__ active) {
  const int32_t m = blockIdx.x / kNormBlocks;
  if (!active[m]) return;
  const GKryJob<V>& J = jobs[m];
  mnorm_partials_block(J.b, J.n * K, J.part, blockIdx.x % kNormBlocks, kNormBlocks);
}

template <class V>
__global__ void k_ggather_scalars(const GKryJob<V>* __restrict__ jobs, int32_t count, int which, uint64_t* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)count * (K + 1)) return;
  const int32_t m = (int32_t)(t / (K + 1));
  const int q = (int)(t % (K + 1));
  const GKryJob<V>& J = jobs[m];
  out[t] = q < K ? __builtin_bit_cast(uint64_t, J.scal[which * K + q]) : (uint64_t)(uint32_t)*J.flags;
}

}  // namespace

// ------------------------------------------------------------ launchers
void mzero_columns(double* x, int64_t n, unsigned mask, hipStream_t s) {
  k_mzero_columns<<<blocks_for(n * K), kBlock, 0, s>>>(x, n, mask);
}

template <class V>
void mgs_sweep(const LevelViewT<V>& v, const Level& lv, hipStream_t s, bool descending) {
  const int C = (int)lv.color_ptr.size() - 1;
  for (int k = 0; k < C; ++k) {
    const int c = descending ? C - 1 - k : k;
    const int32_t r0 = lv.color_ptr[c], r1 = lv.color_ptr[c + 1];
    if (r1 <= r0) continue;
    k_mgs<V><<<blocks_for((int64_t)(r1 - r0) * K), kBlock, 0, s>>>(v.A, v.diag, v.b, v.x, r0, r1);
  }
}

template <class V>
void mresidual(const LevelViewT<V>& v, hipStream_t s) {
  k_mresidual<V><<<blocks_for((int64_t)v.n * K), kBlock, 0, s>>>(v.A, v.b, v.x, v.r, v.n);
}

template <class V>
void mrestrict(const LevelViewT<V>& v, const LevelViewT<V>& c, hipStream_t s) {
  k_mrestrict<V><<<blocks_for((int64_t)c.n * K), kBlock, 0, s>>>(v.T, v.r, c.b, c.x, c.n);
}

template <class V>
void mprolong(const LevelViewT<V>& v, const LevelViewT<V>& c, hipStream_t s) {
  k_mprolong<V><<<blocks_for((int64_t)v.n * K), kBlock, 0, s>>>(v, c.x, v.x);
}

template <class V>
void mcoarse(const double* cinv, const LevelViewT<V>& c, hipStream_t s) {
  k_mgemv<V><<<blocks_for(c.n * K), kBlock, 0, s>>>(cinv, c.b, c.x, c.n);
}

template <class V>
void mtail(const TailDescT<V>& d, hipStream_t s) {
  k_mtail<V><<<1, kTailThreads, (size_t)d.lds_elems * sizeof(V), s>>>(d);
}

void mkry_init(Batch& k, int64_t n, hipStream_t s) {
  k_mkry_init<<<blocks_for(n * K), kBlock, 0, s>>>(k.p, k.r_old, n * K, k.scal);
}

template <class V>
void mkry_direction(Batch& k, const V* z, int64_t n, hipStream_t s) {
  k_mkry_dots<V><<<kNormBlocks, kBlock, 0, s>>>(k.r, k.r_old, z, n * K, k.part);
  k_mkry_beta<<<1, kBlock, 0, s>>>(k.part, k.scal);
  k_mkry_p<V><<<blocks_for(n * K), kBlock, 0, s>>>(z, k.scal, k.p, n * K);
}

void mkry_step(Batch& k, const Level& l0, int32_t* flags, hipStream_t s) {
  const int64_t n = l0.n;
  k_mkry_spmv<<<kNormBlocks, kBlock, 0, s>>>(l0.view.A, k.p, k.q, n, k.part);
  k_mkry_alpha<<<1, kBlock, 0, s>>>(k.part, k.scal, flags);
  k_mkry_update<<<kNormBlocks, kBlock, 0, s>>>(k.x, k.p, k.q, k.r, k.r_old, k.scal, n * K, k.part);
  k_mkry_norm<<<1, kBlock, 0, s>>>(k.part, k.scal + KS_NORM * K);
}

void mresidual_norm(Batch& k, const Level& l0, double* out, hipStream_t s) {
  k_mresidual_norm<<<kNormBlocks, kBlock, 0, s>>>(l0.view.A, k.b, k.x, k.r, l0.n, k.part);
  k_mkry_norm<<<1, kBlock, 0, s>>>(k.part, out);
}

void mnorms(const double* v, int64_t n, double* part, double* out, hipStream_t s) {
  k_mnorm_partials<<<kNormBlocks, kBlock, 0, s>>>(v, n * K, part);
  k_mkry_norm<<<1, kBlock, 0, s>>>(part, out);
}

void mgather(const int32_t* perm, const double* src, int64_t n, int nq, double* dst, hipStream_t s) {
  k_mgather<<<blocks_for(n * K), kBlock, 0, s>>>(perm, src, n, nq, dst);
}

template <class V>
void mscatter(const int32_t* perm, const V* src, int64_t n, int nq, double* dst, hipStream_t s) {
  k_mscatter_v<V><<<blocks_for(n * K), kBlock, 0, s>>>(perm, src, n, nq, dst);
}

// ------------------------------------------------------------ grouped launchers
template <class V>
void gsweep(const GSweepJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s) {
  if (ntiles > 0) k_gsweep<V><<<ntiles, kBlock, 0, s>>>(jobs, tiles, active);
}

template <class V>
void gresidual(const GResJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s) {
  if (ntiles > 0) k_gresidual<V><<<ntiles, kBlock, 0, s>>>(jobs, tiles, active);
}

template <class V>
void grestrict(const GRestJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s) {
  if (ntiles > 0) k_grestrict<V><<<ntiles, kBlock, 0, s>>>(jobs, tiles, active);
}

template <class V>
void gprolong(const GProlJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s) {
  if (ntiles > 0) k_gprolong<V><<<ntiles, kBlock, 0, s>>>(jobs, tiles, active);
}

template <class V>
void ggemv(const GGemvJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s) {
  if (ntiles > 0) k_ggemv<V><<<ntiles, kBlock, 0, s>>>(jobs, tiles, active);
}

template <class V>
void gtail(const TailDescT<V>* descs, const int32_t* members, int32_t count, int32_t lds_bytes, const int32_t* active,
           hipStream_t s) {
  if (count > 0) k_gtail<V><<<count, kTailThreads, (size_t)lds_bytes, s>>>(descs, members, active);
}

template <class V>
void gkry_init(const GKryJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s) {
  if (ntiles > 0) k_gkry_init<V><<<ntiles, kBlock, 0, s>>>(jobs, tiles, active);
}

template <class V>
void gcycle_start(const GKryJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s) {
  if (ntiles > 0) k_gcycle_start<V><<<ntiles, kBlock, 0, s>>>(jobs, tiles, active);
}

template <class V>
void gkry_direction(const GKryJob<V>* jobs, int32_t count, const GTile* tiles, int32_t ntiles, const int32_t* active,
                    hipStream_t s) {
  k_gkry_dots<V><<<count * kNormBlocks, kBlock, 0, s>>>(jobs, active);
  k_gkry_beta<V><<<count, kBlock, 0, s>>>(jobs, active);
  k_gkry_p<V><<<ntiles, kBlock, 0, s>>>(jobs, tiles, active);
}

template <class V>
void gkry_step(const GKryJob<V>* jobs, int32_t count, const int32_t* active, hipStream_t s) {
  k_gkry_spmv<V><<<count * kNormBlocks, kBlock, 0, s>>>(jobs, active);
  k_gkry_alpha<V><<<count, kBlock, 0, s>>>(jobs, active);
  k_gkry_update<V><<<count * kNormBlocks, kBlock, 0, s>>>(jobs, active);
  k_gkry_norm<V><<<count, kBlock, 0, s>>>(jobs, KS_NORM, active);
}

template <class V>
void gnorms_b(const GKryJob<V>* jobs, int32_t count, const int32_t* active, hipStream_t s) {
  k_gnorm_partials_b<V><<<count * kNormBlocks, kBlock, 0, s>>>(jobs, active);
  k_gkry_norm<V><<<count, kBlock, 0, s>>>(jobs, KS_BNORM, active);
}

template <class V>
void gresidual_norms(const GKryJob<V>* jobs, int32_t count, const int32_t* active, hipStream_t s) {
  k_gresidual_norm<V><<<count * kNormBlocks, kBlock, 0, s>>>(jobs, active);
  k_gkry_norm<V><<<count, kBlock, 0, s>>>(jobs, KS_NORM, active);
}

template <class V>
void ggather_scalars(const GKryJob<V>* jobs, int32_t count, int which, uint64_t* out, hipStream_t s) {
  const int64_t nt = (int64_t)count * (K + 1);
  k_ggather_scalars<V><<<blocks_for(nt), kBlock, 0, s>>>(jobs, count, which, out);
}

#define GMG_INSTANTIATE_GROUPED(V)                                                                           \
  template void gsweep<V>(const GSweepJob<V>*, const GTile*, int32_t, const int32_t*, hipStream_t);           \
  template void gresidual<V>(const GResJob<V>*, const GTile*, int32_t, const int32_t*, hipStream_t);          \
  template void grestrict<V>(const GRestJob<V>*, const GTile*, int32_t, const int32_t*, hipStream_t);         \
  template void gprolong<V>(const GProlJob<V>*, const GTile*, int32_t, const int32_t*, hipStream_t);          \
  template void ggemv<V>(const GGemvJob<V>*, const GTile*, int32_t, const int32_t*, hipStream_t);             \
  template void gtail<V>(const TailDescT<V>*, const int32_t*, int32_t, int32_t, const int32_t*, hipStream_t); \
  template void gkry_init<V>(const GKryJob<V>*, const GTile*, int32_t, const int32_t*, hipStream_t);          \
  template void gcycle_start<V>(const GKryJob<V>*, const GTile*, int32_t, const int32_t*, hipStream_t);       \
  template void gkry_direction<V>(const GKryJob<V>*, int32_t, const GTile*, int32_t, const int32_t*,          \
                                  hipStream_t);                                                              \
  template void gkry_step<V>(const GKryJob<V>*, int32_t, const int32_t*, hipStream_t);                        \
  template void gnorms_b<V>(const GKryJob<V>*, int32_t, const int32_t*, hipStream_t);                         \
  template void gresidual_norms<V>(const GKryJob<V>*, int32_t, const int32_t*, hipStream_t);                  \
  template void ggather_scalars<V>(const GKryJob<V>*, int32_t, int, uint64_t*, hipStream_t);
GMG_INSTANTIATE_GROUPED(double)
GMG_INSTANTIATE_GROUPED(float)
#undef GMG_INSTANTIATE_GROUPED

#define GMG_INSTANTIATE_MULTI(V)                                                                 \
  template void mgs_sweep<V>(const LevelViewT<V>&, const Level&, hipStream_t, bool);            \
  template void mresidual<V>(const LevelViewT<V>&, hipStream_t);                                \
  template void mrestrict<V>(const LevelViewT<V>&, const LevelViewT<V>&, hipStream_t);          \
  template void mprolong<V>(const LevelViewT<V>&, const LevelViewT<V>&, hipStream_t);           \
  template void mcoarse<V>(const double*, const LevelViewT<V>&, hipStream_t);                   \
  template void mtail<V>(const TailDescT<V>&, hipStream_t);                                     \
  template void mkry_direction<V>(Batch&, const V*, int64_t, hipStream_t);                      \
  template void mscatter<V>(const int32_t*, const V*, int64_t, int, double*, hipStream_t);
GMG_INSTANTIATE_MULTI(double)
GMG_INSTANTIATE_MULTI(float)
#undef GMG_INSTANTIATE_MULTI

}  // namespace gmg
