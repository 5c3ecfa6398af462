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

template <class V>
__global__ void __launch_bounds__(kBlock) k_mgs(Sell<V> A, const V* __restrict__ diag, const V* __restrict__ b,
                                                V* x, int32_t r0, int32_t r1) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int32_t r = r0 + (int32_t)(t / K);
  const int q = (int)(t % K);
  if (r >= r1) return;
  const V br = b[(int64_t)r * K + q], dr = diag[r];
  const V acc = row_sum_multi(A, r, x, r, q);
  x[(int64_t)r * K + q] = (br - acc) / dr;
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_mresidual(Sell<V> A, const V* __restrict__ b, const V* __restrict__ x,
                                                      V* __restrict__ res, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n * K) return;
  const int32_t r = (int32_t)(t / K);
  const int q = (int)(t % K);
  res[t] = b[t] - row_sum_multi(A, r, x, -1, q);
}

template <class V>
__global__ void __launch_bounds__(kBlock) k_mrestrict(Sell<V> T, const V* __restrict__ r, V* __restrict__ bc,
                                                      V* __restrict__ xc, int64_t nc) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= nc * K) return;
  bc[t] = row_sum_multi(T, (int32_t)(t / K), r, -1, (int)(t % K));
  xc[t] = V(0);                                   // the coarse iterate starts from zero
}

template <class V>
__device__ __forceinline__ void mprolong_entry(const LevelViewT<V>& L, const V* xc, V* x, int64_t t) {
  const int32_t i = (int32_t)(t / K);
  const int q = (int)(t % K);
  const int32_t c = L.q_cnt[i];
  V acc = V(0);
  V v[3], u[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    v[s] = L.q_val[(int64_t)s * L.n + i];
    u[s] = xc[(int64_t)L.q_col[(int64_t)s * L.n + i] * K + q];
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
  mprolong_entry(L, xc, x, t);
}

// x = A_c^-1 b for the K right-hand sides, in double, as the single-vector
// coarse solve: entry (i, q) is the sum over k ascending of (A_c^-1 e_k)_i b_kq.
template <class V>
__device__ __forceinline__ void mgemv_entry(const double* M, const V* b, V* x, int64_t n, int64_t t) {
  const int64_t i = t / K;
  const int q = (int)(t % K);
  double acc = 0.0;
  const int64_t ld = inv_ld(n);
  for (int64_t k = 0; k < n; ++k) acc = acc + M[k * ld + i] * (double)b[k * K + q];
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
__global__ void __launch_bounds__(kTailThreads) k_mtail(TailDescT<V> d) {
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
    for (int64_t t = tid; t < (int64_t)L.n * K; t += kTailThreads) mprolong_entry(L, XC, XL, t);
    __syncthreads();
    for (int s = 0; s < d.nu_post; ++s) mtail_gs(L, XL, d.descending_post != 0);
  }
  if (d.lds_off[0] >= 0)
    for (int64_t i = tid; i < (int64_t)d.lv[0].n * K; i += kTailThreads) d.lv[0].x[i] = X(0)[i];
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

__global__ void k_mkry_init(double* p, double* r_old, int64_t nk, double* scal) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
__global__ void __launch_bounds__(kBlock) k_mkry_dots(const double* __restrict__ r, const double* __restrict__ r_old,
                                                      const V* __restrict__ z, int64_t nk, double* part) {
  __shared__ double o1[K], o2[K];
  double a = 0.0, c = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nk; i += (int64_t)gridDim.x * kBlock) {
    const double zi = (double)z[i];
    a += r[i] * zi;
    c += r_old[i] * zi;
  }
  block_sums_by_rhs(a, o1);
  block_sums_by_rhs(c, o2);
  if (threadIdx.x < K) {
    part[(int64_t)blockIdx.x * K + threadIdx.x] = o1[threadIdx.x];
    part[(int64_t)(kNormBlocks + blockIdx.x) * K + threadIdx.x] = o2[threadIdx.x];
  }
}

__global__ void __launch_bounds__(kBlock) k_mkry_beta(const double* part, double* scal) {
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
__global__ void k_mkry_p(const V* __restrict__ z, const double* __restrict__ scal, double* __restrict__ p,
                         int64_t nk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nk) return;
  p[i] = (double)z[i] + scal[KS_BETA * K + i % K] * p[i];
}

__global__ void __launch_bounds__(kBlock) k_mkry_spmv(SellView A, const double* __restrict__ p, double* __restrict__ qv,
                                                      int64_t n, double* part) {
  __shared__ double o[K];
  double s = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n * K; t += (int64_t)gridDim.x * kBlock) {
    const double v = row_sum_multi(A, (int32_t)(t / K), p, -1, (int)(t % K));
    qv[t] = v;
    s += p[t] * v;
  }
  block_sums_by_rhs(s, o);
  if (threadIdx.x < K) part[(int64_t)(2 * kNormBlocks + blockIdx.x) * K + threadIdx.x] = o[threadIdx.x];
}

// alpha = rho / p.q per right-hand side; rho = 0 (an exactly solved one) gives alpha = 0
__global__ void __launch_bounds__(kBlock) k_mkry_alpha(const double* part, double* scal, int32_t* flags) {
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

__global__ void __launch_bounds__(kBlock) k_mkry_update(double* __restrict__ x, const double* __restrict__ p,
                                                        const double* __restrict__ qv, double* __restrict__ r,
                                                        double* __restrict__ r_old, const double* __restrict__ scal,
                                                        int64_t nk, double* part) {
  __shared__ double o[K];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nk; i += (int64_t)gridDim.x * kBlock) {
    const double alpha = scal[KS_ALPHA * K + i % K];
    x[i] = x[i] + alpha * p[i];
    const double ri = r[i];
    r_old[i] = ri;
    const double rn = ri - alpha * qv[i];
    r[i] = rn;
    s += rn * rn;
  }
  block_sums_by_rhs(s, o);
  if (threadIdx.x < K) part[(int64_t)blockIdx.x * K + threadIdx.x] = o[threadIdx.x];
}

__global__ void __launch_bounds__(kBlock) k_mkry_norm(const double* part, double* out /* [K] */) {
  __shared__ double s[K];
  finish_by_rhs(part, s);
  if (threadIdx.x < K) out[threadIdx.x] = sqrt(s[threadIdx.x]);
}

// r = b - A x (level 0, double) and partials of |r_q|^2
__global__ void __launch_bounds__(kBlock) k_mresidual_norm(SellView A, const double* __restrict__ b,
                                                           const double* __restrict__ x, double* __restrict__ res,
                                                           int64_t n, double* part) {
  __shared__ double o[K];
  double s = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n * K; t += (int64_t)gridDim.x * kBlock) {
    const double v = b[t] - row_sum_multi(A, (int32_t)(t / K), x, -1, (int)(t % K));
    res[t] = v;
    s += v * v;
  }
  block_sums_by_rhs(s, o);
  if (threadIdx.x < K) part[(int64_t)blockIdx.x * K + threadIdx.x] = o[threadIdx.x];
}

__global__ void __launch_bounds__(kBlock) k_mnorm_partials(const double* v, int64_t nk, double* part) {
  __shared__ double o[K];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nk; i += (int64_t)gridDim.x * kBlock)
    s += v[i] * v[i];
  block_sums_by_rhs(s, o);
  if (threadIdx.x < K) part[(int64_t)blockIdx.x * K + threadIdx.x] = o[threadIdx.x];
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
