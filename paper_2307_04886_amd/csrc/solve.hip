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

// Level 0's one-lane row sum: per-slice widths (row lengths read), or the
// uniform slice width (U) when the level's SELL has one.
template <int CH, bool U, class V>
__device__ __forceinline__ V row_sum_fine(const Sell<V>& A, int32_t r, const V* x, int32_t skip) {
  if constexpr (U) return row_sum_uni<CH>(A, r, x, skip);
  else return row_sum_seq<CH>(A, r, x, skip);
}

// One colour of a Gauss-Seidel sweep on level 0, rows [r0, r1):
//   x_r <- (b_r - sum_{j != r} A_rj x_j) / A_rr.
// Rows of one colour are not coupled, so they update in parallel.
template <int CH, bool U, class V>
__global__ void __launch_bounds__(kBlock) k_gs_color_fine(Sell<V> A, const V* __restrict__ diag,
                                                          const V* __restrict__ b, V* x, int32_t r0, int32_t r1) {
  const int32_t r = (r0 & ~(kSlice - 1)) + (int32_t)(xcd_block() * kBlock + threadIdx.x);
  if (r < r0 || r >= r1) return;
  const V br = b[r], dr = diag[r];        // issued with the row's loads
  const V acc = row_sum_fine<CH, U>(A, r, x, r);
  x[r] = (br - acc) / dr;
}

// The same update on a Galerkin level, R lanes per row.
template <int R, class V>
__global__ void __launch_bounds__(kBlock) k_gs_color(Sell<V> A, const V* __restrict__ diag,
                                                     const V* __restrict__ b, V* x, int32_t r0, int32_t r1,
                                                     int32_t maxlen) {
  const int64_t g = ((int64_t)xcd_block() * kBlock + threadIdx.x) / R;
  const int32_t r = r0 + (int32_t)g;
  const bool active = r < r1;
  const int32_t rc = active ? r : r0;     // in range for every lane: the loads need no branch
  const V br = b[rc], dr = diag[rc];
  const V acc = row_sumR<R>(A, r, active, x, r, maxlen);
  if (active && (threadIdx.x & (R - 1)) == 0) x[r] = (br - acc) / dr;
}

// One block colour of a Gauss-Seidel sweep in block order (levels swept by
// blocks): one workgroup per block (grid cell) of that colour.  Rows of one
// block colour in different blocks are never coupled, so the blocks run at
// once; inside a block the colours run one after the other, separated by
// workgroup barriers, with the block's iterates and the values of its halo
// (the rows of other blocks its rows read, which this launch does not change)
// in LDS.  Thread p holds local rows p and p + kBlkThreads (R of them) with
// their entries in registers: the LDS slot of each column and its value, in
// the row's entry order, the diagonal replaced by a zero term (slot `pad`
// holds +0), so x_i <- (b_i - sum_{j != i} A_ij x_j) / A_ii is computed with
// the terms added in entry order, as on the other paths.  NG gather slots per
// thread cover the gather list (NG * kBlkThreads >= its stride); they are
// read branch-free (slots past the stride re-read its last entry), so the
// list's loads are in flight together.  The register budget sets how many
// workgroups a compute unit holds at once (at 168 VGPRs, three: 768 on the
// chip), and so whether a level's blocks of one colour run in a single round;
// a variant that needs more registers must be measured for it.
template <int R, int K, int NG, class V>
__global__ void __launch_bounds__(kBlkThreads) k_gs_block(BlockView<V> B, const V* __restrict__ bvec,
                                                          const V* __restrict__ diag, V* x, int32_t blk0,
                                                          int32_t c_begin, int32_t descending) {
  extern __shared__ double lds_raw[];
  V* xl = reinterpret_cast<V*>(lds_raw);
  const int32_t b = blk0 + (int32_t)blockIdx.x;
  // first: the header and the gather list (addresses from the block index
  // alone), then the entries, row data and iterates they point to
  const BlockHdr hd = B.hdr[b];
  const int32_t* gl = B.glist + (int64_t)b * B.gstride;
  int32_t gi[NG];
#pragma unroll
  for (int j = 0; j < NG; ++j) gi[j] = gl[min((int32_t)threadIdx.x + j * kBlkThreads, B.gstride - 1)];
  const int32_t r0 = hd.r0, rows = hd.rows, nh = hd.nh, w = hd.w, e0 = hd.e0;
  const int C = B.ncls;
  const int32_t pad = rows + nh;
  const uint64_t present = hd.mask;          // colours with rows in the block
  // Row data and entries.  Two forms with the same values in every slot that
  // is used.  Double: per-lane conditional loads (lanes past the block's rows
  // and slots past its width take the zero term), which fit 168 VGPRs.  Float:
  // no branch inside a wavefront (with per-lane conditions the compiler waited
  // for each load before issuing the next): a wavefront without rows of the
  // block skips them (its registers are never read), lanes past the block's
  // rows re-read its last row (masked where the rows are swept) and slots
  // past the width re-read its last slot (their products are replaced by zero
  // where the row is summed).
  constexpr bool kClamp = sizeof(V) == 4;
  const int32_t wbase = __builtin_amdgcn_readfirstlane((int32_t)threadIdx.x & ~(kWave - 1));
  int32_t info[R];
  V bv[R], dv[R];
  int32_t lx[R][K];
  V lv[R][K];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int32_t p = (int32_t)threadIdx.x + q * kBlkThreads;
    if constexpr (kClamp) {
      const int32_t pc = min(p, rows - 1);
      if (wbase + q * kBlkThreads < rows) {
        info[q] = B.rinfo[r0 + pc];
#pragma unroll
        for (int t = 0; t < K; ++t) {
          const int32_t o = e0 + min(t, w - 1) * rows + pc;
          lx[q][t] = B.elx[o];
          lv[q][t] = B.elv[o];
        }
      }
    } else {
      const bool own = p < rows;
      info[q] = own ? B.rinfo[r0 + p] : 0;
#pragma unroll
      for (int t = 0; t < K; ++t) {
        const bool e = own && t < w;
        lx[q][t] = e ? B.elx[e0 + t * rows + p] : pad;
        lv[q][t] = e ? B.elv[e0 + t * rows + p] : V(0);
      }
    }
  }
  // the block's own rows (thread p holds rows p, p + kBlkThreads, ...) and its halo
#pragma unroll
  for (int j = 0; j < NG; ++j) {
    const int32_t k = (int32_t)threadIdx.x + j * kBlkThreads;
    if (k < pad) {
      xl[k] = x[gi[j]];
      if (j < R && k < rows) {
        bv[j] = bvec[gi[j]];
        dv[j] = diag[gi[j]];
      }
    }
  }
  if (threadIdx.x == 0) xl[pad] = V(0);
  __syncthreads();
  for (int kk = c_begin; kk < C; ++kk) {
    const int c = descending ? C - 1 - kk : kk;
    if (!((present >> c) & 1)) continue;                // no row of this colour in the block
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if ((int32_t)threadIdx.x + q * kBlkThreads < rows && (info[q] & 0xFF) == c) {
        const int32_t len = info[q] >> 8;
        // every gather of the row is issued at once, then the products are
        // added in entry order, in chunks of 8 up to the row's length
        // (terms past the row are +0); the largest shape works a chunk at a
        // time, within its registers
        constexpr int G = R * K <= 64 ? K : 8;
        V s = V(0);
#pragma unroll
        for (int g0 = 0; g0 < K; g0 += G) {
          if (g0 < w) {
            V pr[G];
#pragma unroll
            for (int t = 0; t < G; ++t)
              pr[t] = (!kClamp || g0 + t < w ? lv[q][g0 + t] : V(0)) * xl[lx[q][g0 + t]];
#pragma unroll
            for (int t0 = 0; t0 < G; t0 += 8) {
              if (g0 + t0 < len) {
#pragma unroll
                for (int u = 0; u < 8; ++u) s = s + pr[t0 + u];
              }
            }
          }
        }
        xl[(int32_t)threadIdx.x + q * kBlkThreads] = (bv[q] - s) / dv[q];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int32_t p = (int32_t)threadIdx.x + q * kBlkThreads;
    if (p < rows) x[gi[q]] = xl[p];
  }
}

// r = b - A x on level 0
template <int CH, bool U, class V>
__global__ void __launch_bounds__(kBlock) k_residual_fine(Sell<V> A, const V* __restrict__ b,
                                                          const V* __restrict__ x, V* __restrict__ res,
                                                          int64_t n) {
  const int64_t r = (int64_t)xcd_block() * kBlock + threadIdx.x;
  if (r >= n) return;
  res[r] = b[r] - row_sum_fine<CH, U>(A, (int32_t)r, x, -1);
}

// r = b - A x on a Galerkin level, R lanes per row
template <int R, class V>
__global__ void __launch_bounds__(kBlock) k_residual(Sell<V> A, const V* __restrict__ b, const V* __restrict__ x,
                                                     V* __restrict__ res, int64_t n, int32_t maxlen) {
  const int64_t g = ((int64_t)xcd_block() * kBlock + threadIdx.x) / R;
  const bool active = g < n;
  const V acc = row_sumR<R>(A, (int32_t)g, active, x, -1, maxlen);
  if (active && (threadIdx.x & (R - 1)) == 0) res[g] = b[g] - acc;
}

// r = b - A x on level 0 (double), plus per-block partial sums of r^2 (fixed
// grid: deterministic).
template <int CH, bool U>
__global__ void __launch_bounds__(kBlock) k_residual_norm(SellView A, const double* __restrict__ b,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ res, int64_t n,
                                                          double* partials) {
  // logical block lb covers rows lb * kBlock + k * gridDim.x * kBlock and
  // writes partials[lb], whichever XCD runs it
  const uint32_t lb = xcd_block();
  double sq = 0.0;
  for (int64_t r = (int64_t)lb * kBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kBlock) {
    const double v = b[r] - row_sum_fine<CH, U>(A, (int32_t)r, x, -1);
    res[r] = v;
    sq += v * v;
  }
  double t = block_sum(sq);
  if (threadIdx.x == 0) partials[lb] = t;
}

__global__ void __launch_bounds__(kBlock) k_norm_partials(const double* v, int64_t n, double* partials) {
  double sq = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    sq += v[i] * v[i];
  double t = block_sum(sq);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// The norm into out and, when host_out is set (pinned host memory), there too,
// so that the host sees it without a copy.
__global__ void __launch_bounds__(kBlock) k_finish_norm(const double* partials, double* out, double* host_out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < kNormBlocks; i += kBlock) s += partials[i];
  double t = block_sum(s);
  if (threadIdx.x == 0) {
    const double v = sqrt(t);
    *out = v;
    if (host_out)
      __hip_atomic_store(reinterpret_cast<uint64_t*>(host_out), __builtin_bit_cast(uint64_t, v), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// b_c[I] = sum over row I of P^T (ascending original fine index) of P[i,I] r_i,
// and the coarse iterate starts from zero: x_c[I] = 0.  Rows I < first (the
// first colour of the coarse level, when its first pre-smoothing colour is
// folded in here) take that colour's Gauss-Seidel update from the zero
// iterate instead: every neighbour term is a product with +0, the sum is +0,
// and x_c[I] = (b_c[I] - 0) / A_c[I,I], the value the sweep would write.
template <int R, class V>
__global__ void __launch_bounds__(kBlock) k_restrict(Sell<V> T, const V* __restrict__ r, V* __restrict__ bc,
                                                     V* __restrict__ xc, int64_t nc, int32_t maxlen,
                                                     const V* __restrict__ diag_c, int32_t first,
                                                     const int32_t* __restrict__ orow) {
  const int64_t g = ((int64_t)xcd_block() * kBlock + threadIdx.x) / R;
  const bool active = g < nc;
  const V acc = row_sumR<R>(T, (int32_t)g, active, r, -1, maxlen);
  if (active && (threadIdx.x & (R - 1)) == 0) {
    const int64_t o = orow ? orow[g] : g;        // T's row g is coarse row o
    bc[o] = acc;
    xc[o] = o < first ? (acc - V(0)) / diag_c[o] : V(0);
  }
}

// The same restriction with one lane per coarse row (its terms loaded CH at a
// time and added in entry order, as by the R-lane form).
template <int CH, class V>
__global__ void __launch_bounds__(kBlock) k_restrict_seq(Sell<V> T, const V* __restrict__ r, V* __restrict__ bc,
                                                         V* __restrict__ xc, int64_t nc,
                                                         const V* __restrict__ diag_c, int32_t first,
                                                         const int32_t* __restrict__ orow) {
  const int64_t g = (int64_t)xcd_block() * kBlock + threadIdx.x;
  if (g >= nc) return;
  const V acc = row_sum_seq<CH>(T, (int32_t)g, r, -1);
  const int64_t o = orow ? orow[g] : g;          // T's row g is coarse row o
  bc[o] = acc;
  xc[o] = o < first ? (acc - V(0)) / diag_c[o] : V(0);
}

// x_i <- x_i + sum_t P[i, t] x_c[col_t]
template <class V>
__global__ void __launch_bounds__(kBlock) k_prolong_correct(LevelViewT<V> L, const V* __restrict__ xc,
                                                            V* __restrict__ x) {
  const int64_t i = (int64_t)xcd_block() * kBlock + threadIdx.x;
  if (i >= L.n) return;
  prolong_row(L, xc, x, (int32_t)i);
}

// x = A_c^-1 b in double (b widened from V, x rounded to V): row i is the sum
// over k ascending of (A_c^-1 e_k)_i b_k, stored at inv[k ld + i]; one thread
// per row (the loads of a wavefront are coalesced).
template <class V>
__global__ void __launch_bounds__(kBlock) k_dense_gemv(const double* __restrict__ M, const V* __restrict__ b,
                                                       V* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  const int64_t ld = inv_ld(n);
  // the loads of eight terms are issued before they are added (in ascending k)
  int64_t k = 0;
  for (; k + 8 <= n; k += 8) {
    double m[8], v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      m[u] = M[(k + u) * ld + i];
      v[u] = (double)b[k + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = acc + m[u] * v[u];
  }
  for (; k < n; ++k) acc = acc + M[k * ld + i] * (double)b[k];
  x[i] = (V)acc;
}

// The V-cycle below a level with few rows, in one workgroup: every phase
// (colour of a sweep, residual, restriction, coarsest solve, prolongation) is
// separated by a workgroup barrier instead of a kernel boundary, and the tail
// levels' vectors x, b and r live in LDS.  Each phase performs exactly the
// operations of the corresponding multi-launch kernel, in the same order.
//
// One lane per row, four wavefronts (one per SIMD, so that a lane can hold a
// whole row in registers).  Rows are handled in rounds of kTailThreads1 rows;
// the matrix entries of the next round, which do not depend on x, are loaded
// before the current round computes, so that their latency overlaps the
// current round and the barrier that ends a colour.  The matrices are read in
// the per-colour ELL of the tail levels (see LevelViewT), whose padded terms
// are exactly +0.
constexpr int kTailThreads1 = 256;
constexpr int kTailW = 32;                 // entries of a row held in registers; the rest load on demand
constexpr int kTailProlong = 4;            // prolongation rows per thread whose loads are issued together
constexpr int kTailGemv = 16;              // columns of the coarsest inverse per prefetched chunk
constexpr int kTailLoad = 16;              // elements per thread of the first tail level's loads into LDS

struct TailSeg {
  int32_t lo, hi, w, off;                  // rows [lo, hi), ELL width, offset of entry (0, lo)
};

template <class V>
struct TailRow {
  int32_t j[kTailW];
  V v[kTailW];
  V d;
  int32_t w;                               // entries loaded for the wavefront's rows (uniform)
};

__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Tail matrix loads go through buffer resources: a scalar base and bound, a
// uniform (scalar) offset for the entry column and the lane's row offset, so
// that no vector instruction is spent on addresses.
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc make_rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)(uint32_t)bytes, 0x00020000);
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 bload16(Rsrc r, uint32_t voff, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
}
// (the 8-byte form returns one 64-bit integer)
__device__ __forceinline__ uint64_t bload8(Rsrc r, uint32_t voff, uint32_t soff) {
  return (uint64_t)__builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ double as_f64(uint32_t lo, uint32_t hi) {
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Two consecutive values of a tail ELL value array (one block) for one lane.
template <class V>
__device__ __forceinline__ void val_pair(Rsrc r, uint32_t voff, uint32_t soff, V& a, V& b);
template <>
__device__ __forceinline__ void val_pair<double>(Rsrc r, uint32_t voff, uint32_t soff, double& a, double& b) {
  const u32x4 u = bload16(r, voff * 16u, soff * 8u);
  a = as_f64(u.x, u.y);
  b = as_f64(u.z, u.w);
}
template <>
__device__ __forceinline__ void val_pair<float>(Rsrc r, uint32_t voff, uint32_t soff, float& a, float& b) {
  const uint64_t u = bload8(r, voff * 8u, soff * 4u);
  a = __builtin_bit_cast(float, (uint32_t)u);
  b = __builtin_bit_cast(float, (uint32_t)(u >> 32));
}

// An ELL matrix of the tail: column and value arrays.
template <class V>
struct TailMat {
  Rsrc col, val;
};
template <class V>
__device__ __forceinline__ TailMat<V> tail_mat(const int32_t* col, const V* val, int64_t slots) {
  return TailMat<V>{make_rsrc(col, slots * 4), make_rsrc(val, slots * (int64_t)sizeof(V))};
}

// Entries t0..t0+3 of the lane's row (row offset lo in a segment of cnt rows
// at element offset off): one 4-entry column block, two 2-entry value blocks.
template <class V>
__device__ __forceinline__ void tail_quad(const TailMat<V>& M, uint32_t off, uint32_t cnt, uint32_t lo,
                                          uint32_t t0, int32_t* j, V* v) {
  const u32x4 c = bload16(M.col, lo * 16u, (off + (t0 >> 2) * cnt * 4u) * 4u);
  j[0] = (int32_t)c.x;
  j[1] = (int32_t)c.y;
  j[2] = (int32_t)c.z;
  j[3] = (int32_t)c.w;
#pragma unroll
  for (int b = 0; b < 2; ++b) val_pair<V>(M.val, lo, off + ((t0 >> 1) + b) * cnt * 2u, v[2 * b], v[2 * b + 1]);
}

// A row offset whose lane offsets (16 or 8 bytes per row) lie past every tail
// array: such a buffer load reads no memory and returns zeros.
constexpr uint32_t kTailNoRow = 0x08000000u;

// Entries 0..kTailW-1 of row r (clamped into the segment by the caller), up to
// w (uniform over the wavefront, a multiple of 4 within the segment's width),
// and its diagonal when D.  The quads past w are loads out of the buffer's
// range (no memory traffic), so that every round issues the same number of
// loads and the consumer of a round waits only for that round's loads, not
// for the next round's already in flight.
template <bool D, class V>
__device__ __forceinline__ void tail_fetch(const TailMat<V>& M, const V* diag, const TailSeg& sg, int32_t r,
                                           int32_t w, TailRow<V>& q) {
  const uint32_t cnt = (uint32_t)(sg.hi - sg.lo);
  const uint32_t lo = (uint32_t)(r - sg.lo);
  q.w = w;
#pragma unroll
  for (int g = 0; g < kTailW / 4; ++g)
    tail_quad(M, (uint32_t)sg.off, cnt, 4 * g < w ? lo : kTailNoRow, (uint32_t)(4 * g), q.j + 4 * g, q.v + 4 * g);
  if (D) q.d = diag[r];
}

// sum over the row's entries in entry order of val * X[col]; the entries past
// the row's end up to the wavefront's width are padding (+0 terms)
template <class V>
__device__ __forceinline__ V tail_sum(const TailMat<V>& M, const TailSeg& sg, int32_t r, const TailRow<V>& q,
                                      const V* X) {
  const int32_t w = q.w;
  // all gathers first, so that they are in flight together
  V xv[kTailW];
#pragma unroll
  for (int g = 0; g < kTailW / 4; ++g)
    if (4 * g < w) {
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[4 * g + u] = X[q.j[4 * g + u]];
    }
  V acc = V(0);
#pragma unroll
  for (int g = 0; g < kTailW / 4; ++g)
    if (4 * g < w) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = acc + q.v[4 * g + u] * xv[4 * g + u];
    }
  const uint32_t cnt = (uint32_t)(sg.hi - sg.lo);
  const uint32_t lo = (uint32_t)(r - sg.lo);
  for (int32_t t0 = kTailW; t0 < w; t0 += 4) {
    int32_t j[4];
    V v[4];
    tail_quad(M, (uint32_t)sg.off, cnt, lo, (uint32_t)t0, j, v);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = acc + v[u] * X[j[u]];
  }
  return acc;
}

// Runs the rows of segments 0..nseg-1 (seg(s) -> TailSeg) through the
// pipeline; out(r, acc, diag) consumes each row's sum.  A wavefront loads the
// entries up to WW[r] of its rows (WW in LDS, the same for the wavefront's 64
// rows), or up to the segment's width when WW is null.  A workgroup barrier
// follows every segment when `barrier_each` (colours of a sweep), else only
// the last.  Two row buffers alternate (no copies between rounds).
template <bool D, class V, class Seg, class Out>
__device__ __forceinline__ void tail_rows(const TailMat<V>& M, const V* diag, const uint16_t* WW, int nseg, Seg seg,
                                          const V* X, bool barrier_each, Out out) {
  const int32_t tid = threadIdx.x;
  auto width = [&](const TailSeg& g, int32_t r) { return WW ? uniform((int32_t)WW[r]) : g.w; };
  TailSeg sg = seg(0);
  int s = 0;
  int32_t r0 = sg.lo;
  TailRow<V> ra, rb;
  {
    const int32_t r = max(min(r0 + tid, sg.hi - 1), 0);
    tail_fetch<D>(M, diag, sg, r, width(sg, r), ra);
  }
  // one round: loads the next round into nxt, then computes cur; false after the last
  auto round = [&](TailRow<V>& cur, TailRow<V>& nxt) {
    TailSeg sg2 = sg;
    int s2 = s;
    int32_t r2 = r0 + kTailThreads1;
    const bool last_round = r2 >= sg.hi;
    if (last_round) {
      s2 = s + 1;
      if (s2 < nseg) {
        sg2 = seg(s2);
        r2 = sg2.lo;
      }
    }
    const bool more = s2 < nseg;
    if (!more) {                // the loads stay unconditional (same count in flight on every path)
      sg2 = sg;
      r2 = r0;
    }
    {
      const int32_t rn = max(min(r2 + tid, sg2.hi - 1), 0);
      tail_fetch<D>(M, diag, sg2, rn, width(sg2, rn), nxt);
    }
    const int32_t r = r0 + tid;
    const V acc = tail_sum(M, sg, max(min(r, sg.hi - 1), 0), cur, X);
    if (r < sg.hi) out(r, acc, cur.d);
    if (last_round && (barrier_each || !more)) __syncthreads();
    sg = sg2;
    s = s2;
    r0 = r2;
    return more;
  };
  while (round(ra, rb) && round(rb, ra)) {
  }
}

template <class V>
struct TailLds {
  V *x, *b, *r;
  const int4* c;                           // colour table (lo, hi, w, off)
  const uint16_t* w;                       // rows' wavefront widths
};

template <class V>
__device__ __forceinline__ TailLds<V> tail_lds(const TailDescT<V>& d, char* lds, int l) {
  TailLds<V> t;
  t.x = reinterpret_cast<V*>(lds + d.o_x[l]);
  t.b = reinterpret_cast<V*>(lds + d.o_b[l]);
  t.r = reinterpret_cast<V*>(lds + d.o_r[l]);
  t.c = reinterpret_cast<const int4*>(lds + d.o_c[l]);
  t.w = reinterpret_cast<const uint16_t*>(lds + d.o_w[l]);
  return t;
}

__device__ __forceinline__ TailSeg colour_seg(const int4* ct, int c) {
  const int4 e = ct[c];
  return TailSeg{uniform(e.x), uniform(e.y), uniform(e.z), uniform(e.w)};
}

// nsweeps Gauss-Seidel sweeps over the colours of one tail level.
template <class V>
__device__ __forceinline__ void tail_gs(const LevelViewT<V>& L, const TailLds<V>& t, int nsweeps, bool descending) {
  const int nc = L.ncolors;
  if (nsweeps <= 0) return;
  tail_rows<true>(
      tail_mat(L.e_col_gs, L.e_val_gs, L.e_slots), L.diag, t.w, nsweeps * nc,
      [&](int s) {
        const int i = s % nc;
        return colour_seg(t.c, descending ? nc - 1 - i : i);
      },
      t.x, true, [&](int32_t r, V acc, V dr) { t.x[r] = (t.b[r] - acc) / dr; });
}

template <class V>
__global__ void __launch_bounds__(kTailThreads1) k_tail_vcycle(TailDescT<V> d) {
  extern __shared__ double lds_raw[];
  char* lds = reinterpret_cast<char*>(lds_raw);
  const int tid = threadIdx.x;
  const int lc = d.nlev - 1;   // the coarsest level
  // the first tail level's x and b (and, when it is not the coarsest, its
  // rows' widths) with its colour table: each chunk's loads are all issued
  // before its LDS writes, so that they wait on one memory latency
  {
    const LevelViewT<V>& L = d.lv[0];
    const TailLds<V> t = tail_lds(d, lds, 0);
    const int32_t n = L.n;
    const bool smoothed = lc > 0;
    uint16_t* ww = reinterpret_cast<uint16_t*>(lds + d.o_w[0]);
    for (int32_t i0 = 0; i0 < n; i0 += kTailLoad * kTailThreads1) {
      V xv[kTailLoad], bv[kTailLoad];
      uint16_t wv[kTailLoad];
#pragma unroll
      for (int u = 0; u < kTailLoad; ++u) {
        const int32_t i = min(i0 + u * kTailThreads1 + tid, n - 1);
        xv[u] = L.x[i];
        bv[u] = L.b[i];
        wv[u] = smoothed ? L.e_ww[i] : (uint16_t)0;
      }
      if (i0 == 0 && smoothed) {
        int32_t* ct = reinterpret_cast<int32_t*>(lds + d.o_c[0]);
        for (int i = tid; i < 4 * L.ncolors; i += kTailThreads1) ct[i] = L.e_cinfo[i];
      }
#pragma unroll
      for (int u = 0; u < kTailLoad; ++u) {
        const int32_t i = i0 + u * kTailThreads1 + tid;
        if (i < n) {
          t.x[i] = xv[u];
          t.b[i] = bv[u];
          if (smoothed) ww[i] = wv[u];
        }
      }
    }
  }
  // the other smoothed tail levels' colour tables and widths; the zeros behind x and r
  for (int l = 0; l < lc; ++l) {
    const LevelViewT<V>& L = d.lv[l];
    const TailLds<V> t = tail_lds(d, lds, l);
    if (l > 0) {
      int32_t* ct = reinterpret_cast<int32_t*>(lds + d.o_c[l]);
      for (int i = tid; i < 4 * L.ncolors; i += kTailThreads1) ct[i] = L.e_cinfo[i];
      uint16_t* ww = reinterpret_cast<uint16_t*>(lds + d.o_w[l]);
      for (int i = tid; i < L.n; i += kTailThreads1) ww[i] = L.e_ww[i];
    }
    if (tid == 0) {
      t.x[L.n] = V(0);
      t.r[L.n] = V(0);
    }
  }
  __syncthreads();
  for (int l = 0; l < lc; ++l) {
    const LevelViewT<V>& L = d.lv[l];
    const TailLds<V> t = tail_lds(d, lds, l);
    tail_gs(L, t, d.nu_pre, false);
    // r = b - A x, colour by colour
    tail_rows<false>(
        tail_mat(L.e_col, L.e_val, L.e_slots), L.diag, t.w, L.ncolors, [&](int s) { return colour_seg(t.c, s); },
        t.x, false,
        [&](int32_t r, V acc, V) { t.r[r] = t.b[r] - acc; });
    // b_c = P^T r, x_c = 0
    const TailLds<V> tc = tail_lds(d, lds, l + 1);
    const int32_t nc = d.lv[l + 1].n;
    tail_rows<false>(
        tail_mat(L.e_tcol, L.e_tval, L.e_tslots), L.diag, nullptr, 1,
        [&](int) { return TailSeg{0, nc, uniform(L.e_wt), 0}; },
        t.r, false,
        [&](int32_t r, V acc, V) {
          tc.b[r] = acc;
          tc.x[r] = V(0);
        });
  }
  {
    // x_c = A_c^-1 b_c in double: row i is the sum over k ascending of
    // (A_c^-1 e_k)_i b_k, stored at inv[k ld + i].  Each lane sums two rows
    // (2l, 2l + 1: one 16-byte load per column); the next chunk of columns is
    // loaded while one is summed.
    const TailLds<V> t = tail_lds(d, lds, lc);
    const int32_t n = d.lv[lc].n;
    const int32_t ld = (int32_t)inv_ld(n);
    const Rsrc inv = make_rsrc(d.cinv, (int64_t)n * ld * 8);
    for (int32_t i0 = 0; i0 < n; i0 += 2 * kTailThreads1) {
      const int32_t i = min(i0 + 2 * tid, ld - 2);       // even: rows i, i + 1 (i + 1 = ld - 1 may be padding)
      u32x4 m[kTailGemv], mn[kTailGemv];
#pragma unroll
      for (int u = 0; u < kTailGemv; ++u) m[u] = bload16(inv, (uint32_t)i * 8u, (uint32_t)(min(u, n - 1) * ld) * 8u);
      double acc0 = 0.0, acc1 = 0.0;
      for (int32_t k0 = 0; k0 < n; k0 += kTailGemv) {
#pragma unroll
        for (int u = 0; u < kTailGemv; ++u)
          mn[u] = bload16(inv, (uint32_t)i * 8u, (uint32_t)(min(k0 + kTailGemv + u, n - 1) * ld) * 8u);
#pragma unroll
        for (int u = 0; u < kTailGemv; ++u)
          if (k0 + u < n) {
            const double bk = (double)t.b[min(k0 + u, n - 1)];
            acc0 = acc0 + as_f64(m[u].x, m[u].y) * bk;
            acc1 = acc1 + as_f64(m[u].z, m[u].w) * bk;
          }
#pragma unroll
        for (int u = 0; u < kTailGemv; ++u) m[u] = mn[u];
      }
      const int32_t r = i0 + 2 * tid;
      if (r < n) t.x[r] = (V)acc0;
      if (r + 1 < n) t.x[r + 1] = (V)acc1;
    }
    __syncthreads();
  }
  for (int l = lc - 1; l >= 0; --l) {
    const LevelViewT<V>& L = d.lv[l];
    const TailLds<V> t = tail_lds(d, lds, l);
    const V* XC = tail_lds(d, lds, l + 1).x;
    // x_i += sum_t P[i, t] x_c[col_t]; the loads of kTailProlong rows per thread are issued together
    for (int32_t i0 = 0; i0 < L.n; i0 += kTailProlong * kTailThreads1) {
      int32_t c[kTailProlong];
      int32_t j[kTailProlong][3];
      V v[kTailProlong][3];
#pragma unroll
      for (int u = 0; u < kTailProlong; ++u) {
        const int32_t i = min(i0 + u * kTailThreads1 + tid, L.n - 1);
        c[u] = L.q_cnt[i];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          j[u][e] = L.q_col[(int64_t)e * L.n + i];
          v[u][e] = L.q_val[(int64_t)e * L.n + i];
        }
      }
#pragma unroll
      for (int u = 0; u < kTailProlong; ++u) {
        const int32_t i = i0 + u * kTailThreads1 + tid;
        if (i < L.n) {
          V acc = V(0);
#pragma unroll
          for (int e = 0; e < 3; ++e)
            if (e < c[u]) acc = acc + v[u][e] * XC[j[u][e]];
          t.x[i] = t.x[i] + acc;
        }
      }
    }
    __syncthreads();
    tail_gs(L, t, d.nu_post, d.descending_post != 0);
  }
  {
    const TailLds<V> t = tail_lds(d, lds, 0);
    for (int32_t i = tid; i < d.lv[0].n; i += kTailThreads1) d.lv[0].x[i] = t.x[i];
  }
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

// Calls f(std::integral_constant<int, CH>, std::integral_constant<bool, U>) for
// the load chunk CH of the level-0 row kernels and their slice form U (uniform
// width; only where the level's SELL has one).
template <class V, class F>
void with_chunk(const LevelViewT<V>& v, F&& f) {
  auto go = [&](auto UC) {
    switch (v.ch) {
      case 4: f(std::integral_constant<int, 4>{}, UC); break;
      case 16: f(std::integral_constant<int, 16>{}, UC); break;
      default: f(std::integral_constant<int, 8>{}, UC); break;
    }
  };
  if (v.uni && v.A.uw > 0) go(std::integral_constant<bool, true>{});
  else go(std::integral_constant<bool, false>{});
}

// One sweep in block order: the four block colours one launch each.  `skip`
// (ascending sweeps only): the first colour of block colour 0 is already done.
template <class V>
void block_sweep(const LevelViewT<V>& v, const Level& lv, hipStream_t s, bool descending, bool timed, int skip) {
  const BlockView<V>& B = v.B;
  if (!B.hdr || !B.glist || !B.elx || !B.elv || !B.rinfo || B.gstride <= 0 ||
      B.gstride > kBlkGather * kBlkThreads)
    throw Error{GMG_DEVICE_ERROR, "block sweep layout incomplete"};
  for (int k = 0; k < 4; ++k) {
    const int bc = descending ? 3 - k : k;
    const int32_t nb = B.bstart[bc + 1] - B.bstart[bc];
    if (nb <= 0) continue;
    double bytes = 0.0;
    for (int c = 0; c < B.ncls; ++c) bytes += lv.color_bytes[bc * B.ncls + c];
    KernelTimer::Scope t(timed ? (int)KernelTimer::GS_GALERKIN : -1, bytes);
    const int c_begin = !descending && k == 0 ? skip : 0;
    auto go = [&](auto kern) {
      hipExtLaunchKernelGGL(kern, dim3(nb), dim3(kBlkThreads), (size_t)B.lds_bytes, s, t.start, t.stop, 0, B,
                            (const V*)v.b, (const V*)v.diag, v.x, B.bstart[bc], c_begin, descending ? 1 : 0);
    };
    // gather slots: 2 cover lists of up to 512 rows and halo, 8 the largest (2048)
    const bool g2 = B.gstride <= 2 * kBlkThreads;
    if (B.rows_per_thread == 1) {
      if (B.width <= 32) {
        if (g2) go(k_gs_block<1, 32, 2, V>); else go(k_gs_block<1, 32, kBlkGather, V>);
      } else {
        if (g2) go(k_gs_block<1, 64, 2, V>); else go(k_gs_block<1, 64, kBlkGather, V>);
      }
    } else {
      if (B.width <= 32) {
        if (g2) go(k_gs_block<2, 32, 2, V>); else go(k_gs_block<2, 32, kBlkGather, V>);
      } else {
        if (g2) go(k_gs_block<2, 64, 2, V>); else go(k_gs_block<2, 64, kBlkGather, V>);
      }
    }
  }
}

template <class V>
void gs_sweep(const LevelViewT<V>& v, const Level& lv, hipStream_t s, bool finest, bool descending, bool timed,
              int skip) {
  if (!finest && v.B.nblk > 0) {
    block_sweep(v, lv, s, descending, timed, skip);
    return;
  }
  const int C = (int)lv.color_ptr.size() - 1;
  for (int k = skip; k < C; ++k) {
    const int c = descending ? C - 1 - k : k;
    const int32_t r0 = lv.color_ptr[c], r1 = lv.color_ptr[c + 1];
    if (r1 <= r0) continue;
    if (finest) {
      KernelTimer::Scope t(timed ? (int)KernelTimer::GS_FINEST : -1, lv.color_bytes[c]);
      const int32_t span = r1 - (r0 & ~(kSlice - 1));
      with_chunk(v, [&](auto CC, auto UC) {
        constexpr int CH = decltype(CC)::value;
        constexpr bool U = decltype(UC)::value;
        hipExtLaunchKernelGGL(k_gs_color_fine<CH, U, V>, dim3(blocks_for(span)), dim3(kBlock), 0, s, t.start,
                              t.stop, 0, v.A, (const V*)v.diag, (const V*)v.b, v.x, r0, r1);
      });
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
    with_chunk(v, [&](auto CC, auto UC) {
      constexpr int CH = decltype(CC)::value;
      constexpr bool U = decltype(UC)::value;
      k_residual_fine<CH, U, V><<<blocks_for(v.n), kBlock, 0, s>>>(v.A, v.b, v.x, v.r, v.n);
    });
  } else {
    with_lanes(v.ra, [&](auto RC) {
      constexpr int R = decltype(RC)::value;
      k_residual<R, V><<<blocks_for((int64_t)v.n * R), kBlock, 0, s>>>(v.A, v.b, v.x, v.r, v.n, v.maxa);
    });
  }
}

template <class V>
void restrict_to(const LevelViewT<V>& v, const LevelViewT<V>& c, hipStream_t s, int32_t first) {
  // the original-order copy of P^T where the level has one (row map to_row)
  const Sell<V>& T = v.to_row ? v.To : v.T;
  if (v.rt == 1) {
    k_restrict_seq<8, V><<<blocks_for(c.n), kBlock, 0, s>>>(T, v.r, c.b, c.x, c.n, (const V*)c.diag, first,
                                                            v.to_row);
    return;
  }
  with_lanes(v.rt, [&](auto RC) {
    constexpr int R = decltype(RC)::value;
    k_restrict<R, V><<<blocks_for((int64_t)c.n * R), kBlock, 0, s>>>(T, v.r, c.b, c.x, c.n, v.maxt,
                                                                      (const V*)c.diag, first, v.to_row);
  });
}

template <class V>
void prolong_correct(const LevelViewT<V>& v, const LevelViewT<V>& c, hipStream_t s) {
  k_prolong_correct<V><<<blocks_for(v.n), kBlock, 0, s>>>(v, c.x, v.x);
}

template <class V>
void coarse_solve(const double* cinv, const LevelViewT<V>& c, hipStream_t s) {
  k_dense_gemv<V><<<blocks_for(c.n), kBlock, 0, s>>>(cinv, c.b, c.x, c.n);
}

template <class V>
void tail_vcycle(const TailDescT<V>& d, hipStream_t s) {
  k_tail_vcycle<V><<<1, kTailThreads1, (size_t)d.lds_bytes, s>>>(d);
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
  with_chunk(lv.view, [&](auto CC, auto UC) {
    constexpr int CH = decltype(CC)::value;
    constexpr bool U = decltype(UC)::value;
    hipExtLaunchKernelGGL(k_residual_norm<CH, U>, dim3(kNormBlocks), dim3(kBlock), 0, s, t.start, t.stop, 0,
                          lv.view.A, b, x, res, (int64_t)lv.n, partials);
  });
}

void finish_norm(const double* partials, double* out, hipStream_t s, double* host_out) {
  k_finish_norm<<<1, kBlock, 0, s>>>(partials, out, host_out);
}

void check_finite(const double* v, int64_t n, int32_t* flag, hipStream_t s) {
  k_check_finite<<<blocks_for(n), kBlock, 0, s>>>(v, n, flag);
}

#define GMG_INSTANTIATE(V)                                                                              \
  template void gs_sweep<V>(const LevelViewT<V>&, const Level&, hipStream_t, bool, bool, bool, int);  \
  template void residual<V>(const LevelViewT<V>&, hipStream_t, bool);                                  \
  template void restrict_to<V>(const LevelViewT<V>&, const LevelViewT<V>&, hipStream_t, int32_t);      \
  template void prolong_correct<V>(const LevelViewT<V>&, const LevelViewT<V>&, hipStream_t);           \
  template void coarse_solve<V>(const double*, const LevelViewT<V>&, hipStream_t);                     \
  template void tail_vcycle<V>(const TailDescT<V>&, hipStream_t);                                      \
  template void fill_zero<V>(V*, int64_t, hipStream_t);                                                \
  template void permute_out<V>(const int32_t*, const V*, double*, int64_t, hipStream_t);
GMG_INSTANTIATE(double)
GMG_INSTANTIATE(float)
#undef GMG_INSTANTIATE

}  // namespace gmg
