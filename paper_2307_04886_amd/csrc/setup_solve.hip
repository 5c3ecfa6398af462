// Solve-phase setup: the Gauss-Seidel colouring of each A_l, the
// colour-sorted solve layout (SELL-64 matrix, SoA prolongation, restriction
// rows), and the dense factorisation of the coarsest operator (Alg. 2 solves
// the coarsest level directly).
#include "gmg_internal.hpp"

namespace gmg {

namespace {

// ------------------------------------------------------------------ colouring
// Greedy first-fit colouring in hashed key order, run as Jones-Plassmann
// rounds: a row is coloured once all its lower-key neighbours are, with the
// smallest colour none of them uses.  Decisions are final, so colours are
// written in place.
struct ColorKey {
  uint64_t base;
  __device__ uint64_t operator()(int32_t v) const { return mix64(base ^ (uint64_t)v); }
};

__global__ void __launch_bounds__(kBlock) k_color_round(const int32_t* rp, const int32_t* col, int64_t n,
                                                        ColorKey key, int32_t* color, int32_t* ncol,
                                                        int32_t* rounds, int k) {
  if (k > 0 && rounds[k - 1] == 0) return;
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool pending = false;
  if (v < n && color[v] < 0) {
    const uint64_t kv = key((int32_t)v);
    uint64_t mask = 0;
    bool blocked = false, high = false;
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
      int32_t u = col[e];
      if (u == v) continue;
      uint64_t ku = key(u);
      if (!(ku < kv || (ku == kv && u < v))) continue;
      int32_t cu = __atomic_load_n(&color[u], __ATOMIC_RELAXED);
      if (cu < 0) { blocked = true; break; }
      if (cu < 64) mask |= 1ull << cu; else high = true;
    }
    if (blocked) {
      pending = true;
    } else {
      int32_t c = (~mask) ? __builtin_ctzll(~mask) : 64;
      if (c == 64 && high) {
        for (;; ++c) {                              // rare: every colour below 64 is taken
          bool used = false;
          for (int32_t e = rp[v]; e < rp[v + 1] && !used; ++e) {
            int32_t u = col[e];
            if (u == v) continue;
            uint64_t ku = key(u);
            if ((ku < kv || (ku == kv && u < v)) && color[u] == c) used = true;
          }
          if (!used) break;
        }
      }
      color[v] = c;
      atomicMax(ncol, c + 1);
    }
  }
  unsigned long long b = __ballot(pending);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(&rounds[k], __popcll(b));
}

// ------------------------------------------------------------------ stable colour partition
// hist[c * nb + b] = rows of colour c in block b; its exclusive scan gives,
// for every (colour, block), the first new index, so new indices are sorted
// by (colour, old index).
__global__ void __launch_bounds__(kBlock) k_color_hist(const int32_t* color, int64_t n, int nb, int nc,
                                                       int32_t* hist) {
  extern __shared__ int32_t cnt[];
  for (int c = threadIdx.x; c < nc; c += blockDim.x) cnt[c] = 0;
  __syncthreads();
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) atomicAdd(&cnt[color[v]], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < nc; c += blockDim.x) hist[(int64_t)c * nb + blockIdx.x] = cnt[c];
}

__global__ void __launch_bounds__(kBlock) k_color_place(const int32_t* color, int64_t n, int nb,
                                                        const int32_t* off, int32_t* perm, int32_t* iperm) {
  __shared__ int32_t cl[kBlock];
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  cl[threadIdx.x] = v < n ? color[v] : -1;
  __syncthreads();
  if (v >= n) return;
  int32_t c = cl[threadIdx.x], rank = 0;
  for (int t = 0; t < (int)threadIdx.x; ++t) rank += cl[t] == c;
  int32_t nw = off[(int64_t)c * nb + blockIdx.x] + rank;
  perm[nw] = (int32_t)v;
  iperm[v] = nw;
}

__global__ void k_color_ptr(const int32_t* off, int nb, int nc, int32_t* cptr) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= nc) cptr[c] = off[(int64_t)c * nb];
}

// ------------------------------------------------------------------ SELL-64 matrix
__global__ void k_row_len(const int32_t* perm, const int32_t* arp, int64_t n, int32_t* len) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) len[r] = arp[perm[r] + 1] - arp[perm[r]];
}

__global__ void k_slice_width(const int32_t* len, int64_t n, int64_t ns, int32_t* wsz) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  int32_t w = 0;
  for (int64_t r = s * kSlice; r < (s + 1) * kSlice && r < n; ++r) w = len[r] > w ? len[r] : w;
  wsz[s] = w * kSlice;
}

// Entries keep the CSR order of the original row (so every row sum adds its
// terms in the same order as the definition); columns are renumbered.
__global__ void k_sell_fill(const int32_t* perm, const int32_t* iperm, const int32_t* arp,
                            const int32_t* acol, const double* aval, int64_t n, const int32_t* sptr,
                            int32_t* scol, double* sval, double* diag) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int64_t s = r / kSlice, ln = r % kSlice;
  int32_t old = perm[r];
  int32_t b = arp[old], e = arp[old + 1];
  int32_t w = (sptr[s + 1] - sptr[s]) / kSlice;
  for (int32_t t = 0; t < w; ++t) {
    int64_t o = sptr[s] + (int64_t)t * kSlice + ln;
    if (b + t < e) {
      int32_t j = acol[b + t];
      scol[o] = iperm[j];
      sval[o] = aval[b + t];
      if (j == old) diag[r] = aval[b + t];
    } else {
      scol[o] = (int32_t)r;
      sval[o] = 0.0;
    }
  }
}

// P in the new numbering, SoA ELL-3 ([3][n]); padding repeats the first
// column with weight 0.
__global__ void k_p_layout(const int32_t* perm, const int32_t* ciperm, const int32_t* pcol,
                           const double* pval, const int32_t* pcnt, int64_t n, int32_t* qcol, double* qval,
                           int32_t* qcnt) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int32_t old = perm[r];
  int32_t c = pcnt[old];
  qcnt[r] = c;
  int32_t first = c > 0 ? pcol[3 * old] : 0;
  first = (ciperm && c > 0) ? ciperm[first] : first;
  for (int t = 0; t < 3; ++t) {
    int32_t j = t < c ? pcol[3 * old + t] : -1;
    qcol[t * n + r] = t < c ? (ciperm ? ciperm[j] : j) : first;
    qval[t * n + r] = t < c ? pval[3 * old + t] : 0.0;
  }
}

__global__ void k_t_len(const int32_t* trp, const int32_t* ciperm, int64_t nc, int32_t* len) {
  int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I < nc) len[ciperm ? ciperm[I] : I] = trp[I + 1] - trp[I];
}

__global__ void k_t_fill(const int32_t* trp, const int32_t* tcol, const double* tval, const int32_t* ciperm,
                         const int32_t* fiperm, int64_t nc, const int32_t* nrp, int32_t* ncol, double* nval) {
  int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int32_t o = nrp[ciperm ? ciperm[I] : I];
  for (int32_t q = trp[I]; q < trp[I + 1]; ++q, ++o) {
    ncol[o] = fiperm[tcol[q]];
    nval[o] = tval[q];
  }
}

// ------------------------------------------------------------------ coarsest level
__global__ void k_dense_scatter(const int32_t* rp, const int32_t* col, const double* val, int64_t n,
                                double* D) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t e = rp[i]; e < rp[i + 1]; ++e) D[i * n + col[e]] = val[e];
}

// Right-looking dense Cholesky in one workgroup.  Entry (i, c) receives its
// updates -L[i][j] * L[c][j] in ascending j, i.e. the same operations in the
// same order as the column-by-column (left-looking) definition.
__global__ void __launch_bounds__(1024) k_cholesky(double* D, int64_t n, int32_t* flags) {
  __shared__ int bad;
  __shared__ double piv;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int64_t j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double s = D[j * n + j];
      if (!(s > 0.0)) {
        bad = 1;
        atomicOr(flags, F_NOT_SPD);
      } else {
        piv = sqrt(s);
        D[j * n + j] = piv;
      }
    }
    __syncthreads();
    if (bad) return;
    const double d = piv;
    for (int64_t i = j + 1 + threadIdx.x; i < n; i += blockDim.x) D[i * n + j] = D[i * n + j] / d;
    __syncthreads();
    const int64_t m = n - j - 1;
    for (int64_t idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      int64_t a = idx / m, c = idx % m;
      if (c > a) continue;
      int64_t i = j + 1 + a, k = j + 1 + c;
      D[i * n + k] = D[i * n + k] - D[i * n + j] * D[k * n + j];
    }
    __syncthreads();
  }
}

// Lower factor L (zeros above the diagonal) and its transpose U.
__global__ void k_split_factor(const double* D, int64_t n, double* L, double* U) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  int64_t i = idx / n, k = idx % n;
  double v = k <= i ? D[i * n + k] : 0.0;
  L[idx] = v;
  U[k * n + i] = v;
}

// Column c of A^-1 by forward then backward substitution with L, one
// wavefront per column; written as row c (A^-1 is symmetric).
__global__ void __launch_bounds__(kWave) k_chol_inverse(const double* L, const double* U, int64_t n,
                                                        double* inv) {
  extern __shared__ double y[];
  const int64_t c = blockIdx.x;
  const int lane = threadIdx.x;
  for (int64_t i = lane; i < n; i += kWave) y[i] = 0.0;
  __syncthreads();
  for (int64_t i = c; i < n; ++i) {
    double s = 0.0;
    for (int64_t m = c + lane; m < i; m += kWave) s += L[i * n + m] * y[m];
    s = wave_sum(s);
    if (lane == 0) y[i] = ((i == c ? 1.0 : 0.0) - s) / L[i * n + i];
    __syncthreads();
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double s = 0.0;
    for (int64_t m = i + 1 + lane; m < n; m += kWave) s += U[i * n + m] * y[m];
    s = wave_sum(s);
    if (lane == 0) y[i] = (y[i] - s) / U[i * n + i];
    __syncthreads();
  }
  for (int64_t i = lane; i < n; i += kWave) inv[c * n + i] = y[i];
}

}  // namespace

void colouring(Handle& h, Level& lv, int level) {
  hipStream_t s = h.stream;
  int64_t n = lv.n;
  lv.color = (int32_t*)dalloc(h, (size_t)n * 4);
  fill_i32(lv.color, -1, n, s);
  int32_t* ncol = (int32_t*)talloc(s, 4);
  check_hip(hipMemsetAsync(ncol, 0, 4, s), "memset");
  check_hip(hipMemsetAsync(h.rounds, 0, kMaxRounds * 4, s), "memset");
  ColorKey key{(h.opt.seed ^ kColorSalt) ^ ((uint64_t)level << 32)};
  int k = 0;
  for (;;) {
    for (int t = 0; t < kRoundBatch; ++t, ++k)
      k_color_round<<<blocks_for(n), kBlock, 0, s>>>(lv.arp, lv.acol, n, key, lv.color, ncol, h.rounds, k);
    if (read_i64(h, h.rounds + (k - 1), 4) == 0) break;
    if (k + kRoundBatch > kMaxRounds) throw Error{GMG_DEVICE_ERROR, "colouring did not terminate"};
  }
  lv.ncolors = (int32_t)read_i64(h, ncol, 4);
  tfree(s, ncol);
}

void solve_layout(Handle& h, Level& lv, const Level* nx, const int32_t* t_rp, const int32_t* t_col,
                  const double* t_val) {
  hipStream_t s = h.stream;
  const int64_t n = lv.n;
  const int nb = blocks_for(n);
  lv.perm = (int32_t*)dalloc(h, (size_t)n * 4);
  lv.iperm = (int32_t*)dalloc(h, (size_t)n * 4);
  int32_t *hist = nullptr, *off = nullptr, *cptr = nullptr;
  if (lv.color) {
    // rows sorted by (colour, index)
    const int C = lv.ncolors;
    hist = (int32_t*)talloc(s, ((size_t)C * nb + 1) * 4);
    off = (int32_t*)talloc(s, ((size_t)C * nb + 1) * 4);
    k_color_hist<<<nb, kBlock, (size_t)C * 4, s>>>(lv.color, n, nb, C, hist);
    scan_i32(hist, off, (int64_t)C * nb, s);
    k_color_place<<<nb, kBlock, 0, s>>>(lv.color, n, nb, off, lv.perm, lv.iperm);
    cptr = (int32_t*)talloc(s, (size_t)(C + 1) * 4);
    k_color_ptr<<<blocks_for(C + 1), kBlock, 0, s>>>(off, nb, C, cptr);
    lv.color_ptr.assign(C + 1, 0);
    check_hip(hipMemcpyAsync(lv.color_ptr.data(), cptr, (size_t)(C + 1) * 4, hipMemcpyDeviceToHost, s),
              "copy");
  } else {
    // the coarsest level keeps its numbering (it is solved directly)
    iota_i32(lv.perm, n, s);
    iota_i32(lv.iperm, n, s);
    lv.color_ptr = {0, (int32_t)n};
  }
  // SELL-64
  const int64_t ns = (n + kSlice - 1) / kSlice;
  lv.s_len = (int32_t*)dalloc(h, (size_t)n * 4);
  int32_t* wsz = (int32_t*)talloc(s, (size_t)(ns + 1) * 4);
  lv.s_ptr = (int32_t*)dalloc(h, (size_t)(ns + 1) * 4);
  k_row_len<<<blocks_for(n), kBlock, 0, s>>>(lv.perm, lv.arp, n, lv.s_len);
  k_slice_width<<<blocks_for(ns), kBlock, 0, s>>>(lv.s_len, n, ns, wsz);
  scan_i32(wsz, lv.s_ptr, ns, s);
  int64_t tot = read_i64(h, lv.s_ptr + ns, 4);
  lv.s_col = (int32_t*)dalloc(h, (size_t)(tot + 1) * 4);
  lv.s_val = (double*)dalloc(h, (size_t)(tot + 1) * 8);
  lv.diag = (double*)dalloc(h, (size_t)n * 8);
  k_sell_fill<<<blocks_for(n), kBlock, 0, s>>>(lv.perm, lv.iperm, lv.arp, lv.acol, lv.aval, n, lv.s_ptr,
                                               lv.s_col, lv.s_val, lv.diag);
  // vectors
  lv.x = (double*)dalloc(h, (size_t)n * 8);
  lv.b = (double*)dalloc(h, (size_t)n * 8);
  lv.r = (double*)dalloc(h, (size_t)n * 8);
  // prolongation / restriction in the new numbering
  if (nx) {
    const int64_t nc = nx->n;
    const int32_t* ciperm = nx->iperm;           // null on the coarsest level (identity)
    lv.q_col = (int32_t*)dalloc(h, (size_t)3 * n * 4);
    lv.q_val = (double*)dalloc(h, (size_t)3 * n * 8);
    lv.q_cnt = (int32_t*)dalloc(h, (size_t)n * 4);
    k_p_layout<<<blocks_for(n), kBlock, 0, s>>>(lv.perm, ciperm, lv.pcol, lv.pval, lv.pcnt, n, lv.q_col,
                                                lv.q_val, lv.q_cnt);
    int32_t* len = (int32_t*)talloc(s, (size_t)(nc + 1) * 4);
    lv.t_rp = (int32_t*)dalloc(h, (size_t)(nc + 1) * 4);
    k_t_len<<<blocks_for(nc), kBlock, 0, s>>>(t_rp, ciperm, nc, len);
    scan_i32(len, lv.t_rp, nc, s);
    lv.t_col = (int32_t*)dalloc(h, (size_t)(lv.nnzP + 1) * 4);
    lv.t_val = (double*)dalloc(h, (size_t)(lv.nnzP + 1) * 8);
    k_t_fill<<<blocks_for(nc), kBlock, 0, s>>>(t_rp, t_col, t_val, ciperm, lv.iperm, nc, lv.t_rp, lv.t_col,
                                               lv.t_val);
    tfree(s, len);
  }
  sync(s, "solve layout");
  tfree(s, hist);
  tfree(s, off);
  tfree(s, cptr);
  tfree(s, wsz);
}

void coarse_factor(Handle& h, Level& lv) {
  hipStream_t s = h.stream;
  const int64_t n = lv.n;
  double* D = (double*)talloc(s, (size_t)n * n * 8);
  double* U = (double*)talloc(s, (size_t)n * n * 8);
  check_hip(hipMemsetAsync(D, 0, (size_t)n * n * 8, s), "memset");
  k_dense_scatter<<<blocks_for(n), kBlock, 0, s>>>(lv.arp, lv.acol, lv.aval, n, D);
  k_cholesky<<<1, 1024, 0, s>>>(D, n, h.flags);
  h.chol = (double*)dalloc(h, (size_t)n * n * 8);
  h.cinv = (double*)dalloc(h, (size_t)n * n * 8);
  k_split_factor<<<blocks_for(n * n), kBlock, 0, s>>>(D, n, h.chol, U);
  k_chol_inverse<<<(int)n, kWave, (size_t)n * 8, s>>>(h.chol, U, n, h.cinv);
  h.ncoarse = n;
  check_flags(h, "coarsest factorisation");
  tfree(s, D);
  tfree(s, U);
}

}  // namespace gmg
