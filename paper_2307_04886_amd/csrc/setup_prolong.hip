// Hierarchy construction, operator part: the prolongation P_l of Sec. 4.4
// (Voronoi-neighbour candidate triangles, closest-point barycentric weights,
// inverse-distance fallback), its transpose (the restriction), and the
// Galerkin operator A_{l+1} = P_l^T A_l P_l of Alg. 1.
#include "gmg_internal.hpp"

namespace gmg {

namespace {

__device__ inline bool has_edge(const int32_t* rp, const int32_t* col, int32_t a, int32_t b) {
  int32_t lo = rp[a], hi = rp[a + 1];
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (col[mid] < b) lo = mid + 1; else hi = mid;
  }
  return lo < rp[a + 1] && col[lo] == b;
}

// (Nearly) co-linear triangle: |ab x ac|^2 <= (tau |ab|^2) |ac|^2.
__device__ inline bool degenerate(V3 A, V3 B, V3 C) {
  V3 ab = sub3(B, A), ac = sub3(C, A);
  V3 nr = cross3(ab, ac);
  return dot3(nr, nr) <= (kDegenerateTau * dot3(ab, ab)) * dot3(ac, ac);
}

// Barycentric weights of the point of triangle ABC closest to P (face, edge
// or vertex), by the Voronoi-region tests of Ericson, Real-Time Collision
// Detection (2005), Sec. 5.1.5: vertex A, vertex B, edge AB, vertex C, edge
// AC, edge BC, face.
__device__ inline void closest_point(V3 P, V3 A, V3 B, V3 C, double& wa, double& wb, double& wc) {
  V3 ab = sub3(B, A), ac = sub3(C, A), ap = sub3(P, A);
  double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  if (d1 <= 0.0 && d2 <= 0.0) { wa = 1.0; wb = 0.0; wc = 0.0; return; }
  V3 bp = sub3(P, B);
  double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
  if (d3 >= 0.0 && d4 <= d3) { wa = 0.0; wb = 1.0; wc = 0.0; return; }
  double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
    double t = d1 / (d1 - d3);
    wa = 1.0 - t; wb = t; wc = 0.0; return;
  }
  V3 cp = sub3(P, C);
  double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) { wa = 0.0; wb = 0.0; wc = 1.0; return; }
  double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
    double t = d2 / (d2 - d6);
    wa = 1.0 - t; wb = 0.0; wc = t; return;
  }
  double va = d3 * d6 - d5 * d4;
  double e43 = d4 - d3, e56 = d5 - d6;
  if (va <= 0.0 && e43 >= 0.0 && e56 >= 0.0) {
    double t = e43 / (e43 + e56);
    wa = 0.0; wb = 1.0 - t; wc = t; return;
  }
  double a = va < 0.0 ? 0.0 : va, b = vb < 0.0 ? 0.0 : vb, c = vc < 0.0 ? 0.0 : vc;
  double s = (a + b) + c;
  if (!(s > 0.0)) { wa = 1.0; wb = 0.0; wc = 0.0; return; }
  wa = a / s; wb = b / s; wc = c / s;
}

// One thread per fine point p; c = label(p) is the coarse point closest to p.
// Candidates are the triangles (c, j, k), j < k neighbours of c with {j, k} a
// coarse edge, visited in ascending (j, k); the first candidate at the
// smallest point-to-triangle distance is kept.  With no non-degenerate
// candidate, the three points of {c} U N(c) nearest to p (ties by index) get
// inverse-distance weights.  The row keeps its non-zero weights sorted by
// column.
__global__ void __launch_bounds__(kBlock) k_project(const double* X, const int32_t* lab, int64_t n,
                                                    const double* Xc, const int32_t* crp, const int32_t* ccol,
                                                    int32_t* pcol, double* pval, int32_t* pcnt, int32_t* tri,
                                                    unsigned long long* fallback) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool fb = false;
  if (p < n) {
    V3 P = ld3(X, p);
    int32_t c = lab[p];
    V3 A = ld3(Xc, c);
    const int32_t rb = crp[c], re = crp[c + 1];
    bool found = false;
    double best = 0.0, bw0 = 0.0, bw1 = 0.0, bw2 = 0.0;
    int32_t bj = -1, bk = -1;
    for (int32_t e1 = rb; e1 < re; ++e1) {
      int32_t j = ccol[e1];
      V3 B = ld3(Xc, j);
      for (int32_t e2 = e1 + 1; e2 < re; ++e2) {
        int32_t k = ccol[e2];
        if (!has_edge(crp, ccol, j, k)) continue;
        V3 C = ld3(Xc, k);
        if (degenerate(A, B, C)) continue;
        double w0, w1, w2;
        closest_point(P, A, B, C, w0, w1, w2);
        V3 q = {(w0 * A.x + w1 * B.x) + w2 * C.x, (w0 * A.y + w1 * B.y) + w2 * C.y,
                (w0 * A.z + w1 * B.z) + w2 * C.z};
        V3 d = sub3(P, q);
        double d2 = dot3(d, d);
        if (!found || d2 < best) {
          found = true;
          best = d2;
          bj = j;
          bk = k;
          bw0 = w0;
          bw1 = w1;
          bw2 = w2;
        }
      }
    }
    int32_t cols[3];
    double vals[3];
    int cnt;
    if (found) {
      cols[0] = c; cols[1] = bj; cols[2] = bk;
      vals[0] = bw0; vals[1] = bw1; vals[2] = bw2;
      cnt = 3;
    } else {
      fb = true;
      // the (up to) three smallest (d^2, index) pairs among {c} U N(c)
      double sd[3];
      int32_t sq[3];
      int k = 0;
      for (int t = 0; t < 3; ++t) {
        bool have = false;
        double md = 0.0;
        int32_t mq = -1;
        for (int32_t e = rb - 1; e < re; ++e) {
          int32_t q = e < rb ? c : ccol[e];
          V3 d = sub3(P, ld3(Xc, q));
          double d2 = dot3(d, d);
          bool after = t == 0 || d2 > sd[t - 1] || (d2 == sd[t - 1] && q > sq[t - 1]);
          if (after && (!have || d2 < md || (d2 == md && q < mq))) {
            have = true;
            md = d2;
            mq = q;
          }
        }
        if (!have) break;
        sd[t] = md;
        sq[t] = mq;
        k = t + 1;
      }
      if (sd[0] == 0.0) {
        cols[0] = sq[0]; vals[0] = 1.0; cnt = 1;
      } else {
        double inv[3], s = 0.0;
        for (int t = 0; t < k; ++t) { inv[t] = 1.0 / sqrt(sd[t]); s = s + inv[t]; }
        for (int t = 0; t < k; ++t) { cols[t] = sq[t]; vals[t] = inv[t] / s; }
        cnt = k;
      }
    }
    // non-zero weights, sorted by column (columns are distinct)
    int32_t oc[3];
    double ov[3];
    int u = 0;
    for (int t = 0; t < cnt; ++t)
      if (vals[t] != 0.0) { oc[u] = cols[t]; ov[u] = vals[t]; ++u; }
    for (int a = 1; a < u; ++a)
      for (int b = a; b > 0 && oc[b - 1] > oc[b]; --b) {
        int32_t tc = oc[b]; oc[b] = oc[b - 1]; oc[b - 1] = tc;
        double tv = ov[b]; ov[b] = ov[b - 1]; ov[b - 1] = tv;
      }
    for (int t = 0; t < 3; ++t) {
      pcol[3 * p + t] = t < u ? oc[t] : -1;
      pval[3 * p + t] = t < u ? ov[t] : 0.0;
    }
    pcnt[p] = u;
    tri[2 * p] = found ? bj : -1;
    tri[2 * p + 1] = found ? bk : -1;
  }
  unsigned long long b = __ballot(fb);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(fallback, (unsigned long long)__popcll(b));
}

// ------------------------------------------------------------------ P^T
__global__ void k_count_cols(const int32_t* pcol, const int32_t* pcnt, int64_t n, int32_t* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int t = 0; t < pcnt[i]; ++t) atomicAdd(&cnt[pcol[3 * i + t]], 1);
}

__global__ void k_scatter_cols(const int32_t* pcol, const double* pval, const int32_t* pcnt, int64_t n,
                               const int32_t* ptr, int32_t* cur, int32_t* tcol, double* tval) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int t = 0; t < pcnt[i]; ++t) {
    int32_t I = pcol[3 * i + t];
    int32_t pos = ptr[I] + atomicAdd(&cur[I], 1);
    tcol[pos] = (int32_t)i;
    tval[pos] = pval[3 * i + t];
  }
}

// Rows of P^T sorted by fine index (insertion sort on (index, value) pairs).
__global__ void k_sort_pairs(const int32_t* ptr, int32_t* col, double* val, int64_t nrow) {
  int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nrow) return;
  int32_t b = ptr[I], e = ptr[I + 1];
  for (int32_t i = b + 1; i < e; ++i) {
    int32_t c = col[i];
    double v = val[i];
    int32_t j = i - 1;
    while (j >= b && col[j] > c) {
      col[j + 1] = col[j];
      val[j + 1] = val[j];
      --j;
    }
    col[j + 1] = c;
    val[j + 1] = v;
  }
}

// ------------------------------------------------------------------ Galerkin (Alg. 1)
// One wavefront per coarse row I.  The terms of row I are
//   (P[i,I] * A[i,j]) * P[j,J]  for i in row I of P^T (ascending), j in row i
// of A (CSR order), J in row j of P (column order).
// Symbolic pass: the distinct J go into an LDS hash set.  Numeric pass: the
// sorted distinct J are handed one per lane; every lane walks the whole term
// list in the order above and adds the terms of its own column, so each
// entry is summed in exactly the order of the definition's row accumulation.
constexpr int kHash = 1024;

__device__ inline bool hash_insert(int32_t* keys, int32_t J) {
  uint32_t h = ((uint32_t)J * 2654435761u) & (kHash - 1);
  for (int probe = 0; probe < kHash; ++probe) {
    int32_t old = atomicCAS(&keys[h], -1, J);
    if (old == -1 || old == J) return true;
    h = (h + 1) & (kHash - 1);
  }
  return false;
}

__device__ inline bool hash_fill_row(int32_t I, const int32_t* trp, const int32_t* tcol, const int32_t* arp,
                                     const int32_t* acol, const int32_t* pcol, const int32_t* pcnt,
                                     int32_t* keys) {
  const int lane = threadIdx.x;
  for (int s = lane; s < kHash; s += kWave) keys[s] = -1;
  __syncthreads();
  bool ok = true;
  for (int32_t q = trp[I]; q < trp[I + 1]; ++q) {
    int32_t i = tcol[q];
    for (int32_t e = arp[i] + lane; e < arp[i + 1]; e += kWave) {
      int32_t j = acol[e];
      for (int t = 0; t < pcnt[j]; ++t) ok &= hash_insert(keys, pcol[3 * j + t]);
    }
  }
  __syncthreads();
  return ok;
}

__global__ void __launch_bounds__(kWave) k_galerkin_count(const int32_t* trp, const int32_t* tcol,
                                                          const int32_t* arp, const int32_t* acol,
                                                          const int32_t* pcol, const int32_t* pcnt,
                                                          int64_t nc, int32_t* rowcnt, int32_t* flags) {
  __shared__ int32_t keys[kHash];
  int32_t I = blockIdx.x;
  if (I >= nc) return;
  bool ok = hash_fill_row(I, trp, tcol, arp, acol, pcol, pcnt, keys);
  int c = 0;
  for (int s = threadIdx.x; s < kHash; s += kWave) c += keys[s] >= 0;
  c = wave_sum(c);
  if (!ok || c > kHash * 3 / 4) { if (threadIdx.x == 0) atomicOr(flags, F_OVERFLOW); }
  if (threadIdx.x == 0) rowcnt[I] = c;
}

__global__ void __launch_bounds__(kWave) k_galerkin_fill(const int32_t* trp, const int32_t* tcol,
                                                         const double* tval, const int32_t* arp,
                                                         const int32_t* acol, const double* aval,
                                                         const int32_t* pcol, const double* pval,
                                                         const int32_t* pcnt, int64_t nc, const int32_t* crp,
                                                         int32_t* ccol, double* cval, int32_t* flags) {
  __shared__ int32_t keys[kHash];
  __shared__ int32_t list[kHash];
  __shared__ int32_t sorted[kHash];
  __shared__ int32_t nlist;
  int32_t I = blockIdx.x;
  if (I >= nc) return;
  const int lane = threadIdx.x;
  hash_fill_row(I, trp, tcol, arp, acol, pcol, pcnt, keys);
  if (lane == 0) nlist = 0;
  __syncthreads();
  for (int s = lane; s < kHash; s += kWave)
    if (keys[s] >= 0) list[atomicAdd(&nlist, 1)] = keys[s];
  __syncthreads();
  const int k = nlist;
  for (int a = lane; a < k; a += kWave) {
    int32_t key = list[a];
    int rank = 0;
    for (int b = 0; b < k; ++b) rank += list[b] < key;
    sorted[rank] = key;
  }
  __syncthreads();
  const int32_t out = crp[I];
  bool diag_ok = false;
  for (int c0 = 0; c0 < k; c0 += kWave) {
    const bool mine = c0 + lane < k;
    const int32_t myJ = mine ? sorted[c0 + lane] : -1;
    double acc = 0.0;
    for (int32_t q = trp[I]; q < trp[I + 1]; ++q) {
      const int32_t i = tcol[q];
      const double piI = tval[q];
      for (int32_t e = arp[i]; e < arp[i + 1]; ++e) {
        const int32_t j = acol[e];
        const double t1 = piI * aval[e];
        for (int t = 0; t < pcnt[j]; ++t)
          if (pcol[3 * j + t] == myJ) acc = acc + t1 * pval[3 * j + t];
      }
    }
    if (mine) {
      ccol[out + c0 + lane] = myJ;
      cval[out + c0 + lane] = acc;
      if (myJ == I && acc > 0.0) diag_ok = true;
    }
  }
  // a missing or non-positive diagonal makes Gauss-Seidel divide by zero
  unsigned long long b = __ballot(diag_ok);
  if (lane == 0 && b == 0) atomicOr(flags, F_NOT_SPD);
}

}  // namespace

void prolongation(Handle& h, Level& lv, Level& nx) {
  hipStream_t s = h.stream;
  int64_t n = lv.n;
  lv.pcol = (int32_t*)dalloc(h, (size_t)3 * n * 4);
  lv.pval = (double*)dalloc(h, (size_t)3 * n * 8);
  lv.pcnt = (int32_t*)dalloc(h, (size_t)n * 4);
  lv.tri = (int32_t*)dalloc(h, (size_t)2 * n * 4);
  unsigned long long* fb = (unsigned long long*)talloc(s, 8);
  check_hip(hipMemsetAsync(fb, 0, 8, s), "memset");
  k_project<<<blocks_for(n), kBlock, 0, s>>>(lv.X, lv.label, n, nx.X, nx.erp, nx.ecol, lv.pcol, lv.pval,
                                             lv.pcnt, lv.tri, fb);
  lv.fallback = read_i64(h, fb, 8);
  tfree(s, fb);
}

void transpose_p(Handle& h, Level& lv, int64_t nc, int32_t** t_rp, int32_t** t_col, double** t_val) {
  hipStream_t s = h.stream;
  int64_t n = lv.n;
  int32_t* cnt = (int32_t*)talloc(s, (size_t)(nc + 1) * 4);
  int32_t* cur = (int32_t*)talloc(s, (size_t)(nc + 1) * 4);
  int32_t* rp = (int32_t*)talloc(s, (size_t)(nc + 1) * 4);   // freed by the caller
  check_hip(hipMemsetAsync(cnt, 0, (size_t)(nc + 1) * 4, s), "memset");
  check_hip(hipMemsetAsync(cur, 0, (size_t)(nc + 1) * 4, s), "memset");
  k_count_cols<<<blocks_for(n), kBlock, 0, s>>>(lv.pcol, lv.pcnt, n, cnt);
  scan_i32(cnt, rp, nc, s);
  lv.nnzP = read_i64(h, rp + nc, 4);
  int32_t* col = (int32_t*)talloc(s, (size_t)(lv.nnzP + 1) * 4);
  double* val = (double*)talloc(s, (size_t)(lv.nnzP + 1) * 8);
  k_scatter_cols<<<blocks_for(n), kBlock, 0, s>>>(lv.pcol, lv.pval, lv.pcnt, n, rp, cur, col, val);
  k_sort_pairs<<<blocks_for(nc), kBlock, 0, s>>>(rp, col, val, nc);
  tfree(s, cnt);
  tfree(s, cur);
  *t_rp = rp;
  *t_col = col;
  *t_val = val;
}

void galerkin(Handle& h, Level& lv, Level& nx, const int32_t* t_rp, const int32_t* t_col,
              const double* t_val) {
  hipStream_t s = h.stream;
  int64_t nc = nx.n;
  int32_t* cnt = (int32_t*)talloc(s, (size_t)(nc + 1) * 4);
  nx.arp = (int32_t*)dalloc(h, (size_t)(nc + 1) * 4);
  k_galerkin_count<<<(int)nc, kWave, 0, s>>>(t_rp, t_col, lv.arp, lv.acol, lv.pcol, lv.pcnt, nc, cnt,
                                            h.flags);
  scan_i32(cnt, nx.arp, nc, s);
  nx.nnzA = read_i64(h, nx.arp + nc, 4);
  check_flags(h, "Galerkin pattern");
  nx.acol = (int32_t*)dalloc(h, (size_t)(nx.nnzA + 1) * 4);
  nx.aval = (double*)dalloc(h, (size_t)(nx.nnzA + 1) * 8);
  k_galerkin_fill<<<(int)nc, kWave, 0, s>>>(t_rp, t_col, t_val, lv.arp, lv.acol, lv.aval, lv.pcol, lv.pval,
                                           lv.pcnt, nc, nx.arp, nx.acol, nx.aval, h.flags);
  tfree(s, cnt);
}

}  // namespace gmg
