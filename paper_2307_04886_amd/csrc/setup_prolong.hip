// Hierarchy construction, operator part: the prolongation P_l of Sec. 4.4
// (Voronoi-neighbour candidate triangles, closest-point barycentric weights,
// inverse-distance fallback), its transpose (the restriction), and the
// Galerkin operator A_{l+1} = P_l^T A_l P_l of Alg. 1.
#include <algorithm>

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
// AC, edge BC, face.  Returns the region in that order (0 .. 6).
enum : int { kRegionA = 0, kRegionB = 1, kRegionC = 3 };

__device__ inline int closest_point(V3 P, V3 A, V3 B, V3 C, double& wa, double& wb, double& wc) {
  V3 ab = sub3(B, A), ac = sub3(C, A), ap = sub3(P, A);
  double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  if (d1 <= 0.0 && d2 <= 0.0) { wa = 1.0; wb = 0.0; wc = 0.0; return 0; }
  V3 bp = sub3(P, B);
  double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
  if (d3 >= 0.0 && d4 <= d3) { wa = 0.0; wb = 1.0; wc = 0.0; return 1; }
  double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
    double t = d1 / (d1 - d3);
    wa = 1.0 - t; wb = t; wc = 0.0; return 2;
  }
  V3 cp = sub3(P, C);
  double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) { wa = 0.0; wb = 0.0; wc = 1.0; return 3; }
  double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
    double t = d2 / (d2 - d6);
    wa = 1.0 - t; wb = 0.0; wc = t; return 4;
  }
  double va = d3 * d6 - d5 * d4;
  double e43 = d4 - d3, e56 = d5 - d6;
  if (va <= 0.0 && e43 >= 0.0 && e56 >= 0.0) {
    double t = e43 / (e43 + e56);
    wa = 0.0; wb = 1.0 - t; wc = t; return 5;
  }
  double a = va < 0.0 ? 0.0 : va, b = vb < 0.0 ? 0.0 : vb, c = vc < 0.0 ? 0.0 : vc;
  double s = (a + b) + c;
  if (!(s > 0.0)) { wa = 1.0; wb = 0.0; wc = 0.0; return 6; }
  wa = a / s; wb = b / s; wc = c / s;
  return 6;
}

// Candidate triangles of each coarse point c: the pairs (j, k) of its sorted
// neighbour list, positions e1 < e2, with {j, k} a coarse edge and (c, j, k)
// not degenerate, in ascending (e1, e2) -- the candidates, in order, that the
// projection of every fine point of c's cell visits.  kTriLanes lanes per
// coarse point, a pair per lane; tcnt[c] = -1 when there are more than kTriMax.
constexpr int kTriMax = 32;
constexpr int kTriLanes = 16;

__global__ void __launch_bounds__(kBlock) k_tri_candidates(const double* __restrict__ Xc,
                                                           const int32_t* __restrict__ crp,
                                                           const int32_t* __restrict__ ccol, int64_t nc,
                                                           int32_t* __restrict__ tlist, int32_t* __restrict__ tcnt) {
  const int64_t c = (int64_t)blockIdx.x * (kBlock / kTriLanes) + threadIdx.x / kTriLanes;
  const int sub = threadIdx.x & (kTriLanes - 1);
  const int gbase = (threadIdx.x & (kWave - 1)) & ~(kTriLanes - 1);   // the group's first lane in the wavefront
  const bool act = c < nc;
  const int32_t rb = act ? crp[c] : 0, d = act ? crp[c + 1] - rb : 0;
  const int32_t np = d * (d - 1) / 2;
  // trip count uniform over the wavefront: the largest pair count of its groups
  int32_t npw = np;
  for (int o = kTriLanes; o < kWave; o <<= 1) npw = max(npw, __shfl_xor(npw, o, kWave));
  const V3 A = act ? ld3(Xc, c) : V3{0.0, 0.0, 0.0};
  int32_t cnt = 0;
  for (int32_t p0 = 0; p0 < npw; p0 += kTriLanes) {
    const int32_t p = p0 + sub;
    bool ok = false;
    int32_t j = 0, k = 0;
    if (p < np) {
      int32_t e1 = 0, off = 0;                           // pair p -> (e1, e2) in lexicographic order
      while (off + (d - 1 - e1) <= p) {
        off += d - 1 - e1;
        ++e1;
      }
      const int32_t e2 = e1 + 1 + (p - off);
      j = ccol[rb + e1];
      k = ccol[rb + e2];
      if (has_edge(crp, ccol, j, k)) ok = !degenerate(A, ld3(Xc, j), ld3(Xc, k));
    }
    const unsigned long long m = (__ballot(ok) >> gbase) & ((1ull << kTriLanes) - 1ull);
    if (ok) {
      const int32_t pos = cnt + __popcll(m & ((1ull << sub) - 1ull));
      if (pos < kTriMax) {
        tlist[(c * kTriMax + pos) * 2] = j;
        tlist[(c * kTriMax + pos) * 2 + 1] = k;
      }
    }
    cnt += __popcll(m);
  }
  if (act && sub == 0) tcnt[c] = cnt <= kTriMax ? cnt : -1;
}

// One thread per fine point p; c = label(p) is the coarse point closest to p.
// Candidates are the triangles (c, j, k), j < k neighbours of c with {j, k} a
// coarse edge, visited in ascending (j, k); the first candidate at the
// smallest point-to-triangle distance is kept.  With no non-degenerate
// candidate, the three points of {c} U N(c) nearest to p (ties by index) get
// inverse-distance weights.  The row keeps its non-zero weights sorted by
// column.
// Variants (weighting ablation): the chosen triangle's vertices (c, j, k) get
// uniform weights 1/3, or inverse-distance weights 1/|p - X_t| normalised by
// their sum (c, j, k order; a vertex at distance 0 takes weight 1).  With
// fallback_on_vertex, a best projection onto a vertex goes to the fallback.
__global__ void __launch_bounds__(kBlock) k_project(const double* X, const int32_t* lab, int64_t n,
                                                    const double* Xc, const int32_t* crp, const int32_t* ccol,
                                                    int32_t weighting, int32_t fallback_on_vertex,
                                                    int32_t* pcol, double* pval, int32_t* pcnt, int32_t* tri,
                                                    unsigned long long* fallback, const int32_t* tlist,
                                                    const int32_t* tcnt) {
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
    int breg = -1;
    // a candidate (c, j, k); the first at the smallest distance is kept
    auto consider = [&](int32_t j, int32_t k, V3 B, V3 C) {
      double w0, w1, w2;
      const int reg = closest_point(P, A, B, C, w0, w1, w2);
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
        breg = reg;
      }
    };
    const int32_t nt = tcnt[c];
    if (nt >= 0) {
      // the cell's listed candidates, kTriChunk at a time with their loads together
      constexpr int kTriChunk = 4;
      for (int32_t t0 = 0; t0 < nt; t0 += kTriChunk) {
        int32_t jj[kTriChunk], kk[kTriChunk];
        V3 B[kTriChunk], C[kTriChunk];
#pragma unroll
        for (int u = 0; u < kTriChunk; ++u) {
          const int64_t o = ((int64_t)c * kTriMax + min(t0 + u, nt - 1)) * 2;
          jj[u] = tlist[o];
          kk[u] = tlist[o + 1];
        }
#pragma unroll
        for (int u = 0; u < kTriChunk; ++u) {
          B[u] = ld3(Xc, jj[u]);
          C[u] = ld3(Xc, kk[u]);
        }
#pragma unroll
        for (int u = 0; u < kTriChunk; ++u)
          if (t0 + u < nt) consider(jj[u], kk[u], B[u], C[u]);
      }
    } else {
      for (int32_t e1 = rb; e1 < re; ++e1) {
        int32_t j = ccol[e1];
        V3 B = ld3(Xc, j);
        for (int32_t e2 = e1 + 1; e2 < re; ++e2) {
          int32_t k = ccol[e2];
          if (!has_edge(crp, ccol, j, k)) continue;
          V3 C = ld3(Xc, k);
          if (degenerate(A, B, C)) continue;
          consider(j, k, B, C);
        }
      }
    }
    if (found && fallback_on_vertex && (breg == kRegionA || breg == kRegionB || breg == kRegionC)) found = false;
    int32_t cols[3];
    double vals[3];
    int cnt;
    if (found) {
      cols[0] = c; cols[1] = bj; cols[2] = bk;
      vals[0] = bw0; vals[1] = bw1; vals[2] = bw2;
      if (weighting == 1) {
        vals[0] = vals[1] = vals[2] = 1.0 / 3.0;
      } else if (weighting == 2) {
        const V3 T[3] = {A, ld3(Xc, bj), ld3(Xc, bk)};
        double dd[3];
        int zero = -1;
        for (int t = 0; t < 3; ++t) {
          const V3 d = sub3(P, T[t]);
          dd[t] = sqrt(dot3(d, d));
          if (dd[t] == 0.0 && zero < 0) zero = t;
        }
        if (zero >= 0) {
          for (int t = 0; t < 3; ++t) vals[t] = t == zero ? 1.0 : 0.0;
        } else {
          const double i0 = 1.0 / dd[0], i1 = 1.0 / dd[1], i2 = 1.0 / dd[2];
          const double sum = (i0 + i1) + i2;
          vals[0] = i0 / sum;
          vals[1] = i1 / sum;
          vals[2] = i2 / sum;
        }
      }
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
__global__ void k_store_total(const int32_t* total, unsigned long long* out) { *out = (unsigned long long)*total; }

// Entries per column of P; the count a column had before entry (i, t) is that
// entry's slot in row I of P^T (slot[3 i + t]).
// Entries of every column of P, with a slot for each entry (one atomic per run
// of equal columns over consecutive rows: neighbouring fine points mostly
// share their triangle).
__global__ void k_count_cols(const int32_t* pcol, const int32_t* pcnt, int64_t n, int32_t* cnt, int32_t* slot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = i < n ? pcnt[i] : 0;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const bool on = t < c;
    const int32_t k = run_add(cnt, on ? pcol[3 * i + t] : -1, on);
    if (on) slot[3 * i + t] = k;
  }
}

// P^T entries at the slots the count handed out (each row is sorted by fine
// index afterwards).
__global__ void k_scatter_cols(const int32_t* __restrict__ pcol, const double* __restrict__ pval,
                               const int32_t* __restrict__ pcnt, int64_t n, const int32_t* __restrict__ ptr,
                               const int32_t* __restrict__ slot, int32_t* __restrict__ tcol,
                               double* __restrict__ tval) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = pcnt[i];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (t >= c) break;
    const int32_t pos = ptr[pcol[3 * i + t]] + slot[3 * i + t];
    tcol[pos] = (int32_t)i;
    tval[pos] = pval[3 * i + t];
  }
}

// Rows of P^T sorted by fine index: one wavefront per row, a bitonic sort of
// (index, value) pairs across the 64 lanes; longer rows (rare) fall back to
// an insertion sort by the first lane.
__global__ void __launch_bounds__(kBlock) k_sort_pairs(const int32_t* ptr, int32_t* col, double* val,
                                                       int64_t nrow) {
  const int64_t I = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (I >= nrow) return;
  const int32_t b = ptr[I], e = ptr[I + 1], len = e - b;
  if (len <= kWave) {
    int32_t key = lane < len ? col[b + lane] : INT32_MAX;
    double v = lane < len ? val[b + lane] : 0.0;
    for (int k = 2; k <= kWave; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) {
        const int32_t ok = __shfl_xor(key, j, kWave);
        const double ov = __shfl_xor(v, j, kWave);
        const bool up = (lane & k) == 0, lower = (lane & j) == 0;
        const bool take = lower ? (up ? ok < key : ok > key) : (up ? ok > key : ok < key);
        if (take) {
          key = ok;
          v = ov;
        }
      }
    if (lane < len) {
      col[b + lane] = key;
      val[b + lane] = v;
    }
  } else if (lane == 0) {
    for (int32_t i = b + 1; i < e; ++i) {
      int32_t c = col[i];
      double w = val[i];
      int32_t j = i - 1;
      while (j >= b && col[j] > c) {
        col[j + 1] = col[j];
        val[j + 1] = val[j];
        --j;
      }
      col[j + 1] = c;
      val[j + 1] = w;
    }
  }
}

// ------------------------------------------------------------------ Galerkin (Alg. 1)
// One wavefront per coarse row I.  The terms of row I are
//   (P[i,I] * A[i,j]) * P[j,J]  for i in row I of P^T (ascending), j in row i
// of A (CSR order), J in row j of P (column order).
// The (i, j) pairs of a row are enumerated 64 at a time (one per lane, after
// a wavefront prefix sum over the row lengths), so a row's dependent loads
// are issued for 64 pairs at once.
// Symbolic pass: the distinct J go into an LDS hash set.  Numeric pass: for
// every 64 pairs the lane that owns output column J adds the terms of J of
// those pairs in pair order, so each entry is summed exactly like the
// definition's row accumulation.

// Inclusive scan of one int per lane over a wavefront.
__device__ inline int wave_incl_scan(int v) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(v, o, kWave);
    if (lane >= o) v += t;
  }
  return v;
}

template <int HS>
__device__ inline bool hash_insert(int32_t* keys, int32_t J) {
  uint32_t h = ((uint32_t)J * 2654435761u) & (HS - 1);
  for (int probe = 0; probe < HS; ++probe) {
    int32_t old = atomicCAS(&keys[h], -1, J);
    if (old == -1 || old == J) return true;
    h = (h + 1) & (HS - 1);
  }
  return false;
}

struct PairChunk {
  int32_t pre[kWave];                  // exclusive prefix of A-row lengths over a chunk of P^T entries
  int32_t rb[kWave];                   // first A entry of that row
  double piI[kWave];                   // P[i, I]
};

// Loads P^T entries [q0, q0 + 64) of row I and returns the number of (i, j) pairs.
__device__ inline int load_pairs(int32_t q0, int32_t qe, const int32_t* tcol, const double* tval,
                                 const int32_t* arp, PairChunk& pc) {
  const int lane = threadIdx.x;
  const int32_t q = q0 + lane;
  const bool on = q < qe;
  const int32_t i = on ? tcol[q] : 0;
  const int32_t rb = on ? arp[i] : 0;
  const int32_t rl = on ? arp[i + 1] - rb : 0;
  const int incl = wave_incl_scan(rl);
  pc.pre[lane] = incl - rl;
  pc.rb[lane] = rb;
  pc.piI[lane] = on ? tval[q] : 0.0;
  __syncthreads();
  return __shfl(incl, kWave - 1, kWave);
}

// Pair p of the chunk -> (P^T entry index within the chunk, A entry index)
__device__ inline void locate_pair(const PairChunk& pc, int p, int& src, int32_t& e) {
  int lo = 0, hi = kWave;                           // last src with pre[src] <= p
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (pc.pre[mid] <= p) lo = mid; else hi = mid;
  }
  src = lo;
  e = pc.rb[lo] + (p - pc.pre[lo]);
}

template <int HS>
__global__ void __launch_bounds__(kWave) k_galerkin_count(const int32_t* trp, const int32_t* tcol,
                                                          const double* tval, const int32_t* arp,
                                                          const int32_t* acol, const int32_t* pcol,
                                                          const int32_t* pcnt, int64_t nc, int32_t* rowcnt,
                                                          int32_t* flags) {
  __shared__ int32_t keys[HS];
  __shared__ PairChunk pc;
  const int32_t I = (int32_t)xcd_block();        // neighbouring rows share an XCD
  if (I >= nc) return;
  const int lane = threadIdx.x;
  for (int s = lane; s < HS; s += kWave) keys[s] = -1;
  __syncthreads();
  bool ok = true;
  // one chunk of P^T entries and at most kFastSub * 64 pairs: every lane's
  // pairs gathered together (as in the numeric pass); otherwise chunk by chunk
  constexpr int kFastSub = 4;
  const int32_t qb = trp[I], qe = trp[I + 1];
  const int tot1 = qe - qb <= kWave ? load_pairs(qb, qe, tcol, tval, arp, pc) : kFastSub * kWave + 1;
  if (tot1 <= kFastSub * kWave) {                                    // uniform over the wavefront
    int32_t fe[kFastSub], fj[kFastSub], fJ[kFastSub][3];
    int fc[kFastSub];
#pragma unroll
    for (int u = 0; u < kFastSub; ++u) {
      int src = 0;
      fe[u] = 0;
      if (lane + u * kWave < tot1) locate_pair(pc, lane + u * kWave, src, fe[u]);
    }
#pragma unroll
    for (int u = 0; u < kFastSub; ++u) fj[u] = lane + u * kWave < tot1 ? acol[fe[u]] : 0;
#pragma unroll
    for (int u = 0; u < kFastSub; ++u) {
      fc[u] = lane + u * kWave < tot1 ? pcnt[fj[u]] : 0;
#pragma unroll
      for (int t = 0; t < 3; ++t) fJ[u][t] = pcol[3 * fj[u] + t];
    }
#pragma unroll
    for (int u = 0; u < kFastSub; ++u)
#pragma unroll
      for (int t = 0; t < 3; ++t)
        if (t < fc[u]) ok &= hash_insert<HS>(keys, fJ[u][t]);
    __syncthreads();
  } else {
    for (int32_t q0 = qb; q0 < qe; q0 += kWave) {
      const int tot = load_pairs(q0, qe, tcol, tval, arp, pc);
      for (int p0 = 0; p0 < tot; p0 += kWave) {
        const int p = p0 + lane;
        if (p < tot) {
          int src;
          int32_t e;
          locate_pair(pc, p, src, e);
          const int32_t j = acol[e];
          const int c = pcnt[j];
          for (int t = 0; t < c; ++t) ok &= hash_insert<HS>(keys, pcol[3 * j + t]);
        }
      }
      __syncthreads();
    }
  }
  int c = 0;
  for (int s = lane; s < HS; s += kWave) c += keys[s] >= 0;
  c = wave_sum(c);
  bool bad = __ballot(!ok) != 0;
  if (lane == 0) {
    rowcnt[I] = c;
    if (bad || c > HS * 3 / 4) atomicOr(flags, F_OVERFLOW);
  }
}

template <int HS>
__global__ void __launch_bounds__(kWave) k_galerkin_fill(const int32_t* trp, const int32_t* tcol,
                                                         const double* tval, const int32_t* arp,
                                                         const int32_t* acol, const double* aval,
                                                         const int32_t* pcol, const double* pval,
                                                         const int32_t* pcnt, int64_t nc, const int32_t* crp,
                                                         int32_t* ccol, double* cval, int32_t* flags,
                                                         int32_t* rowcnt, int32_t* unfit) {
  // Row I goes to crp[I] (the symbolic pass counted it and checked the bound),
  // or, with crp null, to I * kOut of padded rows with its length in rowcnt[I];
  // a row with more than kOut columns then sets *unfit and is left out.
  constexpr int kOut = HS * 3 / 4;     // distinct columns of a row
  constexpr int kFastSub = 4;          // pairs per lane of the one-chunk form
  constexpr int kPer = (kOut + kWave - 1) / kWave;   // output columns per lane
  __shared__ int32_t keys[HS];
  __shared__ int32_t rank_of[HS];      // hash slot -> position of its column in the sorted row
  __shared__ int32_t sorted[kOut];
  __shared__ double accum[kOut];
  __shared__ unsigned long long hits[kOut];   // per output column: the pairs of the chunk that add to it
  __shared__ int32_t tR[3 * kWave];    // per pair of the chunk: output position of each term (-1: none)
  __shared__ double tV[3 * kWave];     // and its value
  __shared__ PairChunk pc;
  __shared__ int32_t nlist;
  const int32_t I = (int32_t)xcd_block();        // neighbouring rows share an XCD
  if (I >= nc) return;
  const int lane = threadIdx.x;
  // distinct columns (the symbolic pass guaranteed they fit)
  for (int s = lane; s < HS; s += kWave) keys[s] = -1;
  if (lane == 0) nlist = 0;
  __syncthreads();
  // Rows with one chunk of P^T entries and at most kFastSub * 64 pairs keep
  // the chunk and each lane's pairs (pair lane + 64 s) in registers for both
  // passes, with every gather of a pass issued together; other rows reload
  // them chunk by chunk.
  const int32_t qb = trp[I], qe = trp[I + 1];
  int tot = qe - qb <= kWave ? load_pairs(qb, qe, tcol, tval, arp, pc) : kFastSub * kWave + 1;
  const bool fast = tot <= kFastSub * kWave;                        // uniform over the wavefront
  int fsrc[kFastSub], fc[kFastSub];
  int32_t fe[kFastSub], fj[kFastSub], fJ[kFastSub][3];
  if (fast) {
#pragma unroll
    for (int u = 0; u < kFastSub; ++u) {
      fsrc[u] = 0;
      fe[u] = 0;
      if (lane + u * kWave < tot) locate_pair(pc, lane + u * kWave, fsrc[u], fe[u]);
    }
#pragma unroll
    for (int u = 0; u < kFastSub; ++u) fj[u] = lane + u * kWave < tot ? acol[fe[u]] : 0;
#pragma unroll
    for (int u = 0; u < kFastSub; ++u) {
      fc[u] = lane + u * kWave < tot ? pcnt[fj[u]] : 0;
#pragma unroll
      for (int t = 0; t < 3; ++t) fJ[u][t] = pcol[3 * fj[u] + t];
    }
#pragma unroll
    for (int u = 0; u < kFastSub; ++u)
#pragma unroll
      for (int t = 0; t < 3; ++t)
        if (t < fc[u]) hash_insert<HS>(keys, fJ[u][t]);
    __syncthreads();
  } else {
    for (int32_t q0 = qb; q0 < qe; q0 += kWave) {
      const int tc = load_pairs(q0, qe, tcol, tval, arp, pc);
      for (int p0 = 0; p0 < tc; p0 += kWave) {
        const int p = p0 + lane;
        if (p < tc) {
          int src;
          int32_t e;
          locate_pair(pc, p, src, e);
          const int32_t j = acol[e];
          for (int t = 0; t < pcnt[j]; ++t) hash_insert<HS>(keys, pcol[3 * j + t]);
        }
      }
      __syncthreads();
    }
  }
  for (int s = lane; s < HS; s += kWave)
    if (keys[s] >= 0) {                                             // slots, in any order
      const int a = atomicAdd(&nlist, 1);
      if (a < kOut) sorted[a] = s;
    }
  __syncthreads();
  const int k = nlist;
  if (k > kOut) {                                                   // uniform over the wavefront
    if (lane == 0) {
      if (unfit) atomicOr(unfit, 1);
      if (rowcnt) rowcnt[I] = 0;
    }
    return;
  }
  int32_t myslot[kPer], mykey[kPer];
#pragma unroll
  for (int g = 0; g < kPer; ++g) {
    const int a = lane + g * kWave;
    myslot[g] = a < k ? sorted[a] : -1;
    mykey[g] = a < k ? keys[myslot[g]] : 0;
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < kPer; ++g)
    if (lane + g * kWave < k) {
      int rank = 0;
      for (int b = 0; b < k; ++b) rank += keys[sorted[b]] < mykey[g];
      rank_of[myslot[g]] = rank;
    }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < kPer; ++g)
    if (lane + g * kWave < k) {
      sorted[rank_of[myslot[g]]] = mykey[g];
      accum[rank_of[myslot[g]]] = 0.0;
    }
  __syncthreads();
  // Numeric pass, 64 (i, j) pairs at a time in definition order.  Each pair
  // adds at most one term to an output column (the columns of a row of P are
  // distinct), so the owner of column o adds the terms of the pairs flagged in
  // hits[o] in ascending pair order: every entry is summed in the order of the
  // definition.
  // The terms of one 64-pair chunk of the one-chunk form: pair lane has c
  // terms (P row of j, t1 = P[i,I] A[i,j] times P[j,J_t]); the owner of each
  // output column adds them in pair order.  (The general form below does the
  // same with its loads inline.)
  auto add_chunk = [&](int c, const int32_t* J, const double* v) {
    for (int o = lane; o < k; o += kWave) hits[o] = 0ull;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      int32_t r = -1;
      if (t < c) {
        uint32_t h = ((uint32_t)J[t] * 2654435761u) & (HS - 1);
        while (keys[h] != J[t]) h = (h + 1) & (HS - 1);
        r = rank_of[h];
      }
      tR[3 * lane + t] = r;
      tV[3 * lane + t] = t < c ? v[t] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (t < c) atomicOr(&hits[tR[3 * lane + t]], 1ull << lane);
    __syncthreads();
    for (int o = lane; o < k; o += kWave) {
      unsigned long long m = hits[o];
      double acc = accum[o];
      while (m) {
        const int q = __builtin_ctzll(m);
        m &= m - 1;
        const int t = tR[3 * q] == o ? 0 : (tR[3 * q + 1] == o ? 1 : 2);
        acc = acc + tV[3 * q + t];
      }
      accum[o] = acc;
    }
    __syncthreads();
  };
  if (fast) {
    double fa[kFastSub], fp[kFastSub][3];
#pragma unroll
    for (int u = 0; u < kFastSub; ++u) {
      fa[u] = aval[fe[u]];
#pragma unroll
      for (int t = 0; t < 3; ++t) fp[u][t] = pval[3 * fj[u] + t];
    }
#pragma unroll
    for (int u = 0; u < kFastSub; ++u) {
      if (u * kWave >= tot) break;                                   // uniform
      const double t1 = pc.piI[fsrc[u]] * fa[u];
      double v[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) v[t] = t1 * fp[u][t];
      add_chunk(fc[u], fJ[u], v);
    }
  } else {
    for (int32_t q0 = qb; q0 < qe; q0 += kWave) {
      const int tc = load_pairs(q0, qe, tcol, tval, arp, pc);
      for (int p0 = 0; p0 < tc; p0 += kWave) {
        const int p = p0 + lane;
        const bool on = p < tc;
        int32_t j = 0;
        int c = 0;
        double t1 = 0.0;
        if (on) {
          int src;
          int32_t e;
          locate_pair(pc, p, src, e);
          j = acol[e];
          c = pcnt[j];
          t1 = pc.piI[src] * aval[e];
        }
        for (int o = lane; o < k; o += kWave) hits[o] = 0ull;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          int32_t r = -1;
          double v = 0.0;
          if (t < c) {
            const int32_t J = pcol[3 * j + t];
            uint32_t h = ((uint32_t)J * 2654435761u) & (HS - 1);
            while (keys[h] != J) h = (h + 1) & (HS - 1);
            r = rank_of[h];
            v = t1 * pval[3 * j + t];
          }
          tR[3 * lane + t] = r;
          tV[3 * lane + t] = v;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 3; ++t)
          if (t < c) atomicOr(&hits[tR[3 * lane + t]], 1ull << lane);
        __syncthreads();
        for (int o = lane; o < k; o += kWave) {
          unsigned long long m = hits[o];
          double acc = accum[o];
          while (m) {
            const int q = __builtin_ctzll(m);
            m &= m - 1;
            const int t = tR[3 * q] == o ? 0 : (tR[3 * q + 1] == o ? 1 : 2);
            acc = acc + tV[3 * q + t];
          }
          accum[o] = acc;
        }
        __syncthreads();
      }
    }
  }
  const int64_t out = crp ? (int64_t)crp[I] : (int64_t)I * kOut;
  if (rowcnt && lane == 0) rowcnt[I] = k;
  bool diag_ok = false;
  for (int o = lane; o < k; o += kWave) {
    ccol[out + o] = sorted[o];
    cval[out + o] = accum[o];
    if (sorted[o] == I && accum[o] > 0.0) diag_ok = true;
  }
  // a missing or non-positive diagonal makes Gauss-Seidel divide by zero
  unsigned long long bal = __ballot(diag_ok);
  if (lane == 0 && bal == 0) atomicOr(flags, F_NOT_SPD);
}

// Padded rows (stride W) of the first numeric pass into their CSR place, a
// wavefront per row.
__global__ void __launch_bounds__(kBlock) k_galerkin_compact(const int32_t* __restrict__ rowcnt,
                                                             const int32_t* __restrict__ rp,
                                                             const int32_t* __restrict__ pcol,
                                                             const double* __restrict__ pval, int64_t nc, int32_t W,
                                                             int32_t* __restrict__ col, double* __restrict__ val) {
  const int64_t I = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (I >= nc) return;
  const int32_t n = rowcnt[I], o = rp[I];
  for (int32_t t = threadIdx.x & (kWave - 1); t < n; t += kWave) {
    col[o + t] = pcol[I * W + t];
    val[o + t] = pval[I * W + t];
  }
}

__global__ void __launch_bounds__(kBlock) k_max_i32(const int32_t* v, int64_t n, int32_t* out) {
  int32_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    m = v[i] > m ? v[i] : m;
  m = block_reduce(m, [](int32_t a, int32_t b) { return a > b ? a : b; });
  if (threadIdx.x == 0 && m) atomicMax(out, m);
}

}  // namespace

void prolongation(Handle& h, Level& lv, Level& nx) {
  hipStream_t s = h.stream;
  int64_t n = lv.n;
  lv.pcol = (int32_t*)dalloc(h, (size_t)3 * n * 4);
  lv.pval = (double*)dalloc(h, (size_t)3 * n * 8);
  lv.pcnt = (int32_t*)dalloc(h, (size_t)n * 4);
  lv.tri = (int32_t*)dalloc(h, (size_t)2 * n * 4);
  const int64_t nc = nx.n;
  int32_t* tlist = (int32_t*)talloc(s, (size_t)nc * kTriMax * 2 * 4);
  int32_t* tcnt = (int32_t*)talloc(s, (size_t)nc * 4);
  k_tri_candidates<<<blocks_for(nc, kBlock / kTriLanes), kBlock, 0, s>>>(nx.X, nx.erp, nx.ecol, nc, tlist, tcnt);
  k_project<<<blocks_for(n), kBlock, 0, s>>>(lv.X, lv.label, n, nx.X, nx.erp, nx.ecol, h.opt.weighting,
                                             h.opt.fallback_on_vertex, lv.pcol, lv.pval, lv.pcnt, lv.tri,
                                             lv.stats, tlist, tcnt);
  tfree(s, tlist);
  tfree(s, tcnt);
}

void transpose_p(Handle& h, Level& lv, int64_t nc, int32_t** t_rp, int32_t** t_col, double** t_val) {
  hipStream_t s = h.stream;
  int64_t n = lv.n;
  int32_t* cnt = (int32_t*)talloc(s, (size_t)(nc + 1) * 4);
  int32_t* slot = (int32_t*)talloc(s, (size_t)3 * n * 4);
  int32_t* rp = (int32_t*)dalloc(h, (size_t)(nc + 1) * 4);   // kept by the handle
  check_hip(hipMemsetAsync(cnt, 0, (size_t)(nc + 1) * 4, s), "memset");
  k_count_cols<<<blocks_for(n), kBlock, 0, s>>>(lv.pcol, lv.pcnt, n, cnt, slot);
  scan_i32(cnt, rp, nc, s);
  k_store_total<<<1, 1, 0, s>>>(rp + nc, lv.stats + 1);      // nnz(P), read at the end of the build
  int32_t* col = (int32_t*)dalloc(h, (size_t)(3 * n + 1) * 4);   // nnz(P) <= 3n
  double* val = (double*)dalloc(h, (size_t)(3 * n + 1) * 8);
  k_scatter_cols<<<blocks_for(n), kBlock, 0, s>>>(lv.pcol, lv.pval, lv.pcnt, n, rp, slot, col, val);
  k_sort_pairs<<<blocks_for(nc, kBlock / kWave), kBlock, 0, s>>>(rp, col, val, nc);
  tfree(s, cnt);
  tfree(s, slot);
  *t_rp = rp;
  *t_col = col;
  *t_val = val;
}

void galerkin(Handle& h, Level& lv, Level& nx, const int32_t* t_rp, const int32_t* t_col,
              const double* t_val) {
  hipStream_t s = h.stream;
  int64_t nc = nx.n;
  lv.t_rp = (int32_t*)t_rp;
  lv.t_col = (int32_t*)t_col;
  lv.t_val = (double*)t_val;
  // First the numeric pass into padded rows of up to 48 columns (the smallest
  // hash table); its rows then only move into place.  If a row has more
  // columns, the symbolic pass sizes the rows and the numeric pass runs again.
  {
    constexpr int32_t W = 64 * 3 / 4;
    int32_t* cnt = (int32_t*)talloc(s, (size_t)(nc + 1) * 4);
    int32_t* unfit = (int32_t*)talloc(s, 4);
    int32_t* pcol = (int32_t*)talloc(s, (size_t)nc * W * 4);
    double* pval = (double*)talloc(s, (size_t)nc * W * 8);
    fill_i32(unfit, 0, 1, s);
    nx.arp = (int32_t*)dalloc(h, (size_t)(nc + 1) * 4);
    k_galerkin_fill<64><<<(int)nc, kWave, 0, s>>>(t_rp, t_col, t_val, lv.arp, lv.acol, lv.aval, lv.pcol, lv.pval,
                                                  lv.pcnt, nc, nullptr, pcol, pval, h.flags, cnt, unfit);
    scan_i32(cnt, nx.arp, nc, s);
    int64_t bad = 0, f = 0;
    ScalarRead rd[3] = {{nx.arp + nc, 4, &nx.nnzA}, {unfit, 4, &bad}, {h.flags, 4, &f}};
    read_scalars(h, rd, 3);
    if (bad == 0) {
      throw_flags((int32_t)f, "Galerkin operator");
      nx.acol = (int32_t*)dalloc(h, (size_t)(nx.nnzA + 1) * 4);
      nx.aval = (double*)dalloc(h, (size_t)(nx.nnzA + 1) * 8);
      k_galerkin_compact<<<blocks_for(nc, kBlock / kWave), kBlock, 0, s>>>(cnt, nx.arp, pcol, pval, nc, W, nx.acol,
                                                                          nx.aval);
      lv.galerkin_hs = 64;
    }
    tfree(s, pcol);
    tfree(s, pval);
    tfree(s, unfit);
    tfree(s, cnt);
    if (bad == 0) return;
  }
  int32_t* cnt = (int32_t*)talloc(s, (size_t)(nc + 1) * 4);
  int32_t* mx = (int32_t*)talloc(s, 4);
  check_hip(hipMemsetAsync(mx, 0, 4, s), "memset");
  k_galerkin_count<1024><<<(int)nc, kWave, 0, s>>>(t_rp, t_col, t_val, lv.arp, lv.acol, lv.pcol, lv.pcnt, nc,
                                                  cnt, h.flags);
  k_max_i32<<<std::min(blocks_for(nc), kReduceGrid), kBlock, 0, s>>>(cnt, nc, mx);
  scan_i32(cnt, nx.arp, nc, s);
  int64_t maxrow = 0, f = 0;
  ScalarRead rd[3] = {{nx.arp + nc, 4, &nx.nnzA}, {mx, 4, &maxrow}, {h.flags, 4, &f}};
  read_scalars(h, rd, 3);
  throw_flags((int32_t)f, "Galerkin operator");
  nx.acol = (int32_t*)dalloc(h, (size_t)(nx.nnzA + 1) * 4);
  nx.aval = (double*)dalloc(h, (size_t)(nx.nnzA + 1) * 8);
  // the smallest hash table that holds every row (3/4 full at most): a
  // smaller LDS footprint keeps more rows in flight per CU
  lv.galerkin_hs = maxrow <= 64 * 3 / 4 ? 64 : (maxrow <= 256 * 3 / 4 ? 256 : 1024);
  galerkin_values(h, lv, nx);
  tfree(s, cnt);
  tfree(s, mx);
}

// The numeric pass alone: the pattern it writes is the one already there.
void galerkin_values(Handle& h, Level& lv, Level& nx) {
  hipStream_t s = h.stream;
  const int64_t nc = nx.n;
  auto fill = [&](auto kern) {
    kern<<<(int)nc, kWave, 0, s>>>(lv.t_rp, lv.t_col, lv.t_val, lv.arp, lv.acol, lv.aval, lv.pcol, lv.pval, lv.pcnt,
                                   nc, nx.arp, nx.acol, nx.aval, h.flags, nullptr, nullptr);
  };
  if (lv.galerkin_hs == 64) fill(k_galerkin_fill<64>);
  else if (lv.galerkin_hs == 256) fill(k_galerkin_fill<256>);
  else fill(k_galerkin_fill<1024>);
}

}  // namespace gmg
