// Hierarchy construction, graph part (Sec. 4.1-4.3): input canonicalisation,
// edge lengths and the sampling radius (Eq. 1), the greedy sampling sweep as a
// lexicographically-first maximal independent set, graph Voronoi cells by
// parallel Bellman-Ford, coarse positions (cell means) and Voronoi-neighbour
// edges.
//
// Every floating-point decision repeats the exact IEEE binary64 operation
// sequence of the method's definition (no contraction: built with
// -ffp-contract=off), so samples, labels and coarse edges are reproducible bit
// for bit by any correct implementation.
#include <algorithm>

#include "gmg_internal.hpp"

namespace gmg {

namespace {

// ------------------------------------------------------------------ validation
__global__ void k_validate_points(const double* X, int64_t n3, int32_t* flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3 && !isfinite(X[i])) atomicOr(flags, F_INVALID);
}

// Degrees of the edge list's end points; the count each end point had before
// this edge is the edge's slot in that end point's row (slot[2e], slot[2e+1]).
__global__ void k_edge_degree(const int32_t* edges, int64_t m, int64_t n, int32_t* deg, int32_t* slot,
                              int32_t* flags) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = e < m;
  const int32_t u = in ? edges[2 * e] : 0, v = in ? edges[2 * e + 1] : 0;
  const bool bad = in && (u < 0 || v < 0 || u >= n || v >= n);
  if (bad) atomicOr(flags, F_INVALID);
  const bool on = in && !bad && u != v;
  // one atomic per run of equal endpoints (edges are often listed vertex by vertex)
  const int32_t su = run_add(deg, on ? u : -1, on);
  const int32_t sv = run_add(deg, on ? v : -1, on);
  if (on) {
    slot[2 * e] = su;
    slot[2 * e + 1] = sv;
  }
}

// Row entries at the slots the degree count handed out (rows are sorted
// afterwards, so the order of the slots does not matter).
__global__ void k_edge_scatter(const int32_t* __restrict__ edges, int64_t m, int64_t n,
                               const int32_t* __restrict__ ptr, const int32_t* __restrict__ slot,
                               int32_t* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  int32_t u = edges[2 * e], v = edges[2 * e + 1];
  if (u < 0 || v < 0 || u >= n || v >= n || u == v) return;
  out[ptr[u] + slot[2 * e]] = v;
  out[ptr[v] + slot[2 * e + 1]] = u;
}

// Row i of the system matrix: valid offsets, strictly ascending in-range
// columns, finite values, diagonal present and positive, symmetric pattern.
// Per row: offsets in range, columns in range and strictly ascending, values
// finite, a positive diagonal, and every entry (i, j) matched by (j, i) (a
// binary search in row j).  The row's entries are checked kValidChunk at a
// time with their loads and search steps in flight together; the flags do not
// depend on the order of the checks.
constexpr int kValidChunk = 8;

__global__ void k_validate_matrix(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                  const double* __restrict__ val, int64_t n, int64_t nnz, int32_t* flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicOr(flags, F_INVALID);
  if (i >= n) return;
  int32_t b = rp[i], e = rp[i + 1];
  if (b < 0 || e < b || e > nnz) {
    atomicOr(flags, F_INVALID);
    return;
  }
  bool diag = false, bad = false, notspd = false;
  for (int32_t k0 = b; k0 < e; k0 += kValidChunk) {
    int32_t j[kValidChunk], jprev[kValidChunk], lo[kValidChunk], hi[kValidChunk];
    double v[kValidChunk];
    bool on[kValidChunk];
#pragma unroll
    for (int q = 0; q < kValidChunk; ++q) {
      const int32_t k = min(k0 + q, e - 1);
      on[q] = k0 + q < e;
      j[q] = col[k];
      jprev[q] = k > b ? col[k - 1] : -1;
      v[q] = val[k];
    }
#pragma unroll
    for (int q = 0; q < kValidChunk; ++q) {
      const bool jok = j[q] >= 0 && j[q] < n;
      if (on[q] && (!jok || (k0 + q > b && j[q] <= jprev[q]) || !isfinite(v[q]))) bad = true;
      if (on[q] && j[q] == i) {
        diag = true;
        if (!(v[q] > 0.0)) notspd = true;
      }
      lo[q] = 0;
      hi[q] = 0;
      if (on[q] && jok) {
        lo[q] = rp[j[q]];
        hi[q] = rp[j[q] + 1];
      }
    }
    int32_t je[kValidChunk];
#pragma unroll
    for (int q = 0; q < kValidChunk; ++q) {
      je[q] = hi[q];
      if (lo[q] < 0 || hi[q] < lo[q] || hi[q] > nnz) {
        bad = true;
        lo[q] = hi[q] = je[q] = 0;
      }
    }
    // binary searches for i in rows j, one step of each per pass
    for (;;) {
      bool more = false;
#pragma unroll
      for (int q = 0; q < kValidChunk; ++q)
        if (lo[q] < hi[q]) {
          const int32_t mid = (lo[q] + hi[q]) >> 1;
          if (col[mid] < i) lo[q] = mid + 1; else hi[q] = mid;
          more = true;
        }
      if (!more) break;
    }
#pragma unroll
    for (int q = 0; q < kValidChunk; ++q)
      if (on[q] && j[q] >= 0 && j[q] < n && (lo[q] >= je[q] || col[lo[q]] != i)) bad = true;
  }
  if (notspd) atomicOr(flags, F_NOT_SPD);
  if (bad || !diag) atomicOr(flags, F_INVALID);
}

// ------------------------------------------------------------------ edge lengths, Eq. (1)
// The row's end points are loaded kEdgeChunk at a time.
constexpr int kEdgeChunk = 8;

__global__ void k_edge_weights(const double* __restrict__ X, const int32_t* __restrict__ rp,
                               const int32_t* __restrict__ col, int64_t n, double* __restrict__ w) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  V3 pu = ld3(X, u);
  const int32_t b = rp[u], e = rp[u + 1];
  for (int32_t e0 = b; e0 < e; e0 += kEdgeChunk) {
    int32_t c[kEdgeChunk];
    V3 pv[kEdgeChunk];
#pragma unroll
    for (int q = 0; q < kEdgeChunk; ++q) c[q] = col[min(e0 + q, e - 1)];
#pragma unroll
    for (int q = 0; q < kEdgeChunk; ++q) pv[q] = ld3(X, c[q]);
#pragma unroll
    for (int q = 0; q < kEdgeChunk; ++q) {
      if (e0 + q >= e) break;
      V3 d = sub3(pu, pv[q]);
      w[e0 + q] = sqrt(dot3(d, d));
    }
  }
}

// Longest undirected edge, as the bit pattern of a non-negative double
// (ordered like the value), combined with an unsigned 64-bit atomic max.
__global__ void k_edge_max(const int32_t* rp, const int32_t* col, const double* w, int64_t n,
                           unsigned long long* maxbits) {
  unsigned long long m = 0;
  for (int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x; u < n; u += (int64_t)gridDim.x * kBlock)
    for (int32_t e = rp[u]; e < rp[u + 1]; ++e)
      if (u < col[e]) {
        unsigned long long b = (unsigned long long)__double_as_longlong(w[e]);
        m = b > m ? b : m;
      }
  m = block_reduce(m, [](unsigned long long a, unsigned long long b) { return a > b ? a : b; });
  if (threadIdx.x == 0 && m) atomicMax(maxbits, m);
}

__device__ inline int fixed_point_shift(double M, int64_t cnt) {
  int ex = 0;
  frexp(M, &ex);
  int lg = 0;
  while ((int64_t(1) << lg) < cnt) ++lg;
  return 62 - ex - lg;
}

// Exact, order-independent sum of the undirected edge lengths in 64-bit fixed
// point: with the longest edge M < 2^e, each length scaled by 2^F,
// F = 62 - e - ceil(log2 m), rounds to an integer below 2^(62 - ceil log2 m).
__global__ void k_edge_fixsum(const int32_t* rp, const int32_t* col, const double* w, int64_t n,
                              const unsigned long long* maxbits, unsigned long long* sum) {
  const int64_t cnt = rp[n] / 2;
  double M = __longlong_as_double((long long)*maxbits);
  if (M == 0.0) return;
  int F = fixed_point_shift(M, cnt);
  long long s = 0;
  for (int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x; u < n; u += (int64_t)gridDim.x * kBlock)
    for (int32_t e = rp[u]; e < rp[u + 1]; ++e)
      if (u < col[e]) s += (long long)rint(ldexp(w[e], F));
  s = block_reduce(s, [](long long a, long long b) { return a + b; });
  if (threadIdx.x == 0 && s) atomicAdd(sum, (unsigned long long)s);
}

__global__ void k_edge_mean_finish(const unsigned long long* maxbits, const unsigned long long* sum,
                                   const int32_t* total, double rho, double* scal) {
  const int64_t cnt = *total / 2;     // undirected edges
  double M = __longlong_as_double((long long)*maxbits);
  if (cnt == 0 || M == 0.0) {
    scal[0] = 0.0;
    scal[1] = 0.0;
    return;
  }
  int F = fixed_point_shift(M, cnt);
  double ehat = ldexp((double)(long long)*sum, -F) / (double)cnt;
  scal[0] = ehat;
  scal[1] = rho * ehat;
}

// ------------------------------------------------------------------ sampling (Sec. 4.2)
// Sweep order key (hashed or index); ties by index.
struct SweepKey {
  uint64_t base;
  bool by_index;
  __device__ uint64_t operator()(int32_t v) const { return by_index ? 0ull : mix64(base ^ (uint64_t)v); }
};

__device__ inline bool key_less(uint64_t ka, int32_t a, uint64_t kb, int32_t b) {
  return ka < kb || (ka == kb && a < b);
}

// One round of the parallel greedy sweep.  An undecided point joins the
// sample set when every point in conflict with it (within path length r over
// at most two edges) that comes earlier in the sweep order is already
// excluded; it is excluded as soon as one of them is a sample.  Decisions are
// final, so statuses are updated in place; the result equals the sequential
// sweep's for any interleaving.  Round 0 visits every point; later rounds
// visit the worklist of points still undecided after the previous round.
// The loads are issued a chunk at a time: kSweepChunk neighbours m of p with
// their row bounds and statuses, then each m's row kSweepChunk entries at a
// time with the statuses of their ends (positions past a row's end re-read
// its last entry and are not counted).
constexpr int kSweepChunk = 8;

__device__ inline bool lfmis_attempt(const int32_t* rp, const int32_t* col, const double* w, double r,
                                     const SweepKey& key, uint8_t* status, int32_t p) {
  const uint64_t kp = key(p);
  bool blocked = false, out = false;
  auto note = [&](uint8_t s) {
    if (s == 1) out = true; else if (s == 0) blocked = true;
  };
  const int32_t b = rp[p], e = rp[p + 1];
  for (int32_t e0 = b; e0 < e && !out; e0 += kSweepChunk) {
    int32_t m[kSweepChunk], mb[kSweepChunk], me[kSweepChunk];
    double wm[kSweepChunk];
    uint8_t sm[kSweepChunk];
#pragma unroll
    for (int k = 0; k < kSweepChunk; ++k) {
      const int32_t i = min(e0 + k, e - 1);
      m[k] = col[i];
      wm[k] = w[i];
    }
#pragma unroll
    for (int k = 0; k < kSweepChunk; ++k) {
      mb[k] = rp[m[k]];
      me[k] = rp[m[k] + 1];
      sm[k] = __atomic_load_n(&status[m[k]], __ATOMIC_RELAXED);
    }
#pragma unroll
    for (int k = 0; k < kSweepChunk; ++k)
      if (e0 + k < e && wm[k] <= r && key_less(key(m[k]), m[k], kp, p)) note(sm[k]);
    for (int k = 0; k < kSweepChunk && e0 + k < e && !out; ++k) {
      for (int32_t f0 = mb[k]; f0 < me[k] && !out; f0 += kSweepChunk) {
        int32_t q[kSweepChunk];
        double wq[kSweepChunk];
        uint8_t sq[kSweepChunk];
#pragma unroll
        for (int t = 0; t < kSweepChunk; ++t) {
          const int32_t i = min(f0 + t, me[k] - 1);
          q[t] = col[i];
          wq[t] = w[i];
        }
#pragma unroll
        for (int t = 0; t < kSweepChunk; ++t) sq[t] = __atomic_load_n(&status[q[t]], __ATOMIC_RELAXED);
#pragma unroll
        for (int t = 0; t < kSweepChunk; ++t)
          if (f0 + t < me[k] && q[t] != p && wm[k] + wq[t] <= r && key_less(key(q[t]), q[t], kp, p)) note(sq[t]);
      }
    }
  }
  if (out) status[p] = 2;
  else if (!blocked) status[p] = 1;
  return !out && blocked;
}

// On levels of up to kListLevel points the first visit of p also records the
// points in conflict with it that come earlier in the sweep (its whole 2-ring
// search, repeats included) in list[p * kConflicts ..], with
// their number in cnt[p] (kConflicts + 1: too many, later visits search
// again); later visits then only read those points' statuses.  (On larger
// levels the first round streams the graph at full bandwidth, and writing the
// lists cost more than the later rounds saved.)
constexpr int kConflicts = 32;
constexpr int64_t kListLevel = 262144;

__device__ inline bool lfmis_first(const int32_t* rp, const int32_t* col, const double* w, double r,
                                   const SweepKey& key, uint8_t* status, int32_t p, int32_t* list, uint8_t* cnt) {
  const uint64_t kp = key(p);
  bool blocked = false, out = false;
  int32_t k = 0;
  int32_t* lp = list + (int64_t)p * kConflicts;
  auto note = [&](int32_t q, uint8_t s) {
    if (s == 1) out = true; else if (s == 0) blocked = true;
    if (k < kConflicts) lp[k] = q;
    ++k;
  };
  // the same chunked search as lfmis_attempt, recording every conflict
  const int32_t b = rp[p], e = rp[p + 1];
  for (int32_t e0 = b; e0 < e; e0 += kSweepChunk) {
    int32_t m[kSweepChunk], mb[kSweepChunk], me[kSweepChunk];
    double wm[kSweepChunk];
    uint8_t sm[kSweepChunk];
#pragma unroll
    for (int j = 0; j < kSweepChunk; ++j) {
      const int32_t i = min(e0 + j, e - 1);
      m[j] = col[i];
      wm[j] = w[i];
    }
#pragma unroll
    for (int j = 0; j < kSweepChunk; ++j) {
      mb[j] = rp[m[j]];
      me[j] = rp[m[j] + 1];
      sm[j] = __atomic_load_n(&status[m[j]], __ATOMIC_RELAXED);
    }
#pragma unroll
    for (int j = 0; j < kSweepChunk; ++j)
      if (e0 + j < e && wm[j] <= r && key_less(key(m[j]), m[j], kp, p)) note(m[j], sm[j]);
    for (int j = 0; j < kSweepChunk && e0 + j < e; ++j) {
      for (int32_t f0 = mb[j]; f0 < me[j]; f0 += kSweepChunk) {
        int32_t q[kSweepChunk];
        double wq[kSweepChunk];
        uint8_t sq[kSweepChunk];
#pragma unroll
        for (int t = 0; t < kSweepChunk; ++t) {
          const int32_t i = min(f0 + t, me[j] - 1);
          q[t] = col[i];
          wq[t] = w[i];
        }
#pragma unroll
        for (int t = 0; t < kSweepChunk; ++t) sq[t] = __atomic_load_n(&status[q[t]], __ATOMIC_RELAXED);
#pragma unroll
        for (int t = 0; t < kSweepChunk; ++t)
          if (f0 + t < me[j] && q[t] != p && wm[j] + wq[t] <= r && key_less(key(q[t]), q[t], kp, p))
            note(q[t], sq[t]);
      }
    }
  }
  cnt[p] = (uint8_t)(k <= kConflicts ? k : kConflicts + 1);
  if (out) status[p] = 2;
  else if (!blocked) status[p] = 1;
  return !out && blocked;
}

__device__ inline bool lfmis_again(const int32_t* rp, const int32_t* col, const double* w, double r,
                                   const SweepKey& key, uint8_t* status, int32_t p, const int32_t* list,
                                   const uint8_t* cnt) {
  const int32_t k = cnt[p];
  if (k > kConflicts) return lfmis_attempt(rp, col, w, r, key, status, p);
  const int32_t* lp = list + (int64_t)p * kConflicts;
  bool blocked = false, out = false;
  constexpr int kListChunk = 16;
  for (int32_t i0 = 0; i0 < k && !out; i0 += kListChunk) {
    int32_t q[kListChunk];
    uint8_t sq[kListChunk];
#pragma unroll
    for (int t = 0; t < kListChunk; ++t) q[t] = lp[min(i0 + t, k - 1)];
#pragma unroll
    for (int t = 0; t < kListChunk; ++t) sq[t] = __atomic_load_n(&status[q[t]], __ATOMIC_RELAXED);
#pragma unroll
    for (int t = 0; t < kListChunk; ++t) {
      if (i0 + t >= k) continue;
      if (sq[t] == 1) out = true; else if (sq[t] == 0) blocked = true;
    }
  }
  if (out) status[p] = 2;
  else if (!blocked) status[p] = 1;
  return !out && blocked;
}

__global__ void __launch_bounds__(kBlock) k_lfmis_round(const int32_t* rp, const int32_t* col,
                                                        const double* w, int64_t n, const double* scal,
                                                        SweepKey key, uint8_t* status, const int32_t* wl_in,
                                                        int32_t* wl_out, int32_t* rounds, int k, int32_t* list,
                                                        uint8_t* cnt) {
  const int64_t count = k == 0 ? n : rounds[k - 1];
  const double r = scal[1];
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < count; base += (int64_t)gridDim.x * kBlock) {
    const int64_t i = base + threadIdx.x;
    const bool act = i < count;
    const int32_t p = act ? (k == 0 ? (int32_t)i : wl_in[i]) : 0;
    bool pend = false;
    if (act) {
      if (!list) pend = lfmis_attempt(rp, col, w, r, key, status, p);
      else if (k == 0) pend = lfmis_first(rp, col, w, r, key, status, p, list, cnt);
      else pend = lfmis_again(rp, col, w, r, key, status, p, list, cnt);
    }
    block_append(pend, p, wl_out, &rounds[k]);
  }
}

// The remaining rounds of the sweep in one workgroup, once at most
// kDrainItems points are undecided: count_in points in wl_in (or, if wl_in is
// null, all points 0 .. count_in - 1).
__global__ void __launch_bounds__(kDrainItems) k_lfmis_drain(const int32_t* rp, const int32_t* col, const double* w,
                                                             const double* scal, SweepKey key, uint8_t* status,
                                                             const int32_t* wl_in, const int32_t* count_in,
                                                             int64_t n, const int32_t* list, const uint8_t* cnt,
                                                             int32_t* flags) {
  __shared__ int32_t buf[2][kDrainItems];
  __shared__ int32_t c;
  const double r = scal[1];
  int32_t count = wl_in ? *count_in : (int32_t)n;
  int cur = 0;
  for (int round = 0; round < kMaxRounds; ++round) {
    if (threadIdx.x == 0) c = 0;
    __syncthreads();
    if ((int32_t)threadIdx.x < count) {
      const int32_t p = round == 0 ? (wl_in ? wl_in[threadIdx.x] : (int32_t)threadIdx.x) : buf[cur][threadIdx.x];
      bool pend;
      if (!list) pend = lfmis_attempt(rp, col, w, r, key, status, p);
      else if (round == 0 && !wl_in) pend = lfmis_first(rp, col, w, r, key, status, p, (int32_t*)list, (uint8_t*)cnt);
      else pend = lfmis_again(rp, col, w, r, key, status, p, list, cnt);
      if (pend) buf[cur ^ 1][atomicAdd(&c, 1)] = p;
    }
    __syncthreads();
    count = c;
    cur ^= 1;
    __syncthreads();
    if (count == 0) return;
  }
  if (threadIdx.x == 0) atomicOr(flags, F_TIMEOUT);
}

__global__ void k_seed_flags(const uint8_t* status, int64_t n, int32_t* f) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) f[v] = status[v] == 1 ? 1 : 0;
}

__global__ void k_collect_samples(const uint8_t* status, const int32_t* ids, int64_t n, int32_t* samples) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && status[v] == 1) samples[ids[v]] = (int32_t)v;
}

// ------------------------------------------------------------------ graph Voronoi (Sec. 4.3)
__global__ void k_voronoi_init(const uint8_t* status, const int32_t* ids, int64_t n, double* d, int32_t* lab) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  bool seed = status[v] == 1;
  d[v] = seed ? 0.0 : INFINITY;
  lab[v] = seed ? ids[v] : -1;
}

// One Jacobi Bellman-Ford round over (distance, coarse id) pairs compared
// lexicographically: a point takes the smallest (d(u) + w_uv, label(u)) over
// its neighbours.  From +inf this converges to the multi-source shortest-path
// labelling with ties going to the smaller coarse id (same fixed point as a
// multi-source Dijkstra with lexicographic keys).
__global__ void __launch_bounds__(kBlock) k_voronoi_round(const int32_t* rp, const int32_t* col,
                                                          const double* w, const uint8_t* status,
                                                          int64_t n, const double* dA, const int32_t* lA,
                                                          double* dB, int32_t* lB, int32_t* rounds, int k) {
  if (k > 0 && rounds[k - 1] == 0) return;
  int64_t v = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
  bool changed = false;
  if (v < n) {
    double bd = dA[v];
    int32_t bl = lA[v];
    if (status[v] != 1) {
      // the lexicographic minimum of (distance, label): the neighbours' loads
      // are issued kSweepChunk at a time (positions past the row's end
      // re-read its last entry and are not counted)
      const int32_t b = rp[v], e = rp[v + 1];
      for (int32_t e0 = b; e0 < e; e0 += kSweepChunk) {
        int32_t u[kSweepChunk], lu[kSweepChunk];
        double wu[kSweepChunk], du[kSweepChunk];
#pragma unroll
        for (int k = 0; k < kSweepChunk; ++k) {
          const int32_t i = min(e0 + k, e - 1);
          u[k] = col[i];
          wu[k] = w[i];
        }
#pragma unroll
        for (int k = 0; k < kSweepChunk; ++k) {
          lu[k] = lA[u[k]];
          du[k] = dA[u[k]];
        }
#pragma unroll
        for (int k = 0; k < kSweepChunk; ++k) {
          if (e0 + k >= e || lu[k] < 0) continue;
          const double c = du[k] + wu[k];
          if (c < bd || (c == bd && lu[k] < bl)) {
            bd = c;
            bl = lu[k];
          }
        }
      }
      changed = (bd != dA[v]) || (bl != lA[v]);
    }
    dB[v] = bd;
    lB[v] = bl;
  }
  const int32_t c = block_reduce((int32_t)changed, [](int32_t a, int32_t b) { return a + b; });
  if (threadIdx.x == 0 && c) atomicAdd(&rounds[k], c);
}

// ------------------------------------------------------------------ cells, shift (Sec. 4.4)
// Cell sizes; the count a cell had before point v is v's slot in the cell
// (one atomic per run of equal labels: neighbouring points mostly share a cell).
__global__ void k_count_labels(const int32_t* lab, int64_t n, int32_t* cnt, int32_t* slot) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = v < n;
  const int32_t k = run_add(cnt, on ? lab[v] : -1, on);
  if (on) slot[v] = k;
}

// Cell members at their slots (sorted afterwards).
__global__ void k_scatter_labels(const int32_t* __restrict__ lab, int64_t n, const int32_t* __restrict__ ptr,
                                 const int32_t* __restrict__ slot, int32_t* __restrict__ mem) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) mem[ptr[lab[v]] + slot[v]] = (int32_t)v;
}

// Coarse point I = mean of its cell's points, summed in ascending fine index
// from 0.0 (or the sample's own position without the shift).
__global__ void k_cell_mean(const double* X, const int32_t* ptr, const int32_t* mem, const int32_t* samples,
                            int64_t nc, int shift, double* Xc) {
  int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  if (!shift) {
    int64_t s = samples[I];
    Xc[3 * I] = X[3 * s];
    Xc[3 * I + 1] = X[3 * s + 1];
    Xc[3 * I + 2] = X[3 * s + 2];
    return;
  }
  double sx = 0.0, sy = 0.0, sz = 0.0;
  int32_t b = ptr[I], e = ptr[I + 1];
  for (int32_t k = b; k < e; ++k) {
    int64_t i = mem[k];
    sx = sx + X[3 * i];
    sy = sy + X[3 * i + 1];
    sz = sz + X[3 * i + 2];
  }
  double c = (double)(e - b);
  Xc[3 * I] = sx / c;
  Xc[3 * I + 1] = sy / c;
  Xc[3 * I + 2] = sz / c;
}

// ------------------------------------------------------------------ Voronoi-neighbour edges (Sec. 4.3)
__global__ void k_cell_degree(const int32_t* ptr, const int32_t* mem, const int32_t* rp, int64_t nc,
                              int32_t* cdeg) {
  int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int32_t s = 0;
  for (int32_t k = ptr[I]; k < ptr[I + 1]; ++k) s += rp[mem[k] + 1] - rp[mem[k]];
  cdeg[I] = s;
}

// The distinct cells J != I reached by an edge from cell I, written sorted to
// this cell's slot range of `tmp` (cptr[I] .. : one slot per edge of its
// members), their number to ucnt[I].
//
// Cells with more than kCellCand edges: one lane, insertion into the sorted
// range.
// Orders the LDS accesses of a lane group inside one wavefront (its lanes
// run in lockstep and its LDS operations complete in issue order, so only the
// compiler must be kept from moving accesses across).
__device__ __forceinline__ void group_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline void cell_neighbours_serial(const int32_t* ptr, const int32_t* mem, const int32_t* rp,
                                              const int32_t* col, const int32_t* lab, int32_t I, int32_t* out,
                                              int32_t* ucnt) {
  int32_t u = 0;
  for (int32_t k = ptr[I]; k < ptr[I + 1]; ++k) {
    int32_t a = mem[k];
    for (int32_t e = rp[a]; e < rp[a + 1]; ++e) {
      int32_t J = lab[col[e]];
      if (J == I) continue;
      int32_t lo = 0, hi = u;
      while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (out[mid] < J) lo = mid + 1; else hi = mid;
      }
      if (lo < u && out[lo] == J) continue;
      for (int32_t t = u; t > lo; --t) out[t] = out[t - 1];
      out[lo] = J;
      ++u;
    }
  }
  ucnt[I] = u;
}

// Other cells: kCellLanes lanes per cell.  The lanes take the members in turn,
// write the cell label of each member edge's end to LDS (the members' edges
// placed one after another by a scan of their degrees), then every distinct
// label J != I finds its rank among the distinct labels and is written there.
constexpr int kCellLanes = 16;
constexpr int kCellCand = 128;
constexpr int kCellChunk = 8;
constexpr int kCellsPerBlock = kBlock / kCellLanes;

__global__ void __launch_bounds__(kBlock) k_cell_neighbours(const int32_t* ptr, const int32_t* mem,
                                                            const int32_t* rp, const int32_t* col,
                                                            const int32_t* lab, const int32_t* cptr, int64_t nc,
                                                            int32_t* tmp, int32_t* ucnt) {
  __shared__ int32_t cand[kCellsPerBlock][kCellCand];
  const int g = threadIdx.x / kCellLanes, sub = threadIdx.x & (kCellLanes - 1);
  const int64_t I = (int64_t)xcd_block() * kCellsPerBlock + g;
  const bool act = I < nc;
  const int32_t slots = act ? cptr[I + 1] - cptr[I] : 0;   // the members' degree sum
  const bool group = act && slots <= kCellCand;
  int32_t* out = act ? tmp + cptr[I] : tmp;
  int32_t total = 0;
  if (act && !group) {
    if (sub == 0) cell_neighbours_serial(ptr, mem, rp, col, lab, (int32_t)I, out, ucnt);
  } else if (group) {
    const int32_t m0 = ptr[I], m1 = ptr[I + 1];
    for (int32_t k0 = m0; k0 < m1; k0 += kCellLanes) {     // uniform within the group
      const int32_t k = k0 + sub;
      int32_t rb = 0, deg = 0;
      if (k < m1) {
        const int32_t a = mem[k];
        rb = rp[a];
        deg = rp[a + 1] - rb;
      }
      int32_t incl = deg;
      for (int o = 1; o < kCellLanes; o <<= 1) {
        const int32_t t = __shfl_up(incl, o, kCellLanes);
        if (sub >= o) incl += t;
      }
      const int32_t pos = total + incl - deg;
      for (int32_t e0 = 0; e0 < deg; e0 += kCellChunk) {
        int32_t c[kCellChunk], J[kCellChunk];
#pragma unroll
        for (int q = 0; q < kCellChunk; ++q) c[q] = col[rb + min(e0 + q, deg - 1)];
#pragma unroll
        for (int q = 0; q < kCellChunk; ++q) J[q] = lab[c[q]];
#pragma unroll
        for (int q = 0; q < kCellChunk; ++q)
          if (e0 + q < deg) cand[g][pos + e0 + q] = J[q] == (int32_t)I ? INT32_MIN : J[q];
      }
      total += __shfl(incl, kCellLanes - 1, kCellLanes);
    }
  }
  __syncthreads();
  if (group) {
    // the group's candidates sorted (bitonic, padded with INT32_MAX to a power
    // of two; the group's 16 lanes are in one wavefront, whose LDS accesses
    // complete in order), then every distinct label other than the cell's own
    // (INT32_MIN) at the count of distinct labels before it
    int32_t* cg = cand[g];
    int32_t P = 1;
    while (P < total) P <<= 1;
    for (int32_t q = total + sub; q < P; q += kCellLanes) cg[q] = INT32_MAX;
    group_sync();
    for (int32_t k = 2; k <= P; k <<= 1)
      for (int32_t j = k >> 1; j > 0; j >>= 1) {
        for (int32_t q = sub; q < P; q += kCellLanes) {
          const int32_t l = q ^ j;
          if (l > q) {
            const int32_t x = cg[q], y = cg[l];
            if ((x > y) == ((q & k) == 0)) {
              cg[q] = y;
              cg[l] = x;
            }
          }
        }
        group_sync();
      }
    const int32_t per = (total + kCellLanes - 1) / kCellLanes;
    const int32_t q0 = min(total, sub * per), q1 = min(total, q0 + per);
    int32_t u = 0;
    for (int32_t q = q0; q < q1; ++q) u += cg[q] != INT32_MIN && (q == 0 || cg[q - 1] != cg[q]);
    int32_t incl = u;
    for (int o = 1; o < kCellLanes; o <<= 1) {
      const int32_t t = __shfl_up(incl, o, kCellLanes);
      if (sub >= o) incl += t;
    }
    int32_t at = incl - u;
    for (int32_t q = q0; q < q1; ++q)
      if (cg[q] != INT32_MIN && (q == 0 || cg[q - 1] != cg[q])) out[at++] = cg[q];
    if (sub == kCellLanes - 1) ucnt[I] = incl;
  }
}

}  // namespace

void validate_points(const double* X, int64_t n, int32_t* flags, hipStream_t s) {
  k_validate_points<<<blocks_for(3 * n), kBlock, 0, s>>>(X, 3 * n, flags);
}

void edges_to_csr(Handle& h, Level& lv, const int32_t* edges, int64_t m) {
  hipStream_t s = h.stream;
  int64_t n = lv.n;
  int32_t* deg = (int32_t*)talloc(s, (size_t)(n + 1) * 4);
  int32_t* tptr = (int32_t*)talloc(s, (size_t)(n + 1) * 4);
  int32_t* slot = (int32_t*)talloc(s, (size_t)(2 * m + 1) * 4);
  int32_t* tmp = (int32_t*)talloc(s, (size_t)(2 * m + 1) * 4);
  check_hip(hipMemsetAsync(deg, 0, (size_t)(n + 1) * 4, s), "memset");
  if (m > 0) k_edge_degree<<<blocks_for(m), kBlock, 0, s>>>(edges, m, n, deg, slot, h.flags);
  scan_i32(deg, tptr, n, s);
  if (m > 0) k_edge_scatter<<<blocks_for(m), kBlock, 0, s>>>(edges, m, n, tptr, slot, tmp);
  segment_sort_unique(tmp, tptr, deg, n, s);
  lv.erp = (int32_t*)dalloc(h, (size_t)(n + 1) * 4);
  scan_i32(deg, lv.erp, n, s);
  {
    int64_t f = 0;
    ScalarRead rd[2] = {{lv.erp + n, 4, &lv.nnzE}, {h.flags, 4, &f}};
    read_scalars(h, rd, 2);
    throw_flags((int32_t)f, "edge array");
  }
  lv.nnzE_cap = lv.nnzE;
  lv.ecol = (int32_t*)dalloc(h, (size_t)(lv.nnzE + 1) * 4);
  compact_segments(tmp, tptr, lv.erp, lv.ecol, n, s);
  tfree(s, deg);
  tfree(s, tptr);
  tfree(s, slot);
  tfree(s, tmp);
}

void validate_matrix(const int32_t* rp, const int32_t* col, const double* val, int64_t n, int64_t nnz,
                     int32_t* flags, hipStream_t s) {
  k_validate_matrix<<<blocks_for(n), kBlock, 0, s>>>(rp, col, val, n, nnz, flags);
}

void edge_weights(Level& lv, hipStream_t s) {
  k_edge_weights<<<blocks_for(lv.n), kBlock, 0, s>>>(lv.X, lv.erp, lv.ecol, lv.n, lv.ew);
}

void mean_edge(Handle& h, Level& lv, double rho) {
  hipStream_t s = h.stream;
  unsigned long long* acc = (unsigned long long*)talloc(s, 16);
  check_hip(hipMemsetAsync(acc, 0, 16, s), "memset");
  const int rg = std::min(blocks_for(lv.n), kReduceGrid);
  k_edge_max<<<rg, kBlock, 0, s>>>(lv.erp, lv.ecol, lv.ew, lv.n, acc);
  k_edge_fixsum<<<rg, kBlock, 0, s>>>(lv.erp, lv.ecol, lv.ew, lv.n, acc, acc + 1);
  k_edge_mean_finish<<<1, 1, 0, s>>>(acc, acc + 1, lv.erp + lv.n, rho, lv.scal);
  tfree(s, acc);
}

// Runs sweep rounds until every point is decided; returns the number of
// coarse points and fills lv.samples (ascending fine index = coarse id order).
int64_t sample_lfmis(Handle& h, Level& lv, int level) {
  hipStream_t s = h.stream;
  int64_t n = lv.n;
  uint8_t* status = (uint8_t*)talloc(s, (size_t)n);
  check_hip(hipMemsetAsync(status, 0, (size_t)n, s), "memset");
  int32_t* rounds = fresh_rounds(h);
  SweepKey key{h.opt.seed ^ ((uint64_t)level << 32), h.opt.sample_order == 1};
  int32_t* wl = (int32_t*)talloc(s, (size_t)2 * n * 4);
  const int grid = std::min(blocks_for(n), kRoundGrid);
  int32_t* f = (int32_t*)talloc(s, (size_t)(n + 1) * 4);
  int32_t* ids = (int32_t*)talloc(s, (size_t)(n + 1) * 4);
  const bool lists = n <= kListLevel;
  int32_t* list = lists ? (int32_t*)talloc(s, (size_t)n * kConflicts * 4) : nullptr;
  uint8_t* cnt = lists ? (uint8_t*)talloc(s, (size_t)n) : nullptr;
  int k = 0;
  int64_t nc = 0;
  bool drained = false;
  if (n <= kDrainItems) {
    k_lfmis_drain<<<1, kDrainItems, 0, s>>>(lv.erp, lv.ecol, lv.ew, lv.scal, key, status, nullptr, nullptr, n, list,
                                           cnt, h.flags);
    drained = true;
  }
  for (;;) {
    if (!drained)
      for (int t = 0; t < kRoundBatch; ++t, ++k)
        k_lfmis_round<<<grid, kBlock, 0, s>>>(lv.erp, lv.ecol, lv.ew, n, lv.scal, key, status,
                                              wl + ((k + 1) % 2) * n, wl + (k % 2) * n, rounds, k, list, cnt);
    // coarse ids, valid if the sweep has finished (read together with the round count)
    k_seed_flags<<<blocks_for(n), kBlock, 0, s>>>(status, n, f);
    scan_i32(f, ids, n, s);
    int64_t left = 0, fl = 0;
    ScalarRead rd[3] = {{rounds + (drained ? 0 : k - 1), 4, &left}, {ids + n, 4, &nc}, {h.flags, 4, &fl}};
    read_scalars(h, rd, 3);
    if (fl & F_TIMEOUT) throw Error{GMG_DEVICE_ERROR, "sampling did not terminate"};
    if (drained || left == 0) break;
    if (left <= kDrainItems) {
      k_lfmis_drain<<<1, kDrainItems, 0, s>>>(lv.erp, lv.ecol, lv.ew, lv.scal, key, status, wl + ((k - 1) % 2) * n,
                                             rounds + (k - 1), n, list, cnt, h.flags);
      drained = true;
      continue;
    }
    if (k + kRoundBatch > kMaxRounds) throw Error{GMG_DEVICE_ERROR, "sampling did not terminate"};
  }
  tfree(s, wl);
  if (lists) {
    tfree(s, list);
    tfree(s, cnt);
  }
  lv.nc = nc;
  lv.samples = (int32_t*)dalloc(h, (size_t)(nc + 1) * 4);
  k_collect_samples<<<blocks_for(n), kBlock, 0, s>>>(status, ids, n, lv.samples);
  lv.label = (int32_t*)dalloc(h, (size_t)n * 4);
  lv.dist = (double*)dalloc(h, (size_t)n * 8);
  k_voronoi_init<<<blocks_for(n), kBlock, 0, s>>>(status, ids, n, lv.dist, lv.label);
  lv.status = status;                            // released by voronoi()
  tfree(s, f);
  tfree(s, ids);
  return nc;
}

void voronoi(Handle& h, Level& lv) {
  hipStream_t s = h.stream;
  int64_t n = lv.n;
  uint8_t* status = lv.status;
  lv.status = nullptr;
  double* dB = (double*)talloc(s, (size_t)n * 8);
  int32_t* lB = (int32_t*)talloc(s, (size_t)n * 4);
  int32_t* rounds = fresh_rounds(h);
  int k = 0;
  for (;;) {
    for (int t = 0; t < kRoundBatch; ++t, ++k) {
      const double* dA = (k % 2 == 0) ? lv.dist : dB;
      const int32_t* lA = (k % 2 == 0) ? lv.label : lB;
      double* dO = (k % 2 == 0) ? dB : lv.dist;
      int32_t* lO = (k % 2 == 0) ? lB : lv.label;
      k_voronoi_round<<<blocks_for(n), kBlock, 0, s>>>(lv.erp, lv.ecol, lv.ew, status, n, dA, lA, dO, lO,
                                                       rounds, k);
    }
    if (read_i64(h, rounds + (k - 1), 4) == 0) break;
    if (k + kRoundBatch > kMaxRounds) throw Error{GMG_DEVICE_ERROR, "Voronoi rounds did not terminate"};
  }
  // The first round without changes copied its input unchanged, so both
  // buffers hold the fixed point; lv.dist / lv.label are final.
  tfree(s, dB);
  tfree(s, lB);
  tfree(s, status);
}

void cells_and_shift(Handle& h, Level& lv, Level& nx, bool shift, int32_t** cell_ptr, int32_t** cell_mem) {
  hipStream_t s = h.stream;
  int64_t n = lv.n, nc = lv.nc;
  int32_t* cnt = (int32_t*)talloc(s, (size_t)(nc + 1) * 4);
  int32_t* slot = (int32_t*)talloc(s, (size_t)n * 4);
  int32_t* ptr = (int32_t*)talloc(s, (size_t)(nc + 1) * 4);
  int32_t* mem = (int32_t*)talloc(s, (size_t)n * 4);
  check_hip(hipMemsetAsync(cnt, 0, (size_t)(nc + 1) * 4, s), "memset");
  k_count_labels<<<blocks_for(n), kBlock, 0, s>>>(lv.label, n, cnt, slot);
  scan_i32(cnt, ptr, nc, s);
  k_scatter_labels<<<blocks_for(n), kBlock, 0, s>>>(lv.label, n, ptr, slot, mem);
  segment_sort_unique(mem, ptr, cnt, nc, s);     // members ascending (they are distinct)
  nx.n = nc;
  nx.X = (double*)dalloc(h, (size_t)nc * 3 * 8);
  k_cell_mean<<<blocks_for(nc), kBlock, 0, s>>>(lv.X, ptr, mem, lv.samples, nc, shift ? 1 : 0, nx.X);
  tfree(s, cnt);
  tfree(s, slot);
  *cell_ptr = ptr;
  *cell_mem = mem;
}

void coarse_edges(Handle& h, Level& lv, Level& nx, const int32_t* cell_ptr, const int32_t* cell_mem) {
  hipStream_t s = h.stream;
  int64_t nc = nx.n;
  int32_t* cdeg = (int32_t*)talloc(s, (size_t)(nc + 1) * 4);
  int32_t* cptr = (int32_t*)talloc(s, (size_t)(nc + 1) * 4);
  int32_t* tmp = (int32_t*)talloc(s, (size_t)(lv.nnzE_cap + 1) * 4);
  k_cell_degree<<<blocks_for(nc), kBlock, 0, s>>>(cell_ptr, cell_mem, lv.erp, nc, cdeg);
  scan_i32(cdeg, cptr, nc, s);
  k_cell_neighbours<<<blocks_for(nc, kCellsPerBlock), kBlock, 0, s>>>(cell_ptr, cell_mem, lv.erp, lv.ecol,
                                                                      lv.label, cptr, nc, tmp, cdeg);
  nx.erp = (int32_t*)dalloc(h, (size_t)(nc + 1) * 4);
  scan_i32(cdeg, nx.erp, nc, s);
  // every coarse edge entry comes from a distinct fine edge entry: nnz(E_{l+1}) <= nnz(E_l)
  nx.nnzE_cap = lv.nnzE_cap;
  nx.ecol = (int32_t*)dalloc(h, (size_t)(nx.nnzE_cap + 1) * 4);
  compact_segments(tmp, cptr, nx.erp, nx.ecol, nc, s);
  tfree(s, cdeg);
  tfree(s, cptr);
  tfree(s, tmp);
}

}  // namespace gmg
