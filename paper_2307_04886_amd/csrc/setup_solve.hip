// Solve-phase setup: the Gauss-Seidel colouring of each A_l, the
// colour-sorted solve layout (SELL-64 matrix, SoA prolongation, restriction
// rows), and the dense factorisation of the coarsest operator (Alg. 2 solves
// the coarsest level directly).
#include <algorithm>
#include <cstring>

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

constexpr int kColorChunk = 16;

// On levels of up to kColorListLevel rows the first visit of v also records
// the lower-key neighbours not yet coloured, in list[v * kColorList ..] with
// their number in cnt[v], and the colours of those already coloured as a bit
// mask (cnt[v] = kColorList + 1: too many neighbours to list, or a colour of
// 64 or more; later visits read the row again).  Colours are final once
// written, so a later visit reads only the listed neighbours' colours and
// takes the same decision as a visit that reads the whole row.
constexpr int kColorList = 32;
constexpr int64_t kColorListLevel = 262144;

struct ColorLists {
  int32_t* list = nullptr;   // null: no lists, every visit reads the row
  uint64_t* mask = nullptr;
  uint8_t* cnt = nullptr;
};

__device__ inline int32_t first_fit_above(const int32_t* rp, const int32_t* col, const ColorKey& key,
                                          const int32_t* color, int32_t v, uint64_t kv) {
  for (int32_t c = 64;; ++c) {                  // rare: every colour below 64 is taken
    bool used = false;
    for (int32_t e = rp[v]; e < rp[v + 1] && !used; ++e) {
      int32_t u = col[e];
      if (u == v) continue;
      uint64_t ku = key(u);
      if ((ku < kv || (ku == kv && u < v)) && color[u] == c) used = true;
    }
    if (!used) return c;
  }
}

// Returns 0 if v must wait for a lower-key neighbour, else colours v and
// returns its colour + 1.  The row is read kColorChunk entries at a time with
// every column and neighbour-colour load in flight together (positions past
// the row's end re-read its last entry; every row holds its diagonal).  With
// Record, a waiting row also writes its lists.
template <bool Record>
__device__ inline int32_t color_attempt(const int32_t* rp, const int32_t* col, const ColorKey& key,
                                        int32_t* color, int32_t v, const ColorLists& L) {
  const uint64_t kv = key(v);
  uint64_t mask = 0;
  bool high = false, wait = false;
  int32_t nrec = 0;
  const int32_t b = rp[v], e = rp[v + 1];
  for (int32_t e0 = b; e0 < e; e0 += kColorChunk) {
    int32_t u[kColorChunk], cu[kColorChunk];
#pragma unroll
    for (int k = 0; k < kColorChunk; ++k) u[k] = col[min(e0 + k, e - 1)];
#pragma unroll
    for (int k = 0; k < kColorChunk; ++k) cu[k] = __atomic_load_n(&color[u[k]], __ATOMIC_RELAXED);
#pragma unroll
    for (int k = 0; k < kColorChunk; ++k) {
      if (e0 + k >= e || u[k] == v) continue;
      const uint64_t ku = key(u[k]);
      if (!(ku < kv || (ku == kv && u[k] < v))) continue;
      if (cu[k] < 0) {
        wait = true;
        if constexpr (Record) {
          if (nrec < kColorList) L.list[(int64_t)v * kColorList + nrec] = u[k];
          ++nrec;
        }
      } else if (cu[k] < 64) {
        mask |= 1ull << cu[k];
      } else {
        high = true;
      }
    }
  }
  if (wait) {
    if constexpr (Record) {
      L.mask[v] = mask;
      L.cnt[v] = (uint8_t)(nrec <= kColorList && !high ? nrec : kColorList + 1);
    }
    return 0;
  }
  int32_t c = (~mask) ? __builtin_ctzll(~mask) : 64;
  if (c == 64 && high) c = first_fit_above(rp, col, key, color, v, kv);
  color[v] = c;
  return c + 1;
}

// A later visit of a row with lists: the colours of the listed neighbours.
__device__ inline int32_t color_again(const int32_t* rp, const int32_t* col, const ColorKey& key,
                                      int32_t* color, int32_t v, const ColorLists& L) {
  const int32_t n = L.cnt[v];
  if (n > kColorList) return color_attempt<false>(rp, col, key, color, v, L);
  uint64_t mask = L.mask[v];
  bool high = false, wait = false;
  const int32_t* lp = L.list + (int64_t)v * kColorList;
  for (int32_t e0 = 0; e0 < n; e0 += kColorChunk) {
    int32_t u[kColorChunk], cu[kColorChunk];
#pragma unroll
    for (int k = 0; k < kColorChunk; ++k) u[k] = lp[min(e0 + k, n - 1)];
#pragma unroll
    for (int k = 0; k < kColorChunk; ++k) cu[k] = __atomic_load_n(&color[u[k]], __ATOMIC_RELAXED);
#pragma unroll
    for (int k = 0; k < kColorChunk; ++k) {
      if (e0 + k >= n) continue;
      if (cu[k] < 0) wait = true;
      else if (cu[k] < 64) mask |= 1ull << cu[k];
      else high = true;
    }
  }
  if (wait) return 0;
  int32_t c = (~mask) ? __builtin_ctzll(~mask) : 64;
  if (c == 64 && high) c = first_fit_above(rp, col, key, color, v, key(v));
  color[v] = c;
  return c + 1;
}

// Any visit: the first (round 0 over every row) records the lists.
__device__ inline int32_t color_visit(const int32_t* rp, const int32_t* col, const ColorKey& key, int32_t* color,
                                      int32_t v, const ColorLists& L, bool first) {
  if (!L.list) return color_attempt<false>(rp, col, key, color, v, L);
  if (first) return color_attempt<true>(rp, col, key, color, v, L);
  return color_again(rp, col, key, color, v, L);
}

// One Jones-Plassmann round; round 0 visits every row, later rounds the
// worklist of rows still waiting after the previous round.
__global__ void __launch_bounds__(kBlock) k_color_round(const int32_t* rp, const int32_t* col, int64_t n,
                                                        ColorKey key, int32_t* color, const int32_t* wl_in,
                                                        int32_t* wl_out, int32_t* rounds, int k, ColorLists L) {
  const int64_t count = k == 0 ? n : rounds[k - 1];
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < count; base += (int64_t)gridDim.x * kBlock) {
    const int64_t i = base + threadIdx.x;
    const bool act = i < count;
    const int32_t v = act ? (k == 0 ? (int32_t)i : wl_in[i]) : 0;
    int32_t got = 0;
    if (act) got = color_visit(rp, col, key, color, v, L, k == 0);
    block_append(act && got == 0, v, wl_out, &rounds[k]);
  }
}

// One class of an iterated-greedy pass: every vertex v with old[v] == c takes
// the smallest colour not used by a neighbour's new colour (neu[u] >= 0: the
// classes above c, recoloured by earlier launches).  Vertices of one class are
// not adjacent, so they are recoloured in parallel.
__global__ void __launch_bounds__(kBlock) k_ig_class(const int32_t* rp, const int32_t* col, int64_t n,
                                                     const int32_t* old, int32_t* neu, int32_t c) {
  for (int64_t v = (int64_t)xcd_block() * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
    if (old[v] != c) continue;
    const int32_t b = rp[v], e = rp[v + 1];
    uint64_t mask = 0;
    bool high = false;
    for (int32_t e0 = b; e0 < e; e0 += kColorChunk) {
      int32_t u[kColorChunk], cu[kColorChunk];
#pragma unroll
      for (int k = 0; k < kColorChunk; ++k) u[k] = col[min(e0 + k, e - 1)];
#pragma unroll
      for (int k = 0; k < kColorChunk; ++k) cu[k] = neu[u[k]];
#pragma unroll
      for (int k = 0; k < kColorChunk; ++k) {
        if (e0 + k >= e || u[k] == v || cu[k] < 0) continue;
        if (cu[k] < 64) mask |= 1ull << cu[k];
        else high = true;
      }
    }
    int32_t k = (~mask) ? __builtin_ctzll(~mask) : 64;
    if (k == 64 && high) {
      for (;; ++k) {                            // rare: every colour below 64 is taken
        bool used = false;
        for (int32_t t = b; t < e && !used; ++t) used = col[t] != v && neu[col[t]] == k;
        if (!used) break;
      }
    }
    neu[v] = k;
  }
}

// A whole small level in one workgroup of kDrainItems threads, its row
// offsets, 16-bit columns and colours in LDS: the Jones-Plassmann rounds (the
// same first-fit decisions in key order as the multi-launch rounds), then
// `passes` iterated-greedy passes (the classes of the first colouring from the
// highest down, as k_ig_class).  Each row is first partitioned in place, its
// lower-key neighbours first, so that the rounds compute no keys; the rounds
// visit a worklist of the rows still waiting, and each pass lists the rows of
// every class, so that a thread holds at most a few rows of a round or class.
// Writes the colours and their count.
constexpr int kSmallColorRows = 4096;
constexpr int kSmallColorPer = kSmallColorRows / kDrainItems;
constexpr int kSmallColorMax = 256;               // classes a pass can list
constexpr int64_t kSmallColorLds = 150 * 1024;
inline int64_t small_color_lds(int64_t n, int64_t nnz) {
  auto up = [](int64_t b) { return (b + 15) & ~(int64_t)15; };
  return up((n + 1) * 4) + up(nnz * 2) + 5 * up(n * 2) + up(n * 4);
}

// Smallest colour from the neighbours' mask, or, when every colour below 64
// is taken, the smallest colour no entry of scol[lo, hi) other than v has.
__device__ inline int32_t small_first_fit(const uint16_t* scol, int32_t lo, int32_t hi, const int16_t* c,
                                          int32_t v, uint64_t mask, bool high) {
  int32_t k = (~mask) ? __builtin_ctzll(~mask) : 64;
  if (k < 64 || !high) return k;
  for (;; ++k) {                                // rare: every colour below 64 is taken
    bool used = false;
    for (int32_t e = lo; e < hi && !used; ++e) used = scol[e] != v && c[scol[e]] == k;
    if (!used) return k;
  }
}

__global__ void __launch_bounds__(kDrainItems) k_color_small(const int32_t* rp, const int32_t* col, int32_t n,
                                                             ColorKey key, int32_t passes, int32_t* color,
                                                             int32_t* ncolors, int32_t* flags) {
  extern __shared__ int32_t lds_small[];
  auto up = [](int64_t b) { return (int32_t)((b + 15) & ~(int64_t)15); };
  char* base = reinterpret_cast<char*>(lds_small);
  int32_t* srp = reinterpret_cast<int32_t*>(base);
  const int32_t nnz = rp[n];
  uint16_t* scol = reinterpret_cast<uint16_t*>(base + up((int64_t)(n + 1) * 4));
  const int32_t na = up((int64_t)n * 2) / 2;       // int16 elements per n-array
  int16_t* ca = reinterpret_cast<int16_t*>(base + up((int64_t)(n + 1) * 4) + up((int64_t)nnz * 2));
  int16_t* cb = ca + na;
  int16_t* lowc = cb + na;                       // lower-key neighbours of each row
  int16_t* wa = lowc + na;                       // worklists / class lists
  int16_t* wb = wa + na;
  int32_t* waitc = reinterpret_cast<int32_t*>(wb + na);   // uncoloured lower-key neighbours of each row
  __shared__ int32_t s_cnt[3];
  __shared__ int32_t s_cls[kSmallColorMax + 1];
  const int tid = (int)threadIdx.x;
  for (int32_t i = tid; i <= n; i += kDrainItems) srp[i] = rp[i];
  for (int32_t i = tid; i < n; i += kDrainItems) ca[i] = -1;
  if (tid < 3) s_cnt[tid] = 0;
  // columns: 16 loads in flight per thread before their stores
  for (int32_t e0 = 0; e0 < nnz; e0 += 16 * kDrainItems) {
    int32_t cv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) cv[u] = col[min(e0 + u * kDrainItems + tid, nnz - 1)];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (e0 + u * kDrainItems + tid < nnz) scol[e0 + u * kDrainItems + tid] = (uint16_t)cv[u];
  }
  __syncthreads();
  // each thread partitions its own rows
#pragma unroll
  for (int q = 0; q < kSmallColorPer; ++q) {
    const int32_t v = tid + q * kDrainItems;
    if (v >= n) continue;
    const uint64_t kv = key(v);
    const int32_t b = srp[v], e = srp[v + 1];
    int32_t w = b;
    for (int32_t t = b; t < e; ++t) {
      const int32_t u = scol[t];
      if (u == v) continue;
      const uint64_t ku = key(u);
      if (ku < kv || (ku == kv && u < v)) {
        scol[t] = scol[w];
        scol[w] = (uint16_t)u;
        ++w;
      }
    }
    lowc[v] = (int16_t)(w - b);
  }
  __syncthreads();
  // Rounds in dependency order: a row is ready once all its lower-key
  // neighbours are coloured (its count of uncoloured ones, held in wait[],
  // reaches zero); round r colours the rows that became ready in round r - 1
  // (round 0: the rows without lower-key neighbours) and counts down their
  // higher-key neighbours, appending those that become ready, counted in
  // s_cnt[r % 3] (reset at the start of round r - 1, after every thread read
  // the count it held before).  Each coupling is visited twice in all.
  const int lane = tid & (kWave - 1);
  int32_t count = 0;
  if (tid == 0) s_cnt[0] = 0;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kSmallColorPer; ++q) {
    const int32_t v = tid + q * kDrainItems;
    const bool ready = v < n && lowc[v] == 0;
    if (v < n) waitc[v] = lowc[v];
    const unsigned long long m = __ballot(ready);
    if (m) {
      int32_t o = 0;
      if (lane == 0) o = atomicAdd(&s_cnt[0], (int32_t)__popcll(m));
      o = __shfl(o, 0, kWave);
      if (ready) wb[o + __popcll(m & ((1ull << lane) - 1ull))] = (int16_t)v;
    }
  }
  __syncthreads();
  count = s_cnt[0];
  int32_t coloured = 0;
  bool done = count == 0;
  for (int round = 0; round < kMaxRounds && !done; ++round) {
    const int16_t* src = (round & 1) ? wa : wb;
    int16_t* dst = (round & 1) ? wb : wa;
    if (tid == 0) s_cnt[(round + 2) % 3] = 0;
#pragma unroll
    for (int q = 0; q < kSmallColorPer; ++q) {
      const int32_t i = tid + q * kDrainItems;
      if (i >= count) continue;
      const int32_t v = src[i];
      const int32_t b = srp[v], l = b + lowc[v], e = srp[v + 1];
      uint64_t mask = 0;
      bool high = false;
      for (int32_t t0 = b; t0 < l; t0 += 8) {          // the lower-key neighbours, all coloured
        int32_t u[8], cu[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) u[k] = scol[min(t0 + k, l - 1)];
#pragma unroll
        for (int k = 0; k < 8; ++k) cu[k] = ca[u[k]];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (t0 + k >= l) continue;
          if (cu[k] < 64) mask |= 1ull << cu[k];
          else high = true;
        }
      }
      ca[v] = (int16_t)small_first_fit(scol, b, l, ca, v, mask, high);
    }
    __syncthreads();                              // the round's colours are written
    // count down the higher-key neighbours of the round's rows
#pragma unroll
    for (int q = 0; q < kSmallColorPer; ++q) {
      const int32_t i = tid + q * kDrainItems;
      const bool act = i < count;
      const int32_t v = act ? src[i] : 0;
      const int32_t l = act ? srp[v] + lowc[v] : 0, e = act ? srp[v + 1] : 0;
      for (int32_t t0 = l; t0 < e; t0 += 8) {          // eight at a time, the atomics in flight together
        int32_t u[8], old[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) u[k] = t0 + k < e ? (int32_t)scol[t0 + k] : v;
#pragma unroll
        for (int k = 0; k < 8; ++k) old[k] = atomicSub(&waitc[u[k]], u[k] != v ? 1 : 0);   // v itself: minus 0
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (u[k] != v && old[k] == 1) dst[atomicAdd(&s_cnt[(round + 1) % 3], 1)] = (int16_t)u[k];
      }
    }
    coloured += count;
    __syncthreads();
    count = s_cnt[(round + 1) % 3];
    done = count == 0;
  }
  done = coloured == n;
  if (!done) {
    if (tid == 0) atomicOr(flags, F_TIMEOUT);
    return;
  }
  // the count of colours
  if (tid == 0) s_cnt[0] = 0;
  __syncthreads();
  {
    int32_t m = 0;
    for (int32_t v = tid; v < n; v += kDrainItems) m = max(m, (int32_t)ca[v] + 1);
    atomicMax(&s_cnt[0], m);
  }
  __syncthreads();
  const int32_t nc0 = s_cnt[0];
  if (nc0 > kSmallColorMax) {
    if (tid == 0) atomicOr(flags, F_OVERFLOW);
    return;
  }
  int16_t* cur = ca;
  int16_t* nxt = cb;
  if (nc0 > 1) {
    for (int p = 0; p < passes; ++p) {
      // the rows of every class of cur, listed in wa (any order within a class)
      for (int32_t c = tid; c <= nc0; c += kDrainItems) s_cls[c] = 0;
      __syncthreads();
      for (int32_t v = tid; v < n; v += kDrainItems) {
        atomicAdd(&s_cls[cur[v] + 1], 1);
        nxt[v] = -1;
      }
      __syncthreads();
      if (tid == 0)
        for (int32_t c = 1; c <= nc0; ++c) s_cls[c] += s_cls[c - 1];
      __syncthreads();
      for (int32_t v = tid; v < n; v += kDrainItems) wa[atomicAdd(&s_cls[cur[v]], 1)] = (int16_t)v;
      __syncthreads();
      // after the placement s_cls[c] is the end of class c (its start: s_cls[c - 1], or 0)
      for (int32_t c = nc0 - 1; c >= 0; --c) {
        const int32_t lo = c > 0 ? s_cls[c - 1] : 0, hi = s_cls[c];
#pragma unroll
        for (int q = 0; q < kSmallColorPer; ++q) {
          const int32_t i = lo + tid + q * kDrainItems;
          if (i >= hi) continue;
          const int32_t v = wa[i];
          const int32_t b = srp[v], e = srp[v + 1];
          uint64_t mask = 0;
          bool high = false;
          for (int32_t t0 = b; t0 < e; t0 += 8) {           // eight neighbours at a time
            int32_t u[8], cu[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) u[k] = scol[min(t0 + k, e - 1)];
#pragma unroll
            for (int k = 0; k < 8; ++k) cu[k] = nxt[u[k]];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              if (t0 + k >= e || u[k] == v || cu[k] < 0) continue;
              if (cu[k] < 64) mask |= 1ull << cu[k];
              else high = true;
            }
          }
          nxt[v] = (int16_t)small_first_fit(scol, b, e, nxt, v, mask, high);
        }
        __syncthreads();
      }
      int16_t* t = cur;
      cur = nxt;
      nxt = t;
    }
  }
  if (tid == 0) s_cnt[0] = 0;
  __syncthreads();
  int32_t m = 0;
  for (int32_t v = tid; v < n; v += kDrainItems) {
    color[v] = cur[v];
    m = max(m, (int32_t)cur[v] + 1);
  }
  atomicMax(&s_cnt[0], m);
  __syncthreads();
  if (tid == 0) *ncolors = s_cnt[0];
}

// The remaining Jones-Plassmann rounds in one workgroup, once at most
// kDrainItems rows wait: count_in rows in wl_in (or, if wl_in is null, all
// rows 0 .. n - 1).
__global__ void __launch_bounds__(kDrainItems) k_color_drain(const int32_t* rp, const int32_t* col, int64_t n,
                                                             ColorKey key, int32_t* color, const int32_t* wl_in,
                                                             const int32_t* count_in, ColorLists L, int32_t* flags) {
  __shared__ int32_t buf[2][kDrainItems];
  __shared__ int32_t c;
  int32_t count = wl_in ? *count_in : (int32_t)n;
  int cur = 0;
  for (int round = 0; round < kMaxRounds; ++round) {
    if (threadIdx.x == 0) c = 0;
    __syncthreads();
    if ((int32_t)threadIdx.x < count) {
      const int32_t v = round == 0 ? (wl_in ? wl_in[threadIdx.x] : (int32_t)threadIdx.x) : buf[cur][threadIdx.x];
      if (!color_visit(rp, col, key, color, v, L, round == 0 && !wl_in)) buf[cur ^ 1][atomicAdd(&c, 1)] = v;
    }
    __syncthreads();
    count = c;
    cur ^= 1;
    __syncthreads();
    if (count == 0) return;
  }
  if (threadIdx.x == 0) atomicOr(flags, F_TIMEOUT);
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

// cptr[c] = first new index of colour c (keys of stride classes per colour).
__global__ void k_color_ptr(const int32_t* off, int nb, int nc, int stride, int32_t* cptr) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= nc) cptr[c] = off[(int64_t)c * stride * nb];
}

// key = colour * kLenKeys + class, the class counting down from the widest
// rows (in 4-entry quads), so that a colour's rows come longest first.
__global__ void k_len_class(const int32_t* color, const int32_t* rp, int64_t n, int32_t* key) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t quads = (rp[v + 1] - rp[v] + 3) / 4;
  key[v] = color[v] * kLenKeys + (kLenKeys - 1 - min(max(quads - 1, 0), kLenKeys - 1));
}

// ------------------------------------------------------------------ SELL-64 matrices
// Row r of the result is source row perm[r] (or r) of a CSR matrix; columns
// are renumbered through cmap (or kept); entries keep their CSR order, so
// every row sum adds its terms in the same order as the source row.
// Row lengths, slice sizes and the longest row in one pass: one thread per
// row over whole slices (a wavefront's 64 rows are one slice, so the slice
// width is a wavefront maximum); *mx = max(*mx, longest row).
__global__ void __launch_bounds__(kBlock) k_row_len_width(const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ rp, int64_t n, int64_t ns,
                                                          int32_t* __restrict__ len, int32_t* __restrict__ wsz,
                                                          int32_t* mx) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int32_t l = 0;
  if (r < n) {
    const int32_t src = perm ? perm[r] : (int32_t)r;
    l = rp[src + 1] - rp[src];
    len[r] = l;
  }
  int32_t w = l;
  for (int o = kWave / 2; o > 0; o >>= 1) w = max(w, __shfl_xor(w, o, kWave));
  const int64_t sl = r / kSlice;
  if ((threadIdx.x & (kWave - 1)) == 0 && sl < ns) wsz[sl] = w * kSlice;
  const int32_t b = block_reduce(l, [](int32_t a, int32_t c) { return a > c ? a : c; });
  if (threadIdx.x == 0 && b) atomicMax(mx, b);
}

constexpr int kFillChunk = 8;

// The loads of kFillChunk entries of the source row are issued together
// (positions past the row's end re-read its last entry and store padding).
__global__ void k_sell_fill(const int32_t* __restrict__ perm, const int32_t* __restrict__ cmap,
                            const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const double* __restrict__ val, int64_t n, const int32_t* __restrict__ sptr,
                            int32_t* __restrict__ scol, double* __restrict__ sval, double* __restrict__ diag) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int64_t s = r / kSlice, ln = r % kSlice;
  int32_t src = perm ? perm[r] : (int32_t)r;
  const int32_t b = rp[src], len = rp[src + 1] - b;
  const int32_t base = sptr[s];
  const int32_t w = (sptr[s + 1] - base) / kSlice;
  for (int32_t t0 = 0; t0 < w; t0 += kFillChunk) {
    int32_t j[kFillChunk], m[kFillChunk];
    double v[kFillChunk];
    if (len > 0) {
#pragma unroll
      for (int k = 0; k < kFillChunk; ++k) {
        const int32_t q = b + min(t0 + k, len - 1);
        j[k] = col[q];
        v[k] = val[q];
      }
#pragma unroll
      for (int k = 0; k < kFillChunk; ++k) m[k] = cmap ? cmap[j[k]] : j[k];
    }
#pragma unroll
    for (int k = 0; k < kFillChunk; ++k) {
      const int32_t t = t0 + k;
      if (t >= w) break;
      const int64_t o = base + (int64_t)t * kSlice + ln;
      if (t < len) {
        scol[o] = m[k];
        sval[o] = v[k];
        if (diag && j[k] == src) diag[r] = v[k];
      } else {
        scol[o] = 0;
        sval[o] = 0.0;
      }
    }
  }
}

// The same fill, one workgroup per slice of 64 rows, transposed through LDS:
// every source row is read contiguously (its entries across lanes), the slice
// is written column by column (entry t of the 64 rows contiguous).  pitch is
// at least the longest row of the matrix.
constexpr int kSliceFillMax = 64;

__global__ void __launch_bounds__(kBlock) k_sell_fill_slice(const int32_t* __restrict__ perm,
                                                            const int32_t* __restrict__ cmap,
                                                            const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ col,
                                                            const double* __restrict__ val, int64_t n,
                                                            const int32_t* __restrict__ sptr,
                                                            int32_t* __restrict__ scol, double* __restrict__ sval,
                                                            double* __restrict__ diag, int pitch) {
  extern __shared__ double fill_lds[];
  double* lv = fill_lds;                                   // [kSlice][pitch]
  int32_t* lc = (int32_t*)(fill_lds + kSlice * pitch);     // [kSlice][pitch]
  __shared__ int32_t rb[kSlice], rl[kSlice], rs[kSlice];
  const int64_t s = xcd_block();
  const int64_t r0 = s * kSlice;
  const int tid = threadIdx.x;
  if (tid < kSlice) {
    const int64_t r = r0 + tid;
    int32_t src = -1, b = 0, len = 0;
    if (r < n) {
      src = perm ? perm[r] : (int32_t)r;
      b = rp[src];
      len = rp[src + 1] - b;
    }
    rb[tid] = b;
    rl[tid] = len;
    rs[tid] = src;
  }
  __syncthreads();
  const int32_t base = sptr[s];
  const int w = (sptr[s + 1] - base) / kSlice;
  for (int idx = tid; idx < kSlice * w; idx += kBlock) {
    const int row = idx / w, t = idx - row * w;
    int32_t c = 0;
    double v = 0.0;
    if (t < rl[row]) {
      const int32_t j = col[rb[row] + t];
      v = val[rb[row] + t];
      c = cmap ? cmap[j] : j;
      if (diag && j == rs[row]) diag[r0 + row] = v;
    }
    lc[row * pitch + t] = c;
    lv[row * pitch + t] = v;
  }
  __syncthreads();
  for (int idx = tid; idx < kSlice * w; idx += kBlock) {
    const int t = idx / kSlice, ln = idx - t * kSlice;
    const int64_t o = base + (int64_t)t * kSlice + ln;
    scol[o] = lc[ln * pitch + t];
    sval[o] = lv[ln * pitch + t];
  }
}

// *out = max(*out, max_i v[i] + add)
__global__ void __launch_bounds__(kBlock) k_max_i32(const int32_t* v, int64_t n, int32_t add, int32_t* out) {
  int32_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    m = v[i] + add > m ? v[i] + add : m;
  m = block_reduce(m, [](int32_t a, int32_t b) { return a > b ? a : b; });
  if (threadIdx.x == 0 && m) atomicMax(out, m);
}

void max_i32(const int32_t* v, int64_t n, int32_t add, int32_t* out, hipStream_t s) {
  k_max_i32<<<std::min(blocks_for(n), kReduceGrid), kBlock, 0, s>>>(v, n, add, out);
}

// nnz of colour class c = prefix[cptr[c+1]] - prefix[cptr[c]] of the row lengths
__global__ void k_color_nnz(const int32_t* prefix, const int32_t* cptr, int nc, int32_t* cnnz) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nc) cnnz[c] = prefix[cptr[c + 1]] - prefix[cptr[c]];
}

// P in the new numbering, SoA ELL-3 ([3][n]); padding repeats the first
// column with weight 0.
__global__ void k_p_layout(const int32_t* __restrict__ perm, const int32_t* __restrict__ ciperm,
                           const int32_t* __restrict__ pcol, const double* __restrict__ pval,
                           const int32_t* __restrict__ pcnt, int64_t n, int32_t* __restrict__ qcol,
                           double* __restrict__ qval, int32_t* __restrict__ qcnt) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int32_t old = perm[r];
  const int32_t c = pcnt[old];
  int32_t pc[3], cc[3];
  double pv[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    pc[t] = pcol[3 * old + t];
    pv[t] = pval[3 * old + t];
  }
#pragma unroll
  for (int t = 0; t < 3; ++t) cc[t] = t < c ? ciperm[pc[t]] : 0;
  qcnt[r] = c;
  const int32_t first = c > 0 ? cc[0] : 0;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    qcol[t * n + r] = t < c ? cc[t] : first;
    qval[t * n + r] = t < c ? pv[t] : 0.0;
  }
}

// ------------------------------------------------------------------ coarsest level
__global__ void k_dense_scatter(const int32_t* rp, const int32_t* col, const double* val, int64_t n,
                                double* D) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t e = rp[i]; e < rp[i + 1]; ++e) D[i * n + col[e]] = val[e];
}

// Blocked right-looking dense Cholesky (32-column panels).  Entry (i, c)
// receives its updates -L[i][j] * L[c][j] one at a time in ascending j, then
// (below the diagonal) the division by L[c][c]: the same operations in the
// same order as the column-by-column definition, whatever the blocking.
constexpr int kPanel = 32;

// Lane l's value of v, for a lane index known at compile time.
__device__ __forceinline__ double read_lane(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Factor the diagonal block of panel k0 and solve the panel rows below it.
// The diagonal block is factored by the first wavefront, lane i holding row i
// in registers: column c of the block is l_ic = (a_ic - sum_{m<c} l_im l_cm)
// / l_cc (ascending m), l_cc = sqrt(a_cc - sum_{m<c} l_cm^2).
__global__ void __launch_bounds__(256) k_chol_panel(double* D, int64_t n, int64_t k0, int32_t* flags) {
  __shared__ double T[kPanel][kPanel + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int kb = (int)(n - k0 < kPanel ? n - k0 : kPanel);
  if (tid < kWave) {
    const int i = tid;
    double r[kPanel];
#pragma unroll
    for (int c = 0; c < kPanel; ++c) r[c] = (i < kb && c <= i) ? D[(k0 + i) * n + k0 + c] : 0.0;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < kPanel; ++c) {
      if (c < kb) {
        double t = r[c];
#pragma unroll
        for (int m = 0; m < c; ++m) t = t - r[m] * read_lane(r[m], c);
        const double dc = read_lane(t, c);
        ok = ok && dc > 0.0;
        const double d = ok ? sqrt(dc) : 1.0;
        if (i == c) r[c] = d;
        else if (i > c) r[c] = t / d;
      }
      __builtin_amdgcn_sched_barrier(0);   // one column at a time: bounds the live registers
    }
    if (i < kb) {
#pragma unroll
      for (int c = 0; c < kPanel; ++c)
        if (c <= i) T[i][c] = r[c];
    }
    if (ok && i < kb) {
#pragma unroll
      for (int c = 0; c < kPanel; ++c)
        if (c <= i) D[(k0 + i) * n + k0 + c] = r[c];
    }
    if (tid == 0) {
      bad = ok ? 0 : 1;
      if (!ok) atomicOr(flags, F_NOT_SPD);
    }
  }
  __syncthreads();
  if (bad) return;
  // panel rows: l_ij = (a_ij - sum_{k0 <= m < j} l_im l_jm) / l_jj, ascending j
  for (int64_t i = k0 + kb + tid; i < n; i += blockDim.x) {
    double a[kPanel];
#pragma unroll
    for (int j = 0; j < kPanel; ++j) a[j] = j < kb ? D[i * n + k0 + j] : 0.0;
#pragma unroll
    for (int j = 0; j < kPanel; ++j) {
      if (j < kb) {
        double t = a[j];
#pragma unroll
        for (int m = 0; m < j; ++m) t = t - a[m] * T[j][m];
        a[j] = t / T[j][j];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int j = 0; j < kPanel; ++j)
      if (j < kb) D[i * n + k0 + j] = a[j];
  }
}

// Trailing update of the lower triangle below panel k0: one 32x32 tile per
// workgroup, a_ic <- a_ic - l_ij l_cj for the panel columns j in ascending order.
__global__ void __launch_bounds__(1024) k_chol_update(double* D, int64_t n, int64_t k0, int kb) {
  __shared__ double LI[kPanel][kPanel + 1];
  __shared__ double LC[kPanel][kPanel + 1];
  const int64_t base = k0 + kb;
  const int64_t I = blockIdx.y, C = blockIdx.x;
  if (C > I) return;
  const int ti = threadIdx.x / kPanel, tc = threadIdx.x % kPanel;
  const int64_t gi = base + I * kPanel + ti, gc = base + C * kPanel + ti;
  LI[ti][tc] = (gi < n && tc < kb) ? D[gi * n + k0 + tc] : 0.0;
  LC[ti][tc] = (gc < n && tc < kb) ? D[gc * n + k0 + tc] : 0.0;
  __syncthreads();
  const int64_t i = base + I * kPanel + ti, c = base + C * kPanel + tc;
  if (i < n && c <= i) {
    double a = D[i * n + c];
    for (int j = 0; j < kb; ++j) a = a - LI[ti][j] * LC[tc][j];
    D[i * n + c] = a;
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

// Column c of the coarsest inverse, A^-1 e_c, by substitution with the
// factor: forward L y = e_c, row i subtracting L_ik y_k for k ascending, then
// back L^T x = y, row i subtracting L_ki x_k for k descending from n - 1; each
// row is then divided by its pivot.  Both run column-oriented: once y_k (x_k)
// is known, every row that needs it subtracts its term, so each row performs
// its subtractions in the order of the row-by-row definition, bit for bit.
// Rows above c start at +0 and stay +0 (every term they would subtract is a
// product with y_k = +0), so the forward pass starts at row c.
//
// One wavefront per column: lane l holds rows l, l + 64, ... (S slots) in
// registers and the pivot row's value is read across lanes; the factor
// entries of the next D steps are loaded ahead (phase k mod D of a ring).
template <int S, int D>
__global__ void __launch_bounds__(kWave) k_coarse_inverse(const double* __restrict__ L,
                                                         const double* __restrict__ U, int32_t n,
                                                         double* __restrict__ inv) {
  const int32_t c = blockIdx.x;
  const int lane = threadIdx.x;
  double s[S];
#pragma unroll
  for (int q = 0; q < S; ++q) s[q] = q * kWave + lane == c ? 1.0 : 0.0;
  double f[D][S], d[D];                       // ring: factor entries and pivot of step k at phase k mod D
  // forward: step k uses column k of L (row k of U) for rows i > k
  auto load_fwd = [&](int j, int32_t k) {
    if (k >= n) return;
    d[j] = L[(int64_t)k * n + k];
#pragma unroll
    for (int q = 0; q < S; ++q)
      if (q * kWave + kWave - 1 > k) f[j][q] = U[(int64_t)k * n + min(q * kWave + lane, n - 1)];
  };
#pragma unroll
  for (int j = 0; j < D; ++j) load_fwd(j, c + ((j - c) % D + D) % D);
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const int32_t k_lo = max(c, q * kWave), k_hi = min(n, (q + 1) * kWave);
    for (int32_t k0 = k_lo - k_lo % D; k0 < k_hi; k0 += D) {
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const int32_t k = k0 + j;
        if (k >= k_lo && k < k_hi) {
          const double y = read_lane(s[q], k & (kWave - 1)) / d[j];
          if (lane == (k & (kWave - 1))) s[q] = y;
#pragma unroll
          for (int q2 = q; q2 < S; ++q2) {
            const int32_t i = q2 * kWave + lane;
            if (i > k && i < n) s[q2] = s[q2] - f[j][q2] * y;
          }
          load_fwd(j, k + D);
        }
      }
    }
  }
  // back: step i uses row i of L for rows r < i
  auto load_bwd = [&](int j, int32_t i) {
    if (i < 0) return;
    d[j] = L[(int64_t)i * n + i];
#pragma unroll
    for (int q = 0; q < S; ++q)
      if (q * kWave < i) f[j][q] = L[(int64_t)i * n + min(q * kWave + lane, n - 1)];
  };
#pragma unroll
  for (int j = 0; j < D; ++j) load_bwd(j, (n - 1) - (((n - 1 - j) % D) + D) % D);
#pragma unroll
  for (int q = S - 1; q >= 0; --q) {
    const int32_t i_hi = min(n, (q + 1) * kWave) - 1, i_lo = q * kWave;
    if (i_hi < i_lo) continue;
    // groups of D steps aligned to multiples of D, top step i0 first
    for (int32_t i0 = i_hi + (D - 1 - i_hi % D); i0 >= i_lo; i0 -= D) {
#pragma unroll
      for (int jj = D - 1; jj >= 0; --jj) {
        const int32_t i = i0 - (D - 1) + jj;        // descending within the group
        const int j = jj;
        if (i >= i_lo && i <= i_hi) {
          const double x = read_lane(s[q], i & (kWave - 1)) / d[j];
          if (lane == (i & (kWave - 1))) s[q] = x;
#pragma unroll
          for (int q2 = 0; q2 <= q; ++q2) {
            const int32_t r = q2 * kWave + lane;
            if (r < i) s[q2] = s[q2] - f[j][q2] * x;
          }
          load_bwd(j, i - D);
        }
      }
    }
  }
  const int32_t ld = (int32_t)inv_ld(n);
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const int32_t i = q * kWave + lane;
    if (i < ld) inv[(int64_t)c * ld + i] = i < n ? s[q] : 0.0;
  }
}

// The same operations for coarsest levels beyond the register form: the
// column lives in LDS, one workgroup per column, a barrier per step.
__global__ void __launch_bounds__(kBlock) k_coarse_inverse_lds(const double* __restrict__ L,
                                                               const double* __restrict__ U, int32_t n,
                                                               double* __restrict__ inv) {
  extern __shared__ double col[];
  const int32_t c = blockIdx.x;
  for (int32_t i = threadIdx.x; i < n; i += kBlock) col[i] = i == c ? 1.0 : 0.0;
  __syncthreads();
  for (int32_t k = c; k < n; ++k) {
    const double y = col[k] / L[(int64_t)k * n + k];
    for (int32_t i = k + 1 + threadIdx.x; i < n; i += kBlock) col[i] = col[i] - U[(int64_t)k * n + i] * y;
    __syncthreads();                          // every thread has read col[k]
    if (threadIdx.x == 0) col[k] = y;
    __syncthreads();
  }
  for (int32_t i = n - 1; i >= 0; --i) {
    const double x = col[i] / L[(int64_t)i * n + i];
    for (int32_t r = threadIdx.x; r < i; r += kBlock) col[r] = col[r] - L[(int64_t)i * n + r] * x;
    __syncthreads();
    if (threadIdx.x == 0) col[i] = x;
    __syncthreads();
  }
  const int32_t ld = (int32_t)inv_ld(n);
  for (int32_t i = threadIdx.x; i < ld; i += kBlock) inv[(int64_t)c * ld + i] = i < n ? col[i] : 0.0;
}

// Longest row of every colour, rounded up to kTailGroup: w[c].
__global__ void k_color_width(const int32_t* len, const int32_t* cptr, int32_t* w) {
  __shared__ int32_t ws[kBlock / kWave];
  const int c = blockIdx.x;
  int32_t m = 0;
  for (int32_t r = cptr[c] + threadIdx.x; r < cptr[c + 1]; r += kBlock) m = len[r] > m ? len[r] : m;
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t t = __shfl_xor(m, o, kWave);
    m = t > m ? t : m;
  }
  if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kBlock / kWave; ++i) m = ws[i] > m ? ws[i] : m;
    w[c] = (m + kTailGroup - 1) / kTailGroup * kTailGroup;
  }
}

// A_l (SELL) into the tail's per-colour ELL, with and without the diagonal,
// and every row's wavefront width: the longest row of its 64-row chunk of the
// colour, rounded up to 4 entries.
__global__ void k_tail_ell(SellView A, const int32_t* cinfo, int nc, int64_t n, int32_t* col_gs, double* val_gs,
                           int32_t* col, double* val, uint16_t* ww) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int c = 0;
  while (c + 1 < nc && cinfo[4 * (c + 1)] <= r) ++c;
  const int32_t lo = cinfo[4 * c], hi = cinfo[4 * c + 1], w = cinfo[4 * c + 2], off = cinfo[4 * c + 3];
  const int32_t len = A.len[r];
  {
    const int32_t c0 = lo + (int32_t)((r - lo) & ~(int64_t)(kWave - 1));
    const int32_t c1 = min(c0 + kWave, hi);
    int32_t m = 0;
    for (int32_t q = c0; q < c1; ++q) m = max(m, A.len[q]);
    ww[r] = (uint16_t)min((m + 3) & ~3, w);
  }
  const int64_t base = A.ptr[r / kSlice] + (r & (kSlice - 1));
  for (int32_t t = 0; t < w; ++t) {
    const int64_t oc = ell_col_index(off, hi - lo, lo, r, t), ov = ell_val_index(off, hi - lo, lo, r, t);
    int32_t j = (int32_t)n;
    double v = 0.0;
    if (t < len) {
      j = A.col[base + (int64_t)t * kSlice];
      v = A.val[base + (int64_t)t * kSlice];
    }
    col[oc] = j;
    val[ov] = v;
    col_gs[oc] = j == r ? (int32_t)n : j;
    val_gs[ov] = j == r ? 0.0 : v;
  }
}

// P_l^T (SELL, nc rows) into ELL of width w; padding column n (the fine level's size).
__global__ void k_tail_ell_t(SellView T, int64_t nc, int32_t w, int64_t n, int32_t* col, double* val) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int32_t len = T.len[I];
  const int64_t base = T.ptr[I / kSlice] + (I & (kSlice - 1));
  for (int32_t t = 0; t < w; ++t) {
    col[ell_col_index(0, nc, 0, I, t)] = t < len ? T.col[base + (int64_t)t * kSlice] : (int32_t)n;
    val[ell_val_index(0, nc, 0, I, t)] = t < len ? T.val[base + (int64_t)t * kSlice] : 0.0;
  }
}


// ------------------------------------------------------------------ block order
// Order-preserving 64-bit key of a double (a larger double gets a larger
// key), so that minima and maxima are exact integer atomics.
__device__ __forceinline__ unsigned long long ordered_key(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  return (u >> 63) ? ~u : (u | (1ull << 63));
}

__global__ void k_grid_keys_init(unsigned long long* keys) {
  const int i = threadIdx.x;
  if (i < 9) keys[i] = i < 3 ? ~0ull : 0ull;
}

// keys[0..2]: minima and keys[3..5]: maxima of the three coordinates (ordered
// keys); keys[6..8]: largest |X_j,a - X_i,a| over the stored off-diagonal
// entries (i, j) of A_l, per axis a (non-negative doubles, whose bit patterns
// order as integers).
__global__ void __launch_bounds__(kBlock) k_grid_extents(const double* __restrict__ X, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ col, int64_t n,
                                                         unsigned long long* keys) {
  unsigned long long mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0, 0, 0}, dm[3] = {0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double xi[3] = {X[3 * i], X[3 * i + 1], X[3 * i + 2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const unsigned long long k = ordered_key(xi[a]);
      mn[a] = k < mn[a] ? k : mn[a];
      mx[a] = k > mx[a] ? k : mx[a];
    }
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int64_t j = col[e];
      if (j == i) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const unsigned long long d = __builtin_bit_cast(unsigned long long, fabs(X[3 * j + a] - xi[a]));
        dm[a] = d > dm[a] ? d : dm[a];
      }
    }
  }
  auto lo = [](unsigned long long u, unsigned long long v) { return u < v ? u : v; };
  auto hi = [](unsigned long long u, unsigned long long v) { return u > v ? u : v; };
  unsigned long long r[9];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = block_reduce(mn[a], lo);
    __syncthreads();
    r[3 + a] = block_reduce(mx[a], hi);
    __syncthreads();
    r[6 + a] = block_reduce(dm[a], hi);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      atomicMin(&keys[a], r[a]);
      atomicMax(&keys[3 + a], r[3 + a]);
      atomicMax(&keys[6 + a], r[6 + a]);
    }
  }
}

// Colour of brick bx of cell row cy: with a = bx - (cy + 1) div 2, (a - cy)
// mod 3.  A brick holds the cells cx of its row with (cx + cy mod 2) div 2 =
// bx (two cells side by side, shifted by one cell on odd rows); it touches
// two bricks in its row and two in each neighbouring row, and these six
// colours all differ from its own.
__host__ __device__ inline int32_t brick_color(int64_t bx, int64_t cy) {
  const int64_t a = bx - (cy + 1) / 2;
  return (int32_t)(((a - cy) % 3 + 3) % 3);
}

// Block colour of block id c (bricks: cy nbx + bx with nbx = gx div 2 + 1;
// single cells: cy gx + cx, coloured by their parity pair).
__host__ __device__ inline int32_t block_color_of(int32_t c, int32_t gx, bool bricks) {
  if (bricks) {
    const int32_t nbx = gx / 2 + 1;
    return brick_color(c % nbx, c / nbx);
  }
  return (c % gx & 1) + 2 * (c / gx & 1);
}

// Brick (cy nbx + bx) and cell (cy gx + cx) of every point.
__global__ void k_grid_cells(const double* __restrict__ X, int64_t n, int a0, int a1, double lo0, double lo1,
                             double side, int32_t gx, int32_t* brick, int32_t* cell) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t cx = (int64_t)floor((X[3 * i + a0] - lo0) / side);
  const int64_t cy = (int64_t)floor((X[3 * i + a1] - lo1) / side);
  brick[i] = (int32_t)(cy * (gx / 2 + 1) + (cx + (cy & 1)) / 2);
  cell[i] = (int32_t)(cy * gx + cx);
}

// The chosen blocks of every point and their colours.
__global__ void k_block_ids(const int32_t* brick, const int32_t* cell, int64_t n, int32_t gx, int32_t bricks,
                            int32_t* bcell, int32_t* bcolor) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t c = bricks ? brick[i] : cell[i];
  bcell[i] = c;
  bcolor[i] = block_color_of(c, gx, bricks != 0);
}

// Sweep class of a row: block colour, then colour.
__global__ void k_sweep_class(const int32_t* bcolor, const int32_t* color, int64_t n, int32_t C, int32_t* cls) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cls[i] = bcolor[i] * C + color[i];
}

__global__ void k_count_cells(const int32_t* bcell, int64_t n, int32_t* cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = i < n;
  run_add(cnt, on ? bcell[i] : -1, on);
}

// Rows per brick and rows per cell, in one pass.
__global__ void k_count_cells2(const int32_t* brick, const int32_t* cell, int64_t n, int32_t* cntb, int32_t* cntc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = i < n;
  run_add(cntb, on ? brick[i] : -1, on);
  run_add(cntc, on ? cell[i] : -1, on);
}

// ---- per-cell colouring of a level swept in block order (DSATUR in each cell)
constexpr int32_t kMaxCellRows = 512;     // larger blocks send the level back to the colour order
constexpr int32_t kMaxBrickRows = 256;    // a larger brick makes single cells the level's blocks
constexpr int32_t kMaxCellColors = 64;    // likewise a cell that needs this many colours
constexpr int32_t kCellAdjLds = 4096;     // in-cell couplings of a cell kept in LDS (else in HBM)

__global__ void k_cell_slots(const int32_t* bcell, int64_t n, int32_t* cnt, int32_t* slot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = i < n;
  const int32_t t = run_add(cnt, on ? bcell[i] : -1, on);
  if (on) slot[i] = t;
}

__global__ void k_cell_scatter(const int32_t* __restrict__ bcell, int64_t n, const int32_t* __restrict__ cptr,
                               const int32_t* __restrict__ slot, int32_t* __restrict__ rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) rows[cptr[bcell[i]] + slot[i]] = (int32_t)i;
}

// The largest value over the wavefront, in every lane: running maxima within
// each row of 16 lanes (DPP row shifts by 1, 2, 4, 8; lanes shifted in from
// outside the row contribute 0), the row maxima carried across rows (DPP row
// broadcasts of lanes 15 and 31), then lane 63's value read back.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  auto mx = [](uint32_t a, uint32_t b) { return a > b ? a : b; };
  v = mx(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));   // row_shr:1
  v = mx(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));   // row_shr:2
  v = mx(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));   // row_shr:4
  v = mx(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));   // row_shr:8
  v = mx(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));   // row_bcast:15
  v = mx(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));   // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}

// In-cell degree of row i (couplings to other rows of its cell), and the
// cell's total.
__global__ void k_incell_degree(const int32_t* __restrict__ arp, const int32_t* __restrict__ acol,
                                const int32_t* __restrict__ bcell, int64_t n, int32_t* __restrict__ deg,
                                int32_t* __restrict__ cell_deg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = i < n;
  const int32_t c = on ? bcell[i] : -1;
  int32_t d = 0;
  if (on) {
    for (int32_t e = arp[i]; e < arp[i + 1]; ++e) {
      const int32_t j = acol[e];
      d += (j != (int32_t)i && bcell[j] == c) ? 1 : 0;
    }
    deg[i] = d;
  }
  run_sum(cell_deg, c, d, on);                 // one atomic per run of rows of one block
}

// DSATUR in one cell, one wavefront per cell.  The cell's rows are sorted
// ascending in LDS (bitonic), so a row's position is its rank by index; its
// in-cell neighbours become positions (binary search), kept in LDS when they
// fit and otherwise in the cell's segment of adj.  Each step colours the
// uncoloured row of largest saturation (distinct colours among its coloured
// in-cell neighbours), then largest in-cell degree, then smallest position,
// with the smallest colour none of its neighbours has.  A row that would need
// colour kMaxCellColors sets *overflow.
__global__ void __launch_bounds__(kWave) k_cell_dsatur(const int32_t* __restrict__ cptr,
                                                      const int32_t* __restrict__ rows,
                                                      const int32_t* __restrict__ deg_of,
                                                      const int32_t* __restrict__ cadj,
                                                      const int32_t* __restrict__ arp,
                                                      const int32_t* __restrict__ acol,
                                                      const int32_t* __restrict__ bcell, int32_t* __restrict__ adj,
                                                      int32_t* __restrict__ color, int32_t* __restrict__ maxcol,
                                                      int32_t* __restrict__ overflow) {
  __shared__ uint64_t mask[kMaxCellRows];
  __shared__ int32_t r[kMaxCellRows], deg[kMaxCellRows], off[kMaxCellRows + 1];
  __shared__ int32_t ladj[kCellAdjLds];
  const int32_t c = blockIdx.x;
  const int32_t base = cptr[c], m = cptr[c + 1] - base;
  if (m <= 0 || m > kMaxCellRows) return;
  const int lane = threadIdx.x;
  int32_t M = 1;
  while (M < m) M <<= 1;
  for (int32_t p = lane; p < M; p += kWave) r[p] = p < m ? rows[base + p] : INT32_MAX;
  __syncthreads();
  for (int32_t k = 2; k <= M; k <<= 1)
    for (int32_t j = k >> 1; j > 0; j >>= 1) {
      for (int32_t p = lane; p < M; p += kWave) {
        const int32_t q = p ^ j;
        if (q > p) {
          const int32_t x = r[p], y = r[q];
          if ((x > y) == ((p & k) == 0)) {
            r[p] = y;
            r[q] = x;
          }
        }
      }
      __syncthreads();
    }
  for (int32_t p = lane; p < m; p += kWave) {
    mask[p] = 0;
    deg[p] = deg_of[r[p]];
  }
  __syncthreads();
  if (lane == 0) {
    int32_t acc = 0;
    for (int32_t p = 0; p < m; ++p) {
      off[p] = acc;
      acc += deg[p];
    }
    off[m] = acc;
  }
  __syncthreads();
  int32_t* A = off[m] <= kCellAdjLds ? ladj : adj + cadj[c];
  for (int32_t p = lane; p < m; p += kWave) {
    const int32_t i = r[p];
    int32_t t = off[p];
    for (int32_t e = arp[i]; e < arp[i + 1]; ++e) {
      const int32_t j = acol[e];
      if (j == i || bcell[j] != c) continue;
      int32_t lo = 0, hi = m;
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (r[mid] < j) lo = mid + 1;
        else hi = mid;
      }
      A[t++] = lo;
    }
  }
  __threadfence_block();
  __syncthreads();
  // Lane l holds rows l + 64 q: their colour (-1: not yet coloured; rows past
  // m count as coloured) and degree in registers, so a step reads only the
  // rows' masks from LDS, all of them at once.
  constexpr int kQ = kMaxCellRows / kWave;
  int32_t cq[kQ], dq[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int32_t p = lane + q * kWave;
    cq[q] = p < m ? -1 : 0;
    dq[q] = p < m ? deg[p] : 0;
  }
  int32_t used = 0;
  for (int32_t step = 0; step < m; ++step) {
    uint64_t mk[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) mk[q] = mask[lane + q * kWave];
    uint32_t best = 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int32_t p = lane + q * kWave;
      const uint32_t key = ((uint32_t)__popcll(mk[q]) << 20) | ((uint32_t)dq[q] << 10) | (uint32_t)(1023 - p);
      best = cq[q] < 0 && key > best ? key : best;
    }
    best = wave_max_u32(best);
    const int32_t v = 1023 - (int32_t)(best & 1023u);
    const uint64_t free_colours = ~mask[v];
    if (free_colours == 0) {                // every colour below kMaxCellColors is taken
      if (lane == 0) atomicOr(overflow, 1);
      return;
    }
    const int32_t k = __builtin_ctzll(free_colours);
    used = used > k ? used : k;
#pragma unroll
    for (int q = 0; q < kQ; ++q)
      if (lane + q * kWave == v) cq[q] = k;
    __syncthreads();
    for (int32_t t = lane; t < deg[v]; t += kWave) mask[A[off[v] + t]] |= uint64_t(1) << k;
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int32_t p = lane + q * kWave;
    if (p < m) color[r[p]] = cq[q];
  }
  if (lane == 0) atomicMax(maxcol, used);
}

// Slot v of the block numbering, [0, 4 H) with H block ids: id v mod H if its
// colour is k = v div H (else -1); blocks are numbered by colour, then id.
__device__ __forceinline__ int32_t grid_cell_of(int64_t v, int64_t H, int32_t gx, bool bricks) {
  const int32_t k = (int32_t)(v / H);
  const int32_t b = (int32_t)(v % H);
  return block_color_of(b, gx, bricks) == k ? b : -1;
}

__global__ void k_cell_flags(const int32_t* cnt, int64_t H, int32_t gx, int32_t bricks, int32_t* flag) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= 4 * H) return;
  const int32_t c = grid_cell_of(v, H, gx, bricks != 0);
  flag[v] = c >= 0 && cnt[c] > 0 ? 1 : 0;
}

// Block (compact id) of every solve row.
__global__ void k_row_block(const int32_t* perm, const int32_t* bcell, int64_t n, const int32_t* vid, int64_t H,
                            int32_t gx, int32_t bricks, int32_t* blk) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int32_t c = bcell[perm[g]];
  blk[g] = vid[(int64_t)block_color_of(c, gx, bricks != 0) * H + c];
}

// First local row of every colour c = 0..C in every block (rows of a block are
// ascending solve rows, so ascending colours).
__global__ void k_block_cls(const int32_t* boff, const int32_t* brows, const int32_t* perm, const int32_t* color,
                            int32_t nblk, int32_t C, int32_t* bcls) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nblk * (C + 1)) return;
  const int32_t b = (int32_t)(t / (C + 1)), c = (int32_t)(t % (C + 1));
  int32_t lo = boff[b], hi = boff[b + 1];
  const int32_t base = lo;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (color[perm[brows[mid]]] < c) lo = mid + 1; else hi = mid;
  }
  bcls[t] = lo - base;
}

// Per local row: its length (entries of A_l, diagonal included) and colour,
// packed as len << 8 | colour; per block: the mask of its colours.
__global__ void k_block_rowinfo(const int32_t* rp, const int32_t* perm, const int32_t* color, const int32_t* brows,
                                int64_t n, int32_t* rinfo) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t o = perm[brows[k]];
  rinfo[k] = ((rp[o + 1] - rp[o]) << 8) | color[o];
}

// Per block: its header and its gather list (own rows, then halo rows, padded with the
// block's first row, so that loads of padding slots share a line with a real load).
__global__ void k_block_gather(const int32_t* boff, const int32_t* brows, const int32_t* hoff, const int32_t* hlist,
                               const int32_t* bw, const int32_t* beoff, const uint64_t* bmask, int32_t gstride,
                               BlockHdr* hdr, int32_t* glist) {
  const int32_t b = blockIdx.x;
  const int32_t r0 = boff[b], rows = boff[b + 1] - r0, h0 = hoff[b], nh = hoff[b + 1] - h0;
  if (threadIdx.x == 0) {
    BlockHdr hd;
    hd.r0 = r0;
    hd.rows = rows;
    hd.nh = nh;
    hd.w = bw[b];
    hd.e0 = beoff[b];
    hd.pad = 0;
    hd.mask = bmask[b];
    hdr[b] = hd;
  }
  for (int32_t k = threadIdx.x; k < gstride; k += blockDim.x)
    glist[(int64_t)b * gstride + k] = k < rows ? brows[r0 + k] : (k < rows + nh ? hlist[h0 + k - rows] : brows[r0]);
}

__global__ void k_block_mask(const int32_t* bcls, int32_t nblk, int32_t C, uint64_t* bmask) {
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  uint64_t m = 0;
  for (int32_t c = 0; c < C; ++c)
    if (bcls[(int64_t)b * (C + 1) + c] < bcls[(int64_t)b * (C + 1) + c + 1]) m |= uint64_t(1) << c;
  bmask[b] = m;
}


__global__ void k_block_cells(const int32_t* boff, const int32_t* bw, int32_t nblk, int32_t* sz) {
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nblk) sz[b] = bw[b] * (boff[b + 1] - boff[b]);
}

// The halo of every block, one workgroup per block: the rows of other blocks
// that its rows read, collected in LDS, sorted (bitonic) and kept once each,
// written at the block's slot base tmp + tcap[b] (capacity: its entries);
// hcnt[b] receives their number.  A coupling to another block of the same
// block colour (which the grid excludes), or more than kHaloSort collected
// entries, raises *bad.
constexpr int kHaloSort = 4096;
__global__ void __launch_bounds__(kBlock) k_block_halo(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                       const int32_t* __restrict__ perm,
                                                       const int32_t* __restrict__ iperm,
                                                       const int32_t* __restrict__ blk,
                                                       const int32_t* __restrict__ bcolor,
                                                       const int32_t* __restrict__ boff,
                                                       const int32_t* __restrict__ brows, int32_t* tmp,
                                                       const int32_t* __restrict__ tcap, int32_t* hcnt, int32_t* bad) {
  __shared__ int32_t a[kHaloSort];
  __shared__ int32_t part[kBlock + 1];
  __shared__ int32_t na;
  const int32_t b = blockIdx.x;
  const int32_t r0 = boff[b], rows = boff[b + 1] - r0;
  if (threadIdx.x == 0) na = 0;
  __syncthreads();
  for (int32_t p = threadIdx.x; p < rows; p += kBlock) {
    const int32_t g = brows[r0 + p], o = perm[g];
    for (int32_t e = rp[o]; e < rp[o + 1]; ++e) {
      const int32_t oc = col[e];
      if (oc == o) continue;
      const int32_t j = iperm[oc];
      if (blk[j] == b) continue;
      if (bcolor[oc] == bcolor[o]) atomicOr(bad, 1);
      const int32_t k = atomicAdd(&na, 1);
      if (k < kHaloSort) a[k] = j;
    }
  }
  __syncthreads();
  const int32_t len = na;
  if (len > kHaloSort) {
    if (threadIdx.x == 0) {
      atomicOr(bad, 2);
      hcnt[b] = 0;
    }
    return;
  }
  int32_t P = 1;
  while (P < len) P <<= 1;
  for (int32_t i = len + threadIdx.x; i < P; i += kBlock) a[i] = INT32_MAX;
  __syncthreads();
  for (int32_t k = 2; k <= P; k <<= 1)
    for (int32_t j = k >> 1; j > 0; j >>= 1) {
      for (int32_t i = threadIdx.x; i < P; i += kBlock) {
        const int32_t l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const int32_t x = a[i], y = a[l];
          if ((x > y) == up) {
            a[i] = y;
            a[l] = x;
          }
        }
      }
      __syncthreads();
    }
  // distinct values: each thread counts the first occurrences in its chunk
  const int32_t chunk = (len + kBlock - 1) / kBlock;
  const int32_t c0 = threadIdx.x * chunk, c1 = min(len, c0 + chunk);
  int32_t cnt = 0;
  for (int32_t i = c0; i < c1; ++i) cnt += (i == 0 || a[i] != a[i - 1]) ? 1 : 0;
  part[threadIdx.x + 1] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    part[0] = 0;
    for (int t = 1; t <= kBlock; ++t) part[t] += part[t - 1];
    hcnt[b] = part[kBlock];
  }
  __syncthreads();
  int32_t w = tcap[b] + part[threadIdx.x];
  for (int32_t i = c0; i < c1; ++i)
    if (i == 0 || a[i] != a[i - 1]) tmp[w++] = a[i];
}

// Entries of A_l (diagonal included) in the rows of every block: the halo's capacity.
// Entries (cap) and longest row (bw) of every block, a wavefront per block.
__global__ void k_block_entries(const int32_t* rp, const int32_t* perm, const int32_t* brows, const int32_t* boff,
                                int32_t nblk, int32_t* cap, int32_t* bw) {
  const int32_t b = (int32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  if (b >= nblk) return;
  int32_t s = 0, w = 0;
  for (int32_t k = boff[b] + (int32_t)(threadIdx.x & (kWave - 1)); k < boff[b + 1]; k += kWave) {
    const int32_t o = perm[brows[k]];
    const int32_t len = rp[o + 1] - rp[o];
    s += len;
    w = max(w, len);
  }
  s = wave_sum(s);
  for (int o = kWave / 2; o > 0; o >>= 1) w = max(w, __shfl_xor(w, o, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) {
    cap[b] = s;
    bw[b] = w;
  }
}

// The block ELL, one workgroup per block (its halo in LDS): entry t of local
// row p of block b at beoff[b] + t rows_b + p; the LDS slot of its column
// (own row: its local row; another block's row: rows_b + its position in the
// block's halo) and its value; the diagonal and the padding up to the block's
// width point at the zero slot rows_b + halo_b with value 0.
__global__ void __launch_bounds__(kBlock) k_block_ell(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                      const double* __restrict__ val, const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ iperm,
                                                      const int32_t* __restrict__ blk,
                                                      const int32_t* __restrict__ lpos,
                                                      const int32_t* __restrict__ boff,
                                                      const int32_t* __restrict__ brows,
                                                      const int32_t* __restrict__ hoff,
                                                      const int32_t* __restrict__ hlist,
                                                      const int32_t* __restrict__ bw,
                                                      const int32_t* __restrict__ beoff, int32_t* elx, double* elv) {
  __shared__ int32_t hl[kHaloSort];
  const int32_t b = (int32_t)xcd_block();
  const int32_t r0 = boff[b], rows = boff[b + 1] - r0;
  const int32_t h0 = hoff[b], nh = hoff[b + 1] - h0;
  for (int32_t k = threadIdx.x; k < nh; k += kBlock) hl[k] = hlist[h0 + k];
  __syncthreads();
  const int32_t pad = rows + nh, w = bw[b], e0 = beoff[b];
  for (int32_t p = threadIdx.x; p < rows; p += kBlock) {
    const int32_t o = perm[brows[r0 + p]];
    const int32_t len = rp[o + 1] - rp[o];
    for (int32_t t = 0; t < w; ++t) {
      int32_t slot = pad;
      double v = 0.0;
      if (t < len) {
        const int32_t e = rp[o] + t, oc = col[e];
        if (oc != o) {
          const int32_t j = iperm[oc];
          if (blk[j] == b) {
            slot = lpos[j];
          } else {
            int32_t lo = 0, hi = nh;
            while (lo < hi) {
              const int32_t mid = (lo + hi) >> 1;
              if (hl[mid] < j) lo = mid + 1; else hi = mid;
            }
            slot = rows + lo;
          }
          v = val[e];
        }
      }
      elx[e0 + t * rows + p] = slot;
      elv[e0 + t * rows + p] = v;
    }
  }
}

// Local row of every solve row: its position in the block's row list.
__global__ void k_local_rows(const int32_t* bpos, const int32_t* blk, const int32_t* boff, int64_t n, int32_t* lpos) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) lpos[g] = bpos[g] - boff[blk[g]];
}

// mx[0] = most rows, mx[1] = longest halo, mx[2] = widest ELL of any block.
__global__ void __launch_bounds__(kBlock) k_block_maxima(const int32_t* boff, const int32_t* hoff, const int32_t* bw,
                                                         int32_t nblk, int32_t* mx) {
  int32_t r = 0, hl = 0, w = 0;
  for (int32_t b = blockIdx.x * kBlock + threadIdx.x; b < nblk; b += gridDim.x * kBlock) {
    r = max(r, boff[b + 1] - boff[b]);
    hl = max(hl, hoff[b + 1] - hoff[b]);
    w = max(w, bw[b]);
  }
  auto mxop = [](int32_t a, int32_t b) { return a > b ? a : b; };
  r = block_reduce(r, mxop);
  __syncthreads();
  hl = block_reduce(hl, mxop);
  __syncthreads();
  w = block_reduce(w, mxop);
  if (threadIdx.x == 0) {
    atomicMax(&mx[0], r);
    atomicMax(&mx[1], hl);
    atomicMax(&mx[2], w);
  }
}

constexpr int32_t kMaxBlocks = 8192;         // blocks of a level (the partition's LDS histogram)
constexpr int64_t kBlkLdsMax = 64 * 1024;    // LDS of a block sweep (its rows, halo and zero slot)

// New values of A_l into the block ELL (same slots).
__global__ void k_block_values(const int32_t* rp, const int32_t* col, const double* val, const int32_t* perm,
                               const int32_t* boff, const int32_t* brows, const int32_t* bw, const int32_t* beoff,
                               int32_t nblk, double* elv) {
  const int32_t b = blockIdx.x;
  if (b >= nblk) return;
  const int32_t r0 = boff[b], rows = boff[b + 1] - r0, w = bw[b], e0 = beoff[b];
  for (int32_t p = threadIdx.x; p < rows; p += blockDim.x) {
    const int32_t o = perm[brows[r0 + p]];
    const int32_t len = rp[o + 1] - rp[o];
    for (int32_t t = 0; t < w; ++t) {
      double v = 0.0;
      if (t < len && col[rp[o] + t] != o) v = val[rp[o] + t];
      elv[e0 + t * rows + p] = v;
    }
  }
}
}  // namespace

// Jones-Plassmann colouring takes tens of rounds on the Galerkin levels (about
// the degree): the host checks the worklist every kColorBatch rounds.
constexpr int kColorBatch = 16;

void colouring(Handle& h, Level& lv, int level) {
  hipStream_t s = h.stream;
  int64_t n = lv.n;
  lv.color = (int32_t*)dalloc(h, (size_t)n * 4);
  fill_i32(lv.color, -1, n, s);
  int32_t* ncol = (int32_t*)talloc(s, 4);
  ColorKey key{(h.opt.seed ^ kColorSalt) ^ ((uint64_t)level << 32)};
  int32_t* wl = (int32_t*)talloc(s, (size_t)2 * n * 4);
  ColorLists L;
  if (n <= kColorListLevel) {
    L.list = (int32_t*)talloc(s, (size_t)n * kColorList * 4);
    L.mask = (uint64_t*)talloc(s, (size_t)n * 8);
    L.cnt = (uint8_t*)talloc(s, (size_t)n);
  }
  const int grid = std::min(blocks_for(n), 4 * kRoundGrid);
  int k = 0;
  const int64_t lds_small = small_color_lds(n, lv.nnzA);
  if (n <= kSmallColorRows && lds_small <= kSmallColorLds) {
    // the whole level, passes included, in one workgroup
    k_color_small<<<1, kDrainItems, (size_t)lds_small, s>>>(lv.arp, lv.acol, (int32_t)n, key, h.opt.color_passes,
                                                            lv.color, ncol, h.flags);
    int64_t nco = 0, fl = 0;
    ScalarRead rd[2] = {{ncol, 4, &nco}, {h.flags, 4, &fl}};
    read_scalars(h, rd, 2);
    if (fl & F_TIMEOUT) throw Error{GMG_DEVICE_ERROR, "colouring did not terminate"};
    if (fl & F_OVERFLOW) throw Error{GMG_DEVICE_ERROR, "colouring: too many colours"};
    lv.ncolors = (int32_t)nco;
    tfree(s, wl);
    if (L.list) {
      tfree(s, L.list);
      tfree(s, L.mask);
      tfree(s, L.cnt);
    }
    tfree(s, ncol);
    return;
  }
  check_hip(hipMemsetAsync(ncol, 0, 4, s), "memset");
  int32_t* rounds = fresh_rounds(h);
  if (n <= kDrainItems) {
    k_color_drain<<<1, kDrainItems, 0, s>>>(lv.arp, lv.acol, n, key, lv.color, nullptr, nullptr, L, h.flags);
  } else {
    for (;;) {
      for (int t = 0; t < kColorBatch; ++t, ++k)
        k_color_round<<<grid, kBlock, 0, s>>>(lv.arp, lv.acol, n, key, lv.color, wl + ((k + 1) % 2) * n,
                                              wl + (k % 2) * n, rounds, k, L);
      int64_t left = 0;
      ScalarRead rd[1] = {{rounds + (k - 1), 4, &left}};
      read_scalars(h, rd, 1);
      if (left == 0) break;
      if (left <= kDrainItems) {
        k_color_drain<<<1, kDrainItems, 0, s>>>(lv.arp, lv.acol, n, key, lv.color, wl + ((k - 1) % 2) * n,
                                               rounds + (k - 1), L, h.flags);
        break;
      }
      if (k + kColorBatch > kMaxRounds) throw Error{GMG_DEVICE_ERROR, "colouring did not terminate"};
    }
  }
  {
    max_i32(lv.color, n, 1, ncol, s);
    int64_t nco = 0, fl = 0;
    ScalarRead rd[2] = {{ncol, 4, &nco}, {h.flags, 4, &fl}};
    read_scalars(h, rd, 2);
    if (fl & F_TIMEOUT) throw Error{GMG_DEVICE_ERROR, "colouring did not terminate"};
    lv.ncolors = (int32_t)nco;
  }
  // iterated-greedy passes: classes of the previous colouring from the highest
  // colour down (a pass never needs more colours, so the first count bounds
  // the classes of every pass)
  if (h.opt.color_passes > 0 && lv.ncolors > 1) {
    int32_t* other = (int32_t*)talloc(s, (size_t)n * 4);
    int32_t* cur = lv.color;
    int32_t* nxt = other;
    for (int p = 0; p < h.opt.color_passes; ++p) {
      fill_i32(nxt, -1, n, s);
      for (int32_t c = lv.ncolors - 1; c >= 0; --c)
        k_ig_class<<<grid, kBlock, 0, s>>>(lv.arp, lv.acol, n, cur, nxt, c);
      std::swap(cur, nxt);
    }
    check_hip(hipMemsetAsync(ncol, 0, 4, s), "memset");
    max_i32(cur, n, 1, ncol, s);
    if (cur != lv.color) check_hip(hipMemcpyAsync(lv.color, cur, (size_t)n * 4, hipMemcpyDeviceToDevice, s), "copy");
    int64_t nco = 0;
    ScalarRead rd[1] = {{ncol, 4, &nco}};
    read_scalars(h, rd, 1);
    lv.ncolors = (int32_t)nco;
    tfree(s, other);
  }
  tfree(s, wl);
  if (L.list) {
    tfree(s, L.list);
    tfree(s, L.mask);
    tfree(s, L.cnt);
  }
  tfree(s, ncol);
}

// ------------------------------------------------------------------ block order
// The grid of a level swept in block order (gmg_options.block_min_rows): the
// two coordinate axes of largest extent (the first smallest one dropped),
// cells of side w (1 + 2^-20), w the longest coupling of A_l along those axes.
// The host reads the extents and w, decides the grid, and the device assigns
// every point its brick (two cells of a row, shifted by one cell on odd rows)
// and its cell; block_colouring chooses between them.  The level keeps the
// colour order when it has no couplings or more than kMaxGridCells cells.
constexpr double kBlockMargin = 1.0 + 1.0 / (1 << 20);
constexpr int64_t kMaxGridCells = int64_t(1) << 22;

void block_order(Handle& h, Level& lv) {
  hipStream_t s = h.stream;
  const int64_t n = lv.n;
  unsigned long long* keys = (unsigned long long*)talloc(s, 9 * 8);
  k_grid_keys_init<<<1, kWave, 0, s>>>(keys);
  k_grid_extents<<<std::min(blocks_for(n), kReduceGrid), kBlock, 0, s>>>(lv.X, lv.arp, lv.acol, n, keys);
  int64_t kv[9];
  ScalarRead rd[9];
  for (int i = 0; i < 9; ++i) rd[i] = {keys + i, 8, &kv[i]};
  read_scalars(h, rd, 9);
  tfree(s, keys);
  auto from_key = [](int64_t k) {
    const uint64_t u = (uint64_t)k;
    const uint64_t b = (u >> 63) ? (u & ~(uint64_t(1) << 63)) : ~u;
    double d;
    std::memcpy(&d, &b, 8);
    return d;
  };
  double lo[3], ext[3], d[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = from_key(kv[a]);
    ext[a] = from_key(kv[3 + a]) - lo[a];
    std::memcpy(&d[a], &kv[6 + a], 8);
  }
  int drop = 0;
  for (int a = 1; a < 3; ++a)
    if (ext[a] < ext[drop]) drop = a;
  const int a0 = drop == 0 ? 1 : 0, a1 = drop == 2 ? 1 : 2;
  const double w = std::max(d[a0], d[a1]);
  if (!(w > 0.0)) return;
  const double side = w * kBlockMargin;
  const int64_t gx = (int64_t)std::floor(ext[a0] / side) + 1, gy = (int64_t)std::floor(ext[a1] / side) + 1;
  if (gx * gy > kMaxGridCells) return;
  lv.gx = (int32_t)gx;
  lv.gy = (int32_t)gy;
  lv.bcolor = (int32_t*)dalloc(h, (size_t)n * 4);
  lv.bcell = (int32_t*)talloc(s, (size_t)n * 4);
  lv.ccell = (int32_t*)talloc(s, (size_t)n * 4);
  k_grid_cells<<<blocks_for(n), kBlock, 0, s>>>(lv.X, n, a0, a1, lo[a0], lo[a1], side, lv.gx, lv.bcell, lv.ccell);
}

// The blocks and colouring of a level swept in block order: bricks of two
// cells, or single cells where a brick would hold more than kMaxBrickRows rows
// (lv.bcell receives the block of every row, lv.bcolor its colour), then
// DSATUR in every block (its rows numbered by ascending index).  Returns false,
// with the level's grid dropped, when a block has more than kMaxCellRows rows
// or needs kMaxCellColors colours; the level then takes the colour order.
bool block_colouring(Handle& h, Level& lv) {
  hipStream_t s = h.stream;
  const int64_t n = lv.n;
  // rows per brick and per cell: bricks are the blocks unless one of them
  // holds more than kMaxBrickRows rows
  const int64_t nbrick = (int64_t)(lv.gx / 2 + 1) * lv.gy, ncells = (int64_t)lv.gx * lv.gy;
  const int64_t cap = std::max(nbrick, ncells);
  int32_t* cnt = (int32_t*)talloc(s, (size_t)(cap + 1) * 4);
  int32_t* cnt2 = (int32_t*)talloc(s, (size_t)(ncells + 1) * 4);
  int32_t* slot = (int32_t*)talloc(s, (size_t)n * 4);
  int32_t* mx = (int32_t*)talloc(s, 4 * 4);
  fill_i32(cnt, 0, nbrick, s);
  fill_i32(cnt2, 0, ncells, s);
  fill_i32(mx, 0, 4, s);
  k_count_cells2<<<blocks_for(n), kBlock, 0, s>>>(lv.bcell, lv.ccell, n, cnt, cnt2);
  max_i32(cnt, nbrick, 0, mx, s);
  max_i32(cnt2, ncells, 0, mx + 3, s);
  int64_t mb = 0, mc = 0;
  {
    ScalarRead rd[2] = {{mx, 4, &mb}, {mx + 3, 4, &mc}};
    read_scalars(h, rd, 2);
  }
  tfree(s, cnt2);
  lv.bricks = mb <= kMaxBrickRows ? 1 : 0;
  const int64_t ncell = lv.bricks ? nbrick : ncells;
  const int64_t biggest = lv.bricks ? mb : mc;
  k_block_ids<<<blocks_for(n), kBlock, 0, s>>>(lv.bcell, lv.ccell, n, lv.gx, lv.bricks, lv.bcell, lv.bcolor);
  tfree(s, lv.ccell);
  lv.ccell = nullptr;
  fill_i32(cnt, 0, ncell + 1, s);
  k_cell_slots<<<blocks_for(n), kBlock, 0, s>>>(lv.bcell, n, cnt, slot);
  bool ok = biggest <= kMaxCellRows;
  if (ok) {
    int32_t* cptr = (int32_t*)talloc(s, (size_t)(ncell + 1) * 4);
    int32_t* rows = (int32_t*)talloc(s, (size_t)n * 4);
    scan_i32(cnt, cptr, ncell, s);
    k_cell_scatter<<<blocks_for(n), kBlock, 0, s>>>(lv.bcell, n, cptr, slot, rows);
    int32_t* deg = slot;                               // reused: in-cell degree of every row
    fill_i32(cnt, 0, ncell + 1, s);                    // reused: in-cell couplings of every cell
    k_incell_degree<<<blocks_for(n), kBlock, 0, s>>>(lv.arp, lv.acol, lv.bcell, n, deg, cnt);
    int32_t* cadj = (int32_t*)talloc(s, (size_t)(ncell + 1) * 4);
    scan_i32(cnt, cadj, ncell, s);
    int32_t* adj = (int32_t*)talloc(s, (size_t)std::max<int64_t>(lv.nnzA, 1) * 4);
    lv.color = (int32_t*)dalloc(h, (size_t)n * 4);
    k_cell_dsatur<<<(unsigned)ncell, kWave, 0, s>>>(cptr, rows, deg, cadj, lv.arp, lv.acol, lv.bcell, adj, lv.color,
                                                   mx + 1, mx + 2);
    int64_t top = 0, over = 0;
    ScalarRead rd[2] = {{mx + 1, 4, &top}, {mx + 2, 4, &over}};
    read_scalars(h, rd, 2);
    ok = over == 0;
    lv.ncolors = (int32_t)top + 1;
    tfree(s, cptr);
    tfree(s, rows);
    tfree(s, cadj);
    tfree(s, adj);
  }
  tfree(s, cnt);
  tfree(s, slot);
  tfree(s, mx);
  if (!ok) {                                           // the level takes the colour order
    tfree(s, lv.bcell);
    lv.bcell = nullptr;
    lv.bcolor = nullptr;
    lv.color = nullptr;
  }
  return ok;
}

namespace {

// The block sweep's layout of a level swept in block order (its solve
// numbering already sorted by (block colour, colour, index)).  The level keeps
// the launches per sweep class when a block does not fit the block kernel.
void block_layout(Handle& h, Level& lv, int32_t C) {
  hipStream_t s = h.stream;
  const int64_t n = lv.n;
  const int64_t ncell = lv.bricks ? (int64_t)(lv.gx / 2 + 1) * lv.gy : (int64_t)lv.gx * lv.gy;   // block ids
  const int64_t H = ncell;
  int32_t* cnt = (int32_t*)talloc(s, (size_t)ncell * 4);
  fill_i32(cnt, 0, ncell, s);
  k_count_cells<<<blocks_for(n), kBlock, 0, s>>>(lv.bcell, n, cnt);
  int32_t* flag = (int32_t*)talloc(s, (size_t)(4 * H + 1) * 4);
  int32_t* vid = (int32_t*)talloc(s, (size_t)(4 * H + 1) * 4);
  k_cell_flags<<<blocks_for(4 * H), kBlock, 0, s>>>(cnt, H, lv.gx, lv.bricks, flag);
  scan_i32(flag, vid, 4 * H, s);
  int64_t bs[5];
  {
    ScalarRead rd[5];
    for (int k = 0; k < 5; ++k) rd[k] = {vid + (int64_t)k * H, 4, &bs[k]};
    read_scalars(h, rd, 5);
  }
  const int32_t nblk = (int32_t)bs[4];
  tfree(s, cnt);
  tfree(s, flag);
  BlockView<double>& B = lv.view.B;
  B = BlockView<double>();
  if (nblk <= 0 || nblk > kMaxBlocks || C > kBlkMaxColors) {
    tfree(s, vid);
    return;
  }
  // rows of every block, ascending (a stable partition of the solve rows by block)
  int32_t* blk = (int32_t*)talloc(s, (size_t)n * 4);
  k_row_block<<<blocks_for(n), kBlock, 0, s>>>(lv.perm, lv.bcell, n, vid, H, lv.gx, lv.bricks, blk);
  tfree(s, vid);
  const int nb = blocks_for(n);
  int32_t* hist = (int32_t*)talloc(s, ((size_t)nblk * nb + 1) * 4);
  int32_t* hoffs = (int32_t*)talloc(s, ((size_t)nblk * nb + 1) * 4);
  int32_t* boff = (int32_t*)dalloc(h, (size_t)(nblk + 1) * 4);
  int32_t* brows = (int32_t*)dalloc(h, (size_t)n * 4);
  int32_t* bpos = (int32_t*)talloc(s, (size_t)n * 4);
  k_color_hist<<<nb, kBlock, (size_t)nblk * 4, s>>>(blk, n, nb, nblk, hist);
  scan_i32(hist, hoffs, (int64_t)nblk * nb, s);
  k_color_place<<<nb, kBlock, 0, s>>>(blk, n, nb, hoffs, brows, bpos);
  k_color_ptr<<<blocks_for(nblk + 1), kBlock, 0, s>>>(hoffs, nb, nblk, 1, boff);
  tfree(s, hist);
  tfree(s, hoffs);
  // local row of every solve row; first local row of every colour
  int32_t* lpos = (int32_t*)talloc(s, (size_t)n * 4);
  k_local_rows<<<blocks_for(n), kBlock, 0, s>>>(bpos, blk, boff, n, lpos);
  tfree(s, bpos);
  int32_t* bcls = (int32_t*)dalloc(h, (size_t)nblk * (C + 1) * 4);
  k_block_cls<<<blocks_for((int64_t)nblk * (C + 1)), kBlock, 0, s>>>(boff, brows, lv.perm, lv.color, nblk, C, bcls);
  // halos (at most the blocks' entries each, compacted afterwards)
  int32_t* bad = (int32_t*)talloc(s, 4);
  fill_i32(bad, 0, 1, s);
  int32_t* cap = (int32_t*)talloc(s, (size_t)(nblk + 1) * 4);
  int32_t* tcap = (int32_t*)talloc(s, (size_t)(nblk + 1) * 4);
  int32_t* bw = (int32_t*)dalloc(h, (size_t)(nblk + 1) * 4);   // longest row of every block
  k_block_entries<<<blocks_for(nblk, kBlock / kWave), kBlock, 0, s>>>(lv.arp, lv.perm, brows, boff, nblk, cap, bw);
  scan_i32(cap, tcap, nblk, s);
  int32_t* tmp = (int32_t*)talloc(s, (size_t)std::max<int64_t>(lv.nnzA, 1) * 4);
  int32_t* hcnt = cap;                       // reused: distinct halo rows per block
  k_block_halo<<<nblk, kBlock, 0, s>>>(lv.arp, lv.acol, lv.perm, lv.iperm, blk, lv.bcolor, boff, brows, tmp, tcap,
                                       hcnt, bad);
  int32_t* hoff = (int32_t*)dalloc(h, (size_t)(nblk + 1) * 4);
  scan_i32(hcnt, hoff, nblk, s);
  int32_t* hlist = (int32_t*)dalloc(h, (size_t)std::max<int64_t>(lv.nnzA, 1) * 4);
  compact_long_segments(tmp, tcap, hoff, hlist, nblk, s);
  tfree(s, tmp);
  tfree(s, tcap);
  tfree(s, cap);
  // widths and the ELL offsets
  int32_t* sz = (int32_t*)talloc(s, (size_t)(nblk + 1) * 4);
  k_block_cells<<<blocks_for(nblk), kBlock, 0, s>>>(boff, bw, nblk, sz);
  int32_t* beoff = (int32_t*)dalloc(h, (size_t)(nblk + 1) * 4);
  scan_i32(sz, beoff, nblk, s);
  tfree(s, sz);
  int32_t* mx = (int32_t*)talloc(s, 3 * 4);
  fill_i32(mx, 0, 3, s);
  k_block_maxima<<<std::min(blocks_for(nblk), kReduceGrid), kBlock, 0, s>>>(boff, hoff, bw, nblk, mx);
  int64_t v[5] = {0, 0, 0, 0, 0};
  {
    ScalarRead rd[5] = {{beoff + nblk, 4, &v[0]}, {mx, 4, &v[1]}, {mx + 1, 4, &v[2]}, {mx + 2, 4, &v[3]},
                        {bad, 4, &v[4]}};
    read_scalars(h, rd, 5);
  }
  tfree(s, mx);
  tfree(s, bad);
  const int64_t total = v[0], maxrows = v[1], maxhalo = v[2], maxw = v[3];
  const int64_t lds = (maxrows + maxhalo + 1) * 8;
  const bool fits = v[4] == 0 && maxrows <= 2 * kBlkThreads && maxw <= 64 && lds <= kBlkLdsMax &&
                    maxrows + maxhalo <= kBlkGather * kBlkThreads;
  if (fits) {
    int32_t* elx = (int32_t*)dalloc(h, (size_t)std::max<int64_t>(total, 1) * 4);
    double* elv = (double*)dalloc(h, (size_t)std::max<int64_t>(total, 1) * 8);
    k_block_ell<<<nblk, kBlock, 0, s>>>(lv.arp, lv.acol, lv.aval, lv.perm, lv.iperm, blk, lpos, boff, brows, hoff,
                                        hlist, bw, beoff, elx, elv);
    B.nblk = nblk;
    for (int k = 0; k < 5; ++k) B.bstart[k] = (int32_t)bs[k];
    B.ncls = C;
    B.rows_per_thread = maxrows <= kBlkThreads ? 1 : 2;
    B.width = maxw <= 32 ? 32 : 64;
    B.lds_bytes = (int32_t)lds;
    B.boff = boff;
    B.brows = brows;
    B.bcls = bcls;
    B.hoff = hoff;
    B.hlist = hlist;
    B.bw = bw;
    B.beoff = beoff;
    B.elx = elx;
    B.elv = elv;
    int32_t* rinfo = (int32_t*)dalloc(h, (size_t)n * 4);
    uint64_t* bmask = (uint64_t*)dalloc(h, (size_t)nblk * 8);
    k_block_rowinfo<<<blocks_for(n), kBlock, 0, s>>>(lv.arp, lv.perm, lv.color, brows, n, rinfo);
    k_block_mask<<<blocks_for(nblk), kBlock, 0, s>>>(bcls, nblk, C, bmask);
    B.rinfo = rinfo;
    B.bmask = bmask;
    // headers and gather lists (stride: the largest block plus the largest halo, in wavefronts)
    const int32_t gstride = (int32_t)((maxrows + maxhalo + kWave - 1) / kWave * kWave);
    BlockHdr* hdr = (BlockHdr*)dalloc(h, (size_t)nblk * sizeof(BlockHdr));
    int32_t* glist = (int32_t*)dalloc(h, (size_t)nblk * gstride * 4);
    k_block_gather<<<nblk, kBlock, 0, s>>>(boff, brows, hoff, hlist, bw, beoff, bmask, gstride, hdr, glist);
    B.hdr = hdr;
    B.glist = glist;
    B.gstride = gstride;
    lv.blk_entries = total;
  }
  tfree(s, blk);
  tfree(s, lpos);
}

}  // namespace

void block_values(Handle& h, Level& lv) {
  const BlockView<double>& B = lv.view.B;
  if (B.nblk == 0) return;
  k_block_values<<<B.nblk, kBlock, 0, h.stream>>>(lv.arp, lv.acol, lv.aval, lv.perm, B.boff, B.brows, B.bw, B.beoff,
                                                  B.nblk, (double*)B.elv);
}

namespace {

// CSR (source rows perm[r], columns through cmap) -> SELL-64 owned by the
// handle; *maxlen receives the longest row, *slots the allocated entry slots.
// uniform_nnz > 0 (the matrix's entries): every slice gets the width of the
// longest row when that stores at most kUniformSlack times the entries.
constexpr double kUniformSlack = 1.15;

// Coarse levels of at least this many rows also get P_l^T in original row order.
constexpr int64_t kRestrictOrigRows = 65536;

SellView make_sell(Handle& h, const int32_t* perm, const int32_t* cmap, const int32_t* rp, const int32_t* col,
                   const double* val, int64_t n, double* diag, int32_t* maxlen, int64_t* slots,
                   int64_t uniform_nnz = 0) {
  hipStream_t s = h.stream;
  const int64_t ns = (n + kSlice - 1) / kSlice;
  int32_t* len = (int32_t*)dalloc(h, (size_t)(n + 1) * 4);
  int32_t* ptr = (int32_t*)dalloc(h, (size_t)(ns + 1) * 4);
  int32_t* wsz = (int32_t*)talloc(s, (size_t)(ns + 1) * 4);
  int32_t* mx = (int32_t*)talloc(s, 4);
  check_hip(hipMemsetAsync(mx, 0, 4, s), "memset");
  k_row_len_width<<<blocks_for(ns * kSlice), kBlock, 0, s>>>(perm, rp, n, ns, len, wsz, mx);
  scan_i32(wsz, ptr, ns, s);
  int64_t tot = 0, ml = 0;
  ScalarRead rd[2] = {{ptr + ns, 4, &tot}, {mx, 4, &ml}};
  read_scalars(h, rd, 2);
  int32_t uw = 0;
  if (uniform_nnz > 0 && ml > 0 && (double)(ns * kSlice * ml) <= kUniformSlack * (double)uniform_nnz) {
    fill_i32(wsz, (int32_t)(ml * kSlice), ns, s);
    scan_i32(wsz, ptr, ns, s);
    tot = ns * kSlice * ml;
    uw = (int32_t)ml;
  }
  *maxlen = (int32_t)ml;
  *slots = tot + 1;
  int32_t* scol = (int32_t*)dalloc(h, (size_t)(tot + 1) * 4);
  double* sval = (double*)dalloc(h, (size_t)(tot + 1) * 8);
  if (ml <= kSliceFillMax) {
    const int pitch = (int)ml | 1;                 // odd: rows of the tile fall in different banks
    k_sell_fill_slice<<<(int)ns, kBlock, (size_t)kSlice * pitch * 12, s>>>(perm, cmap, rp, col, val, n, ptr, scol,
                                                                          sval, diag, pitch);
  } else {
    k_sell_fill<<<blocks_for(n), kBlock, 0, s>>>(perm, cmap, rp, col, val, n, ptr, scol, sval, diag);
  }
  tfree(s, wsz);
  tfree(s, mx);
  SellView v;
  v.ptr = ptr;
  v.col = scol;
  v.val = sval;
  v.len = len;
  v.uw = uw;
  return v;
}

// Lanes per row for the lane-parallel row kernels: each lane loads up to
// kLaneEntries entries of its row per pass.
int32_t lanes_for(int32_t maxlen) {
  int32_t r = 4;
  while (r < 64 && r * kLaneEntries < maxlen) r *= 2;
  return r;
}

}  // namespace

void solve_layout(Handle& h, Level& lv, const Level* nx, const int32_t* t_rp, const int32_t* t_col,
                  const double* t_val) {
  hipStream_t s = h.stream;
  const int64_t n = lv.n;
  const int nb = blocks_for(n);
  const int C0 = lv.color ? lv.ncolors : 1;
  // sweep classes: the colours, or (block colour, colour) on a level swept in block order
  const int C = lv.bcolor ? 4 * C0 : C0;
  lv.perm = (int32_t*)dalloc(h, (size_t)n * 4);
  lv.iperm = (int32_t*)dalloc(h, (size_t)n * 4);
  int32_t* cptr = (int32_t*)dalloc(h, (size_t)(C + 1) * 4);
  int32_t *hist = nullptr, *off = nullptr;
  int32_t* stage = (int32_t*)pinned_staging((size_t)(2 * C + 1) * 4);
  if (lv.color) {
    // rows sorted by (sweep class, index); on levels small enough for the
    // single-workgroup tail by (colour, width class, index)
    const int32_t* key = lv.color;
    int32_t* cls = nullptr;
    int K = 1;
    if (lv.bcolor) {
      cls = (int32_t*)talloc(s, (size_t)n * 4);
      k_sweep_class<<<blocks_for(n), kBlock, 0, s>>>(lv.bcolor, lv.color, n, C0, cls);
      key = cls;
    } else if (n <= kTailRows && (int64_t)C * kLenKeys * 4 <= 48 * 1024) {
      K = kLenKeys;
      cls = (int32_t*)talloc(s, (size_t)n * 4);
      k_len_class<<<blocks_for(n), kBlock, 0, s>>>(lv.color, lv.arp, n, cls);
      key = cls;
    }
    const int64_t classes = (int64_t)C * K;
    hist = (int32_t*)talloc(s, ((size_t)classes * nb + 1) * 4);
    off = (int32_t*)talloc(s, ((size_t)classes * nb + 1) * 4);
    k_color_hist<<<nb, kBlock, (size_t)classes * 4, s>>>(key, n, nb, (int)classes, hist);
    scan_i32(hist, off, classes * nb, s);
    k_color_place<<<nb, kBlock, 0, s>>>(key, n, nb, off, lv.perm, lv.iperm);
    k_color_ptr<<<blocks_for(C + 1), kBlock, 0, s>>>(off, nb, C, K, cptr);
    if (cls) tfree(s, cls);
  } else {
    // the coarsest level keeps its numbering (it is solved directly)
    iota_i32(lv.perm, n, s);
    iota_i32(lv.iperm, n, s);
    stage[0] = 0;
    stage[1] = (int32_t)n;
    check_hip(hipMemcpyAsync(cptr, stage, 8, hipMemcpyHostToDevice, s), "copy");
  }
  lv.diag = (double*)dalloc(h, (size_t)n * 8);
  LevelView& v = lv.view;
  v.n = (int32_t)n;
  v.ncolors = C;
  v.cptr = cptr;
  v.A = make_sell(h, lv.perm, lv.iperm, lv.arp, lv.acol, lv.aval, n, lv.diag, &v.maxa, &lv.a_slots,
                  &lv == &h.L[0] ? lv.nnzA : 0);
  v.ra = lanes_for(v.maxa);
  v.diag = lv.diag;
  lv.x = (double*)dalloc(h, (size_t)n * 8);
  lv.b = (double*)dalloc(h, (size_t)n * 8);
  lv.r = (double*)dalloc(h, (size_t)n * 8);
  v.x = lv.x;
  v.b = lv.b;
  v.r = lv.r;
  if (lv.bcolor) {
    block_layout(h, lv, C0);
    tfree(s, lv.bcell);
    lv.bcell = nullptr;
  }
  // algorithmic bytes: 12 per entry (column + value), 28 per row (b, diagonal, row length, x write)
  lv.residual_bytes = 12.0 * (double)lv.nnzA + 28.0 * (double)n;
  int32_t* pre = nullptr;
  int32_t* cn = nullptr;
  if (lv.color) {
    pre = (int32_t*)talloc(s, (size_t)(n + 1) * 4);
    cn = (int32_t*)talloc(s, (size_t)C * 4);
    scan_i32(v.A.len, pre, n, s);
    k_color_nnz<<<blocks_for(C), kBlock, 0, s>>>(pre, cptr, C, cn);
  }
  if (nx) {
    // P: rows in this level's new numbering, columns in the next level's
    int32_t* qcol = (int32_t*)dalloc(h, (size_t)3 * n * 4);
    double* qval = (double*)dalloc(h, (size_t)3 * n * 8);
    int32_t* qcnt = (int32_t*)dalloc(h, (size_t)n * 4);
    k_p_layout<<<blocks_for(n), kBlock, 0, s>>>(lv.perm, nx->iperm, lv.pcol, lv.pval, lv.pcnt, n, qcol, qval,
                                                qcnt);
    v.q_col = qcol;
    v.q_val = qval;
    v.q_cnt = qcnt;
    // P^T: row I' = coarse row perm_c[I'], entries in ascending original fine index
    v.T = make_sell(h, nx->perm, lv.iperm, t_rp, t_col, t_val, nx->n, nullptr, &v.maxt, &lv.t_slots);
    if (nx->n >= kRestrictOrigRows) {
      int32_t mt = 0;
      v.To = make_sell(h, nullptr, lv.iperm, t_rp, t_col, t_val, nx->n, nullptr, &mt, &lv.to_slots);
      v.to_row = nx->iperm;
    }
    v.rt = lanes_for(v.maxt);
  }
  // colour ranges and per-colour entry counts (staging is reused by make_sell's reads, so copy last)
  stage = (int32_t*)pinned_staging((size_t)(2 * C + 1) * 4);
  check_hip(hipMemcpyAsync(stage, cptr, (size_t)(C + 1) * 4, hipMemcpyDeviceToHost, s), "copy");
  if (lv.color) check_hip(hipMemcpyAsync(stage + C + 1, cn, (size_t)C * 4, hipMemcpyDeviceToHost, s), "copy");
  sync(s, "solve layout");
  lv.color_ptr.assign(stage, stage + C + 1);
  lv.color_bytes.assign(C, 0.0);
  if (lv.color)
    for (int c = 0; c < C; ++c)
      lv.color_bytes[c] = 12.0 * (double)stage[C + 1 + c] + 28.0 * (double)(lv.color_ptr[c + 1] - lv.color_ptr[c]);
  tfree(s, pre);
  tfree(s, cn);
  tfree(s, hist);
  tfree(s, off);
}

// Slots per lane of the register form, with the depth of its load ring.
template <int S>
void launch_inverse(const double* L, const double* U, int32_t n, double* inv, hipStream_t s) {
  constexpr int D = S <= 4 ? 8 : (S <= 8 ? 4 : 2);
  k_coarse_inverse<S, D><<<n, kWave, 0, s>>>(L, U, n, inv);
}

void coarse_inverse(const double* L, const double* U, int64_t n64, double* inv, hipStream_t s) {
  const int32_t n = (int32_t)n64;
  switch ((n + kWave - 1) / kWave) {
    case 1: launch_inverse<1>(L, U, n, inv, s); break;
    case 2: launch_inverse<2>(L, U, n, inv, s); break;
    case 3: launch_inverse<3>(L, U, n, inv, s); break;
    case 4: launch_inverse<4>(L, U, n, inv, s); break;
    case 5: launch_inverse<5>(L, U, n, inv, s); break;
    case 6: launch_inverse<6>(L, U, n, inv, s); break;
    case 7: launch_inverse<7>(L, U, n, inv, s); break;
    case 8: launch_inverse<8>(L, U, n, inv, s); break;
    case 9: case 10: case 11: case 12: launch_inverse<12>(L, U, n, inv, s); break;
    case 13: case 14: case 15: case 16: launch_inverse<16>(L, U, n, inv, s); break;
    default:
      k_coarse_inverse_lds<<<n, kBlock, (size_t)n * 8, s>>>(L, U, n, inv);
  }
}

void coarse_factor(Handle& h, Level& lv) {
  hipStream_t s = h.stream;
  const int64_t n = lv.n;
  double* D = (double*)talloc(s, (size_t)n * n * 8);
  double* U = (double*)talloc(s, (size_t)n * n * 8);
  check_hip(hipMemsetAsync(D, 0, (size_t)n * n * 8, s), "memset");
  k_dense_scatter<<<blocks_for(n), kBlock, 0, s>>>(lv.arp, lv.acol, lv.aval, n, D);
  for (int64_t k0 = 0; k0 < n; k0 += kPanel) {
    const int kb = (int)std::min<int64_t>(kPanel, n - k0);
    k_chol_panel<<<1, 256, 0, s>>>(D, n, k0, h.flags);
    const int64_t m = n - k0 - kb;
    if (m > 0) {
      const int t = (int)((m + kPanel - 1) / kPanel);
      k_chol_update<<<dim3(t, t), 1024, 0, s>>>(D, n, k0, kb);
    }
  }
  if (!h.chol) h.chol = (double*)dalloc(h, (size_t)n * n * 8);
  if (!h.cinv) h.cinv = (double*)dalloc(h, (size_t)n * inv_ld(n) * 8);
  k_split_factor<<<blocks_for(n * n), kBlock, 0, s>>>(D, n, h.chol, U);
  coarse_inverse(h.chol, U, n, h.cinv, s);
  h.ncoarse = n;
  check_flags(h, "coarsest factorisation");
  tfree(s, D);
  tfree(s, U);
}

// New values of A_l (same pattern) into its SELL layout and diagonal.
void refresh_values(Handle& h, Level& lv) {
  const LevelView& v = lv.view;
  k_sell_fill<<<blocks_for(lv.n), kBlock, 0, h.stream>>>(lv.perm, lv.iperm, lv.arp, lv.acol, lv.aval, lv.n, v.A.ptr,
                                                         (int32_t*)v.A.col, (double*)v.A.val, lv.diag);
}

// The levels of the single-workgroup tail keep blocked ELL copies of A_l and
// P_l^T.  (The same layout for the multi-launch Gauss-Seidel kernels of the
// Galerkin levels measured no faster than SELL: their launches are bound by
// the per-launch cost.)
int ell_first_level(const Handle& h) { return h.tail_start; }

// Blocked ELL copies of A_l and P_l^T (see LevelViewT): colour widths are read
// back once to lay the colours out.
void ell_layout(Handle& h, Level& lv, const Level& nx) {
  hipStream_t s = h.stream;
  LevelView& v = lv.view;
  const int C = v.ncolors;
  int32_t* w = (int32_t*)talloc(s, (size_t)C * 4);
  k_color_width<<<C, kBlock, 0, s>>>(v.A.len, v.cptr, w);
  int32_t* stage = (int32_t*)pinned_staging((size_t)C * 4);
  check_hip(hipMemcpyAsync(stage, w, (size_t)C * 4, hipMemcpyDeviceToHost, s), "copy");
  sync(s, "tail layout");
  tfree(s, w);
  lv.e_cinfo_h.assign((size_t)4 * C, 0);
  int64_t off = 0;
  for (int c = 0; c < C; ++c) {
    const int32_t lo = lv.color_ptr[c], hi = lv.color_ptr[c + 1];
    lv.e_cinfo_h[4 * c] = lo;
    lv.e_cinfo_h[4 * c + 1] = hi;
    lv.e_cinfo_h[4 * c + 2] = stage[c];
    lv.e_cinfo_h[4 * c + 3] = (int32_t)off;
    off += (int64_t)stage[c] * (hi - lo);
  }
  lv.e_slots = off;
  v.e_slots = (int32_t)off;
  int32_t* cinfo = (int32_t*)dalloc(h, (size_t)4 * C * 4);
  int32_t* st = (int32_t*)pinned_staging((size_t)4 * C * 4);
  std::copy(lv.e_cinfo_h.begin(), lv.e_cinfo_h.end(), st);
  check_hip(hipMemcpyAsync(cinfo, st, (size_t)4 * C * 4, hipMemcpyHostToDevice, s), "copy");
  v.e_cinfo = cinfo;
  const size_t e = (size_t)std::max<int64_t>(off, 1);
  v.e_col_gs = (int32_t*)dalloc(h, e * 4);
  v.e_col = (int32_t*)dalloc(h, e * 4);
  v.e_val_gs = (double*)dalloc(h, e * 8);
  v.e_val = (double*)dalloc(h, e * 8);
  v.e_ww = (uint16_t*)dalloc(h, (size_t)lv.n * 2);
  ell_values(h, lv);
  v.e_wt = (v.maxt + kTailGroup - 1) / kTailGroup * kTailGroup;
  lv.e_tslots = (int64_t)v.e_wt * nx.n;
  v.e_tslots = (int32_t)lv.e_tslots;
  const size_t et = (size_t)std::max<int64_t>(lv.e_tslots, 1);
  int32_t* tcol = (int32_t*)dalloc(h, et * 4);
  double* tval = (double*)dalloc(h, et * 8);
  k_tail_ell_t<<<blocks_for(nx.n), kBlock, 0, s>>>(v.T, nx.n, v.e_wt, lv.n, tcol, tval);
  v.e_tcol = tcol;
  v.e_tval = tval;
  sync(s, "tail layout");   // the staging buffer is reused by the next call
}

void ell_values(Handle& h, Level& lv) {
  const LevelView& v = lv.view;
  k_tail_ell<<<blocks_for(lv.n), kBlock, 0, h.stream>>>(v.A, v.e_cinfo, v.ncolors, lv.n, (int32_t*)v.e_col_gs,
                                                        (double*)v.e_val_gs, (int32_t*)v.e_col, (double*)v.e_val,
                                                        (uint16_t*)v.e_ww);
}

}  // namespace gmg
