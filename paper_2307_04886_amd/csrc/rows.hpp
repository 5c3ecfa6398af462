// Row sums over a SELL-64 matrix, shared by the V-cycle and Krylov kernels.
//
// Matrices (A_l and P_l^T) are in the colour-sorted SELL-64 layout: slice s
// holds rows 64s..64s+63, entry t of row r at ptr[s] + 64 t + (r mod 64).
// Every row sum adds its terms sequentially in the CSR order of the original
// row, so each row is the same floating-point computation as in the method's
// definition, in the value type V of the matrix and vectors.  Two forms:
//  - one lane per row (level 0: about 7 entries, streaming, coalesced across
//    the 64 consecutive rows of a slice), loads issued CH at a time;
//  - R lanes per row (Galerkin levels: 15-40 entries, latency-bound): the R
//    lanes load and multiply the row's entries in parallel and the first lane
//    of the group adds the products in entry order (DPP quad broadcasts for
//    R = 4, wavefront shuffles for wider groups, where DPP measured slower).
#pragma once

#include <type_traits>

#include "gmg_internal.hpp"

namespace gmg {

// One lane per row: sum_t val[t] * x[col[t]] in entry order, skipping column
// `skip`; the row's loads are issued CH at a time before any is consumed.
// Every row has at least one entry (the diagonal of A_l; the seed of a row of
// P_l^T), so the first chunk runs unconditionally and the row length and
// slice offset are loaded together.
template <int CH, class V>
__device__ __forceinline__ V row_sum_seq(const Sell<V>& A, int32_t r, const V* x, int32_t skip) {
  const int32_t len = A.len[r];
  const int32_t base = A.ptr[r / kSlice] + (r & (kSlice - 1));
  V acc = V(0);
  int32_t t0 = 0;
  do {
    int32_t j[CH];
    V v[CH], xv[CH];
    // Branch-free loads: positions past the row's end re-read its last entry
    // (and its x), so that all loads of the chunk are in flight together;
    // only entries t < len enter the sum.
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int32_t o = base + min(t0 + u, len - 1) * kSlice;
      j[u] = A.col[o];
      v[u] = A.val[o];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) xv[u] = x[j[u]];
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (t0 + u < len && j[u] != skip) acc = acc + v[u] * xv[u];
    t0 += CH;
  } while (t0 < len);
  return acc;
}

// Value of lane S of each group of 4 consecutive lanes, as seen by every lane
// of the group: a DPP quad permutation, with no LDS round trip.
template <int S>
__device__ __forceinline__ uint32_t quad_bcast(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, S * 0x55, 0xF, 0xF, false);
}

template <int S, class V>
__device__ __forceinline__ V quad_lane(V v) {
  if constexpr (sizeof(V) == 4) {
    return __builtin_bit_cast(V, quad_bcast<S>(__builtin_bit_cast(uint32_t, v)));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = quad_bcast<S>((uint32_t)u);
    const uint32_t hi = quad_bcast<S>((uint32_t)(u >> 32));
    return __builtin_bit_cast(V, ((uint64_t)hi << 32) | lo);
  }
}

// Calls f(std::integral_constant<int, S>) for S = 0 .. N-1 in order.
template <int N, class F, int S = 0>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (S < N) {
    f(std::integral_constant<int, S>{});
    static_for<N, F, S + 1>(static_cast<F&&>(f));
  }
}

// R lanes per row (R divides 64; the lanes of a group are consecutive).  All
// lanes of the wavefront must call this (shuffles); `active` marks lanes whose
// group has a row.  maxlen bounds every row length (uniform).  The result is
// valid on the group's first lane.
template <int R, class V>
__device__ __forceinline__ V row_sumR(const Sell<V>& A, int32_t r, bool active, const V* x, int32_t skip,
                                      int32_t maxlen) {
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (R - 1);
  const int lane0 = lane - sub;
  int32_t base = 0, len = 0;
  if (active) {
    base = A.ptr[r / kSlice] + (r & (kSlice - 1));
    len = A.len[r];
  }
  V acc = V(0);
  for (int32_t t0 = 0; t0 < maxlen; t0 += R * kLaneEntries) {
    int32_t j[kLaneEntries];
    V v[kLaneEntries], p[kLaneEntries];
    uint32_t mask = 0;
    // Branch-free loads, as in row_sum_seq: positions past the row's end (or
    // of an inactive group: row 0's first entry) re-read a valid entry.
#pragma unroll
    for (int k = 0; k < kLaneEntries; ++k) {
      const int32_t t = t0 + sub + R * k;
      const int32_t o = base + max(min(t, len - 1), 0) * kSlice;
      j[k] = A.col[o];
      v[k] = A.val[o];
    }
    V xv[kLaneEntries];
#pragma unroll
    for (int k = 0; k < kLaneEntries; ++k) xv[k] = x[j[k]];
#pragma unroll
    for (int k = 0; k < kLaneEntries; ++k) {
      const bool ok = (t0 + sub + R * k < len) && j[k] != skip;
      p[k] = ok ? v[k] * xv[k] : V(0);
      mask |= ok ? (1u << k) : 0u;
    }
    uint32_t m[R];
    if constexpr (R == 4) {
      V q[kLaneEntries][R];
      static_for<R>([&](auto S) {
        m[S] = quad_bcast<S>(mask);
#pragma unroll
        for (int k = 0; k < kLaneEntries; ++k) q[k][S] = quad_lane<S>(p[k]);
      });
#pragma unroll
      for (int k = 0; k < kLaneEntries; ++k)
#pragma unroll
        for (int s = 0; s < R; ++s)
          if ((m[s] >> k) & 1u) acc = acc + q[k][s];
    } else {
#pragma unroll
      for (int s = 0; s < R; ++s) m[s] = __shfl(mask, lane0 + s, kWave);
#pragma unroll
      for (int k = 0; k < kLaneEntries; ++k)
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const V q = __shfl(p[k], lane0 + s, kWave);
          if ((m[s] >> k) & 1u) acc = acc + q;
        }
    }
  }
  return acc;
}

// Block-level sum in a fixed tree order (every thread of the block calls it).
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

// Calls f(std::integral_constant<int, R>) for the lane count R of a row kernel.
template <class F>
void with_lanes(int R, F&& f) {
  switch (R) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 32: f(std::integral_constant<int, 32>{}); break;
    default: f(std::integral_constant<int, 64>{}); break;
  }
}

}  // namespace gmg
