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
//    lanes load and multiply consecutive runs of the row's entries in
//    parallel and the running sum passes from lane to lane (DPP row shifts),
//    so the terms are added in entry order.
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

// The same sum over a SELL of uniform slice width A.uw: the row's entries sit
// at addresses known from r alone, so they load with x's first gathers' index
// loads and without the row length.  Slots past the row's end hold column 0
// and value 0; their products are +-0 and leave the sum unchanged (a sum that
// starts at +0 is never -0), so the bits equal row_sum_seq's.
template <int CH, class V>
__device__ __forceinline__ V row_sum_uni(const Sell<V>& A, int32_t r, const V* x, int32_t skip) {
  const int32_t w = A.uw;
  const int64_t base = (int64_t)(r >> 6) * (kSlice * (int64_t)w) + (r & (kSlice - 1));
  V acc = V(0);
  for (int32_t t0 = 0; t0 < w; t0 += CH) {
    int32_t j[CH];
    V v[CH], xv[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int64_t o = base + (int64_t)min(t0 + u, w - 1) * kSlice;
      j[u] = A.col[o];
      v[u] = A.val[o];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) xv[u] = x[j[u]];
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (t0 + u < w && j[u] != skip) acc = acc + v[u] * xv[u];
  }
  return acc;
}

// Calls f(std::integral_constant<int, S>) for S = 0 .. N-1 in order.
template <int N, class F, int S = 0>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (S < N) {
    f(std::integral_constant<int, S>{});
    static_for<N, F, S + 1>(static_cast<F&&>(f));
  }
}

// DPP move of a 32-bit value (CTRL: a row shift or quad permutation; all
// lanes of the wavefront active).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

template <int CTRL, class V>
__device__ __forceinline__ V dpp(V v) {
  if constexpr (sizeof(V) == 4) {
    return __builtin_bit_cast(V, dpp_u32<CTRL>(__builtin_bit_cast(uint32_t, v)));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = dpp_u32<CTRL>((uint32_t)u);
    const uint32_t hi = dpp_u32<CTRL>((uint32_t)(u >> 32));
    return __builtin_bit_cast(V, ((uint64_t)hi << 32) | lo);
  }
}

// Within groups of R consecutive lanes: lane i receives lane i - 1's value
// (meaningful for every lane but the group's first).  Groups of up to 16
// lanes lie in one DPP row: a row shift by one.
template <int R, class V>
__device__ __forceinline__ V lane_up(V v) {
  if constexpr (R <= 16) return dpp<0x111>(v);
  else return __shfl_up(v, 1, kWave);
}

// The value of the group's last lane, as seen by its first lane: a quad
// permutation for R = 4, a row shift by R - 1 lanes for R = 8 and 16.
template <int R, class V>
__device__ __forceinline__ V last_to_first(V v) {
  if constexpr (R == 4) return dpp<0xFF>(v);
  else if constexpr (R <= 16) return dpp<0x100 + R - 1>(v);
  else return __shfl(v, (int)(threadIdx.x & (kWave - 1)) - (int)(threadIdx.x & (R - 1)) + R - 1, kWave);
}

// R lanes per row (R divides 64; the lanes of a group are consecutive).  All
// lanes of the wavefront must call this (cross-lane moves); `active` marks
// lanes whose group has a row.  maxlen bounds every row length.  The result is
// valid on the group's first lane.
//
// A pass covers R * kLaneEntries entries of every row: lane s of a group holds
// entries [s K, s K + K) of the pass (K = kLaneEntries).  The running sum
// starts on lane 0, which adds its products in entry order; it then moves one
// lane up (a DPP row shift) and the next lane continues, so the row is summed
// in entry order with R - 1 cross-lane moves per pass.  A wavefront stops
// after the pass that covers its longest row.
template <int R, class V>
__device__ __forceinline__ V row_sumR(const Sell<V>& A, int32_t r, bool active, const V* x, int32_t skip,
                                      int32_t maxlen) {
  constexpr int K = kLaneEntries;
  const int sub = threadIdx.x & (R - 1);
  int32_t base = 0, len = 0;
  if (active) {
    base = A.ptr[r / kSlice] + (r & (kSlice - 1));
    len = A.len[r];
  }
  V carry = V(0);
  for (int32_t t0 = 0; t0 < maxlen && __ballot(t0 < len) != 0; t0 += R * K) {
    int32_t j[K];
    V v[K], xv[K], p[K];
    bool ok[K];
    // Branch-free loads, as in row_sum_seq: positions past the row's end (or
    // of an inactive group: row 0's first entry) re-read a valid entry.
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int32_t t = t0 + sub * K + k;
      const int32_t o = base + max(min(t, len - 1), 0) * kSlice;
      j[k] = A.col[o];
      v[k] = A.val[o];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) xv[k] = x[j[k]];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ok[k] = (t0 + sub * K + k < len) && j[k] != skip;
      p[k] = v[k] * xv[k];
    }
    V in = carry, a = carry;
    static_for<R>([&](auto S) {
      a = in;
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (ok[k]) a = a + p[k];
      if constexpr (S + 1 < R) in = lane_up<R>(a);
    });
    carry = last_to_first<R>(a);
  }
  return carry;
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
