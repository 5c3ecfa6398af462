// Device-wide primitives: exclusive scan, fills, segmented sort/unique.
#include "gmg_internal.hpp"

namespace gmg {

namespace {

constexpr int kScanItems = 16;                         // items per thread
constexpr int kScanTile = kBlock * kScanItems;         // items per block

// Exclusive scan of one value per thread over a 256-thread block.
__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t* total) {
  __shared__ int32_t wsum[kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int32_t inc = v;
  for (int o = 1; o < kWave; o <<= 1) {
    int32_t t = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += t;
  }
  if (lane == kWave - 1) wsum[wid] = inc;
  __syncthreads();
  int32_t off = 0, tot = 0;
  for (int w = 0; w < kBlock / kWave; ++w) {
    if (w < wid) off += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ void __launch_bounds__(kBlock) k_tile_sums(const int32_t* in, int64_t n, int32_t* sums) {
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int32_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
    if (i < n) s += in[i];
  }
  int32_t tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// The last block also writes out[n] = the total.
__global__ void __launch_bounds__(kBlock) k_tile_scan(const int32_t* in, int64_t n,
                                                      const int32_t* offs, int32_t* out) {
  __shared__ int32_t tile[kScanTile];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
    tile[k * kBlock + threadIdx.x] = i < n ? in[i] : 0;
  }
  __syncthreads();
  int32_t loc[kScanItems];
  int32_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    loc[k] = s;
    s += tile[threadIdx.x * kScanItems + k];
  }
  int32_t tot;
  const int32_t off = offs ? offs[blockIdx.x] : 0;
  int32_t ex = block_exclusive_scan(s, &tot) + off;
  for (int k = 0; k < kScanItems; ++k) tile[threadIdx.x * kScanItems + k] = ex + loc[k];
  __syncthreads();
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
    if (i < n) out[i] = tile[k * kBlock + threadIdx.x];
  }
  if (threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) out[n] = off + tot;
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_iota(int32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

// Thread per segment: insertion sort, then drop repeated keys in place.
__global__ void k_segment_sort_unique(int32_t* keys, const int32_t* ptr, int32_t* cnt, int64_t nseg) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  int32_t b = ptr[s], e = ptr[s + 1];
  for (int32_t i = b + 1; i < e; ++i) {
    int32_t v = keys[i];
    int32_t j = i - 1;
    while (j >= b && keys[j] > v) {
      keys[j + 1] = keys[j];
      --j;
    }
    keys[j + 1] = v;
  }
  int32_t u = 0;
  for (int32_t i = b; i < e; ++i)
    if (u == 0 || keys[b + u - 1] != keys[i]) keys[b + u++] = keys[i];
  cnt[s] = u;
}

__global__ void k_compact_segments(const int32_t* src, const int32_t* src_ptr, const int32_t* dst_ptr,
                                   int32_t* dst, int64_t nseg) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  int32_t b = src_ptr[s], d = dst_ptr[s], len = dst_ptr[s + 1] - d;
  for (int32_t t = 0; t < len; ++t) dst[d + t] = src[b + t];
}

// Wavefront per segment (segments of many entries: block halo lists).
__global__ void k_compact_segments_wave(const int32_t* src, const int32_t* src_ptr, const int32_t* dst_ptr,
                                        int32_t* dst, int64_t nseg) {
  const int64_t sg = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (sg >= nseg) return;
  const int32_t b = src_ptr[sg], d = dst_ptr[sg], len = dst_ptr[sg + 1] - d;
  for (int32_t t = threadIdx.x & (kWave - 1); t < len; t += kWave) dst[d + t] = src[b + t];
}

}  // namespace

void scan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) {
    fill_i32(out, 0, 1, s);
    return;
  }
  int64_t nt = (n + kScanTile - 1) / kScanTile;
  if (nt == 1) {
    k_tile_scan<<<1, kBlock, 0, s>>>(in, n, nullptr, out);
  } else {
    int32_t* sums = (int32_t*)talloc(s, (size_t)nt * 4);
    int32_t* offs = (int32_t*)talloc(s, (size_t)(nt + 1) * 4);
    k_tile_sums<<<(int)nt, kBlock, 0, s>>>(in, n, sums);
    scan_i32(sums, offs, nt, s);
    k_tile_scan<<<(int)nt, kBlock, 0, s>>>(in, n, offs, out);
    tfree(s, sums);
    tfree(s, offs);
  }
}

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n > 0) k_fill<int32_t><<<blocks_for(n), kBlock, 0, s>>>(p, v, n);
}

void fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  if (n > 0) k_fill<double><<<blocks_for(n), kBlock, 0, s>>>(p, v, n);
}

void iota_i32(int32_t* p, int64_t n, hipStream_t s) {
  if (n > 0) k_iota<<<blocks_for(n), kBlock, 0, s>>>(p, n);
}

void segment_sort_unique(int32_t* keys, const int32_t* ptr, int32_t* cnt_out, int64_t nseg,
                         hipStream_t s) {
  if (nseg > 0) k_segment_sort_unique<<<blocks_for(nseg), kBlock, 0, s>>>(keys, ptr, cnt_out, nseg);
}

void compact_segments(const int32_t* src, const int32_t* src_ptr, const int32_t* dst_ptr,
                      int32_t* dst, int64_t nseg, hipStream_t s) {
  if (nseg > 0) k_compact_segments<<<blocks_for(nseg), kBlock, 0, s>>>(src, src_ptr, dst_ptr, dst, nseg);
}

void compact_long_segments(const int32_t* src, const int32_t* src_ptr, const int32_t* dst_ptr,
                           int32_t* dst, int64_t nseg, hipStream_t s) {
  if (nseg > 0)
    k_compact_segments_wave<<<blocks_for(nseg, kBlock / kWave), kBlock, 0, s>>>(src, src_ptr, dst_ptr, dst, nseg);
}

}  // namespace gmg
