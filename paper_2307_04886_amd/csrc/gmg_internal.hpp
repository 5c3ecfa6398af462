// Internal declarations of the MI355X Gravo MG library: device helpers shared
// by the kernels, the hierarchy data layout in HBM and the host launchers.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gmg.h"

namespace gmg {

constexpr int kBlock = 256;          // threads per block of the streaming kernels
constexpr int kWave = 64;            // CDNA wavefront
constexpr int kSlice = 64;           // rows per SELL slice = one wavefront
constexpr double kDegenerateTau = 1e-12;
constexpr int64_t kMaxDenseCoarse = 4096;
constexpr uint64_t kColorSalt = 0xC2B2AE3D27D4EB4FULL;
constexpr int kRoundBatch = 8;       // rounds launched between host checks of a frontier loop
// A frontier loop whose worklist has shrunk to kDrainItems finishes in one
// workgroup of that many threads (one item per thread and round, rounds
// separated by barriers, worklists in LDS).
constexpr int kDrainItems = 1024;
constexpr int kMaxRounds = 4096;
constexpr int kRoundsSlices = 32;

// Device error flags (bit set in Handle::flags[0]).
enum : int { F_INVALID = 1, F_NOT_SPD = 2, F_OVERFLOW = 4, F_TIMEOUT = 8 };

// ------------------------------------------------------------------ device helpers
// SplitMix64 finaliser (Steele, Lea & Flood 2014), the hashed sweep/colour order key.
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Workgroups are dealt to the 8 XCDs round-robin, and each XCD has its own L2.
// The logical block index below gives every XCD one contiguous range of
// logical blocks (a bijection on [0, gridDim.x)), so blocks of neighbouring
// rows, which gather the same cache lines, share an L2.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block() {
  const uint32_t b = blockIdx.x, nb = gridDim.x;
  const uint32_t q = nb / kXcds, r = nb % kXcds, x = b % kXcds, i = b / kXcds;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

struct V3 { double x, y, z; };
__device__ inline V3 ld3(const double* X, int64_t i) { return {X[3 * i], X[3 * i + 1], X[3 * i + 2]}; }
__device__ inline V3 sub3(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
// Fixed association order ((x + y) + z); the library is built with -ffp-contract=off.
__device__ inline double dot3(V3 a, V3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ inline V3 cross3(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

template <typename T>
__device__ inline T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Adds one to cnt[key] for every lane with `on` set, with one atomic per run
// of equal keys in consecutive lanes with `on` set (rows of one cell, edges of
// one vertex, are mostly consecutive), and returns the lane's slot: the count
// before its own increment.  Every lane of the wavefront calls it.
__device__ inline int32_t run_add(int32_t* cnt, int32_t key, bool on) {
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t prev = __shfl_up(key, 1, kWave);
  const int prev_on = __shfl_up((int)on, 1, kWave);
  const bool head = on && (lane == 0 || !prev_on || prev != key);
  const uint64_t heads = __ballot(head);
  const uint64_t offs = ~__ballot(on);
  const uint64_t upto = lane == kWave - 1 ? ~0ull : (2ull << lane) - 1;   // lanes 0..lane
  int32_t base = 0;
  if (head) {
    const uint64_t after = (heads | offs) & ~upto;     // the run ends before the next head or idle lane
    const int next = after ? __builtin_ctzll(after) : kWave;
    base = atomicAdd(&cnt[key], next - lane);
  }
  const uint64_t mine = heads & upto;
  const int h = mine ? 63 - __builtin_clzll(mine) : lane;
  base = __shfl(base, h, kWave);
  return base + (lane - h);
}

// Adds val to cnt[key] for every lane with `on` set, with one atomic per run of
// equal keys in consecutive lanes with `on` set (the run's values summed in
// the wavefront first).  Every lane of the wavefront calls it.
__device__ inline void run_sum(int32_t* cnt, int32_t key, int32_t val, bool on) {
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t v = on ? val : 0;
  int32_t incl = v;
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t t = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += t;
  }
  const int32_t prev = __shfl_up(key, 1, kWave);
  const int prev_on = __shfl_up((int)on, 1, kWave);
  const bool head = on && (lane == 0 || !prev_on || prev != key);
  const uint64_t heads = __ballot(head);
  const uint64_t offs = ~__ballot(on);
  const uint64_t upto = lane == kWave - 1 ? ~0ull : (2ull << lane) - 1;   // lanes 0..lane
  const uint64_t after = (heads | offs) & ~upto;
  const int end = head ? (after ? __builtin_ctzll(after) : kWave) - 1 : lane;   // the run's last lane
  const int32_t upto_end = __shfl(incl, end, kWave);
  if (head) atomicAdd(&cnt[key], upto_end - (incl - v));
}

// Reduction of one value per thread over a block of kBlock threads (every
// thread calls it); the result is valid on thread 0.  Reductions into one
// global counter combine a block first: atomics on one address from every
// wavefront of a large grid serialise.
template <class T, class Op>
__device__ inline T block_reduce(T v, Op op) {
  __shared__ T ws[kBlock / kWave];
  for (int o = kWave / 2; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < kBlock / kWave; ++w) v = op(v, ws[w]);
  return v;
}
constexpr int kReduceGrid = 256;     // blocks of a grid-stride reduction into one counter

// Appends v to out[] (counter *cnt) for the threads where pred holds, with
// one atomic per block of kBlock threads.  Every thread of the block must call
// it.
__device__ inline void block_append(bool pred, int32_t v, int32_t* out, int32_t* cnt) {
  __shared__ int32_t wc[kBlock / kWave + 1];     // per-wavefront offsets, then the block's base
  const unsigned long long m = __ballot(pred);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == 0) wc[w] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t tot = 0;
    for (int i = 0; i < kBlock / kWave; ++i) {
      const int32_t c = wc[i];
      wc[i] = tot;
      tot += c;
    }
    wc[kBlock / kWave] = tot ? atomicAdd(cnt, tot) : 0;
  }
  __syncthreads();
  if (pred) out[wc[kBlock / kWave] + wc[w] + __popcll(m & ((1ull << lane) - 1ull))] = v;
  __syncthreads();                               // wc is reused by the next call
}

constexpr int kRoundGrid = 1024;     // blocks of a worklist round (grid-stride)

inline int blocks_for(int64_t n, int per_block = kBlock) {
  int64_t b = (n + per_block - 1) / per_block;
  return (int)(b < 1 ? 1 : b);
}

// ------------------------------------------------------------------ hierarchy layout
constexpr int kTailThreads = 1024;   // one workgroup runs the V-cycle below kTailRows
constexpr int64_t kTailRows = 4096;
constexpr int kMaxTail = 8;
constexpr int kLaneEntries = 8;      // entries per lane per pass of a lane-parallel row

// A matrix in SELL-64: entry t of row r at ptr[r/64] + 64 t + r%64.
template <class V>
struct Sell {
  const int32_t* ptr = nullptr;
  const int32_t* col = nullptr;
  const V* val = nullptr;
  const int32_t* len = nullptr;
  // > 0: every slice has this width (rows padded with column 0, value 0), so
  // entry t of row r sits at (r / 64) * 64 * uw + 64 t + r % 64
  int32_t uw = 0;
};
using SellView = Sell<double>;

// Block layout of a level swept in block order (gmg_options.block_min_rows):
// blocks are the occupied grid cells, numbered block colour by block colour.
// Block b has rows brows[boff[b] .. boff[b+1]) (solve numbering, ascending,
// so grouped by colour), its local rows of colour c start at
// bcls[b (C + 1) + c], its halo (rows of other blocks that its rows read) is
// hlist[hoff[b] .. hoff[b+1]), and entry t of its local row p, in the row's
// entry order, is at beoff[b] + t rows_b + p: elx the LDS slot of the column
// (local row, rows_b + halo position, or the zero slot rows_b + halo_b for
// the diagonal and padding up to the block's width bw[b]) and elv its value
// (0 for the diagonal and padding).  rinfo packs each local row's length and
// colour, bmask the colours present in each block.
constexpr int kBlkThreads = 256;     // threads of a block-sweep workgroup
constexpr int kBlkGather = 8;        // gather-list entries per thread (rows + halo of a block <= 2048)
struct alignas(32) BlockHdr {
  int32_t r0, rows, nh, w, e0, pad;    // first local row (boff), rows, halo rows, ELL width, first ELL element
  uint64_t mask;                       // colours with rows in the block
};
constexpr int kBlkMaxColors = 64;    // colours a block sweep handles
template <class V>
struct BlockView {
  int32_t nblk = 0;                     // 0: no block sweep (the colour classes are launched one by one)
  int32_t bstart[5] = {};               // blocks of block colour k: [bstart[k], bstart[k + 1])
  int32_t ncls = 0;                     // colours C of the level
  int32_t rows_per_thread = 1, width = 32;   // kernel shape: local rows per thread, register entries per row
  int32_t lds_bytes = 0;                // (largest block + largest halo + 1) values
  const int32_t* boff = nullptr;
  const int32_t* brows = nullptr;
  const int32_t* bcls = nullptr;
  const int32_t* hoff = nullptr;
  const int32_t* hlist = nullptr;
  const int32_t* bw = nullptr;
  const int32_t* beoff = nullptr;
  const int32_t* elx = nullptr;
  const V* elv = nullptr;
  const int32_t* rinfo = nullptr;       // per local row (boff order): row length << 8 | colour
  const uint64_t* bmask = nullptr;      // [nblk] colours with rows in the block
  // What a block sweep reads first, at addresses known from the block index
  // alone: its header and its gather list glist[b gstride + k] = the block's
  // k-th row (k < rows), then its halo rows, padded with row 0.
  const struct BlockHdr* hdr = nullptr;
  const int32_t* glist = nullptr;
  int32_t gstride = 0;

  // The same layout with values of another type (the float cycle's copy).
  template <class W>
  BlockView<W> with_values(const W* values) const {
    BlockView<W> o;
    o.nblk = nblk;
    for (int k = 0; k < 5; ++k) o.bstart[k] = bstart[k];
    o.ncls = ncls;
    o.rows_per_thread = rows_per_thread;
    o.width = width;
    o.lds_bytes = lds_bytes;
    o.boff = boff;
    o.brows = brows;
    o.bcls = bcls;
    o.hoff = hoff;
    o.hlist = hlist;
    o.bw = bw;
    o.beoff = beoff;
    o.elx = elx;
    o.elv = values;
    o.rinfo = rinfo;
    o.bmask = bmask;
    o.hdr = hdr;
    o.glist = glist;
    o.gstride = gstride;
    return o;
  }
};

// What the V-cycle kernels need of one level (device pointers, new numbering),
// with values and vectors in V (double; float for the mixed-precision cycle).
template <class V>
struct LevelViewT {
  int32_t n = 0;
  int32_t ncolors = 0;
  const int32_t* cptr = nullptr;        // device colour ranges [ncolors + 1]
  Sell<V> A;                            // A_l
  Sell<V> T;                            // P_l^T (rows: coarse points)
  // On large levels, also P_l^T with its rows in the coarse level's original
  // numbering (row k is coarse row to_row[k] of the solve numbering), which
  // is spatially ordered: the restriction takes it, so that the fine-level
  // residuals each XCD gathers form a compact band (read once, not by all).
  Sell<V> To;
  const int32_t* to_row = nullptr;
  int32_t ra = 1, rt = 1;               // lanes per row for A_l / P_l^T (power of two)
  int32_t ch = 8;                       // entries per load chunk of the one-lane-per-row kernels (level 0)
  int32_t uni = 0;                      // 1: level 0's one-lane kernels use the uniform slice width A.uw
  int32_t maxa = 0, maxt = 0;           // longest row of A_l / P_l^T
  const V* diag = nullptr;
  const int32_t* q_col = nullptr;       // P_l, SoA ELL-3 [3][n]
  const V* q_val = nullptr;
  const int32_t* q_cnt = nullptr;
  V* x = nullptr;
  V* b = nullptr;
  V* r = nullptr;
  // Levels of the single-workgroup tail (not the coarsest): A_l in per-colour
  // blocked ELL
  // (colour c: rows [lo, hi), width w a multiple of kTailGroup, element
  // offset off; entry positions from ell_col_index / ell_val_index), once with
  // its diagonal (residual) and once without (Gauss-Seidel: the diagonal's
  // column is n, its value 0), and P_l^T likewise as one segment of n_c rows
  // and width e_wt.  Padding entries have column n and value 0: the tail keeps
  // a zero at x[n] and r[n], so that every padded term is +0 and leaves the sum
  // unchanged.
  // A tail level's rows are sorted within each colour by length, longest
  // first, and e_ww[r] is the width (entries, a multiple of 4) of the longest
  // row among the 64 rows of r's wavefront (64-row chunks from the colour's
  // first row): a wavefront loads only that many entries of its rows.
  const int32_t* e_cinfo = nullptr;     // [ncolors][4]: lo, hi, w, off
  const uint16_t* e_ww = nullptr;
  const int32_t* e_col_gs = nullptr;
  const V* e_val_gs = nullptr;
  const int32_t* e_col = nullptr;
  const V* e_val = nullptr;
  const int32_t* e_tcol = nullptr;
  const V* e_tval = nullptr;
  int32_t e_wt = 0;
  int32_t e_slots = 0, e_tslots = 0;    // entries of the ELL arrays of A_l / P_l^T
  BlockView<V> B;                       // block sweep of a level swept in block order
};
using LevelView = LevelViewT<double>;

template <class V>
struct TailDescT {
  int32_t nlev = 0;                     // tail levels, the last one is the coarsest
  int32_t nu_pre = 0, nu_post = 0;
  int32_t descending_post = 0;          // 1: post-smoothing visits the colours in descending order
  // single-vector tail: byte offsets in LDS of every tail level's x (n + 1),
  // b (n), r (n + 1) and colour table (the coarsest level: x and b)
  int32_t lds_bytes = 0;
  int32_t o_x[kMaxTail] = {}, o_b[kMaxTail] = {}, o_r[kMaxTail] = {}, o_c[kMaxTail] = {}, o_w[kMaxTail] = {};
  // batched tail: LDS (elements of V) holding the tail levels' iterates
  int32_t lds_elems = 0;
  int32_t lds_off[kMaxTail] = {};       // offset of level l's x in LDS, or -1 (global)
  const double* cinv = nullptr;
  LevelViewT<V> lv[kMaxTail];
};
constexpr int32_t kTailLdsBytes = 96 * 1024;      // batched tail
constexpr int32_t kTailLdsMax = 144 * 1024;       // single-vector tail (gfx950: 160 KiB per workgroup)
constexpr int kTailGroup = 8;                     // tail ELL widths are multiples of this

// Row stride of the dense coarsest inverse: n rounded up to even, so that two
// consecutive entries of a row are one 16-byte aligned load.
inline __host__ __device__ int64_t inv_ld(int64_t n) { return (n + 1) & ~(int64_t)1; }

// Element index of entry t of row r in a tail ELL segment (first row lo, cnt
// rows, element offset off): columns in blocks of 4 entries per row, values in
// blocks of 2 (one 16-byte load per block and lane).
inline __host__ __device__ int64_t ell_col_index(int64_t off, int64_t cnt, int64_t lo, int64_t r, int64_t t) {
  return off + (t >> 2) * (cnt * 4) + (r - lo) * 4 + (t & 3);
}
inline __host__ __device__ int64_t ell_val_index(int64_t off, int64_t cnt, int64_t lo, int64_t r, int64_t t) {
  return off + (t >> 1) * (cnt * 2) + (r - lo) * 2 + (t & 1);
}

// LDS bytes of one level in the single-vector tail (value type V): x and r with
// their zero, b, the colour table and the rows' wavefront widths; the coarsest
// level keeps x and b only.  Arrays start on 16-byte boundaries.
inline int64_t tail_lds_bytes(int64_t n, int64_t ncolors, bool coarsest, int64_t vbytes) {
  auto up = [](int64_t b) { return (b + 15) & ~(int64_t)15; };
  if (coarsest) return 2 * up(n * vbytes);
  return 2 * up((n + 1) * vbytes) + up(n * vbytes) + up(ncolors * 16) + up(n * 2);
}

// Rows of a level with at most kTailRows rows are sorted within each colour by
// their width in 4-entry quads (longest first; kLenKeys classes, longer rows
// share the last), then by index.
constexpr int kLenKeys = 32;

// One variant of the V-cycle: its per-level views and its tail descriptor.
// symmetric: post-smoothing runs the colours in descending order, so that the
// cycle from a zero guess is a symmetric operator (a CG preconditioner).
template <class V>
struct Cycle {
  std::vector<LevelViewT<V>> v;
  TailDescT<V> tail;
  bool symmetric = false;
};

// One level.  "Original" arrays use the level's own point numbering (what the
// method defines and what is exported); the solve arrays use the colour-sorted
// numbering new = iperm[old] in which every colour class is a contiguous row
// range, so that a Gauss-Seidel colour sweep streams contiguous memory.
struct Level {
  int64_t n = 0;
  double* X = nullptr;                  // n x 3 AoS positions
  int32_t* erp = nullptr;               // edge CSR (symmetric, sorted, no loops)
  int32_t* ecol = nullptr;
  double* ew = nullptr;                 // edge lengths per CSR entry
  int64_t nnzE = 0;                     // exact once the build has finished
  int64_t nnzE_cap = 0;                 // allocation bound for the edge arrays
  double* scal = nullptr;               // device [e_hat, r]
  unsigned long long* stats = nullptr;  // device [fallback rows, nnz(P)], read at the end of the build
  // coarsening products (levels that are not the coarsest)
  int64_t nc = 0;                       // coarse points taken from this level
  int32_t* samples = nullptr;           // [nc] fine index of each coarse point
  int32_t* label = nullptr;             // [n]
  double* dist = nullptr;               // [n]
  uint8_t* status = nullptr;            // [n] sweep status, alive from sampling to the Voronoi step
  int32_t* pcol = nullptr;              // [3n] ELL-3, unused -1
  double* pval = nullptr;               // [3n] unused 0
  int32_t* pcnt = nullptr;              // [n]
  int32_t* tri = nullptr;               // [2n]
  int64_t nnzP = 0, fallback = 0;
  // operator A_l (original numbering)
  int32_t* arp = nullptr;
  int32_t* acol = nullptr;
  double* aval = nullptr;
  int64_t nnzA = 0;
  // Gauss-Seidel colouring
  int32_t* color = nullptr;
  int32_t ncolors = 0;
  // block order (levels swept in block order): grid cell and its parity class per row
  int32_t* bcolor = nullptr;            // [n] block colour 0..3, original numbering
  int32_t* bcell = nullptr;             // [n] cell cy * gx + cx (until the solve layout is built)
  int32_t gx = 0, gy = 0;               // grid cells along the two kept axes (block order)
  int32_t bricks = 0;                   // 1: the blocks are bricks of two cells (three colours), else cells
  int32_t* ccell = nullptr;             // cell of every point, until the blocks are chosen
  int64_t blk_entries = 0;              // elements of the block ELL
  std::vector<int32_t> color_ptr;       // host: rows [color_ptr[c], color_ptr[c+1]) in new numbering
  std::vector<double> color_bytes;      // algorithmic bytes of one colour's sweep
  double residual_bytes = 0;            // algorithmic bytes of one residual
  // solve layout (new numbering)
  int32_t* perm = nullptr;              // perm[new] = old
  int32_t* iperm = nullptr;             // iperm[old] = new
  double* diag = nullptr;
  double* x = nullptr;                  // work vectors
  double* b = nullptr;
  double* r = nullptr;
  int64_t a_slots = 0, t_slots = 0;     // SELL entry slots of A_l and P_l^T (with padding)
  int64_t to_slots = 0;                 // the same for the original-order copy of P_l^T
  LevelView view;
  // P_l^T in the original numbering (rows: coarse points, entries in ascending
  // fine index), kept for recomputing A_{l+1} when A changes
  int32_t* t_rp = nullptr;
  int32_t* t_col = nullptr;
  double* t_val = nullptr;
  int32_t galerkin_hs = 1024;           // hash slots of the numeric Galerkin pass (3/4 hold the longest row)
  // tail levels: the per-colour ELL of A_l and the ELL of P_l^T (LevelViewT)
  std::vector<int32_t> e_cinfo_h;       // host copy of view.e_cinfo
  int64_t e_slots = 0, e_tslots = 0;
};

// Preconditioned conjugate gradients (double) around a symmetric V-cycle in
// double or float; the level-0 vectors use the colour-sorted numbering.
struct Krylov {
  double* r = nullptr;
  double* r_old = nullptr;
  double* p = nullptr;
  double* q = nullptr;
  double* z = nullptr;
  double* part = nullptr;               // 3 x kNormBlocks partial sums
  double* scal = nullptr;               // device scalars (KS_* below)
  bool ready[2] = {false, false};       // cycle views built, per precision
  Cycle<double> c64;
  Cycle<float> c32;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  bool graph_failed[2] = {false, false};
};
enum : int { KS_RHO = 0, KS_BETA = 1, KS_ALPHA = 2, KS_NORM = 3, KS_BNORM = 4, KS_COUNT = 8 };

// The same CG for kBatch right-hand sides at once; vectors interleaved,
// entry (i, q) at i * kBatch + q.
constexpr int kBatch = 8;
struct Batch {
  double* x = nullptr;                  // level 0, colour-sorted numbering, [n][kBatch]
  double* b = nullptr;
  double* r = nullptr;
  double* r_old = nullptr;
  double* p = nullptr;
  double* q = nullptr;
  double* z = nullptr;
  double* part = nullptr;               // 3 x kNormBlocks x kBatch partial sums
  double* scal = nullptr;               // KS_COUNT x kBatch device scalars
  bool ready[2] = {false, false};
  Cycle<double> c64;                    // cycle views with [n][kBatch] iterates
  Cycle<float> c32;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  bool graph_failed[2] = {false, false};
};

struct Handle {
  int device = 0;
  hipStream_t stream = nullptr;         // build stream (frees are ordered on it)
  gmg_options opt{};
  std::vector<Level> L;
  int64_t ncoarse = 0;
  double* chol = nullptr;               // dense lower factor of the coarsest A
  double* cinv = nullptr;               // dense inverse of the coarsest A: inv[k inv_ld(n) + i] = (A^-1 e_k)_i
  int32_t* flags = nullptr;             // device error flags and counters
  int32_t* rounds = nullptr;            // device per-round counters of frontier loops: kRoundsSlices
                                        // slices of kMaxRounds, zeroed once per build (fresh_rounds)
  int32_t rounds_next = 0;              // slices handed out
  double* red = nullptr;                // reduction partials
  double* norm_host = nullptr;          // pinned: the solve's residual norm, written by the cycle's last kernel
  double* norm_dev = nullptr;           // its device address
  int tail_start = -1;                  // first level solved by the single-workgroup tail kernel
  Cycle<double> plain;                  // the V-cycle of the solve (Alg. 2)
  Cycle<double> noalloc64;              // the symmetric double cycle on the no-allocation scratch
  const double* noalloc_base = nullptr; // scratch address noalloc64 was made for
  Krylov kry;
  Batch bat;
  // one V-cycle plus the convergence residual, captured once and replayed
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool graph_failed = false;
  int graph_mode = 0;                   // 0 whole cycle, 1 without level-0 smoothing, 2 without residual
  std::vector<void*> allocs;
};

// Per-kernel timing with HIP events on the launch stream (measurement only;
// inactive unless gmg_timer_start was called).
// The events are passed to hipExtLaunchKernelGGL, which has the dispatch
// itself record them at the kernel's start and end.
struct KernelTimer {
  enum Kind { GS_FINEST = 0, RESIDUAL_FINEST = 1, GS_GALERKIN = 2, KINDS = 3 };
  static int active;
  struct Scope {
    hipEvent_t start = nullptr, stop = nullptr;   // null unless this launch is timed
    Scope(int kind, double bytes);
  };
};

// ------------------------------------------------------------------ host utilities
struct Error {
  int status;
  std::string msg;
};

void set_error(const std::string& m);
void check_hip(hipError_t e, const char* what);           // throws Error
void* dalloc(Handle& h, size_t bytes);                      // owned by the handle
void* talloc(hipStream_t s, size_t bytes);                  // temporary (stream-ordered)
void tfree(hipStream_t s, void* p);
void sync(hipStream_t s, const char* what);
int64_t read_i64(Handle& h, const void* dev_ptr, int bytes); // D2H of a 4- or 8-byte scalar (syncs)
void check_flags(Handle& h, const char* phase);             // throws on device error flags
void throw_flags(int32_t f, const char* phase);             // throws if f has error bits
// Several device scalars (4 or 8 bytes each) copied to the host with one synchronisation.
struct ScalarRead {
  const void* src;
  int bytes;
  int64_t* dst;
};
void read_scalars(Handle& h, const ScalarRead* items, int count);
int32_t* fresh_rounds(Handle& h);                           // zeroed per-round counters for one frontier loop
void* pinned_staging(size_t bytes);                         // per-thread pinned host buffer

// ------------------------------------------------------------------ launchers (prims.hip)
// out[0..n] = exclusive prefix sum of in[0..n-1]; out[n] = total.  Returns nothing; total stays on device.
void scan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s);
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void fill_f64(double* p, double v, int64_t n, hipStream_t s);
void iota_i32(int32_t* p, int64_t n, hipStream_t s);
void segment_sort_unique(int32_t* keys, const int32_t* ptr, int32_t* cnt_out, int64_t nseg,
                         hipStream_t s);
void compact_segments(const int32_t* src, const int32_t* src_ptr, const int32_t* dst_ptr,
                      int32_t* dst, int64_t nseg, hipStream_t s);
void compact_long_segments(const int32_t* src, const int32_t* src_ptr, const int32_t* dst_ptr,
                           int32_t* dst, int64_t nseg, hipStream_t s);  // a wavefront per segment

// ------------------------------------------------------------------ launchers (setup_graph.hip)
void validate_points(const double* X, int64_t n, int32_t* flags, hipStream_t s);
void edges_to_csr(Handle& h, Level& lv, const int32_t* edges, int64_t m);
void validate_matrix(const int32_t* rp, const int32_t* col, const double* val, int64_t n,
                     int64_t nnz, int32_t* flags, hipStream_t s);
void edge_weights(Level& lv, hipStream_t s);
void mean_edge(Handle& h, Level& lv, double rho);
int64_t sample_lfmis(Handle& h, Level& lv, int level);     // returns number of coarse points
void voronoi(Handle& h, Level& lv);
void cells_and_shift(Handle& h, Level& lv, Level& nx, bool shift, int32_t** cell_ptr,
                     int32_t** cell_mem);
void coarse_edges(Handle& h, Level& lv, Level& nx, const int32_t* cell_ptr, const int32_t* cell_mem);

// ------------------------------------------------------------------ launchers (setup_prolong.hip)
void prolongation(Handle& h, Level& lv, Level& nx);
void transpose_p(Handle& h, Level& lv, int64_t nc, int32_t** t_rp, int32_t** t_col, double** t_val);
void galerkin(Handle& h, Level& lv, Level& nx, const int32_t* t_rp, const int32_t* t_col,
              const double* t_val);
void galerkin_values(Handle& h, Level& lv, Level& nx);     // same pattern, values from the current A_l

// ------------------------------------------------------------------ launchers (setup_solve.hip)
void colouring(Handle& h, Level& lv, int level);
void block_order(Handle& h, Level& lv);                     // grid cells and block colours of a level
// DSATUR colouring in every cell of a level with a grid; false (grid dropped)
// when a cell has more than 512 rows or needs 64 colours
bool block_colouring(Handle& h, Level& lv);
void block_values(Handle& h, Level& lv);                    // block ELL values from the current A_l
void autotune(Handle& h);                                   // row-kernel shapes of the multi-launch levels (tune.hip)
void solve_layout(Handle& h, Level& lv, const Level* nx, const int32_t* t_rp, const int32_t* t_col,
                  const double* t_val);
void coarse_factor(Handle& h, Level& lv);
void refresh_values(Handle& h, Level& lv);                 // SELL values and diagonal from lv.aval
void ell_layout(Handle& h, Level& lv, const Level& nx);    // blocked ELL of A_l and P_l^T (view.e_*)
void ell_values(Handle& h, Level& lv);                     // blocked ELL values of A_l from its SELL
int ell_first_level(const Handle& h);                      // levels ell_first_level.. (not the coarsest) have it

// ------------------------------------------------------------------ launchers (solve.hip)
// V-cycle phases on one level, for V = double and V = float.  gs_sweep visits
// the colours of lv (host ranges) in ascending or descending order; `timed`
// lets the level-0 measurement timer see the launches.
template <class V>
// skip: colours at the start of the sweep already done (the first pre-sweep
// colour of a coarse level, folded into the restriction)
void gs_sweep(const LevelViewT<V>& v, const Level& lv, hipStream_t s, bool finest, bool descending, bool timed,
              int skip = 0);
template <class V>
void residual(const LevelViewT<V>& v, hipStream_t s, bool finest);
template <class V>
// first > 0: rows [0, first) of the coarse level also take their first
// pre-smoothing Gauss-Seidel update from the zero iterate
void restrict_to(const LevelViewT<V>& v, const LevelViewT<V>& c, hipStream_t s, int32_t first = 0);
template <class V>
void prolong_correct(const LevelViewT<V>& v, const LevelViewT<V>& c, hipStream_t s);
template <class V>
void coarse_solve(const double* cinv, const LevelViewT<V>& c, hipStream_t s);
template <class V>
void tail_vcycle(const TailDescT<V>& d, hipStream_t s);
template <class V>
void fill_zero(V* p, int64_t n, hipStream_t s);
void to_f32(const double* src, float* dst, int64_t n, hipStream_t s);
void permute_in(const int32_t* perm, const double* src, double* dst, int64_t n, hipStream_t s);
template <class V>
void permute_out(const int32_t* perm, const V* src, double* dst, int64_t n, hipStream_t s);
void norm2_partials(const double* v, int64_t n, double* partials, hipStream_t s);
void residual_norm(const Level& lv, const double* b, const double* x, double* res, double* partials,
                   hipStream_t s);
void finish_norm(const double* partials, double* out, hipStream_t s, double* host_out = nullptr);
void check_finite(const double* v, int64_t n, int32_t* flag, hipStream_t s);
void pattern_outer(int64_t n, const int32_t* rp, const int32_t* col, const double* u, const double* v,
                   double scale, double* out, hipStream_t s);
// batched right-hand sides (multi.hip): vectors [n][kBatch]
template <class V>
void mgs_sweep(const LevelViewT<V>& v, const Level& lv, hipStream_t s, bool descending);
template <class V>
void mresidual(const LevelViewT<V>& v, hipStream_t s);
template <class V>
void mrestrict(const LevelViewT<V>& v, const LevelViewT<V>& c, hipStream_t s);
template <class V>
void mprolong(const LevelViewT<V>& v, const LevelViewT<V>& c, hipStream_t s);
template <class V>
void mcoarse(const double* cinv, const LevelViewT<V>& c, hipStream_t s);
template <class V>
void mtail(const TailDescT<V>& d, hipStream_t s);
void mkry_init(Batch& k, int64_t n, hipStream_t s);
template <class V>
void mkry_direction(Batch& k, const V* z, int64_t n, hipStream_t s);
void mkry_step(Batch& k, const Level& l0, int32_t* flags, hipStream_t s);
void mresidual_norm(Batch& k, const Level& l0, double* out, hipStream_t s);
void mnorms(const double* v, int64_t n, double* part, double* out, hipStream_t s);
void mgather(const int32_t* perm, const double* src, int64_t n, int nq, double* dst, hipStream_t s);
template <class V>
void mscatter(const int32_t* perm, const V* src, int64_t n, int nq, double* dst, hipStream_t s);
void mzero_columns(double* x, int64_t n, unsigned mask, hipStream_t s);
// Grouped launches (multi.hip): one launch runs one step of the batched cycle
// or CG for a group of hierarchies.  A row-parallel step lists each member's
// piece as a job and every workgroup's (job, tile of kBlock elements, member)
// in a tile map; the CG steps index a job per member and run kNormBlocks
// blocks per member where the single-hierarchy kernel does, so each member
// gets that kernel's arithmetic, reductions included.  Workgroups of members
// with active[member] == 0 return at once.
struct GTile {
  int32_t job, tile, member, pad;
};
template <class V>
struct GSweepJob {                      // one colour class [r0, r1) of A_l
  Sell<V> A;
  const V* diag;
  const V* b;
  V* x;
  int32_t r0, r1;
};
template <class V>
struct GResJob {                        // r = b - A x on a level
  Sell<V> A;
  const V* b;
  const V* x;
  V* r;
  int64_t n;
};
template <class V>
struct GRestJob {                       // b_c = P^T r, x_c = 0
  Sell<V> T;
  const V* r;
  V* bc;
  V* xc;
  int64_t nc;
};
template <class V>
struct GProlJob {                       // x += P x_c
  const int32_t* q_col;
  const V* q_val;
  const int32_t* q_cnt;
  const V* xc;
  V* x;
  int64_t n;
};
template <class V>
struct GGemvJob {                       // x = A_c^-1 b
  const double* M;
  const V* b;
  V* x;
  int64_t n;
};
template <class V>
struct GKryJob {                        // a member's CG state (level 0, double) and cycle ends
  SellView A0;
  double *x, *b, *r, *r_old, *p, *q, *part, *scal;
  V* cb;                                // the cycle's level-0 right-hand side (float copy of r, or r)
  V* cx;                                // the cycle's level-0 output z
  int32_t* flags;
  int64_t n;
};
template <class V>
void gsweep(const GSweepJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s);
template <class V>
void gresidual(const GResJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s);
template <class V>
void grestrict(const GRestJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s);
template <class V>
void gprolong(const GProlJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s);
template <class V>
void ggemv(const GGemvJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s);
// one workgroup per listed member: descs[i] is member members[i]'s tail
template <class V>
void gtail(const TailDescT<V>* descs, const int32_t* members, int32_t count, int32_t lds_bytes, const int32_t* active,
           hipStream_t s);
// CG steps over the members' jobs (count of them); `tiles` cover each member's n * kBatch elements
template <class V>
void gkry_init(const GKryJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s);
template <class V>
void gcycle_start(const GKryJob<V>* jobs, const GTile* tiles, int32_t ntiles, const int32_t* active, hipStream_t s);
template <class V>
void gkry_direction(const GKryJob<V>* jobs, int32_t count, const GTile* tiles, int32_t ntiles, const int32_t* active,
                    hipStream_t s);
template <class V>
void gkry_step(const GKryJob<V>* jobs, int32_t count, const int32_t* active, hipStream_t s);
// norms of b (into KS_BNORM) or true residuals r = b - A x (into KS_NORM, r replaced)
template <class V>
void gnorms_b(const GKryJob<V>* jobs, int32_t count, const int32_t* active, hipStream_t s);
template <class V>
void gresidual_norms(const GKryJob<V>* jobs, int32_t count, const int32_t* active, hipStream_t s);
// out[m * (kBatch + 1) + q] = scal_m[which * kBatch + q], out[m * (kBatch + 1) + kBatch] = *flags_m
template <class V>
void ggather_scalars(const GKryJob<V>* jobs, int32_t count, int which, uint64_t* out, hipStream_t s);
// preconditioned CG steps (level 0, double; z in V)
void kry_init(Krylov& k, int64_t n, hipStream_t s);
template <class V>
void kry_direction(Krylov& k, const V* z, int64_t n, hipStream_t s);
void kry_step(Krylov& k, const Level& l0, double* x, int32_t* flags, hipStream_t s);
constexpr int kNormBlocks = 1024;

}  // namespace gmg
