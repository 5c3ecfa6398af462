// C ABI of the library (include/gmg.h): argument checks, the level loop of
// the hierarchy construction (Sec. 4, Alg. 1), the V-cycle driver (Alg. 1,
// Alg. 2) and the inspection exports.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <type_traits>

#include "gmg_internal.hpp"

namespace gmg {

namespace {
thread_local std::string g_last_error;

// Device memory cache.  hipFreeAsync costs 0.1-0.3 ms per call on this
// platform and a hierarchy owns a few hundred arrays, so the library keeps
// its own per-device cache of blocks in size classes (quarter steps between
// powers of two).  A block freed in stream order is tagged with its stream
// and reused only on that stream until the stream has been synchronised; a
// block of a released handle (its stream synchronised) is reusable anywhere.
// Idle blocks beyond kCacheIdleMax are returned to the driver, and so is the
// whole cache when an allocation fails.
constexpr size_t kCacheIdleMax = size_t(16) << 30;

// A free block: reusable on any stream once `settled` (every use of it on
// the device has finished), before that only on `stream`, the stream that
// freed it (which may be the null stream).
struct FreeBlock {
  void* p;
  hipStream_t stream;
  bool settled;
};

struct Cache {
  std::mutex m;
  std::multimap<size_t, FreeBlock> idle;       // size class -> free block
  std::unordered_map<void*, size_t> live;      // block -> size class
  size_t idle_bytes = 0;
};
Cache g_cache[64];

size_t size_class(size_t b) {
  b = std::max<size_t>(b, 256);
  size_t base = size_t(1) << (63 - __builtin_clzll((unsigned long long)b));
  if (b == base) return base;
  const size_t step = base / 4;
  return (b + step - 1) / step * step;
}

Cache& cache_for_current() {
  int dev = 0;
  check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) throw Error{GMG_DEVICE_ERROR, "device index out of range"};
  return g_cache[dev];
}

// Returns idle blocks to the driver until at most `keep` bytes stay idle
// (the caller holds the lock; blocks tagged with a stream are synchronised first).
void trim_locked(Cache& c, size_t keep) {
  if (c.idle_bytes <= keep) return;
  bool synced = false;
  for (auto it = c.idle.end(); it != c.idle.begin() && c.idle_bytes > keep;) {
    --it;
    if (!it->second.settled && !synced) {
      (void)hipDeviceSynchronize();
      synced = true;
    }
    (void)hipFree(it->second.p);
    c.idle_bytes -= it->first;
    it = c.idle.erase(it);
  }
}

void* cache_get(size_t bytes, hipStream_t s) {
  Cache& c = cache_for_current();
  const size_t cls = size_class(bytes);
  std::lock_guard<std::mutex> lock(c.m);
  auto range = c.idle.equal_range(cls);
  for (auto it = range.first; it != range.second; ++it) {
    if (it->second.settled || it->second.stream == s) {
      void* p = it->second.p;
      c.idle.erase(it);
      c.idle_bytes -= cls;
      c.live[p] = cls;
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, cls);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    trim_locked(c, 0);
    e = hipMalloc(&p, cls);
  }
  check_hip(e, "device allocation");
  c.live[p] = cls;
  return p;
}

// idle: every use of the block on the device has finished
void cache_put(void* p, hipStream_t s, bool idle) {
  if (!p) return;
  Cache& c = cache_for_current();
  std::lock_guard<std::mutex> lock(c.m);
  auto it = c.live.find(p);
  if (it == c.live.end()) return;
  const size_t cls = it->second;
  c.live.erase(it);
  c.idle.emplace(cls, FreeBlock{p, s, idle});
  c.idle_bytes += cls;
  if (idle) trim_locked(c, kCacheIdleMax);
}

// After a synchronisation of stream s: its freed blocks become reusable anywhere.
void cache_settle(hipStream_t s) {
  Cache& c = cache_for_current();
  std::lock_guard<std::mutex> lock(c.m);
  for (auto& kv : c.idle)
    if (kv.second.stream == s) kv.second.settled = true;
}

constexpr size_t kStaging = 1 << 16;
constexpr int kNormSpins = 1 << 22;   // host polls of a V-cycle's norm (tens of ms) before a blocking wait

double* pinned_scratch() {
  static thread_local double* p = nullptr;
  if (!p) {
    check_hip(hipHostMalloc((void**)&p, kStaging, hipHostMallocDefault), "pinned host buffer");
    std::memset(p, 0, kStaging);
  }
  return p;
}
}  // namespace

void* pinned_staging(size_t bytes) {
  if (bytes > kStaging / 2) throw Error{GMG_DEVICE_ERROR, "staging buffer too small"};
  return (char*)pinned_scratch() + kStaging / 2;      // second half: bulk staging
}

// Up to kScalarGather device scalars copied by one launch into 8-byte slots
// of the pinned buffer (lane k takes item k; a 4-byte item fills the low half).
constexpr int kScalarGather = 8;
constexpr int kScalarMark = 256;      // 8-byte slot of the pinned buffer that marks a finished read
struct ScalarGather {
  const void* src[kScalarGather];
  int32_t bytes[kScalarGather];
};

// The last launch of a read also stores seq at mark (after the values), which
// the host polls for.
__global__ void k_read_scalars(ScalarGather g, int count, uint64_t* out, uint64_t* mark, uint64_t seq) {
  const int k = (int)threadIdx.x;
  if (k >= count) return;
  const void* src = g.src[0];
  int32_t bytes = g.bytes[0];
#pragma unroll
  for (int j = 1; j < kScalarGather; ++j)
    if (j == k) {
      src = g.src[j];
      bytes = g.bytes[j];
    }
  out[k] = bytes == 4 ? (uint64_t)*(const uint32_t*)src : *(const uint64_t*)src;
  if (mark && k == 0) __hip_atomic_store(mark, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Waits until the stream's last kernel has stored seq at *mark (pinned host
// memory); after kNormSpins polls, for the stream itself (which also reports
// any device error).
void wait_mark(hipStream_t s, volatile uint64_t* mark, uint64_t seq, const char* what) {
  check_hip(hipGetLastError(), what);
  for (int spin = 0; spin < kNormSpins; ++spin) {
    if (*mark == seq) return;
    __builtin_ia32_pause();
  }
  sync(s, what);
}

void read_scalars(Handle& h, const ScalarRead* items, int count) {
  char* buf = (char*)pinned_scratch();
  static thread_local uint64_t* dbuf = nullptr;      // the buffer's device address
  static thread_local uint64_t seq = 0;
  if (!dbuf) check_hip(hipHostGetDevicePointer((void**)&dbuf, buf, 0), "pinned host buffer");
  if (count > kScalarMark) throw Error{GMG_DEVICE_ERROR, "too many scalars in one read"};
  ++seq;
  for (int k0 = 0; k0 < count; k0 += kScalarGather) {
    ScalarGather g{};
    const int c = std::min(count - k0, kScalarGather);
    for (int k = 0; k < c; ++k) {
      g.src[k] = items[k0 + k].src;
      g.bytes[k] = items[k0 + k].bytes;
    }
    const bool last = k0 + kScalarGather >= count;
    k_read_scalars<<<1, kWave, 0, h.stream>>>(g, c, dbuf + k0, last ? dbuf + kScalarMark : nullptr, seq);
  }
  wait_mark(h.stream, reinterpret_cast<volatile uint64_t*>(buf) + kScalarMark, seq, "device-to-host copy");
  for (int k = 0; k < count; ++k) {
    if (items[k].bytes == 4) {
      int32_t v;
      std::memcpy(&v, buf + 8 * k, 4);
      *items[k].dst = v;
    } else {
      std::memcpy(items[k].dst, buf + 8 * k, 8);
    }
  }
}

void throw_flags(int32_t f, const char* phase) {
  if (f & F_INVALID) throw Error{GMG_INVALID_ARGUMENT, std::string(phase) + ": invalid input"};
  if (f & F_NOT_SPD) throw Error{GMG_NOT_SPD, std::string(phase) + ": non-positive diagonal or pivot"};
  if (f & F_OVERFLOW) throw Error{GMG_DEVICE_ERROR, std::string(phase) + ": a coarse row is too dense"};
  if (f & F_TIMEOUT) throw Error{GMG_DEVICE_ERROR, std::string(phase) + ": rounds did not terminate"};
}

void set_error(const std::string& m) { g_last_error = m; }

void check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  (void)hipGetLastError();
  int st = (e == hipErrorOutOfMemory) ? GMG_OUT_OF_MEMORY : GMG_DEVICE_ERROR;
  throw Error{st, std::string(what) + ": " + hipGetErrorString(e)};
}

void* dalloc(Handle& h, size_t bytes) {
  void* p = cache_get(bytes, h.stream);
  h.allocs.push_back(p);
  return p;
}

void* talloc(hipStream_t s, size_t bytes) { return cache_get(bytes, s); }

void tfree(hipStream_t s, void* p) { cache_put(p, s, false); }

void sync(hipStream_t s, const char* what) {
  check_hip(hipGetLastError(), what);
  check_hip(hipStreamSynchronize(s), what);
}

// The next unused slice of the build's rounds arena (zeroed with the arena),
// or, once all are used, the last slice zeroed again.
int32_t* fresh_rounds(Handle& h) {
  if (h.rounds_next < kRoundsSlices) return h.rounds + (size_t)(h.rounds_next++) * kMaxRounds;
  int32_t* r = h.rounds + (size_t)(kRoundsSlices - 1) * kMaxRounds;
  check_hip(hipMemsetAsync(r, 0, (size_t)kMaxRounds * 4, h.stream), "memset");
  return r;
}

int64_t read_i64(Handle& h, const void* dev_ptr, int bytes) {
  int64_t v = 0;
  ScalarRead rd{dev_ptr, bytes, &v};
  read_scalars(h, &rd, 1);
  return v;
}

void check_flags(Handle& h, const char* phase) { throw_flags((int32_t)read_i64(h, h.flags, 4), phase); }

// ------------------------------------------------------------------ kernel timer
int KernelTimer::active = -1;

namespace {
std::vector<hipEvent_t> g_ev;        // pairs (start, stop)
size_t g_ev_used = 0;
double g_bytes = 0.0;
int64_t g_launches = 0;
}  // namespace

KernelTimer::Scope::Scope(int kind, double bytes) {
  if (kind < 0 || active != kind) return;
  if (g_ev_used + 2 > g_ev.size()) {
    for (int k = 0; k < 256; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      g_ev.push_back(e);
    }
  }
  start = g_ev[g_ev_used];
  stop = g_ev[g_ev_used + 1];
  g_ev_used += 2;
  g_bytes += bytes;
  g_launches += 1;
}

namespace {

// GMG_PROFILE_BUILD=1: host wall time of phases outside the build (diagnostics)
struct HostMark {
  bool on = std::getenv("GMG_PROFILE_BUILD") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void operator()(const char* what) {
    if (!on) return;
    auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[gmg] %-28s %8.3f ms\n", what, std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};

template <typename H>
void release(H* h) {
  if (!h) return;
  HostMark mark;
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  for (int p = 0; p < 2; ++p) {
    if (h->kry.exec[p]) (void)hipGraphExecDestroy(h->kry.exec[p]);
    if (h->kry.graph[p]) (void)hipGraphDestroy(h->kry.graph[p]);
    if (h->bat.exec[p]) (void)hipGraphExecDestroy(h->bat.exec[p]);
    if (h->bat.graph[p]) (void)hipGraphDestroy(h->bat.graph[p]);
  }
  mark("release: graphs");
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  (void)hipStreamSynchronize(h->stream);
  if (h->norm_host) (void)hipHostFree(h->norm_host);
  mark("release: capture stream");
  (void)hipStreamSynchronize(h->stream);
  try {
    cache_settle(h->stream);
    for (void* p : h->allocs) cache_put(p, h->stream, true);
  } catch (const Error&) {
  }
  mark("release: memory");
  delete h;
}

bool options_ok(const gmg_options& o) {
  return o.struct_size == (int32_t)sizeof(gmg_options) && o.coarsening_ratio > 0.0 &&
         o.coarsening_ratio < 1.0 && o.min_coarse_points >= 1 && o.max_levels >= 1 && o.nu_pre >= 0 &&
         o.nu_post >= 0 && (o.sample_order == 0 || o.sample_order == 1) && o.weighting >= 0 && o.weighting <= 2 &&
         (o.fallback_on_vertex == 0 || o.fallback_on_vertex == 1) && o.color_passes >= 0 && o.color_passes <= 64 &&
         o.block_min_rows >= 0 && (o.autotune == 0 || o.autotune == 1);
}

// The single-workgroup tail of a cycle: levels tail_start.. with their views
// and the LDS offsets of their arrays (batched layout: make_tail_batched).
template <class V>
void make_tail_at(const Handle& h, const Cycle<V>& c, int start, TailDescT<V>& t) {
  const int nl = (int)h.L.size();
  t = TailDescT<V>();
  t.nlev = nl - start;
  t.nu_pre = h.opt.nu_pre;
  t.nu_post = h.opt.nu_post;
  t.descending_post = c.symmetric ? 1 : 0;
  t.cinv = h.cinv;
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int32_t o = (int32_t)off;
    off += (bytes + 15) & ~(int64_t)15;
    return o;
  };
  for (int l = start; l < nl; ++l) {
    const LevelViewT<V>& v = c.v[l];
    const int i = l - start;
    t.lv[i] = v;
    const bool coarsest = l + 1 == nl;
    t.o_x[i] = take(((int64_t)v.n + (coarsest ? 0 : 1)) * sizeof(V));
    t.o_b[i] = take((int64_t)v.n * sizeof(V));
    if (!coarsest) {
      t.o_r[i] = take(((int64_t)v.n + 1) * sizeof(V));
      t.o_c[i] = take((int64_t)v.ncolors * 16);
      t.o_w[i] = take((int64_t)v.n * 2);
    }
  }
  if (off > kTailLdsMax) throw Error{GMG_DEVICE_ERROR, "tail LDS layout exceeds its budget"};
  t.lds_bytes = (int32_t)off;
}

template <class V>
void make_tail(const Handle& h, Cycle<V>& c) {
  make_tail_at(h, c, h.tail_start, c.tail);
}

struct PT {
  int32_t* rp = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
};

void build(Handle& h, int64_t n, const double* points, int64_t m, const int32_t* edges, const int32_t* arp,
           const int32_t* acol, const double* aval, int64_t nnz) {
  hipStream_t s = h.stream;
  const gmg_options& o = h.opt;
  const double rho = std::cbrt(1.0 / o.coarsening_ratio);
  // GMG_PROFILE_BUILD=1: synchronise after every phase and print host wall times (diagnostics)
  const bool prof = std::getenv("GMG_PROFILE_BUILD") != nullptr;
  const auto t_start = std::chrono::steady_clock::now();
  double t_last = 0.0;
  auto mark = [&](const char* what, int level) {
    if (!prof) return;
    sync(s, what);
    double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    std::fprintf(stderr, "[gmg build] level %d %-22s %8.3f ms (+%.3f)\n", level, what, t, t - t_last);
    t_last = t;
  };
  h.flags = (int32_t*)dalloc(h, 64 * 4);
  h.rounds = (int32_t*)dalloc(h, (size_t)kMaxRounds * kRoundsSlices * 4);
  h.rounds_next = 0;
  h.red = (double*)dalloc(h, (kNormBlocks + 8) * 8);
  check_hip(hipMemsetAsync(h.flags, 0, 64 * 4, s), "memset");
  check_hip(hipMemsetAsync(h.rounds, 0, (size_t)kMaxRounds * kRoundsSlices * 4, s), "memset");

  h.L.emplace_back();
  {
    Level& lv = h.L[0];
    lv.n = n;
    lv.X = (double*)dalloc(h, (size_t)n * 3 * 8);
    check_hip(hipMemcpyAsync(lv.X, points, (size_t)n * 3 * 8, hipMemcpyDeviceToDevice, s), "copy points");
    validate_points(lv.X, n, h.flags, s);
    edges_to_csr(h, lv, edges, m);
    lv.arp = (int32_t*)dalloc(h, (size_t)(n + 1) * 4);
    lv.acol = (int32_t*)dalloc(h, (size_t)nnz * 4);
    lv.aval = (double*)dalloc(h, (size_t)nnz * 8);
    lv.nnzA = nnz;
    check_hip(hipMemcpyAsync(lv.arp, arp, (size_t)(n + 1) * 4, hipMemcpyDeviceToDevice, s), "copy A");
    check_hip(hipMemcpyAsync(lv.acol, acol, (size_t)nnz * 4, hipMemcpyDeviceToDevice, s), "copy A");
    check_hip(hipMemcpyAsync(lv.aval, aval, (size_t)nnz * 8, hipMemcpyDeviceToDevice, s), "copy A");
    validate_matrix(lv.arp, lv.acol, lv.aval, n, nnz, h.flags, s);
    check_flags(h, "input");
    lv.scal = (double*)dalloc(h, 16);
    check_hip(hipMemsetAsync(lv.scal, 0, 16, s), "memset");
    lv.stats = (unsigned long long*)dalloc(h, 16);
    check_hip(hipMemsetAsync(lv.stats, 0, 16, s), "memset");
    mark("input", 0);
  }

  std::vector<PT> pts;
  // Sec. 4.2: coarsen while a level has more than min_coarse_points points.
  while (h.L.back().n > o.min_coarse_points && (int)h.L.size() < o.max_levels) {
    const int l = (int)h.L.size() - 1;
    Level nx;
    {
      Level& lv = h.L[l];
      lv.ew = (double*)dalloc(h, (size_t)(lv.nnzE_cap + 1) * 8);
      edge_weights(lv, s);
      mean_edge(h, lv, rho);
      mark("edge lengths", l);
      int64_t nc = sample_lfmis(h, lv, l);
      mark("sampling", l);
      if (nc == lv.n) {                       // no progress: this level becomes the coarsest
        tfree(s, lv.status);
        lv.status = nullptr;
        break;
      }
      voronoi(h, lv);
      mark("voronoi", l);
      int32_t *cptr = nullptr, *cmem = nullptr;
      cells_and_shift(h, lv, nx, o.shift_coarse_points != 0, &cptr, &cmem);
      coarse_edges(h, lv, nx, cptr, cmem);
      tfree(s, cptr);
      tfree(s, cmem);
      mark("cells, coarse edges", l);
      prolongation(h, lv, nx);
      mark("prolongation", l);
      PT pt;
      transpose_p(h, lv, nx.n, &pt.rp, &pt.col, &pt.val);
      mark("transpose", l);
      galerkin(h, lv, nx, pt.rp, pt.col, pt.val);
      mark("galerkin", l);
      pts.push_back(pt);
      nx.scal = (double*)dalloc(h, 16);
      check_hip(hipMemsetAsync(nx.scal, 0, 16, s), "memset");
      nx.stats = (unsigned long long*)dalloc(h, 16);
      check_hip(hipMemsetAsync(nx.stats, 0, 16, s), "memset");
    }
    h.L.push_back(nx);
  }
  Level& last = h.L.back();
  if (!last.ew) {
    last.ew = (double*)dalloc(h, (size_t)(last.nnzE_cap + 1) * 8);
    edge_weights(last, s);
  }
  last.nc = 0;                                // the coarsest level keeps no coarsening products
  last.samples = nullptr;
  last.label = nullptr;
  last.dist = nullptr;
  if (last.n > kMaxDenseCoarse) throw Error{GMG_DEGENERATE, "coarsening stalled above the dense-solve limit"};
  const int nl = (int)h.L.size();
  for (int l = 0; l + 1 < nl; ++l) {
    // block-ordered levels are coloured cell by cell; the others (and a level
    // whose cells do not allow it) take the colouring of the whole level
    bool blocked = false;
    if (l >= 1 && h.L[l].n > o.block_min_rows) {
      block_order(h, h.L[l]);
      if (h.L[l].bcolor) blocked = block_colouring(h, h.L[l]);
    }
    if (!blocked) colouring(h, h.L[l], l);
    mark("colouring", l);
  }
  solve_layout(h, h.L[nl - 1], nullptr, nullptr, nullptr, nullptr);
  for (int l = nl - 2; l >= 0; --l) {
    solve_layout(h, h.L[l], &h.L[l + 1], pts[l].rp, pts[l].col, pts[l].val);
    mark("solve layout", l);
  }
  coarse_factor(h, last);
  mark("coarse factor", nl - 1);
  // deferred sizes and statistics, with the error flags, in one synchronisation
  {
    std::vector<ScalarRead> rd;
    std::vector<int64_t> vals(1 + 3 * nl);
    rd.push_back({h.flags, 4, &vals[0]});
    for (int l = 0; l < nl; ++l) {
      rd.push_back({h.L[l].erp + h.L[l].n, 4, &vals[1 + 3 * l]});
      rd.push_back({h.L[l].stats, 8, &vals[2 + 3 * l]});
      rd.push_back({h.L[l].stats + 1, 8, &vals[3 + 3 * l]});
    }
    read_scalars(h, rd.data(), (int)rd.size());
    throw_flags((int32_t)vals[0], "build");
    for (int l = 0; l < nl; ++l) {
      h.L[l].nnzE = vals[1 + 3 * l];
      h.L[l].fallback = vals[2 + 3 * l];
      h.L[l].nnzP = vals[3 + 3 * l];
    }
  }
  // levels with few rows run their part of the V-cycle in one workgroup
  // (the coarsest level always; above it while the levels are small and their
  // arrays fit the LDS of one workgroup, counted in double)
  h.tail_start = nl - 1;
  int64_t tail_bytes = tail_lds_bytes(h.L[nl - 1].n, 0, true, 8);
  while (h.tail_start > 0 && h.L[h.tail_start - 1].n <= kTailRows && nl - (h.tail_start - 1) <= kMaxTail) {
    const Level& up = h.L[h.tail_start - 1];
    const int64_t more = tail_lds_bytes(up.n, (int64_t)up.color_ptr.size() - 1, false, 8);
    if (tail_bytes + more > kTailLdsMax) break;
    tail_bytes += more;
    --h.tail_start;
  }
  for (int l = ell_first_level(h); l + 1 < nl; ++l) ell_layout(h, h.L[l], h.L[l + 1]);
  autotune(h);
  h.plain.v.clear();
  for (int l = 0; l < nl; ++l) h.plain.v.push_back(h.L[l].view);
  h.plain.symmetric = false;
  make_tail(h, h.plain);
  sync(s, "build");
  cache_settle(s);
}

// MGI(x, b, l) of Alg. 2: pre-relax, restrict the residual, recurse from a
// zero guess, prolong and correct the pre-relaxed iterate, post-relax.  In a
// symmetric cycle the post-relaxation visits the colours in descending order.
// Rows of level l whose first pre-smoothing update the restriction into l
// performs (its first colour; 0 when level l is solved by the tail kernel or
// has no pre-smoothing).
int32_t folded_rows(const Handle& h, size_t l) {
  const Level& lv = h.L[l];
  if ((int)l >= h.tail_start || h.opt.nu_pre < 1 || lv.color_ptr.size() < 2) return 0;
  return lv.color_ptr[1];
}

template <class V>
void vcycle(Handle& h, const Cycle<V>& c, size_t l, hipStream_t s) {
  const LevelViewT<V>& v = c.v[l];
  if ((int)l == h.tail_start) {
    if (c.tail.nlev == 1) coarse_solve(h.cinv, v, s); else tail_vcycle(c.tail, s);
    return;
  }
  const LevelViewT<V>& cv = c.v[l + 1];
  const Level& lv = h.L[l];
  const bool timed = !c.symmetric;            // the solve's cycle is the measured one
  // on a coarse level the restriction into it already did the first colour
  const int skip = l > 0 && folded_rows(h, l) > 0 ? 1 : 0;
  for (int k = 0; k < h.opt.nu_pre; ++k) gs_sweep(v, lv, s, l == 0, false, timed, k == 0 ? skip : 0);
  residual(v, s, l == 0);
  restrict_to(v, cv, s, folded_rows(h, l + 1));
  vcycle(h, c, l + 1, s);
  prolong_correct(v, cv, s);
  for (int k = 0; k < h.opt.nu_post; ++k) gs_sweep(v, lv, s, l == 0, c.symmetric, timed);
}

// The part of the level-0 V-cycle between pre- and post-smoothing.
void cycle_inner(Handle& h, hipStream_t s) {
  const Cycle<double>& c = h.plain;
  residual(c.v[0], s, true);
  restrict_to(c.v[0], c.v[1], s, folded_rows(h, 1));
  vcycle(h, c, 1, s);
  prolong_correct(c.v[0], c.v[1], s);
}

// One iteration of the solve: a V-cycle and the convergence residual norm.
// Graph mode 0 replays all of it; when a level-0 kernel class is being timed
// with events (which cannot be read back from inside a graph), that class is
// launched directly around the replayed remainder (modes 1 and 2).
void run_iteration(Handle& h, hipStream_t s) {
  Level& l0 = h.L[0];
  const bool graph = h.graph_exec != nullptr;
  if (graph && h.graph_mode == 0) {
    check_hip(hipGraphLaunch(h.graph_exec, s), "graph launch");
    return;
  }
  if (graph && h.graph_mode == 1) {
    for (int k = 0; k < h.opt.nu_pre; ++k) gs_sweep(h.plain.v[0], l0, s, true, false, true);
    check_hip(hipGraphLaunch(h.graph_exec, s), "graph launch");
    for (int k = 0; k < h.opt.nu_post; ++k) gs_sweep(h.plain.v[0], l0, s, true, false, true);
  } else if (graph && h.graph_mode == 2) {
    check_hip(hipGraphLaunch(h.graph_exec, s), "graph launch");
  } else {
    vcycle(h, h.plain, 0, s);
  }
  residual_norm(l0, l0.b, l0.x, l0.r, h.red, s);
  finish_norm(h.red, h.red + kNormBlocks, s, h.norm_dev);
}

// Captures the iteration into a graph (one launch instead of ~100) on a
// private stream; it is replayed on the caller's stream.  Any failure leaves
// the handle on direct launches.
void capture_cycle(Handle& h) {
  if (h.graph_exec || h.graph_failed) return;
  if (std::getenv("GMG_DISABLE_GRAPHS")) {
    h.graph_failed = true;
    return;
  }
  if (KernelTimer::active == KernelTimer::GS_GALERKIN) return;   // those launches are inside the cycle
  if (!h.cap_stream && hipStreamCreateWithFlags(&h.cap_stream, hipStreamNonBlocking) != hipSuccess) {
    h.graph_failed = true;
    (void)hipGetLastError();
    return;
  }
  Level& l0 = h.L[0];
  const bool multi = h.L.size() > 1 && h.tail_start > 0;
  h.graph_mode = 0;
  if (multi && KernelTimer::active == KernelTimer::GS_FINEST) h.graph_mode = 1;
  if (KernelTimer::active == KernelTimer::RESIDUAL_FINEST) h.graph_mode = 2;
  HostMark mark;
  const int saved = KernelTimer::active;
  KernelTimer::active = -1;                    // no event records inside the capture
  bool ok = hipStreamBeginCapture(h.cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    if (h.graph_mode == 1) {
      cycle_inner(h, h.cap_stream);
    } else {
      vcycle(h, h.plain, 0, h.cap_stream);
      if (h.graph_mode == 0) {
        residual_norm(l0, l0.b, l0.x, l0.r, h.red, h.cap_stream);
        finish_norm(h.red, h.red + kNormBlocks, h.cap_stream, h.norm_dev);
      }
    }
    ok = hipStreamEndCapture(h.cap_stream, &h.graph) == hipSuccess && h.graph;
  }
  KernelTimer::active = saved;
  mark("capture: record");
  if (ok) ok = hipGraphInstantiate(&h.graph_exec, h.graph, nullptr, nullptr, 0) == hipSuccess;
  mark("capture: instantiate");
  if (!ok) {
    (void)hipGetLastError();
    if (h.graph) (void)hipGraphDestroy(h.graph);
    h.graph = nullptr;
    h.graph_exec = nullptr;
    h.graph_failed = true;
  }
}

// ------------------------------------------------------------------ preconditioned CG
void kry_alloc(Handle& h) {
  Krylov& k = h.kry;
  if (k.r) return;
  const int64_t n = h.L[0].n;
  k.r = (double*)dalloc(h, (size_t)n * 8);
  k.r_old = (double*)dalloc(h, (size_t)n * 8);
  k.p = (double*)dalloc(h, (size_t)n * 8);
  k.q = (double*)dalloc(h, (size_t)n * 8);
  k.z = (double*)dalloc(h, (size_t)n * 8);
  k.part = (double*)dalloc(h, (size_t)3 * kNormBlocks * 8);
  k.scal = (double*)dalloc(h, (size_t)KS_COUNT * 8);
}

float* to_f32_copy(Handle& h, const double* src, int64_t n, hipStream_t s) {
  float* d = (float*)dalloc(h, (size_t)std::max<int64_t>(n, 1) * 4);
  if (n > 0) to_f32(src, d, n, s);
  return d;
}

// The symmetric cycle in double shares the solve's level data; only level 0
// reads the CG residual and writes the preconditioned vector z.
void kry_prepare(Handle& h, Cycle<double>& c) {
  c.v = h.plain.v;
  c.symmetric = true;
  c.v[0].b = h.kry.r;
  c.v[0].x = h.kry.z;
  make_tail(h, c);
}

// The float cycle: float copies of every level's A_l, P_l^T, P_l and diagonal
// values (same SELL / ELL-3 layout and index arrays), float iterates.
void kry_prepare(Handle& h, Cycle<float>& c) {
  hipStream_t s = h.stream;
  const int nl = (int)h.L.size();
  c.v.assign(nl, LevelViewT<float>());
  c.symmetric = true;
  for (int l = 0; l < nl; ++l) {
    const LevelView& d = h.plain.v[l];
    const Level& lv = h.L[l];
    LevelViewT<float>& f = c.v[l];
    f.n = d.n;
    f.ncolors = d.ncolors;
    f.cptr = d.cptr;
    f.ra = d.ra;
    f.rt = d.rt;
    f.ch = d.ch;
    f.uni = d.uni;
    f.maxa = d.maxa;
    f.maxt = d.maxt;
    f.q_col = d.q_col;
    f.q_cnt = d.q_cnt;
    f.x = (float*)dalloc(h, (size_t)d.n * 4);
    f.b = (float*)dalloc(h, (size_t)d.n * 4);
    f.r = (float*)dalloc(h, (size_t)d.n * 4);
    if (l + 1 < nl) {                        // the coarsest level only uses b and x
      f.A = {d.A.ptr, d.A.col, to_f32_copy(h, d.A.val, lv.a_slots, s), d.A.len, d.A.uw};
      f.T = {d.T.ptr, d.T.col, to_f32_copy(h, d.T.val, lv.t_slots, s), d.T.len};
      if (d.to_row) {
        f.To = {d.To.ptr, d.To.col, to_f32_copy(h, d.To.val, lv.to_slots, s), d.To.len};
        f.to_row = d.to_row;
      }
      f.diag = to_f32_copy(h, d.diag, d.n, s);
      f.q_val = to_f32_copy(h, d.q_val, (int64_t)3 * d.n, s);
      if (d.B.nblk > 0)                      // block sweep: same layout, float values
        f.B = d.B.with_values(to_f32_copy(h, d.B.elv, lv.blk_entries, s));
      if (d.e_cinfo) {                       // a tail level
        f.e_cinfo = d.e_cinfo;
        f.e_ww = d.e_ww;
        f.e_col_gs = d.e_col_gs;
        f.e_col = d.e_col;
        f.e_tcol = d.e_tcol;
        f.e_wt = d.e_wt;
        f.e_slots = d.e_slots;
        f.e_tslots = d.e_tslots;
        f.e_val_gs = to_f32_copy(h, d.e_val_gs, lv.e_slots, s);
        f.e_val = to_f32_copy(h, d.e_val, lv.e_slots, s);
        f.e_tval = to_f32_copy(h, d.e_tval, lv.e_tslots, s);
      }
    }
  }
  make_tail(h, c);
}

template <class V>
Cycle<V>& kry_cycle(Handle& h);
template <>
Cycle<double>& kry_cycle<double>(Handle& h) { return h.kry.c64; }
template <>
Cycle<float>& kry_cycle<float>(Handle& h) { return h.kry.c32; }

template <class V>
Cycle<V>& kry_ready(Handle& h) {
  const int prec = std::is_same<V, float>::value ? 1 : 0;
  kry_alloc(h);
  Cycle<V>& c = kry_cycle<V>(h);
  if (!h.kry.ready[prec]) {
    kry_prepare(h, c);
    h.kry.ready[prec] = true;
  }
  return c;
}

// z = B r: the level-0 right-hand side is the CG residual (rounded to float
// for the float cycle), the cycle starts from zero.
template <class V>
void kry_precondition(Handle& h, const Cycle<V>& c, hipStream_t s) {
  const int64_t n = h.L[0].n;
  if (std::is_same<V, float>::value) to_f32(h.kry.r, (float*)c.v[0].b, n, s);
  fill_zero(c.v[0].x, n, s);
  vcycle(h, c, 0, s);
}

template <class V>
void kry_iteration(Handle& h, const Cycle<V>& c, hipStream_t s) {
  kry_precondition(h, c, s);
  kry_direction<V>(h.kry, c.v[0].x, h.L[0].n, s);
  kry_step(h.kry, h.L[0], h.L[0].x, h.flags, s);
}

template <class V>
void kry_capture(Handle& h, const Cycle<V>& c) {
  const int prec = std::is_same<V, float>::value ? 1 : 0;
  Krylov& k = h.kry;
  if (k.exec[prec] || k.graph_failed[prec]) return;
  if (std::getenv("GMG_DISABLE_GRAPHS")) {
    k.graph_failed[prec] = true;
    return;
  }
  if (!h.cap_stream && hipStreamCreateWithFlags(&h.cap_stream, hipStreamNonBlocking) != hipSuccess) {
    k.graph_failed[prec] = true;
    (void)hipGetLastError();
    return;
  }
  const int saved = KernelTimer::active;
  KernelTimer::active = -1;
  bool ok = hipStreamBeginCapture(h.cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    kry_iteration(h, c, h.cap_stream);
    ok = hipStreamEndCapture(h.cap_stream, &k.graph[prec]) == hipSuccess && k.graph[prec];
  }
  KernelTimer::active = saved;
  if (ok) ok = hipGraphInstantiate(&k.exec[prec], k.graph[prec], nullptr, nullptr, 0) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    if (k.graph[prec]) (void)hipGraphDestroy(k.graph[prec]);
    k.graph[prec] = nullptr;
    k.exec[prec] = nullptr;
    k.graph_failed[prec] = true;
  }
}

// True residual r = b - A x of the CG iterate into the CG residual vector;
// returns |r|.
double kry_true_residual(Handle& h, hipStream_t s) {
  Level& l0 = h.L[0];
  residual_norm(l0, l0.b, l0.x, h.kry.r, h.red, s);
  finish_norm(h.red, h.red + kNormBlocks, s);
  int64_t v = 0;
  ScalarRead rd{h.red + kNormBlocks, 8, &v};
  read_scalars(h, &rd, 1);
  double d;
  std::memcpy(&d, &v, 8);
  return d;
}

template <class V>
int pcg(Handle& h, double nb, double tol, int32_t max_iters, hipStream_t s, int32_t* iters, double* rel_out,
        double* hist) {
  Cycle<V>& c = kry_ready<V>(h);
  const int prec = std::is_same<V, float>::value ? 1 : 0;
  Krylov& k = h.kry;
  double rel = kry_true_residual(h, s) / nb;
  *iters = 0;
  *rel_out = rel;
  if (rel <= tol) return GMG_OK;
  kry_init(k, h.L[0].n, s);
  kry_capture(h, c);
  int status = GMG_NOT_CONVERGED;
  int32_t it = 0;
  while (it < max_iters) {
    if (k.exec[prec])
      check_hip(hipGraphLaunch(k.exec[prec], s), "graph launch");
    else
      kry_iteration(h, c, s);
    int64_t vals[2] = {0, 0};
    ScalarRead rd[2] = {{k.scal + KS_NORM, 8, &vals[0]}, {h.flags, 4, &vals[1]}};
    read_scalars(h, rd, 2);
    ++it;
    if (vals[1] & F_NOT_SPD) throw Error{GMG_NOT_SPD, "CG: non-positive curvature (A or the cycle not SPD)"};
    double norm;
    std::memcpy(&norm, &vals[0], 8);
    rel = norm / nb;
    if (hist) hist[it - 1] = rel;
    if (rel <= tol) {
      const double t = kry_true_residual(h, s) / nb;
      rel = t;
      if (t <= tol) {
        status = GMG_OK;
        break;
      }
    }
  }
  if (status != GMG_OK) rel = kry_true_residual(h, s) / nb;
  *iters = it;
  *rel_out = rel;
  return status;
}

// ------------------------------------------------------------------ batched right-hand sides
// The single-workgroup tail of a batched cycle: as make_tail, iterates of
// n * kBatch elements.
// LDS places of the batched tail's iterates, level by level while they fit.
template <class V>
void place_batched_tail(TailDescT<V>& t) {
  const int32_t cap = kTailLdsBytes / (int32_t)sizeof(V);
  t.lds_elems = 0;
  for (int l = 0; l < t.nlev; ++l) {
    const int32_t e = t.lv[l].n * kBatch;
    if (t.lds_elems + e <= cap) {
      t.lds_off[l] = t.lds_elems;
      t.lds_elems += e;
    } else {
      t.lds_off[l] = -1;
    }
  }
}

template <class V>
void make_tail_batched(const Handle& h, Cycle<V>& c) {
  make_tail(h, c);
  place_batched_tail(c.tail);
}

void bat_alloc(Handle& h) {
  Batch& k = h.bat;
  if (k.x) return;
  const size_t nk = (size_t)h.L[0].n * kBatch;
  for (double** v : {&k.x, &k.b, &k.r, &k.r_old, &k.p, &k.q, &k.z}) *v = (double*)dalloc(h, nk * 8);
  k.part = (double*)dalloc(h, (size_t)3 * kNormBlocks * kBatch * 8);
  k.scal = (double*)dalloc(h, (size_t)KS_COUNT * kBatch * 8);
}

// Views of a batched cycle: the matrices of the single-vector cycle of the same
// precision, iterates of n * kBatch elements.  Level 0 reads the CG residual
// (rounded to float for the float cycle) and writes z.
template <class V>
void bat_prepare(Handle& h, Cycle<V>& c, const Cycle<V>& single) {
  const int nl = (int)h.L.size();
  c.v = single.v;
  c.symmetric = true;
  for (int l = 0; l < nl; ++l) {
    const size_t nk = (size_t)c.v[l].n * kBatch;
    c.v[l].x = (V*)dalloc(h, nk * sizeof(V));
    c.v[l].b = (V*)dalloc(h, nk * sizeof(V));
    c.v[l].r = (V*)dalloc(h, nk * sizeof(V));
  }
  if (std::is_same<V, double>::value) {
    c.v[0].b = (V*)h.bat.r;
    c.v[0].x = (V*)h.bat.z;
  }
  make_tail_batched(h, c);
}

template <class V>
Cycle<V>& bat_cycle(Handle& h);
template <>
Cycle<double>& bat_cycle<double>(Handle& h) { return h.bat.c64; }
template <>
Cycle<float>& bat_cycle<float>(Handle& h) { return h.bat.c32; }

template <class V>
Cycle<V>& bat_ready(Handle& h) {
  const int prec = std::is_same<V, float>::value ? 1 : 0;
  bat_alloc(h);
  Cycle<V>& single = kry_ready<V>(h);                // matrices of that precision
  Cycle<V>& c = bat_cycle<V>(h);
  if (!h.bat.ready[prec]) {
    bat_prepare(h, c, single);
    h.bat.ready[prec] = true;
  }
  return c;
}

// The symmetric V-cycle on kBatch right-hand sides (each gets the arithmetic
// of vcycle() on a single one).
template <class V>
void mvcycle(Handle& h, const Cycle<V>& c, size_t l, hipStream_t s) {
  const LevelViewT<V>& v = c.v[l];
  if ((int)l == h.tail_start) {
    if (c.tail.nlev == 1) mcoarse(h.cinv, v, s); else mtail(c.tail, s);
    return;
  }
  const LevelViewT<V>& cv = c.v[l + 1];
  const Level& lv = h.L[l];
  for (int k = 0; k < h.opt.nu_pre; ++k) mgs_sweep(v, lv, s, false);
  mresidual(v, s);
  mrestrict(v, cv, s);
  mvcycle(h, c, l + 1, s);
  mprolong(v, cv, s);
  for (int k = 0; k < h.opt.nu_post; ++k) mgs_sweep(v, lv, s, c.symmetric);
}

template <class V>
void bat_precondition(Handle& h, const Cycle<V>& c, hipStream_t s) {
  const int64_t nk = h.L[0].n * kBatch;
  if (std::is_same<V, float>::value) to_f32(h.bat.r, (float*)c.v[0].b, nk, s);
  fill_zero(c.v[0].x, nk, s);
  mvcycle(h, c, 0, s);
}

template <class V>
void bat_iteration(Handle& h, const Cycle<V>& c, hipStream_t s) {
  bat_precondition(h, c, s);
  mkry_direction<V>(h.bat, c.v[0].x, h.L[0].n, s);
  mkry_step(h.bat, h.L[0], h.flags, s);
}

template <class V>
void bat_capture(Handle& h, const Cycle<V>& c) {
  const int prec = std::is_same<V, float>::value ? 1 : 0;
  Batch& k = h.bat;
  if (k.exec[prec] || k.graph_failed[prec]) return;
  if (std::getenv("GMG_DISABLE_GRAPHS")) {
    k.graph_failed[prec] = true;
    return;
  }
  if (!h.cap_stream && hipStreamCreateWithFlags(&h.cap_stream, hipStreamNonBlocking) != hipSuccess) {
    k.graph_failed[prec] = true;
    (void)hipGetLastError();
    return;
  }
  const int saved = KernelTimer::active;
  KernelTimer::active = -1;
  bool ok = hipStreamBeginCapture(h.cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    bat_iteration(h, c, h.cap_stream);
    ok = hipStreamEndCapture(h.cap_stream, &k.graph[prec]) == hipSuccess && k.graph[prec];
  }
  KernelTimer::active = saved;
  if (ok) ok = hipGraphInstantiate(&k.exec[prec], k.graph[prec], nullptr, nullptr, 0) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    if (k.graph[prec]) (void)hipGraphDestroy(k.graph[prec]);
    k.graph[prec] = nullptr;
    k.exec[prec] = nullptr;
    k.graph_failed[prec] = true;
  }
}

// Reads kBatch doubles (and optionally the flags) with one synchronisation.
void read_batch(Handle& h, const double* src, double* dst, int32_t* flags_out) {
  int64_t v[kBatch + 1];
  ScalarRead rd[kBatch + 1];
  for (int q = 0; q < kBatch; ++q) rd[q] = {src + q, 8, &v[q]};
  rd[kBatch] = {h.flags, 4, &v[kBatch]};
  read_scalars(h, rd, kBatch + 1);
  for (int q = 0; q < kBatch; ++q) std::memcpy(&dst[q], &v[q], 8);
  if (flags_out) *flags_out = (int32_t)v[kBatch];
}

// CG on one group of nq <= kBatch right-hand sides already in h.bat.b / h.bat.x.
// Iterates until every right-hand side with b != 0 meets tol by its recursive
// residual and then by its true residual (true residuals that fail replace the
// recursive ones and the iteration goes on).
template <class V>
int pcg_batched(Handle& h, int nq, double tol, int32_t max_iters, hipStream_t s, gmg_solve_info* infos) {
  Cycle<V>& c = bat_ready<V>(h);
  const int prec = std::is_same<V, float>::value ? 1 : 0;
  Batch& k = h.bat;
  const Level& l0 = h.L[0];
  const int64_t n = l0.n;
  double nb[kBatch], rel[kBatch], norm[kBatch];
  int32_t flags = 0;
  mnorms(k.b, n, k.part, k.scal + KS_BNORM * kBatch, s);
  read_batch(h, k.scal + KS_BNORM * kBatch, nb, &flags);
  if (flags & F_INVALID) throw Error{GMG_INVALID_ARGUMENT, "non-finite b or x"};
  unsigned zero = 0;
  for (int q = 0; q < kBatch; ++q)
    if (q >= nq || nb[q] == 0.0) zero |= 1u << q;
  if (zero) mzero_columns(k.x, n, zero, s);            // b = 0 (or padding): x = 0
  int32_t first[kBatch];
  for (int q = 0; q < kBatch; ++q) first[q] = (zero >> q) & 1u ? 0 : -1;
  auto true_residuals = [&]() {
    mresidual_norm(k, l0, k.scal + KS_NORM * kBatch, s);
    read_batch(h, k.scal + KS_NORM * kBatch, norm, nullptr);
    bool all = true;
    for (int q = 0; q < kBatch; ++q) {
      rel[q] = (zero >> q) & 1u ? 0.0 : norm[q] / nb[q];
      all = all && rel[q] <= tol;
    }
    return all;
  };
  int32_t it = 0;
  int status = GMG_OK;
  if (!true_residuals()) {
    mkry_init(k, n, s);
    bat_capture(h, c);
    status = GMG_NOT_CONVERGED;
    while (it < max_iters) {
      if (k.exec[prec])
        check_hip(hipGraphLaunch(k.exec[prec], s), "graph launch");
      else
        bat_iteration(h, c, s);
      read_batch(h, k.scal + KS_NORM * kBatch, norm, &flags);
      ++it;
      if (flags & F_NOT_SPD) throw Error{GMG_NOT_SPD, "CG: non-positive curvature (A or the cycle not SPD)"};
      bool all = true;
      for (int q = 0; q < kBatch; ++q) {
        if ((zero >> q) & 1u) continue;
        const double r = norm[q] / nb[q];
        if (r <= tol && first[q] < 0) first[q] = it;
        all = all && r <= tol;
      }
      if (all) {
        if (true_residuals()) {
          status = GMG_OK;
          break;
        }
        for (int q = 0; q < kBatch; ++q)
          if (rel[q] > tol) first[q] = -1;
      }
    }
    if (status != GMG_OK) true_residuals();
  }
  for (int q = 0; q < nq; ++q) {
    infos[q].iterations = first[q] >= 0 ? first[q] : it;
    infos[q].converged = rel[q] <= tol;
    infos[q].rel_residual = rel[q];
  }
  return status;
}

// ------------------------------------------------------------------ preconditioner without allocation
// Scratch of gmg_precondition_noalloc: the residual in the solve numbering
// (first half) and the cycle's level-0 output (second half).  Each device
// holds its own copy of the array; host code uses only the address returned
// by hipGetSymbolAddress for the current device, never the array's name.
constexpr int64_t kNoAllocMaxPoints = int64_t(1) << 21;
static __device__ __align__(256) double scratch[2 * kNoAllocMaxPoints];

std::mutex g_scratch_mutex;
double* g_scratch_dev[64] = {};

// The scratch address on the current device, looked up on the first call
// there (with that device current).
double* scratch_on_current_device() {
  int dev = 0;
  check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) throw Error{GMG_DEVICE_ERROR, "device index out of range"};
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  return g_scratch_dev[dev];
}

// z = B r with the scratch above; nothing is allocated and nothing waits.
void precondition_noalloc(Handle& h, const double* r, double* z, int32_t precision, hipStream_t s) {
  const Level& l0 = h.L[0];
  const int64_t n = l0.n;
  double* sr = scratch_on_current_device();
  permute_in(l0.perm, r, sr, n, s);
  if (precision == GMG_PRECISION_F32) {
    const Cycle<float>& c = h.kry.c32;
    to_f32(sr, (float*)c.v[0].b, n, s);
    fill_zero(c.v[0].x, n, s);
    vcycle(h, c, 0, s);
    permute_out(l0.perm, (const float*)c.v[0].x, z, n, s);
  } else {
    if (h.noalloc_base != sr) {             // host-side views of the cycle, made once per handle
      h.noalloc64.v = h.plain.v;
      h.noalloc64.symmetric = true;
      h.noalloc64.v[0].b = sr;
      h.noalloc64.v[0].x = sr + kNoAllocMaxPoints;
      make_tail(h, h.noalloc64);
      h.noalloc_base = sr;
    }
    const Cycle<double>& c = h.noalloc64;
    fill_zero(c.v[0].x, n, s);
    vcycle(h, c, 0, s);
    permute_out(l0.perm, (const double*)c.v[0].x, z, n, s);
  }
  check_hip(hipGetLastError(), "preconditioner launch");
}

// ------------------------------------------------------------------ grouped solve
// The batched CG (pcg_batched) for a group of hierarchies at once, each member
// with up to kBatch right-hand sides already in its h.bat.b / h.bat.x: every
// step of a CG iteration is one grouped launch over all members still
// iterating, and the iteration is one hipGraph for the whole group.  Each
// member goes through exactly pcg_batched's steps in pcg_batched's order (its
// true-residual checks included), so its results are bitwise those of a
// pcg_batched call on it alone.

// Device copies of host tables, returned to the block cache when the group ends.
struct DeviceTables {
  hipStream_t s;
  std::vector<void*> blocks;
  template <class T>
  T* put(const std::vector<T>& v) {
    if (v.empty()) return nullptr;
    T* d = (T*)talloc(s, v.size() * sizeof(T));
    blocks.push_back(d);
    check_hip(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s), "group tables");
    return d;
  }
  ~DeviceTables() {
    for (void* p : blocks) tfree(s, p);
  }
};

// One row-parallel step: each listed member's job and the tiles covering it.
template <class J>
struct RowStep {
  std::vector<J> jobs;
  std::vector<GTile> tiles;
  const J* djobs = nullptr;
  const GTile* dtiles = nullptr;
  void add(const J& j, int32_t member, int64_t elements) {
    const int32_t job = (int32_t)jobs.size();
    jobs.push_back(j);
    const int64_t nt = (elements + kBlock - 1) / kBlock;
    for (int64_t t = 0; t < nt; ++t) tiles.push_back(GTile{job, (int32_t)t, member, 0});
  }
  void upload(DeviceTables& d) {
    djobs = d.put(jobs);
    dtiles = d.put(tiles);
  }
  int32_t ntiles() const { return (int32_t)tiles.size(); }
};

template <class V>
struct GroupPlan {
  // the cycle as a sequence of steps, in launch order
  enum Kind { SWEEP, RESIDUAL, RESTRICT, PROLONG, GEMV, TAIL };
  struct Step {
    Kind kind;
    int32_t index;
  };
  std::vector<Step> order;
  std::vector<RowStep<GSweepJob<V>>> sweeps;
  std::vector<RowStep<GResJob<V>>> residuals;
  std::vector<RowStep<GRestJob<V>>> restricts;
  std::vector<RowStep<GProlJob<V>>> prolongs;
  RowStep<GGemvJob<V>> gemv;
  std::vector<TailDescT<V>> tails;
  std::vector<int32_t> tail_members;
  const TailDescT<V>* dtails = nullptr;
  const int32_t* dtail_members = nullptr;
  int32_t tail_lds = 0;
  // CG: one job per member, tiles over each member's n * kBatch elements
  RowStep<GKryJob<V>> kry;
  int32_t count = 0;
};

template <class V>
void build_group_plan(std::vector<Handle*>& H, GroupPlan<V>& P, DeviceTables& dt) {
  const int M = (int)H.size();
  P.count = M;
  std::vector<Cycle<V>*> C(M);
  // Each member's tail starts where all of its levels' iterates fit the
  // batched tail's LDS (the levels above it run as grouped launches, with the
  // same arithmetic as in the tail): one workgroup then carries only small
  // levels, and the group waits for the slowest member's tail once per cycle.
  std::vector<int> ts(M);
  int Lmax = 0, pre = 0, post = 0;
  for (int m = 0; m < M; ++m) {
    const Handle& h = *H[m];
    C[m] = &bat_ready<V>(*H[m]);
    const int nl = (int)h.L.size();
    int start = nl - 1;
    int64_t elems = h.L[nl - 1].n * kBatch;
    while (start > h.tail_start && elems + h.L[start - 1].n * kBatch <= kTailLdsBytes / (int64_t)sizeof(V)) {
      elems += h.L[start - 1].n * kBatch;
      --start;
    }
    ts[m] = start;
    Lmax = std::max(Lmax, start);
    pre = std::max(pre, h.opt.nu_pre);
    post = std::max(post, h.opt.nu_post);
  }
  auto classes = [&](int m, int l) { return (int)H[m]->L[l].color_ptr.size() - 1; };
  auto sweep_step = [&](int l, int sweep, bool descending) {
    int kmax = 0;
    for (int m = 0; m < M; ++m)
      if (l < ts[m]) kmax = std::max(kmax, classes(m, l));
    for (int k = 0; k < kmax; ++k) {
      RowStep<GSweepJob<V>> st;
      for (int m = 0; m < M; ++m) {
        const Handle& h = *H[m];
        const int nu = descending ? h.opt.nu_post : h.opt.nu_pre;
        const int K = l < ts[m] ? classes(m, l) : 0;
        if (sweep >= nu || k >= K) continue;
        const int c = descending ? K - 1 - k : k;      // the batched cycle is symmetric
        const int32_t r0 = h.L[l].color_ptr[c], r1 = h.L[l].color_ptr[c + 1];
        if (r1 <= r0) continue;
        const LevelViewT<V>& v = C[m]->v[l];
        st.add(GSweepJob<V>{v.A, v.diag, v.b, v.x, r0, r1}, m, (int64_t)(r1 - r0) * kBatch);
      }
      if (st.ntiles() == 0) continue;
      P.order.push_back({GroupPlan<V>::SWEEP, (int32_t)P.sweeps.size()});
      P.sweeps.push_back(std::move(st));
    }
  };
  for (int l = 0; l < Lmax; ++l) {
    for (int sweep = 0; sweep < pre; ++sweep) sweep_step(l, sweep, false);
    RowStep<GResJob<V>> rs;
    RowStep<GRestJob<V>> rt;
    for (int m = 0; m < M; ++m) {
      if (l >= ts[m]) continue;
      const LevelViewT<V>& v = C[m]->v[l];
      const LevelViewT<V>& cv = C[m]->v[l + 1];
      rs.add(GResJob<V>{v.A, v.b, v.x, v.r, v.n}, m, (int64_t)v.n * kBatch);
      rt.add(GRestJob<V>{v.T, v.r, cv.b, cv.x, cv.n}, m, (int64_t)cv.n * kBatch);
    }
    P.order.push_back({GroupPlan<V>::RESIDUAL, (int32_t)P.residuals.size()});
    P.residuals.push_back(std::move(rs));
    P.order.push_back({GroupPlan<V>::RESTRICT, (int32_t)P.restricts.size()});
    P.restricts.push_back(std::move(rt));
  }
  for (int m = 0; m < M; ++m) {
    const Handle& h = *H[m];
    const Cycle<V>& c = *C[m];
    if (ts[m] + 1 == (int)h.L.size()) {
      const LevelViewT<V>& v = c.v[ts[m]];
      P.gemv.add(GGemvJob<V>{h.cinv, v.b, v.x, v.n}, m, (int64_t)v.n * kBatch);
    } else {
      TailDescT<V> t;
      make_tail_at(h, c, ts[m], t);
      place_batched_tail(t);
      P.tails.push_back(t);
      P.tail_members.push_back(m);
      P.tail_lds = std::max(P.tail_lds, t.lds_elems * (int32_t)sizeof(V));
    }
  }
  P.order.push_back({GroupPlan<V>::TAIL, 0});
  P.order.push_back({GroupPlan<V>::GEMV, 0});
  for (int l = Lmax - 1; l >= 0; --l) {
    RowStep<GProlJob<V>> pr;
    for (int m = 0; m < M; ++m) {
      if (l >= ts[m]) continue;
      const LevelViewT<V>& v = C[m]->v[l];
      const LevelViewT<V>& cv = C[m]->v[l + 1];
      pr.add(GProlJob<V>{v.q_col, v.q_val, v.q_cnt, cv.x, v.x, v.n}, m, (int64_t)v.n * kBatch);
    }
    P.order.push_back({GroupPlan<V>::PROLONG, (int32_t)P.prolongs.size()});
    P.prolongs.push_back(std::move(pr));
    for (int sweep = 0; sweep < post; ++sweep) sweep_step(l, sweep, true);
  }
  for (int m = 0; m < M; ++m) {
    Handle& h = *H[m];
    Batch& k = h.bat;
    const int64_t n = h.L[0].n;
    P.kry.add(GKryJob<V>{h.L[0].view.A, k.x, k.b, k.r, k.r_old, k.p, k.q, k.part, k.scal, C[m]->v[0].b,
                         C[m]->v[0].x, h.flags, n},
              m, n * kBatch);
  }
  for (auto& st : P.sweeps) st.upload(dt);
  for (auto& st : P.residuals) st.upload(dt);
  for (auto& st : P.restricts) st.upload(dt);
  for (auto& st : P.prolongs) st.upload(dt);
  P.gemv.upload(dt);
  P.kry.upload(dt);
  P.dtails = dt.put(P.tails);
  P.dtail_members = dt.put(P.tail_members);
}

// One CG iteration of every member with active[m] != 0 (bat_iteration).
template <class V>
void group_iteration(const GroupPlan<V>& P, const int32_t* active, hipStream_t s) {
  gcycle_start(P.kry.djobs, P.kry.dtiles, P.kry.ntiles(), active, s);
  for (const auto& st : P.order) {
    switch (st.kind) {
      case GroupPlan<V>::SWEEP: {
        const auto& r = P.sweeps[st.index];
        gsweep(r.djobs, r.dtiles, r.ntiles(), active, s);
        break;
      }
      case GroupPlan<V>::RESIDUAL: {
        const auto& r = P.residuals[st.index];
        gresidual(r.djobs, r.dtiles, r.ntiles(), active, s);
        break;
      }
      case GroupPlan<V>::RESTRICT: {
        const auto& r = P.restricts[st.index];
        grestrict(r.djobs, r.dtiles, r.ntiles(), active, s);
        break;
      }
      case GroupPlan<V>::PROLONG: {
        const auto& r = P.prolongs[st.index];
        gprolong(r.djobs, r.dtiles, r.ntiles(), active, s);
        break;
      }
      case GroupPlan<V>::GEMV:
        ggemv(P.gemv.djobs, P.gemv.dtiles, P.gemv.ntiles(), active, s);
        break;
      case GroupPlan<V>::TAIL:
        gtail(P.dtails, P.dtail_members, (int32_t)P.tails.size(), P.tail_lds, active, s);
        break;
    }
  }
  gkry_direction(P.kry.djobs, P.count, P.kry.dtiles, P.kry.ntiles(), active, s);
  gkry_step(P.kry.djobs, P.count, active, s);
}

// Pinned host memory for the group's masks and scalar reads.
struct PinnedBuffer {
  void* p = nullptr;
  explicit PinnedBuffer(size_t bytes) {
    check_hip(hipHostMalloc(&p, bytes, hipHostMallocDefault), "pinned host buffer");
  }
  ~PinnedBuffer() {
    if (p) (void)hipHostFree(p);
  }
};

struct GroupGraph {
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~GroupGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// nq[m] right-hand sides of member m (1..kBatch); infos[m * kBatch + q]; status[m].
template <class V>
void pcg_grouped(std::vector<Handle*>& H, const std::vector<int>& nq, double tol, int32_t max_iters, hipStream_t s,
                 gmg_solve_info* infos, int32_t* status) {
  const int M = (int)H.size();
  DeviceTables dt{s, {}};
  GroupPlan<V> P;
  build_group_plan<V>(H, P, dt);
  // masks (iterating, checking) and the gathered scalars, in pinned memory
  const size_t mask_bytes = (size_t)M * 4, read_elems = (size_t)M * (kBatch + 1);
  PinnedBuffer pin(2 * mask_bytes + read_elems * 8);
  int32_t* h_iter = (int32_t*)pin.p;
  int32_t* h_check = h_iter + M;
  uint64_t* h_read = (uint64_t*)((char*)pin.p + 2 * mask_bytes);
  uint64_t* d_read = nullptr;
  check_hip(hipHostGetDevicePointer((void**)&d_read, h_read, 0), "pinned host buffer");
  int32_t* d_masks = (int32_t*)talloc(s, 2 * mask_bytes);
  dt.blocks.push_back(d_masks);
  int32_t* d_iter = d_masks;
  int32_t* d_check = d_masks + M;
  auto set_mask = [&](int32_t* hm, int32_t* dm, const std::vector<char>& on) {
    for (int m = 0; m < M; ++m) hm[m] = on[m] ? 1 : 0;
    check_hip(hipMemcpyAsync(dm, hm, mask_bytes, hipMemcpyHostToDevice, s), "group mask");
  };
  // reads one kBatch-vector of scalars (and the flags) of every member
  auto read_all = [&](int which, std::vector<std::array<double, kBatch>>& vals, std::vector<int32_t>& flags) {
    ggather_scalars(P.kry.djobs, M, which, d_read, s);
    check_hip(hipGetLastError(), "group read");
    sync(s, "group read");
    for (int m = 0; m < M; ++m) {
      for (int q = 0; q < kBatch; ++q) std::memcpy(&vals[m][q], &h_read[m * (kBatch + 1) + q], 8);
      flags[m] = (int32_t)h_read[m * (kBatch + 1) + kBatch];
    }
  };
  std::vector<std::array<double, kBatch>> nb(M), norm(M), rel(M);
  std::vector<int32_t> flags(M, 0);
  std::vector<std::array<int32_t, kBatch>> first(M);
  std::vector<unsigned> zero(M, 0);
  std::vector<int32_t> it(M, 0);
  std::vector<char> all_members(M, 1), iterating(M, 0), checking(M, 0);
  // norms of b, zero right-hand sides (and padding columns) solved by x = 0
  set_mask(h_check, d_check, all_members);
  gnorms_b(P.kry.djobs, M, d_check, s);
  read_all(KS_BNORM, nb, flags);
  for (int m = 0; m < M; ++m) {
    if (flags[m] & F_INVALID) throw Error{GMG_INVALID_ARGUMENT, "non-finite b or x"};
    for (int q = 0; q < kBatch; ++q)
      if (q >= nq[m] || nb[m][q] == 0.0) zero[m] |= 1u << q;
    if (zero[m]) mzero_columns(H[m]->bat.x, H[m]->L[0].n, zero[m], s);
    for (int q = 0; q < kBatch; ++q) first[m][q] = (zero[m] >> q) & 1u ? 0 : -1;
  }
  // true residuals of the members in `on`: rel, and whether all of a member's meet tol
  std::vector<char> passed(M, 0);
  auto true_residuals = [&](const std::vector<char>& on) {
    set_mask(h_check, d_check, on);
    gresidual_norms(P.kry.djobs, M, d_check, s);
    read_all(KS_NORM, norm, flags);
    for (int m = 0; m < M; ++m) {
      if (!on[m]) continue;
      bool all = true;
      for (int q = 0; q < kBatch; ++q) {
        rel[m][q] = (zero[m] >> q) & 1u ? 0.0 : norm[m][q] / nb[m][q];
        all = all && rel[m][q] <= tol;
      }
      passed[m] = all;
    }
  };
  true_residuals(all_members);
  int remaining = 0;
  for (int m = 0; m < M; ++m) {
    status[m] = passed[m] ? GMG_OK : GMG_NOT_CONVERGED;
    iterating[m] = !passed[m];
    remaining += iterating[m];
  }
  if (remaining > 0) {
    set_mask(h_iter, d_iter, iterating);
    gkry_init(P.kry.djobs, P.kry.dtiles, P.kry.ntiles(), d_iter, s);
    GroupGraph g;
    bool graphs = !std::getenv("GMG_DISABLE_GRAPHS");
    if (graphs) {
      const int saved = KernelTimer::active;
      KernelTimer::active = -1;
      bool ok = hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking) == hipSuccess;
      if (ok) ok = hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        group_iteration(P, d_iter, g.cap);
        ok = hipStreamEndCapture(g.cap, &g.graph) == hipSuccess && g.graph;
      }
      KernelTimer::active = saved;
      if (ok) ok = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0) == hipSuccess;
      if (!ok) {
        (void)hipGetLastError();
        graphs = false;
      }
    }
    int32_t done_iters = 0;
    while (remaining > 0 && done_iters < max_iters) {
      set_mask(h_iter, d_iter, iterating);
      if (graphs) check_hip(hipGraphLaunch(g.exec, s), "graph launch");
      else group_iteration(P, d_iter, s);
      check_hip(hipGetLastError(), "group iteration");
      read_all(KS_NORM, norm, flags);
      ++done_iters;
      std::fill(checking.begin(), checking.end(), 0);
      bool any_check = false;
      for (int m = 0; m < M; ++m) {
        if (!iterating[m]) continue;
        it[m] = done_iters;
        if (flags[m] & F_NOT_SPD) throw Error{GMG_NOT_SPD, "CG: non-positive curvature (A or the cycle not SPD)"};
        bool all = true;
        for (int q = 0; q < kBatch; ++q) {
          if ((zero[m] >> q) & 1u) continue;
          const double r = norm[m][q] / nb[m][q];
          if (r <= tol && first[m][q] < 0) first[m][q] = done_iters;
          all = all && r <= tol;
        }
        checking[m] = all;
        any_check = any_check || all;
      }
      if (any_check) {
        true_residuals(checking);
        for (int m = 0; m < M; ++m) {
          if (!checking[m]) continue;
          if (passed[m]) {
            status[m] = GMG_OK;
            iterating[m] = 0;
            --remaining;
          } else {
            for (int q = 0; q < kBatch; ++q)
              if (rel[m][q] > tol) first[m][q] = -1;
          }
        }
      }
    }
    if (remaining > 0) true_residuals(iterating);
  }
  for (int m = 0; m < M; ++m)
    for (int q = 0; q < nq[m]; ++q) {
      gmg_solve_info& inf = infos[(int64_t)m * kBatch + q];
      inf.iterations = first[m][q] >= 0 ? first[m][q] : it[m];
      inf.converged = rel[m][q] <= tol;
      inf.rel_residual = rel[m][q];
    }
  sync(s, "grouped solve");
}

const char* status_text(int st) {
  switch (st) {
    case GMG_OK: return "ok";
    case GMG_NOT_CONVERGED: return "not converged";
    case GMG_INVALID_ARGUMENT: return "invalid argument";
    case GMG_OUT_OF_MEMORY: return "out of memory";
    case GMG_DEVICE_ERROR: return "device error";
    case GMG_NOT_SPD: return "matrix not symmetric positive definite";
    case GMG_DEGENERATE: return "degenerate coarsening";
    default: return "unknown status";
  }
}

}  // namespace
}  // namespace gmg

using namespace gmg;

// The opaque handle of the C ABI is the library's hierarchy object.
struct gmg_handle_s : public gmg::Handle {};

extern "C" {

int gmg_default_options(gmg_options* o) {
  if (!o) return GMG_INVALID_ARGUMENT;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = (int32_t)sizeof(gmg_options);
  o->coarsening_ratio = 1.0 / 8.0;
  o->min_coarse_points = 1000;
  o->max_levels = 32;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->shift_coarse_points = 1;
  o->sample_order = 0;
  o->seed = 0;
  o->color_passes = 3;
  o->block_min_rows = 4096;
  o->autotune = 1;
  return GMG_OK;
}

int gmg_build_hierarchy(int64_t n, const double* points_dev, int64_t m, const int32_t* edges_dev,
                        const int32_t* A_rowptr_dev, const int32_t* A_col_dev, const double* A_val_dev,
                        int64_t A_nnz, const gmg_options* opt, void* stream, gmg_handle* out) {
  set_error("");
  if (!out) {
    set_error("out is NULL");
    return GMG_INVALID_ARGUMENT;
  }
  *out = nullptr;
  if (n <= 0 || n > INT32_MAX - 1 || m < 0 || m > INT32_MAX / 2 || A_nnz < n || A_nnz > INT32_MAX - 1 ||
      !points_dev || (m > 0 && !edges_dev) || !A_rowptr_dev || !A_col_dev || !A_val_dev) {
    set_error("invalid sizes or null pointers");
    return GMG_INVALID_ARGUMENT;
  }
  gmg_handle_s* h = new gmg_handle_s();
  h->stream = (hipStream_t)stream;
  if (opt) h->opt = *opt; else gmg_default_options(&h->opt);
  if (!options_ok(h->opt)) {
    delete h;
    set_error("invalid options");
    return GMG_INVALID_ARGUMENT;
  }
  try {
    check_hip(hipGetDevice(&h->device), "hipGetDevice");
    build(*h, n, points_dev, m, edges_dev, A_rowptr_dev, A_col_dev, A_val_dev, A_nnz);
  } catch (const Error& e) {
    set_error(e.msg);
    release(h);
    return e.status;
  }
  *out = h;
  return GMG_OK;
}

int gmg_solve(gmg_handle hh, const double* b_dev, double* x_dev, double tol, int32_t max_iters, void* stream,
              gmg_solve_info* info, double* residual_history) {
  set_error("");
  Handle* h = hh;
  if (!h || !b_dev || !x_dev || max_iters < 1 || !(tol >= 0.0)) {
    set_error("invalid solve arguments");
    return GMG_INVALID_ARGUMENT;
  }
  hipStream_t s = (hipStream_t)stream;
  hipStream_t saved = h->stream;
  h->stream = s;                               // synchronous reads below use the solve stream
  int status = GMG_OK;
  try {
    Level& l0 = h->L[0];
    const int64_t n = l0.n;
    double* red = h->red;
    double* hs = pinned_scratch();
    check_hip(hipMemsetAsync(h->flags, 0, 4, s), "memset");
    check_finite(b_dev, n, h->flags, s);
    check_finite(x_dev, n, h->flags, s);
    norm2_partials(b_dev, n, red, s);
    finish_norm(red, red + kNormBlocks, s);
    const double nb = [&] {
      check_hip(hipMemcpyAsync(hs, red + kNormBlocks, 8, hipMemcpyDeviceToHost, s), "copy");
      sync(s, "norm of b");
      return hs[0];
    }();
    if ((int32_t)read_i64(*h, h->flags, 4) & F_INVALID) throw Error{GMG_INVALID_ARGUMENT, "non-finite b or x"};
    if (info) {
      info->iterations = 0;
      info->converged = 0;
      info->rel_residual = 0.0;
    }
    if (nb == 0.0) {
      fill_f64(x_dev, 0.0, n, s);
      sync(s, "solve");
      if (info) info->converged = 1;
      h->stream = saved;
      return GMG_OK;
    }
    permute_in(l0.perm, b_dev, l0.b, n, s);
    permute_in(l0.perm, x_dev, l0.x, n, s);
    status = GMG_NOT_CONVERGED;
    double rel = 0.0;
    int32_t it = 0;
    if (!h->norm_host) {
      check_hip(hipHostMalloc((void**)&h->norm_host, 64, hipHostMallocDefault), "pinned host buffer");
      check_hip(hipHostGetDevicePointer((void**)&h->norm_dev, h->norm_host, 0), "pinned host buffer");
    }
    capture_cycle(*h);
    volatile uint64_t* nh = reinterpret_cast<volatile uint64_t*>(h->norm_host);
    while (it < max_iters) {
      // the cycle's last kernel stores the norm in pinned memory: the host
      // waits for that store (a norm is never the all-ones pattern) rather
      // than for a copy and the stream, then for the stream's completion only
      // when the solve ends or the wait runs long
      *nh = ~0ull;
      run_iteration(*h, s);
      uint64_t u = ~0ull;
      for (int spin = 0; spin < kNormSpins && (u = *nh) == ~0ull; ++spin) __builtin_ia32_pause();
      if (u == ~0ull) {
        sync(s, "V-cycle");
        u = *nh;
      }
      ++it;
      rel = __builtin_bit_cast(double, u) / nb;
      if (residual_history) residual_history[it - 1] = rel;
      if (rel <= tol) {
        status = GMG_OK;
        break;
      }
    }
    permute_out(l0.perm, l0.x, x_dev, n, s);
    sync(s, "solve");
    if (info) {
      info->iterations = it;
      info->converged = status == GMG_OK;
      info->rel_residual = rel;
    }
  } catch (const Error& e) {
    set_error(e.msg);
    status = e.status;
  }
  h->stream = saved;
  return status;
}

int gmg_solve_pcg(gmg_handle hh, const double* b_dev, double* x_dev, double tol, int32_t max_iters,
                  int32_t precision, void* stream, gmg_solve_info* info, double* residual_history) {
  set_error("");
  Handle* h = hh;
  if (!h || !b_dev || !x_dev || max_iters < 1 || !(tol >= 0.0) ||
      (precision != GMG_PRECISION_F64 && precision != GMG_PRECISION_F32)) {
    set_error("invalid solve arguments");
    return GMG_INVALID_ARGUMENT;
  }
  hipStream_t s = (hipStream_t)stream;
  hipStream_t saved = h->stream;
  h->stream = s;
  int status = GMG_OK;
  try {
    Level& l0 = h->L[0];
    const int64_t n = l0.n;
    double* red = h->red;
    check_hip(hipMemsetAsync(h->flags, 0, 4, s), "memset");
    check_finite(b_dev, n, h->flags, s);
    check_finite(x_dev, n, h->flags, s);
    norm2_partials(b_dev, n, red, s);
    finish_norm(red, red + kNormBlocks, s);
    int64_t vals[2] = {0, 0};
    ScalarRead rd[2] = {{red + kNormBlocks, 8, &vals[0]}, {h->flags, 4, &vals[1]}};
    read_scalars(*h, rd, 2);
    if (vals[1] & F_INVALID) throw Error{GMG_INVALID_ARGUMENT, "non-finite b or x"};
    double nb;
    std::memcpy(&nb, &vals[0], 8);
    if (info) {
      info->iterations = 0;
      info->converged = 0;
      info->rel_residual = 0.0;
    }
    if (nb == 0.0) {
      fill_zero(x_dev, n, s);
      sync(s, "solve");
      if (info) info->converged = 1;
      h->stream = saved;
      return GMG_OK;
    }
    permute_in(l0.perm, b_dev, l0.b, n, s);
    permute_in(l0.perm, x_dev, l0.x, n, s);
    int32_t it = 0;
    double rel = 0.0;
    if (precision == GMG_PRECISION_F32)
      status = pcg<float>(*h, nb, tol, max_iters, s, &it, &rel, residual_history);
    else
      status = pcg<double>(*h, nb, tol, max_iters, s, &it, &rel, residual_history);
    permute_out(l0.perm, (const double*)l0.x, x_dev, n, s);
    sync(s, "solve");
    if (info) {
      info->iterations = it;
      info->converged = status == GMG_OK;
      info->rel_residual = rel;
    }
  } catch (const Error& e) {
    set_error(e.msg);
    status = e.status;
  }
  h->stream = saved;
  return status;
}

int gmg_precondition(gmg_handle hh, const double* r_dev, double* z_dev, int32_t precision, void* stream) {
  set_error("");
  Handle* h = hh;
  if (!h || !r_dev || !z_dev || (precision != GMG_PRECISION_F64 && precision != GMG_PRECISION_F32)) {
    set_error("invalid preconditioner arguments");
    return GMG_INVALID_ARGUMENT;
  }
  hipStream_t s = (hipStream_t)stream;
  hipStream_t saved = h->stream;
  h->stream = s;
  int status = GMG_OK;
  try {
    Level& l0 = h->L[0];
    const int64_t n = l0.n;
    check_hip(hipMemsetAsync(h->flags, 0, 4, s), "memset");
    check_finite(r_dev, n, h->flags, s);
    if ((int32_t)read_i64(*h, h->flags, 4) & F_INVALID) throw Error{GMG_INVALID_ARGUMENT, "non-finite r"};
    kry_alloc(*h);
    permute_in(l0.perm, r_dev, h->kry.r, n, s);
    if (precision == GMG_PRECISION_F32) {
      Cycle<float>& c = kry_ready<float>(*h);
      kry_precondition(*h, c, s);
      permute_out(l0.perm, (const float*)c.v[0].x, z_dev, n, s);
    } else {
      Cycle<double>& c = kry_ready<double>(*h);
      kry_precondition(*h, c, s);
      permute_out(l0.perm, (const double*)c.v[0].x, z_dev, n, s);
    }
    sync(s, "preconditioner");
  } catch (const Error& e) {
    set_error(e.msg);
    status = e.status;
  }
  h->stream = saved;
  return status;
}

int gmg_update_matrix(gmg_handle hh, const double* A_val_dev, void* stream) {
  set_error("");
  Handle* h = hh;
  if (!h || !A_val_dev) {
    set_error("invalid update arguments");
    return GMG_INVALID_ARGUMENT;
  }
  hipStream_t s = (hipStream_t)stream;
  hipStream_t saved = h->stream;
  h->stream = s;
  int status = GMG_OK;
  try {
    const int nl = (int)h->L.size();
    Level& l0 = h->L[0];
    check_hip(hipMemsetAsync(h->flags, 0, 4, s), "memset");
    validate_matrix(l0.arp, l0.acol, A_val_dev, l0.n, l0.nnzA, h->flags, s);
    check_hip(hipMemcpyAsync(l0.aval, A_val_dev, (size_t)l0.nnzA * 8, hipMemcpyDeviceToDevice, s), "copy values");
    for (int l = 0; l + 1 < nl; ++l) galerkin_values(*h, h->L[l], h->L[l + 1]);
    for (int l = 0; l < nl; ++l) {
      refresh_values(*h, h->L[l]);
      block_values(*h, h->L[l]);
    }
    for (int l = ell_first_level(*h); l + 1 < nl; ++l) ell_values(*h, h->L[l]);
    coarse_factor(*h, h->L[nl - 1]);                 // also raises the flags of the steps above
    if (h->kry.ready[1])
      for (int l = 0; l + 1 < nl; ++l) {
        const LevelView& d = h->plain.v[l];
        LevelViewT<float>& f = h->kry.c32.v[l];
        to_f32(d.A.val, (float*)f.A.val, h->L[l].a_slots, s);
        to_f32(d.diag, (float*)f.diag, d.n, s);
        if (d.B.nblk > 0) to_f32(d.B.elv, (float*)f.B.elv, h->L[l].blk_entries, s);
        if (d.e_cinfo) {
          to_f32(d.e_val_gs, (float*)f.e_val_gs, h->L[l].e_slots, s);
          to_f32(d.e_val, (float*)f.e_val, h->L[l].e_slots, s);
        }
      }
    sync(s, "update");
  } catch (const Error& e) {
    set_error(e.msg);
    status = e.status;
  }
  h->stream = saved;
  return status;
}

int gmg_pattern_outer(int64_t n, const int32_t* rowptr_dev, const int32_t* col_dev, const double* u_dev,
                      const double* v_dev, double scale, double* out_dev, void* stream) {
  set_error("");
  if (n < 0 || (n > 0 && (!rowptr_dev || !col_dev || !u_dev || !v_dev || !out_dev))) {
    set_error("invalid pattern product arguments");
    return GMG_INVALID_ARGUMENT;
  }
  try {
    if (n > 0) pattern_outer(n, rowptr_dev, col_dev, u_dev, v_dev, scale, out_dev, (hipStream_t)stream);
    check_hip(hipGetLastError(), "pattern product");
  } catch (const Error& e) {
    set_error(e.msg);
    return e.status;
  }
  return GMG_OK;
}

int gmg_solve_pcg_batched(gmg_handle hh, int32_t nrhs, const double* B_dev, double* X_dev, double tol,
                          int32_t max_iters, int32_t precision, void* stream, gmg_solve_info* infos) {
  set_error("");
  Handle* h = hh;
  if (!h || nrhs < 0 || (nrhs > 0 && (!B_dev || !X_dev || !infos)) || max_iters < 1 || !(tol >= 0.0) ||
      (precision != GMG_PRECISION_F64 && precision != GMG_PRECISION_F32)) {
    set_error("invalid batched solve arguments");
    return GMG_INVALID_ARGUMENT;
  }
  hipStream_t s = (hipStream_t)stream;
  hipStream_t saved = h->stream;
  h->stream = s;
  int status = GMG_OK;
  try {
    Level& l0 = h->L[0];
    const int64_t n = l0.n;
    check_hip(hipMemsetAsync(h->flags, 0, 4, s), "memset");
    check_finite(B_dev, n * nrhs, h->flags, s);
    check_finite(X_dev, n * nrhs, h->flags, s);
    bat_alloc(*h);
    for (int g = 0; g < nrhs; g += kBatch) {
      const int nq = std::min(kBatch, nrhs - g);
      mgather(l0.perm, B_dev + (int64_t)g * n, n, nq, h->bat.b, s);
      mgather(l0.perm, X_dev + (int64_t)g * n, n, nq, h->bat.x, s);
      const int st = precision == GMG_PRECISION_F32
                         ? pcg_batched<float>(*h, nq, tol, max_iters, s, infos + g)
                         : pcg_batched<double>(*h, nq, tol, max_iters, s, infos + g);
      mscatter(l0.perm, (const double*)h->bat.x, n, nq, X_dev + (int64_t)g * n, s);
      if (st != GMG_OK) status = st;
    }
    sync(s, "batched solve");
  } catch (const Error& e) {
    set_error(e.msg);
    status = e.status;
  }
  h->stream = saved;
  return status;
}

int gmg_solve_pcg_grouped(int32_t count, const gmg_handle* handles, const int32_t* nrhs, const double* const* B_dev,
                          double* const* X_dev, double tol, int32_t max_iters, int32_t precision, void* stream,
                          gmg_solve_info* infos, int32_t* status_out) {
  set_error("");
  bool ok = count >= 0 && (count == 0 || (handles && nrhs && B_dev && X_dev && infos && status_out)) &&
            max_iters >= 1 && tol >= 0.0 &&
            (precision == GMG_PRECISION_F64 || precision == GMG_PRECISION_F32);
  std::vector<Handle*> H;
  std::vector<int> nq, idx;
  for (int32_t m = 0; ok && m < count; ++m) {
    Handle* h = handles[m];
    if (!h || nrhs[m] < 0 || nrhs[m] > kBatch || (nrhs[m] > 0 && (!B_dev[m] || !X_dev[m]))) {
      ok = false;
      break;
    }
    status_out[m] = GMG_OK;
    if (nrhs[m] == 0) continue;
    if (std::find(H.begin(), H.end(), h) != H.end() || (!H.empty() && h->device != H[0]->device)) {
      ok = false;
      break;
    }
    H.push_back(h);
    nq.push_back(nrhs[m]);
    idx.push_back(m);
  }
  if (!ok) {
    set_error("invalid grouped solve arguments (handles distinct, on one device, 0..8 right-hand sides each)");
    return GMG_INVALID_ARGUMENT;
  }
  if (H.empty()) return GMG_OK;
  hipStream_t s = (hipStream_t)stream;
  std::vector<hipStream_t> saved;
  for (Handle* h : H) {
    saved.push_back(h->stream);
    h->stream = s;
  }
  int status = GMG_OK;
  try {
    for (size_t m = 0; m < H.size(); ++m) {
      Handle& h = *H[m];
      const Level& l0 = h.L[0];
      const int64_t n = l0.n;
      const int32_t i = idx[m];
      check_hip(hipMemsetAsync(h.flags, 0, 4, s), "memset");
      check_finite(B_dev[i], n * nq[m], h.flags, s);
      check_finite(X_dev[i], n * nq[m], h.flags, s);
      bat_alloc(h);
      mgather(l0.perm, B_dev[i], n, nq[m], h.bat.b, s);
      mgather(l0.perm, X_dev[i], n, nq[m], h.bat.x, s);
    }
    std::vector<gmg_solve_info> inf(H.size() * kBatch);
    std::vector<int32_t> st(H.size(), GMG_OK);
    if (precision == GMG_PRECISION_F32) pcg_grouped<float>(H, nq, tol, max_iters, s, inf.data(), st.data());
    else pcg_grouped<double>(H, nq, tol, max_iters, s, inf.data(), st.data());
    for (size_t m = 0; m < H.size(); ++m) {
      const int32_t i = idx[m];
      mscatter(H[m]->L[0].perm, (const double*)H[m]->bat.x, H[m]->L[0].n, nq[m], X_dev[i], s);
      for (int q = 0; q < nq[m]; ++q) infos[(int64_t)i * kBatch + q] = inf[m * kBatch + q];
      status_out[i] = st[m];
      if (st[m] != GMG_OK) status = st[m];
    }
    sync(s, "grouped solve");
  } catch (const Error& e) {
    set_error(e.msg);
    status = e.status;
  }
  for (size_t m = 0; m < H.size(); ++m) H[m]->stream = saved[m];
  return status;
}

int gmg_precondition_batched(gmg_handle hh, int32_t nrhs, const double* R_dev, double* Z_dev, int32_t precision,
                             void* stream) {
  set_error("");
  Handle* h = hh;
  if (!h || nrhs < 0 || (nrhs > 0 && (!R_dev || !Z_dev)) ||
      (precision != GMG_PRECISION_F64 && precision != GMG_PRECISION_F32)) {
    set_error("invalid batched preconditioner arguments");
    return GMG_INVALID_ARGUMENT;
  }
  hipStream_t s = (hipStream_t)stream;
  hipStream_t saved = h->stream;
  h->stream = s;
  int status = GMG_OK;
  try {
    Level& l0 = h->L[0];
    const int64_t n = l0.n;
    check_hip(hipMemsetAsync(h->flags, 0, 4, s), "memset");
    check_finite(R_dev, n * nrhs, h->flags, s);
    if ((int32_t)read_i64(*h, h->flags, 4) & F_INVALID) throw Error{GMG_INVALID_ARGUMENT, "non-finite r"};
    bat_alloc(*h);
    for (int g = 0; g < nrhs; g += kBatch) {
      const int nq = std::min(kBatch, nrhs - g);
      mgather(l0.perm, R_dev + (int64_t)g * n, n, nq, h->bat.r, s);
      if (precision == GMG_PRECISION_F32) {
        Cycle<float>& c = bat_ready<float>(*h);
        bat_precondition(*h, c, s);
        mscatter(l0.perm, (const float*)c.v[0].x, n, nq, Z_dev + (int64_t)g * n, s);
      } else {
        Cycle<double>& c = bat_ready<double>(*h);
        bat_precondition(*h, c, s);
        mscatter(l0.perm, (const double*)c.v[0].x, n, nq, Z_dev + (int64_t)g * n, s);
      }
    }
    sync(s, "batched preconditioner");
  } catch (const Error& e) {
    set_error(e.msg);
    status = e.status;
  }
  h->stream = saved;
  return status;
}

int gmg_precondition_noalloc(gmg_handle hh, const double* r_dev, double* z_dev, int32_t precision, void* stream) {
  set_error("");
  Handle* h = hh;
  if (!h || !r_dev || !z_dev || (precision != GMG_PRECISION_F64 && precision != GMG_PRECISION_F32)) {
    set_error("invalid preconditioner arguments");
    return GMG_INVALID_ARGUMENT;
  }
  if (h->L[0].n > kNoAllocMaxPoints) {
    set_error("gmg_precondition_noalloc: more points than its scratch holds (2,097,152)");
    return GMG_INVALID_ARGUMENT;
  }
  if (precision == GMG_PRECISION_F32 && !h->kry.ready[1]) {
    set_error("gmg_precondition_noalloc: the float level data is made by a first GMG_PRECISION_F32 call of "
              "gmg_precondition or gmg_solve_pcg");
    return GMG_INVALID_ARGUMENT;
  }
  try {
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (dev != h->device) throw Error{GMG_INVALID_ARGUMENT, "the handle's device is not the current device"};
    precondition_noalloc(*h, r_dev, z_dev, precision, (hipStream_t)stream);
  } catch (const Error& e) {
    set_error(e.msg);
    return e.status;
  }
  return GMG_OK;
}

void gmg_free(gmg_handle h) { release(h); }

int gmg_timer_start(int32_t kernel, int32_t expected_launches) {
  if (kernel < 0 || kernel >= KernelTimer::KINDS || expected_launches < 0) return GMG_INVALID_ARGUMENT;
  g_ev_used = 0;
  g_bytes = 0.0;
  g_launches = 0;
  while ((int64_t)g_ev.size() < 2 * (int64_t)expected_launches) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return GMG_DEVICE_ERROR;
    g_ev.push_back(e);
  }
  KernelTimer::active = kernel;
  return GMG_OK;
}

int gmg_timer_stop(double* total_ms, int64_t* launches, double* bytes) {
  KernelTimer::active = -1;
  double ms = 0.0;
  for (size_t k = 0; k + 1 < g_ev_used + 1 && k < g_ev_used; k += 2) {
    if (hipEventSynchronize(g_ev[k + 1]) != hipSuccess) return GMG_DEVICE_ERROR;
    float t = 0.f;
    if (hipEventElapsedTime(&t, g_ev[k], g_ev[k + 1]) != hipSuccess) return GMG_DEVICE_ERROR;
    ms += t;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = g_launches;
  if (bytes) *bytes = g_bytes;
  return GMG_OK;
}

const char* gmg_status_string(int status) { return status_text(status); }

const char* gmg_last_error(void) { return g_last_error.c_str(); }

int gmg_num_levels(gmg_handle h, int32_t* levels) {
  if (!h || !levels) return GMG_INVALID_ARGUMENT;
  *levels = (int32_t)h->L.size();
  return GMG_OK;
}

int gmg_level_sizes(gmg_handle h, int32_t l, int64_t* sz) {
  if (!h || !sz || l < 0 || l >= (int32_t)h->L.size()) return GMG_INVALID_ARGUMENT;
  const Level& lv = h->L[l];
  sz[0] = lv.n;
  sz[1] = lv.nnzE / 2;
  sz[2] = lv.nnzA;
  sz[3] = lv.nc ? lv.nnzP : 0;
  sz[4] = lv.color ? lv.ncolors : 0;
  sz[5] = lv.nc ? lv.fallback : 0;
  sz[6] = lv.nc;
  sz[7] = lv.nnzE;
  sz[8] = lv.bcolor ? 1 : 0;
  return GMG_OK;
}

int gmg_level_tuning(gmg_handle h, int32_t l, int32_t* out) {
  if (!h || !out || l < 0 || l >= (int32_t)h->L.size()) return GMG_INVALID_ARGUMENT;
  const LevelView& v = h->L[l].view;
  const bool multi = l < h->tail_start;
  out[0] = multi && l > 0 ? v.ra : 0;
  out[1] = multi ? v.rt : 0;
  out[2] = multi && l == 0 ? v.ch : 0;
  out[3] = multi && l > 0 && v.B.nblk > 0 ? 1 : 0;
  out[4] = multi && l == 0 && v.uni && v.A.uw > 0 ? v.A.uw : 0;
  return GMG_OK;
}

int gmg_export_level(gmg_handle h, int32_t l, int32_t what, void* dst, int64_t bytes) {
  set_error("");
  if (!h || l < 0 || l >= (int32_t)h->L.size() || (!dst && bytes)) return GMG_INVALID_ARGUMENT;
  const Level& lv = h->L[l];
  const bool coarse = l + 1 == (int32_t)h->L.size();
  const int64_t n = lv.n, has = lv.nc ? n : 0;
  const void* src = nullptr;
  int64_t nb = 0;
  switch (what) {
    case GMG_EXPORT_POSITIONS: src = lv.X; nb = 24 * n; break;
    case GMG_EXPORT_EDGE_ROWPTR: src = lv.erp; nb = 4 * (n + 1); break;
    case GMG_EXPORT_EDGE_COL: src = lv.ecol; nb = 4 * lv.nnzE; break;
    case GMG_EXPORT_EDGE_W: src = lv.ew; nb = lv.ew ? 8 * lv.nnzE : 0; break;
    case GMG_EXPORT_SCALARS: src = lv.scal; nb = 16; break;
    case GMG_EXPORT_SAMPLES: src = lv.samples; nb = 4 * lv.nc; break;
    case GMG_EXPORT_LABELS: src = lv.label; nb = 4 * has; break;
    case GMG_EXPORT_DIST: src = lv.dist; nb = 8 * has; break;
    case GMG_EXPORT_P_COL: src = lv.pcol; nb = 12 * has; break;
    case GMG_EXPORT_P_VAL: src = lv.pval; nb = 24 * has; break;
    case GMG_EXPORT_P_CNT: src = lv.pcnt; nb = 4 * has; break;
    case GMG_EXPORT_TRI: src = lv.tri; nb = 8 * has; break;
    case GMG_EXPORT_A_ROWPTR: src = lv.arp; nb = 4 * (n + 1); break;
    case GMG_EXPORT_A_COL: src = lv.acol; nb = 4 * lv.nnzA; break;
    case GMG_EXPORT_A_VAL: src = lv.aval; nb = 8 * lv.nnzA; break;
    case GMG_EXPORT_COLORS: src = lv.color; nb = lv.color ? 4 * n : 0; break;
    case GMG_EXPORT_BLOCK_COLORS: src = lv.bcolor; nb = lv.bcolor ? 4 * n : 0; break;
    case GMG_EXPORT_CHOL:
      if (!coarse) return GMG_INVALID_ARGUMENT;
      src = h->chol; nb = 8 * n * n; break;
    case GMG_EXPORT_COARSE_INVERSE: {
      // stored with the padded column stride inv_ld(n): copied column by column
      if (!coarse) return GMG_INVALID_ARGUMENT;
      if (bytes != 8 * n * n) {
        set_error("export size mismatch");
        return GMG_INVALID_ARGUMENT;
      }
      if (n == 0) return GMG_OK;
      hipError_t e = hipMemcpy2D(dst, (size_t)n * 8, h->cinv, (size_t)inv_ld(n) * 8, (size_t)n * 8, (size_t)n,
                                 hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        set_error(hipGetErrorString(e));
        return GMG_DEVICE_ERROR;
      }
      return GMG_OK;
    }
    default: return GMG_INVALID_ARGUMENT;
  }
  if (bytes != nb) {
    set_error("export size mismatch");
    return GMG_INVALID_ARGUMENT;
  }
  if (nb == 0) return GMG_OK;
  hipError_t e = hipMemcpy(dst, src, (size_t)nb, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    set_error(hipGetErrorString(e));
    return GMG_DEVICE_ERROR;
  }
  return GMG_OK;
}

}  // extern "C"
