// Autotuner of the row kernels' shapes: for every level solved by separate
// launches, the lanes per row of the SELL row kernels of A_l (residual and
// colour sweeps) and of P_l^T (restriction, where one lane per row is also a
// candidate), and the load chunk of level 0's one-lane-per-row kernels (with
// the uniform slice width as a candidate where level 0's SELL has one), are
// picked by timing the candidates on the level's own data.  A shape only
// distributes a row's terms over lanes or loads: every row is still summed in
// its entry order (uniform slices add their padding's +-0 products after the
// row's own, which leaves the sum unchanged), so the choice never changes a
// result bit.  Choices are cached per shape class (kind, rows to a factor of
// sqrt 2, mean row, longest row to a power of two), so later builds of
// similar levels reuse them; the first build of a class pays for the
// measurement.  Lane counts wider than half the longest row are not timed,
// and a restriction is timed right after the residual it reads.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "gmg_internal.hpp"

namespace gmg {

namespace {

enum TuneKind : int32_t { TUNE_CHUNK0 = 0, TUNE_LANES_A = 1, TUNE_LANES_T = 2, TUNE_CHUNK0_UNIFORM = 3 };

struct TuneKey {
  int32_t kind, rows, mean, maxlen;
  bool operator<(const TuneKey& o) const {
    return std::tie(kind, rows, mean, maxlen) < std::tie(o.kind, o.rows, o.mean, o.maxlen);
  }
};

std::mutex g_tune_mutex;
std::map<TuneKey, int32_t> g_tune;

TuneKey key_of(int32_t kind, int64_t rows, int64_t entries, int32_t maxlen) {
  const double r = (double)std::max<int64_t>(rows, 1);
  int32_t m = 1;                                  // the longest row, rounded up to a power of two
  while (m < maxlen) m *= 2;
  return TuneKey{kind, (int32_t)std::floor(2.0 * std::log2(r)), (int32_t)std::lround((double)entries / r), m};
}

// Smallest time of kTuneReps launches after one warm-up, in milliseconds.
constexpr int kTuneReps = 3;
template <class F>
double time_launch(hipStream_t s, hipEvent_t e0, hipEvent_t e1, F launch) {
  launch();
  double best = 1e30;
  for (int k = 0; k < kTuneReps; ++k) {
    check_hip(hipEventRecord(e0, s), "tuning event");
    launch();
    check_hip(hipEventRecord(e1, s), "tuning event");
    check_hip(hipEventSynchronize(e1), "tuning event");
    float ms = 0.f;
    check_hip(hipEventElapsedTime(&ms, e0, e1), "tuning event");
    best = std::min(best, (double)ms);
  }
  return best;
}

// Lane counts worth timing for rows of at most maxlen entries: one lane (when
// allowed) and the powers of two from 4 up to half the longest row (at least
// 4); wider groups leave most of their lanes idle.
std::vector<int32_t> lane_candidates(int32_t maxlen, bool one) {
  std::vector<int32_t> c;
  if (one) c.push_back(1);
  for (int32_t r = 4; r <= 64; r *= 2)
    if (r == 4 || 2 * r <= maxlen) c.push_back(r);
  return c;
}

// The cached choice for key, or the fastest candidate (then cached).
template <class F>
int32_t choose(const TuneKey& key, const std::vector<int32_t>& cand, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
               F launch_with) {
  {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  // two sweeps over the candidates, each candidate's smallest time (a
  // candidate's launches are not all timed in one stretch of the box's state)
  std::vector<double> tmin(cand.size(), 1e30);
  for (int sweep = 0; sweep < 2; ++sweep) {
    int i = 0;
    for (int32_t c : cand) {
      tmin[i] = std::min(tmin[i], time_launch(s, e0, e1, [&] { launch_with(c); }));
      ++i;
    }
  }
  int32_t best = *cand.begin();
  double tbest = 1e30;
  int i = 0;
  for (int32_t c : cand) {
    if (tmin[i] < tbest) {
      tbest = tmin[i];
      best = c;
    }
    ++i;
  }
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  g_tune[key] = best;
  return best;
}

}  // namespace

void autotune(Handle& h) {
  const int nl = (int)h.L.size();
  if (!h.opt.autotune || nl < 2 || h.tail_start < 1) return;
  hipStream_t s = h.stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  check_hip(hipEventCreate(&e0), "tuning event");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    check_hip(hipErrorOutOfMemory, "tuning event");
  }
  try {
    for (int l = 0; l < h.tail_start; ++l) {
      Level& lv = h.L[l];
      LevelView& v = lv.view;
      const LevelView& cv = h.L[l + 1].view;
      // the residual writes the level's residual vector and the restriction the next
      // level's right-hand side and iterate: all of them are rewritten by every cycle
      if (l == 0) {
        // chunk c % 100; c >= 100: the uniform slice width (where the layout has one)
        const std::vector<int32_t> sell = {4, 8, 16}, both = {4, 8, 16, 104, 108, 116};
        const int32_t c = choose(key_of(v.A.uw > 0 ? TUNE_CHUNK0_UNIFORM : TUNE_CHUNK0, v.n, lv.nnzA, v.maxa),
                                 v.A.uw > 0 ? both : sell, s, e0, e1, [&](int32_t c) {
                                   LevelView t = v;
                                   t.ch = c % 100;
                                   t.uni = c >= 100 ? 1 : 0;
                                   residual(t, s, true);
                                 });
        v.ch = c % 100;
        v.uni = c >= 100 ? 1 : 0;
      } else {
        v.ra = choose(key_of(TUNE_LANES_A, v.n, lv.nnzA, v.maxa), lane_candidates(v.maxa, false), s, e0, e1,
                      [&](int32_t c) {
          LevelView t = v;
          t.ra = c;
          residual(t, s, false);
        });
      }
      // each restriction candidate is timed after the residual it reads, as in
      // the cycle (the residual just written, not yet in this compute unit's
      // cache): the pair's time ranks the candidates
      v.rt = choose(key_of(TUNE_LANES_T, cv.n, lv.nnzP, v.maxt), lane_candidates(v.maxt, true), s, e0, e1,
                    [&](int32_t c) {
        LevelView t = v;
        t.rt = c;
        residual(t, s, l == 0);
        restrict_to(t, cv, s, 0);
      });
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

}  // namespace gmg
