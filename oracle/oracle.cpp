// CPU oracle of the Gravo MG setup + solve pipeline (Wiersma, Nasikun, Eisemann &
// Hildebrandt, "A Fast Geometric Multigrid Method for Curved Surfaces", SIGGRAPH 2023).
//
// TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the smoke
// check and the benchmark's CPU-baseline leg may load this library.  It is a
// plain, slow, single-threaded restatement of the method: sequential loops,
// a binary heap, dense buffers.  It shares no code, header or constant table
// with the GPU library.
//
// Arithmetic convention: every floating-point operation is one IEEE-754
// binary64 operation in round-to-nearest-even, evaluated in the order written
// (built with -ffp-contract=off, no fast-math; x86-64 SSE2).  A 3-vector dot
// product is ((u.x*v.x + u.y*v.y) + u.z*v.z).  Under this convention every
// discrete decision (samples, Voronoi labels, coarse edges, triangle choices,
// sparsity patterns, colours) is reproducible bit for bit by any
// implementation that performs the same operations.
//
// Step map (paper section / algorithm / equation each step follows):
//   canonicalise            - Sec. 4.1 (input is points + an edge array)
//   edge_weights, mean_edge - Sec. 4.2, Eq. (1): r = phi^(-1/3) * e_hat
//   conflicts, sample       - Sec. 4.2: greedy sweep, radius r, 2-ring search
//   voronoi                 - Sec. 4.3: multi-source Dijkstra graph Voronoi
//   cells_and_shift         - Sec. 4.4 "Reducing single-entry rows"
//   coarse_edges            - Sec. 4.3: Voronoi-neighbour edges E_{l+1}
//   prolongation            - Sec. 4.4: candidate triangles, closest-point
//                             barycentric weights, inverse-distance fallback
//   galerkin                - Alg. 1: A_{l+1} = P_l^T A_l P_l
//   colouring               - Gauss-Seidel order (Sec. 3 leaves it open)
//   cholesky                - Alg. 2: direct solve on the coarsest level
//   solve / vcycle          - Alg. 1 and Alg. 2 (V-cycle, nu_pre/nu_post GS)
//   vcycle_sym, solve_pcg   - the V-cycle as a symmetric CG preconditioner
//                             (the Krylov-preconditioner use named in Sec. 6),
//                             in double or float, inside double-precision CG
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <queue>
#include <set>
#include <tuple>
#include <vector>

namespace {

// ---------------------------------------------------------------- options
struct Options {                 // field order mirrors the public options struct
  int32_t struct_size;
  double coarsening_ratio;       // phi (Sec. 4.2), default 1/8
  int32_t min_coarse_points;     // stop coarsening at this many points (Sec. 4.2), 1000
  int32_t max_levels;            // guard against non-terminating coarsening
  int32_t nu_pre, nu_post;       // Gauss-Seidel sweeps (Sec. 5.1): 2, 2
  int32_t shift_coarse_points;   // move coarse points to their cell mean (Sec. 4.4)
  int32_t sample_order;          // 0: hashed sweep order, 1: input (index) order
  uint64_t seed;
  int32_t weighting;             // 0 barycentric (Sec. 4.4), 1 uniform, 2 inverse distance (Sec. 5.3)
  int32_t fallback_on_vertex;    // 1: a best projection onto a triangle vertex uses the fallback
  int32_t color_passes;          // iterated-greedy passes after the first colouring (default 3)
  int32_t block_min_rows;        // levels 1.. above this many points sweep in block order (4096)
  int32_t autotune;              // GPU kernel shapes only (mirrors the public struct; no effect here)
};

enum Status { OK = 0, NOT_CONVERGED = 1, INVALID_ARGUMENT = -1, NOT_SPD = -4, DEGENERATE = -5 };

// What can be exported per level (same codes as the public inspection call).
enum What {
  W_POSITIONS = 0,   // double[n*3]
  W_EDGE_ROWPTR = 1, // int32[n+1]
  W_EDGE_COL = 2,    // int32[2m]
  W_EDGE_W = 3,      // double[2m]
  W_SCALARS = 4,     // double[2]: e_hat, r
  W_SAMPLES = 5,     // int32[n_{l+1}] fine indices of the coarse points, ascending
  W_LABELS = 6,      // int32[n] coarse id of the Voronoi cell of each point
  W_DIST = 7,        // double[n] graph distance to the cell's seed
  W_P_COL = 8,       // int32[3n] ELL-3 columns (unused slots: -1)
  W_P_VAL = 9,       // double[3n] ELL-3 values (unused slots: 0)
  W_P_CNT = 10,      // int32[n] entries per row (1..3)
  W_TRI = 11,        // int32[2n] chosen triangle (j,k) with apex label(p); -1,-1 = fallback
  W_A_ROWPTR = 12,   // int32[n+1]
  W_A_COL = 13,      // int32[nnz]
  W_A_VAL = 14,      // double[nnz]
  W_COLORS = 15,     // int32[n]
  W_CHOL = 16,       // double[n*n] row-major lower Cholesky factor (coarsest level only)
  W_CINV = 17,       // double[n*n] coarsest inverse by columns: [k*n + i] = (A^-1 e_k)_i
  W_BLOCK_COLORS = 18, // int32[n] block colour 0..3 of each row (levels swept in block order; else empty)
};

constexpr double kDegenerateTau = 1e-12;   // sin^2 of the smallest accepted triangle angle
constexpr int64_t kMaxDenseCoarse = 4096;  // largest coarsest level factored densely
constexpr uint64_t kColorSalt = 0xC2B2AE3D27D4EB4FULL;
constexpr double kBlockMargin = 1.0 + 1.0 / (1 << 20);   // cell side over the largest coupling distance
constexpr int64_t kMaxGridCells = int64_t(1) << 22;       // grids with more cells keep the colour order
constexpr int32_t kMaxCellRows = 512;                      // blocks with more rows keep the level in colour order
constexpr int32_t kMaxBrickRows = 256;                     // bricks with more rows: single cells are the blocks
constexpr int32_t kMaxCellColors = 64;                     // likewise a block that needs this many colours

// SplitMix64 finaliser (Steele, Lea & Flood 2014): a bijective 64-bit mixer.
uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

struct V3 { double x, y, z; };
V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
double dot(V3 a, V3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

struct Level {
  int64_t n = 0;
  std::vector<double> X;                        // n*3 positions
  std::vector<int32_t> erp, ecol;               // symmetric, sorted, loop-free CSR of E_l
  std::vector<double> ew;                       // Euclidean edge lengths per CSR entry
  double ehat = 0, r = 0;
  std::vector<int32_t> samples;                 // coarse points (fine indices), ascending
  std::vector<int32_t> label;                   // Voronoi cell (coarse id) per point
  std::vector<double> dist;                     // graph distance to the cell's seed
  std::vector<int32_t> pcol, pcnt, tri;         // prolongation P_l (ELL-3) and triangle choice
  std::vector<double> pval;
  int64_t fallback = 0;
  std::vector<int32_t> arp, acol;               // A_l
  std::vector<double> aval, adiag;
  std::vector<int32_t> color;
  int32_t ncolors = 0;
  std::vector<int32_t> block_color;             // block colour 0..3 per row (block order), or empty
  std::vector<int32_t> color_rows;              // rows in sweep order: (block colour, colour, index)
  std::vector<int32_t> color_ptr;               // colour c rows: color_rows[color_ptr[c] .. color_ptr[c+1])
};

struct Hier {
  Options opt;
  std::vector<Level> L;                         // L[0] finest ... L.back() coarsest
  std::vector<double> chol;                     // dense lower Cholesky factor of the coarsest A
  std::vector<double> cinv;                     // its inverse by columns: cinv[k n + i] = (A^-1 e_k)_i
};

V3 pos(const Level& lv, int64_t i) { return {lv.X[3 * i], lv.X[3 * i + 1], lv.X[3 * i + 2]}; }

// ---------------------------------------------------------------- input
// Sec. 4.1: the input is a point set and an edge array.  E is made a symmetric
// adjacency without self loops or duplicate edges, rows sorted ascending.
int canonicalise(Level& lv, int64_t n, const double* pts, int64_t m, const int32_t* edges) {
  lv.n = n;
  lv.X.assign(pts, pts + 3 * n);
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(lv.X[i])) return INVALID_ARGUMENT;
  std::vector<std::vector<int32_t>> adj(n);
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = edges[2 * e], v = edges[2 * e + 1];
    if (u < 0 || v < 0 || u >= n || v >= n) return INVALID_ARGUMENT;
    if (u == v) continue;
    adj[u].push_back(v);
    adj[v].push_back(u);
  }
  lv.erp.assign(n + 1, 0);
  lv.ecol.clear();
  for (int64_t i = 0; i < n; ++i) {
    std::sort(adj[i].begin(), adj[i].end());
    adj[i].erase(std::unique(adj[i].begin(), adj[i].end()), adj[i].end());
    lv.ecol.insert(lv.ecol.end(), adj[i].begin(), adj[i].end());
    lv.erp[i + 1] = (int32_t)lv.ecol.size();
  }
  return OK;
}

// The system matrix must be an n x n CSR with sorted in-range columns, a
// symmetric pattern, finite values and a positive diagonal.
int take_matrix(Level& lv, const int32_t* rp, const int32_t* col, const double* val, int64_t nnz) {
  int64_t n = lv.n;
  if (rp[0] != 0 || rp[n] != nnz) return INVALID_ARGUMENT;
  lv.arp.assign(rp, rp + n + 1);
  lv.acol.assign(col, col + nnz);
  lv.aval.assign(val, val + nnz);
  lv.adiag.assign(n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return INVALID_ARGUMENT;
    bool has_diag = false;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n) return INVALID_ARGUMENT;
      if (e > rp[i] && col[e] <= col[e - 1]) return INVALID_ARGUMENT;
      if (!std::isfinite(val[e])) return INVALID_ARGUMENT;
      if (col[e] == i) { has_diag = true; lv.adiag[i] = val[e]; }
      // pattern symmetry: (col, i) must exist
      const int32_t* b = col + rp[col[e]];
      const int32_t* en = col + rp[col[e] + 1];
      if (!std::binary_search(b, en, (int32_t)i)) return INVALID_ARGUMENT;
    }
    if (!has_diag) return INVALID_ARGUMENT;
    if (!(lv.adiag[i] > 0.0)) return NOT_SPD;
  }
  return OK;
}

// ---------------------------------------------------------------- sampling (Sec. 4.2)
void edge_weights(Level& lv) {
  lv.ew.resize(lv.ecol.size());
  for (int64_t u = 0; u < lv.n; ++u)
    for (int32_t e = lv.erp[u]; e < lv.erp[u + 1]; ++e) {
      V3 d = sub(pos(lv, u), pos(lv, lv.ecol[e]));
      lv.ew[e] = std::sqrt(dot(d, d));
    }
}

// Average edge length e_hat over the undirected edges, then r = phi^(-1/3) e_hat
// (Eq. 1).  The sum is taken exactly in 64-bit fixed point so that its value
// does not depend on summation order: with M the longest edge, M < 2^e, and
// F = 62 - e - ceil(log2 m), every edge length scaled by 2^F rounds to an
// integer below 2^(62 - ceil log2 m), so the m-term sum stays below 2^62.
void mean_edge(Level& lv, double rho) {
  double M = 0.0;
  int64_t cnt = 0;
  for (int64_t u = 0; u < lv.n; ++u)
    for (int32_t e = lv.erp[u]; e < lv.erp[u + 1]; ++e)
      if (u < lv.ecol[e]) { M = std::max(M, lv.ew[e]); ++cnt; }
  if (cnt == 0 || M == 0.0) { lv.ehat = 0.0; lv.r = 0.0; return; }
  int ex = 0;
  std::frexp(M, &ex);
  int lg = 0;
  while ((int64_t(1) << lg) < cnt) ++lg;
  int F = 62 - ex - lg;
  int64_t S = 0;
  for (int64_t u = 0; u < lv.n; ++u)
    for (int32_t e = lv.erp[u]; e < lv.erp[u + 1]; ++e)
      if (u < lv.ecol[e]) S += std::llrint(std::ldexp(lv.ew[e], F));
  lv.ehat = std::ldexp((double)S, -F) / (double)cnt;
  lv.r = rho * lv.ehat;
}

// Points within graph distance r of p, the search limited to the 2-ring: q is in
// conflict with p when q is a neighbour with w_pq <= r, or when some path
// p - m - q has w_pm + w_mq <= r.  (Duplicates are harmless to the callers.)
void conflicts(const Level& lv, int64_t p, std::vector<int32_t>& out) {
  out.clear();
  for (int32_t e = lv.erp[p]; e < lv.erp[p + 1]; ++e) {
    int32_t m = lv.ecol[e];
    double wpm = lv.ew[e];
    if (wpm <= lv.r) out.push_back(m);
    for (int32_t f = lv.erp[m]; f < lv.erp[m + 1]; ++f) {
      int32_t q = lv.ecol[f];
      if (q != p && wpm + lv.ew[f] <= lv.r) out.push_back(q);
    }
  }
}

// The greedy sweep: visit points in sweep order; an eligible point becomes a
// sample and makes every point in conflict with it ineligible.
void sample(Level& lv, int level, const Options& o) {
  int64_t n = lv.n;
  std::vector<std::pair<uint64_t, int32_t>> order(n);
  for (int64_t v = 0; v < n; ++v) {
    uint64_t key = (o.sample_order == 1) ? 0
                 : mix64(o.seed ^ ((uint64_t)level << 32) ^ (uint64_t)v);
    order[v] = {key, (int32_t)v};
  }
  std::sort(order.begin(), order.end());
  std::vector<char> eligible(n, 1);
  std::vector<int32_t> c;
  lv.samples.clear();
  for (auto& kv : order) {
    int32_t v = kv.second;
    if (!eligible[v]) continue;
    lv.samples.push_back(v);
    eligible[v] = 0;
    conflicts(lv, v, c);
    for (int32_t q : c) eligible[q] = 0;
  }
  // coarse point ids: rank of the sample by ascending fine index
  std::sort(lv.samples.begin(), lv.samples.end());
}

// ---------------------------------------------------------------- graph Voronoi (Sec. 4.3)
// Multi-source Dijkstra.  Keys are (distance, coarse id) compared
// lexicographically, so a point equidistant from two seeds joins the cell with
// the smaller id; a key is replaced only by a strictly smaller one.
void voronoi(Level& lv) {
  int64_t n = lv.n;
  const double inf = INFINITY;
  lv.dist.assign(n, inf);
  lv.label.assign(n, -1);
  typedef std::tuple<double, int32_t, int32_t> Item;   // (d, label, vertex)
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (size_t id = 0; id < lv.samples.size(); ++id) {
    int32_t s = lv.samples[id];
    lv.dist[s] = 0.0;
    lv.label[s] = (int32_t)id;
    heap.push(Item(0.0, (int32_t)id, s));
  }
  while (!heap.empty()) {
    Item it = heap.top();
    heap.pop();
    double d = std::get<0>(it);
    int32_t lab = std::get<1>(it), u = std::get<2>(it);
    if (d != lv.dist[u] || lab != lv.label[u]) continue;   // stale entry
    for (int32_t e = lv.erp[u]; e < lv.erp[u + 1]; ++e) {
      int32_t v = lv.ecol[e];
      double nd = d + lv.ew[e];
      if (nd < lv.dist[v] || (nd == lv.dist[v] && lab < lv.label[v])) {
        lv.dist[v] = nd;
        lv.label[v] = lab;
        heap.push(Item(nd, lab, v));
      }
    }
  }
}

// ---------------------------------------------------------------- next level points and edges
// Sec. 4.4 "Reducing single-entry rows": each coarse point moves to the mean of
// its cell, summed in ascending fine index from 0.0.  The moved point is used
// for the projection and as the point of level l+1.
void cells_and_shift(const Level& lv, Level& nx, bool shift) {
  int64_t nc = (int64_t)lv.samples.size();
  nx.n = nc;
  nx.X.assign(3 * nc, 0.0);
  if (!shift) {
    for (int64_t I = 0; I < nc; ++I)
      for (int k = 0; k < 3; ++k) nx.X[3 * I + k] = lv.X[3 * (int64_t)lv.samples[I] + k];
    return;
  }
  std::vector<int64_t> count(nc, 0);
  for (int64_t i = 0; i < lv.n; ++i) {            // ascending fine index
    int32_t I = lv.label[i];
    for (int k = 0; k < 3; ++k) nx.X[3 * I + k] = nx.X[3 * I + k] + lv.X[3 * i + k];
    count[I] += 1;
  }
  for (int64_t I = 0; I < nc; ++I)
    for (int k = 0; k < 3; ++k) nx.X[3 * I + k] = nx.X[3 * I + k] / (double)count[I];
}

// Sec. 4.3: {I, J} is an edge of level l+1 iff some edge of level l joins a
// point of cell I and a point of cell J.
void coarse_edges(const Level& lv, Level& nx) {
  std::vector<std::set<int32_t>> adj(nx.n);
  for (int64_t u = 0; u < lv.n; ++u)
    for (int32_t e = lv.erp[u]; e < lv.erp[u + 1]; ++e) {
      int32_t a = lv.label[u], b = lv.label[lv.ecol[e]];
      if (a != b) adj[a].insert(b);
    }
  nx.erp.assign(nx.n + 1, 0);
  nx.ecol.clear();
  for (int64_t I = 0; I < nx.n; ++I) {
    nx.ecol.insert(nx.ecol.end(), adj[I].begin(), adj[I].end());
    nx.erp[I + 1] = (int32_t)nx.ecol.size();
  }
}

// ---------------------------------------------------------------- prolongation (Sec. 4.4)
bool has_edge(const Level& lv, int32_t a, int32_t b) {
  return std::binary_search(lv.ecol.begin() + lv.erp[a], lv.ecol.begin() + lv.erp[a + 1], b);
}

// A triangle is rejected as (nearly) co-linear when the squared sine of its
// angle at A is at most tau: |ab x ac|^2 <= (tau |ab|^2) |ac|^2.
bool degenerate(V3 A, V3 B, V3 C) {
  V3 ab = sub(B, A), ac = sub(C, A);
  V3 nrm = cross(ab, ac);
  return dot(nrm, nrm) <= (kDegenerateTau * dot(ab, ab)) * dot(ac, ac);
}

// Closest point of triangle ABC to P as barycentric weights (wA, wB, wC): the
// point may lie in the face, on an edge or at a vertex (Sec. 4.4).  The
// region is found by the Voronoi-region tests of Ericson, Real-Time Collision
// Detection (2005), Sec. 5.1.5, taken in the order vertex A, vertex B, edge AB,
// vertex C, edge AC, edge BC, face.  Returns the region index 0..6.
int closest_point(V3 P, V3 A, V3 B, V3 C, double w[3]) {
  V3 ab = sub(B, A), ac = sub(C, A), ap = sub(P, A);
  double d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0.0 && d2 <= 0.0) { w[0] = 1.0; w[1] = 0.0; w[2] = 0.0; return 0; }
  V3 bp = sub(P, B);
  double d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0.0 && d4 <= d3) { w[0] = 0.0; w[1] = 1.0; w[2] = 0.0; return 1; }
  double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
    double t = d1 / (d1 - d3);
    w[0] = 1.0 - t; w[1] = t; w[2] = 0.0; return 2;
  }
  V3 cp = sub(P, C);
  double d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) { w[0] = 0.0; w[1] = 0.0; w[2] = 1.0; return 3; }
  double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
    double t = d2 / (d2 - d6);
    w[0] = 1.0 - t; w[1] = 0.0; w[2] = t; return 4;
  }
  double va = d3 * d6 - d5 * d4;
  double e43 = d4 - d3, e56 = d5 - d6;
  if (va <= 0.0 && e43 >= 0.0 && e56 >= 0.0) {
    double t = e43 / (e43 + e56);
    w[0] = 0.0; w[1] = 1.0 - t; w[2] = t; return 5;
  }
  double a = std::max(va, 0.0), b = std::max(vb, 0.0), c = std::max(vc, 0.0);
  double s = (a + b) + c;
  if (!(s > 0.0)) { w[0] = 1.0; w[1] = 0.0; w[2] = 0.0; return 6; }
  w[0] = a / s; w[1] = b / s; w[2] = c / s;
  return 6;
}

double dist2_to(V3 P, V3 A, V3 B, V3 C, const double w[3]) {
  V3 q = {(w[0] * A.x + w[1] * B.x) + w[2] * C.x,
          (w[0] * A.y + w[1] * B.y) + w[2] * C.y,
          (w[0] * A.z + w[1] * B.z) + w[2] * C.z};
  V3 d = sub(P, q);
  return dot(d, d);
}

// Row p of P_l: c = label(p) is the coarse point closest to p.  Candidates are
// the triangles (c, j, k) of E_{l+1} with j < k both neighbours of c, visited
// in ascending (j, k); the first one with the smallest point-to-triangle
// distance wins.  Without any non-degenerate candidate, the three points of
// {c} U N(c) nearest to p get inverse-distance weights.
// Variants of the weighting ablation (Sec. 5.3) replace the barycentric
// weights on the chosen triangle (c, j, k) by 1/3 each (uniform) or by
// 1/|p - X_t| normalised by their sum (inverse distance; a vertex at distance 0
// takes weight 1).  fallback_on_vertex sends a best projection that lands on a
// triangle vertex to the inverse-distance fallback.
void prolongation(Level& L, const Level& nx, const Options& o) {
  const Level& lv = L;
  int64_t n = lv.n;
  L.pcol.assign(3 * n, -1);
  L.pval.assign(3 * n, 0.0);
  L.pcnt.assign(n, 0);
  L.tri.assign(2 * n, -1);
  L.fallback = 0;
  for (int64_t p = 0; p < n; ++p) {
    V3 P = pos(lv, p);
    int32_t c = lv.label[p];
    V3 A = pos(nx, c);
    bool found = false;
    double best = 0.0, bw[3] = {0, 0, 0};
    int32_t bj = -1, bk = -1;
    int breg = -1;
    for (int32_t e1 = nx.erp[c]; e1 < nx.erp[c + 1]; ++e1) {
      int32_t j = nx.ecol[e1];
      for (int32_t e2 = e1 + 1; e2 < nx.erp[c + 1]; ++e2) {
        int32_t k = nx.ecol[e2];
        if (!has_edge(nx, j, k)) continue;
        V3 B = pos(nx, j), C = pos(nx, k);
        if (degenerate(A, B, C)) continue;
        double w[3];
        int reg = closest_point(P, A, B, C, w);
        double d2 = dist2_to(P, A, B, C, w);
        if (!found || d2 < best) {
          found = true; best = d2; bj = j; bk = k; breg = reg;
          bw[0] = w[0]; bw[1] = w[1]; bw[2] = w[2];
        }
      }
    }
    // regions 0, 1, 3 are the vertices A, B, C (see closest_point)
    if (found && o.fallback_on_vertex && (breg == 0 || breg == 1 || breg == 3)) found = false;
    int32_t cols[3];
    double vals[3];
    int cnt = 0;
    if (found) {
      L.tri[2 * p] = bj;
      L.tri[2 * p + 1] = bk;
      cols[0] = c; cols[1] = bj; cols[2] = bk;
      vals[0] = bw[0]; vals[1] = bw[1]; vals[2] = bw[2];
      if (o.weighting == 1) {
        vals[0] = vals[1] = vals[2] = 1.0 / 3.0;
      } else if (o.weighting == 2) {
        V3 T[3] = {A, pos(nx, bj), pos(nx, bk)};
        double d[3];
        for (int t = 0; t < 3; ++t) { V3 e = sub(P, T[t]); d[t] = std::sqrt(dot(e, e)); }
        int zero = d[0] == 0.0 ? 0 : d[1] == 0.0 ? 1 : d[2] == 0.0 ? 2 : -1;
        if (zero >= 0) {
          for (int t = 0; t < 3; ++t) vals[t] = t == zero ? 1.0 : 0.0;
        } else {
          double inv[3] = {1.0 / d[0], 1.0 / d[1], 1.0 / d[2]};
          double s = (inv[0] + inv[1]) + inv[2];
          for (int t = 0; t < 3; ++t) vals[t] = inv[t] / s;
        }
      }
      cnt = 3;
    } else {
      L.fallback += 1;
      std::vector<std::pair<double, int32_t>> cand;
      std::vector<int32_t> nb;
      nb.push_back(c);
      for (int32_t e = nx.erp[c]; e < nx.erp[c + 1]; ++e) nb.push_back(nx.ecol[e]);
      for (int32_t q : nb) {
        V3 d = sub(P, pos(nx, q));
        cand.push_back({dot(d, d), q});
      }
      std::sort(cand.begin(), cand.end());
      int k = (int)std::min<size_t>(3, cand.size());
      if (cand[0].first == 0.0) {
        cols[0] = cand[0].second; vals[0] = 1.0; cnt = 1;
      } else {
        double inv[3], s = 0.0;
        for (int t = 0; t < k; ++t) { inv[t] = 1.0 / std::sqrt(cand[t].first); s = s + inv[t]; }
        for (int t = 0; t < k; ++t) { cols[t] = cand[t].second; vals[t] = inv[t] / s; }
        cnt = k;
      }
    }
    // keep the non-zero weights, sorted by column
    std::vector<std::pair<int32_t, double>> row;
    for (int t = 0; t < cnt; ++t)
      if (vals[t] != 0.0) row.push_back({cols[t], vals[t]});
    std::sort(row.begin(), row.end());
    L.pcnt[p] = (int32_t)row.size();
    for (size_t t = 0; t < row.size(); ++t) {
      L.pcol[3 * p + t] = row[t].first;
      L.pval[3 * p + t] = row[t].second;
    }
  }
}

// ---------------------------------------------------------------- Galerkin operator (Alg. 1)
// A_{l+1}[I, J] = sum_i sum_j P[i, I] A[i, j] P[j, J] over the structural
// pattern, accumulated per coarse row in a dense buffer: fine rows i in
// ascending order, then the CSR order of row i of A, then the order of row j
// of P; every term is (P_iI * A_ij) * P_jJ.
int galerkin(const Level& lv, Level& nx) {
  int64_t nc = nx.n;
  std::vector<std::vector<std::pair<int32_t, double>>> pt(nc);   // P^T rows, ascending fine index
  for (int64_t i = 0; i < lv.n; ++i)
    for (int t = 0; t < lv.pcnt[i]; ++t) pt[lv.pcol[3 * i + t]].push_back({(int32_t)i, lv.pval[3 * i + t]});
  std::vector<double> acc(nc, 0.0);
  std::vector<char> touched(nc, 0);
  std::vector<int32_t> cols;
  nx.arp.assign(nc + 1, 0);
  nx.acol.clear();
  nx.aval.clear();
  nx.adiag.assign(nc, 0.0);
  for (int64_t I = 0; I < nc; ++I) {
    cols.clear();
    for (auto& ip : pt[I]) {
      int32_t i = ip.first;
      double piI = ip.second;
      for (int32_t e = lv.arp[i]; e < lv.arp[i + 1]; ++e) {
        int32_t j = lv.acol[e];
        double t1 = piI * lv.aval[e];
        for (int t = 0; t < lv.pcnt[j]; ++t) {
          int32_t J = lv.pcol[3 * j + t];
          if (!touched[J]) { touched[J] = 1; acc[J] = 0.0; cols.push_back(J); }
          acc[J] = acc[J] + t1 * lv.pval[3 * j + t];
        }
      }
    }
    std::sort(cols.begin(), cols.end());
    bool has_diag = false;
    for (int32_t J : cols) {
      nx.acol.push_back(J);
      nx.aval.push_back(acc[J]);
      if (J == I) { has_diag = true; nx.adiag[I] = acc[J]; }
      touched[J] = 0;
    }
    nx.arp[I + 1] = (int32_t)nx.acol.size();
    // a zero diagonal would make Gauss-Seidel divide by zero (the paper's NaN case)
    if (!has_diag || !(nx.adiag[I] > 0.0)) return NOT_SPD;
  }
  return OK;
}

// ---------------------------------------------------------------- Gauss-Seidel order
// First-fit colour of v given the colours of the other vertices (-1: none yet).
int32_t first_fit(const Level& lv, int32_t v, const std::vector<int32_t>& color, std::vector<char>& used) {
  used.assign(lv.arp[v + 1] - lv.arp[v] + 1, 0);
  for (int32_t e = lv.arp[v]; e < lv.arp[v + 1]; ++e) {
    int32_t u = lv.acol[e];
    if (u != v && color[u] >= 0 && color[u] < (int32_t)used.size()) used[color[u]] = 1;
  }
  int32_t c = 0;
  while (used[c]) ++c;
  return c;
}

// Multicolour ordering of A_l: first-fit greedy colouring in hashed key order
// (equal to Jones-Plassmann colouring), then o.color_passes passes of iterated
// greedy colouring (Culberson): every vertex is coloured first-fit again, the
// colour classes of the previous colouring visited from the highest colour
// down.  The vertices of one class are not adjacent, so their order within
// the class does not matter; a pass never needs more colours than the
// colouring it starts from.  A Gauss-Seidel sweep then visits the colours in
// ascending order.
void colouring(Level& lv, int level, const Options& o) {
  int64_t n = lv.n;
  std::vector<std::pair<uint64_t, int32_t>> order(n);
  for (int64_t v = 0; v < n; ++v)
    order[v] = {mix64((o.seed ^ kColorSalt) ^ ((uint64_t)level << 32) ^ (uint64_t)v), (int32_t)v};
  std::sort(order.begin(), order.end());
  lv.color.assign(n, -1);
  lv.ncolors = 0;
  std::vector<char> used;
  for (auto& kv : order) {
    int32_t v = kv.second;
    int32_t c = first_fit(lv, v, lv.color, used);
    lv.color[v] = c;
    lv.ncolors = std::max(lv.ncolors, c + 1);
  }
  for (int32_t p = 0; p < o.color_passes && lv.ncolors > 1; ++p) {
    std::vector<std::vector<int32_t>> cls(lv.ncolors);
    for (int64_t v = 0; v < n; ++v) cls[lv.color[v]].push_back((int32_t)v);
    std::vector<int32_t> next(n, -1);
    int32_t nc = 0;
    for (int32_t c = lv.ncolors - 1; c >= 0; --c)
      for (int32_t v : cls[c]) {
        next[v] = first_fit(lv, v, next, used);
        nc = std::max(nc, next[v] + 1);
      }
    lv.color.swap(next);
    lv.ncolors = nc;
  }
}

// Block order of the sweeps on a level (a reading: the paper leaves the
// Gauss-Seidel order open).  The level's points are projected onto the two
// coordinate axes of largest extent (the axis of smallest extent is dropped,
// the first on ties) and binned into square cells whose side is slightly more
// than w, the largest distance along either kept axis between two points
// coupled by A_l.  Two coupled points then lie in the same cell or in
// neighbouring ones (sharing a side or a corner).  The blocks are bricks of
// two cells side by side, shifted by one cell on every odd row of cells:
// brick bx of row cy holds cells cx with (cx + (cy mod 2)) div 2 = bx.  A
// brick then touches exactly six others (two in its row, two in each
// neighbouring row), the pattern of a triangular lattice, and with
// a = bx - (cy + 1) div 2 the brick colour (a - cy) mod 3 differs between
// any two touching bricks.  A level with a brick of more than kMaxBrickRows
// rows takes single cells as blocks instead, coloured by the parity pair
// (cx mod 2) + 2 (cy mod 2), which differs between touching cells.  The block
// colours are swept one after the other, all blocks of a colour at once and
// within a block the colours in ascending order.  Without couplings (w = 0),
// or with more than kMaxGridCells cells, the level keeps the colour order.
// cell[i] receives row i's block (bricks: cy * nbx + bx, nbx = ncx div 2 + 1
// bricks per row; cells: cy * ncx + cx); returns whether the level has a grid.
bool block_order(Level& lv, std::vector<int64_t>& cell) {
  const int64_t n = lv.n;
  lv.block_color.clear();
  cell.clear();
  double lo[3], hi[3], ext[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = lv.X[a];
    hi[a] = lv.X[a];
    for (int64_t i = 1; i < n; ++i) {
      lo[a] = std::min(lo[a], lv.X[3 * i + a]);
      hi[a] = std::max(hi[a], lv.X[3 * i + a]);
    }
    ext[a] = hi[a] - lo[a];
  }
  int drop = 0;
  for (int a = 1; a < 3; ++a)
    if (ext[a] < ext[drop]) drop = a;
  const int a0 = drop == 0 ? 1 : 0, a1 = drop == 2 ? 1 : 2;
  double w = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int32_t e = lv.arp[i]; e < lv.arp[i + 1]; ++e) {
      const int64_t j = lv.acol[e];
      if (j == i) continue;
      w = std::max(w, std::fabs(lv.X[3 * j + a0] - lv.X[3 * i + a0]));
      w = std::max(w, std::fabs(lv.X[3 * j + a1] - lv.X[3 * i + a1]));
    }
  if (!(w > 0.0)) return false;
  const double side = w * kBlockMargin;
  const int64_t ncx = (int64_t)std::floor(ext[a0] / side) + 1, ncy = (int64_t)std::floor(ext[a1] / side) + 1;
  if (ncx * ncy > kMaxGridCells) return false;
  const int64_t nbx = ncx / 2 + 1;
  std::vector<int64_t> cx(n), cy(n);
  std::vector<int64_t> brick_rows((size_t)(nbx * ncy), 0);
  for (int64_t i = 0; i < n; ++i) {
    cx[i] = (int64_t)std::floor((lv.X[3 * i + a0] - lo[a0]) / side);
    cy[i] = (int64_t)std::floor((lv.X[3 * i + a1] - lo[a1]) / side);
    brick_rows[cy[i] * nbx + (cx[i] + cy[i] % 2) / 2] += 1;
  }
  const bool bricks = *std::max_element(brick_rows.begin(), brick_rows.end()) <= kMaxBrickRows;
  lv.block_color.assign(n, 0);
  cell.assign(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (bricks) {
      const int64_t bx = (cx[i] + cy[i] % 2) / 2;
      const int64_t a = bx - (cy[i] + 1) / 2;
      lv.block_color[i] = (int32_t)(((a - cy[i]) % 3 + 3) % 3);
      cell[i] = cy[i] * nbx + bx;
    } else {
      lv.block_color[i] = (int32_t)((cx[i] & 1) + 2 * (cy[i] & 1));
      cell[i] = cy[i] * ncx + cx[i];
    }
  }
  return true;
}

// DSATUR colouring (Brelaz) of a graph on m vertices given by adjacency
// lists: repeatedly the uncoloured vertex with the most distinct colours
// among its coloured neighbours (its saturation) is coloured, ties going to
// the larger degree and then to the smaller vertex number, with the smallest
// colour none of its neighbours has.  Returns the number of colours, or -1 if
// a vertex would need colour kMaxCellColors or more.
int32_t dsatur(int32_t m, const std::vector<std::vector<int32_t>>& adj, std::vector<int32_t>& col) {
  col.assign(m, -1);
  std::vector<std::vector<char>> seen(m, std::vector<char>(kMaxCellColors, 0));
  std::vector<int32_t> sat(m, 0);
  int32_t ncol = 0;
  for (int32_t step = 0; step < m; ++step) {
    int32_t v = -1;
    for (int32_t u = 0; u < m; ++u) {
      if (col[u] >= 0) continue;
      if (v < 0 || sat[u] > sat[v] || (sat[u] == sat[v] && adj[u].size() > adj[v].size())) v = u;
    }
    int32_t c = 0;
    while (c < kMaxCellColors && seen[v][c]) ++c;
    if (c == kMaxCellColors) return -1;
    col[v] = c;
    ncol = std::max(ncol, c + 1);
    for (int32_t u : adj[v])
      if (!seen[u][c]) {
        seen[u][c] = 1;
        ++sat[u];
      }
  }
  return ncol;
}

// The colouring of a level swept in block order (a reading, like the block
// order itself): each block's rows are coloured on their own, by DSATUR on
// the couplings of A_l between rows of that block (rows numbered by ascending
// index within the block), since rows of different blocks of one block colour
// are never coupled.  A block with more than kMaxCellRows rows, or one that
// needs kMaxCellColors colours or more, sends the level back to the colour
// order (returns false).  cell[i] is row i's block.
bool cell_colouring(Level& lv, const std::vector<int64_t>& cell) {
  const int64_t n = lv.n;
  std::vector<int64_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cell[a] < cell[b]; });
  std::vector<int32_t> local(n, -1), color(n, -1);
  int32_t ncolors = 0;
  for (int64_t a = 0; a < n;) {
    int64_t b = a;
    while (b < n && cell[order[b]] == cell[order[a]]) ++b;
    const int32_t m = (int32_t)(b - a);
    if (m > kMaxCellRows) return false;
    for (int32_t p = 0; p < m; ++p) local[order[a + p]] = p;
    std::vector<std::vector<int32_t>> adj(m);
    for (int32_t p = 0; p < m; ++p) {
      const int64_t i = order[a + p];
      for (int32_t e = lv.arp[i]; e < lv.arp[i + 1]; ++e) {
        const int64_t j = lv.acol[e];
        if (j != i && cell[j] == cell[i]) adj[p].push_back(local[j]);
      }
    }
    std::vector<int32_t> col;
    const int32_t nc = dsatur(m, adj, col);
    if (nc < 0) return false;
    for (int32_t p = 0; p < m; ++p) color[order[a + p]] = col[p];
    ncolors = std::max(ncolors, nc);
    a = b;
  }
  lv.color.swap(color);
  lv.ncolors = ncolors;
  return true;
}

// The rows in sweep order, sorted by (block colour, colour, index); rows of
// one (block colour, colour) class are never coupled.
void sweep_order(Level& lv) {
  const int64_t n = lv.n;
  const int32_t C = lv.ncolors;
  const int32_t K = lv.block_color.empty() ? C : 4 * C;
  auto key = [&](int64_t v) { return (lv.block_color.empty() ? 0 : lv.block_color[v] * C) + lv.color[v]; };
  lv.color_ptr.assign(K + 1, 0);
  for (int64_t v = 0; v < n; ++v) lv.color_ptr[key(v) + 1] += 1;
  for (int32_t c = 0; c < K; ++c) lv.color_ptr[c + 1] += lv.color_ptr[c];
  lv.color_rows.assign(n, 0);
  std::vector<int32_t> fill(lv.color_ptr.begin(), lv.color_ptr.end() - 1);
  for (int64_t v = 0; v < n; ++v) lv.color_rows[fill[key(v)]++] = (int32_t)v;
}

// ---------------------------------------------------------------- coarsest level (Alg. 2)
// Dense Cholesky A = L L^T, column by column; each inner sum subtracts the
// terms in ascending k.  A non-positive pivot means A is not SPD.
int cholesky(const Level& lv, std::vector<double>& Lf) {
  int64_t n = lv.n;
  std::vector<double> A(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t e = lv.arp[i]; e < lv.arp[i + 1]; ++e) A[i * n + lv.acol[e]] = lv.aval[e];
  Lf.assign(n * n, 0.0);
  for (int64_t j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int64_t k = 0; k < j; ++k) s = s - Lf[j * n + k] * Lf[j * n + k];
    if (!(s > 0.0)) return NOT_SPD;
    double d = std::sqrt(s);
    Lf[j * n + j] = d;
    for (int64_t i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int64_t k = 0; k < j; ++k) t = t - Lf[i * n + k] * Lf[j * n + k];
      Lf[i * n + j] = t / d;
    }
  }
  return OK;
}

// A x = b by forward (L y = b) and back (L^T x = y) substitution.  Forward,
// row i subtracts L_ik y_k for k ascending; back, row i subtracts L_ki x_k for
// k descending from n-1 (the order in which the x_k become known).
void cholesky_solve(const std::vector<double>& Lf, int64_t n, const double* b, double* x) {
  std::vector<double> y(n);
  for (int64_t i = 0; i < n; ++i) {
    double s = b[i];
    for (int64_t k = 0; k < i; ++k) s = s - Lf[i * n + k] * y[k];
    y[i] = s / Lf[i * n + i];
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int64_t k = n - 1; k > i; --k) s = s - Lf[k * n + i] * x[k];
    x[i] = s / Lf[i * n + i];
  }
}

// The direct solve of the coarsest level (Alg. 2) as a product with A^-1:
// column k of A^-1 is A^-1 e_k, by the substitutions above (inv[k n + i]).
void coarse_inverse(const std::vector<double>& Lf, int64_t n, std::vector<double>& inv) {
  inv.assign(n * n, 0.0);
  std::vector<double> e(n, 0.0);
  for (int64_t k = 0; k < n; ++k) {
    e[k] = 1.0;
    cholesky_solve(Lf, n, e.data(), &inv[k * n]);
    e[k] = 0.0;
  }
}

// x = A^-1 b: x_i = sum over k ascending of (A^-1 e_k)_i b_k.
void coarse_solve(const std::vector<double>& inv, int64_t n, const double* b, double* x) {
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t k = 0; k < n; ++k) s = s + inv[k * n + i] * b[k];
    x[i] = s;
  }
}

// ---------------------------------------------------------------- solve (Alg. 1, Alg. 2)
// One Gauss-Seidel update: x_i <- (b_i - sum_{j != i} A_ij x_j) / A_ii, the
// sum taken in the CSR order of row i.
inline void gs_row(const Level& lv, int32_t i, const double* b, double* x) {
  double s = 0.0;
  for (int32_t e = lv.arp[i]; e < lv.arp[i + 1]; ++e) {
    int32_t j = lv.acol[e];
    if (j != i) s = s + lv.aval[e] * x[j];
  }
  x[i] = (b[i] - s) / lv.adiag[i];
}

void gs_sweep(const Level& lv, const double* b, double* x, int mode) {
  if (mode == 1) {                               // lexicographic (input order)
    for (int64_t i = 0; i < lv.n; ++i) gs_row(lv, (int32_t)i, b, x);
  } else {                                       // multicolour: colours ascending
    for (int64_t t = 0; t < lv.n; ++t) gs_row(lv, lv.color_rows[t], b, x);
  }
}

void residual(const Level& lv, const double* b, const double* x, double* r) {
  for (int64_t i = 0; i < lv.n; ++i) {
    double s = 0.0;
    for (int32_t e = lv.arp[i]; e < lv.arp[i + 1]; ++e) s = s + lv.aval[e] * x[lv.acol[e]];
    r[i] = b[i] - s;
  }
}

double norm2(const double* v, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s = s + v[i] * v[i];
  return std::sqrt(s);
}

// MGI(x, b, l): pre-relax, restrict the residual, recurse from zero, prolong
// and correct the pre-relaxed iterate, post-relax; solve directly at the
// coarsest level.  (The correction is added to the pre-relaxed iterate y.)
void vcycle(const Hier& h, size_t l, const double* b, double* x, int mode) {
  const Level& lv = h.L[l];
  if (l + 1 == h.L.size()) {
    coarse_solve(h.cinv, lv.n, b, x);
    return;
  }
  for (int s = 0; s < h.opt.nu_pre; ++s) gs_sweep(lv, b, x, mode);
  std::vector<double> r(lv.n);
  residual(lv, b, x, r.data());
  const Level& cl = h.L[l + 1];
  std::vector<double> bc(cl.n, 0.0), xc(cl.n, 0.0);
  for (int64_t i = 0; i < lv.n; ++i)                     // b_c = P^T r, ascending i
    for (int t = 0; t < lv.pcnt[i]; ++t) {
      int32_t I = lv.pcol[3 * i + t];
      bc[I] = bc[I] + lv.pval[3 * i + t] * r[i];
    }
  vcycle(h, l + 1, bc.data(), xc.data(), mode);
  for (int64_t i = 0; i < lv.n; ++i) {                   // x <- x + P x_c
    double s = 0.0;
    for (int t = 0; t < lv.pcnt[i]; ++t) s = s + lv.pval[3 * i + t] * xc[lv.pcol[3 * i + t]];
    x[i] = x[i] + s;
  }
  for (int s = 0; s < h.opt.nu_post; ++s) gs_sweep(lv, b, x, mode);
}

// ---------------------------------------------------------------- CG preconditioner, mixed precision
// A V-cycle used as the preconditioner B of conjugate gradients (the paper's
// conclusion, Sec. 6, names the method as a Krylov preconditioner).  For B to
// be symmetric the post-smoothing sweeps are the adjoints of the
// pre-smoothing sweeps: pre-smoothing visits the colours in ascending order,
// post-smoothing in descending order.  The cycle starts from x = 0 on every
// level.  Its arithmetic runs in T (double, or float for the mixed form): the
// values of A_l and P_l are rounded to T once per use and every product and
// sum is one T operation in the order written.  The coarsest level is solved
// in double with the Cholesky factor; its right-hand side is widened from T
// and its solution rounded to T.
template <class T>
inline void gs_row_t(const Level& lv, int32_t i, const T* b, T* x) {
  T s = T(0);
  for (int32_t e = lv.arp[i]; e < lv.arp[i + 1]; ++e) {
    int32_t j = lv.acol[e];
    if (j != i) s = s + (T)lv.aval[e] * x[j];
  }
  x[i] = (b[i] - s) / (T)lv.adiag[i];
}

template <class T>
void gs_sweep_t(const Level& lv, const T* b, T* x, bool descending) {
  if (!descending)
    for (int64_t t = 0; t < lv.n; ++t) gs_row_t(lv, lv.color_rows[t], b, x);
  else
    for (int64_t t = lv.n - 1; t >= 0; --t) gs_row_t(lv, lv.color_rows[t], b, x);
}

template <class T>
void vcycle_sym(const Hier& h, size_t l, const T* b, T* x) {
  const Level& lv = h.L[l];
  for (int64_t i = 0; i < lv.n; ++i) x[i] = T(0);
  if (l + 1 == h.L.size()) {
    std::vector<double> bd(lv.n), xd(lv.n);
    for (int64_t i = 0; i < lv.n; ++i) bd[i] = (double)b[i];
    coarse_solve(h.cinv, lv.n, bd.data(), xd.data());
    for (int64_t i = 0; i < lv.n; ++i) x[i] = (T)xd[i];
    return;
  }
  for (int s = 0; s < h.opt.nu_pre; ++s) gs_sweep_t(lv, b, x, false);
  std::vector<T> r(lv.n);
  for (int64_t i = 0; i < lv.n; ++i) {                   // r = b - A y
    T s = T(0);
    for (int32_t e = lv.arp[i]; e < lv.arp[i + 1]; ++e) s = s + (T)lv.aval[e] * x[lv.acol[e]];
    r[i] = b[i] - s;
  }
  const Level& cl = h.L[l + 1];
  std::vector<T> bc(cl.n, T(0)), xc(cl.n);
  for (int64_t i = 0; i < lv.n; ++i)                     // b_c = P^T r, ascending i
    for (int t = 0; t < lv.pcnt[i]; ++t) {
      int32_t I = lv.pcol[3 * i + t];
      bc[I] = bc[I] + (T)lv.pval[3 * i + t] * r[i];
    }
  vcycle_sym(h, l + 1, bc.data(), xc.data());
  for (int64_t i = 0; i < lv.n; ++i) {                   // x <- y + P x_c
    T s = T(0);
    for (int t = 0; t < lv.pcnt[i]; ++t) s = s + (T)lv.pval[3 * i + t] * xc[lv.pcol[3 * i + t]];
    x[i] = x[i] + s;
  }
  for (int s = 0; s < h.opt.nu_post; ++s) gs_sweep_t(lv, b, x, true);
}

// z = B r.  precision 0: double throughout; 1: r is rounded to float, the
// cycle runs in float, z is widened back.
void precondition(const Hier& h, const double* r, double* z, int precision) {
  const int64_t n = h.L[0].n;
  if (precision == 0) {
    vcycle_sym<double>(h, 0, r, z);
    return;
  }
  std::vector<float> rf(n), zf(n);
  for (int64_t i = 0; i < n; ++i) rf[i] = (float)r[i];
  vcycle_sym<float>(h, 0, rf.data(), zf.data());
  for (int64_t i = 0; i < n; ++i) z[i] = (double)zf[i];
}

double dotp(const double* u, const double* v, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s = s + u[i] * v[i];
  return s;
}

void matvec(const Level& lv, const double* x, double* y) {
  for (int64_t i = 0; i < lv.n; ++i) {
    double s = 0.0;
    for (int32_t e = lv.arp[i]; e < lv.arp[i + 1]; ++e) s = s + lv.aval[e] * x[lv.acol[e]];
    y[i] = s;
  }
}

int check_options(const Options& o) {
  if (o.struct_size != (int32_t)sizeof(Options)) return INVALID_ARGUMENT;
  if (!(o.coarsening_ratio > 0.0 && o.coarsening_ratio < 1.0)) return INVALID_ARGUMENT;
  if (o.min_coarse_points < 1 || o.max_levels < 1 || o.nu_pre < 0 || o.nu_post < 0) return INVALID_ARGUMENT;
  if (o.sample_order != 0 && o.sample_order != 1) return INVALID_ARGUMENT;
  if (o.weighting < 0 || o.weighting > 2 || (o.fallback_on_vertex != 0 && o.fallback_on_vertex != 1) ||
      o.color_passes < 0 || o.color_passes > 64 || o.block_min_rows < 0 || (o.autotune != 0 && o.autotune != 1))
    return INVALID_ARGUMENT;
  return OK;
}

}  // namespace

// ================================================================ C interface
extern "C" {

int orc_options_size() { return (int)sizeof(Options); }

int orc_build(int64_t n, const double* pts, int64_t m, const int32_t* edges, const int32_t* arp,
              const int32_t* acol, const double* aval, int64_t nnz, const void* opt_in, void** out) {
  *out = nullptr;
  if (n <= 0 || m < 0 || nnz < n || !pts || (m > 0 && !edges) || !arp || !acol || !aval || !opt_in)
    return INVALID_ARGUMENT;
  Hier* h = new Hier();
  std::memcpy(&h->opt, opt_in, sizeof(Options));
  int st = check_options(h->opt);
  if (st != OK) { delete h; return st; }
  const Options& o = h->opt;
  const double rho = std::cbrt(1.0 / o.coarsening_ratio);
  h->L.emplace_back();
  st = canonicalise(h->L[0], n, pts, m, edges);
  if (st == OK) st = take_matrix(h->L[0], arp, acol, aval, nnz);
  if (st != OK) { delete h; return st; }
  // Sec. 4.2: coarsen while a level has more than min_coarse_points points.
  while (h->L.back().n > o.min_coarse_points && (int)h->L.size() < o.max_levels) {
    int l = (int)h->L.size() - 1;
    Level& lv = h->L[l];
    edge_weights(lv);
    mean_edge(lv, rho);
    sample(lv, l, o);
    if ((int64_t)lv.samples.size() == lv.n) break;          // no progress: stop here
    voronoi(lv);
    Level nx;
    cells_and_shift(lv, nx, o.shift_coarse_points != 0);
    coarse_edges(lv, nx);
    prolongation(lv, nx, o);
    st = galerkin(lv, nx);
    if (st != OK) { delete h; return st; }
    h->L.push_back(std::move(nx));
  }
  Level& last = h->L.back();
  if (last.ew.empty() && !last.ecol.empty()) edge_weights(last);
  last.samples.clear();
  last.label.clear();
  last.dist.clear();
  if (last.n > kMaxDenseCoarse) { delete h; return DEGENERATE; }
  for (size_t l = 0; l + 1 < h->L.size(); ++l) {
    Level& lv = h->L[l];
    bool blocked = false;
    if (l >= 1 && lv.n > o.block_min_rows) {
      std::vector<int64_t> cell;
      blocked = block_order(lv, cell) && cell_colouring(lv, cell);
      if (!blocked) lv.block_color.clear();
    }
    if (!blocked) colouring(lv, (int)l, o);
    sweep_order(lv);
  }
  st = cholesky(last, h->chol);
  if (st != OK) { delete h; return st; }
  coarse_inverse(h->chol, last.n, h->cinv);
  *out = h;
  return OK;
}

void orc_free(void* hp) { delete static_cast<Hier*>(hp); }

int orc_num_levels(void* hp) { return hp ? (int)static_cast<Hier*>(hp)->L.size() : 0; }

// sizes[0..8]: n, undirected edges, nnz(A), nnz(P), colours, fallback rows, samples, nnz(E CSR),
// 1 if the level sweeps in block order
int orc_level_sizes(void* hp, int32_t l, int64_t* sizes) {
  Hier* h = static_cast<Hier*>(hp);
  if (!h || l < 0 || l >= (int32_t)h->L.size()) return INVALID_ARGUMENT;
  const Level& lv = h->L[l];
  int64_t nnzp = 0;
  for (int32_t c : lv.pcnt) nnzp += c;
  sizes[0] = lv.n;
  sizes[1] = (int64_t)lv.ecol.size() / 2;
  sizes[2] = (int64_t)lv.acol.size();
  sizes[3] = nnzp;
  sizes[4] = lv.ncolors;
  sizes[5] = lv.fallback;
  sizes[6] = (int64_t)lv.samples.size();
  sizes[7] = (int64_t)lv.ecol.size();
  sizes[8] = lv.block_color.empty() ? 0 : 1;
  return OK;
}

int orc_export(void* hp, int32_t l, int32_t what, void* dst, int64_t bytes) {
  Hier* h = static_cast<Hier*>(hp);
  if (!h || l < 0 || l >= (int32_t)h->L.size() || !dst) return INVALID_ARGUMENT;
  const Level& lv = h->L[l];
  const void* src = nullptr;
  int64_t nb = 0;
  double sc[2] = {lv.ehat, lv.r};
  switch (what) {
    case W_POSITIONS: src = lv.X.data(); nb = 8 * (int64_t)lv.X.size(); break;
    case W_EDGE_ROWPTR: src = lv.erp.data(); nb = 4 * (int64_t)lv.erp.size(); break;
    case W_EDGE_COL: src = lv.ecol.data(); nb = 4 * (int64_t)lv.ecol.size(); break;
    case W_EDGE_W: src = lv.ew.data(); nb = 8 * (int64_t)lv.ew.size(); break;
    case W_SCALARS: src = sc; nb = 16; break;
    case W_SAMPLES: src = lv.samples.data(); nb = 4 * (int64_t)lv.samples.size(); break;
    case W_LABELS: src = lv.label.data(); nb = 4 * (int64_t)lv.label.size(); break;
    case W_DIST: src = lv.dist.data(); nb = 8 * (int64_t)lv.dist.size(); break;
    case W_P_COL: src = lv.pcol.data(); nb = 4 * (int64_t)lv.pcol.size(); break;
    case W_P_VAL: src = lv.pval.data(); nb = 8 * (int64_t)lv.pval.size(); break;
    case W_P_CNT: src = lv.pcnt.data(); nb = 4 * (int64_t)lv.pcnt.size(); break;
    case W_TRI: src = lv.tri.data(); nb = 4 * (int64_t)lv.tri.size(); break;
    case W_A_ROWPTR: src = lv.arp.data(); nb = 4 * (int64_t)lv.arp.size(); break;
    case W_A_COL: src = lv.acol.data(); nb = 4 * (int64_t)lv.acol.size(); break;
    case W_A_VAL: src = lv.aval.data(); nb = 8 * (int64_t)lv.aval.size(); break;
    case W_COLORS: src = lv.color.data(); nb = 4 * (int64_t)lv.color.size(); break;
    case W_CHOL:
      if (l + 1 != (int32_t)h->L.size()) return INVALID_ARGUMENT;
      src = h->chol.data(); nb = 8 * (int64_t)h->chol.size(); break;
    case W_BLOCK_COLORS: src = lv.block_color.data(); nb = 4 * (int64_t)lv.block_color.size(); break;
    case W_CINV:
      if (l + 1 != (int32_t)h->L.size()) return INVALID_ARGUMENT;
      src = h->cinv.data(); nb = 8 * (int64_t)h->cinv.size(); break;
    default: return INVALID_ARGUMENT;
  }
  if (bytes != nb) return INVALID_ARGUMENT;
  if (nb) std::memcpy(dst, src, nb);
  return OK;
}

// gs_mode 0: multicolour Gauss-Seidel (colours ascending), 1: lexicographic.
// hist (may be null) receives the relative residual after each V-cycle.
int orc_solve(void* hp, const double* b, double* x, double tol, int32_t max_iters, int32_t gs_mode,
              int32_t* iters, double* hist) {
  Hier* h = static_cast<Hier*>(hp);
  if (!h || !b || !x || max_iters < 1 || !(tol >= 0.0)) return INVALID_ARGUMENT;
  const Level& l0 = h->L[0];
  int64_t n = l0.n;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(b[i]) || !std::isfinite(x[i])) return INVALID_ARGUMENT;
  double nb = norm2(b, n);
  *iters = 0;
  if (nb == 0.0) {
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    return OK;
  }
  std::vector<double> r(n);
  for (int32_t it = 1; it <= max_iters; ++it) {
    vcycle(*h, 0, b, x, gs_mode);
    residual(l0, b, x, r.data());
    double rel = norm2(r.data(), n) / nb;
    if (hist) hist[it - 1] = rel;
    *iters = it;
    if (rel <= tol) return OK;
  }
  return NOT_CONVERGED;
}

// z = B r: one symmetric V-cycle from zero (precision 0: double, 1: float).
int orc_precondition(void* hp, const double* r, double* z, int32_t precision) {
  Hier* h = static_cast<Hier*>(hp);
  if (!h || !r || !z || (precision != 0 && precision != 1)) return INVALID_ARGUMENT;
  precondition(*h, r, z, precision);
  return OK;
}

// Conjugate gradients in double on A x = b, preconditioned by B (above),
// flexible form (Polak-Ribiere beta, which stays a CG method when B carries
// rounding of a lower precision):
//   r = b - A x, z = B r, p = z, rho = r.z
//   repeat: q = A p; alpha = rho / p.q; x += alpha p; r_old = r; r -= alpha q;
//           stop if |r| <= tol |b| and the true residual |b - A x| agrees;
//           z = B r; beta = (r.z - r_old.z) / rho; rho = r.z; p = z + beta p.
// If the recursive residual passes the test and the true one does not, r is
// replaced by the true residual and the iteration goes on.  hist[k] is the
// recursive |r| / |b| after iteration k+1; *final_rel the true one at the end.
int orc_solve_pcg(void* hp, const double* b, double* x, double tol, int32_t max_iters, int32_t precision,
                  int32_t* iters, double* hist, double* final_rel) {
  Hier* h = static_cast<Hier*>(hp);
  if (!h || !b || !x || !iters || !final_rel || max_iters < 1 || !(tol >= 0.0) ||
      (precision != 0 && precision != 1))
    return INVALID_ARGUMENT;
  const Level& l0 = h->L[0];
  const int64_t n = l0.n;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(b[i]) || !std::isfinite(x[i])) return INVALID_ARGUMENT;
  *iters = 0;
  *final_rel = 0.0;
  const double nb = norm2(b, n);
  if (nb == 0.0) {
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    return OK;
  }
  std::vector<double> r(n), r_old(n), z(n), p(n), q(n);
  matvec(l0, x, q.data());
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
  double rel = norm2(r.data(), n) / nb;
  *final_rel = rel;
  if (rel <= tol) return OK;
  precondition(*h, r.data(), z.data(), precision);
  p = z;
  double rho = dotp(r.data(), z.data(), n);
  for (int32_t it = 1; it <= max_iters; ++it) {
    matvec(l0, p.data(), q.data());
    const double pq = dotp(p.data(), q.data(), n);
    if (!(pq > 0.0) || !(rho > 0.0)) return NOT_SPD;
    const double alpha = rho / pq;
    for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
    r_old = r;
    for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
    rel = norm2(r.data(), n) / nb;
    if (hist) hist[it - 1] = rel;
    *iters = it;
    if (rel <= tol) {
      matvec(l0, x, q.data());
      for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
      *final_rel = norm2(r.data(), n) / nb;
      if (*final_rel <= tol) return OK;
    }
    precondition(*h, r.data(), z.data(), precision);
    const double rho_new = dotp(r.data(), z.data(), n);
    const double beta = (rho_new - dotp(r_old.data(), z.data(), n)) / rho;
    rho = rho_new;
    for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
  matvec(l0, x, q.data());
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
  *final_rel = norm2(r.data(), n) / nb;
  return NOT_CONVERGED;
}

// Single-step entry points, exposed so that tests can pin them in isolation.
// DSATUR on a graph given as CSR (rows 0..m-1, neighbour lists, no loops):
// writes every vertex's colour, returns the number of colours or -1.
int orc_dsatur(int32_t m, const int32_t* rp, const int32_t* col, int32_t* out) {
  if (m < 0) return -1;
  std::vector<std::vector<int32_t>> adj(m);
  for (int32_t v = 0; v < m; ++v) adj[v].assign(col + rp[v], col + rp[v + 1]);
  std::vector<int32_t> c;
  const int32_t nc = dsatur(m, adj, c);
  if (nc >= 0) std::copy(c.begin(), c.end(), out);
  return nc;
}

int orc_closest_point(const double* p, const double* a, const double* b, const double* c, double* w) {
  return closest_point({p[0], p[1], p[2]}, {a[0], a[1], a[2]}, {b[0], b[1], b[2]}, {c[0], c[1], c[2]}, w);
}

int orc_degenerate(const double* a, const double* b, const double* c) {
  return degenerate({a[0], a[1], a[2]}, {b[0], b[1], b[2]}, {c[0], c[1], c[2]}) ? 1 : 0;
}

uint64_t orc_mix64(uint64_t z) { return mix64(z); }

}  // extern "C"
