// Tile-sparse solve of the regularised normal equations of eq. (7) with the epsilon ladder of the text
// after it, for the fixed keyframe-pair pattern of a pose graph:
//   (H + lambda diag H + eps_r I) tau = -g,  eps_r = eps0 * mult^r,  r = 0 .. attempts-1,
// and a zero update (status -1) when every factorisation fails.
//
// The dense solver runs one dependent launch per 32-row panel, each ending in the factorisation of the
// next diagonal tile: its time is the number of panels times a launch and a tile factorisation. Here the
// 32x32 float64 tiles keep that machinery, but the rows are laid out so that independent parts of the
// pose graph fall into different tiles, and the launches follow the elimination tree of the tiles rather
// than the panel order:
//
// Symbolic analysis (host, once per pattern):
//   * two elimination orders of the keyframe graph, minimum degree and nested dissection, and their
//     elimination trees (every layout below is tried for both);
//   * a layout of the keyframes' 7-row blocks along a postorder of that tree in which every child
//     subtree of a node except its largest (the last one laid out before the node) is aligned to whole
//     tiles when it holds at least `thr` keyframes, so that sibling subtrees share no tile (padding rows
//     are identity rows with a zero right-hand side); the order and threshold with the fewest tree levels
//     win, then the fewest factor tiles;
//   * the tile pattern of H in that layout, its symbolic tile Cholesky factorisation (column K's rows,
//     closed under the elimination: fill included), the tile elimination tree and its levels;
//   * per level l, the trailing tiles (I, J) that the level's pivot columns K update (I, J both rows of
//     column K), each with the list of its pivots.
// Numeric solve (one launch per level, so that kernel boundaries order everything):
//   init      every factor tile from H (only the blocks of the keyframe pattern are read) and -g; the
//             level-0 diagonal tiles are factored at once;
//   level l   one workgroup per trailing tile (I, J) with updates in this launch: for each of its pivots
//             K (of level l, or of earlier levels for an off-diagonal tile whose updates are spread over
//             the launches before it is read) it forms L_IK = A_IK Inv_K^T and L_JK, subtracts
//             L_IK L_JK^T; the workgroup of a diagonal tile (I, I) also stores L_IK and eliminates
//             b_I -= L_IK y_K, and factors the tile when it is on the next level;
//   backsub   one workgroup per tile column, dataflow over the tree: column K waits for the solution of
//             the tile rows of its column (its ancestors), solves x_K = Inv_K^T (y_K - sum L_IK^T x_I) with
//             everything but its parent's term done before the parent's solution arrives, and publishes
//             it; every wait is bounded.
// The diagonal factorisations, the tile products and the inverse of each diagonal factor are the dense
// solver's (shared tile primitives). Attempt 0 runs this way; when it fails, the dense solver's
// persistent fallback runs attempts 1.. from H in the caller's dense workspace.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "chol_tile.hpp"
#include "internal.hpp"

namespace ds3 {

constexpr int kTcThreads = 256;
constexpr int kTcMaxKf = 8192 / 7;      // the order limit of the dense solver, in keyframes
constexpr int kTcMaxTiles = 1024;       // tile columns: the back substitution keeps one workgroup per column
constexpr int kTcMaxAttempts = 16;
constexpr long kTcSpinLimit = 1L << 20;  // polls of about a microsecond each
constexpr int kTgtWords = 6;            // per trailing tile of a level: slot, I, J, pivot begin, end, flags
constexpr int kPivWords = 3;            // per pivot of a trailing tile: K, slot of (I, K), slot of (J, K)

// ---------------------------------------------------------------------------------------------------
// Host: symbolic analysis
// ---------------------------------------------------------------------------------------------------
struct TcSymbolic {
  int n_kf = 0, n = 0, np = 0, nt = 0, nlev = 0, thr = 0;
  int64_t nslot = 0, nupd = 0;
  std::vector<int32_t> kf_row0;     // n_kf: first layout row of each keyframe's 7 rows
  std::vector<int32_t> rowmap;      // np: row of H of each layout row, -1 for padding
  std::vector<int32_t> col_ptr;     // nt + 1: slots of tile column K, the diagonal tile first
  std::vector<int32_t> slot_row;    // tile row of each slot (rows increase within a column)
  std::vector<int32_t> slot_col;    // tile column of each slot
  std::vector<int32_t> tlevel;      // nt: level in the tile elimination tree (leaves 0)
  std::vector<int32_t> init_order;  // slots in the order the init launch takes them (level-0 diagonals first)
  std::vector<int32_t> lt_ptr;      // nlev: trailing tiles of the launch after level l: [lt_ptr[l], lt_ptr[l+1])
  std::vector<int32_t> tgt;         // kTgtWords per trailing tile
  std::vector<int32_t> piv;         // kPivWords per pivot
  std::vector<uint32_t> pat;        // n_kf^2 bits: keyframe pairs (and diagonals) whose block H holds
};

namespace {

struct Tree {
  std::vector<int> order;                // elimination order (keyframes)
  std::vector<int> parent, size;         // per keyframe
  std::vector<std::vector<int>> child;   // per keyframe, by (subtree size, id)
  std::vector<int> roots;                // by (subtree size, id)
};

// Keyframe order of the tile layout: a postorder of the tree; `pad[k]` after keyframe order[k] means the
// next keyframe starts a new tile.
void layout_order(const Tree& T, int thr, std::vector<int>& out, std::vector<uint8_t>& pad) {
  out.clear();
  pad.clear();
  // explicit stack: (node, next child index); children of a node are laid out in increasing size, and
  // every child but the last one that holds >= thr keyframes is fenced by tile boundaries
  struct Frame { int v, i; };
  std::vector<Frame> st;
  auto fence = [&]() {
    if (!pad.empty()) pad.back() = 1;
  };
  auto run = [&](int r) {
    st.push_back({r, 0});
    while (!st.empty()) {
      Frame& f = st.back();
      const std::vector<int>& ch = T.child[f.v];
      if (f.i > 0) {  // child f.i - 1 just finished
        const int c = ch[f.i - 1];
        if (f.i - 1 != int(ch.size()) - 1 && T.size[c] >= thr) fence();
      }
      if (f.i < int(ch.size())) {
        const int c = ch[f.i];
        if (f.i != int(ch.size()) - 1 && T.size[c] >= thr) fence();
        ++f.i;
        st.push_back({c, 0});
        continue;
      }
      out.push_back(f.v);
      pad.push_back(0);
      st.pop_back();
    }
  };
  for (size_t k = 0; k < T.roots.size(); ++k) {
    const int r = T.roots[k];
    const bool fenced = (k + 1 != T.roots.size()) && T.size[r] >= thr;
    if (fenced) fence();
    run(r);
    if (fenced) fence();
  }
}

struct TileShape {
  int np = 0, nt = 0, nlev = 0;
  int64_t nslot = 0;
  std::vector<int32_t> row0;
  std::vector<std::vector<int>> cols;  // per tile column: rows I > K of the filled factor, increasing
  std::vector<int> level;
};

// Layout rows, tile pattern, its symbolic factorisation and levels for one keyframe order.
void tile_shape(int n_kf, const std::vector<std::vector<int>>& adj, const std::vector<int>& ord,
                const std::vector<uint8_t>& pad, TileShape& S) {
  S.row0.assign(n_kf, 0);
  int r = 0;
  for (size_t k = 0; k < ord.size(); ++k) {
    S.row0[ord[k]] = r;
    r += 7;
    if (pad[k]) r = (r + NB - 1) / NB * NB;
  }
  S.np = std::max(NB, (r + NB - 1) / NB * NB);
  S.nt = S.np / NB;
  const int nt = S.nt, words = (nt + 63) / 64;
  std::vector<uint64_t> cur(size_t(nt) * words, 0);
  auto add = [&](int I, int J) {  // I > J
    cur[size_t(J) * words + I / 64] |= 1ull << (I % 64);
  };
  for (int v = 0; v < n_kf; ++v) {
    const int a0 = S.row0[v] / NB, a1 = (S.row0[v] + 6) / NB;
    auto tiles_of = [&](int u, int& b0, int& b1) {
      b0 = S.row0[u] / NB;
      b1 = (S.row0[u] + 6) / NB;
    };
    if (a1 > a0) add(a1, a0);
    for (int u : adj[v]) {
      int b0, b1;
      tiles_of(u, b0, b1);
      for (int I = a0; I <= a1; ++I)
        for (int J = b0; J <= b1; ++J)
          if (I > J) add(I, J);
    }
  }
  S.cols.assign(nt, {});
  S.level.assign(nt, 0);
  S.nslot = nt;
  for (int K = 0; K < nt; ++K) {
    const uint64_t* c = &cur[size_t(K) * words];
    std::vector<int>& rows = S.cols[K];
    for (int w = 0; w < words; ++w)
      for (uint64_t m = c[w]; m; m &= m - 1) rows.push_back(64 * w + __builtin_ctzll(m));
    S.nslot += int64_t(rows.size());
    if (rows.empty()) continue;
    const int p = rows[0];  // parent: the first row below the diagonal
    uint64_t* cp = &cur[size_t(p) * words];
    for (int w = 0; w < words; ++w) cp[w] |= c[w];
    cp[p / 64] &= ~(1ull << (p % 64));
    S.level[p] = std::max(S.level[p], S.level[K] + 1);
  }
  S.nlev = 1;
  for (int K = 0; K < nt; ++K) S.nlev = std::max(S.nlev, S.level[K] + 1);
}

// Symbolic elimination of the keyframe graph (bit rows `adj`, W words each) in a given order: rows[v] =
// the neighbours of v when it is eliminated, i.e. its column of the filled factor.
void eliminate(int n, std::vector<uint64_t> adj, const std::vector<int>& order, std::vector<std::vector<int>>& rows) {
  const int W = (n + 63) / 64;
  rows.assign(n, {});
  for (int v : order) {
    const uint64_t* av = &adj[size_t(v) * W];
    std::vector<int>& nb = rows[v];
    for (int w = 0; w < W; ++w)
      for (uint64_t m = av[w]; m; m &= m - 1) nb.push_back(64 * w + __builtin_ctzll(m));
    for (int a : nb) {
      uint64_t* aa = &adj[size_t(a) * W];
      for (int w = 0; w < W; ++w) aa[w] |= av[w];
      aa[a / 64] &= ~(1ull << (a % 64));
      aa[v / 64] &= ~(1ull << (v % 64));
    }
  }
}

// Nested-dissection order of the keyframe graph. A vertex set (taken in increasing id) is ordered so:
//   * several connected components: each in turn, in order of their smallest id;
//   * at most kNdLeaf keyframes: increasing id;
//   * otherwise a breadth-first search of the set from its smallest id, repeated three times from the
//     farthest vertex found (the smallest id among the farthest), gives levels from a pseudo-peripheral
//     vertex; with fewer than three levels (too dense to split) the set keeps increasing id; else the
//     balanced level c0 is the smallest of 1 .. L-1 (L the last level) holding half the set with the
//     levels below it (L-1 if none does). A cut at level c splits the set into the near side (the levels
//     below c plus the level-c vertices with no neighbour on level c+1), the far side (the levels above c)
//     and the separator (the rest of level c); among the cuts c0 - window .. c0 + window within 1 .. L-1
//     the one with the smallest separator, then the smallest difference of the sides, then the lowest
//     level is taken. The near side, then the far side are ordered recursively, then the separator in
//     increasing id.
// On chains of keyframes the elimination tree is then about logarithmic in height instead of linear.
constexpr int kNdLeaf = 4;
void nd_order(int n, const std::vector<std::vector<int>>& adj, int window, std::vector<int>& order) {
  order.clear();
  std::vector<int> stamp(n, 0), lev(n, -1), comp(n, -1);
  int epoch = 0;
  // components of S (sorted by id), each as its own sorted list, in order of their smallest member
  auto components = [&](const std::vector<int>& S, std::vector<std::vector<int>>& out) {
    out.clear();
    ++epoch;
    for (int v : S) stamp[v] = epoch;
    for (int v : S) comp[v] = -1;
    for (int r : S) {
      if (comp[r] >= 0) continue;
      out.push_back({r});
      comp[r] = int(out.size()) - 1;
      for (size_t h = 0; h < out.back().size(); ++h)
        for (int u : adj[out.back()[h]])
          if (stamp[u] == epoch && comp[u] < 0) {
            comp[u] = comp[r];
            out.back().push_back(u);
          }
      std::sort(out.back().begin(), out.back().end());
    }
  };
  // breadth-first levels within S (stamped with the current epoch) from r; returns the farthest vertex
  auto bfs = [&](const std::vector<int>& S, int r, int& maxlev) {
    for (int v : S) lev[v] = -1;
    std::vector<int> q{r};
    lev[r] = 0;
    int far = r;
    for (size_t h = 0; h < q.size(); ++h) {
      const int v = q[h];
      if (lev[v] > lev[far] || (lev[v] == lev[far] && v < far)) far = v;
      for (int u : adj[v])
        if (stamp[u] == epoch && lev[u] < 0) {
          lev[u] = lev[v] + 1;
          q.push_back(u);
        }
    }
    maxlev = lev[far];
    return far;
  };
  // explicit stack of tasks: a vertex set to order, or a separator to append (emit)
  struct Task { std::vector<int> set; bool emit; };
  std::vector<Task> st(1);
  for (int v = 0; v < n; ++v) st[0].set.push_back(v);
  st[0].emit = false;
  while (!st.empty()) {
    Task t = std::move(st.back());
    st.pop_back();
    if (t.emit) {
      for (int v : t.set) order.push_back(v);
      continue;
    }
    std::sort(t.set.begin(), t.set.end());
    std::vector<std::vector<int>> cs;
    components(t.set, cs);
    if (cs.size() > 1) {
      for (size_t c = cs.size(); c-- > 0;) st.push_back({std::move(cs[c]), false});
      continue;
    }
    std::vector<int>& S = cs[0];
    if (int(S.size()) <= kNdLeaf) {
      std::sort(S.begin(), S.end());
      for (int v : S) order.push_back(v);
      continue;
    }
    ++epoch;
    for (int v : S) stamp[v] = epoch;
    int L = 0;
    int r = *std::min_element(S.begin(), S.end());
    for (int sweep = 0; sweep < 3; ++sweep) r = bfs(S, r, L);
    bfs(S, r, L);
    if (L < 2) {
      std::sort(S.begin(), S.end());
      for (int v : S) order.push_back(v);
      continue;
    }
    std::vector<int> cnt(L + 1, 0);
    for (int v : S) ++cnt[lev[v]];
    int c0 = 1, below = cnt[0];
    while (c0 < L - 1 && 2 * (below + cnt[c0]) < int(S.size())) below += cnt[c0++];
    std::vector<int> a, b, sep;
    long best_key = -1;
    for (int cut = std::max(1, c0 - window); cut <= std::min(L - 1, c0 + window); ++cut) {
      std::vector<int> ca, cb, cs2;
      for (int v : S) {
        if (lev[v] < cut) ca.push_back(v);
        else if (lev[v] > cut) cb.push_back(v);
        else {
          bool far = false;
          for (int u : adj[v])
            if (stamp[u] == epoch && lev[u] == cut + 1) far = true;
          (far ? cs2 : ca).push_back(v);
        }
      }
      const long key = long(cs2.size()) * (n + 1) + std::abs(int(ca.size()) - int(cb.size()));
      if (best_key < 0 || key < best_key) {
        best_key = key;
        a.swap(ca);
        b.swap(cb);
        sep.swap(cs2);
      }
    }
    std::sort(sep.begin(), sep.end());
    st.push_back({std::move(sep), true});
    st.push_back({std::move(b), false});
    st.push_back({std::move(a), false});
  }
}

}  // namespace

static int tc_symbolic(int n_kf, int n_pairs, const int32_t* pair_ij, TcSymbolic& S) {
  if (n_kf < 1 || n_kf > kTcMaxKf) return fail(DS3_EINVAL, "tilechol: n_kf must be in 1 .. 1170");
  std::vector<std::vector<int>> md_rows;
  std::vector<uint64_t> bits;
  std::vector<int> md;
  DS3_TRY(min_degree_order(n_kf, n_pairs, pair_ij, md, md_rows, &bits));
  const int n = n_kf, W = (n + 63) / 64;
  std::vector<std::vector<int>> adj(n);
  for (int v = 0; v < n; ++v)
    for (int w = 0; w < W; ++w)
      for (uint64_t m = bits[size_t(v) * W + w]; m; m &= m - 1) adj[v].push_back(64 * w + __builtin_ctzll(m));
  // elimination tree of an order (parent = the earliest-eliminated row of a keyframe's factor column)
  auto build_tree = [&](const std::vector<int>& order, const std::vector<std::vector<int>>& rows, Tree& T) {
    T.order = order;
    std::vector<int> pos(n);
    for (int k = 0; k < n; ++k) pos[order[k]] = k;
    T.parent.assign(n, -1);
    T.size.assign(n, 1);
    T.child.assign(n, {});
    T.roots.clear();
    for (int v : order) {
      int p = -1;
      for (int u : rows[v])
        if (p < 0 || pos[u] < pos[p]) p = u;
      T.parent[v] = p;
    }
    for (int v : order)  // children are eliminated before their parent
      if (T.parent[v] >= 0) T.size[T.parent[v]] += T.size[v];
    for (int v = 0; v < n; ++v)
      if (T.parent[v] >= 0) T.child[T.parent[v]].push_back(v);
      else T.roots.push_back(v);
    auto by_size = [&](int a, int b) { return T.size[a] != T.size[b] ? T.size[a] < T.size[b] : a < b; };
    for (auto& c : T.child) std::sort(c.begin(), c.end(), by_size);
    std::sort(T.roots.begin(), T.roots.end(), by_size);
  };
  // elimination orders x the alignment thresholds: the fewest tree levels, then the fewest factor tiles
  // candidates: minimum degree, nested dissection at the balanced cut, and with the smallest separator
  // among the cuts one level around it
  Tree trees[3];
  build_tree(md, md_rows, trees[0]);
  for (int window = 0; window < 2; ++window) {
    std::vector<int> nd;
    std::vector<std::vector<int>> nd_rows;
    nd_order(n, adj, window, nd);
    eliminate(n, bits, nd, nd_rows);
    build_tree(nd, nd_rows, trees[1 + window]);
  }
  const int cand[] = {2, 3, 4, 6, 9, 14, 20, 1 << 30};
  TileShape best;
  std::vector<int> best_ord;
  int best_thr = 0;
  for (const Tree& T : trees)
    for (int thr : cand) {
      std::vector<int> ord;
      std::vector<uint8_t> pad;
      layout_order(T, thr, ord, pad);
      TileShape sh;
      tile_shape(n, adj, ord, pad, sh);
      if (sh.nt > kTcMaxTiles) continue;
      if (best_thr == 0 || sh.nlev < best.nlev || (sh.nlev == best.nlev && sh.nslot < best.nslot)) {
        best = std::move(sh);
        best_ord = ord;
        best_thr = thr;
      }
    }
  if (best_thr == 0) return fail(DS3_ENOSPACE, "tilechol: more than 1024 tiles in every layout");
  S.n_kf = n;
  S.n = 7 * n;
  S.np = best.np;
  S.nt = best.nt;
  S.nlev = best.nlev;
  S.thr = best_thr;
  S.kf_row0 = best.row0;
  S.rowmap.assign(S.np, -1);
  for (int v = 0; v < n; ++v)
    for (int d = 0; d < 7; ++d) S.rowmap[best.row0[v] + d] = 7 * v + d;
  // slots
  const int nt = S.nt;
  S.col_ptr.assign(nt + 1, 0);
  S.slot_row.clear();
  S.slot_col.clear();
  for (int K = 0; K < nt; ++K) {
    S.slot_row.push_back(K);
    S.slot_col.push_back(K);
    for (int I : best.cols[K]) {
      S.slot_row.push_back(I);
      S.slot_col.push_back(K);
    }
    S.col_ptr[K + 1] = int(S.slot_row.size());
  }
  S.nslot = int64_t(S.slot_row.size());
  S.tlevel.assign(best.level.begin(), best.level.end());
  auto slot_of = [&](int I, int K) -> int {
    if (I == K) return S.col_ptr[K];
    const auto b = S.slot_row.begin() + S.col_ptr[K] + 1, e = S.slot_row.begin() + S.col_ptr[K + 1];
    const auto it = std::lower_bound(b, e, I);
    return (it != e && *it == I) ? int(it - S.slot_row.begin()) : -1;
  };
  // init order: the level-0 diagonal tiles (factored by the init launch) first
  S.init_order.clear();
  for (int K = 0; K < nt; ++K)
    if (S.tlevel[K] == 0) S.init_order.push_back(S.col_ptr[K]);
  for (int s = 0; s < int(S.nslot); ++s)
    if (!(S.slot_row[s] == S.slot_col[s] && S.tlevel[S.slot_col[s]] == 0)) S.init_order.push_back(s);
  // trailing tiles per launch: target slot -> pivots. An update of (I, J) by pivot K can run in any launch
  // from level(K) on, as long as it is done before the tile is read: an off-diagonal tile (I, J) is read
  // as a pivot tile in the launch of level(J), so its updates may be spread over the launches up to
  // level(J) - 1; a diagonal tile (I, I) is factored in the launch of level(I) - 1, right after that
  // launch's own updates (its workgroup is on the critical path), so its earlier updates are spread over
  // the launches up to level(I) - 2. A launch takes at most kSpread of a tile's pending updates, or more
  // when the deadline needs it, so that no workgroup carries many more products than the factoring ones.
  constexpr int kSpread = 2;
  std::vector<std::vector<int>> lev_cols(S.nlev);
  for (int K = 0; K < nt; ++K) lev_cols[S.tlevel[K]].push_back(K);
  S.lt_ptr.assign(S.nlev, 0);
  S.tgt.clear();
  S.piv.clear();
  S.nupd = 0;
  std::vector<std::vector<int>> pending(S.nslot);
  std::vector<int> open;  // slots with pending updates
  for (int l = 0; l + 1 < S.nlev; ++l) {
    for (int K : lev_cols[l]) {
      const std::vector<int>& r = best.cols[K];
      for (size_t a = 0; a < r.size(); ++a)
        for (size_t b = 0; b <= a; ++b) {
          const int s = slot_of(r[a], r[b]);
          if (s < 0) return fail(DS3_EINVAL, "tilechol: internal error (update outside the factor pattern)");
          if (pending[s].empty()) open.push_back(s);
          pending[s].push_back(K);
        }
    }
    auto is_factor = [&](int s) { return S.slot_row[s] == S.slot_col[s] && S.tlevel[S.slot_row[s]] == l + 1; };
    std::vector<std::pair<int, int>> take;  // (slot, updates taken in this launch)
    std::vector<int> still;
    for (int s : open) {
      const int I = S.slot_row[s], J = S.slot_col[s];
      const int npend = int(pending[s].size());
      int t = npend;
      const int deadline = (I != J) ? S.tlevel[J] - 1 : S.tlevel[I] - 2;
      if (I != J && deadline < l) return fail(DS3_EINVAL, "tilechol: internal error (update after its deadline)");
      if (deadline >= l) {
        const int left = deadline - l + 1;
        t = std::min(npend, std::max((npend + left - 1) / left, kSpread));
      }
      take.push_back({s, t});
      if (t < npend) still.push_back(s);
    }
    std::sort(take.begin(), take.end(), [&](const std::pair<int, int>& a, const std::pair<int, int>& b) {
      const bool fa = is_factor(a.first), fb = is_factor(b.first);
      if (fa != fb) return fa;
      if (a.second != b.second) return a.second > b.second;
      return a.first < b.first;
    });
    S.lt_ptr[l] = int(S.tgt.size() / kTgtWords);
    for (const auto& st : take) {
      const int s = st.first, I = S.slot_row[s], J = S.slot_col[s];
      const int pb = int(S.piv.size() / kPivWords);
      for (int k = 0; k < st.second; ++k) {
        const int K = pending[s][k];
        S.piv.push_back(K);
        S.piv.push_back(slot_of(I, K));
        S.piv.push_back(slot_of(J, K));
      }
      const int pe = int(S.piv.size() / kPivWords);
      S.tgt.insert(S.tgt.end(), {s, I, J, pb, pe, is_factor(s) ? 1 : 0});
      S.nupd += pe - pb;
      pending[s].erase(pending[s].begin(), pending[s].begin() + st.second);
    }
    open.swap(still);
  }
  if (!open.empty()) return fail(DS3_EINVAL, "tilechol: internal error (updates left after the last launch)");
  if (S.nlev >= 1) S.lt_ptr.back() = int(S.tgt.size() / kTgtWords);
  // lt_ptr[l] .. lt_ptr[l + 1] for l < nlev - 1; the last entry closes the list
  // keyframe-pair pattern bits (diagonal blocks included)
  S.pat.assign((size_t(n) * n + 31) / 32, 0u);
  for (int a = 0; a < n; ++a) {
    const size_t d = size_t(a) * n + a;
    S.pat[d / 32] |= 1u << (d % 32);
    for (int b : adj[a]) {
      const size_t e = size_t(a) * n + b;
      S.pat[e / 32] |= 1u << (e % 32);
    }
  }
  return DS3_OK;
}

// ---------------------------------------------------------------------------------------------------
// Device side
// ---------------------------------------------------------------------------------------------------
struct TcArgs {
  const double* H;
  const double* g;
  int n, n_kf, np, nt;
  double lambda, eps0;
  int attempts;
  const int32_t* rowmap;
  const int32_t* slot_row;
  const int32_t* slot_col;
  const int32_t* col_ptr;
  const int32_t* tlevel;
  const int32_t* init_order;
  const int32_t* tgt;
  const int32_t* piv;
  const uint32_t* pat;
  double* W;    // nslot tiles: the trailing matrix (row-major 32x32 each)
  double* L;    // nslot tiles: the factor's off-diagonal tiles
  double* Inv;  // nt tiles: inverse of each diagonal factor
  double* b;    // np: -g after forward elimination
  double* y;    // np: L^-1 (-g) per tile
  double* x;    // np: solution tiles as published by the back substitution
  double* tau;
  int32_t* status;
  unsigned* sync;  // the dense workspace's words: [2] error, [3] attempt 0 failed
  unsigned* done;  // tile columns solved by the back substitution
};

__device__ inline bool in_pattern(const TcArgs& a, int rr, int cc) {
  const size_t e = size_t(rr / 7) * a.n_kf + cc / 7;
  return (a.pat[e / 32] >> (e % 32)) & 1u;
}

// Regularised lower tile (I, J) of the laid-out H as a fragment: entries of H outside the blocks of the
// keyframe pattern count as zero; padding rows are identity rows; zero above the diagonal.
__device__ inline void tc_frag_from_H(const TcArgs& a, int I, int J, f64x4& q) {
  const int C = J * NB + fcol();
  const int cc = a.rowmap[C];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int R = I * NB + frow(v);
    const int rr = a.rowmap[R];
    double x = 0.0;
    if (C <= R) {
      if (rr >= 0 && cc >= 0) {
        if (in_pattern(a, rr, cc)) {
          x = a.H[int64_t(max(rr, cc)) * a.n + min(rr, cc)];
          if (R == C) x += a.lambda * x + a.eps0;
        }
      } else if (R == C) {
        x = 1.0;
      }
    }
    q[v] = x;
  }
}

__global__ __launch_bounds__(kTcThreads) void k_tc_init(TcArgs a) {
  __shared__ double S[NB * LDT];
  __shared__ double fb[kFactorScratch];
  const int s = a.init_order[blockIdx.x];
  const int I = a.slot_row[s], J = a.slot_col[s];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *a.status = -2;  // replaced by the back substitution or the fallback
    *a.done = 0u;
  }
  f64x4 q;
  tc_frag_from_H(a, I, J, q);
  if (I != J) {
    frag_store(q, a.W + int64_t(s) * NB * NB, NB);
    return;
  }
  double* sb = fb + 4 * kFw * NB;
  if (threadIdx.x < NB) {
    const int R = I * NB + threadIdx.x, rr = a.rowmap[R];
    const double bv = (rr >= 0) ? -a.g[rr] : 0.0;
    a.b[R] = bv;
    sb[threadIdx.x] = bv;
    reinterpret_cast<unsigned long long*>(a.x)[R] = kXPending;
  }
  if (a.tlevel[I] != 0) {
    frag_store(q, a.W + int64_t(s) * NB * NB, NB);
    return;
  }
  __syncthreads();
  f64x4 Xq;
  if (!factor_frag(q, fb, Xq)) {
    if (threadIdx.x == 0) atomicOr(&a.sync[3], 1u);
    return;
  }
  diag_out(a.Inv + int64_t(I) * NB * NB, a.y + I * NB, Xq, S, sb);
}

// The trailing tiles of one level: workgroup -> target tgt[t0 + blockIdx.x].
__global__ __launch_bounds__(kTcThreads) void k_tc_level(TcArgs a, int t0) {
  if (a.sync[3] != 0u) return;  // attempt 0 already failed (uniform)
  __shared__ double S0[NB * LDT];
  __shared__ double S1[NB * LDT];
  __shared__ double S2[NB * LDT];
  __shared__ double fb[kFactorScratch];
  const int32_t* t = a.tgt + int64_t(t0 + blockIdx.x) * kTgtWords;
  const int s = t[0], I = t[1], J = t[2], pb = t[3], pe = t[4];
  const bool factor = t[5] != 0;
  const bool diag = (I == J);
  // the diagonal tiles factored in this launch are on the critical path of the whole solve: their waves
  // get issue priority over the other workgroups sharing their compute unit
  if (factor) __builtin_amdgcn_s_setprio(3);
  f64x4 acc;
  frag_load(acc, a.W + int64_t(s) * NB * NB, NB);
  double* sy = fb + 2 * kFw * NB;  // y_K while the factor scratch is unused (parity-1 buffer)
  double* sb = fb + 4 * kFw * NB;
  const int r8 = threadIdx.x >> 3, p8 = threadIdx.x & 7;
  double bi = 0.0;
  if (diag && p8 == 0) bi = a.b[I * NB + r8];
  // operands of pivot p: Inv_K, A_IK, A_JK (off-diagonal targets) and y_K (diagonal ones); the next
  // pivot's are loaded while the current one's products run
  f64x4 qinv, qi, qj = {0.0, 0.0, 0.0, 0.0};
  double yk = 0.0;
  auto load_pivot = [&](int p) {
    const int K = a.piv[kPivWords * p], sIK = a.piv[kPivWords * p + 1], sJK = a.piv[kPivWords * p + 2];
    frag_load(qinv, a.Inv + int64_t(K) * NB * NB, NB);
    frag_load(qi, a.W + int64_t(sIK) * NB * NB, NB);
    if (!diag) frag_load(qj, a.W + int64_t(sJK) * NB * NB, NB);
    if (diag && threadIdx.x < NB) yk = a.y[K * NB + threadIdx.x];
  };
  if (pb < pe) load_pivot(pb);
  for (int p = pb; p < pe; ++p) {
    const int sIK = a.piv[kPivWords * p + 1];
    __syncthreads();  // the previous pivot's readers of S0..S2 and sy are done
    frag_to_lds(qinv, S0);
    frag_to_lds(qi, S1);
    if (!diag) frag_to_lds(qj, S2);
    if (diag && threadIdx.x < NB) sy[threadIdx.x] = yk;
    if (p + 1 < pe) load_pivot(p + 1);
    __syncthreads();
    f64x4 li = {0.0, 0.0, 0.0, 0.0}, lj = {0.0, 0.0, 0.0, 0.0};
    frag_gemm_abt<false>(S1, S0, li);  // L_IK = A_IK Inv_K^T
    if (!diag) frag_gemm_abt<false>(S2, S0, lj);
    __syncthreads();
    frag_to_lds(li, S1);
    if (!diag) frag_to_lds(lj, S2);
    __syncthreads();
    frag_gemm_abt<true>(S1, diag ? S1 : S2, acc);  // A_IJ -= L_IK L_JK^T
    if (diag) {
      frag_store(li, a.L + int64_t(sIK) * NB * NB, NB);
      // forward elimination b_I -= L_IK y_K on 8 threads per row, reduced with lane shuffles
      double d = 0.0;
#pragma unroll
      for (int q = 0; q < NB / 8; ++q) d = fma(S1[r8 * LDT + p8 + 8 * q], sy[p8 + 8 * q], d);
      d += __shfl_xor(d, 1, 8);
      d += __shfl_xor(d, 2, 8);
      d += __shfl_xor(d, 4, 8);
      bi -= d;
    }
  }
  if (factor) {
    if (p8 == 0) sb[r8] = bi;
    __syncthreads();
    f64x4 Xq;
    if (!factor_frag(acc, fb, Xq)) {
      if (threadIdx.x == 0) atomicOr(&a.sync[3], 1u);
      return;
    }
    diag_out(a.Inv + int64_t(I) * NB * NB, a.y + I * NB, Xq, S0, sb);
    return;
  }
  if (diag && p8 == 0) a.b[I * NB + r8] = bi;
  frag_store(acc, a.W + int64_t(s) * NB * NB, NB);
}

__device__ inline unsigned tc_ld_acq(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline unsigned long long tc_x_load(const double* p) {
  return __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Back substitution, one workgroup per tile column K (the highest columns, the tree's roots, first):
//   x_K = Inv_K^T (y_K - sum_I L_IK^T x_I) = z_K - M_K x_p,
//   z_K = Inv_K^T (y_K - sum_{I != p} L_IK^T x_I),   M_K = Inv_K^T L_pK^T,
// p the parent of K (its lowest tile row). The rows I of the column are K's ancestors, and every one but
// p is also a row of p's column, so x_p is the last solution K waits for. Everything except the last
// product is done before it arrives: M_K on the matrix cores at the start; for the other rows, from the
// highest (solved first) down, the waves poll the 32 values of x_I (each value is its own ready flag: the
// signalling-NaN pending pattern until its owner stores it) and accumulate L_IK^T x_I with the next tile
// of L already loading, then z_K. One wave then polls x_p with two loads in flight, broadcasts its values
// from the lanes and finishes x_K[c] = z_K[c] - sum_r M_K[c][r] x_p[r] in each lane, without a barrier, and
// publishes it with relaxed agent-scope stores. A wait that times out sets sync[2]; the status then stays
// -2.
__device__ inline double lane_value(double v, int r) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), r);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), r);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

__global__ __launch_bounds__(kTcThreads) void k_tc_backsub(TcArgs a) {
  const int K = a.nt - 1 - int(blockIdx.x);
  if (a.sync[3] != 0u) {  // attempt 0 failed: the fallback takes over, or gives up with one attempt
    if (a.attempts == 1) {
      if (threadIdx.x < NB) {
        const int rr = a.rowmap[K * NB + threadIdx.x];
        if (rr >= 0) a.tau[rr] = 0.0;
      }
      if (blockIdx.x == 0 && threadIdx.x == 0) *a.status = -1;
    }
    return;
  }
  __shared__ double sInvT[NB * LDT];  // Inv_K transposed
  __shared__ double sM[NB * LDT];     // L_pK, then M_K
  __shared__ double red[2][NB];
  __shared__ double rs[NB];
  __shared__ double zs[NB];
  __shared__ int s_bad;
  const int c = fcol(), l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int sb = a.col_ptr[K] + 1, se = a.col_ptr[K + 1];
  const bool has_parent = se > sb;  // slot sb holds the parent row
  {
    f64x4 q, qL = {0.0, 0.0, 0.0, 0.0};
    frag_load(q, a.Inv + int64_t(K) * NB * NB, NB);
    if (has_parent) frag_load(qL, a.L + int64_t(sb) * NB * NB, NB);
#pragma unroll
    for (int v = 0; v < 4; ++v) sInvT[c * LDT + frow(v)] = q[v];
    frag_to_lds(qL, sM);
  }
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  f64x4 M = {0.0, 0.0, 0.0, 0.0};
  frag_gemm_abt<false>(sInvT, sM, M);  // M[c][r] = sum_u Inv_K[u][c] L_pK[r][u]
  // the other rows of the column, highest first
  double acc = 0.0;
  bool ok = true;
  f64x4 Lc = {0.0, 0.0, 0.0, 0.0}, Ln = {0.0, 0.0, 0.0, 0.0};
  if (se - 1 > sb) frag_load(Lc, a.L + int64_t(se - 1) * NB * NB, NB);
  for (int q = se - 1; q > sb; --q) {
    if (q - 1 > sb) frag_load(Ln, a.L + int64_t(q - 1) * NB * NB, NB);
    const int I = a.slot_row[q];
    const double* px = a.x + I * NB;
    unsigned long long v[4];
    long spins = 0;
    bool ready;
    do {
      ready = true;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        v[k] = tc_x_load(px + frow(k));
        ready = ready && (v[k] != kXPending);
      }
      if (__all(ready)) break;
      if (++spins > kTcSpinLimit ||
          __hip_atomic_load(&a.sync[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    } while (true);
    if (!ok) break;
#pragma unroll
    for (int k = 0; k < 4; ++k) acc = fma(Lc[k], __longlong_as_double(static_cast<long long>(v[k])), acc);
    Lc = Ln;
  }
  __syncthreads();  // every wave is past the product's reads of sM
  if (!ok) s_bad = 1;
  frag_to_lds(M, sM);
  // column c's partial sums: lanes l, l^16, l^32, l^48 of a wave, then the two row halves
  acc += __shfl_xor(acc, 16);
  acc += __shfl_xor(acc, 32);
  if (l < 16) red[w >> 1][c] = acc;
  __syncthreads();
  if (threadIdx.x < NB) rs[threadIdx.x] = a.y[K * NB + threadIdx.x] - (red[0][threadIdx.x] + red[1][threadIdx.x]);
  __syncthreads();
  {  // z_K[cz] = sum_u Inv_K[u][cz] rs[u], 8 threads per entry
    const int cz = threadIdx.x >> 3, p8 = threadIdx.x & 7;
    double z = 0.0;
#pragma unroll
    for (int q = 0; q < NB / 8; ++q) z = fma(sInvT[cz * LDT + p8 + 8 * q], rs[p8 + 8 * q], z);
    z += __shfl_xor(z, 1, 8);
    z += __shfl_xor(z, 2, 8);
    z += __shfl_xor(z, 4, 8);
    if (p8 == 0) zs[cz] = z;
  }
  __syncthreads();
  if (w != 0) return;
  const int cl = l & 31;
  bool good = !s_bad;
  double xk = zs[cl];
  if (good && has_parent) {
    double m[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) m[r] = sM[cl * LDT + r];
    const double* px = a.x + a.slot_row[sb] * NB + cl;
    unsigned long long cur = tc_x_load(px);
    long spins = 0;
    while (true) {
      const unsigned long long nxt = tc_x_load(px);  // the next poll is in flight while this one is tested
      if (__all(cur != kXPending)) break;
      if (++spins > kTcSpinLimit ||
          ((spins & 255) == 0 &&
           __hip_atomic_load(&a.sync[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
        good = false;
        break;
      }
      cur = nxt;
    }
    if (good) {
      const double xp = __longlong_as_double(static_cast<long long>(cur));
#pragma unroll
      for (int r = 0; r < NB; ++r) xk = fma(-m[r], lane_value(xp, r), xk);
    }
  }
  if (!good) {
    if (l == 0) atomicOr(&a.sync[2], 1u);
    if (l < NB) {
      const int rr = a.rowmap[K * NB + l];
      if (rr >= 0) a.tau[rr] = 0.0;
    }
    return;
  }
  if (l < NB) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(a.x + K * NB + l),
                       static_cast<unsigned long long>(__double_as_longlong(xk)), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    const int rr = a.rowmap[K * NB + l];
    if (rr >= 0) a.tau[rr] = xk;
  }
  if (l == 0) {
    const unsigned prev = atomicAdd(a.done, 1u);
    if (prev == unsigned(a.nt - 1)) *a.status = (tc_ld_acq(&a.sync[2]) != 0u) ? -2 : 0;
  }
}

// ---------------------------------------------------------------------------------------------------
// Host objects
// ---------------------------------------------------------------------------------------------------
struct TileChol {
  TcSymbolic S;
  void* mem = nullptr;
  int32_t *rowmap = nullptr, *slot_row = nullptr, *slot_col = nullptr, *col_ptr = nullptr, *tlevel = nullptr,
          *init_order = nullptr, *tgt = nullptr, *piv = nullptr;
  uint32_t* pat = nullptr;
  double *W = nullptr, *L = nullptr, *Inv = nullptr, *b = nullptr, *y = nullptr, *x = nullptr;
  unsigned* done = nullptr;
};

template <typename T>
static T* carve_copy(Carver& d, const std::vector<T>& v, std::vector<std::pair<void*, const void*>>& cp,
                     std::vector<size_t>& sz) {
  T* p = d.take<T>(std::max<size_t>(v.size(), 1));
  cp.push_back({p, v.data()});
  sz.push_back(sizeof(T) * v.size());
  return p;
}

int tilechol_create(int n_kf, int n_pairs, const int32_t* pair_ij, TileChol** out) {
  *out = nullptr;
  TileChol* P = new TileChol();
  int rc = tc_symbolic(n_kf, n_pairs, pair_ij, P->S);
  if (rc != DS3_OK) {
    delete P;
    return rc;
  }
  const TcSymbolic& S = P->S;
  auto plan = [&](Carver& c, std::vector<std::pair<void*, const void*>>& cp, std::vector<size_t>& sz) {
    P->rowmap = carve_copy(c, S.rowmap, cp, sz);
    P->slot_row = carve_copy(c, S.slot_row, cp, sz);
    P->slot_col = carve_copy(c, S.slot_col, cp, sz);
    P->col_ptr = carve_copy(c, S.col_ptr, cp, sz);
    P->tlevel = carve_copy(c, S.tlevel, cp, sz);
    P->init_order = carve_copy(c, S.init_order, cp, sz);
    P->tgt = carve_copy(c, S.tgt, cp, sz);
    P->piv = carve_copy(c, S.piv, cp, sz);
    P->pat = carve_copy(c, S.pat, cp, sz);
    P->W = c.take<double>(size_t(S.nslot) * NB * NB);
    P->L = c.take<double>(size_t(S.nslot) * NB * NB);
    P->Inv = c.take<double>(size_t(S.nt) * NB * NB);
    P->b = c.take<double>(S.np);
    P->y = c.take<double>(S.np);
    P->x = c.take<double>(S.np);
    P->done = c.take<unsigned>(1);
  };
  std::vector<std::pair<void*, const void*>> cp;
  std::vector<size_t> sz;
  Carver c(nullptr);
  plan(c, cp, sz);
  rc = check_hip(hipMalloc(&P->mem, c.used), "hipMalloc(tile-sparse Cholesky)");
  if (rc != DS3_OK) {
    delete P;
    return rc;
  }
  cp.clear();
  sz.clear();
  Carver d(P->mem);
  plan(d, cp, sz);
  for (size_t k = 0; k < cp.size() && rc == DS3_OK; ++k)
    if (sz[k]) rc = check_hip(hipMemcpy(cp[k].first, cp[k].second, sz[k], hipMemcpyHostToDevice),
                              "hipMemcpy(tile-sparse Cholesky tables)");
  if (rc != DS3_OK) {
    (void)hipFree(P->mem);
    delete P;
    return rc;
  }
  *out = P;
  return DS3_OK;
}

void tilechol_destroy(TileChol* P) {
  if (!P) return;
  if (P->mem) (void)hipFree(P->mem);
  delete P;
}

void tilechol_stats(const TileChol* P, int64_t* info) {
  const TcSymbolic& S = P->S;
  const int64_t v[7] = {S.n_kf, S.nt, S.nslot, S.nlev, S.nupd, S.np - S.n, S.thr};
  for (int k = 0; k < 7; ++k) info[k] = v[k];
}

int launch_tilechol(const TileChol* P, const double* H, const double* g, double lambda, double eps0,
                    double mult, int attempts, double* tau, int32_t* status, void* ws, hipStream_t s,
                    bool sync_cleared) {
  if (!P || !H || !g || !tau || !status || !ws) return fail(DS3_EINVAL, "tilechol: null pointer");
  if (attempts < 1 || attempts > kTcMaxAttempts) return fail(DS3_EINVAL, "tilechol: attempts out of range");
  const TcSymbolic& S = P->S;
  TcArgs a;
  a.H = H; a.g = g;
  a.n = S.n; a.n_kf = S.n_kf; a.np = S.np; a.nt = S.nt;
  a.lambda = lambda; a.eps0 = eps0; a.attempts = attempts;
  a.rowmap = P->rowmap; a.slot_row = P->slot_row; a.slot_col = P->slot_col; a.col_ptr = P->col_ptr;
  a.tlevel = P->tlevel; a.init_order = P->init_order; a.tgt = P->tgt; a.piv = P->piv; a.pat = P->pat;
  a.W = P->W; a.L = P->L; a.Inv = P->Inv; a.b = P->b; a.y = P->y; a.x = P->x;
  a.tau = tau; a.status = status;
  a.sync = chol_sync_words(ws, S.n);
  a.done = P->done;
  // the dense fallback's barrier words and the attempt-0 flag start at zero (a fill kernel, not a memset,
  // so the sequence can be captured)
  if (!sync_cleared) DS3_TRY(launch_fill_u32(a.sync, 4, 0u, s));
  hipLaunchKernelGGL(k_tc_init, dim3(unsigned(S.nslot)), dim3(kTcThreads), 0, s, a);
  DS3_TRY(check_hip(hipGetLastError(), "k_tc_init"));
  for (int l = 0; l + 1 < S.nlev; ++l) {
    const int t0 = S.lt_ptr[l], t1 = S.lt_ptr[l + 1];
    if (t1 <= t0) continue;
    hipLaunchKernelGGL(k_tc_level, dim3(t1 - t0), dim3(kTcThreads), 0, s, a, t0);
    DS3_TRY(check_hip(hipGetLastError(), "k_tc_level"));
  }
  hipLaunchKernelGGL(k_tc_backsub, dim3(S.nt), dim3(kTcThreads), 0, s, a);
  DS3_TRY(check_hip(hipGetLastError(), "k_tc_backsub"));
  if (attempts > 1)
    DS3_TRY(launch_chol_fallback(H, g, S.n, lambda, eps0, mult, attempts, tau, status, ws, s));
  return DS3_OK;
}

}  // namespace ds3

using namespace ds3;

extern "C" {

struct ds3_tilechol {
  TileChol* impl;
};

int ds3_tilechol_analyse(int32_t n_kf, int32_t n_pairs, const int32_t* pair_ij, int32_t* kf_row0,
                         int64_t* info) {
  if (!info) return fail(DS3_EINVAL, "tilechol: null info");
  TcSymbolic S;
  DS3_TRY(tc_symbolic(n_kf, n_pairs, pair_ij, S));
  if (kf_row0) std::memcpy(kf_row0, S.kf_row0.data(), sizeof(int32_t) * size_t(n_kf));
  const int64_t v[7] = {S.n_kf, S.nt, S.nslot, S.nlev, S.nupd, S.np - S.n, S.thr};
  for (int k = 0; k < 7; ++k) info[k] = v[k];
  return DS3_OK;
}

int ds3_tilechol_create(int32_t n_kf, int32_t n_pairs, const int32_t* pair_ij, ds3_tilechol** out) {
  if (!out) return fail(DS3_EINVAL, "tilechol: null output");
  *out = nullptr;
  TileChol* P = nullptr;
  DS3_TRY(tilechol_create(n_kf, n_pairs, pair_ij, &P));
  *out = new ds3_tilechol{P};
  return DS3_OK;
}

int ds3_tilechol_info(const ds3_tilechol* S, int64_t* info) {
  if (!S || !info) return fail(DS3_EINVAL, "tilechol: null pointer");
  tilechol_stats(S->impl, info);
  return DS3_OK;
}

int ds3_tilechol_solve(ds3_tilechol* S, const double* H, const double* g, double lambda, double eps0,
                       double mult, int32_t attempts, double* tau, int32_t* status, void* workspace,
                       size_t workspace_bytes, void* stream) {
  if (!S) return fail(DS3_EINVAL, "tilechol: null plan");
  if (workspace_bytes < chol_workspace_bytes(S->impl->S.n))
    return fail(DS3_ENOSPACE, "tilechol: workspace smaller than ds3_chol_workspace_bytes(7 n_kf)");
  return launch_tilechol(S->impl, H, g, lambda, eps0, mult, attempts, tau, status, workspace,
                         static_cast<hipStream_t>(stream));
}

void ds3_tilechol_destroy(ds3_tilechol* S) {
  if (!S) return;
  tilechol_destroy(S->impl);
  delete S;
}

}  // extern "C"
