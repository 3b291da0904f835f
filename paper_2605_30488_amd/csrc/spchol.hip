// Block-sparse solve of the regularised normal equations of eq. (7) with the epsilon ladder of the text
// after it, for the fixed block pattern of a pose graph:
//   (H + lambda diag H + eps_r I) tau = -g,  eps_r = eps0 * mult^r,  r = 0 .. attempts-1,
// and a zero update (status -1) when every factorisation fails. H couples keyframes a and b only when an
// edge joins them, so it is a pattern of 7x7 blocks that stays fixed while Gauss-Newton moves the poses.
//
// Symbolic analysis (host, once per pattern): a minimum-degree elimination order of the keyframe graph,
// the filled pattern of the block Cholesky factor L (the cliques that elimination leaves), its
// elimination tree, and an order of the columns by tree level (leaves first), which is a topological
// order of the tree and therefore has exactly the same fill. For every block (x, k) of L the list of
// products L_xj L_kj^T that left-looking elimination subtracts from it (j runs over the descendants of
// k whose columns hold both rows), in increasing j.
//
// Numeric solve: a gather kernel over the device copies attempt 0's blocks of H and -g into the factor's
// storage; then one workgroup does the rest in one launch. Level by level, every block of the level's
// columns is A_xk minus its products (float64 matrix-core products, one wave per block, the operand loads
// of a batch of products issued together); the wave of a diagonal block carries the right-hand side as an
// extra row of its products, then factors the block (Cholesky of the 7x7 block and the inverse of its
// factor, carried out redundantly in every lane) and forms y_k; then every off-diagonal block is
// multiplied by the inverse of its column's diagonal factor. Columns of one level never depend on each
// other, so a level needs two workgroup barriers. A non-positive or non-finite pivot fails the attempt,
// and the next attempt starts over from H (read again inside the workgroup) with the next eps. The back
// substitution runs the levels in reverse with the solution blocks in LDS. No step waits on another
// workgroup, so nothing can hang.
//
// The index tables and the solution blocks live in LDS for the whole launch; patterns whose tables do not
// fit are refused at creation (the dense solver takes any pattern). One compute unit's load pipeline bounds
// the solve (every product is four 64-lane operand loads), which is why the plans use it only when asked
// (the tile-sparse solver is faster on the pose graphs measured here).
#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace ds3 {

constexpr int kSpThreads = 768;  // 12 waves: 168 VGPRs each, enough for a batch of products without spills
constexpr int kSpWaves = kSpThreads / kWave;
constexpr int kSpMaxAttempts = 16;
constexpr int kSpLdsWords = 28 * 1024;  // int32 words of index tables held in LDS (112 KiB)
constexpr int kSpMaxCols = 512;         // keyframes whose solution blocks the back substitution keeps in LDS
constexpr int kSpMaxKf = 8192 / 7;      // the order limit of the dense solver, in keyframes
constexpr int32_t kOrigBit = 1 << 30;   // block-column word: the block is in the pattern of H

// Host result of the symbolic analysis.
struct SpSymbolic {
  int n_kf = 0, nlev = 0;
  int64_t nblk = 0, nfill = 0, npair = 0, nyup = 0;
  std::vector<int32_t> perm;     // column -> keyframe
  std::vector<int32_t> level;    // keyframe -> elimination-tree level
  std::vector<int32_t> lev_ptr;  // nlev + 1: columns of level l are [lev_ptr[l], lev_ptr[l + 1])
  std::vector<int32_t> blk_ptr;  // n_kf + 1: blocks of column c, the diagonal block first
  std::vector<int32_t> blk_row;  // row (column index) of each block
  std::vector<int32_t> blk_col;  // column of each block, | kOrigBit when it is in the pattern of H
  std::vector<int32_t> upd_ptr;  // nblk + 1
  std::vector<int32_t> upd_src;  // 2 per product: block of L_xj, block of L_kj
  std::vector<int32_t> yup_ptr;  // n_kf + 1
  std::vector<int32_t> yup_src;  // 2 per term of the forward elimination of column k: block of L_kj, j
  // word offsets of the tables in the packed image (the order the kernel copies into LDS)
  int o_perm = 0, o_lev = 0, o_bptr = 0, o_brow = 0, o_bcol = 0, o_uptr = 0, o_usrc = 0, o_yptr = 0,
      o_ysrc = 0, words = 0;
  std::vector<int32_t> image;
};

static int popcount_row(const uint64_t* r, int W) {
  int s = 0;
  for (int w = 0; w < W; ++w) s += __builtin_popcountll(r[w]);
  return s;
}

// Minimum-degree elimination order of the keyframe graph given by the pairs (a, b), a != b (repeated pairs
// allowed), on the exact elimination graph with ties to the lowest keyframe id. rows[v]: the neighbours of
// v when it is eliminated, i.e. the rows of its column in the filled factor. pattern (optional): the
// adjacency bitset of the pairs themselves, ceil(n / 64) words per keyframe.
int min_degree_order(int n, int n_pairs, const int32_t* pair_ij, std::vector<int>& order,
                     std::vector<std::vector<int>>& rows, std::vector<uint64_t>* pattern) {
  if (n_pairs < 0 || (n_pairs > 0 && !pair_ij)) return fail(DS3_EINVAL, "min_degree: bad pair table");
  const int W = (n + 63) / 64;
  std::vector<uint64_t> adj(size_t(n) * W, 0);
  for (int p = 0; p < n_pairs; ++p) {
    const int a = pair_ij[2 * p], b = pair_ij[2 * p + 1];
    if (a < 0 || b < 0 || a >= n || b >= n || a == b)
      return fail(DS3_EINVAL, "pair " + std::to_string(p) + " out of range or on the diagonal");
    adj[size_t(a) * W + b / 64] |= 1ull << (b % 64);
    adj[size_t(b) * W + a / 64] |= 1ull << (a % 64);
  }
  if (pattern) *pattern = adj;
  std::vector<int> deg(n);
  order.clear();
  order.reserve(n);
  rows.assign(n, {});
  for (int v = 0; v < n; ++v) deg[v] = popcount_row(&adj[size_t(v) * W], W);
  std::vector<uint8_t> alive(n, 1);
  for (int step = 0; step < n; ++step) {
    int v = -1;
    for (int u = 0; u < n; ++u)
      if (alive[u] && (v < 0 || deg[u] < deg[v])) v = u;
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
    for (int a : nb) deg[a] = popcount_row(&adj[size_t(a) * W], W);
    alive[v] = 0;
    order.push_back(v);
  }
  return DS3_OK;
}

// Symbolic analysis of the block pattern given by the keyframe pairs (a, b), a != b; repeated pairs are
// allowed. Returns DS3_EINVAL for bad arguments.
static int spchol_symbolic(int n_kf, int n_pairs, const int32_t* pair_ij, SpSymbolic& S) {
  if (n_kf < 1 || n_kf > kSpMaxKf) return fail(DS3_EINVAL, "spchol: n_kf must be in 1 .. 1170");
  if (n_pairs < 0 || (n_pairs > 0 && !pair_ij)) return fail(DS3_EINVAL, "spchol: bad pair table");
  const int n = n_kf, W = (n + 63) / 64;
  std::vector<uint64_t> in_pattern;
  std::vector<int> order, pos(n, -1);
  std::vector<std::vector<int>> rows;
  DS3_TRY(min_degree_order(n, n_pairs, pair_ij, order, rows, &in_pattern));
  for (int k = 0; k < n; ++k) pos[order[k]] = k;
  // elimination tree (parent = earliest-eliminated row) and levels from the leaves
  S.level.assign(n, 0);
  for (int v : order) {
    int parent = -1;
    for (int u : rows[v])
      if (parent < 0 || pos[u] < pos[parent]) parent = u;
    if (parent >= 0) S.level[parent] = std::max(S.level[parent], S.level[v] + 1);
  }
  S.perm = order;
  std::stable_sort(S.perm.begin(), S.perm.end(), [&](int a, int b) { return S.level[a] < S.level[b]; });
  std::vector<int> col(n);
  for (int c = 0; c < n; ++c) col[S.perm[c]] = c;
  S.n_kf = n;
  S.nlev = S.level[S.perm[n - 1]] + 1;
  S.lev_ptr.assign(S.nlev + 1, 0);
  for (int c = 0; c < n; ++c) S.lev_ptr[S.level[S.perm[c]] + 1] = c + 1;
  for (int l = 1; l <= S.nlev; ++l) S.lev_ptr[l] = std::max(S.lev_ptr[l], S.lev_ptr[l - 1]);
  // blocks, column by column: the diagonal, then the rows in increasing column index
  S.blk_ptr.assign(n + 1, 0);
  S.blk_row.clear();
  S.blk_col.clear();
  S.nfill = 0;
  for (int c = 0; c < n; ++c) {
    const int v = S.perm[c];
    std::vector<int> r;
    for (int u : rows[v]) r.push_back(col[u]);
    std::sort(r.begin(), r.end());
    S.blk_row.push_back(c);
    S.blk_col.push_back(c | kOrigBit);
    for (int x : r) {
      if (x <= c) return fail(DS3_EINVAL, "spchol: internal error (row above the diagonal)");
      const int px = S.perm[x];
      const bool orig = (in_pattern[size_t(v) * W + px / 64] >> (px % 64)) & 1ull;
      S.blk_row.push_back(x);
      S.blk_col.push_back(c | (orig ? kOrigBit : 0));
      if (!orig) ++S.nfill;
    }
    S.blk_ptr[c + 1] = int(S.blk_row.size());
  }
  S.nblk = int64_t(S.blk_row.size());
  auto find_blk = [&](int x, int j) -> int {  // block (x, j) of L, -1 if structurally zero
    const auto b = S.blk_row.begin() + S.blk_ptr[j], e = S.blk_row.begin() + S.blk_ptr[j + 1];
    const auto it = std::lower_bound(b, e, x);
    return (it != e && *it == x) ? int(it - S.blk_row.begin()) : -1;
  };
  // descendants contributing to each column, in increasing order
  std::vector<std::vector<int>> contrib(n);
  for (int j = 0; j < n; ++j)
    for (int b = S.blk_ptr[j] + 1; b < S.blk_ptr[j + 1]; ++b) contrib[S.blk_row[b]].push_back(j);
  S.upd_ptr.assign(S.nblk + 1, 0);
  S.upd_src.clear();
  S.yup_ptr.assign(n + 1, 0);
  S.yup_src.clear();
  for (int k = 0; k < n; ++k) {
    for (int b = S.blk_ptr[k]; b < S.blk_ptr[k + 1]; ++b) {
      const int x = S.blk_row[b];
      if (x == k) {  // the diagonal block's products come from the right-hand side list below
        S.upd_ptr[b + 1] = int(S.upd_src.size() / 2);
        continue;
      }
      for (int j : contrib[k]) {
        const int bkj = find_blk(k, j);
        const int bxj = find_blk(x, j);
        if (bkj < 0) return fail(DS3_EINVAL, "spchol: internal error (missing contribution)");
        if (bxj >= 0) {
          S.upd_src.push_back(bxj);
          S.upd_src.push_back(bkj);
        }
      }
      S.upd_ptr[b + 1] = int(S.upd_src.size() / 2);
    }
    // every row of a contributing column below k must be a row of k (the elimination graph's cliques)
    for (int j : contrib[k])
      for (int b = S.blk_ptr[j] + 1; b < S.blk_ptr[j + 1]; ++b)
        if (S.blk_row[b] > k && find_blk(S.blk_row[b], k) < 0)
          return fail(DS3_EINVAL, "spchol: internal error (fill outside the factor pattern)");
    for (int j : contrib[k]) {
      S.yup_src.push_back(find_blk(k, j));
      S.yup_src.push_back(j);
    }
    S.yup_ptr[k + 1] = int(S.yup_src.size() / 2);
  }
  S.npair = int64_t(S.upd_src.size() / 2);
  S.nyup = int64_t(S.yup_src.size() / 2);
  // packed image of the tables
  S.image.clear();
  auto put = [&](const std::vector<int32_t>& v) {
    const int off = int(S.image.size());
    S.image.insert(S.image.end(), v.begin(), v.end());
    return off;
  };
  S.o_perm = put(S.perm);
  S.o_lev = put(S.lev_ptr);
  S.o_bptr = put(S.blk_ptr);
  S.o_brow = put(S.blk_row);
  S.o_bcol = put(S.blk_col);
  S.o_uptr = put(S.upd_ptr);
  S.o_usrc = put(S.upd_src);
  S.o_yptr = put(S.yup_ptr);
  S.o_ysrc = put(S.yup_src);
  S.words = int(S.image.size());
  return DS3_OK;
}

// ---------------------------------------------------------------------------------------------------
// Device side
// ---------------------------------------------------------------------------------------------------
constexpr int kSpInvSlots = 16;  // inverses of the diagonal factors of a level's first columns, in LDS

struct SpArgs {
  const int32_t* image;
  int words;
  int o_perm, o_lev, o_bptr, o_brow, o_bcol, o_uptr, o_usrc, o_yptr, o_ysrc;
  int n_kf, nlev;
  const double* H;
  const double* g;
  double lambda, eps0, mult;
  int attempts;
  double* L;    // 49 per block: the regularised block of H, then the factor's block (row-major)
  double* Inv;  // 49 per column: inverse of the diagonal factor, row-major
  double* y;    // 8 per column: -g, then L^-1 (-g)
  double* tau;
  int32_t* status;
};

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ inline double sp_rsqrt(double d) {  // hardware estimate refined by two Newton steps
  double r = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}

__device__ inline double rdlane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffff), lane);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// The float64 matrix-core product (16x16x4, two of them for an inner dimension of 7) as used here: lane
// i + 16 kq (i < 16, kq < 4) feeds P[i][kq] and P[i][kq + 4] of the left factor and Q[kq][i], Q[kq + 4][i]
// of the right one; register v of lane c + 16 kq receives row kq + 4 v, column c of the result. A
// result's registers 0 and 1 are therefore, as they are, the right operand of a product whose inner
// index runs over the result's rows.
__device__ inline f64x4 mma2(double p0, double p1, double q0, double q1, f64x4 acc) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(p0, q0, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f64_16x16x4f64(p1, q1, acc, 0, 0, 0);
}

// Operands of one product acc[m][n] -= sum_q X[m][q] Z[n][q] for 7x7 row-major blocks X, Z (with r7
// non-null, row 7 of the left factor is r7, so row 7 of acc takes -Z r7). The loads are branch-free
// (clamped addresses, then selects) so that the loads of a batch of products issue back to back.
struct Ops {
  double a0, a1, b0, b1;
};

// Raw loads of one product's operands (clamped addresses, nothing selected yet), so that the loads of a
// batch issue back to back; mask_ops then zeroes what lies outside the blocks.
__device__ inline Ops load_ops(const double* X, const double* Z, const double* r7, int i, int kq) {
  const bool row7 = (r7 != nullptr) && i == 7;
  const int ii = (i < 7) ? i : 0, q1 = (kq < 3) ? kq + 4 : kq;
  const double* px = row7 ? r7 : X + 7 * ii;
  Ops o;
  o.a0 = px[kq];
  o.a1 = px[q1];
  o.b0 = Z[7 * ii + kq];
  o.b1 = Z[7 * ii + q1];
  return o;
}

__device__ inline Ops mask_ops(Ops o, bool diag, int i, int kq) {
  const bool in = i < 7, left = in || (diag && i == 7);
  o.a0 = left ? o.a0 : 0.0;
  o.a1 = (left && kq < 3) ? o.a1 : 0.0;
  o.b0 = in ? o.b0 : 0.0;
  o.b1 = (in && kq < 3) ? o.b1 : 0.0;
  return o;
}

constexpr int kSpBatch = 6;  // products whose loads are in flight together

// Lower-triangle read of the symmetric H at (row a, column b).
__device__ inline double h_lower(const double* H, int64_t n, int64_t a, int64_t b) {
  return (a >= b) ? H[a * n + b] : H[b * n + a];
}

// Element t of the factor storage at the start of an attempt: the block's entry of H (lower triangle read;
// zero for fill blocks), plus lambda times itself and eps on the diagonal. tab: the index tables (LDS or
// global copy).
__device__ inline double sp_init_value(const SpArgs& a, const int32_t* tab, int64_t t, double eps) {
  const int64_t n = 7 * int64_t(a.n_kf);
  const int b = int(t / 49), e = int(t - 49 * int64_t(b)), r = e / 7, c = e - 7 * r;
  const int cw = tab[a.o_bcol + b], k = cw & (kOrigBit - 1), xr = tab[a.o_brow + b];
  if (!(cw & kOrigBit)) return 0.0;
  const int64_t ra = 7 * int64_t(tab[a.o_perm + xr]) + r, cb = 7 * int64_t(tab[a.o_perm + k]) + c;
  double v = (ra >= cb) ? a.H[ra * n + cb] : a.H[cb * n + ra];
  if (xr == k && r == c) v += a.lambda * v + eps;
  return v;
}

// Right-hand side slot t (column t / 8, entry t % 8; entry 7 is padding).
__device__ inline double sp_init_rhs(const SpArgs& a, const int32_t* tab, int t) {
  const int k = t >> 3, r = t & 7;
  return (r < 7) ? -a.g[7 * int64_t(tab[a.o_perm + k]) + r] : 0.0;
}

// The factor storage and the right-hand side for attempt 0, over the whole device.
__global__ __launch_bounds__(256) void k_spchol_gather(SpArgs a, int64_t nblk) {
  const int64_t total = 49 * nblk, stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total + 8 * a.n_kf; t += stride) {
    if (t < total)
      a.L[t] = sp_init_value(a, a.image, t, a.eps0);
    else
      a.y[t - total] = sp_init_rhs(a, a.image, int(t - total));
  }
}

// The same inside the solve's workgroup, for the ladder's later attempts.
__device__ void sp_prologue(const SpArgs& a, const int32_t* sm, int64_t nblk, double eps) {
  for (int64_t t = threadIdx.x; t < 49 * nblk; t += kSpThreads) a.L[t] = sp_init_value(a, sm, t, eps);
  for (int t = threadIdx.x; t < 8 * a.n_kf; t += kSpThreads) a.y[t] = sp_init_rhs(a, sm, t);
}

// Reads the factor storage and the right-hand side once (16 B per load, eight loads in flight per thread)
// so that the levels find them in this workgroup's L2. Returns a value that is never a particular bit
// pattern in practice; the caller consumes it so that the loads stay.
__device__ double sp_warm(const SpArgs& a, int64_t nblk) {
  const double2* L2v = reinterpret_cast<const double2*>(a.L);
  const int64_t nl = (49 * nblk) / 2;  // 49 * nblk doubles; the odd last one is read with the rhs below
  double s = 0.0;
  for (int64_t base = threadIdx.x; base < nl; base += 8 * int64_t(kSpThreads)) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t q = base + int64_t(u) * kSpThreads;
      v[u] = L2v[(q < nl) ? q : base];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u].x + v[u].y;
  }
  for (int t = threadIdx.x; t < 8 * a.n_kf; t += kSpThreads) s += a.y[t];
  return s;
}

// Block (x, k) of L before its scaling, transposed: (A_xk - sum_j L_xj L_kj^T)^T. The diagonal block's wave
// carries the right-hand side as row 7 (b_k - sum_j L_kj y_j), then factors the block, forms the inverse
// of the factor and y_k, and publishes the inverse (global, and LDS slot k - c0 when there is one). An
// off-diagonal block goes to `keep` when it is the wave's first of the level, else to the factor storage.
// Returns false (uniformly) when a pivot is not positive and finite.
__device__ inline int sp_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Products of one block: a batch of kSpBatch products at a time with all their loads issued first, summed
// into four independent accumulators. DIAG: the pairs are (block of L_kj, j) and row 7 carries L_kj y_j;
// else (block of L_xj, block of L_kj) and the products are L_kj L_xj^T.
template <bool DIAG>
__device__ inline void sp_products(const SpArgs& a, const int32_t* lst, int p0, int p1, int i, int kq,
                                   f64x4 (&acc)[4]) {
  for (int p = p0; p < p1; p += kSpBatch) {
    // the batch's index pairs first (LDS reads back to back), then every operand load, then the products;
    // past the end of the list a product repeats the last pair with its operands zeroed (no branches, so
    // that no load is sunk behind one)
    int2 ev[kSpBatch];
#pragma unroll
    for (int u = 0; u < kSpBatch; ++u) ev[u] = *reinterpret_cast<const int2*>(lst + 2 * min(p + u, p1 - 1));
    __builtin_amdgcn_sched_barrier(0);
    Ops o[kSpBatch];
#pragma unroll
    for (int u = 0; u < kSpBatch; ++u) {
      const int e0 = sp_uniform(ev[u].x), e1 = sp_uniform(ev[u].y);
      if (DIAG) {
        const double* Lb = a.L + 49 * int64_t(e0);
        o[u] = load_ops(Lb, Lb, a.y + 8 * int64_t(e1), i, kq);
      } else {
        o[u] = load_ops(a.L + 49 * int64_t(e1), a.L + 49 * int64_t(e0), nullptr, i, kq);
      }
    }
    __builtin_amdgcn_sched_barrier(0);  // every load of the batch is issued before the first product waits
#pragma unroll
    for (int u = 0; u < kSpBatch; ++u) {
      const Ops m = mask_ops(o[u], DIAG, i, kq);
      const double w = (p + u < p1) ? -1.0 : 0.0;
      acc[u & 3] = mma2(w * m.a0, w * m.a1, m.b0, m.b1, acc[u & 3]);
    }
  }
}

__device__ bool sp_target(const SpArgs& a, const int32_t* sm, double* s_inv, int tb, int c0, bool first,
                          f64x4& keep) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
  const int k = sp_uniform(sm[a.o_bcol + tb] & (kOrigBit - 1));
  const bool diag = sp_uniform(sm[a.o_brow + tb]) == k;
  const double* init = a.L + 49 * int64_t(tb);
  f64x4 part[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) part[u] = f64x4{0.0, 0.0, 0.0, 0.0};
  {
    const int ii = (i < 7) ? i : 0, q1 = (kq < 3) ? kq + 4 : kq;
    const double v0 = init[7 * ii + kq], v1 = init[7 * ii + q1], yk = a.y[8 * int64_t(k) + ii];
    part[0][0] = (i < 7) ? v0 : 0.0;
    part[0][1] = (i < 7) ? ((kq < 3) ? v1 : (diag ? yk : 0.0)) : 0.0;
  }
  // diagonal block: products L_kj L_kj^T with L_kj y_j in row 7, over the descendants j of k; off-diagonal
  // block: products L_kj L_xj^T (the transposed contributions)
  if (diag)
    sp_products<true>(a, sm + a.o_ysrc, sp_uniform(sm[a.o_yptr + k]), sp_uniform(sm[a.o_yptr + k + 1]), i, kq,
                      part);
  else
    sp_products<false>(a, sm + a.o_usrc, sp_uniform(sm[a.o_uptr + tb]), sp_uniform(sm[a.o_uptr + tb + 1]), i,
                       kq, part);
  const f64x4 acc01 = (part[0] + part[1]) + (part[2] + part[3]);
  const f64x4 acc = acc01;
  if (!diag) {
    if (first) {
      keep = acc;
    } else if (i < 7) {
      double* dst = a.L + 49 * int64_t(tb);
      dst[7 * kq + i] = acc[0];
      if (kq < 3) dst[7 * (kq + 4) + i] = acc[1];
    }
    return true;
  }
  // the block's lower triangle, uniform in every lane
  double A[7][7];
#pragma unroll
  for (int rr = 0; rr < 7; ++rr)
#pragma unroll
    for (int c = 0; c <= rr; ++c) A[rr][c] = rdlane(acc[rr >> 2], c + 16 * (rr & 3));
  // Cholesky of the block (left-looking inside it); the diagonal slot takes 1 / L_qq
  bool ok = true;
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    double d = A[q][q];
#pragma unroll
    for (int t = 0; t < q; ++t) d = fma(-A[q][t], A[q][t], d);
    ok = ok && (d > 0.0) && isfinite(d);
    A[q][q] = sp_rsqrt(d);
#pragma unroll
    for (int rr = q + 1; rr < 7; ++rr) {
      double s = A[rr][q];
#pragma unroll
      for (int t = 0; t < q; ++t) s = fma(-A[rr][t], A[q][t], s);
      A[rr][q] = s * A[q][q];
    }
  }
  // forward substitution L z = e_lane (lanes 0..6: column `lane` of the inverse) or L z = y' (lane 7; y'
  // is row 7 of the product, in register 1 of lanes 48..54)
  double z[7];
#pragma unroll
  for (int rr = 0; rr < 7; ++rr) {
    const double yr = rdlane(acc[1], rr + 48);
    double s = (lane < 7) ? ((lane == rr) ? 1.0 : 0.0) : yr;
#pragma unroll
    for (int t = 0; t < rr; ++t) s = fma(-A[rr][t], z[t], s);
    z[rr] = s * A[rr][rr];
  }
  const int slot = k - c0;
  if (lane < 7) {
    double* inv = a.Inv + 49 * int64_t(k);
#pragma unroll
    for (int rr = 0; rr < 7; ++rr) inv[7 * rr + lane] = z[rr];
    if (slot < kSpInvSlots)
#pragma unroll
      for (int rr = 0; rr < 7; ++rr) s_inv[49 * slot + 7 * rr + lane] = z[rr];
  } else if (lane == 7) {
#pragma unroll
    for (int rr = 0; rr < 7; ++rr) a.y[8 * int64_t(k) + rr] = z[rr];
  }
  return ok;
}

// L_xk = (A'_xk) Inv_k^T, formed as its transpose Inv_k (A'_xk)^T from the transposed block (kept in
// registers, or stored by sp_target) and written row-major.
__device__ void sp_scale(const SpArgs& a, const int32_t* sm, const double* s_inv, int tb, int c0, bool first,
                         const f64x4& keep) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
  const bool in = i < 7, in1 = in && kq < 3;
  const int k = sp_uniform(sm[a.o_bcol + tb] & (kOrigBit - 1));
  double* blk = a.L + 49 * int64_t(tb);
  const int slot = k - c0;
  double p0, p1;
  if (slot < kSpInvSlots) {
    const double* M = s_inv + 49 * slot;
    p0 = in ? M[7 * i + kq] : 0.0;
    p1 = in1 ? M[7 * i + kq + 4] : 0.0;
  } else {
    const double* M = a.Inv + 49 * int64_t(k);
    p0 = in ? M[7 * i + kq] : 0.0;
    p1 = in1 ? M[7 * i + kq + 4] : 0.0;
  }
  double q0, q1;
  if (first) {
    q0 = keep[0];
    q1 = keep[1];
  } else {
    q0 = in ? blk[7 * kq + i] : 0.0;
    q1 = in1 ? blk[7 * (kq + 4) + i] : 0.0;
  }
  const f64x4 C = mma2(p0, p1, q0, q1, f64x4{0.0, 0.0, 0.0, 0.0});
  if (in) {
    blk[7 * i + kq] = C[0];
    if (kq < 3) blk[7 * i + kq + 4] = C[1];
  }
}

// Back substitution of column c: x_c = Inv_c^T (y_c - sum_x L_xc^T x_x), the solution blocks x in LDS (sx).
// Lane (column r of the blocks, slot grp) sums over the column's off-diagonal blocks grp, grp + 8, ....
__device__ void sp_backsolve(const SpArgs& a, const int32_t* sm, double* sx, int c) {
  const int lane = threadIdx.x & 63, r = lane & 7, grp = lane >> 3, rc = (r < 7) ? r : 0;
  const double yc = a.y[8 * int64_t(c) + rc];
  const double* inv = a.Inv + 49 * int64_t(c) + ((lane < 7) ? lane : 0);
  double m[7];
#pragma unroll
  for (int t = 0; t < 7; ++t) m[t] = inv[7 * t];
  double acc = 0.0;
  const int bb = sp_uniform(sm[a.o_bptr + c]) + 1, b1 = sp_uniform(sm[a.o_bptr + c + 1]);
  for (int b = bb + grp; b < b1; b += 8) {
    const double* Lb = a.L + 49 * int64_t(b) + rc;
    const double* xx = sx + 8 * sm[a.o_brow + b];
    double lv[7];
#pragma unroll
    for (int t = 0; t < 7; ++t) lv[t] = Lb[7 * t];
#pragma unroll
    for (int t = 0; t < 7; ++t) acc = fma(lv[t], xx[t], acc);
  }
  acc += __shfl_xor(acc, 8, kWave);
  acc += __shfl_xor(acc, 16, kWave);
  acc += __shfl_xor(acc, 32, kWave);
  const double s = (r < 7) ? yc - acc : 0.0;
  double sv[7];
#pragma unroll
  for (int t = 0; t < 7; ++t) sv[t] = rdlane(s, t);
  if (lane < 7) {
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < 7; ++t) v = fma(m[t], sv[t], v);  // entries above the diagonal are zero
    sx[8 * c + lane] = v;
    a.tau[7 * int64_t(sm[a.o_perm + c]) + lane] = v;
  }
}

__global__ __launch_bounds__(kSpThreads) void k_spchol(SpArgs a) {
  __shared__ int32_t sm[kSpLdsWords];
  __shared__ double s_inv[kSpInvSlots * 49];
  __shared__ double s_x[kSpMaxCols * 8];
  __shared__ int s_fail[kSpMaxAttempts];
  for (int t = threadIdx.x; t < a.words; t += kSpThreads) sm[t] = a.image[t];
  if (threadIdx.x < kSpMaxAttempts) s_fail[threadIdx.x] = 0;
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int32_t* lev = sm + a.o_lev;
  const int32_t* bptr = sm + a.o_bptr;
  const int64_t nblk = bptr[a.n_kf];
  int result = -1;
  double eps = a.eps0;
  for (int r = 0; r < a.attempts; ++r, eps *= a.mult) {
    if (r == 0) {  // k_spchol_gather wrote attempt 0's storage
      const double w = sp_warm(a, nblk);
      if (__double_as_longlong(w) == 0x7ff4dead0badf00dll) s_fail[kSpMaxAttempts - 1] = 0;
    } else {
      sp_prologue(a, sm, nblk, eps);
    }
    __syncthreads();
    bool failed = false;
    for (int l = 0; l < a.nlev; ++l) {
      const int c0 = lev[l], b0 = bptr[c0], b1 = bptr[lev[l + 1]];
      // this wave's blocks b0 + wave + kSpWaves m: a diagonal block first (its factorisation is on the
      // critical path), else the first block (m = 0) last, so that the one block kept in registers for the
      // scaling is not held across the others
      const int nm = (b1 - b0 - wave + kSpWaves - 1) / kSpWaves;
      const bool diag_first = nm > 0 && sm[a.o_brow + b0 + wave] == (sm[a.o_bcol + b0 + wave] & (kOrigBit - 1));
      f64x4 keep;
      for (int u = 0; u < nm; ++u) {
        const int m = diag_first ? u : nm - 1 - u;
        if (!sp_target(a, sm, s_inv, b0 + wave + kSpWaves * m, c0, m == 0, keep) && (threadIdx.x & 63) == 0)
          s_fail[r] = 1;
      }
      __syncthreads();
      if (s_fail[r]) {  // one slot per attempt: the flag read here was written before this barrier
        failed = true;
        break;
      }
      for (int tb = b0 + wave; tb < b1; tb += kSpWaves)
        if (sm[a.o_brow + tb] != (sm[a.o_bcol + tb] & (kOrigBit - 1)))
          sp_scale(a, sm, s_inv, tb, c0, tb == b0 + wave, keep);
      __syncthreads();
    }
    if (!failed) {
      result = r;
      break;
    }
  }
  if (result < 0) {
    for (int t = threadIdx.x; t < 7 * a.n_kf; t += kSpThreads) a.tau[t] = 0.0;
    if (threadIdx.x == 0) *a.status = -1;
    return;
  }
  // the solution blocks stay in LDS, so the levels are separated by LDS-only barriers (the stores of tau
  // need not complete before the next level)
  for (int l = a.nlev - 1; l >= 0; --l) {
    for (int c = lev[l] + wave; c < lev[l + 1]; c += kSpWaves) sp_backsolve(a, sm, s_x, c);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  }
  if (threadIdx.x == 0) *a.status = result;
}

// ---------------------------------------------------------------------------------------------------
// Host objects
// ---------------------------------------------------------------------------------------------------
struct SpChol {
  SpSymbolic S;
  void* mem = nullptr;
  int32_t* image = nullptr;
  double *L = nullptr, *Inv = nullptr, *y = nullptr;
};

int spchol_create(int n_kf, int n_pairs, const int32_t* pair_ij, SpChol** out) {
  *out = nullptr;
  SpChol* P = new SpChol();
  int rc = spchol_symbolic(n_kf, n_pairs, pair_ij, P->S);
  if (rc == DS3_OK && n_kf > kSpMaxCols)
    rc = fail(DS3_ENOSPACE, "spchol: more than " + std::to_string(kSpMaxCols) + " keyframes");
  if (rc == DS3_OK && P->S.words > kSpLdsWords)
    rc = fail(DS3_ENOSPACE, "spchol: the factor's index tables (" + std::to_string(P->S.words) +
                                " words) exceed the " + std::to_string(kSpLdsWords) + "-word LDS budget");
  if (rc == DS3_OK && (P->S.nblk > (int64_t(1) << 29) / 49))
    rc = fail(DS3_ENOSPACE, "spchol: factor too large");
  if (rc != DS3_OK) {
    delete P;
    return rc;
  }
  Carver c(nullptr);
  c.take<int32_t>(P->S.words);
  c.take<double>(49 * size_t(P->S.nblk));
  c.take<double>(49 * size_t(n_kf));
  c.take<double>(8 * size_t(n_kf));
  rc = check_hip(hipMalloc(&P->mem, c.used), "hipMalloc(sparse Cholesky)");
  if (rc != DS3_OK) {
    delete P;
    return rc;
  }
  Carver d(P->mem);
  P->image = d.take<int32_t>(P->S.words);
  P->L = d.take<double>(49 * size_t(P->S.nblk));
  P->Inv = d.take<double>(49 * size_t(n_kf));
  P->y = d.take<double>(8 * size_t(n_kf));
  rc = check_hip(hipMemcpy(P->image, P->S.image.data(), sizeof(int32_t) * P->S.words, hipMemcpyHostToDevice),
                 "hipMemcpy(sparse Cholesky tables)");
  if (rc != DS3_OK) {
    (void)hipFree(P->mem);
    delete P;
    return rc;
  }
  *out = P;
  return DS3_OK;
}

void spchol_destroy(SpChol* P) {
  if (!P) return;
  if (P->mem) (void)hipFree(P->mem);
  delete P;
}

int launch_spchol(const SpChol* P, const double* H, const double* g, double lambda, double eps0, double mult,
                  int attempts, double* tau, int32_t* status, hipStream_t s) {
  if (!P || !H || !g || !tau || !status) return fail(DS3_EINVAL, "spchol: null pointer");
  if (attempts < 1 || attempts > kSpMaxAttempts) return fail(DS3_EINVAL, "spchol: attempts out of range");
  const SpSymbolic& S = P->S;
  SpArgs a;
  a.image = P->image;
  a.words = S.words;
  a.o_perm = S.o_perm; a.o_lev = S.o_lev; a.o_bptr = S.o_bptr; a.o_brow = S.o_brow; a.o_bcol = S.o_bcol;
  a.o_uptr = S.o_uptr; a.o_usrc = S.o_usrc; a.o_yptr = S.o_yptr; a.o_ysrc = S.o_ysrc;
  a.n_kf = S.n_kf;
  a.nlev = S.nlev;
  a.H = H; a.g = g;
  a.lambda = lambda; a.eps0 = eps0; a.mult = mult; a.attempts = attempts;
  a.L = P->L; a.Inv = P->Inv; a.y = P->y;
  a.tau = tau; a.status = status;
  const int64_t total = 49 * S.nblk + 8 * int64_t(S.n_kf);
  const int gb = int(std::min<int64_t>((total + 255) / 256, 4096));
  hipLaunchKernelGGL(k_spchol_gather, dim3(gb), dim3(256), 0, s, a, int64_t(S.nblk));
  DS3_TRY(check_hip(hipGetLastError(), "k_spchol_gather"));
  hipLaunchKernelGGL(k_spchol, dim3(1), dim3(kSpThreads), 0, s, a);
  return check_hip(hipGetLastError(), "k_spchol");
}

void spchol_stats(const SpChol* P, int64_t* info) {
  const SpSymbolic& S = P->S;
  info[0] = S.n_kf;
  info[1] = S.nblk;
  info[2] = S.nfill;
  info[3] = S.nlev;
  info[4] = S.npair + S.nyup;
  info[5] = S.words;
}

}  // namespace ds3

using namespace ds3;

extern "C" {

struct ds3_spchol {
  SpChol* impl;
};

int ds3_spchol_analyse(int32_t n_kf, int32_t n_pairs, const int32_t* pair_ij, int32_t* perm, int32_t* level,
                       int64_t* info) {
  if (!info) return fail(DS3_EINVAL, "spchol: null info");
  SpSymbolic S;
  DS3_TRY(spchol_symbolic(n_kf, n_pairs, pair_ij, S));
  if (perm) std::memcpy(perm, S.perm.data(), sizeof(int32_t) * size_t(n_kf));
  if (level) std::memcpy(level, S.level.data(), sizeof(int32_t) * size_t(n_kf));
  info[0] = S.n_kf;
  info[1] = S.nblk;
  info[2] = S.nfill;
  info[3] = S.nlev;
  info[4] = S.npair + S.nyup;
  info[5] = S.words;
  return DS3_OK;
}

int ds3_spchol_create(int32_t n_kf, int32_t n_pairs, const int32_t* pair_ij, ds3_spchol** out) {
  if (!out) return fail(DS3_EINVAL, "spchol: null output");
  *out = nullptr;
  SpChol* P = nullptr;
  DS3_TRY(spchol_create(n_kf, n_pairs, pair_ij, &P));
  *out = new ds3_spchol{P};
  return DS3_OK;
}

int ds3_spchol_info(const ds3_spchol* S, int64_t* info) {
  if (!S || !info) return fail(DS3_EINVAL, "spchol: null pointer");
  spchol_stats(S->impl, info);
  return DS3_OK;
}

int ds3_spchol_solve(ds3_spchol* S, const double* H, const double* g, double lambda, double eps0, double mult,
                     int32_t attempts, double* tau, int32_t* status, void* stream) {
  if (!S) return fail(DS3_EINVAL, "spchol: null plan");
  return launch_spchol(S->impl, H, g, lambda, eps0, mult, attempts, tau, status,
                       static_cast<hipStream_t>(stream));
}

void ds3_spchol_destroy(ds3_spchol* S) {
  if (!S) return;
  spchol_destroy(S->impl);
  delete S;
}

}  // extern "C"
