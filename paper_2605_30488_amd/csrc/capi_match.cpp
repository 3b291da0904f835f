// C ABI of the matching and gauge-synchronisation entry points (declared in include/ds3.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.hpp"
#include "match_internal.hpp"
#include "umeyama.hpp"

namespace ds3 {

size_t gauge_ws_bytes();
int launch_gauge_align(const void* Xi, int64_t npx_i, const void* Xj, int64_t npx_j, ds3_dtype dt,
                       const int32_t* idx, const uint8_t* valid, const double* poses, int i, int j,
                       int ref_is_i, int nc_min, double* T_out, int32_t* used, void* ws, hipStream_t s);
int launch_apply_gauge(double* poses, int n, const uint8_t* mask, const double* T, hipStream_t s);

static hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

static int check_match_params(const ds3_match_params* p) {
  if (!p) return fail(DS3_EINVAL, "null match params");
  if (p->max_iters < 0 || p->max_iters > 1000) return fail(DS3_EINVAL, "max_iters out of range");
  if (!(p->lambda0 > 0) || !(p->lambda_min > 0) || !(p->step_tol_px >= 0) || !(p->ang_tol_px >= 0) ||
      !(p->range_rel_tol >= 0) || p->mutual_radius_px < 0)
    return fail(DS3_EINVAL, "match params out of range");
  return DS3_OK;
}

static MatchConst make_match_const(const ds3_match_params& p) {
  MatchConst c;
  c.max_iters = p.max_iters;
  c.lambda0 = float(p.lambda0);
  c.lambda_min = float(p.lambda_min);
  c.step_tol = float(p.step_tol_px);
  c.ang_tol = float(p.ang_tol_px);
  c.range_tol = float(p.range_rel_tol);
  c.radius = p.mutual_radius_px;
  c.q_min = p.q_min;
  return c;
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

static int check_image(const ds3_image& im, bool ref) {
  if (im.H < (ref ? 2 : 1) || im.W < (ref ? 2 : 1) || im.px_offset < 0 ||
      int64_t(im.H) * im.W > INT32_MAX)
    return fail(DS3_EINVAL, ref ? "reference image must be at least 2x2" : "bad query image");
  return DS3_OK;
}

template <class T>
static int upload(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return DS3_OK;
  return check_hip(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s),
                   "hipMemcpyAsync(upload)");
}

// Deal entries with `tiles[k]` 256-px tiles into 8 bins (greedy, largest first) and lay the item map out:
// `order` lists the entries bin by bin; prefix/bin_start/bin_tiles as in ItemMap. Returns the grid size.
static int bin_items(const std::vector<int32_t>& tiles, std::vector<int32_t>& order,
                     std::vector<int32_t>& prefix, std::vector<int32_t>& bin_start,
                     std::vector<int32_t>& bin_tiles) {
  const int n = int(tiles.size());
  std::vector<int32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return tiles[a] > tiles[b]; });
  std::vector<std::vector<int32_t>> bins(8);
  std::vector<int64_t> load(8, 0);
  for (int k : idx) {
    int b = int(std::min_element(load.begin(), load.end()) - load.begin());
    bins[b].push_back(k);
    load[b] += tiles[k];
  }
  order.clear();
  prefix.clear();
  bin_start.assign(9, 0);
  bin_tiles.assign(8, 0);
  int max_tiles = 0;
  for (int b = 0; b < 8; ++b) {
    bin_start[b] = int32_t(order.size());
    int32_t acc = 0;
    for (int k : bins[b]) {
      order.push_back(k);
      prefix.push_back(acc);
      acc += tiles[k];
    }
    bin_tiles[b] = acc;
    max_tiles = std::max(max_tiles, int(acc));
  }
  bin_start[8] = int32_t(order.size());
  return 8 * max_tiles;
}

struct ItemMapBufs {
  int32_t *bin_start, *prefix, *bin_tiles;
};

static void carve_map(Carver& c, int n_entries, ItemMapBufs& m) {
  m.bin_start = c.take<int32_t>(9);
  m.prefix = c.take<int32_t>(std::max(n_entries, 1));
  m.bin_tiles = c.take<int32_t>(8);
}

static ItemMap as_map(const ItemMapBufs& m) { return ItemMap{m.bin_start, m.prefix, m.bin_tiles}; }

// Workspace of a batched match over `dirs` directions and `sides` mutual sides.
struct MatchWs {
  float4* rays;
  float* conf;
  int32_t* idx_tmp;
  MatchDir* dirs;
  MutualDir* md;
  ItemMapBufs map_m, map_u;
  unsigned* counts;
  int64_t* npx;
  unsigned* step_stripes;
  unsigned* part;   // per-tile mutual counts
  int64_t* side;    // per count slot: first partial, number of partials
};

static size_t carve_match(void* base, int64_t ray_px, int64_t tmp_idx, int n_dirs, int n_sides, int n_edges,
                          MatchWs& W) {
  Carver c(base);
  W.rays = c.take<float4>(size_t(std::max<int64_t>(ray_px, 1)));
  W.conf = c.take<float>(size_t(std::max<int64_t>(ray_px, 1)));
  W.idx_tmp = c.take<int32_t>(size_t(std::max<int64_t>(tmp_idx, 1)));
  W.dirs = c.take<MatchDir>(std::max(n_dirs, 1));
  W.md = c.take<MutualDir>(std::max(n_sides, 1));
  carve_map(c, n_dirs, W.map_m);
  carve_map(c, n_sides, W.map_u);
  W.counts = c.take<unsigned>(2 * size_t(std::max(n_edges, 1)));
  W.npx = c.take<int64_t>(2 * size_t(std::max(n_edges, 1)));
  W.step_stripes = c.take<unsigned>(size_t(kStepStripes) * kStripeStride);
  // every side has at most npx / 256 + 1 tiles and the sides' pixels add up to tmp_idx
  W.part = c.take<unsigned>(size_t(std::max<int64_t>(tmp_idx / 256 + n_sides + 1, 1)));
  W.side = c.take<int64_t>(2 * size_t(std::max(n_sides, 1)));
  return c.used;
}

// Per-tile partial slots of the sides (in their original order) and the per-slot table for the sums.
static void assign_parts(std::vector<MutualDir>& sides, const std::vector<int32_t>& stiles,
                         std::vector<int64_t>& side_tab) {
  side_tab.assign(2 * sides.size(), 0);
  int64_t off = 0;
  for (size_t k = 0; k < sides.size(); ++k) {
    sides[k].part_off = off;
    side_tab[2 * size_t(sides[k].count_slot)] = off;
    side_tab[2 * size_t(sides[k].count_slot) + 1] = stiles[k];
    off += stiles[k];
  }
}

// Shared driver: ray images, both directions of every edge, mutual check, nu.
struct EdgeSpec {
  const void* ref_i;  // canonical arena of i (pixel 0)
  const void* ref_j;
  int64_t ray_i, ray_j;   // pixel offsets of the two ray images in W.rays
  int64_t q_ji, q_ij;     // pixel offsets of the cross-view pointmaps in their arena
  int Hi, Wi, Hj, Wj;
  int64_t tmp_ji, tmp_ij;  // offsets in idx_tmp
  int64_t out_off;         // output offset (idx, valid)
};

static int run_match(const std::vector<EdgeSpec>& es, const void* cross, ds3_dtype dt, const MatchConst& C,
                     double nu_min, MatchWs& W, int32_t* idx_out, uint8_t* valid_out, float* nu,
                     int32_t* admit, uint64_t* lm_steps, ds3_timer* timer, hipStream_t s) {
  const int ne = int(es.size());
  std::vector<MatchDir> dirs;
  std::vector<int32_t> dtiles;
  std::vector<MutualDir> sides;
  std::vector<int32_t> stiles;
  std::vector<int64_t> npx;
  for (int e = 0; e < ne; ++e) {
    const EdgeSpec& E = es[e];
    MatchDir a{E.ray_i, E.q_ji, E.tmp_ji, E.Hi, E.Wi, E.Hj, E.Wj};   // queries: pixels of j
    MatchDir b{E.ray_j, E.q_ij, E.tmp_ij, E.Hj, E.Wj, E.Hi, E.Wi};   // queries: pixels of i
    dirs.push_back(a);
    dtiles.push_back(match_tiles(E.Hj, E.Wj));
    dirs.push_back(b);
    dtiles.push_back(match_tiles(E.Hi, E.Wi));
    MutualDir sj{E.tmp_ji, E.tmp_ij, E.out_off, W.conf + E.ray_j, W.conf + E.ray_i, E.Hj, E.Wj, E.Hi, E.Wi,
                 2 * e + 1, 1};
    MutualDir si{E.tmp_ij, E.tmp_ji, 0, W.conf + E.ray_i, W.conf + E.ray_j, E.Hi, E.Wi, E.Hj, E.Wj, 2 * e, 0};
    sides.push_back(sj);
    stiles.push_back(int32_t((int64_t(E.Hj) * E.Wj + kMutualPx - 1) / kMutualPx));
    sides.push_back(si);
    stiles.push_back(int32_t((int64_t(E.Hi) * E.Wi + kMutualPx - 1) / kMutualPx));
    npx.push_back(int64_t(E.Hi) * E.Wi);
    npx.push_back(int64_t(E.Hj) * E.Wj);
  }
  std::vector<int32_t> order, prefix, bs, bt;
  const int grid_m = bin_items(dtiles, order, prefix, bs, bt);
  std::vector<MatchDir> dirs_o;
  for (int k : order) dirs_o.push_back(dirs[k]);
  DS3_TRY(upload(W.dirs, dirs_o, s));
  DS3_TRY(upload(W.map_m.bin_start, bs, s));
  DS3_TRY(upload(W.map_m.prefix, prefix, s));
  DS3_TRY(upload(W.map_m.bin_tiles, bt, s));
  std::vector<int64_t> side_tab;
  assign_parts(sides, stiles, side_tab);
  DS3_TRY(upload(W.side, side_tab, s));
  std::vector<int32_t> order2, prefix2, bs2, bt2;
  const int grid_u = bin_items(stiles, order2, prefix2, bs2, bt2);
  std::vector<MutualDir> sides_o;
  for (int k : order2) sides_o.push_back(sides[k]);
  DS3_TRY(upload(W.md, sides_o, s));
  DS3_TRY(upload(W.map_u.bin_start, bs2, s));
  DS3_TRY(upload(W.map_u.prefix, prefix2, s));
  DS3_TRY(upload(W.map_u.bin_tiles, bt2, s));
  DS3_TRY(upload(W.npx, npx, s));
  unsigned* stripes = lm_steps ? W.step_stripes : nullptr;
  if (stripes) DS3_TRY(launch_fill_u32(stripes, size_t(kStepStripes) * kStripeStride, 0u, s));
  DS3_TRY(timer_record(timer, true, s));
  DS3_TRY(launch_match_batched(W.rays, cross, dt, W.dirs, as_map(W.map_m), grid_m, C, W.idx_tmp, stripes, s));
  DS3_TRY(timer_record(timer, false, s));
  if (stripes) DS3_TRY(launch_sum_stripes(stripes, reinterpret_cast<unsigned long long*>(lm_steps), s));
  DS3_TRY(launch_mutual(W.md, as_map(W.map_u), grid_u, dt, C, W.idx_tmp, idx_out, valid_out, W.part, s));
  DS3_TRY(launch_side_counts(W.part, W.side, 2 * ne, W.counts, s));
  return launch_nu_finalize(W.counts, W.npx, ne, nu_min, nu, admit, s);
}

static int check_arch_local() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(DS3_EHIP, "no HIP device");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(DS3_EHIP, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(DS3_ENOTSUP, std::string("libds3 is built for gfx950, device is ") + prop.gcnArchName);
  return DS3_OK;
}

}  // namespace ds3

using namespace ds3;

extern "C" {

size_t ds3_match_workspace_bytes(int32_t H_ref, int32_t W_ref) {
  if (H_ref <= 0 || W_ref <= 0) return 0;
  Carver c(nullptr);
  c.take<float4>(size_t(H_ref) * W_ref);
  return c.used;
}

int ds3_match(const void* ref_xyzc, ds3_image ref, const void* qry_xyzc, ds3_image qry, ds3_dtype dtype,
              const ds3_match_params* params, int32_t* idx_out, float* p_out, int32_t* iters_out,
              void* workspace, size_t ws_bytes, void* stream) {
  if (!ref_xyzc || !qry_xyzc || !idx_out || !workspace) return fail(DS3_EINVAL, "match: null pointer");
  if (dtype != DS3_F32 && dtype != DS3_BF16) return fail(DS3_ENOTSUP, "match: dtype");
  if (!aligned16(ref_xyzc) || !aligned16(qry_xyzc) || !aligned16(workspace))
    return fail(DS3_EINVAL, "match: arenas must be 16 B aligned");
  DS3_TRY(check_match_params(params));
  DS3_TRY(check_image(ref, true));
  DS3_TRY(check_image(qry, false));
  if (ws_bytes < ds3_match_workspace_bytes(ref.H, ref.W)) return fail(DS3_ENOSPACE, "match: workspace");
  DS3_TRY(check_arch_local());
  hipStream_t s = S(stream);
  const int pxb = dtype == DS3_F32 ? 16 : 8;
  const char* rp = static_cast<const char*>(ref_xyzc) + ref.px_offset * pxb;
  const char* qp = static_cast<const char*>(qry_xyzc) + qry.px_offset * pxb;
  float4* rays = static_cast<float4*>(workspace);
  DS3_TRY(launch_raymap(rp, int64_t(ref.H) * ref.W, dtype, rays, nullptr, s));
  return launch_match_one(rays, ref.H, ref.W, qp, qry.H, qry.W, dtype, make_match_const(*params), idx_out,
                          p_out, iters_out, s);
}

size_t ds3_match_bidir_workspace_bytes(int32_t H_i, int32_t W_i, int32_t H_j, int32_t W_j) {
  if (H_i <= 0 || W_i <= 0 || H_j <= 0 || W_j <= 0) return 0;
  MatchWs W;
  const int64_t ni = int64_t(H_i) * W_i, nj = int64_t(H_j) * W_j;
  return carve_match(nullptr, ni + nj, ni + nj, 2, 2, 1, W);
}

int ds3_match_bidir(const void* X_ii, const void* X_ji, const void* X_jj, const void* X_ij,
                    ds3_image img_i, ds3_image img_j, ds3_dtype dtype, const ds3_match_params* params,
                    int32_t* idx_j2i, uint8_t* valid_j, float* nu, int32_t* admit, void* workspace,
                    size_t ws_bytes, void* stream) {
  if (!X_ii || !X_ji || !X_jj || !X_ij || !idx_j2i || !valid_j || !workspace)
    return fail(DS3_EINVAL, "match_bidir: null pointer");
  if (dtype != DS3_F32 && dtype != DS3_BF16) return fail(DS3_ENOTSUP, "match_bidir: dtype");
  if (!aligned16(X_ii) || !aligned16(X_ji) || !aligned16(X_jj) || !aligned16(X_ij) || !aligned16(workspace))
    return fail(DS3_EINVAL, "match_bidir: arenas must be 16 B aligned");
  DS3_TRY(check_match_params(params));
  DS3_TRY(check_image(img_i, true));
  DS3_TRY(check_image(img_j, true));
  if (ws_bytes < ds3_match_bidir_workspace_bytes(img_i.H, img_i.W, img_j.H, img_j.W))
    return fail(DS3_ENOSPACE, "match_bidir: workspace");
  DS3_TRY(check_arch_local());
  hipStream_t s = S(stream);
  const int64_t ni = int64_t(img_i.H) * img_i.W, nj = int64_t(img_j.H) * img_j.W;
  MatchWs W;
  carve_match(workspace, ni + nj, ni + nj, 2, 2, 1, W);
  const int pxb = dtype == DS3_F32 ? 16 : 8;
  auto at = [&](const void* p, int64_t off) { return static_cast<const char*>(p) + off * pxb; };
  const void* ii = at(X_ii, img_i.px_offset);
  const void* jj = at(X_jj, img_j.px_offset);
  DS3_TRY(launch_raymap(ii, ni, dtype, W.rays, W.conf, s));
  DS3_TRY(launch_raymap(jj, nj, dtype, W.rays + ni, W.conf + ni, s));
  // the two cross-view maps live in different buffers: run the two directions as single launches and
  // reuse the batched mutual kernel over both sides
  const MatchConst C = make_match_const(*params);
  DS3_TRY(launch_match_one(W.rays, img_i.H, img_i.W, at(X_ji, img_j.px_offset), img_j.H, img_j.W, dtype, C,
                           W.idx_tmp, nullptr, nullptr, s));
  DS3_TRY(launch_match_one(W.rays + ni, img_j.H, img_j.W, at(X_ij, img_i.px_offset), img_i.H, img_i.W,
                           dtype, C, W.idx_tmp + nj, nullptr, nullptr, s));
  std::vector<MutualDir> sides = {
      MutualDir{0, nj, 0, W.conf + ni, W.conf, img_j.H, img_j.W, img_i.H, img_i.W, 1, 1},
      MutualDir{nj, 0, 0, W.conf, W.conf + ni, img_i.H, img_i.W, img_j.H, img_j.W, 0, 0}};
  std::vector<int32_t> stiles = {int32_t((nj + kMutualPx - 1) / kMutualPx), int32_t((ni + kMutualPx - 1) / kMutualPx)};
  std::vector<int64_t> side_tab;
  assign_parts(sides, stiles, side_tab);
  DS3_TRY(upload(W.side, side_tab, s));
  std::vector<int32_t> order, prefix, bs, bt;
  const int grid = bin_items(stiles, order, prefix, bs, bt);
  std::vector<MutualDir> sides_o;
  for (int k : order) sides_o.push_back(sides[k]);
  DS3_TRY(upload(W.md, sides_o, s));
  DS3_TRY(upload(W.map_u.bin_start, bs, s));
  DS3_TRY(upload(W.map_u.prefix, prefix, s));
  DS3_TRY(upload(W.map_u.bin_tiles, bt, s));
  std::vector<int64_t> npx = {ni, nj};
  DS3_TRY(upload(W.npx, npx, s));
  DS3_TRY(launch_mutual(W.md, as_map(W.map_u), grid, dtype, C, W.idx_tmp, idx_j2i, valid_j, W.part, s));
  DS3_TRY(launch_side_counts(W.part, W.side, 2, W.counts, s));
  return launch_nu_finalize(W.counts, W.npx, 1, params->nu_min, nu, admit, s);
}

size_t ds3_match_batch_workspace_bytes(int32_t n_kf, const ds3_image* kf, int32_t n_edges,
                                       const ds3_edge* edges) {
  if (n_kf <= 0 || !kf || n_edges < 0 || (n_edges > 0 && !edges)) return 0;
  int64_t ray_px = 0, tmp = 0;
  for (int k = 0; k < n_kf; ++k) ray_px = std::max(ray_px, kf[k].px_offset + int64_t(kf[k].H) * kf[k].W);
  for (int e = 0; e < n_edges; ++e) {
    if (edges[e].i < 0 || edges[e].i >= n_kf || edges[e].j < 0 || edges[e].j >= n_kf) return 0;
    tmp += int64_t(kf[edges[e].i].H) * kf[edges[e].i].W + int64_t(kf[edges[e].j].H) * kf[edges[e].j].W;
  }
  MatchWs W;
  return carve_match(nullptr, ray_px, tmp, 2 * n_edges, 2 * n_edges, n_edges, W);
}

int ds3_match_batch(const void* kf_arena, const ds3_image* kf, int32_t n_kf, const void* cross_arena,
                    const int64_t* cross_off, const ds3_edge* edges, int32_t n_edges, ds3_dtype dtype,
                    const ds3_match_params* params, int32_t* idx_arena, uint8_t* valid_arena, float* nu,
                    int32_t* admit, uint64_t* lm_steps, ds3_timer* match_timer, void* workspace,
                    size_t ws_bytes, void* stream) {
  if (!kf_arena || !kf || !cross_arena || !cross_off || !edges || !idx_arena || !valid_arena || !workspace)
    return fail(DS3_EINVAL, "match_batch: null pointer");
  if (n_kf <= 0 || n_edges <= 0) return fail(DS3_EINVAL, "match_batch: empty graph");
  if (dtype != DS3_F32 && dtype != DS3_BF16) return fail(DS3_ENOTSUP, "match_batch: dtype");
  if (!aligned16(kf_arena) || !aligned16(cross_arena) || !aligned16(workspace))
    return fail(DS3_EINVAL, "match_batch: arenas must be 16 B aligned");
  DS3_TRY(check_match_params(params));
  for (int k = 0; k < n_kf; ++k) DS3_TRY(check_image(kf[k], true));
  const size_t need = ds3_match_batch_workspace_bytes(n_kf, kf, n_edges, edges);
  if (need == 0) return fail(DS3_EINVAL, "match_batch: bad edge table");
  if (ws_bytes < need) return fail(DS3_ENOSPACE, "match_batch: workspace");
  DS3_TRY(check_arch_local());
  hipStream_t s = S(stream);
  int64_t ray_px = 0, tmp = 0;
  for (int k = 0; k < n_kf; ++k) ray_px = std::max(ray_px, kf[k].px_offset + int64_t(kf[k].H) * kf[k].W);
  std::vector<EdgeSpec> es(n_edges);
  const int pxb = dtype == DS3_F32 ? 16 : 8;
  for (int e = 0; e < n_edges; ++e) {
    const ds3_image &I = kf[edges[e].i], &J = kf[edges[e].j];
    if (cross_off[2 * e] < 0 || cross_off[2 * e + 1] < 0 || edges[e].idx_offset < 0)
      return fail(DS3_EINVAL, "match_batch: negative offset");
    EdgeSpec& E = es[e];
    E.ref_i = static_cast<const char*>(kf_arena) + I.px_offset * pxb;
    E.ref_j = static_cast<const char*>(kf_arena) + J.px_offset * pxb;
    E.ray_i = I.px_offset;
    E.ray_j = J.px_offset;
    E.q_ji = cross_off[2 * e];
    E.q_ij = cross_off[2 * e + 1];
    E.Hi = I.H; E.Wi = I.W; E.Hj = J.H; E.Wj = J.W;
    E.tmp_ji = tmp;
    tmp += int64_t(J.H) * J.W;
    E.tmp_ij = tmp;
    tmp += int64_t(I.H) * I.W;
    E.out_off = edges[e].idx_offset;
  }
  MatchWs W;
  carve_match(workspace, ray_px, tmp, 2 * n_edges, 2 * n_edges, n_edges, W);
  DS3_TRY(launch_raymap(kf_arena, ray_px, dtype, W.rays, W.conf, s));
  return run_match(es, cross_arena, dtype, make_match_const(*params), params->nu_min, W, idx_arena,
                   valid_arena, nu, admit, lm_steps, match_timer, s);
}

// ---- gauge -------------------------------------------------------------------------------------------
int ds3_umeyama(const double* x, const double* y, int64_t n, double* T_out) {
  if (!x || !y || !T_out || n < 1) return fail(DS3_EINVAL, "umeyama: null pointer or no correspondences");
  // two passes in float64, index order: centroids, then the centred cross-covariance and spread of y
  double xb[3] = {0, 0, 0}, yb[3] = {0, 0, 0};
  for (int64_t l = 0; l < n; ++l)
    for (int k = 0; k < 3; ++k) {
      xb[k] += x[3 * l + k];
      yb[k] += y[3 * l + k];
    }
  for (int k = 0; k < 3; ++k) {
    xb[k] /= double(n);
    yb[k] /= double(n);
  }
  double A[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, sy2 = 0.0;
  for (int64_t l = 0; l < n; ++l) {
    double xc[3], yc[3];
    for (int k = 0; k < 3; ++k) {
      xc[k] = x[3 * l + k] - xb[k];
      yc[k] = y[3 * l + k] - yb[k];
    }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) A[3 * r + c] += xc[r] * yc[c];
    sy2 += yc[0] * yc[0] + yc[1] * yc[1] + yc[2] * yc[2];
  }
  for (int e = 0; e < 9; ++e) A[e] /= double(n);
  sy2 /= double(n);
  for (int e = 0; e < 9 + 1; ++e)
    if (!std::isfinite(e < 9 ? A[e] : sy2)) return fail(DS3_EINVAL, "umeyama: non-finite correspondences");
  Sim3 T;
  if (!umeyama_solve(xb, yb, A, sy2, T))
    return fail(DS3_EDEGENERATE, "umeyama: degenerate correspondences (rank of the cross-covariance < 2)");
  sim3_store(T, T_out);
  return DS3_OK;
}

size_t ds3_gauge_workspace_bytes(int32_t n_kf) {
  Carver c(nullptr);
  c.take<char>(gauge_ws_bytes());
  c.take<double>(8);
  c.take<int32_t>(4);
  c.take<uint8_t>(size_t(std::max(n_kf, 1)));
  return c.used;
}

int ds3_gauge_align(const void* X_i, ds3_image img_i, const void* X_j, ds3_image img_j, ds3_dtype dtype,
                    const int32_t* idx_j2i, const uint8_t* valid_j, const double* poses, int32_t i,
                    int32_t j, int32_t ref_is_i, int32_t nc_min, double* T_out, int32_t* used_umeyama,
                    void* workspace, size_t ws_bytes, void* stream) {
  if (!X_i || !X_j || !idx_j2i || !valid_j || !poses || !T_out || !used_umeyama || !workspace)
    return fail(DS3_EINVAL, "gauge_align: null pointer");
  if (dtype != DS3_F32 && dtype != DS3_BF16) return fail(DS3_ENOTSUP, "gauge_align: dtype");
  if (i < 0 || j < 0 || i == j) return fail(DS3_EINVAL, "gauge_align: bad keyframe ids");
  if (ws_bytes < gauge_ws_bytes()) return fail(DS3_ENOSPACE, "gauge_align: workspace");
  DS3_TRY(check_image(img_i, false));
  DS3_TRY(check_image(img_j, false));
  DS3_TRY(check_arch_local());
  const int pxb = dtype == DS3_F32 ? 16 : 8;
  const char* pi = static_cast<const char*>(X_i) + img_i.px_offset * pxb;
  const char* pj = static_cast<const char*>(X_j) + img_j.px_offset * pxb;
  return launch_gauge_align(pi, int64_t(img_i.H) * img_i.W, pj, int64_t(img_j.H) * img_j.W, dtype, idx_j2i,
                            valid_j, poses, i, j, ref_is_i ? 1 : 0, nc_min, T_out, used_umeyama, workspace,
                            S(stream));
}

int ds3_apply_gauge(double* poses, int32_t n_kf, const uint8_t* mask, const double* T, void* stream) {
  if (!poses || !mask || !T || n_kf < 0) return fail(DS3_EINVAL, "apply_gauge: bad arguments");
  DS3_TRY(check_arch_local());
  return launch_apply_gauge(poses, n_kf, mask, T, S(stream));
}

int ds3_gauge_sync(double* poses, int32_t n_kf, const int32_t* agent_of_kf, const void* kf_arena,
                   const ds3_image* kf, ds3_dtype dtype, const ds3_edge* edges, int32_t n_edges,
                   const int32_t* idx_arena, const uint8_t* valid_arena, const int32_t* admit,
                   int32_t nc_min, int32_t* n_links_out, void* workspace, size_t ws_bytes,
                   void* stream) {
  if (!poses || !agent_of_kf || !kf_arena || !kf || !edges || !idx_arena || !valid_arena || !admit ||
      !workspace)
    return fail(DS3_EINVAL, "gauge_sync: null pointer");
  if (n_kf <= 0 || n_edges < 0) return fail(DS3_EINVAL, "gauge_sync: bad sizes");
  if (ws_bytes < ds3_gauge_workspace_bytes(n_kf)) return fail(DS3_ENOSPACE, "gauge_sync: workspace");
  DS3_TRY(check_arch_local());
  hipStream_t s = S(stream);
  Carver w(workspace);
  void* gws = w.take<char>(gauge_ws_bytes());
  double* T = w.take<double>(8);
  int32_t* used = w.take<int32_t>(4);
  uint8_t* mask = w.take<uint8_t>(n_kf);
  std::vector<int32_t> adm(n_edges);
  if (n_edges > 0) {
    DS3_TRY(check_hip(hipMemcpyAsync(adm.data(), admit, sizeof(int32_t) * n_edges, hipMemcpyDeviceToHost, s),
                      "hipMemcpyAsync(admit)"));
    DS3_TRY(check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"));
  }
  int n_agents = 0;
  for (int k = 0; k < n_kf; ++k) {
    if (agent_of_kf[k] < 0) return fail(DS3_EINVAL, "gauge_sync: negative agent id");
    n_agents = std::max(n_agents, agent_of_kf[k] + 1);
  }
  std::vector<int> comp(n_agents);
  std::iota(comp.begin(), comp.end(), 0);  // label = smallest agent id of the component
  const int pxb = dtype == DS3_F32 ? 16 : 8;
  int links = 0;
  for (int e = 0; e < n_edges; ++e) {
    const int i = edges[e].i, j = edges[e].j;
    if (i < 0 || i >= n_kf || j < 0 || j >= n_kf) return fail(DS3_EINVAL, "gauge_sync: bad edge");
    const int ai = agent_of_kf[i], aj = agent_of_kf[j];
    if (ai == aj || !adm[e] || comp[ai] == comp[aj]) continue;
    const bool ref_is_i = comp[ai] < comp[aj];
    const int ref_c = ref_is_i ? comp[ai] : comp[aj], mov_c = ref_is_i ? comp[aj] : comp[ai];
    const char* pi = static_cast<const char*>(kf_arena) + kf[i].px_offset * pxb;
    const char* pj = static_cast<const char*>(kf_arena) + kf[j].px_offset * pxb;
    DS3_TRY(launch_gauge_align(pi, int64_t(kf[i].H) * kf[i].W, pj, int64_t(kf[j].H) * kf[j].W, dtype,
                               idx_arena + edges[e].idx_offset, valid_arena + edges[e].idx_offset, poses,
                               i, j, ref_is_i ? 1 : 0, nc_min, T, used, gws, s));
    std::vector<uint8_t> m(n_kf, 0);
    for (int k = 0; k < n_kf; ++k) m[k] = comp[agent_of_kf[k]] == mov_c ? 1 : 0;
    DS3_TRY(upload(mask, m, s));
    DS3_TRY(launch_apply_gauge(poses, n_kf, mask, T, s));
    // the mask upload of the next link must not overwrite this one before the kernel ran
    DS3_TRY(check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"));
    for (int a = 0; a < n_agents; ++a)
      if (comp[a] == mov_c) comp[a] = ref_c;
    ++links;
  }
  if (n_links_out) *n_links_out = links;
  return DS3_OK;
}

// ---- cost and adjoint (implemented in adjoint.hip) -------------------------------------------------------
}  // extern "C"
