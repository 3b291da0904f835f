// C ABI of libds3 (declared in include/ds3.h): argument checks, workspace layout, launch sequences of the
// plain form, and the batched plan (work-item ordering, tile autotuning, hipGraph capture).
#include <hip/hip_runtime.h>
#include <sys/stat.h>
#include <sys/types.h>

#include <algorithm>
#include <cerrno>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "internal.hpp"
#include "match_internal.hpp"

namespace ds3 {

// ---- error state -----------------------------------------------------------------------------------
static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return DS3_OK;
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return DS3_EHIP;
}

int device_cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return 256;
  return cus;
}

static int check_arch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(DS3_EHIP, "no HIP device");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(DS3_EHIP, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(DS3_ENOTSUP, std::string("libds3 is built for gfx950, device is ") + prop.gcnArchName);
  return DS3_OK;
}

static hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

// Upload a host vector into a device region (the copy is staged before the call returns).
template <class T>
static int upload(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return DS3_OK;
  return check_hip(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s),
                   "hipMemcpyAsync(upload)");
}

// ---- graph topology on the host ---------------------------------------------------------------------
struct Topology {
  int n_kf = 0, n_edges = 0, n_pairs = 0, total_tiles = 0, max_tiles = 0, tile_px = 0;
  std::vector<EdgeDev> edges;
  std::vector<int64_t> kf_off;
  std::vector<int32_t> kf_npx, kf_w, node_ptr, node_adj, pair_ptr, pair_edges, pair_ij;
  std::vector<uint8_t> anchor;
};

static int build_topology(int n_kf, const ds3_image* kf, int n_edges, const ds3_edge* edges,
                          const int32_t* anchors, int n_anchors, int tile_px, Topology& T) {
  if (n_kf <= 0 || !kf) return fail(DS3_EINVAL, "n_kf must be positive with a keyframe table");
  if (n_edges < 0 || (n_edges > 0 && !edges)) return fail(DS3_EINVAL, "bad edge table");
  if (n_anchors < 0 || (n_anchors > 0 && !anchors)) return fail(DS3_EINVAL, "bad anchor list");
  T.n_kf = n_kf;
  T.n_edges = n_edges;
  T.tile_px = tile_px;
  T.kf_off.resize(n_kf);
  T.kf_npx.resize(n_kf);
  T.kf_w.resize(n_kf);
  for (int k = 0; k < n_kf; ++k) {
    if (kf[k].H <= 0 || kf[k].W <= 0 || kf[k].px_offset < 0 || int64_t(kf[k].H) * kf[k].W > INT32_MAX)
      return fail(DS3_EINVAL, "bad keyframe image " + std::to_string(k));
    T.kf_off[k] = kf[k].px_offset;
    T.kf_npx[k] = kf[k].H * kf[k].W;
    T.kf_w[k] = kf[k].W;
  }
  T.edges.resize(n_edges);
  T.total_tiles = 0;
  T.max_tiles = 0;
  for (int e = 0; e < n_edges; ++e) {
    const ds3_edge& E = edges[e];
    if (E.i < 0 || E.i >= n_kf || E.j < 0 || E.j >= n_kf || E.i == E.j || E.idx_offset < 0)
      return fail(DS3_EINVAL, "bad edge " + std::to_string(e));
    EdgeDev D;
    D.off_i = kf[E.i].px_offset;
    D.off_j = kf[E.j].px_offset;
    D.idx_off = E.idx_offset;
    D.npx_i = kf[E.i].H * kf[E.i].W;
    D.npx_j = kf[E.j].H * kf[E.j].W;
    D.i = E.i;
    D.j = E.j;
    D.tile0 = T.total_tiles;
    D.n_tiles = (D.npx_j + tile_px - 1) / tile_px;
    T.total_tiles += D.n_tiles;
    T.max_tiles = std::max(T.max_tiles, D.n_tiles);
    T.edges[e] = D;
  }
  // incidence lists (edge index order) and keyframe pairs
  std::vector<std::vector<int32_t>> inc(n_kf);
  std::map<std::pair<int, int>, std::vector<int32_t>> pairs;
  for (int e = 0; e < n_edges; ++e) {
    inc[edges[e].i].push_back(e << 1);
    inc[edges[e].j].push_back((e << 1) | 1);
    int a = std::min(edges[e].i, edges[e].j), b = std::max(edges[e].i, edges[e].j);
    pairs[{a, b}].push_back(e);
  }
  T.node_ptr.assign(n_kf + 1, 0);
  T.node_adj.clear();
  for (int k = 0; k < n_kf; ++k) {
    T.node_ptr[k] = int32_t(T.node_adj.size());
    T.node_adj.insert(T.node_adj.end(), inc[k].begin(), inc[k].end());
  }
  T.node_ptr[n_kf] = int32_t(T.node_adj.size());
  T.pair_ptr.clear();
  T.pair_edges.clear();
  T.pair_ij.clear();
  for (auto& kv : pairs) {
    T.pair_ptr.push_back(int32_t(T.pair_edges.size()));
    T.pair_edges.insert(T.pair_edges.end(), kv.second.begin(), kv.second.end());
    T.pair_ij.push_back(kv.first.first);
    T.pair_ij.push_back(kv.first.second);
  }
  T.n_pairs = int(pairs.size());
  T.pair_ptr.push_back(int32_t(T.pair_edges.size()));
  T.anchor.assign(n_kf, 0);
  for (int a = 0; a < n_anchors; ++a) {
    if (anchors[a] < 0 || anchors[a] >= n_kf) return fail(DS3_EINVAL, "anchor out of range");
    T.anchor[anchors[a]] = 1;
  }
  return DS3_OK;
}

// Device buffers of one graph step, carved from a workspace.
struct GnBuffers {
  EdgeDev* edges;
  EdgeXf* xf;
  double* Ad;
  float* partials;
  double *A_e, *b_e, *cost_e;
  int64_t* count_e;
  int64_t* kf_off;
  int32_t *kf_npx, *node_ptr, *node_adj, *pair_ptr, *pair_edges, *pair_ij;
  uint8_t* anchor;
  double *H, *g, *tau;
  double* cost_tmp;
  int64_t* count_tmp;
  unsigned* counter;
  float* part7;
  void* chol_ws;
};

int adjoint_part_floats(int n_edges, int max_npx_j);
int launch_adjoint(ds3_dtype dt, const void* arena, const EdgeDev* edges, int n_edges, int max_npx_j,
                   int max_npx_kf, const EdgeXf* xf, const double* Ad, const int32_t* idx, GnConst c,
                   float dcost, float* grad_xyz, float* grad_conf, float* part7, double* b_e, int n_kf,
                   const int64_t* kf_off, const int32_t* kf_npx, const int32_t* node_ptr,
                   const int32_t* node_adj, double* grad_tau, ds3_timer* timer, hipStream_t s);

int launch_inverse_maps(const EdgeDev* edges, int n_edges, int max_npx_j, int max_npx_i, const int32_t* idx,
                        const int64_t* cbase, const int64_t* obase, const int64_t* sbase, int32_t* cnt,
                        size_t cnt_len, int32_t* off, int32_t* src, int32_t* head, hipStream_t s);
int launch_adjoint_gather(ds3_dtype dt, const void* arena, const EdgeDev* edges, int n_edges, int max_npx_j,
                          int max_npx_kf, const EdgeXf* xf, const double* Ad, const int32_t* idx, GnConst c,
                          float dcost, float* grad_xyz, float* grad_conf, float* part7, double* b_e,
                          double* cost_e, int64_t* count_e, int n_kf, const int64_t* kf_off,
                          const int32_t* kf_npx, const int32_t* node_ptr, const int32_t* node_adj,
                          const int64_t* obase, const int64_t* sbase, const int64_t* cbase,
                          const int32_t* inv_off, const int32_t* inv_src, const int32_t* inv_head, double* grad_tau,
                          ds3_timer* timer, hipStream_t s);
int launch_cost_batched(ds3_dtype dt, const void* arena, const EdgeDev* edges, int n_edges, int max_npx_j,
                        const EdgeXf* xf, const int32_t* idx, GnConst c, float* part, double* cost_e,
                        int64_t* count_e, hipStream_t s);
static int max_npx_j(const Topology& T) {
  int m = 0;
  for (auto& E : T.edges) m = std::max(m, int(E.npx_j));
  return m;
}

static size_t carve_gn(void* base, const Topology& T, GnBuffers& B) {
  Carver c(base);
  const int E = std::max(T.n_edges, 1);
  const size_t n = 7 * size_t(T.n_kf);
  B.edges = c.take<EdgeDev>(E);
  B.xf = c.take<EdgeXf>(E);
  B.Ad = c.take<double>(49 * size_t(E));
  B.partials = c.take<float>(size_t(std::max(T.total_tiles, 1)) * kPartial);
  B.A_e = c.take<double>(49 * size_t(E));
  B.b_e = c.take<double>(7 * size_t(E));
  B.cost_e = c.take<double>(E);
  B.count_e = c.take<int64_t>(E);
  B.kf_off = c.take<int64_t>(T.n_kf);
  B.kf_npx = c.take<int32_t>(T.n_kf);
  B.node_ptr = c.take<int32_t>(T.n_kf + 1);
  B.node_adj = c.take<int32_t>(2 * size_t(E));
  B.pair_ptr = c.take<int32_t>(size_t(E) + 1);
  B.pair_edges = c.take<int32_t>(E);
  B.pair_ij = c.take<int32_t>(2 * size_t(E));
  B.anchor = c.take<uint8_t>(T.n_kf);
  B.H = c.take<double>(n * n);
  B.g = c.take<double>(n);
  B.tau = c.take<double>(n);
  B.cost_tmp = c.take<double>(1);
  B.count_tmp = c.take<int64_t>(1);
  B.counter = c.take<unsigned>(64);
  B.part7 = c.take<float>(size_t(std::max(adjoint_part_floats(T.n_edges, max_npx_j(T)), 8)));
  B.chol_ws = c.take<char>(chol_workspace_bytes(int(n)));
  return c.used;
}

static int upload_topology(const Topology& T, GnBuffers& B, hipStream_t s) {
  DS3_TRY(upload(B.edges, T.edges, s));
  DS3_TRY(upload(B.kf_off, T.kf_off, s));
  DS3_TRY(upload(B.kf_npx, T.kf_npx, s));
  DS3_TRY(upload(B.node_ptr, T.node_ptr, s));
  DS3_TRY(upload(B.node_adj, T.node_adj, s));
  DS3_TRY(upload(B.pair_ptr, T.pair_ptr, s));
  DS3_TRY(upload(B.pair_edges, T.pair_edges, s));
  DS3_TRY(upload(B.pair_ij, T.pair_ij, s));
  DS3_TRY(upload(B.anchor, T.anchor, s));
  return DS3_OK;
}

constexpr int kPlainPPT = 16;

static int check_gn_args(const double* poses, const void* arena, const int32_t* idx, ds3_dtype dt,
                         const ds3_gn_params* p) {
  if (!poses || !arena || !idx || !p) return fail(DS3_EINVAL, "null pointer");
  if (dt != DS3_F32 && dt != DS3_BF16) return fail(DS3_ENOTSUP, "dtype");
  if ((reinterpret_cast<uintptr_t>(arena) & 15) != 0) return fail(DS3_EINVAL, "arena must be 16 B aligned");
  if (!(p->sigma_ray > 0) || !(p->sigma_dist > 0) || !(p->huber_k > 0))
    return fail(DS3_EINVAL, "sigma and kappa must be positive");
  if (p->max_attempts < 1 || p->max_attempts > 16) return fail(DS3_EINVAL, "max_attempts out of range");
  if (p->K && (!(p->sigma_pix > 0) || !(p->sigma_logz > 0)))
    return fail(DS3_EINVAL, "calibrated mode: sigma_pix and sigma_logz must be positive");
  return DS3_OK;
}

// The calls without a calibrated form.
static int no_calibrated(const ds3_gn_params* p, const char* what) {
  if (p && p->K) return fail(DS3_ENOTSUP, std::string(what) + ": no calibrated mode (K must be NULL)");
  return DS3_OK;
}

static int edge_cal_table(const ds3_gn_params& p, const Topology& T, std::vector<EdgeCal>& out) {
  out.assign(std::max(T.n_edges, 1), EdgeCal{});
  if (!p.K) return DS3_OK;
  return make_edge_cal(p.K, T.n_kf, T.kf_w.data(), T.edges.data(), T.n_edges, out.data());
}

// Plain-form linearisation: prep, one residual launch per edge, finalize, assembly, cost sum.
static int gn_linearize_plain(const double* poses, const Topology& T, const GnBuffers& B,
                              const void* arena, ds3_dtype dt, const int32_t* idx,
                              const ds3_gn_params& p, double* H, double* g, double* cost_out,
                              int64_t* count_out, hipStream_t s) {
  const GnConst c = make_gn_const(p);
  std::vector<EdgeCal> cal;
  DS3_TRY(edge_cal_table(p, T, cal));
  DS3_TRY(launch_gn_prep(poses, B.edges, T.n_edges, B.xf, B.Ad, s));
  for (int e = 0; e < T.n_edges; ++e)
    DS3_TRY(launch_edge_reduce_one(dt, kPlainPPT, arena, T.edges[e], e, B.xf, idx, B.partials, c, s,
                                   p.K ? &cal[e] : nullptr));
  DS3_TRY(launch_edge_finalize(B.edges, T.n_edges, B.partials, B.Ad, B.A_e, B.b_e, B.cost_e, B.count_e, s));
  const size_t n = 7 * size_t(T.n_kf);
  DS3_TRY(launch_fill(H, n * n, 0.0, s));
  DS3_TRY(launch_assemble(T.n_kf, B.node_ptr, B.node_adj, B.pair_ptr, B.pair_edges, B.pair_ij, T.n_pairs,
                          B.A_e, B.b_e, B.anchor, H, g, s));
  return launch_sum_costs(B.cost_e, B.count_e, T.n_edges, cost_out, count_out, s);
}

}  // namespace ds3

using namespace ds3;

// =====================================================================================================
// Basics
// =====================================================================================================
extern "C" {

void ds3_default_match_params(ds3_match_params* p) {
  if (!p) return;
  p->max_iters = 10;
  p->lambda0 = 1e-4;
  p->lambda_min = 1e-9;
  p->step_tol_px = 1e-4;
  p->ang_tol_px = 0.5;
  p->range_rel_tol = 0.10;
  p->mutual_radius_px = 1;
  p->q_min = 1.5;
  p->nu_min = 0.1;
}

void ds3_default_gn_params(ds3_gn_params* p) {
  if (!p) return;
  p->sigma_ray = 0.003;
  p->sigma_dist = 10.0;
  p->huber_k = 1.345;
  p->lambda = 0.0;
  p->eps0 = 1e-6;
  p->eps_mult = 100.0;
  p->max_attempts = 6;
  p->K = nullptr;
  p->sigma_pix = 1.0;
  p->sigma_logz = 0.1;
}

const char* ds3_status_string(int code) {
  static thread_local std::string msg;
  const char* name = code == DS3_OK ? "ok"
                     : code == DS3_EINVAL ? "invalid argument"
                     : code == DS3_ENOTSUP ? "not supported"
                     : code == DS3_EHIP ? "HIP error"
                     : code == DS3_ENOSPACE ? "workspace too small"
                     : code == DS3_EDEGENERATE ? "degenerate input"
                                            : "unknown";
  msg = std::string(name) + (g_last_error.empty() ? "" : " (" + g_last_error + ")");
  return msg.c_str();
}

int ds3_version(void) { return 100; }

int ds3_pack_xyzc(const float* xyz, const float* conf, int64_t n_px, ds3_dtype dtype, void* out,
                  void* stream) {
  if (n_px < 0 || (n_px > 0 && (!xyz || !conf || !out))) return fail(DS3_EINVAL, "pack: bad arguments");
  if (dtype != DS3_F32 && dtype != DS3_BF16) return fail(DS3_ENOTSUP, "pack: dtype");
  if ((reinterpret_cast<uintptr_t>(out) & 15) != 0) return fail(DS3_EINVAL, "pack: output not 16 B aligned");
  DS3_TRY(check_arch());
  return launch_pack(xyz, conf, n_px, dtype, out, S(stream));
}

// =====================================================================================================
// Sim(3)
// =====================================================================================================
int ds3_sim3_exp(const double* tau, double* poses_out, int32_t n, void* stream) {
  if (n < 0 || (n > 0 && (!tau || !poses_out))) return fail(DS3_EINVAL, "sim3_exp: bad arguments");
  DS3_TRY(check_arch());
  return launch_sim3_exp(tau, poses_out, n, S(stream));
}

int ds3_sim3_log(const double* poses, double* tau_out, int32_t n, void* stream) {
  if (n < 0 || (n > 0 && (!poses || !tau_out))) return fail(DS3_EINVAL, "sim3_log: bad arguments");
  DS3_TRY(check_arch());
  return launch_sim3_log(poses, tau_out, n, S(stream));
}

int ds3_sim3_update(double* poses, const double* tau, const uint8_t* fixed, int32_t n, void* stream) {
  if (n < 0 || (n > 0 && (!poses || !tau))) return fail(DS3_EINVAL, "sim3_update: bad arguments");
  DS3_TRY(check_arch());
  return launch_sim3_update(poses, tau, fixed, n, S(stream));
}

// =====================================================================================================
// Cholesky ladder
// =====================================================================================================
size_t ds3_chol_workspace_bytes(int32_t n) { return n > 0 ? chol_workspace_bytes(n) : 0; }

int ds3_chol_ladder_solve(const double* H, const double* g, int32_t n, double lambda, double eps0,
                          double mult, int32_t attempts, double* tau, int32_t* status, void* workspace,
                          size_t ws_bytes, void* stream) {
  if (n <= 0 || !H || !g || !tau || !status || !workspace) return fail(DS3_EINVAL, "chol: bad arguments");
  if (ws_bytes < chol_workspace_bytes(n)) return fail(DS3_ENOSPACE, "chol: workspace too small");
  DS3_TRY(check_arch());
  return launch_chol_ladder(H, g, n, lambda, eps0, mult, attempts, tau, status, workspace, S(stream));
}

// =====================================================================================================
// Graph step, plain form
// =====================================================================================================
size_t ds3_gn_workspace_bytes(int32_t n_kf, const ds3_image* kf, int32_t n_edges, const ds3_edge* edges,
                              ds3_dtype dtype) {
  (void)dtype;
  Topology T;
  if (build_topology(n_kf, kf, n_edges, edges, nullptr, 0, kReduceThreads * kPlainPPT, T) != DS3_OK) return 0;
  GnBuffers B;
  return carve_gn(nullptr, T, B);
}

int ds3_gn_linearize(const double* poses, int32_t n_kf, const ds3_image* kf, const void* arena,
                     ds3_dtype dtype, const ds3_edge* edges, int32_t n_edges, const int32_t* idx,
                     const ds3_gn_params* params, const int32_t* anchors, int32_t n_anchors, double* H,
                     double* g, double* cost_out, int64_t* count_out, void* workspace, size_t ws_bytes,
                     void* stream) {
  DS3_TRY(check_gn_args(poses, arena, idx, dtype, params));
  if (!H || !g || !cost_out || !workspace) return fail(DS3_EINVAL, "null output or workspace");
  Topology T;
  DS3_TRY(build_topology(n_kf, kf, n_edges, edges, anchors, n_anchors, kReduceThreads * kPlainPPT, T));
  GnBuffers B;
  if (ws_bytes < carve_gn(nullptr, T, B)) return fail(DS3_ENOSPACE, "gn: workspace too small");
  carve_gn(workspace, T, B);
  DS3_TRY(check_arch());
  hipStream_t s = S(stream);
  DS3_TRY(upload_topology(T, B, s));
  return gn_linearize_plain(poses, T, B, arena, dtype, idx, *params, H, g, cost_out, count_out, s);
}

int ds3_sim3_gn_step(double* poses, int32_t n_kf, const ds3_image* kf, const void* arena, ds3_dtype dtype,
                     const ds3_edge* edges, int32_t n_edges, const int32_t* idx,
                     const ds3_gn_params* params, const int32_t* anchors, int32_t n_anchors,
                     double* cost_out, int32_t* status_out, double* tau_out, void* workspace,
                     size_t ws_bytes, void* stream) {
  DS3_TRY(check_gn_args(poses, arena, idx, dtype, params));
  if (!cost_out || !status_out || !workspace) return fail(DS3_EINVAL, "null output or workspace");
  Topology T;
  DS3_TRY(build_topology(n_kf, kf, n_edges, edges, anchors, n_anchors, kReduceThreads * kPlainPPT, T));
  GnBuffers B;
  if (ws_bytes < carve_gn(nullptr, T, B)) return fail(DS3_ENOSPACE, "gn: workspace too small");
  carve_gn(workspace, T, B);
  DS3_TRY(check_arch());
  hipStream_t s = S(stream);
  DS3_TRY(upload_topology(T, B, s));
  DS3_TRY(gn_linearize_plain(poses, T, B, arena, dtype, idx, *params, B.H, B.g, cost_out, nullptr, s));
  const int n = 7 * n_kf;
  double* tau = tau_out ? tau_out : B.tau;
  DS3_TRY(launch_chol_ladder(B.H, B.g, n, params->lambda, params->eps0, params->eps_mult,
                             params->max_attempts, tau, status_out, B.chol_ws, s));
  return launch_sim3_update(poses, tau, B.anchor, n_kf, s);
}

int ds3_gn_cost(const double* poses, int32_t n_kf, const ds3_image* kf, const void* arena, ds3_dtype dtype,
                const ds3_edge* edges, int32_t n_edges, const int32_t* idx, const ds3_gn_params* params,
                double* cost_out, void* workspace, size_t ws_bytes, void* stream) {
  DS3_TRY(check_gn_args(poses, arena, idx, dtype, params));
  DS3_TRY(no_calibrated(params, "gn_cost"));
  if (!cost_out || !workspace) return fail(DS3_EINVAL, "null output or workspace");
  Topology T;
  DS3_TRY(build_topology(n_kf, kf, n_edges, edges, nullptr, 0, kReduceThreads * kPlainPPT, T));
  GnBuffers B;
  if (ws_bytes < carve_gn(nullptr, T, B)) return fail(DS3_ENOSPACE, "gn_cost: workspace too small");
  carve_gn(workspace, T, B);
  DS3_TRY(check_arch());
  hipStream_t s = S(stream);
  DS3_TRY(upload_topology(T, B, s));
  DS3_TRY(launch_gn_prep(poses, B.edges, T.n_edges, B.xf, B.Ad, s));
  DS3_TRY(launch_cost_batched(dtype, arena, B.edges, T.n_edges, max_npx_j(T), B.xf, idx, make_gn_const(*params),
                              B.part7, B.cost_e, B.count_e, s));
  return launch_sum_costs(B.cost_e, B.count_e, T.n_edges, cost_out, nullptr, s);
}

int ds3_gn_cost_adjoint(const double* poses, int32_t n_kf, const ds3_image* kf, const void* arena,
                        ds3_dtype dtype, const ds3_edge* edges, int32_t n_edges, const int32_t* idx,
                        const ds3_gn_params* params, float dcost, float* grad_xyz, float* grad_conf,
                        double* grad_tau, ds3_timer* adjoint_timer, void* workspace, size_t ws_bytes,
                        void* stream) {
  DS3_TRY(check_gn_args(poses, arena, idx, dtype, params));
  DS3_TRY(no_calibrated(params, "gn_cost_adjoint"));
  if (!grad_xyz || !grad_conf || !grad_tau || !workspace) return fail(DS3_EINVAL, "null output or workspace");
  Topology T;
  DS3_TRY(build_topology(n_kf, kf, n_edges, edges, nullptr, 0, kReduceThreads * kPlainPPT, T));
  GnBuffers B;
  if (ws_bytes < carve_gn(nullptr, T, B)) return fail(DS3_ENOSPACE, "gn_adjoint: workspace too small");
  carve_gn(workspace, T, B);
  DS3_TRY(check_arch());
  hipStream_t s = S(stream);
  DS3_TRY(upload_topology(T, B, s));
  DS3_TRY(launch_gn_prep(poses, B.edges, T.n_edges, B.xf, B.Ad, s));
  const int max_npx_kf = *std::max_element(T.kf_npx.begin(), T.kf_npx.end());
  return launch_adjoint(dtype, arena, B.edges, T.n_edges, max_npx_j(T), max_npx_kf, B.xf, B.Ad, idx,
                        make_gn_const(*params), dcost, grad_xyz, grad_conf, B.part7, B.b_e, T.n_kf, B.kf_off,
                        B.kf_npx, B.node_ptr, B.node_adj, grad_tau, adjoint_timer, s);
}

}  // extern "C"

// =====================================================================================================
// Batched plan
// =====================================================================================================
namespace ds3 {

constexpr int kHistory = 4096;

struct Plan {
  Topology T;
  GnBuffers B;
  void* ws = nullptr;
  const void* arena = nullptr;
  const int32_t* idx = nullptr;
  double* poses = nullptr;
  ds3_dtype dt = DS3_F32;
  ds3_gn_params p;
  GnConst c;
  int ppt = 16;         // segment = kReduceThreads * ppt pixels of keyframe j
  int unroll = 2;       // match records in flight per thread in the residual kernel
  int n_items = 0;
  WorkItem* items = nullptr;
  void* stream = nullptr;      // match stream: records of every segment (capacity for the largest segment)
  int32_t* seg_count = nullptr;  // records per segment
  size_t stream_cap = 0;       // records the stream holds
  int64_t n_records = 0;       // records gathered at creation (matches passing the static checks)
  int reserved_tiles = 0;      // partial and count slots (tiles of the smallest segment size)
  double* cost_hist = nullptr;
  int32_t* status_hist = nullptr;
  unsigned* hist_ctr = nullptr;
  unsigned* time_ctrs = nullptr;
  int64_t px_scanned = 0, px_valid = 0;
  EdgeCal* ecal = nullptr;     // calibrated mode: per-edge intrinsics (device), else NULL
  bool use_graph = true;
  ds3_timer* timer = nullptr;
  hipGraph_t graph = nullptr;  // one iteration
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph_chunk = nullptr;  // kGraphChunk iterations in one graph (one launch gap per chunk)
  hipGraphExec_t exec_chunk = nullptr;
  SpChol* sp = nullptr;        // block-sparse solver of the plan's pattern, NULL otherwise
  TileChol* tc = nullptr;      // tile-sparse solver of the plan's pattern, NULL otherwise
};

constexpr int kGraphChunk = 8;  // iterations per chunk graph of a plan

// One GN iteration; `timed` records the plan's timer around the residual launch (never inside a capture).
static int plan_iteration(Plan& P, hipStream_t s, bool timed) {
  DS3_TRY(launch_gn_prep(P.poses, P.B.edges, P.T.n_edges, P.B.xf, P.B.Ad, s));
  if (timed) DS3_TRY(timer_record(P.timer, true, s));
  DS3_TRY(launch_reduce_stream(P.dt, P.unroll, P.stream, P.seg_count, P.B.edges, P.items, P.n_items, P.B.xf,
                               P.T.tile_px, P.B.partials, P.c, nullptr, s, nullptr, nullptr, P.ecal));
  if (timed) DS3_TRY(timer_record(P.timer, false, s));
  DS3_TRY(launch_edge_finalize(P.B.edges, P.T.n_edges, P.B.partials, P.B.Ad, P.B.A_e, P.B.b_e, P.B.cost_e,
                               P.B.count_e, s));
  const size_t n = 7 * size_t(P.T.n_kf);
  // H was cleared once at plan creation: the assembly rewrites every block of its fixed nonzero pattern
  // with the tile-sparse solver, the assembly also clears the solve's barrier words and attempt-0 flag (one
  // launch fewer per iteration)
  unsigned* sync = P.tc ? chol_sync_words(P.B.chol_ws, int(n)) : nullptr;
  DS3_TRY(launch_assemble(P.T.n_kf, P.B.node_ptr, P.B.node_adj, P.B.pair_ptr, P.B.pair_edges, P.B.pair_ij,
                          P.T.n_pairs, P.B.A_e, P.B.b_e, P.B.anchor, P.B.H, P.B.g, s, sync, sync ? 4 : 0));
  int32_t* status = reinterpret_cast<int32_t*>(P.B.counter + 8);
  if (P.sp)
    DS3_TRY(launch_spchol(P.sp, P.B.H, P.B.g, P.p.lambda, P.p.eps0, P.p.eps_mult, P.p.max_attempts, P.B.tau,
                          status, s));
  else if (P.tc)
    DS3_TRY(launch_tilechol(P.tc, P.B.H, P.B.g, P.p.lambda, P.p.eps0, P.p.eps_mult, P.p.max_attempts, P.B.tau,
                            status, P.B.chol_ws, s, true));
  else
    DS3_TRY(launch_chol_ladder(P.B.H, P.B.g, int(n), P.p.lambda, P.p.eps0, P.p.eps_mult, P.p.max_attempts,
                               P.B.tau, status, P.B.chol_ws, s));
  // the update, and the cost at the iteration's input poses (cost_e is rewritten only by the next iteration)
  // with the ladder status to the history, in one launch
  return launch_update_record(P.poses, P.B.tau, P.B.anchor, P.T.n_kf, P.B.cost_e, P.B.count_e, P.T.n_edges,
                              P.B.cost_tmp, P.B.count_tmp, status, P.hist_ctr, P.cost_hist, P.status_hist, kHistory, s);
}

// Order (edge, tile) items by descending valid count for the current tile shape.
static int plan_build_items(Plan& P, int ppt, hipStream_t s) {
  const int tile_px = kReduceThreads * ppt;
  Topology T2 = P.T;
  int total = 0, mx = 0;
  for (auto& E : T2.edges) {
    E.tile0 = total;
    E.n_tiles = (E.npx_j + tile_px - 1) / tile_px;
    total += E.n_tiles;
    mx = std::max(mx, E.n_tiles);
  }
  if (total > P.reserved_tiles) return fail(DS3_EINVAL, "plan: tile table larger than reserved");
  T2.total_tiles = total;
  T2.max_tiles = mx;
  T2.tile_px = tile_px;
  DS3_TRY(upload(P.B.edges, T2.edges, s));
  int32_t* counts_dev = reinterpret_cast<int32_t*>(P.B.partials);  // scratch (re-written every iteration)
  DS3_TRY(launch_count_valid(P.B.edges, T2.n_edges, P.idx, tile_px, mx, counts_dev, s));
  std::vector<int32_t> counts(std::max(total, 1));
  DS3_TRY_HIP(hipMemcpyAsync(counts.data(), counts_dev, sizeof(int32_t) * total, hipMemcpyDeviceToHost, s));
  DS3_TRY_HIP(hipStreamSynchronize(s));
  std::vector<WorkItem> items;
  items.reserve(total);
  P.px_valid = 0;
  for (int e = 0; e < T2.n_edges; ++e)
    for (int t = 0; t < T2.edges[e].n_tiles; ++t) {
      P.px_valid += counts[T2.edges[e].tile0 + t];
      items.push_back(WorkItem{e, t});  // every tile: the plan stays valid when the matches change
    }
  std::stable_sort(items.begin(), items.end(), [&](const WorkItem& a, const WorkItem& b) {
    return counts[T2.edges[a.edge].tile0 + a.tile] > counts[T2.edges[b.edge].tile0 + b.tile];
  });
  DS3_TRY(upload(P.items, items, s));
  P.n_items = int(items.size());
  P.ppt = ppt;
  P.T.edges = T2.edges;
  P.T.total_tiles = total;
  P.T.max_tiles = mx;
  P.T.tile_px = tile_px;
  if (size_t(total) * size_t(tile_px) > P.stream_cap) return fail(DS3_EINVAL, "plan: stream larger than reserved");
  // gather the match stream for this segment size and read back how many records it holds
  DS3_TRY(launch_gather_stream(P.dt, P.arena, P.B.edges, P.items, P.n_items, P.idx, tile_px, P.stream,
                               P.seg_count, s, P.ecal));
  DS3_TRY_HIP(hipMemcpyAsync(counts.data(), P.seg_count, sizeof(int32_t) * total, hipMemcpyDeviceToHost, s));
  DS3_TRY_HIP(hipStreamSynchronize(s));
  P.n_records = 0;
  for (int t = 0; t < total; ++t) P.n_records += counts[t];
  return DS3_OK;
}

static int plan_time_reduce(Plan& P, int reps, float* ms, hipStream_t s) {
  DS3_TRY(launch_gn_prep(P.poses, P.B.edges, P.T.n_edges, P.B.xf, P.B.Ad, s));
  DS3_TRY(launch_fill_u32(P.time_ctrs, size_t(reps), 0u, s));
  hipEvent_t a, b;
  DS3_TRY_HIP(hipEventCreate(&a));
  DS3_TRY_HIP(hipEventCreate(&b));
  int rc = check_hip(hipEventRecord(a, s), "hipEventRecord");
  for (int r = 0; r < reps && rc == DS3_OK; ++r)
    rc = launch_reduce_stream(P.dt, P.unroll, P.stream, P.seg_count, P.B.edges, P.items, P.n_items, P.B.xf,
                              P.T.tile_px, P.B.partials, P.c, nullptr, s, nullptr, nullptr, P.ecal);
  if (rc == DS3_OK) rc = check_hip(hipEventRecord(b, s), "hipEventRecord");
  if (rc == DS3_OK) rc = check_hip(hipEventSynchronize(b), "hipEventSynchronize");
  float t = 0.f;
  if (rc == DS3_OK) rc = check_hip(hipEventElapsedTime(&t, a, b), "hipEventElapsedTime");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc == DS3_OK) *ms = t / float(reps);
  return rc;
}

static std::string tune_key(const Plan& P) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  (void)hipGetDeviceProperties(&prop, dev);
  std::map<std::pair<int, int>, int> shapes;
  for (auto& E : P.T.edges) shapes[{E.npx_j, E.npx_i}]++;
  std::ostringstream k;
  k << prop.gcnArchName << "|stream|" << (P.dt == DS3_F32 ? "f32" : "bf16") << (P.ecal ? "|cal" : "") << "|cu"
    << prop.multiProcessorCount;
  for (auto& kv : shapes) k << "|" << kv.first.first << "x" << kv.first.second;
  return k.str();
}

static std::string tune_cache_path() {
  const char* env = std::getenv("DS3_TUNE_CACHE");
  if (env && *env) return env;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/ds3_tune.txt";
}

static bool tune_lookup(const std::string& key, int& ppt, int& bpc) {
  std::ifstream f(tune_cache_path());
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    auto tab = line.rfind('\t');
    if (tab == std::string::npos) continue;
    if (line.substr(0, tab) != key) continue;
    int a = 0, b = 0;
    if (std::sscanf(line.c_str() + tab + 1, "%d %d", &a, &b) == 2 && a > 0 && b > 0) {
      ppt = a;
      bpc = b;
      found = true;
    }
  }
  return found;
}

// Creates every missing directory of `dir` with mkdir(2) (no child process: the caller has already
// initialised the GPU). Errors are ignored; the cache write that follows simply fails.
void make_dirs(const std::string& dir) {
  for (size_t pos = 1; pos <= dir.size(); ++pos) {
    if (pos == dir.size() || dir[pos] == '/') (void)::mkdir(dir.substr(0, pos).c_str(), 0755);
  }
}

static void tune_store(const std::string& key, int ppt, int bpc) {
  std::string path = tune_cache_path();
  auto slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) make_dirs(path.substr(0, slash));
  std::ofstream f(path, std::ios::app);
  if (f) f << key << "\t" << ppt << " " << bpc << "\n";
}

static std::string tune_cache_dir() {
  const std::string path = tune_cache_path();
  const auto slash = path.rfind('/');
  return (slash != std::string::npos && slash > 0) ? path.substr(0, slash) : std::string();
}

static int plan_autotune(Plan& P, hipStream_t s) {
  const std::string key = tune_key(P);
  int best_ppt = 16, best_unroll = 2;
  if (tune_lookup(key, best_ppt, best_unroll) && (best_unroll == 1 || best_unroll == 2 || best_unroll == 4) &&
      (best_ppt == 8 || best_ppt == 16 || best_ppt == 32 || best_ppt == 64)) {
    P.unroll = best_unroll;
    return plan_build_items(P, best_ppt, s);
  }
  // per segment size, the records-in-flight variants are timed in interleaved passes and each keeps its
  // fastest pass: the variants differ by a few percent, less than the clock drifts over a sweep
  constexpr int kPasses = 3;
  constexpr int kUnrolls[3] = {1, 2, 4};
  float best = 1e30f;
  for (int ppt : {8, 16, 32, 64}) {
    DS3_TRY(plan_build_items(P, ppt, s));
    float t[3] = {1e30f, 1e30f, 1e30f};
    for (int r = 0; r < kPasses; ++r)
      for (int u = 0; u < 3; ++u) {
        P.unroll = kUnrolls[u];
        float ms = 0.f;
        if (r == 0) DS3_TRY(plan_time_reduce(P, 2, &ms, s));  // warm
        DS3_TRY(plan_time_reduce(P, 5, &ms, s));
        t[u] = std::min(t[u], ms);
      }
    for (int u = 0; u < 3; ++u)
      if (t[u] < best) {
        best = t[u];
        best_ppt = ppt;
        best_unroll = kUnrolls[u];
      }
  }
  tune_store(key, best_ppt, best_unroll);
  P.unroll = best_unroll;
  return plan_build_items(P, best_ppt, s);
}

static void plan_free(Plan* P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->exec_chunk) (void)hipGraphExecDestroy(P->exec_chunk);
  if (P->graph_chunk) (void)hipGraphDestroy(P->graph_chunk);
  if (P->ws) (void)hipFree(P->ws);
  if (P->items) (void)hipFree(P->items);
  if (P->cost_hist) (void)hipFree(P->cost_hist);
  if (P->status_hist) (void)hipFree(P->status_hist);
  if (P->hist_ctr) (void)hipFree(P->hist_ctr);
  if (P->time_ctrs) (void)hipFree(P->time_ctrs);
  if (P->stream) (void)hipFree(P->stream);
  if (P->seg_count) (void)hipFree(P->seg_count);
  if (P->ecal) (void)hipFree(P->ecal);
  spchol_destroy(P->sp);
  tilechol_destroy(P->tc);
  delete P;
}

// Solver of the normal equations: 1 the dense one, 2 the block-sparse one and 3 the tile-sparse one for
// the plan's pattern (pairs that touch an anchor are zero blocks of H and stay out of the pattern); 0 the
// tile-sparse one when its elimination tree has fewer levels than the dense solver has panels, else the
// dense one.
static int plan_pick_solver(Plan& P, int solver) {
  if (solver < 0 || solver > 3) return fail(DS3_EINVAL, "plan: solver must be 0, 1, 2 or 3");
  if (solver == 1) return DS3_OK;
  std::vector<int32_t> pairs;
  for (int p = 0; p < P.T.n_pairs; ++p) {
    const int a = P.T.pair_ij[2 * p], b = P.T.pair_ij[2 * p + 1];
    if (P.T.anchor[a] || P.T.anchor[b]) continue;
    pairs.push_back(a);
    pairs.push_back(b);
  }
  if (solver == 2) return spchol_create(P.T.n_kf, int(pairs.size() / 2), pairs.data(), &P.sp);
  DS3_TRY(tilechol_create(P.T.n_kf, int(pairs.size() / 2), pairs.data(), &P.tc));
  if (solver == 0) {
    int64_t info[7];
    tilechol_stats(P.tc, info);
    const int64_t panels = (7 * int64_t(P.T.n_kf) + 31) / 32;
    if (info[3] >= panels) {
      tilechol_destroy(P.tc);
      P.tc = nullptr;
    }
  }
  return DS3_OK;
}

int timer_record(ds3_timer* t, bool begin, hipStream_t s) {
  if (!t) return DS3_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  DS3_TRY_HIP(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return fail(DS3_ENOTSUP, "timer: not recordable inside a capture");
  DS3_TRY_HIP(hipEventRecord(t->ev[begin ? 0 : 1], s));
  if (!begin) t->recorded = true;
  return DS3_OK;
}

}  // namespace ds3

extern "C" {

int ds3_timer_create(ds3_timer** out) {
  if (!out) return fail(DS3_EINVAL, "timer: out is null");
  *out = nullptr;
  ds3_timer* t = new ds3_timer();
  for (int k = 0; k < 2; ++k) {
    const int rc = check_hip(hipEventCreate(&t->ev[k]), "hipEventCreate");
    if (rc != DS3_OK) {
      if (k == 1) (void)hipEventDestroy(t->ev[0]);
      delete t;
      return rc;
    }
  }
  *out = t;
  return DS3_OK;
}

int ds3_timer_elapsed_ms(ds3_timer* t, float* ms) {
  if (!t || !ms) return fail(DS3_EINVAL, "timer: bad arguments");
  if (!t->recorded) return fail(DS3_EINVAL, "timer: nothing recorded yet");
  DS3_TRY_HIP(hipEventSynchronize(t->ev[1]));
  DS3_TRY_HIP(hipEventElapsedTime(ms, t->ev[0], t->ev[1]));
  return DS3_OK;
}

int ds3_timer_destroy(ds3_timer* t) {
  if (!t) return DS3_OK;
  (void)hipEventDestroy(t->ev[0]);
  (void)hipEventDestroy(t->ev[1]);
  delete t;
  return DS3_OK;
}

int ds3_gn_plan_create(int32_t n_kf, const ds3_image* kf, const void* arena, ds3_dtype dtype,
                       const ds3_edge* edges, int32_t n_edges, const int32_t* idx,
                       const ds3_gn_params* params, const int32_t* anchors, int32_t n_anchors,
                       const ds3_plan_opts* opts, double* poses, void** plan_out, void* stream) {
  if (!plan_out) return fail(DS3_EINVAL, "plan_out is null");
  *plan_out = nullptr;
  DS3_TRY(check_gn_args(poses, arena, idx, dtype, params));
  DS3_TRY(check_arch());
  hipStream_t s = S(stream);
  Plan* P = new Plan();
  // reserve partial slots for the smallest tile (4 px per thread)
  int rc = build_topology(n_kf, kf, n_edges, edges, anchors, n_anchors, kReduceThreads * 4, P->T);
  if (rc != DS3_OK) { plan_free(P); return rc; }
  const size_t ws = carve_gn(nullptr, P->T, P->B);
  rc = check_hip(hipMalloc(&P->ws, ws), "hipMalloc(plan)");
  if (rc == DS3_OK) rc = check_hip(hipMalloc(&P->items, sizeof(WorkItem) * std::max(P->T.total_tiles, 1)), "hipMalloc(items)");
  if (rc == DS3_OK) rc = check_hip(hipMalloc(&P->cost_hist, sizeof(double) * kHistory), "hipMalloc");
  if (rc == DS3_OK) rc = check_hip(hipMalloc(&P->status_hist, sizeof(int32_t) * kHistory), "hipMalloc");
  if (rc == DS3_OK) rc = check_hip(hipMalloc(&P->hist_ctr, sizeof(unsigned) * 4), "hipMalloc");
  if (rc == DS3_OK) rc = check_hip(hipMalloc(&P->time_ctrs, sizeof(unsigned) * 64), "hipMalloc");
  // match stream: room for every pixel of every edge at the largest segment size (the padding of the
  // last segment of each edge included); segment counts for the smallest segment size
  for (int ppt : {4, 8, 16, 32, 64}) {
    const size_t seg = size_t(kReduceThreads) * ppt;
    size_t cap = 0;
    for (auto& E : P->T.edges) cap += (size_t(E.npx_j) + seg - 1) / seg * seg;
    P->stream_cap = std::max(P->stream_cap, cap);
  }
  if (rc == DS3_OK)
    rc = check_hip(hipMalloc(&P->stream, std::max<size_t>(P->stream_cap, 1) * stream_record_bytes(dtype, params->K)),
                   "hipMalloc(match stream)");
  if (rc == DS3_OK && params->K) {
    std::vector<EdgeCal> cal;
    rc = edge_cal_table(*params, P->T, cal);
    if (rc == DS3_OK) rc = check_hip(hipMalloc(&P->ecal, sizeof(EdgeCal) * cal.size()), "hipMalloc(intrinsics)");
    if (rc == DS3_OK) rc = upload(P->ecal, cal, s);
    if (rc == DS3_OK) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize(intrinsics)");
  }
  if (rc == DS3_OK)
    rc = check_hip(hipMalloc(&P->seg_count, sizeof(int32_t) * std::max(P->T.total_tiles, 1)), "hipMalloc");
  P->reserved_tiles = P->T.total_tiles;
  if (rc != DS3_OK) { plan_free(P); return rc; }
  carve_gn(P->ws, P->T, P->B);
  P->arena = arena;
  P->idx = idx;
  P->poses = poses;
  P->dt = dtype;
  P->p = *params;
  P->p.K = nullptr;  // the caller's intrinsics were copied into ecal; the plan keeps no host pointer
  P->c = make_gn_const(*params);
  P->use_graph = !opts || opts->use_graph != 0;
  P->timer = opts ? opts->reduce_timer : nullptr;
  rc = upload_topology(P->T, P->B, s);
  if (rc == DS3_OK) rc = plan_pick_solver(*P, opts ? opts->solver : 0);
  if (rc == DS3_OK) rc = launch_fill(P->B.H, 49 * size_t(P->T.n_kf) * size_t(P->T.n_kf), 0.0, s);
  if (rc == DS3_OK) rc = launch_fill_u32(P->B.counter, 64, 0u, s);
  if (rc == DS3_OK) rc = launch_fill_u32(P->hist_ctr, 4, 0u, s);
  if (rc == DS3_OK) {
    if (opts && opts->autotune) {
      rc = plan_autotune(*P, s);
    } else {
      int ppt = (opts && opts->px_per_thread > 0) ? opts->px_per_thread : 16;
      int unroll = (opts && opts->unroll > 0) ? opts->unroll : 2;
      if (ppt != 4 && ppt != 8 && ppt != 16 && ppt != 32 && ppt != 64)
        rc = fail(DS3_EINVAL, "px_per_thread must be 4, 8, 16, 32 or 64");
      if (unroll != 1 && unroll != 2 && unroll != 4) rc = fail(DS3_EINVAL, "unroll must be 1, 2 or 4");
      P->unroll = unroll;
      if (rc == DS3_OK) rc = plan_build_items(*P, ppt, s);
    }
  }
  if (rc == DS3_OK) {
    P->px_scanned = 0;
    for (auto& E : P->T.edges) P->px_scanned += E.npx_j;
  }
  if (rc == DS3_OK && P->use_graph) {
    // one iteration, and kGraphChunk iterations back to back: a replayed graph pays a launch gap of about
    // 8 us before its first kernel, so runs replay the chunk graph as often as they can
    hipStream_t cs;
    rc = check_hip(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
    if (rc == DS3_OK) {
      for (int reps : {1, kGraphChunk}) {
        if (rc != DS3_OK) break;
        rc = check_hip(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        if (rc != DS3_OK) break;
        int rc2 = DS3_OK;
        for (int r = 0; r < reps && rc2 == DS3_OK; ++r) rc2 = plan_iteration(*P, cs, false);
        hipGraph_t g = nullptr;
        int rc3 = check_hip(hipStreamEndCapture(cs, &g), "hipStreamEndCapture");
        rc = rc2 != DS3_OK ? rc2 : rc3;
        hipGraph_t& gp = reps == 1 ? P->graph : P->graph_chunk;
        hipGraphExec_t& ep = reps == 1 ? P->exec : P->exec_chunk;
        gp = g;
        if (rc == DS3_OK) rc = check_hip(hipGraphInstantiate(&ep, gp, nullptr, nullptr, 0), "hipGraphInstantiate");
      }
      (void)hipStreamDestroy(cs);
    }
  }
  if (rc != DS3_OK) { plan_free(P); return rc; }
  *plan_out = P;
  return DS3_OK;
}

int ds3_gn_plan_run(void* plan, int32_t iters, double* cost_per_iter, int32_t* status_per_iter,
                    void* stream) {
  Plan* P = static_cast<Plan*>(plan);
  if (!P || iters < 0) return fail(DS3_EINVAL, "plan_run: bad arguments");
  if (iters > kHistory) return fail(DS3_EINVAL, "plan_run: at most 4096 iterations per call");
  hipStream_t s = S(stream);
  DS3_TRY(launch_fill_u32(P->hist_ctr, 1, 0u, s));
  // with a timer, the last iteration runs as direct launches so that the events bracket its residual
  // launch (event records are not captured into the graph)
  const int replayed = P->use_graph ? iters - (P->timer && iters > 0 ? 1 : 0) : 0;
  int it = 0;
  for (; it + kGraphChunk <= replayed; it += kGraphChunk) DS3_TRY_HIP(hipGraphLaunch(P->exec_chunk, s));
  for (; it < replayed; ++it) DS3_TRY_HIP(hipGraphLaunch(P->exec, s));
  for (; it < iters; ++it) DS3_TRY(plan_iteration(*P, s, P->timer && it == iters - 1));
  if (iters > 0 && cost_per_iter)
    DS3_TRY_HIP(hipMemcpyAsync(cost_per_iter, P->cost_hist, sizeof(double) * iters, hipMemcpyDeviceToDevice, s));
  if (iters > 0 && status_per_iter)
    DS3_TRY_HIP(hipMemcpyAsync(status_per_iter, P->status_hist, sizeof(int32_t) * iters, hipMemcpyDeviceToDevice, s));
  return DS3_OK;
}

int ds3_gn_plan_time_reduce(void* plan, int32_t reps, float* ms_out, void* stream) {
  Plan* P = static_cast<Plan*>(plan);
  if (!P || reps < 1 || reps > 64 || !ms_out) return fail(DS3_EINVAL, "plan_time_reduce: bad arguments");
  return plan_time_reduce(*P, reps, ms_out, S(stream));
}

int ds3_gn_plan_info(void* plan, int64_t* info, int32_t n_info) {
  Plan* P = static_cast<Plan*>(plan);
  if (!P || !info || n_info < 0) return fail(DS3_EINVAL, "plan_info: bad arguments");
  const int64_t px_bytes = P->dt == DS3_F32 ? 16 : 8;
  const int64_t rec = int64_t(stream_record_bytes(P->dt, P->ecal != nullptr));
  int64_t sp[7] = {0, 0, 0, 0, 0, 0, 0};
  int64_t solver = 1, blocks = 0, levels = 0;
  if (P->sp) {
    spchol_stats(P->sp, sp);
    solver = 2, blocks = sp[1], levels = sp[3];
  } else if (P->tc) {
    tilechol_stats(P->tc, sp);
    solver = 3, blocks = sp[2], levels = sp[3];
  }
  const int64_t v[11] = {P->n_items, P->ppt, P->px_scanned, P->px_valid,
                         4 * P->px_scanned + 2 * px_bytes * P->px_valid,
                         rec * P->n_records + 4 * int64_t(P->n_items),
                         4 * P->px_scanned + 2 * px_bytes * P->px_valid + rec * P->n_records + 4 * int64_t(P->n_items),
                         P->unroll, solver, blocks, levels};
  for (int k = 0; k < n_info && k < 11; ++k) info[k] = v[k];
  return DS3_OK;
}

int ds3_gn_plan_refresh(void* plan, void* stream) {
  Plan* P = static_cast<Plan*>(plan);
  if (!P) return fail(DS3_EINVAL, "plan_refresh: null plan");
  return launch_gather_stream(P->dt, P->arena, P->B.edges, P->items, P->n_items, P->idx, P->T.tile_px, P->stream,
                              P->seg_count, S(stream), P->ecal);
}

int ds3_tune_cache_reset(void) {
  const std::string dir = tune_cache_dir();
  if (!dir.empty()) make_dirs(dir);
  const std::string path = tune_cache_path();
  if (std::remove(path.c_str()) != 0 && errno != ENOENT) return fail(DS3_EINVAL, "tune cache: cannot remove " + path);
  return DS3_OK;
}

int ds3_gn_plan_set_timer(void* plan, ds3_timer* timer) {
  Plan* P = static_cast<Plan*>(plan);
  if (!P) return fail(DS3_EINVAL, "plan_set_timer: null plan");
  P->timer = timer;
  return DS3_OK;
}

int ds3_gn_plan_destroy(void* plan) {
  plan_free(static_cast<Plan*>(plan));
  return DS3_OK;
}

// ---- cost + adjoint plan over a graph with fixed matches ----------------------------------------------
struct AdjPlan {
  Topology T;
  void* ws = nullptr;
  EdgeDev* edges = nullptr;
  EdgeXf* xf = nullptr;
  double *Ad = nullptr, *b_e = nullptr, *cost_e = nullptr;
  int64_t* count_e = nullptr;
  int64_t* kf_off = nullptr;
  int32_t *kf_npx = nullptr, *node_ptr = nullptr, *node_adj = nullptr;
  float* part7 = nullptr;
  int64_t *obase = nullptr, *sbase = nullptr, *cbase = nullptr;
  int32_t *inv_off = nullptr, *inv_src = nullptr, *inv_head = nullptr;
  const void* arena = nullptr;
  const int32_t* idx = nullptr;
  ds3_dtype dt = DS3_F32;
  GnConst c;
  int max_npx_j = 0, max_npx_kf = 0;
};

static size_t carve_adj(void* base, const Topology& T, AdjPlan& A, size_t off_len, size_t src_len,
                        size_t cnt_len) {
  Carver c(base);
  const int E = std::max(T.n_edges, 1);
  A.edges = c.take<EdgeDev>(E);
  A.xf = c.take<EdgeXf>(E);
  A.Ad = c.take<double>(49 * size_t(E));
  A.b_e = c.take<double>(7 * size_t(E));
  A.cost_e = c.take<double>(E);
  A.count_e = c.take<int64_t>(E);
  A.kf_off = c.take<int64_t>(T.n_kf);
  A.kf_npx = c.take<int32_t>(T.n_kf);
  A.node_ptr = c.take<int32_t>(T.n_kf + 1);
  A.node_adj = c.take<int32_t>(2 * size_t(E));
  A.part7 = c.take<float>(size_t(std::max(adjoint_part_floats(T.n_edges, max_npx_j(T)), 8)));
  A.obase = c.take<int64_t>(E);
  A.sbase = c.take<int64_t>(E);
  A.cbase = c.take<int64_t>(E);
  A.inv_off = c.take<int32_t>(std::max<size_t>(off_len, 1));
  A.inv_src = c.take<int32_t>(std::max<size_t>(src_len, 1));
  A.inv_head = c.take<int32_t>(std::max<size_t>(cnt_len, 1));
  return c.used;
}

static void adj_plan_free(AdjPlan* A) {
  if (!A) return;
  if (A->ws) (void)hipFree(A->ws);
  delete A;
}

int ds3_adjoint_plan_create(int32_t n_kf, const ds3_image* kf, const void* arena, ds3_dtype dtype,
                            const ds3_edge* edges, int32_t n_edges, const int32_t* idx,
                            const ds3_gn_params* params, void** plan_out, void* stream) {
  if (!plan_out) return fail(DS3_EINVAL, "plan_out is null");
  *plan_out = nullptr;
  static const double kNotPoses = 0.0;  // the plan takes its poses at run time
  DS3_TRY(check_gn_args(&kNotPoses, arena, idx, dtype, params));
  DS3_TRY(no_calibrated(params, "adjoint_plan"));
  DS3_TRY(check_arch());
  hipStream_t s = S(stream);
  AdjPlan* A = new AdjPlan();
  int rc = build_topology(n_kf, kf, n_edges, edges, nullptr, 0, kReduceThreads * kPlainPPT, A->T);
  if (rc != DS3_OK) { adj_plan_free(A); return rc; }
  const Topology& T = A->T;
  std::vector<int64_t> cbase(std::max(T.n_edges, 1), 0), obase(std::max(T.n_edges, 1), 0),
      sbase(std::max(T.n_edges, 1), 0);
  size_t cnt_len = 0, off_len = 0, src_len = 0;
  int max_npx_i = 0;
  for (int e = 0; e < T.n_edges; ++e) {
    cbase[e] = int64_t(cnt_len);
    obase[e] = int64_t(off_len);
    sbase[e] = int64_t(src_len);
    cnt_len += size_t(T.edges[e].npx_i);
    off_len += size_t(T.edges[e].npx_i) + 1;
    src_len += size_t(T.edges[e].npx_j);
    max_npx_i = std::max(max_npx_i, int(T.edges[e].npx_i));
  }
  const size_t ws = carve_adj(nullptr, T, *A, off_len, src_len, cnt_len);
  rc = check_hip(hipMalloc(&A->ws, ws), "hipMalloc(adjoint plan)");
  if (rc != DS3_OK) { adj_plan_free(A); return rc; }
  carve_adj(A->ws, T, *A, off_len, src_len, cnt_len);
  A->arena = arena;
  A->idx = idx;
  A->dt = dtype;
  A->c = make_gn_const(*params);
  A->max_npx_j = max_npx_j(T);
  A->max_npx_kf = *std::max_element(T.kf_npx.begin(), T.kf_npx.end());
  // the counts live in a temporary allocation
  void* tmp = nullptr;
  Carver tc(nullptr);
  tc.take<int32_t>(std::max<size_t>(cnt_len, 1));
  rc = check_hip(hipMalloc(&tmp, tc.used), "hipMalloc(adjoint plan build)");
  if (rc != DS3_OK) { adj_plan_free(A); return rc; }
  Carver tcc(tmp);
  int32_t* d_cnt = tcc.take<int32_t>(std::max<size_t>(cnt_len, 1));
  rc = upload(A->edges, T.edges, s);
  if (rc == DS3_OK) rc = upload(A->kf_off, T.kf_off, s);
  if (rc == DS3_OK) rc = upload(A->kf_npx, T.kf_npx, s);
  if (rc == DS3_OK) rc = upload(A->node_ptr, T.node_ptr, s);
  if (rc == DS3_OK) rc = upload(A->node_adj, T.node_adj, s);
  if (rc == DS3_OK) rc = upload(A->obase, obase, s);
  if (rc == DS3_OK) rc = upload(A->sbase, sbase, s);
  if (rc == DS3_OK) rc = upload(A->cbase, cbase, s);
  if (rc == DS3_OK)
    rc = launch_inverse_maps(A->edges, T.n_edges, A->max_npx_j, max_npx_i, idx, A->cbase, A->obase, A->sbase,
                             d_cnt, cnt_len, A->inv_off, A->inv_src, A->inv_head, s);
  const int rs = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize(adjoint plan build)");
  (void)hipFree(tmp);
  if (rc == DS3_OK) rc = rs;
  if (rc != DS3_OK) { adj_plan_free(A); return rc; }
  *plan_out = A;
  return DS3_OK;
}

int ds3_adjoint_plan_run(void* plan, const double* poses, float dcost, float* grad_xyz, float* grad_conf,
                         double* grad_tau, double* cost_out, ds3_timer* timer, void* stream) {
  AdjPlan* A = static_cast<AdjPlan*>(plan);
  if (!A || !poses || !grad_xyz || !grad_conf || !grad_tau) return fail(DS3_EINVAL, "null pointer");
  hipStream_t s = S(stream);
  const Topology& T = A->T;
  DS3_TRY(launch_gn_prep(poses, A->edges, T.n_edges, A->xf, A->Ad, s));
  DS3_TRY(launch_adjoint_gather(A->dt, A->arena, A->edges, T.n_edges, A->max_npx_j, A->max_npx_kf, A->xf, A->Ad,
                                A->idx, A->c, dcost, grad_xyz, grad_conf, A->part7, A->b_e, A->cost_e,
                                A->count_e, T.n_kf, A->kf_off, A->kf_npx, A->node_ptr, A->node_adj, A->obase,
                                A->sbase, A->cbase, A->inv_off, A->inv_src, A->inv_head, grad_tau, timer, s));
  if (cost_out) DS3_TRY(launch_sum_costs(A->cost_e, A->count_e, T.n_edges, cost_out, nullptr, s));
  return DS3_OK;
}

int ds3_adjoint_plan_destroy(void* plan) {
  adj_plan_free(static_cast<AdjPlan*>(plan));
  return DS3_OK;
}

}  // extern "C"
