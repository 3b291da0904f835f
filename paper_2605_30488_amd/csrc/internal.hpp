// Host-side declarations shared by the translation units of libds3 (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ds3.h"

struct ds3_timer {
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool recorded = false;
};

namespace ds3 {

// ---- error state -----------------------------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);
#define DS3_TRY_HIP(expr)                                        \
  do {                                                           \
    int _rc = ::ds3::check_hip((expr), #expr);                   \
    if (_rc != DS3_OK) return _rc;                               \
  } while (0)
#define DS3_TRY(expr)            \
  do {                           \
    int _rc = (expr);            \
    if (_rc != DS3_OK) return _rc; \
  } while (0)

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Records the begin (or end) event of a kernel timer on s; inside a stream capture the record becomes an
// event node of the graph. A null timer records nothing.
int timer_record(ds3_timer* t, bool begin, hipStream_t s);

// Carves aligned sub-buffers out of one workspace block (or only measures when base == nullptr).
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    size_t off = align_up(used);
    used = off + count * sizeof(T);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

// ---- graph-step device structures --------------------------------------------------------------------
// One edge as the kernels see it.
struct EdgeDev {
  int64_t off_i, off_j;  // arena pixel offsets of keyframes i and j
  int64_t idx_off;       // idx arena offset
  int32_t npx_i, npx_j;  // pixel counts
  int32_t i, j;          // keyframe ids
  int32_t tile0;         // first tile slot of the edge in the partial buffer
  int32_t n_tiles;
};

// Per-edge relative transform T_ij = T_i^-1 T_j in float32 (sR row-major, t) for the residual kernel.
struct EdgeXf {
  float m[12];
  float pad[4];
};

// Constants of the residual kernel.
struct GnConst {
  float inv_sr, inv_sd, inv_sr2, inv_sd2, kappa;
  double inv_sr_d, inv_sd_d, kappa_d;  // the same constants in float64 (float64 cost evaluation)
  float inv_sp, inv_sz, inv_sp2, inv_sz2;  // calibrated mode: 1/sigma_pix, 1/sigma_logz and their squares
};

// Residual of the graph step: the ray-range residual of eq. (1), or the calibrated mode's pixel
// reprojection and log-depth (Sec. IV-C).
enum ResidualMode { kRayRange = 0, kCalibrated = 1 };

// Per-edge intrinsics of the calibrated mode: K_i (projection into keyframe i), K_j^-1 (calibrated rays of
// keyframe j) and both image widths (pixel index -> (u, v)).
struct EdgeCal {
  float fxi, fyi, cxi, cyi;
  float ifxj, ifyj, cxj, cyj;
  int32_t Wi, Wj, Hi, pad;
};

// Host: per-edge EdgeCal from the supplied intrinsics (n_kf x 4) and the keyframe widths; checks that
// every focal length is positive and finite.
int make_edge_cal(const double* K, int n_kf, const int32_t* kf_w, const EdgeDev* edges, int n_edges,
                  EdgeCal* out);

constexpr int kPartial = 40;  // floats per tile partial: H upper 28, b 7, cost, count, 3 pad
constexpr int kReduceThreads = 256;

// One (edge, tile) work item of the batched form: a segment of the match stream.
struct WorkItem {
  int32_t edge;
  int32_t tile;
};

GnConst make_gn_const(const ds3_gn_params& p);

// Constants of the tracker's LM loop (track.hip).
struct TrackConst {
  double lambda0, lambda_min, lambda_up, lambda_down, step_tol, eps0, eps_mult;
  int32_t max_trials, attempts;
};

// gn.hip
int launch_gn_prep(const double* poses, const EdgeDev* edges, int n_edges, EdgeXf* xf, double* Ad,
                   hipStream_t s);
int launch_edge_reduce_one(ds3_dtype dt, int ppt, const void* arena, const EdgeDev& e, int edge_id,
                           const EdgeXf* xf, const int32_t* idx_arena, float* partials, GnConst c,
                           hipStream_t s, const EdgeCal* cal = nullptr);
// match stream of the batched form (gn.hip)
// Calibrated mode (ecal != NULL, device, one EdgeCal per edge): float32 records of the calibrated point
// and the target (u_m, v_m, 1/z_i[m]) whatever the arena dtype.
size_t stream_record_bytes(ds3_dtype dt, bool calibrated = false);
int launch_gather_stream(ds3_dtype dt, const void* arena, const EdgeDev* edges, const WorkItem* items,
                         int n_items, const int32_t* idx_arena, int seg_px, void* stream, int32_t* seg_count,
                         hipStream_t s, const EdgeCal* ecal = nullptr);
int launch_reduce_stream(ds3_dtype dt, int unroll, const void* stream, const int32_t* seg_count,
                         const EdgeDev* edges, const WorkItem* items, int n_items, const EdgeXf* xf, int seg_px,
                         float* partials, GnConst c, const int32_t* skip, hipStream_t s,
                         const double* xf64 = nullptr, double* cost64 = nullptr, const EdgeCal* ecal = nullptr);
int launch_edge_finalize(const EdgeDev* edges, int n_edges, const float* partials, const double* Ad,
                         double* A_out, double* b_out, double* cost_e, int64_t* count_e, hipStream_t s);
int launch_assemble(int n_kf, const int32_t* node_ptr, const int32_t* node_adj, const int32_t* pair_ptr,
                    const int32_t* pair_edges, const int32_t* pair_ij, int n_pairs, const double* A_e,
                    const double* b_e, const uint8_t* anchor_mask, double* H, double* g, hipStream_t s,
                    unsigned* zero = nullptr, int n_zero = 0);  // also clears zero[0 .. n_zero), n_zero <= 64
int launch_sum_costs(const double* cost_e, const int64_t* count_e, int n_edges, double* cost_out,
                     int64_t* count_out, hipStream_t s);
int launch_sim3_update(double* poses, const double* tau, const uint8_t* fixed, int n, hipStream_t s);
// T <- Exp(tau) T (as launch_sim3_update) and the sum of the edge costs with the ladder status appended to the
// history (the history counter is advanced), in one launch
int launch_update_record(double* poses, const double* tau, const uint8_t* fixed, int n, const double* cost_e,
                         const int64_t* count_e, int n_edges, double* cost_out, int64_t* count_out,
                         const int32_t* status, unsigned* ctr, double* cost_hist, int32_t* status_hist, int hist_len,
                         hipStream_t s);
int launch_fill(double* p, size_t n, double v, hipStream_t s);
int launch_fill_u32(unsigned* p, size_t n, unsigned v, hipStream_t s);
int launch_copy_f64(const double* src, double* dst, size_t n, hipStream_t s);
int launch_count_valid(const EdgeDev* edges, int n_edges, const int32_t* idx_arena, int tile_px,
                       int max_tiles, int32_t* counts, hipStream_t s);

// track.hip
size_t track_state_bytes();
int launch_track_init(const double* T_io, int n, EdgeXf* xf, double* xf64, int32_t* done, hipStream_t s);
int launch_track_step(const EdgeDev* edges, int n, const float* partials, const double* cost64, void* states,
                      int32_t* done, EdgeXf* xf, double* xf64, double* T_io, double* cost_out, int32_t* trials_out,
                      int32_t* status_out, TrackConst tc, int phase, hipStream_t s);

// chol.hip
size_t chol_workspace_bytes(int n);
int launch_chol_ladder(const double* H, const double* g, int n, double lambda, double eps0, double mult,
                       int attempts, double* tau, int32_t* status, void* ws, hipStream_t s);

// the dense workspace's synchronisation words ([2] error, [3] attempt 0 failed) and its persistent
// fallback alone (attempts 1.., run only when attempt 0 failed)
unsigned* chol_sync_words(void* ws, int n);
int launch_chol_fallback(const double* H, const double* g, int n, double lambda, double eps0, double mult,
                         int attempts, double* tau, int32_t* status, void* ws, hipStream_t s);

// spchol.hip: block-sparse ladder solve for a fixed keyframe-pair pattern, and the minimum-degree order
// both sparse solvers start from
int min_degree_order(int n, int n_pairs, const int32_t* pair_ij, std::vector<int>& order,
                     std::vector<std::vector<int>>& rows, std::vector<uint64_t>* pattern);
struct SpChol;
int spchol_create(int n_kf, int n_pairs, const int32_t* pair_ij, SpChol** out);
void spchol_destroy(SpChol* P);
void spchol_stats(const SpChol* P, int64_t* info);  // n_kf, blocks, fill blocks, levels, products, words
int launch_spchol(const SpChol* P, const double* H, const double* g, double lambda, double eps0, double mult,
                  int attempts, double* tau, int32_t* status, hipStream_t s);

// tilechol.hip: tile-sparse ladder solve for a fixed keyframe-pair pattern (attempt 0 over the tile
// elimination tree, the dense fallback after it in the dense workspace ws)
struct TileChol;
int tilechol_create(int n_kf, int n_pairs, const int32_t* pair_ij, TileChol** out);
void tilechol_destroy(TileChol* P);
void tilechol_stats(const TileChol* P, int64_t* info);  // n_kf, tiles, factor tiles, levels, updates, pad rows, thr
// sync_cleared: the first four words of ws's barrier block (chol_sync_words) were already cleared on stream s
// (by the plan's assembly), so the solve does not clear them itself
int launch_tilechol(const TileChol* P, const double* H, const double* g, double lambda, double eps0,
                    double mult, int attempts, double* tau, int32_t* status, void* ws, hipStream_t s,
                    bool sync_cleared = false);

// sim3.hip
int launch_sim3_exp(const double* tau, double* poses, int n, hipStream_t s);
int launch_sim3_log(const double* poses, double* tau, int n, hipStream_t s);

// pack / match / gauge / adjoint
int launch_pack(const float* xyz, const float* conf, int64_t n, ds3_dtype dt, void* out, hipStream_t s);
int device_cu_count();

}  // namespace ds3
