// Ray-range tracking (Sec. III-A): each of n independent problems estimates the pose T_kf of a frame f
// relative to a keyframe k by minimising E_track(T_kf), the component-wise Huber cost of the whitened
// residual of eq. (1) over the frame-to-keyframe matches, with Levenberg-Marquardt damping (the tracker's
// form of eq. 7: (H + lambda diag H + eps_r I) tau = -g, T <- Exp(tau) T).
//
// Execution: the matches of every problem are gathered once into a match stream (the batched graph
// step's records: X_f[n], X_k[m], (C_k C_f)^(1/4)); then 1 + max_trials rounds of two launches run with
// no host synchronisation: the stream reduction at every problem's trial pose (the graph step's
// residual / Jacobian / Huber / Hessian kernel, one edge per problem with the keyframe at the identity,
// so H = H_L and g = b_L), and k_track_step, one block per problem, which sums the segment partials in
// a fixed order, takes the LM decision, solves the damped 7x7 system and writes the next trial pose.
// Problems that have stopped are skipped by both launches.
//
// The accept test compares E_track at two nearby poses. Near the optimum their difference falls below
// what a float32 evaluation resolves (each whitened ray residual is a difference of unit vectors over
// sigma_r = 0.003, so float32 rounding alone moves a pixel's cost by ~1e-4, and a 3k-pixel sum by ~1e-3
// while the true decrease per step reaches 1e-8): a float32 test rejects good steps there, inflates the
// damping and stops short of the optimum. The reduction therefore also evaluates each segment's cost in
// float64 (from the stored values and the float64 trial pose), and only that cost enters the decision;
// H and g stay float32.
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "sim3.hpp"

namespace ds3 {

struct TrackState {
  double T[8];    // kept pose
  double Tt[8];   // trial pose the last reduction evaluated
  double tau[7];  // the step that produced Tt
  double H[28];   // upper triangle of H at T (row-major pairs r <= c)
  double b[7];
  double E;       // E_track at T
  double lam;
  int32_t trials, status, count, pad;
};

size_t track_state_bytes() { return sizeof(TrackState); }

__device__ inline int hidx(int r, int c) { return r * 7 - (r * (r - 1)) / 2 + (c - r); }

// (H + lam diag H + eps_r I) tau = -b by Cholesky with the epsilon ladder; returns the attempt used or -1
// (tau = 0) when every attempt fails (a non-positive or non-finite pivot).
__device__ int solve7(const double* H, const double* b, double lam, double eps0, double mult, int attempts,
                      double* tau) {
  double eps = eps0;
  for (int r = 0; r < attempts; ++r, eps *= mult) {
    double L[49];
    for (int i = 0; i < 7; ++i)
      for (int j = 0; j <= i; ++j) L[7 * i + j] = H[hidx(j, i)];
    for (int i = 0; i < 7; ++i) L[8 * i] += lam * H[hidx(i, i)] + eps;
    bool ok = true;
    for (int j = 0; j < 7 && ok; ++j) {
      double d = L[8 * j];
      for (int k = 0; k < j; ++k) d -= L[7 * j + k] * L[7 * j + k];
      if (!(d > 0.0) || !isfinite(d)) {
        ok = false;
        break;
      }
      const double ljj = sqrt(d);
      L[8 * j] = ljj;
      for (int i = j + 1; i < 7; ++i) {
        double v = L[7 * i + j];
        for (int k = 0; k < j; ++k) v -= L[7 * i + k] * L[7 * j + k];
        L[7 * i + j] = v / ljj;
      }
    }
    if (!ok) continue;
    double y[7];
    for (int i = 0; i < 7; ++i) {
      double v = -b[i];
      for (int k = 0; k < i; ++k) v -= L[7 * i + k] * y[k];
      y[i] = v / L[8 * i];
    }
    for (int i = 6; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < 7; ++k) v -= L[7 * k + i] * tau[k];
      tau[i] = v / L[8 * i];
    }
    return r;
  }
  for (int i = 0; i < 7; ++i) tau[i] = 0.0;
  return -1;
}

// The trial transform for the next reduction: float32 (H, g) and float64 (the cost of the accept test).
__device__ inline void write_xf(const Sim3& T, EdgeXf* xf, double* xf64) {
  double R[9];
  quat_to_mat(T.q, R);
  EdgeXf X;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) {
      xf64[3 * r + c] = T.s * R[3 * r + c];
      X.m[3 * r + c] = float(T.s * R[3 * r + c]);
    }
    xf64[9 + r] = T.t[r];
    X.m[9 + r] = float(T.t[r]);
  }
  for (int k = 0; k < 4; ++k) X.pad[k] = 0.0f;
  *xf = X;
}

// phase 0: the partials hold the sums at the initial poses (T_io); later phases: at the trial poses.
__global__ __launch_bounds__(64) void k_track_step(const EdgeDev* __restrict__ edges,
                                                   const float* __restrict__ partials,
                                                   const double* __restrict__ cost64,
                                                   TrackState* __restrict__ states, int32_t* __restrict__ done,
                                                   EdgeXf* __restrict__ xf, double* __restrict__ xf64,
                                                   double* __restrict__ T_io,
                                                   double* __restrict__ cost_out, int32_t* __restrict__ trials_out,
                                                   int32_t* __restrict__ status_out, TrackConst tc, int phase) {
  const int p = blockIdx.x;
  const int t = threadIdx.x;
  if (phase > 0 && done[p]) return;
  __shared__ double S[37];
  __shared__ double Ecost;
  const EdgeDev E = edges[p];
  if (t == 63) {  // the float64 cost, summed over the segments in order
    double s = 0.0;
    for (int k = 0; k < E.n_tiles; ++k) s += cost64[E.tile0 + k];
    Ecost = s;
  }
  if (t < 37) {
    double s = 0.0;
    const float* q = partials + int64_t(E.tile0) * kPartial + t;
    int k = 0;
    for (; k + 8 <= E.n_tiles; k += 8) {  // eight loads in flight, summed in segment order
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = q[int64_t(k + u) * kPartial];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += double(v[u]);
    }
    for (; k < E.n_tiles; ++k) s += double(q[int64_t(k) * kPartial]);
    S[t] = s;
  }
  __syncthreads();
  if (t != 0) return;
  TrackState& st = states[p];
  bool stop = false;
  if (phase == 0) {
    for (int k = 0; k < 8; ++k) st.T[k] = T_io[8 * int64_t(p) + k];
    for (int k = 0; k < 28; ++k) st.H[k] = S[k];
    for (int k = 0; k < 7; ++k) st.b[k] = S[28 + k];
    st.E = Ecost;
    st.count = int32_t(S[36] + 0.5);
    st.lam = tc.lambda0;
    st.trials = 0;
    st.status = 0;
  } else {
    st.trials += 1;
    if (Ecost < st.E) {  // accept: keep the trial pose and its linearisation
      for (int k = 0; k < 8; ++k) st.T[k] = st.Tt[k];
      for (int k = 0; k < 28; ++k) st.H[k] = S[k];
      for (int k = 0; k < 7; ++k) st.b[k] = S[28 + k];
      st.E = Ecost;
      st.count = int32_t(S[36] + 0.5);
      st.lam = fmax(st.lam * tc.lambda_down, tc.lambda_min);
      double m = 0.0;
      for (int k = 0; k < 7; ++k) m = fmax(m, fabs(st.tau[k]));
      if (m < tc.step_tol) stop = true;
    } else {
      st.lam *= tc.lambda_up;
    }
    if (st.trials >= tc.max_trials) stop = true;
  }
  if (!stop) {
    st.status = solve7(st.H, st.b, st.lam, tc.eps0, tc.eps_mult, tc.attempts, st.tau);
    const Sim3 Tt = sim3_mul(sim3_exp(st.tau), sim3_load(st.T));
    Sim3 Tn = Tt;
    quat_normalize(Tn.q);
    sim3_store(Tn, st.Tt);
    write_xf(Tn, xf + p, xf64 + 12 * int64_t(p));
  } else {
    done[p] = 1;
  }
  for (int k = 0; k < 8; ++k) T_io[8 * int64_t(p) + k] = st.T[k];
  cost_out[p] = st.E;
  trials_out[p] = st.trials;
  if (status_out) status_out[p] = st.status;
}

// Initial transform of every problem (float32 and float64 copies of T_io) for the phase-0 reduction.
__global__ void k_track_init(const double* __restrict__ T_io, int n, EdgeXf* __restrict__ xf,
                             double* __restrict__ xf64, int32_t* __restrict__ done) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  Sim3 T = sim3_load(T_io + 8 * int64_t(p));
  quat_normalize(T.q);
  write_xf(T, xf + p, xf64 + 12 * int64_t(p));
  done[p] = 0;
}

int launch_track_init(const double* T_io, int n, EdgeXf* xf, double* xf64, int32_t* done, hipStream_t s) {
  if (n <= 0) return DS3_OK;
  hipLaunchKernelGGL(k_track_init, dim3((n + 63) / 64), dim3(64), 0, s, T_io, n, xf, xf64, done);
  return check_hip(hipGetLastError(), "k_track_init");
}

int launch_track_step(const EdgeDev* edges, int n, const float* partials, const double* cost64, void* states,
                      int32_t* done, EdgeXf* xf, double* xf64, double* T_io, double* cost_out, int32_t* trials_out,
                      int32_t* status_out, TrackConst tc, int phase, hipStream_t s) {
  if (n <= 0) return DS3_OK;
  hipLaunchKernelGGL(k_track_step, dim3(n), dim3(64), 0, s, edges, partials, cost64,
                     static_cast<TrackState*>(states), done, xf, xf64, T_io, cost_out, trials_out, status_out, tc,
                     phase);
  return check_hip(hipGetLastError(), "k_track_step");
}

}  // namespace ds3

// ------------------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------------------
namespace ds3 {

constexpr int kTrackPPT = 16;  // segment = 4096 frame pixels

struct TrackBuffers {
  EdgeDev* edges;
  WorkItem* items;
  EdgeXf* xf;
  double* xf64;
  float* partials;
  double* cost64;
  void* stream;
  int32_t* seg_count;
  void* states;
  int32_t* done;
};

static int track_topology(int n, const ds3_track_problem* probs, std::vector<EdgeDev>& edges,
                          std::vector<WorkItem>& items) {
  if (n < 0 || (n > 0 && !probs)) return fail(DS3_EINVAL, "track: bad problem table");
  const int seg = kReduceThreads * kTrackPPT;
  edges.resize(n);
  items.clear();
  int64_t tiles = 0;
  for (int p = 0; p < n; ++p) {
    const ds3_track_problem& q = probs[p];
    const ds3_image& K = q.keyframe;
    const ds3_image& F = q.frame;
    if (K.H <= 0 || K.W <= 0 || F.H <= 0 || F.W <= 0 || K.px_offset < 0 || F.px_offset < 0 || q.idx_offset < 0 ||
        int64_t(K.H) * K.W > INT32_MAX || int64_t(F.H) * F.W > INT32_MAX)
      return fail(DS3_EINVAL, "track: bad problem " + std::to_string(p));
    EdgeDev D;
    D.off_i = K.px_offset;
    D.off_j = F.px_offset;
    D.idx_off = q.idx_offset;
    D.npx_i = K.H * K.W;
    D.npx_j = F.H * F.W;
    D.i = 0;
    D.j = 0;
    D.tile0 = int32_t(tiles);
    D.n_tiles = (D.npx_j + seg - 1) / seg;
    for (int t = 0; t < D.n_tiles; ++t) items.push_back(WorkItem{p, t});
    tiles += D.n_tiles;
    if (tiles > INT32_MAX / seg) return fail(DS3_EINVAL, "track: too many frame pixels for one call");
    edges[p] = D;
  }
  return DS3_OK;
}

static size_t carve_track(void* base, int n, int tiles, ds3_dtype dt, TrackBuffers& B) {
  Carver c(base);
  const size_t seg = size_t(kReduceThreads) * kTrackPPT;
  B.edges = c.take<EdgeDev>(std::max(n, 1));
  B.items = c.take<WorkItem>(std::max(tiles, 1));
  B.xf = c.take<EdgeXf>(std::max(n, 1));
  B.xf64 = c.take<double>(size_t(std::max(n, 1)) * 12);
  B.partials = c.take<float>(size_t(std::max(tiles, 1)) * kPartial);
  B.cost64 = c.take<double>(std::max(tiles, 1));
  B.stream = c.take<char>(size_t(std::max(tiles, 1)) * seg * stream_record_bytes(dt));
  B.seg_count = c.take<int32_t>(std::max(tiles, 1));
  B.states = c.take<char>(size_t(std::max(n, 1)) * track_state_bytes());
  B.done = c.take<int32_t>(std::max(n, 1));
  return c.used;
}

// Static scratch of ds3_track_noalloc: a file-scope device array, one copy per GPU, held until the
// process ends. Host code reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's own name is a host-side stand-in, not a device address).
constexpr size_t kTrackScratchBytes = size_t(DS3_TRACK_SCRATCH_BYTES);
static __device__ __align__(256) char scratch[kTrackScratchBytes];

static int track_scratch(void** out) {
  static std::mutex mu;
  static std::vector<void*> addr;
  int dev = 0;
  DS3_TRY_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if (int(addr.size()) <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    DS3_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    addr[dev] = p;
  }
  *out = addr[dev];
  return DS3_OK;
}

static int track_impl(const void* arena, ds3_dtype dtype, const ds3_track_problem* probs, int32_t n,
                      const int32_t* idx_arena, const ds3_gn_params* gn, const ds3_track_params* tp, double* T,
                      double* cost_out, int32_t* trials_out, int32_t* status_out, ds3_timer* reduce_timer,
                      void* workspace, size_t ws_bytes, void* stream) {
  if (n < 0) return fail(DS3_EINVAL, "track: n < 0");
  if (n == 0) return DS3_OK;
  if (!arena || !idx_arena || !gn || !tp || !T || !cost_out || !trials_out || !workspace)
    return fail(DS3_EINVAL, "track: null pointer");
  if (dtype != DS3_F32 && dtype != DS3_BF16) return fail(DS3_ENOTSUP, "track: dtype");
  if ((reinterpret_cast<uintptr_t>(arena) & 15) != 0) return fail(DS3_EINVAL, "track: arena must be 16 B aligned");
  if (!(gn->sigma_ray > 0) || !(gn->sigma_dist > 0) || !(gn->huber_k > 0) || gn->max_attempts < 1 ||
      gn->max_attempts > 16)
    return fail(DS3_EINVAL, "track: bad graph-step constants");
  if (gn->K) return fail(DS3_ENOTSUP, "track: no calibrated mode (K must be NULL)");
  if (tp->max_trials < 0 || tp->max_trials > 1000 || !(tp->lambda0 >= 0) || !(tp->lambda_up >= 1) ||
      !(tp->lambda_down > 0) || !(tp->lambda_down <= 1) || !(tp->lambda_min >= 0) || !(tp->step_tol >= 0))
    return fail(DS3_EINVAL, "track: bad LM schedule");
  std::vector<EdgeDev> edges;
  std::vector<WorkItem> items;
  DS3_TRY(track_topology(n, probs, edges, items));
  const int tiles = int(items.size());
  TrackBuffers B;
  if (ws_bytes < carve_track(nullptr, n, tiles, dtype, B)) return fail(DS3_ENOSPACE, "track: workspace too small");
  carve_track(workspace, n, tiles, dtype, B);
  hipStream_t s = static_cast<hipStream_t>(stream);
  DS3_TRY_HIP(hipMemcpyAsync(B.edges, edges.data(), sizeof(EdgeDev) * n, hipMemcpyHostToDevice, s));
  DS3_TRY_HIP(hipMemcpyAsync(B.items, items.data(), sizeof(WorkItem) * tiles, hipMemcpyHostToDevice, s));
  const int seg = kReduceThreads * kTrackPPT;
  const GnConst c = make_gn_const(*gn);
  TrackConst tc;
  tc.lambda0 = tp->lambda0;
  tc.lambda_min = tp->lambda_min;
  tc.lambda_up = tp->lambda_up;
  tc.lambda_down = tp->lambda_down;
  tc.step_tol = tp->step_tol;
  tc.eps0 = gn->eps0;
  tc.eps_mult = gn->eps_mult;
  tc.max_trials = tp->max_trials;
  tc.attempts = gn->max_attempts;
  DS3_TRY(launch_gather_stream(dtype, arena, B.edges, B.items, tiles, idx_arena, seg, B.stream, B.seg_count, s));
  DS3_TRY(launch_track_init(T, n, B.xf, B.xf64, B.done, s));
  for (int phase = 0; phase <= tp->max_trials; ++phase) {
    const bool timed = reduce_timer && phase == 0;
    if (timed) DS3_TRY(timer_record(reduce_timer, true, s));
    DS3_TRY(launch_reduce_stream(dtype, 2, B.stream, B.seg_count, B.edges, B.items, tiles, B.xf, seg, B.partials,
                                 c, B.done, s, B.xf64, B.cost64));
    if (timed) DS3_TRY(timer_record(reduce_timer, false, s));
    DS3_TRY(launch_track_step(B.edges, n, B.partials, B.cost64, B.states, B.done, B.xf, B.xf64, T, cost_out,
                              trials_out, status_out, tc, phase, s));
  }
  return DS3_OK;
}


}  // namespace ds3

using namespace ds3;

extern "C" {

void ds3_default_track_params(ds3_track_params* p) {
  if (!p) return;
  p->lambda0 = 1e-4;
  p->lambda_min = 1e-9;
  p->lambda_up = 10.0;
  p->lambda_down = 0.1;
  p->max_trials = 20;
  p->step_tol = 1e-7;
}

size_t ds3_track_workspace_bytes(int32_t n, const ds3_track_problem* probs, ds3_dtype dtype) {
  std::vector<EdgeDev> edges;
  std::vector<WorkItem> items;
  if (n <= 0 || track_topology(n, probs, edges, items) != DS3_OK) return 0;
  TrackBuffers B;
  return carve_track(nullptr, n, int(items.size()), dtype, B);
}

int ds3_track(const void* arena, ds3_dtype dtype, const ds3_track_problem* probs, int32_t n,
              const int32_t* idx_arena, const ds3_gn_params* gn, const ds3_track_params* tp, double* T,
              double* cost_out, int32_t* trials_out, int32_t* status_out, ds3_timer* reduce_timer,
              void* workspace, size_t ws_bytes, void* stream) {
  return track_impl(arena, dtype, probs, n, idx_arena, gn, tp, T, cost_out, trials_out, status_out, reduce_timer,
                    workspace, ws_bytes, stream);
}

int ds3_track_noalloc(const void* arena, ds3_dtype dtype, const ds3_track_problem* probs, int32_t n,
                      const int32_t* idx_arena, const ds3_gn_params* gn, const ds3_track_params* tp, double* T,
                      double* cost_out, int32_t* trials_out, int32_t* status_out, void* stream) {
  if (n < 0) return fail(DS3_EINVAL, "track_noalloc: n < 0");
  if (n == 0) return DS3_OK;
  std::vector<EdgeDev> edges;
  std::vector<WorkItem> items;
  DS3_TRY(track_topology(n, probs, edges, items));
  TrackBuffers B;
  const size_t need = carve_track(nullptr, n, int(items.size()), dtype, B);
  if (need > kTrackScratchBytes)
    return fail(DS3_ENOSPACE, "track_noalloc: these problems need " + std::to_string(need) +
                                  " bytes of scratch; the static scratch holds " +
                                  std::to_string(kTrackScratchBytes) + " (DS3_TRACK_SCRATCH_BYTES)");
  void* ws = nullptr;
  DS3_TRY(track_scratch(&ws));
  return track_impl(arena, dtype, probs, n, idx_arena, gn, tp, T, cost_out, trials_out, status_out, nullptr, ws,
                    kTrackScratchBytes, stream);
}

}  // extern "C"
