// Canonical pointmap fusion of eq. (2) (Sec. III-A): the confidence-weighted running average that folds
// registered point predictions into the keyframes' canonical pointmaps, one launch over every
// (keyframe, frame) pair. A streaming kernel: 16 B read from each arena and 16 B written per pixel.
#include <algorithm>
#include <climits>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "sim3.hpp"

namespace ds3 {

struct FusePairDev {
  int64_t canon_off, pred_off, n_px;
  int32_t tile0;  // first block of the pair
  int32_t pad;
};

constexpr int kFuseThreads = 256;
constexpr int kFusePpt = 8;                         // pixels per thread, strided by the block size
constexpr int kFuseTile = kFuseThreads * kFusePpt;  // pixels per block

typedef float vf4 __attribute__((ext_vector_type(4)));

// Block b fuses pixels [t kFuseTile, (t + 1) kFuseTile) of the pair whose blocks hold b (pairs in tile0
// order). y = s R x + t and the weighted average are evaluated in float64 from the float32 inputs and
// rounded once; every load of a thread is issued before its arithmetic. Both arenas are touched once per
// launch, so loads and stores are non-temporal (0.28-0.30 ms against 0.31-0.32 ms per launch over the
// 34.4 Mpx of 200 keyframes with cached accesses).
__global__ __launch_bounds__(kFuseThreads) void k_fuse(vf4* __restrict__ canon, const vf4* __restrict__ pred,
                                                       const FusePairDev* __restrict__ pairs, int n_pairs,
                                                       const double* __restrict__ T) {
  const int b = blockIdx.x;
  int lo = 0, hi = n_pairs - 1;  // the last pair with tile0 <= b (uniform per block)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pairs[mid].tile0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const FusePairDev P = pairs[lo];
  const int64_t base = int64_t(b - P.tile0) * kFuseTile;
  vf4 c[kFusePpt], x[kFusePpt];
  bool in[kFusePpt];
#pragma unroll
  for (int u = 0; u < kFusePpt; ++u) {
    const int64_t m = base + u * kFuseThreads + threadIdx.x;
    in[u] = m < P.n_px;
    if (in[u]) {
      c[u] = __builtin_nontemporal_load(canon + P.canon_off + m);
      x[u] = __builtin_nontemporal_load(pred + P.pred_off + m);
    }
  }
  const Sim3 S = sim3_load(T + 8 * int64_t(lo));
  double R[9];
  quat_to_mat(S.q, R);
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] *= S.s;
#pragma unroll
  for (int u = 0; u < kFusePpt; ++u) {
    if (!in[u]) continue;
    const double c0 = c[u].w, c1 = x[u].w, tot = c0 + c1;
    if (!(finite3(x[u].x, x[u].y, x[u].z) && isfinite(x[u].w) && tot > 0.0)) continue;
    const double px = x[u].x, py = x[u].y, pz = x[u].z;
    const double yx = R[0] * px + R[1] * py + R[2] * pz + S.t[0];
    const double yy = R[3] * px + R[4] * py + R[5] * pz + S.t[1];
    const double yz = R[6] * px + R[7] * py + R[8] * pz + S.t[2];
    vf4 o;
    o.x = float((c0 * double(c[u].x) + c1 * yx) / tot);
    o.y = float((c0 * double(c[u].y) + c1 * yy) / tot);
    o.z = float((c0 * double(c[u].z) + c1 * yz) / tot);
    o.w = float(tot);
    __builtin_nontemporal_store(o, canon + P.canon_off + base + u * kFuseThreads + threadIdx.x);
  }
}

static size_t fuse_workspace(int n_pairs) {
  Carver c(nullptr);
  c.take<FusePairDev>(size_t(std::max(n_pairs, 1)));
  return c.used;
}

static hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

}  // namespace ds3

using namespace ds3;

extern "C" size_t ds3_fuse_workspace_bytes(int32_t n_pairs) { return n_pairs > 0 ? fuse_workspace(n_pairs) : 0; }

extern "C" int ds3_fuse(float* canon, int64_t n_canon_px, const float* pred, int64_t n_pred_px,
                        const ds3_fuse_pair* pairs, int32_t n_pairs, const double* T, int32_t n_T,
                        void* workspace, size_t ws_bytes, void* stream) {
  if (n_pairs < 0) return fail(DS3_EINVAL, "fuse: n_pairs < 0");
  if (n_pairs == 0) return DS3_OK;
  if (!canon || !pred || !pairs || !T || !workspace) return fail(DS3_EINVAL, "fuse: null pointer");
  if (n_canon_px < 0 || n_pred_px < 0) return fail(DS3_EINVAL, "fuse: negative arena size");
  if (n_T < n_pairs) return fail(DS3_EINVAL, "fuse: fewer poses than pairs");
  if ((reinterpret_cast<uintptr_t>(canon) | reinterpret_cast<uintptr_t>(pred)) & 15u)
    return fail(DS3_EINVAL, "fuse: arenas must be 16-byte aligned (float4 per pixel)");
  {
    // the canonical arena is written in place: it may not share memory with the prediction arena
    const uintptr_t c0 = reinterpret_cast<uintptr_t>(canon), c1 = c0 + 16u * uint64_t(n_canon_px);
    const uintptr_t p0 = reinterpret_cast<uintptr_t>(pred), p1 = p0 + 16u * uint64_t(n_pred_px);
    if (c0 < p1 && p0 < c1) return fail(DS3_EINVAL, "fuse: canonical and prediction arenas overlap");
  }
  if (ws_bytes < fuse_workspace(n_pairs)) return fail(DS3_ENOSPACE, "fuse: workspace too small");
  std::vector<FusePairDev> dev(n_pairs);
  int64_t tiles = 0;
  for (int p = 0; p < n_pairs; ++p) {
    const ds3_fuse_pair& q = pairs[p];
    if (q.n_px < 0 || q.canon_off < 0 || q.pred_off < 0) return fail(DS3_EINVAL, "fuse: negative offset or size");
    if (q.canon_off > n_canon_px - q.n_px || q.pred_off > n_pred_px - q.n_px)
      return fail(DS3_EINVAL, "fuse: pair " + std::to_string(p) + " reaches past the end of an arena");
    dev[p] = FusePairDev{q.canon_off, q.pred_off, q.n_px, int32_t(tiles), 0};
    tiles += (q.n_px + kFuseTile - 1) / kFuseTile;
    if (tiles > INT_MAX) return fail(DS3_EINVAL, "fuse: too many pixels for one call");
  }
  // pairs within one launch may not share canonical pixels
  std::vector<int> order(n_pairs);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return pairs[a].canon_off < pairs[b].canon_off; });
  int64_t end = -1;
  for (int k : order) {
    if (pairs[k].n_px == 0) continue;
    if (pairs[k].canon_off < end) return fail(DS3_EINVAL, "fuse: two pairs share canonical pixels");
    end = pairs[k].canon_off + pairs[k].n_px;
  }
  if (tiles == 0) return DS3_OK;
  FusePairDev* d_pairs = static_cast<FusePairDev*>(workspace);
  DS3_TRY_HIP(hipMemcpyAsync(d_pairs, dev.data(), sizeof(FusePairDev) * dev.size(), hipMemcpyHostToDevice, S(stream)));
  hipLaunchKernelGGL(k_fuse, dim3(unsigned(tiles)), dim3(kFuseThreads), 0, S(stream), reinterpret_cast<vf4*>(canon),
                     reinterpret_cast<const vf4*>(pred), d_pairs, n_pairs, T);
  return check_hip(hipGetLastError(), "k_fuse");
}
