// Terminal segment-level depth refinement (Sec. III-E, eqs. (8)-(10)).
//
// Segmentation (once per plan): per keyframe, SLIC over canonical surface normals and normalised
// log-range, pixels with confidence below C_min excluded, segments with fewer than min_seg_px valid pixels
// excluded. Features are computed in float64 in a fixed operation order and quantised to integers, and the
// clustering runs in exact int64 arithmetic, so the labels do not depend on summation order:
//   F = (round(Q (n + 1)) x3, round(Q l)), Q = 1024; S = round(sqrt(HW / M_k)); one centre per grid cell;
//   D = S^2 |F_p - F_c|^2 + 512^2 |xy_p - xy_c|^2 over the centres of the 3x3 cells around the pixel's cell
//   (ties: lowest centre index); centres move to the floor of their members' mean; fixed iteration count.
// Centre updates gather their members from the 3x3 cells around their own (a pixel can only join a centre
// of an adjacent cell), so each centre's sums are formed by one block without atomics.
// Boundary table: for 4-adjacent pixels of two valid segments g != h of a keyframe, the log-range difference
// ln|X(p)| - ln|X(p')| (p in g) is summed into slot (g -> h) and its negative into (h -> g); h's grid cell is
// within 3 cells of g's, so each segment keeps 7 x 7 slots indexed by the cell offset. Sums are int64 fixed
// point (2^-40), so the table is independent of the order of the atomic adds.
//
// One refinement iteration (Jacobi-style damped Newton, eqs. 8-10):
//   data: for every match (m, n) of edge (i, j), X_j(eta) = X_j exp(eta_h), X_i(eta) = X_i exp(eta_g),
//     r = sqrt(q)/sigma_point (T_ij X_j(eta) - X_i(eta)), Huber weights w; the segments' diagonal
//     H += w |J|^2 and gradient g += w J.r with J_h = sqrt(q)/sigma (sR_ij X_j(eta)), J_g = -sqrt(q)/sigma
//     X_i(eta) -- one block per (edge, 4096-pixel tile of j) accumulates into LDS tables indexed by the
//     segment's slot in its keyframe (at most 256 per keyframe) and flushes them with float64 atomics;
//   step: per segment, boundary (lambda_smooth per pair, lambda_smooth r_b in the gradient) and prior
//     (lambda_prior, lambda_prior eta) terms, delta = clip(-g / ((1 + lambda_lm) H), +-eta_max), anchor
//     keyframes' segments fixed; eta is double-buffered so every segment reads the iteration's input.
// The objective reported per iteration is E' = sum rho + (lambda_smooth/2) sum_B r_b^2 +
// (lambda_prior/2) sum eta^2 at the iteration's input eta.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "sim3.hpp"

namespace ds3 {

constexpr int kMaxSegPerKf = 256;  // LDS tables of the data kernel are indexed by a keyframe's segment slot
constexpr int kSlots = 49;         // 7 x 7 grid-cell offsets of a boundary neighbour
constexpr double kFix = 1099511627776.0;  // 2^40, fixed-point scale of the boundary sums
constexpr int kDepthThreads = 256;
constexpr int kDepthPPT = 16;      // data kernel tile = 4096 pixels of keyframe j

struct DepthKf {
  int64_t off;      // arena pixel offset
  int32_t H, W, S, nx, ny;
  int32_t seg_base;  // first global segment id
  int32_t anchor;
  int32_t pad;
};

struct DepthConst {
  double conf_min;
  float inv_sigma, kappa;
  double lambda_smooth, lambda_prior, lambda_lm, eta_max;
};

// ---- features --------------------------------------------------------------------------------------
template <int DT>
__device__ inline void load_xyz(const void* arena, int64_t px, double* X, double& C) {
  const float4 v = Px<DT>::load(arena, px);
  X[0] = v.x;
  X[1] = v.y;
  X[2] = v.z;
  C = v.w;
}

// A hole: a non-finite component or |X| <= 1e-9 (products, sums and the square root in the order of the
// reference: (x x + y y) + z z).
__device__ inline bool is_hole(const double* X) {
  const double n = sqrt((X[0] * X[0] + X[1] * X[1]) + X[2] * X[2]);
  return !(isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2]) && n > 1e-9);
}

__device__ inline double log_range(const double* X) {
  const double a = isfinite(X[0]) ? X[0] : 0.0, b = isfinite(X[1]) ? X[1] : 0.0, c = isfinite(X[2]) ? X[2] : 0.0;
  const double n = sqrt((a * a + b * b) + c * c);
  return log(fmax(n, 1e-300));
}

// Per keyframe: min and max of ln|X| over its valid pixels (one block per keyframe).
template <int DT>
__global__ __launch_bounds__(kDepthThreads) void k_dr_logrange(const void* __restrict__ arena,
                                                               const DepthKf* __restrict__ kfs, DepthConst dc,
                                                               double* __restrict__ lmin, double* __restrict__ lmax) {
  const DepthKf K = kfs[blockIdx.x];
  const int n = K.H * K.W;
  double lo = INFINITY, hi = -INFINITY;
  for (int p = threadIdx.x; p < n; p += kDepthThreads) {
    double X[3], C;
    load_xyz<DT>(arena, K.off + p, X, C);
    if (is_hole(X) || !(C >= dc.conf_min)) continue;
    const double L = log_range(X);
    lo = fmin(lo, L);
    hi = fmax(hi, L);
  }
  __shared__ double slo[kDepthThreads / kWave], shi[kDepthThreads / kWave];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, kWave));
    hi = fmax(hi, __shfl_xor(hi, off, kWave));
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    slo[threadIdx.x / kWave] = lo;
    shi[threadIdx.x / kWave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kDepthThreads / kWave; ++w) {
      lo = fmin(slo[0], slo[w]);
      slo[0] = lo;
      hi = fmax(shi[0], shi[w]);
      shi[0] = hi;
    }
    lmin[blockIdx.x] = slo[0];
    lmax[blockIdx.x] = shi[0];
  }
}

// Quantised features of every pixel of keyframe blockIdx.y (4 x uint16, packed) and its label set to -1
// (invalid) or 0 (valid, to be assigned). Normal: cross product of central differences (one-sided at the
// border), unit length, oriented towards the camera; zero where a pixel used is a hole.
template <int DT>
__global__ __launch_bounds__(kDepthThreads) void k_dr_features(const void* __restrict__ arena,
                                                               const DepthKf* __restrict__ kfs, DepthConst dc,
                                                               const double* __restrict__ lmin,
                                                               const double* __restrict__ lmax,
                                                               uint2* __restrict__ feat, int32_t* __restrict__ label) {
  const DepthKf K = kfs[blockIdx.y];
  const int p = blockIdx.x * kDepthThreads + threadIdx.x;
  if (p >= K.H * K.W) return;
  const int v = p / K.W, u = p - v * K.W;
  double X[3], C;
  load_xyz<DT>(arena, K.off + p, X, C);
  const bool hole = is_hole(X);
  const bool valid = !hole && C >= dc.conf_min;
  const int64_t gp = K.off + p;
  if (!valid) {
    feat[gp] = make_uint2(0u, 0u);
    label[gp] = -1;
    return;
  }
  auto nb = [&](int uu, int vv, double* Y) {
    double c;
    load_xyz<DT>(arena, K.off + int64_t(vv) * K.W + uu, Y, c);
    const bool h = is_hole(Y);
    if (h) Y[0] = Y[1] = Y[2] = 0.0;
    return h;
  };
  double A[3], B[3], Cc[3], Dd[3];
  const int u0 = max(u - 1, 0), u1 = min(u + 1, K.W - 1), v0 = max(v - 1, 0), v1 = min(v + 1, K.H - 1);
  bool bad = nb(u1, v, A);
  bad |= nb(u0, v, B);
  bad |= nb(u, v1, Cc);
  bad |= nb(u, v0, Dd);
  const double du[3] = {A[0] - B[0], A[1] - B[1], A[2] - B[2]};
  const double dv[3] = {Cc[0] - Dd[0], Cc[1] - Dd[1], Cc[2] - Dd[2]};
  double c[3] = {du[1] * dv[2] - du[2] * dv[1], du[2] * dv[0] - du[0] * dv[2], du[0] * dv[1] - du[1] * dv[0]};
  const double ln = sqrt((c[0] * c[0] + c[1] * c[1]) + c[2] * c[2]);
  double n[3] = {0.0, 0.0, 0.0};
  if (!bad && ln > 0.0 && isfinite(ln)) {
    n[0] = c[0] / ln;
    n[1] = c[1] / ln;
    n[2] = c[2] / ln;
  }
  if ((n[0] * X[0] + n[1] * X[1]) + n[2] * X[2] > 0.0) {
    n[0] = -n[0];
    n[1] = -n[1];
    n[2] = -n[2];
  }
  const double lo = lmin[blockIdx.y], hi = lmax[blockIdx.y];
  const double ell = hi > lo ? (log_range(X) - lo) / (hi - lo) : 0.0;
  const uint32_t f0 = uint32_t(floor(1024.0 * (n[0] + 1.0) + 0.5));
  const uint32_t f1 = uint32_t(floor(1024.0 * (n[1] + 1.0) + 0.5));
  const uint32_t f2 = uint32_t(floor(1024.0 * (n[2] + 1.0) + 0.5));
  const uint32_t f3 = uint32_t(floor(1024.0 * ell + 0.5));
  feat[gp] = make_uint2(f0 | (f1 << 16), f2 | (f3 << 16));
  label[gp] = 0;
}

__device__ inline void unpack_feat(uint2 w, int64_t* F) {
  F[0] = int64_t(w.x & 0xffffu);
  F[1] = int64_t(w.x >> 16);
  F[2] = int64_t(w.y & 0xffffu);
  F[3] = int64_t(w.y >> 16);
}

// ---- SLIC --------------------------------------------------------------------------------------------
// Centre c of keyframe k: cen[6 (seg_base + c) + {x, y, F0..F3}] (int64).
__global__ void k_slic_init(const DepthKf* __restrict__ kfs, int n_kf, const uint2* __restrict__ feat,
                            int64_t* __restrict__ cen) {
  const int k = blockIdx.y;
  if (k >= n_kf) return;
  const DepthKf K = kfs[k];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K.nx * K.ny) return;
  const int cy = c / K.nx, cx = c - cy * K.nx;
  const int px = min(cx * K.S + K.S / 2, K.W - 1), py = min(cy * K.S + K.S / 2, K.H - 1);
  int64_t F[4];
  unpack_feat(feat[K.off + int64_t(py) * K.W + px], F);
  int64_t* o = cen + 6 * int64_t(K.seg_base + c);
  o[0] = px;
  o[1] = py;
  for (int q = 0; q < 4; ++q) o[2 + q] = F[q];
}

// Each valid pixel takes the nearest of the centres of the 3x3 grid cells around its own.
__global__ __launch_bounds__(kDepthThreads) void k_slic_assign(const DepthKf* __restrict__ kfs,
                                                               const uint2* __restrict__ feat,
                                                               const int64_t* __restrict__ cen,
                                                               int32_t* __restrict__ label) {
  const DepthKf K = kfs[blockIdx.y];
  const int p = blockIdx.x * kDepthThreads + threadIdx.x;
  if (p >= K.H * K.W) return;
  const int64_t gp = K.off + p;
  if (label[gp] < 0) return;
  const int v = p / K.W, u = p - v * K.W;
  const int gx = min(u / K.S, K.nx - 1), gy = min(v / K.S, K.ny - 1);
  int64_t F[4];
  unpack_feat(feat[gp], F);
  const int64_t S2 = int64_t(K.S) * K.S, w2 = 512 * 512;
  int64_t best = INT64_MAX;
  int lab = 0;
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      const int cx = gx + dx, cy = gy + dy;
      if (cx < 0 || cx >= K.nx || cy < 0 || cy >= K.ny) continue;
      const int c = cy * K.nx + cx;
      const int64_t* o = cen + 6 * int64_t(K.seg_base + c);
      int64_t d = 0;
      for (int q = 0; q < 4; ++q) {
        const int64_t e = F[q] - o[2 + q];
        d += e * e;
      }
      const int64_t ex = u - o[0], ey = v - o[1];
      d = S2 * d + w2 * (ex * ex + ey * ey);
      if (d < best) {
        best = d;
        lab = c;
      }
    }
  label[gp] = lab;
}

// One block per centre: sums its members over the 3x3 cells around its own cell, moves it to the floor of
// their mean (no members: unchanged) and writes the member count.
__global__ __launch_bounds__(kDepthThreads) void k_slic_update(const DepthKf* __restrict__ kfs,
                                                               const uint2* __restrict__ feat,
                                                               const int32_t* __restrict__ label,
                                                               int64_t* __restrict__ cen, int32_t* __restrict__ cnt) {
  const DepthKf K = kfs[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= K.nx * K.ny) return;
  const int cy = c / K.nx, cx = c - cy * K.nx;
  const int x0 = max(cx - 1, 0) * K.S, x1 = min((cx + 2) * K.S, K.W);
  const int y0 = max(cy - 1, 0) * K.S, y1 = min((cy + 2) * K.S, K.H);
  // the last cell also holds the pixels beyond nx S (resp. ny S): widen to the image edge
  const int xe = (cx + 1 >= K.nx - 1) ? K.W : x1, ye = (cy + 1 >= K.ny - 1) ? K.H : y1;
  const int w = xe - x0, h = ye - y0;
  int64_t s[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int q = threadIdx.x; q < w * h; q += kDepthThreads) {
    const int yy = y0 + q / w, xx = x0 + q % w;
    const int64_t gp = K.off + int64_t(yy) * K.W + xx;
    if (label[gp] != c) continue;
    int64_t F[4];
    unpack_feat(feat[gp], F);
    s[0] += xx;
    s[1] += yy;
    for (int k = 0; k < 4; ++k) s[2 + k] += F[k];
    s[6] += 1;
  }
  __shared__ int64_t red[kDepthThreads / kWave][7];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    int64_t a = s[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave][k] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t[7];
    for (int k = 0; k < 7; ++k) {
      t[k] = 0;
      for (int ww = 0; ww < kDepthThreads / kWave; ++ww) t[k] += red[ww][k];
    }
    const int g = K.seg_base + c;
    if (t[6] > 0)
      for (int k = 0; k < 6; ++k) cen[6 * int64_t(g) + k] = t[k] / t[6];  // members' sums are >= 0: floor
    cnt[g] = int32_t(t[6]);
  }
}

// Final labels: global segment id, or -1 for invalid pixels and for segments with fewer than min_px pixels.
__global__ __launch_bounds__(kDepthThreads) void k_label_finalize(const DepthKf* __restrict__ kfs,
                                                                  const int32_t* __restrict__ cnt, int min_px,
                                                                  int32_t* __restrict__ label,
                                                                  uint8_t* __restrict__ seg_valid) {
  const DepthKf K = kfs[blockIdx.y];
  const int p = blockIdx.x * kDepthThreads + threadIdx.x;
  if (p < K.nx * K.ny) seg_valid[K.seg_base + p] = cnt[K.seg_base + p] >= min_px ? 1 : 0;
  if (p >= K.H * K.W) return;
  const int64_t gp = K.off + p;
  const int l = label[gp];
  if (l < 0) return;
  label[gp] = cnt[K.seg_base + l] >= min_px ? K.seg_base + l : -1;
}

// ---- boundary table -------------------------------------------------------------------------------------
__device__ inline int slot_of(const DepthKf& K, int g_local, int h_local) {
  const int gy = g_local / K.nx, gx = g_local - gy * K.nx;
  const int hy = h_local / K.nx, hx = h_local - hy * K.nx;
  return (hy - gy + 3) * 7 + (hx - gx + 3);
}

template <int DT>
__global__ __launch_bounds__(kDepthThreads) void k_dr_boundary(const void* __restrict__ arena,
                                                               const DepthKf* __restrict__ kfs,
                                                               const int32_t* __restrict__ label,
                                                               unsigned long long* __restrict__ bsum,
                                                               int32_t* __restrict__ bcnt) {
  const DepthKf K = kfs[blockIdx.y];
  const int p = blockIdx.x * kDepthThreads + threadIdx.x;
  if (p >= K.H * K.W) return;
  const int v = p / K.W, u = p - v * K.W;
  const int64_t gp = K.off + p;
  const int g = label[gp];
  if (g < 0) return;
  double X[3], C;
  load_xyz<DT>(arena, gp, X, C);
  const double Lp = log_range(X);
  for (int dir = 0; dir < 2; ++dir) {
    const int uu = u + (dir == 0), vv = v + (dir == 1);
    if (uu >= K.W || vv >= K.H) continue;
    const int64_t gq = K.off + int64_t(vv) * K.W + uu;
    const int h = label[gq];
    if (h < 0 || h == g) continue;
    double Y[3];
    load_xyz<DT>(arena, gq, Y, C);
    const double d = Lp - log_range(Y);
    const long long q = llrint(d * kFix);
    const int gl = g - K.seg_base, hl = h - K.seg_base;
    atomicAdd(&bsum[int64_t(g) * kSlots + slot_of(K, gl, hl)], (unsigned long long)q);
    atomicAdd(&bcnt[int64_t(g) * kSlots + slot_of(K, gl, hl)], 1);
    atomicAdd(&bsum[int64_t(h) * kSlots + slot_of(K, hl, gl)], (unsigned long long)(-q));
    atomicAdd(&bcnt[int64_t(h) * kSlots + slot_of(K, hl, gl)], 1);
  }
}

// ---- refinement iteration -------------------------------------------------------------------------------
struct DepthEdge {
  int64_t off_i, off_j, idx_off;
  int32_t npx_i, npx_j;
  int32_t base_i, base_j;  // first global segment id of keyframes i and j
  int32_t tile0, n_tiles;
};

// One block per (edge, tile of keyframe j): data-term sums of the segments it touches, flushed with float64
// atomics; the block's cost into its partial. The scale factors exp(eta) of both keyframes' segments are
// formed once per block into LDS. A thread takes groups of kGrp consecutive pixels of j: all loads of a
// group are issued together (matches, both points, both labels), and
// consecutive matches of one segment (the usual case: segments are tens of pixels wide and neighbouring
// matches land in neighbouring pixels of i) are summed in registers before one LDS add per run.
constexpr int kGrp = 4;

__device__ inline void run_flush(float* H, float* G, int base, int& cur, float& h, float& g) {
  if (cur >= 0) {
    atomicAdd(&H[cur - base], h);
    atomicAdd(&G[cur - base], g);
  }
  cur = -1;
  h = 0.0f;
  g = 0.0f;
}

template <int DT>
__global__ __launch_bounds__(kDepthThreads) void k_dr_data(const void* __restrict__ arena,
                                                           const DepthEdge* __restrict__ edges,
                                                           const int2* __restrict__ items,
                                                           const EdgeXf* __restrict__ xf,
                                                           const int32_t* __restrict__ idx_arena,
                                                           const int32_t* __restrict__ label,
                                                           const double* __restrict__ eta, int n_seg, DepthConst dc,
                                                           double* __restrict__ Hd, double* __restrict__ gd,
                                                           float* __restrict__ cost_part) {
  __shared__ float sHj[kMaxSegPerKf], sGj[kMaxSegPerKf], sHi[kMaxSegPerKf], sGi[kMaxSegPerKf];
  __shared__ float sEj[kMaxSegPerKf], sEi[kMaxSegPerKf];  // exp(eta) of the two keyframes' segments, eq. (8)
  __shared__ float red[kDepthThreads / kWave];
  const int2 W = items[blockIdx.x];
  const DepthEdge E = edges[W.x];
  for (int q = threadIdx.x; q < kMaxSegPerKf; q += kDepthThreads) {
    sHj[q] = sGj[q] = sHi[q] = sGi[q] = 0.0f;
    sEj[q] = (E.base_j + q < n_seg) ? expf(float(eta[E.base_j + q])) : 1.0f;
    sEi[q] = (E.base_i + q < n_seg) ? expf(float(eta[E.base_i + q])) : 1.0f;
  }
  __syncthreads();
  float M[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) M[q] = xf[W.x].m[q];
  const int32_t* __restrict__ idx = idx_arena + E.idx_off;
  float cost = 0.0f;
  int curj = -1, curi = -1;
  float hj = 0.0f, gj = 0.0f, hi = 0.0f, gi = 0.0f;
  const int base = W.y * (kDepthThreads * kDepthPPT);
#pragma unroll 1
  for (int k = 0; k < kDepthPPT / kGrp; ++k) {
    const int n0 = base + (k * kDepthThreads + int(threadIdx.x)) * kGrp;
    int m[kGrp];
#pragma unroll
    for (int u = 0; u < kGrp; ++u) {
      const int n = n0 + u;
      m[u] = (n < E.npx_j) ? idx[n] : -1;
      if (m[u] >= E.npx_i) m[u] = -1;
    }
    float4 Xj[kGrp], Xi[kGrp];
    int h[kGrp], g[kGrp];
#pragma unroll
    for (int u = 0; u < kGrp; ++u) {
      h[u] = g[u] = -1;
      if (m[u] >= 0) {
        Xj[u] = Px<DT>::load(arena, E.off_j + n0 + u);
        Xi[u] = Px<DT>::load(arena, E.off_i + m[u]);
        h[u] = label[E.off_j + n0 + u];
        g[u] = label[E.off_i + m[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < kGrp; ++u) {
      if (m[u] < 0) continue;
      const float4 A = Xj[u], B = Xi[u];
      const float dj2 = fmaf(A.x, A.x, fmaf(A.y, A.y, A.z * A.z));
      const float di2 = fmaf(B.x, B.x, fmaf(B.y, B.y, B.z * B.z));
      const float cc = B.w * A.w;
      if (!(fminf(dj2, di2) > 1e-18f) || !(dj2 + di2 + cc < __builtin_huge_valf()) || !(cc >= 0.0f)) continue;
      const float fh = h[u] >= 0 ? sEj[h[u] - E.base_j] : 1.0f;  // exp(0) for a pixel without a segment
      const float fg = g[u] >= 0 ? sEi[g[u] - E.base_i] : 1.0f;
      const float a0 = A.x * fh, a1 = A.y * fh, a2 = A.z * fh;   // X_j(eta), eq. (8)
      const float b0 = B.x * fg, b1 = B.y * fg, b2 = B.z * fg;   // X_i(eta)
      const float s = __builtin_amdgcn_sqrtf(__builtin_amdgcn_sqrtf(cc)) * dc.inv_sigma;
      const float R0 = fmaf(M[0], a0, fmaf(M[1], a1, M[2] * a2));  // sR_ij X_j(eta)
      const float R1 = fmaf(M[3], a0, fmaf(M[4], a1, M[5] * a2));
      const float R2 = fmaf(M[6], a0, fmaf(M[7], a1, M[8] * a2));
      const float r0 = s * (R0 + M[9] - b0), r1 = s * (R1 + M[10] - b1), r2 = s * (R2 + M[11] - b2);
      const float e0 = fabsf(r0), e1 = fabsf(r1), e2 = fabsf(r2);
      const float w0 = fminf(1.0f, dc.kappa * __builtin_amdgcn_rcpf(e0));
      const float w1 = fminf(1.0f, dc.kappa * __builtin_amdgcn_rcpf(e1));
      const float w2 = fminf(1.0f, dc.kappa * __builtin_amdgcn_rcpf(e2));
      const float t0 = w0 * e0, t1 = w1 * e1, t2 = w2 * e2;
      cost += t0 * fmaf(-0.5f, t0, e0) + t1 * fmaf(-0.5f, t1, e1) + t2 * fmaf(-0.5f, t2, e2);
      if (h[u] >= 0) {
        if (h[u] != curj) {
          run_flush(sHj, sGj, E.base_j, curj, hj, gj);
          curj = h[u];
        }
        const float J0 = s * R0, J1 = s * R1, J2 = s * R2;
        hj += w0 * J0 * J0 + w1 * J1 * J1 + w2 * J2 * J2;
        gj += w0 * J0 * r0 + w1 * J1 * r1 + w2 * J2 * r2;
      }
      if (g[u] >= 0) {
        if (g[u] != curi) {
          run_flush(sHi, sGi, E.base_i, curi, hi, gi);
          curi = g[u];
        }
        const float J0 = -s * b0, J1 = -s * b1, J2 = -s * b2;
        hi += w0 * J0 * J0 + w1 * J1 * J1 + w2 * J2 * J2;
        gi += w0 * J0 * r0 + w1 * J1 * r1 + w2 * J2 * r2;
      }
    }
  }
  run_flush(sHj, sGj, E.base_j, curj, hj, gj);
  run_flush(sHi, sGi, E.base_i, curi, hi, gi);
  float c = wave_sum(cost);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < kDepthThreads / kWave; ++w) t += red[w];
    cost_part[blockIdx.x] = t;
  }
  for (int q = threadIdx.x; q < kMaxSegPerKf; q += kDepthThreads) {
    if (sHj[q] != 0.0f || sGj[q] != 0.0f) {
      atomicAdd(&Hd[E.base_j + q], double(sHj[q]));
      atomicAdd(&gd[E.base_j + q], double(sGj[q]));
    }
    if (sHi[q] != 0.0f || sGi[q] != 0.0f) {
      atomicAdd(&Hd[E.base_i + q], double(sHi[q]));
      atomicAdd(&gd[E.base_i + q], double(sGi[q]));
    }
  }
}

// One thread per segment: boundary and prior terms, the damped and clipped step (free segments only), and
// the segment's share of the boundary and prior cost (each unordered pair once, at its lower id).
__global__ __launch_bounds__(kDepthThreads) void k_dr_step(const DepthKf* __restrict__ kfs, int n_kf,
                                                           const int32_t* __restrict__ seg_kf,
                                                           const uint8_t* __restrict__ seg_valid,
                                                           const unsigned long long* __restrict__ bsum,
                                                           const int32_t* __restrict__ bcnt,
                                                           const double* __restrict__ Hd, const double* __restrict__ gd,
                                                           const double* __restrict__ eta, double* __restrict__ eta_out,
                                                           int n_seg, DepthConst dc, double* __restrict__ cost_part) {
  const int s = blockIdx.x * kDepthThreads + threadIdx.x;
  double cost = 0.0;
  if (s < n_seg) {
    const double e = eta[s];
    double out = e;
    if (seg_valid[s]) {
      const DepthKf K = kfs[seg_kf[s]];
      const int l = s - K.seg_base;
      const int gy = l / K.nx, gx = l - gy * K.nx;
      double H = Hd[s] + dc.lambda_prior, g = gd[s] + dc.lambda_prior * e;
      cost += 0.5 * dc.lambda_prior * e * e;
      for (int q = 0; q < kSlots; ++q) {
        const int c = bcnt[int64_t(s) * kSlots + q];
        if (c == 0) continue;
        const int hx = gx + q % 7 - 3, hy = gy + q / 7 - 3;
        const int h = K.seg_base + hy * K.nx + hx;
        const double dlt = double((long long)bsum[int64_t(s) * kSlots + q]) / kFix / double(c);
        const double rb = e - eta[h] + dlt;
        H += dc.lambda_smooth;
        g += dc.lambda_smooth * rb;
        if (s < h) cost += 0.5 * dc.lambda_smooth * rb * rb;
      }
      if (!K.anchor) {
        const double d = fmin(fmax(-g / ((1.0 + dc.lambda_lm) * H), -dc.eta_max), dc.eta_max);
        out = e + d;
      }
    }
    eta_out[s] = out;
  }
  __shared__ double red[kDepthThreads / kWave];
  const double c = wave_sum(cost);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kDepthThreads / kWave; ++w) t += red[w];
    cost_part[blockIdx.x] = t;
  }
}

// Cost of the iteration: the data partials (float, per block) and the step partials (float64, per block)
// summed in a fixed order into hist[it]. Also clears Hd and gd for the next iteration.
__global__ __launch_bounds__(kDepthThreads) void k_dr_cost(const float* __restrict__ data_part, int n_data,
                                                           const double* __restrict__ step_part, int n_step,
                                                           double* __restrict__ hist, int it,
                                                           double* __restrict__ Hd, double* __restrict__ gd,
                                                           int n_seg) {
  for (int s = blockIdx.x * kDepthThreads + threadIdx.x; s < n_seg; s += gridDim.x * kDepthThreads) {
    Hd[s] = 0.0;
    gd[s] = 0.0;
  }
  if (blockIdx.x != 0) return;
  double acc = 0.0;
  for (int q = threadIdx.x; q < n_data; q += kDepthThreads) acc += double(data_part[q]);
  for (int q = threadIdx.x; q < n_step; q += kDepthThreads) acc += step_part[q];
  __shared__ double red[kDepthThreads / kWave];
  const double c = wave_sum(acc);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kDepthThreads / kWave; ++w) t += red[w];
    hist[it] = t;
  }
}

// X(eta) for every arena pixel: xyz scaled by exp(eta_g), confidence copied (float32 xyzc out).
template <int DT>
__global__ __launch_bounds__(kDepthThreads) void k_dr_apply(const void* __restrict__ arena, int64_t n_px,
                                                            const int32_t* __restrict__ label,
                                                            const double* __restrict__ eta, float4* __restrict__ out) {
  const int64_t p = int64_t(blockIdx.x) * kDepthThreads + threadIdx.x;
  if (p >= n_px) return;
  const float4 X = Px<DT>::load(arena, p);
  const int g = label[p];
  const double f = g >= 0 ? exp(eta[g]) : 1.0;
  out[p] = make_float4(float(double(X.x) * f), float(double(X.y) * f), float(double(X.z) * f), X.w);
}

// ---- plan -----------------------------------------------------------------------------------------------
struct DepthPlan {
  ds3_dtype dt = DS3_F32;
  const void* arena = nullptr;
  const int32_t* idx = nullptr;
  int n_kf = 0, n_edges = 0, n_seg = 0, n_items = 0;
  int64_t n_px = 0;
  DepthConst dc;
  std::vector<DepthKf> kf_host;
  void* mem = nullptr;
  DepthKf* kfs = nullptr;
  DepthEdge* edges = nullptr;
  EdgeDev* gedges = nullptr;  // for the pose prep
  int2* items = nullptr;
  EdgeXf* xf = nullptr;
  double* Ad = nullptr;
  int32_t* label = nullptr;
  uint2* feat = nullptr;
  int64_t* cen = nullptr;
  int32_t* cnt = nullptr;
  uint8_t* seg_valid = nullptr;
  int32_t* seg_kf = nullptr;
  unsigned long long* bsum = nullptr;
  int32_t* bcnt = nullptr;
  double *eta = nullptr, *eta2 = nullptr, *Hd = nullptr, *gd = nullptr;
  double *lmin = nullptr, *lmax = nullptr;
  float* data_part = nullptr;
  double* step_part = nullptr;
  double* hist = nullptr;
  int64_t valid_segments = 0, pairs = 0, px_scanned = 0;
};

static size_t carve_depth(void* base, DepthPlan& P) {
  Carver c(base);
  P.kfs = c.take<DepthKf>(P.n_kf);
  P.edges = c.take<DepthEdge>(std::max(P.n_edges, 1));
  P.gedges = c.take<EdgeDev>(std::max(P.n_edges, 1));
  P.items = c.take<int2>(std::max(P.n_items, 1));
  P.xf = c.take<EdgeXf>(std::max(P.n_edges, 1));
  P.Ad = c.take<double>(49 * size_t(std::max(P.n_edges, 1)));
  P.label = c.take<int32_t>(size_t(P.n_px));
  P.feat = c.take<uint2>(size_t(P.n_px));
  P.cen = c.take<int64_t>(6 * size_t(P.n_seg));
  P.cnt = c.take<int32_t>(P.n_seg);
  P.seg_valid = c.take<uint8_t>(P.n_seg);
  P.seg_kf = c.take<int32_t>(P.n_seg);
  P.bsum = c.take<unsigned long long>(size_t(kSlots) * P.n_seg);
  P.bcnt = c.take<int32_t>(size_t(kSlots) * P.n_seg);
  P.eta = c.take<double>(P.n_seg);
  P.eta2 = c.take<double>(P.n_seg);
  P.Hd = c.take<double>(P.n_seg);
  P.gd = c.take<double>(P.n_seg);
  P.lmin = c.take<double>(P.n_kf);
  P.lmax = c.take<double>(P.n_kf);
  P.data_part = c.take<float>(std::max(P.n_items, 1));
  P.step_part = c.take<double>((P.n_seg + kDepthThreads - 1) / kDepthThreads);
  P.hist = c.take<double>(1024);
  return c.used;
}

template <class T>
static int upload_vec(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return DS3_OK;
  return check_hip(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s), "upload");
}

static int depth_segment(DepthPlan& P, int slic_iters, int min_px, hipStream_t s) {
  int max_px = 0, max_m = 0;
  for (auto& K : P.kf_host) {
    max_px = std::max(max_px, K.H * K.W);
    max_m = std::max(max_m, K.nx * K.ny);
  }
  const dim3 gpx((max_px + kDepthThreads - 1) / kDepthThreads, P.n_kf);
  if (P.dt == DS3_F32) {
    hipLaunchKernelGGL(k_dr_logrange<DS3_F32>, dim3(P.n_kf), dim3(kDepthThreads), 0, s, P.arena, P.kfs, P.dc, P.lmin, P.lmax);
    hipLaunchKernelGGL(k_dr_features<DS3_F32>, gpx, dim3(kDepthThreads), 0, s, P.arena, P.kfs, P.dc, P.lmin, P.lmax, P.feat, P.label);
  } else {
    hipLaunchKernelGGL(k_dr_logrange<DS3_BF16>, dim3(P.n_kf), dim3(kDepthThreads), 0, s, P.arena, P.kfs, P.dc, P.lmin, P.lmax);
    hipLaunchKernelGGL(k_dr_features<DS3_BF16>, gpx, dim3(kDepthThreads), 0, s, P.arena, P.kfs, P.dc, P.lmin, P.lmax, P.feat, P.label);
  }
  DS3_TRY(check_hip(hipGetLastError(), "k_dr_features"));
  hipLaunchKernelGGL(k_slic_init, dim3((max_m + 63) / 64, P.n_kf), dim3(64), 0, s, P.kfs, P.n_kf, P.feat, P.cen);
  DS3_TRY(check_hip(hipGetLastError(), "k_slic_init"));
  for (int it = 0; it < slic_iters; ++it) {
    hipLaunchKernelGGL(k_slic_assign, gpx, dim3(kDepthThreads), 0, s, P.kfs, P.feat, P.cen, P.label);
    hipLaunchKernelGGL(k_slic_update, dim3(max_m, P.n_kf), dim3(kDepthThreads), 0, s, P.kfs, P.feat, P.label, P.cen,
                       P.cnt);
    DS3_TRY(check_hip(hipGetLastError(), "k_slic"));
  }
  const dim3 gfin((std::max(max_px, max_m) + kDepthThreads - 1) / kDepthThreads, P.n_kf);
  hipLaunchKernelGGL(k_label_finalize, gfin, dim3(kDepthThreads), 0, s, P.kfs, P.cnt, min_px, P.label, P.seg_valid);
  DS3_TRY(check_hip(hipGetLastError(), "k_label_finalize"));
  DS3_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(P.bsum), 2 * kSlots * size_t(P.n_seg), 0u, s));
  DS3_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(P.bcnt), kSlots * size_t(P.n_seg), 0u, s));
  if (P.dt == DS3_F32)
    hipLaunchKernelGGL(k_dr_boundary<DS3_F32>, gpx, dim3(kDepthThreads), 0, s, P.arena, P.kfs, P.label, P.bsum, P.bcnt);
  else
    hipLaunchKernelGGL(k_dr_boundary<DS3_BF16>, gpx, dim3(kDepthThreads), 0, s, P.arena, P.kfs, P.label, P.bsum, P.bcnt);
  return check_hip(hipGetLastError(), "k_dr_boundary");
}

static void depth_free(DepthPlan* P) {
  if (!P) return;
  if (P->mem) (void)hipFree(P->mem);
  delete P;
}

}  // namespace ds3

using namespace ds3;

extern "C" {

void ds3_default_depth_params(ds3_depth_params* p) {
  if (!p) return;
  p->segments_per_kf = 200;
  p->conf_min = 1.5;
  p->min_seg_px = 16;
  p->slic_iters = 10;
  p->sigma_point = 0.05;
  p->huber_k = 1.345;
  p->lambda_smooth = 1.0;
  p->lambda_prior = 1.0;
  p->lambda_lm = 0.05;
  p->eta_max = 0.5;
}

int ds3_depth_plan_create(int32_t n_kf, const ds3_image* kf, const void* arena, ds3_dtype dtype, const ds3_edge* edges,
                          int32_t n_edges, const int32_t* idx_arena, const int32_t* anchors, int32_t n_anchors,
                          const ds3_depth_params* params, void** plan_out, void* stream) {
  if (!plan_out) return fail(DS3_EINVAL, "depth: plan_out is null");
  *plan_out = nullptr;
  if (n_kf <= 0 || !kf || !arena || !params || n_edges < 0 || (n_edges > 0 && (!edges || !idx_arena)) ||
      n_anchors < 0 || (n_anchors > 0 && !anchors))
    return fail(DS3_EINVAL, "depth: bad arguments");
  if (dtype != DS3_F32 && dtype != DS3_BF16) return fail(DS3_ENOTSUP, "depth: dtype");
  if ((reinterpret_cast<uintptr_t>(arena) & 15) != 0) return fail(DS3_EINVAL, "depth: arena must be 16 B aligned");
  const ds3_depth_params& p = *params;
  if (p.segments_per_kf < 1 || p.min_seg_px < 0 || p.slic_iters < 1 || p.slic_iters > 100 || !(p.sigma_point > 0) ||
      !(p.huber_k > 0) || !(p.lambda_smooth >= 0) || !(p.lambda_prior >= 0) || !(p.lambda_lm >= 0) ||
      !(p.eta_max > 0))
    return fail(DS3_EINVAL, "depth: bad parameters");
  DepthPlan* P = new DepthPlan();
  P->dt = dtype;
  P->arena = arena;
  P->idx = idx_arena;
  P->n_kf = n_kf;
  P->n_edges = n_edges;
  P->dc.conf_min = p.conf_min;
  P->dc.inv_sigma = float(1.0 / p.sigma_point);
  P->dc.kappa = float(p.huber_k);
  P->dc.lambda_smooth = p.lambda_smooth;
  P->dc.lambda_prior = p.lambda_prior;
  P->dc.lambda_lm = p.lambda_lm;
  P->dc.eta_max = p.eta_max;
  std::vector<uint8_t> is_anchor(n_kf, 0);
  for (int a = 0; a < n_anchors; ++a) {
    if (anchors[a] < 0 || anchors[a] >= n_kf) { depth_free(P); return fail(DS3_EINVAL, "depth: anchor out of range"); }
    is_anchor[anchors[a]] = 1;
  }
  int seg = 0;
  int64_t px = 0;
  std::vector<int32_t> seg_kf;
  for (int k = 0; k < n_kf; ++k) {
    const ds3_image& I = kf[k];
    if (I.H <= 0 || I.W <= 0 || I.px_offset < 0 || int64_t(I.H) * I.W > INT32_MAX) {
      depth_free(P);
      return fail(DS3_EINVAL, "depth: bad keyframe image " + std::to_string(k));
    }
    DepthKf K;
    K.off = I.px_offset;
    K.H = I.H;
    K.W = I.W;
    K.S = std::max(1, int(std::floor(std::sqrt(double(I.H) * I.W / p.segments_per_kf) + 0.5)));
    K.nx = (I.W + K.S - 1) / K.S;
    K.ny = (I.H + K.S - 1) / K.S;
    if (K.nx * K.ny > kMaxSegPerKf) {
      depth_free(P);
      return fail(DS3_EINVAL, "depth: more than 256 segments in keyframe " + std::to_string(k));
    }
    K.seg_base = seg;
    K.anchor = is_anchor[k];
    K.pad = 0;
    for (int q = 0; q < K.nx * K.ny; ++q) seg_kf.push_back(k);
    seg += K.nx * K.ny;
    px = std::max(px, I.px_offset + int64_t(I.H) * I.W);
    P->kf_host.push_back(K);
  }
  P->n_seg = seg;
  P->n_px = px;
  // edges and their tiles
  std::vector<DepthEdge> de(std::max(n_edges, 1));
  std::vector<EdgeDev> ge(std::max(n_edges, 1));
  std::vector<int2> items;
  const int tile = kDepthThreads * kDepthPPT;
  for (int e = 0; e < n_edges; ++e) {
    const ds3_edge& Ed = edges[e];
    if (Ed.i < 0 || Ed.i >= n_kf || Ed.j < 0 || Ed.j >= n_kf || Ed.i == Ed.j || Ed.idx_offset < 0) {
      depth_free(P);
      return fail(DS3_EINVAL, "depth: bad edge " + std::to_string(e));
    }
    DepthEdge D;
    D.off_i = kf[Ed.i].px_offset;
    D.off_j = kf[Ed.j].px_offset;
    D.idx_off = Ed.idx_offset;
    D.npx_i = kf[Ed.i].H * kf[Ed.i].W;
    D.npx_j = kf[Ed.j].H * kf[Ed.j].W;
    D.base_i = P->kf_host[Ed.i].seg_base;
    D.base_j = P->kf_host[Ed.j].seg_base;
    D.tile0 = int32_t(items.size());
    D.n_tiles = (D.npx_j + tile - 1) / tile;
    for (int t = 0; t < D.n_tiles; ++t) items.push_back(make_int2(e, t));
    de[e] = D;
    EdgeDev G{};
    G.off_i = D.off_i;
    G.off_j = D.off_j;
    G.idx_off = D.idx_off;
    G.npx_i = D.npx_i;
    G.npx_j = D.npx_j;
    G.i = Ed.i;
    G.j = Ed.j;
    ge[e] = G;
    P->px_scanned += D.npx_j;
  }
  P->n_items = int(items.size());
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t bytes = carve_depth(nullptr, *P);
  int rc = check_hip(hipMalloc(&P->mem, bytes), "hipMalloc(depth plan)");
  if (rc == DS3_OK) {
    carve_depth(P->mem, *P);
    rc = upload_vec(P->kfs, P->kf_host, s);
    if (rc == DS3_OK) rc = upload_vec(P->edges, de, s);
    if (rc == DS3_OK) rc = upload_vec(P->gedges, ge, s);
    if (rc == DS3_OK) rc = upload_vec(P->items, items, s);
    if (rc == DS3_OK) rc = upload_vec(P->seg_kf, seg_kf, s);
    if (rc == DS3_OK) rc = launch_fill(P->eta, size_t(P->n_seg), 0.0, s);
    if (rc == DS3_OK) rc = launch_fill(P->Hd, size_t(P->n_seg), 0.0, s);
    if (rc == DS3_OK) rc = launch_fill(P->gd, size_t(P->n_seg), 0.0, s);
    if (rc == DS3_OK) rc = depth_segment(*P, p.slic_iters, p.min_seg_px, s);
    // facts for the caller (synchronises once, at creation)
    std::vector<uint8_t> sv(P->n_seg);
    std::vector<int32_t> bc(size_t(kSlots) * P->n_seg);
    if (rc == DS3_OK) rc = check_hip(hipMemcpyAsync(sv.data(), P->seg_valid, sv.size(), hipMemcpyDeviceToHost, s), "d2h");
    if (rc == DS3_OK)
      rc = check_hip(hipMemcpyAsync(bc.data(), P->bcnt, sizeof(int32_t) * bc.size(), hipMemcpyDeviceToHost, s), "d2h");
    if (rc == DS3_OK) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize(depth plan)");
    if (rc == DS3_OK) {
      for (auto v : sv) P->valid_segments += v;
      for (auto v : bc) P->pairs += v > 0;
    }
  }
  if (rc != DS3_OK) { depth_free(P); return rc; }
  *plan_out = P;
  return DS3_OK;
}

int ds3_depth_plan_run(void* plan, const double* poses, int32_t iters, double* cost_per_iter, ds3_timer* data_timer,
                       void* stream) {
  DepthPlan* P = static_cast<DepthPlan*>(plan);
  if (!P || !poses || iters < 0 || iters > 1024) return fail(DS3_EINVAL, "depth_run: bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nstep = (P->n_seg + kDepthThreads - 1) / kDepthThreads;
  for (int it = 0; it < iters; ++it) {
    DS3_TRY(launch_gn_prep(poses, P->gedges, P->n_edges, P->xf, P->Ad, s));
    const bool timed = data_timer && it == iters - 1;
    if (timed) DS3_TRY(timer_record(data_timer, true, s));
    if (P->n_items > 0) {
      if (P->dt == DS3_F32)
        hipLaunchKernelGGL(k_dr_data<DS3_F32>, dim3(P->n_items), dim3(kDepthThreads), 0, s, P->arena, P->edges, P->items,
                           P->xf, P->idx, P->label, P->eta, P->n_seg, P->dc, P->Hd, P->gd, P->data_part);
      else
        hipLaunchKernelGGL(k_dr_data<DS3_BF16>, dim3(P->n_items), dim3(kDepthThreads), 0, s, P->arena, P->edges, P->items,
                           P->xf, P->idx, P->label, P->eta, P->n_seg, P->dc, P->Hd, P->gd, P->data_part);
      DS3_TRY(check_hip(hipGetLastError(), "k_dr_data"));
    }
    if (timed) DS3_TRY(timer_record(data_timer, false, s));
    hipLaunchKernelGGL(k_dr_step, dim3(std::max(nstep, 1)), dim3(kDepthThreads), 0, s, P->kfs, P->n_kf, P->seg_kf,
                       P->seg_valid, P->bsum, P->bcnt, P->Hd, P->gd, P->eta, P->eta2, P->n_seg, P->dc, P->step_part);
    DS3_TRY(check_hip(hipGetLastError(), "k_dr_step"));
    hipLaunchKernelGGL(k_dr_cost, dim3(std::max(1, std::min(256, nstep))), dim3(kDepthThreads), 0, s, P->data_part,
                       P->n_items, P->step_part, nstep, P->hist, it, P->Hd, P->gd, P->n_seg);
    DS3_TRY(check_hip(hipGetLastError(), "k_dr_cost"));
    std::swap(P->eta, P->eta2);
  }
  if (iters > 0 && cost_per_iter)
    DS3_TRY(check_hip(hipMemcpyAsync(cost_per_iter, P->hist, sizeof(double) * iters, hipMemcpyDeviceToDevice, s), "copy"));
  return DS3_OK;
}

int ds3_depth_plan_info(void* plan, int64_t* info, int32_t n_info) {
  DepthPlan* P = static_cast<DepthPlan*>(plan);
  if (!P || !info || n_info < 0) return fail(DS3_EINVAL, "depth_info: bad arguments");
  const int64_t v[6] = {P->n_seg, P->valid_segments, P->pairs, P->n_items, P->px_scanned, P->n_px};
  for (int k = 0; k < n_info && k < 6; ++k) info[k] = v[k];
  return DS3_OK;
}

int ds3_depth_plan_get(void* plan, int32_t* labels_out, double* eta_out, void* stream) {
  DepthPlan* P = static_cast<DepthPlan*>(plan);
  if (!P) return fail(DS3_EINVAL, "depth_get: null plan");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (labels_out)
    DS3_TRY(check_hip(hipMemcpyAsync(labels_out, P->label, sizeof(int32_t) * size_t(P->n_px), hipMemcpyDeviceToDevice, s),
                      "copy labels"));
  if (eta_out)
    DS3_TRY(check_hip(hipMemcpyAsync(eta_out, P->eta, sizeof(double) * size_t(P->n_seg), hipMemcpyDeviceToDevice, s),
                      "copy eta"));
  return DS3_OK;
}

int ds3_depth_plan_set_eta(void* plan, const double* eta, void* stream) {
  DepthPlan* P = static_cast<DepthPlan*>(plan);
  if (!P || !eta) return fail(DS3_EINVAL, "depth_set_eta: bad arguments");
  return check_hip(hipMemcpyAsync(P->eta, eta, sizeof(double) * size_t(P->n_seg), hipMemcpyDeviceToDevice,
                                  static_cast<hipStream_t>(stream)),
                   "copy eta");
}

int ds3_depth_plan_apply(void* plan, float* xyzc_out, void* stream) {
  DepthPlan* P = static_cast<DepthPlan*>(plan);
  if (!P || !xyzc_out) return fail(DS3_EINVAL, "depth_apply: bad arguments");
  if ((reinterpret_cast<uintptr_t>(xyzc_out) & 15) != 0) return fail(DS3_EINVAL, "depth_apply: output not 16 B aligned");
  if (P->n_px == 0) return DS3_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 g(unsigned((P->n_px + kDepthThreads - 1) / kDepthThreads));
  if (P->dt == DS3_F32)
    hipLaunchKernelGGL(k_dr_apply<DS3_F32>, g, dim3(kDepthThreads), 0, s, P->arena, P->n_px, P->label, P->eta,
                       reinterpret_cast<float4*>(xyzc_out));
  else
    hipLaunchKernelGGL(k_dr_apply<DS3_BF16>, g, dim3(kDepthThreads), 0, s, P->arena, P->n_px, P->label, P->eta,
                       reinterpret_cast<float4*>(xyzc_out));
  return check_hip(hipGetLastError(), "k_dr_apply");
}

int ds3_depth_plan_destroy(void* plan) {
  depth_free(static_cast<DepthPlan*>(plan));
  return DS3_OK;
}

}  // extern "C"
