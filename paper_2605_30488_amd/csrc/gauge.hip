// Gauge synchronisation of map components (Sec. III-C): the closed-form similarity of eq. (4) between
// the matches of an admitted edge lifted to world frames, x = T_i X_i[m] and y = T_j X_j[n], with the
// endpoint fallback T* = T_ref T_mov^-1 below N_c^min correspondences; and the left-multiplication of T*
// onto the moving component.
//
// Moments are float64 sums in two passes (centroids, then centred products) over per-block partials
// reduced in block order; the 3x3 SVD is a one-sided Jacobi iteration on the cross-covariance.
#include "common.hpp"
#include "internal.hpp"
#include "sim3.hpp"
#include "umeyama.hpp"

namespace ds3 {

constexpr int kGaugeBlocks = 256;
constexpr int kGaugeThreads = 256;

__device__ inline void world_point(const Sim3& T, const double* R, float4 X, double* w) {
  const double p[3] = {double(X.x), double(X.y), double(X.z)};
  for (int r = 0; r < 3; ++r) w[r] = T.s * (R[3 * r] * p[0] + R[3 * r + 1] * p[1] + R[3 * r + 2] * p[2]) + T.t[r];
}

// pass 0: sums of x, y and the count; pass 1: sums of (x - xb)(y - yb)^T, |y - yb|^2 and |x - xb|^2.
constexpr int kMom = 12;  // accumulator slots per block partial
template <int DT>
__global__ __launch_bounds__(kGaugeThreads) void k_gauge_moments(
    const void* __restrict__ Xi, const void* __restrict__ Xj, int64_t npx_j, int64_t npx_i,
    const int32_t* __restrict__ idx, const uint8_t* __restrict__ valid, const double* __restrict__ poses,
    int i, int j, int pass, const double* __restrict__ centroids, double* __restrict__ partials) {
  const Sim3 Ti = sim3_load(poses + 8 * i), Tj = sim3_load(poses + 8 * j);
  double Ri[9], Rj[9];
  quat_to_mat(Ti.q, Ri);
  quat_to_mat(Tj.q, Rj);
  double acc[11];
  for (int k = 0; k < 11; ++k) acc[k] = 0.0;
  double xb[3] = {0, 0, 0}, yb[3] = {0, 0, 0};
  if (pass == 1)
    for (int k = 0; k < 3; ++k) { xb[k] = centroids[k]; yb[k] = centroids[3 + k]; }
  for (int64_t n = int64_t(blockIdx.x) * kGaugeThreads + threadIdx.x; n < npx_j;
       n += int64_t(gridDim.x) * kGaugeThreads) {
    const int32_t m = idx[n];
    if (!valid[n] || m < 0 || m >= npx_i) continue;
    double x[3], y[3];
    world_point(Ti, Ri, Px<DT>::load(Xi, m), x);
    world_point(Tj, Rj, Px<DT>::load(Xj, n), y);
    if (pass == 0) {
      for (int k = 0; k < 3; ++k) { acc[k] += x[k]; acc[3 + k] += y[k]; }
      acc[6] += 1.0;
    } else {
      double xc[3], yc[3];
      for (int k = 0; k < 3; ++k) { xc[k] = x[k] - xb[k]; yc[k] = y[k] - yb[k]; }
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) acc[3 * r + c] += xc[r] * yc[c];
      acc[9] += yc[0] * yc[0] + yc[1] * yc[1] + yc[2] * yc[2];
      acc[10] += xc[0] * xc[0] + xc[1] * xc[1] + xc[2] * xc[2];
    }
  }
  __shared__ double red[kGaugeThreads / kWave][11];
  for (int k = 0; k < 11; ++k) {
    double s = wave_sum(acc[k]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < 11) {
    double s = 0.0;
    for (int w = 0; w < kGaugeThreads / kWave; ++w) s += red[w][threadIdx.x];
    partials[int64_t(blockIdx.x) * kMom + threadIdx.x] = s;
  }
}

// Sum block partials in block order (single block of 64 threads). out: [0..5] centroids of x and y,
// [6] count, [10..20] pass-1 sums.
// Fixed-order sum of the per-block moments: thread t takes blocks t, t + 256, ..., then a fixed tree.
__global__ __launch_bounds__(256) void k_gauge_reduce(const double* __restrict__ partials, int nblocks,
                                                      int pass, double* __restrict__ out) {
  __shared__ double red[11][256];
  const int t = threadIdx.x;
  double a[11];
  for (int q = 0; q < 11; ++q) a[q] = 0.0;
  for (int b = t; b < nblocks; b += 256)
    for (int q = 0; q < 11; ++q) a[q] += partials[int64_t(b) * kMom + q];
  for (int q = 0; q < 11; ++q) red[q][t] = a[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int q = 0; q < 11; ++q) red[q][t] += red[q][t + w];
    __syncthreads();
  }
  if (t >= 64) return;  // the first wave writes the results
  const int k = t;
  const double s = (k < 11) ? red[k][0] : 0.0;
  if (pass == 0) {
    // centroids x (0..2), y (3..5), count (6)
    const double cnt = __shfl(s, 6, kWave);
    if (k < 6) out[k] = (cnt > 0.0) ? s / cnt : 0.0;
    if (k == 6) out[6] = s;
  } else if (k < 11) {
    out[10 + k] = s;
  }
}

// Solve eq. (4) (or take the endpoint transform) and write T* as a pose.
__global__ void k_gauge_solve(const double* __restrict__ mom, const double* __restrict__ poses, int i,
                              int j, int ref_is_i, int nc_min, double* __restrict__ T_out,
                              int32_t* __restrict__ used) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double cnt = mom[6];
  const int ref = ref_is_i ? i : j, mov = ref_is_i ? j : i;
  bool ok = cnt >= double(nc_min) && cnt > 0.0;
  Sim3 T;
  if (ok) {
    // x in the reference component, y in the moving one
    const double* xb = ref_is_i ? mom : mom + 3;
    const double* yb = ref_is_i ? mom + 3 : mom;
    double A[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        A[3 * r + c] = (ref_is_i ? mom[10 + 3 * r + c] : mom[10 + 3 * c + r]) / cnt;
    // spread of the moving side: |y_j - yb|^2 (slot 19) when j moves, |x_i - xb|^2 (slot 20) when i moves
    const double sy2 = (ref_is_i ? mom[19] : mom[20]) / cnt;
    ok = umeyama_solve(xb, yb, A, sy2, T);
  }
  if (!ok) T = sim3_mul(sim3_load(poses + 8 * ref), sim3_inv(sim3_load(poses + 8 * mov)));
  sim3_store(T, T_out);
  *used = ok ? 1 : 0;
}

__global__ void k_apply_gauge(double* __restrict__ poses, int n, const uint8_t* __restrict__ mask,
                              const double* __restrict__ T) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || !mask[k]) return;
  sim3_store(sim3_mul(sim3_load(T), sim3_load(poses + 8 * int64_t(k))), poses + 8 * int64_t(k));
}

size_t gauge_ws_bytes() {
  Carver c(nullptr);
  c.take<double>(size_t(kGaugeBlocks) * kMom);
  c.take<double>(24);
  return c.used;
}

int launch_gauge_align(const void* Xi, int64_t npx_i, const void* Xj, int64_t npx_j, ds3_dtype dt,
                       const int32_t* idx, const uint8_t* valid, const double* poses, int i, int j,
                       int ref_is_i, int nc_min, double* T_out, int32_t* used, void* ws, hipStream_t s) {
  Carver c(ws);
  double* partials = c.take<double>(size_t(kGaugeBlocks) * kMom);
  double* mom = c.take<double>(24);
  for (int pass = 0; pass < 2; ++pass) {
    if (dt == DS3_F32)
      hipLaunchKernelGGL(k_gauge_moments<DS3_F32>, dim3(kGaugeBlocks), dim3(kGaugeThreads), 0, s, Xi, Xj,
                         npx_j, npx_i, idx, valid, poses, i, j, pass, mom, partials);
    else
      hipLaunchKernelGGL(k_gauge_moments<DS3_BF16>, dim3(kGaugeBlocks), dim3(kGaugeThreads), 0, s, Xi, Xj,
                         npx_j, npx_i, idx, valid, poses, i, j, pass, mom, partials);
    DS3_TRY(check_hip(hipGetLastError(), "k_gauge_moments"));
    hipLaunchKernelGGL(k_gauge_reduce, dim3(1), dim3(256), 0, s, partials, kGaugeBlocks, pass, mom);
    DS3_TRY(check_hip(hipGetLastError(), "k_gauge_reduce"));
  }
  hipLaunchKernelGGL(k_gauge_solve, dim3(1), dim3(64), 0, s, mom, poses, i, j, ref_is_i, nc_min, T_out, used);
  return check_hip(hipGetLastError(), "k_gauge_solve");
}

int launch_apply_gauge(double* poses, int n, const uint8_t* mask, const double* T, hipStream_t s) {
  if (n <= 0) return DS3_OK;
  hipLaunchKernelGGL(k_apply_gauge, dim3((n + 63) / 64), dim3(64), 0, s, poses, n, mask, T);
  return check_hip(hipGetLastError(), "k_apply_gauge");
}

}  // namespace ds3
