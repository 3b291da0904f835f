// Hand-written adjoint of E_global (eq. 5) with the matches held fixed: gradients with respect to the
// canonical pointmaps, the confidences and a left tangent per pose, recomputing every edge's forward pass
// instead of storing Jacobians.
//
// With r_c = sqrt(q) e_c / sigma_c, q = sqrt(C_i C_j) and rho'(r) = w r (Sec. III-A):
//   gamma_c = dE/de_c = w_c q e_c / sigma_c^2,
//   dE/dx = P gamma_ray / d + gamma_range psi          (x = T_ij X_j, P = I - psi psi^T),
//   dE/dX_j[n] = (s_ij R_ij)^T dE/dx,  dE/dX_i[m] = -(P_i gamma_ray / d_i + gamma_range psi_i),
//   dE/dC = sum_c w_c r_c^2 / (4 C) for both endpoint confidences (r_c scales with (C_i C_j)^(1/4)),
//   dE/dtau_j = Ad^T [dE/dx; x x dE/dx; x . dE/dx] summed over the edge,  dE/dtau_i = -(the same)
//   (the chain of eq. 6 and the -/+Ad endpoint maps; equal to the Gauss-Newton gradient g).
// The pointmap / confidence scatter uses float atomics (many matches of one edge can land on one pixel
// of i, and keyframes belong to several edges).
#include "common.hpp"
#include "internal.hpp"
#include "sim3.hpp"

namespace ds3 {

constexpr int kAdjThreads = 256;
constexpr int kAdjPPT = 8;

template <int DT>
__global__ __launch_bounds__(kAdjThreads) void k_edge_adjoint(
    const void* __restrict__ arena, const EdgeDev* __restrict__ edges, const EdgeXf* __restrict__ xf,
    const int32_t* __restrict__ idx_arena, GnConst k, float dcost, float* __restrict__ grad_xyz,
    float* __restrict__ grad_conf, float* __restrict__ part7) {
  const int e = blockIdx.y;
  const EdgeDev E = edges[e];
  const int tile = blockIdx.x;
  const int tiles_e = (E.npx_j + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  if (tile >= tiles_e) return;  // uniform per block
  float M[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) M[q] = xf[e].m[q];
  float g7[7] = {0, 0, 0, 0, 0, 0, 0};
  const int32_t* idx = idx_arena + E.idx_off;
  for (int u = 0; u < kAdjPPT; ++u) {
    const int64_t n = int64_t(tile) * kAdjThreads * kAdjPPT + int64_t(u) * kAdjThreads + threadIdx.x;
    if (n >= E.npx_j) continue;
    const int32_t m = idx[n];
    if (m < 0 || m >= E.npx_i) continue;
    const float4 Xj = Px<DT>::load(arena, E.off_j + n);
    const float4 Xi = Px<DT>::load(arena, E.off_i + m);
    const float x0 = fmaf(M[0], Xj.x, fmaf(M[1], Xj.y, fmaf(M[2], Xj.z, M[9])));
    const float x1 = fmaf(M[3], Xj.x, fmaf(M[4], Xj.y, fmaf(M[5], Xj.z, M[10])));
    const float x2 = fmaf(M[6], Xj.x, fmaf(M[7], Xj.y, fmaf(M[8], Xj.z, M[11])));
    const float d2 = fmaf(x0, x0, fmaf(x1, x1, x2 * x2));
    const float di2 = fmaf(Xi.x, Xi.x, fmaf(Xi.y, Xi.y, Xi.z * Xi.z));
    const float dj2 = fmaf(Xj.x, Xj.x, fmaf(Xj.y, Xj.y, Xj.z * Xj.z));
    const float cc = Xi.w * Xj.w;
    if (!(d2 > 1e-18f) || !(di2 > 1e-18f) || !(dj2 > 1e-18f) || !(cc >= 0.0f) || !isfinite(d2) ||
        !isfinite(di2) || !isfinite(cc) || !isfinite(dj2))
      continue;
    const float rd = rsqrtf(d2), rdi = rsqrtf(di2);
    const float d = d2 * rd, di = di2 * rdi;
    const float p[3] = {x0 * rd, x1 * rd, x2 * rd};
    const float pi[3] = {Xi.x * rdi, Xi.y * rdi, Xi.z * rdi};
    const float e4[4] = {p[0] - pi[0], p[1] - pi[1], p[2] - pi[2], d - di};
    const float q = sqrtf(cc), sq = sqrtf(q);
    const float isg[4] = {k.inv_sr, k.inv_sr, k.inv_sr, k.inv_sd};
    float gam[4], dc = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float r = sq * e4[c] * isg[c];
      const float a = fabsf(r);
      const float w = (a <= k.kappa) ? 1.0f : k.kappa / a;
      gam[c] = w * r * sq * isg[c] * dcost;
      dc = fmaf(w * r, r, dc);
    }
    dc *= dcost;
    // dE/dx
    const float pg = p[0] * gam[0] + p[1] * gam[1] + p[2] * gam[2];
    float gx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) gx[a] = (gam[a] - p[a] * pg) * rd + gam[3] * p[a];
    // dE/dX_j = (sR)^T gx
    float* gj = grad_xyz + 3 * (E.off_j + n);
    atomicAdd(gj + 0, M[0] * gx[0] + M[3] * gx[1] + M[6] * gx[2]);
    atomicAdd(gj + 1, M[1] * gx[0] + M[4] * gx[1] + M[7] * gx[2]);
    atomicAdd(gj + 2, M[2] * gx[0] + M[5] * gx[1] + M[8] * gx[2]);
    // dE/dX_i
    const float pgi = pi[0] * gam[0] + pi[1] * gam[1] + pi[2] * gam[2];
    float* gi = grad_xyz + 3 * (E.off_i + m);
#pragma unroll
    for (int a = 0; a < 3; ++a) atomicAdd(gi + a, -((gam[a] - pi[a] * pgi) * rdi + gam[3] * pi[a]));
    atomicAdd(grad_conf + E.off_j + n, dc / (4.0f * Xj.w));
    atomicAdd(grad_conf + E.off_i + m, dc / (4.0f * Xi.w));
    // pose tangent pieces [g; x cross g; x . g]
    g7[0] += gx[0];
    g7[1] += gx[1];
    g7[2] += gx[2];
    g7[3] += x1 * gx[2] - x2 * gx[1];
    g7[4] += x2 * gx[0] - x0 * gx[2];
    g7[5] += x0 * gx[1] - x1 * gx[0];
    g7[6] += x0 * gx[0] + x1 * gx[1] + x2 * gx[2];
  }
  __shared__ float red[kAdjThreads / kWave][7];
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    float s = wave_sum(g7[c]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = s;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    float s = 0.0f;
    for (int w = 0; w < kAdjThreads / kWave; ++w) s += red[w][threadIdx.x];
    part7[(int64_t(e) * gridDim.x + tile) * 8 + threadIdx.x] = s;
  }
}

// Per edge: b_e = Ad^T (sum of tile pieces), float64.
__global__ void k_adjoint_edge_finalize(const EdgeDev* __restrict__ edges, int tiles_stride,
                                        const float* __restrict__ part7, const double* __restrict__ Ad,
                                        double* __restrict__ b_e, int n_edges) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_edges) return;
  const EdgeDev E = edges[e];
  const int tiles_e = (E.npx_j + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  double s[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int t = 0; t < tiles_e; ++t)
    for (int c = 0; c < 7; ++c) s[c] += double(part7[(int64_t(e) * tiles_stride + t) * 8 + c]);
  const double* A = Ad + 49 * int64_t(e);
  for (int r = 0; r < 7; ++r) {
    double v = 0.0;
    for (int a = 0; a < 7; ++a) v += A[7 * a + r] * s[a];
    b_e[7 * int64_t(e) + r] = v;
  }
}

// Per keyframe: dE/dtau_k = sum over incident edges (edge order) of +b_e (k = j) or -b_e (k = i).
__global__ void k_grad_tau(int n_kf, const int32_t* __restrict__ node_ptr, const int32_t* __restrict__ node_adj,
                           const double* __restrict__ b_e, double* __restrict__ grad_tau) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 7 * n_kf) return;
  const int k = t / 7, r = t % 7;
  double s = 0.0;
  for (int p = node_ptr[k]; p < node_ptr[k + 1]; ++p) {
    const int code = node_adj[p];
    const double v = b_e[7 * int64_t(code >> 1) + r];
    s += (code & 1) ? v : -v;
  }
  grad_tau[t] = s;
}

int adjoint_part_floats(int n_edges, int max_npx_j) {
  const int tiles = (max_npx_j + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  return n_edges * tiles * 8;
}

int launch_adjoint(ds3_dtype dt, const void* arena, const EdgeDev* edges, int n_edges, int max_npx_j,
                   const EdgeXf* xf, const double* Ad, const int32_t* idx, GnConst c, float dcost,
                   float* grad_xyz, float* grad_conf, float* part7, double* b_e, int n_kf,
                   const int32_t* node_ptr, const int32_t* node_adj, double* grad_tau, ds3_timer* timer,
                   hipStream_t s) {
  const int tiles = (max_npx_j + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  if (n_edges > 0 && tiles > 0) {
    dim3 grid(tiles, n_edges), block(kAdjThreads);
    DS3_TRY(timer_record(timer, true, s));
    if (dt == DS3_F32)
      hipLaunchKernelGGL(k_edge_adjoint<DS3_F32>, grid, block, 0, s, arena, edges, xf, idx, c, dcost, grad_xyz, grad_conf, part7);
    else
      hipLaunchKernelGGL(k_edge_adjoint<DS3_BF16>, grid, block, 0, s, arena, edges, xf, idx, c, dcost, grad_xyz, grad_conf, part7);
    DS3_TRY(check_hip(hipGetLastError(), "k_edge_adjoint"));
    DS3_TRY(timer_record(timer, false, s));
    hipLaunchKernelGGL(k_adjoint_edge_finalize, dim3((n_edges + 63) / 64), dim3(64), 0, s, edges, tiles, part7,
                       Ad, b_e, n_edges);
    DS3_TRY(check_hip(hipGetLastError(), "k_adjoint_edge_finalize"));
  }
  hipLaunchKernelGGL(k_grad_tau, dim3((7 * n_kf + 127) / 128), dim3(128), 0, s, n_kf, node_ptr, node_adj, b_e,
                     grad_tau);
  return check_hip(hipGetLastError(), "k_grad_tau");
}

}  // namespace ds3
