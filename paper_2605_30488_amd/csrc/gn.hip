// Graph-step kernels: per-edge pose prep, the fused residual / Jacobian / Huber / Hessian reduction,
// per-edge adjoint transform, block assembly with anchor pinning, cost sum and the Sim(3) update.
//
// Paper map (CoMo3R-SLAM, Sec. III): residual eq. (1); whitening Sigma_mn = Sigma/q_mn with
// Sigma = diag(sigma_r^2 I3, sigma_d^2) and component-wise Huber/IRLS (Sec. III-A, "Ray-range
// tracking"); E_global eq. (5); Jacobian blocks eq. (6) and the endpoint maps -/+ Ad_{T_i^-1} (text after
// eq. 6); normal equations eq. (7); left update T <- Exp(tau) T (Sec. III-D).
//
// Because J_i = -J_j = -J_x Ad, an edge's 14x14 block of J^T W J is [[A, -A], [-A, A]] with
// A = Ad^T H_L Ad, where H_L = sum J_x^T W J_x over the edge's matches. The streaming kernel therefore
// reduces only the 28 unique entries of H_L, the 7 of b_L = J_x^T W e, the cost and the count per tile.
// J_x = [[P/d, -[psi]x, 0], [psi^T, 0, d]] (P = I - psi psi^T) has structural zeros that the
// accumulation skips: column 6 of the ray rows, column 3+c of ray row c, columns 3-5 of the range row.
//
// Calibrated mode (Sec. IV-C, "Calibration"): the same reduction of J_x^T W J_x with the pixel
// reprojection and log-depth residual on the pointmaps constrained to the calibrated rays; with
// iz = 1/x2, px = x0 iz, py = x1 iz, J_x = (dr/dx) [I  -[x]x  x] has the rows
//   u: [fx iz, 0, -fx px iz, -fx px py, fx (1 + px^2), -fx py, 0]
//   v: [0, fy iz, -fy py iz, -fy (1 + py^2), fy px py, fy px, 0]
//   z: [0, 0, iz, py, -px, 0, 1]            (the pixel rows do not see the scale)
#include <cmath>
#include <string>

#include "common.hpp"
#include "internal.hpp"
#include "sim3.hpp"

namespace ds3 {

GnConst make_gn_const(const ds3_gn_params& p) {
  GnConst c;
  c.inv_sr = float(1.0 / p.sigma_ray);
  c.inv_sd = float(1.0 / p.sigma_dist);
  c.inv_sr2 = float(1.0 / (p.sigma_ray * p.sigma_ray));
  c.inv_sd2 = float(1.0 / (p.sigma_dist * p.sigma_dist));
  c.kappa = float(p.huber_k);
  c.inv_sr_d = 1.0 / p.sigma_ray;
  c.inv_sd_d = 1.0 / p.sigma_dist;
  c.kappa_d = p.huber_k;
  const double sp = p.sigma_pix > 0 ? p.sigma_pix : 1.0, sz = p.sigma_logz > 0 ? p.sigma_logz : 1.0;
  c.inv_sp = float(1.0 / sp);
  c.inv_sz = float(1.0 / sz);
  c.inv_sp2 = float(1.0 / (sp * sp));
  c.inv_sz2 = float(1.0 / (sz * sz));
  return c;
}

// --------------------------------------------------------------------------------------------------
// Pose prep: T_ij = T_i^-1 T_j (float32 copy for the residual kernel) and Ad_{T_i^-1} (float64).
// --------------------------------------------------------------------------------------------------
__global__ void k_gn_prep(const double* __restrict__ poses, const EdgeDev* __restrict__ edges,
                          int n_edges, EdgeXf* __restrict__ xf, double* __restrict__ Ad) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_edges) return;
  const EdgeDev E = edges[e];
  Sim3 Ti = sim3_load(poses + 8 * E.i);
  Sim3 Tj = sim3_load(poses + 8 * E.j);
  Sim3 Tinv = sim3_inv(Ti);
  Sim3 Tij = sim3_mul(Tinv, Tj);
  double R[9];
  quat_to_mat(Tij.q, R);
  EdgeXf X;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) X.m[3 * r + c] = float(Tij.s * R[3 * r + c]);
    X.m[9 + r] = float(Tij.t[r]);
  }
  for (int k = 0; k < 4; ++k) X.pad[k] = 0.0f;
  xf[e] = X;
  sim3_adjoint(Tinv, Ad + 49 * int64_t(e));
}

int launch_gn_prep(const double* poses, const EdgeDev* edges, int n_edges, EdgeXf* xf, double* Ad,
                   hipStream_t s) {
  int threads = 128;
  int blocks = (n_edges + threads - 1) / threads;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_gn_prep, dim3(blocks), dim3(threads), 0, s, poses, edges, n_edges, xf, Ad);
  return check_hip(hipGetLastError(), "k_gn_prep");
}

// --------------------------------------------------------------------------------------------------
// Fused residual / Jacobian / Huber / Hessian reduction of one tile of an edge
// --------------------------------------------------------------------------------------------------
#define HIDX(r, c) ((r) * 7 - ((r) * ((r) - 1)) / 2 + ((c) - (r)))

struct Acc {
  float h[28];
  float b[7];
  float cost;
  float cnt;
};

__device__ inline void acc_zero(Acc& a) {
#pragma unroll
  for (int k = 0; k < 28; ++k) a.h[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < 7; ++k) a.b[k] = 0.0f;
  a.cost = 0.0f;
  a.cnt = 0.0f;
}

// Ray row c of J_x: J[0..2] = P_c / d, J[3..5] = row c of -[psi]x (its entry 3+c is zero), J[6] = 0.
template <int Z>
__device__ inline void acc_ray_row(Acc& a, const float* J, float W, float e) {
  float wj[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) wj[k] = (k == Z) ? 0.0f : W * J[k];
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    if (r == Z) continue;
#pragma unroll
    for (int c = r; c < 6; ++c) {
      if (c == Z) continue;
      a.h[HIDX(r, c)] = fmaf(wj[r], J[c], a.h[HIDX(r, c)]);
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    if (k == Z) continue;
    a.b[k] = fmaf(wj[k], e, a.b[k]);
  }
}

// One match after its checks: x = T_ij X_j (d2 = |x|^2 > 0), X_i with di2 = |X_i|^2 > 0 and
// sq = (C_i C_j)^(1/4): e of eq. (1), whitening, Huber weights, J_x, accumulation.
__device__ inline void acc_core(Acc& a, float x0, float x1, float x2, float d2, float xi0, float xi1, float xi2,
                                float di2, float sq, const GnConst& k) {
  const float rd = rsqrtf(d2);
  const float rdi = rsqrtf(di2);
  const float d = d2 * rd;
  const float di = di2 * rdi;
  const float p0 = x0 * rd, p1 = x1 * rd, p2 = x2 * rd;
  const float e0 = p0 - xi0 * rdi;
  const float e1 = p1 - xi1 * rdi;
  const float e2 = p2 - xi2 * rdi;
  const float e3 = d - di;
  // Sigma_mn^-1/2 = sqrt(q) Sigma^-1/2 with q = sqrt(C_i C_j) = sq^2
  const float q = sq * sq;
  const float sr = sq * k.inv_sr;
  const float r0 = sr * e0, r1 = sr * e1, r2 = sr * e2;
  const float r3 = sq * k.inv_sd * e3;
  const float a0 = fabsf(r0), a1 = fabsf(r1), a2 = fabsf(r2), a3 = fabsf(r3);
  // IRLS weight min(1, kappa/|r|); the reciprocal is the hardware one (1 ulp)
  // (min(1, kappa * rcp(|r|)): |r| = 0 gives rcp = inf and weight 1)
  const float w0 = fminf(1.0f, k.kappa * __builtin_amdgcn_rcpf(a0));
  const float w1 = fminf(1.0f, k.kappa * __builtin_amdgcn_rcpf(a1));
  const float w2 = fminf(1.0f, k.kappa * __builtin_amdgcn_rcpf(a2));
  const float w3 = fminf(1.0f, k.kappa * __builtin_amdgcn_rcpf(a3));
  // rho(r) = t (|r| - t/2) with t = w |r|: r^2/2 inside kappa, kappa |r| - kappa^2/2 outside
  const float t0 = w0 * a0, t1 = w1 * a1, t2 = w2 * a2, t3 = w3 * a3;
  a.cost += t0 * fmaf(-0.5f, t0, a0) + t1 * fmaf(-0.5f, t1, a1) + t2 * fmaf(-0.5f, t2, a2) +
            t3 * fmaf(-0.5f, t3, a3);
  a.cnt += 1.0f;
  const float qr = q * k.inv_sr2;
  const float W0 = w0 * qr, W1 = w1 * qr, W2 = w2 * qr, W3 = w3 * q * k.inv_sd2;
  // P/d rows: (delta_ca - psi_c psi_a) / d
  const float s0 = p0 * rd, s1 = p1 * rd, s2 = p2 * rd;
  {
    float J[6] = {rd - s0 * p0, -s0 * p1, -s0 * p2, 0.0f, p2, -p1};
    acc_ray_row<3>(a, J, W0, e0);
  }
  {
    float J[6] = {-s1 * p0, rd - s1 * p1, -s1 * p2, -p2, 0.0f, p0};
    acc_ray_row<4>(a, J, W1, e1);
  }
  {
    float J[6] = {-s2 * p0, -s2 * p1, rd - s2 * p2, p1, -p0, 0.0f};
    acc_ray_row<5>(a, J, W2, e2);
  }
  // range row [psi^T, 0, 0, 0, d]
  {
    const float j0 = W3 * p0, j1 = W3 * p1, j2 = W3 * p2, j6 = W3 * d;
    a.h[HIDX(0, 0)] = fmaf(j0, p0, a.h[HIDX(0, 0)]);
    a.h[HIDX(0, 1)] = fmaf(j0, p1, a.h[HIDX(0, 1)]);
    a.h[HIDX(0, 2)] = fmaf(j0, p2, a.h[HIDX(0, 2)]);
    a.h[HIDX(0, 6)] = fmaf(j0, d, a.h[HIDX(0, 6)]);
    a.h[HIDX(1, 1)] = fmaf(j1, p1, a.h[HIDX(1, 1)]);
    a.h[HIDX(1, 2)] = fmaf(j1, p2, a.h[HIDX(1, 2)]);
    a.h[HIDX(1, 6)] = fmaf(j1, d, a.h[HIDX(1, 6)]);
    a.h[HIDX(2, 2)] = fmaf(j2, p2, a.h[HIDX(2, 2)]);
    a.h[HIDX(2, 6)] = fmaf(j2, d, a.h[HIDX(2, 6)]);
    a.h[HIDX(6, 6)] = fmaf(j6, d, a.h[HIDX(6, 6)]);
    a.b[0] = fmaf(j0, e3, a.b[0]);
    a.b[1] = fmaf(j1, e3, a.b[1]);
    a.b[2] = fmaf(j2, e3, a.b[2]);
    a.b[6] = fmaf(j6, e3, a.b[6]);
  }
}

// x = T_ij X_j with T_ij = [M[0..8] | M[9..11]] (sR row-major, t)
__device__ inline void transform(const float* M, float X0, float X1, float X2, float& x0, float& x1, float& x2) {
  x0 = fmaf(M[0], X0, fmaf(M[1], X1, fmaf(M[2], X2, M[9])));
  x1 = fmaf(M[3], X0, fmaf(M[4], X1, fmaf(M[5], X2, M[10])));
  x2 = fmaf(M[6], X0, fmaf(M[7], X1, fmaf(M[8], X2, M[11])));
}

// The checks of one match that do not depend on the poses: no hole (|X| <= 1e-9, or a NaN or infinity)
// on either side and a non-negative finite confidence product. sq = (C_i C_j)^(1/4) by the hardware
// square root (1 ulp each; the product of confidences is never denormal here).
__device__ inline bool match_static_ok(const float4 Xj, const float4 Xi, float& dj2, float& di2, float& sq) {
  di2 = fmaf(Xi.x, Xi.x, fmaf(Xi.y, Xi.y, Xi.z * Xi.z));
  dj2 = fmaf(Xj.x, Xj.x, fmaf(Xj.y, Xj.y, Xj.z * Xj.z));
  const float cc = Xi.w * Xj.w;
  // a NaN or infinity anywhere makes the sum non-finite
  const float sum = (di2 + dj2) + cc;
  if (!(fminf(di2, dj2) > 1e-18f) || !(cc >= 0.0f) || !(sum < __builtin_huge_valf())) return false;
  sq = __builtin_amdgcn_sqrtf(__builtin_amdgcn_sqrtf(cc));
  return true;
}

// One match from the two arena entries. Returns false (nothing accumulated) for holes, non-finite
// values, zero ranges or a negative confidence product.
__device__ inline bool acc_pixel(Acc& a, const float4 Xj, const float4 Xi, const float* M, const GnConst& k) {
  float dj2, di2, sq;
  if (!match_static_ok(Xj, Xi, dj2, di2, sq)) return false;
  float x0, x1, x2;
  transform(M, Xj.x, Xj.y, Xj.z, x0, x1, x2);
  const float d2 = fmaf(x0, x0, fmaf(x1, x1, x2 * x2));
  if (!(d2 > 1e-18f) || !(d2 < __builtin_huge_valf())) return false;
  acc_core(a, x0, x1, x2, d2, Xi.x, Xi.y, Xi.z, di2, sq, k);
  return true;
}

// One residual row J (7 entries, nonzero only where MASK has a bit) with weight W and residual e:
// H_L += W J^T J (upper triangle), b_L += W J^T e.
template <unsigned MASK>
__device__ inline void acc_row(Acc& a, const float* J, float W, float e) {
  float wj[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) wj[k] = ((MASK >> k) & 1u) ? W * J[k] : 0.0f;
#pragma unroll
  for (int r = 0; r < 7; ++r) {
    if (!((MASK >> r) & 1u)) continue;
#pragma unroll
    for (int c = r; c < 7; ++c) {
      if (!((MASK >> c) & 1u)) continue;
      a.h[HIDX(r, c)] = fmaf(wj[r], J[c], a.h[HIDX(r, c)]);
    }
    a.b[r] = fmaf(wj[r], e, a.b[r]);
  }
}

// Calibrated mode, one match after its pose-independent checks: x = T_ij Xcal_j (x2 > 1e-9), target pixel
// (um, vm) of keyframe i and izm = 1/z_i[m], sq = (C_i C_j)^(1/4), K_i = (fx, fy, cx, cy). Nothing is
// accumulated unless the reprojection lands on keyframe i's image: -0.5 <= u < W_i - 0.5 (lim.x = W_i - 0.5)
// and likewise v with H_i (lim.y).
__device__ inline void acc_core_cal(Acc& a, float x0, float x1, float x2, float um, float vm, float izm, float sq,
                                    const float4 Ki, const float2 lim, const GnConst& k) {
  const float iz = __builtin_amdgcn_rcpf(x2);
  const float px = x0 * iz, py = x1 * iz;
  const float pu = fmaf(Ki.x, px, Ki.z), pv = fmaf(Ki.y, py, Ki.w);
  if (!(pu >= -0.5f && pu < lim.x && pv >= -0.5f && pv < lim.y)) return;
  const float e0 = pu - um;
  const float e1 = pv - vm;
  const float e2 = logf(x2 * izm);
  const float q = sq * sq;
  const float sp = sq * k.inv_sp;
  const float r0 = sp * e0, r1 = sp * e1, r2 = sq * k.inv_sz * e2;
  const float a0 = fabsf(r0), a1 = fabsf(r1), a2 = fabsf(r2);
  const float w0 = fminf(1.0f, k.kappa * __builtin_amdgcn_rcpf(a0));
  const float w1 = fminf(1.0f, k.kappa * __builtin_amdgcn_rcpf(a1));
  const float w2 = fminf(1.0f, k.kappa * __builtin_amdgcn_rcpf(a2));
  const float t0 = w0 * a0, t1 = w1 * a1, t2 = w2 * a2;
  a.cost += t0 * fmaf(-0.5f, t0, a0) + t1 * fmaf(-0.5f, t1, a1) + t2 * fmaf(-0.5f, t2, a2);
  a.cnt += 1.0f;
  const float qp = q * k.inv_sp2;
  const float fx = Ki.x, fy = Ki.y;
  {
    const float J[7] = {fx * iz, 0.0f, -fx * px * iz, -fx * px * py, fmaf(fx * px, px, fx), -fx * py, 0.0f};
    acc_row<0x3Du>(a, J, w0 * qp, e0);
  }
  {
    const float J[7] = {0.0f, fy * iz, -fy * py * iz, -fmaf(fy * py, py, fy), fy * px * py, fy * px, 0.0f};
    acc_row<0x3Eu>(a, J, w1 * qp, e1);
  }
  {
    const float J[7] = {0.0f, 0.0f, iz, py, -px, 0.0f, 1.0f};
    acc_row<0x5Cu>(a, J, w2 * q * k.inv_sz2, e2);
  }
}

// Pose-independent checks of the calibrated mode: no hole, a non-negative finite confidence product and
// both depths above 1e-9.
__device__ inline bool cal_static_ok(const float4 Xj, const float4 Xi, float& sq) {
  float dj2, di2;
  if (!match_static_ok(Xj, Xi, dj2, di2, sq)) return false;
  return Xj.z > 1e-9f && Xi.z > 1e-9f;
}

// The calibrated point of pixel n of keyframe j: z_j (u_n - cx_j, v_n - cy_j) / (fx_j, fy_j), z_j.
__device__ inline void cal_point(float zj, int n, const EdgeCal& C, float& X0, float& X1) {
  const int vn = n / C.Wj, un = n - vn * C.Wj;
  X0 = zj * ((float(un) - C.cxj) * C.ifxj);
  X1 = zj * ((float(vn) - C.cyj) * C.ifyj);
}

// Plain form, calibrated mode: one match (n of j, m of i) from the two arena entries.
__device__ inline void acc_pixel_cal(Acc& a, const float4 Xj, const float4 Xi, int n, int m, const float* M,
                                     const EdgeCal& C, const GnConst& k) {
  float sq;
  if (!cal_static_ok(Xj, Xi, sq)) return;
  float X0, X1;
  cal_point(Xj.z, n, C, X0, X1);
  float x0, x1, x2;
  transform(M, X0, X1, Xj.z, x0, x1, x2);
  if (!(x2 > 1e-9f) || !(x2 < __builtin_huge_valf()) || !isfinite(x0) || !isfinite(x1)) return;
  const int vm = m / C.Wi, um = m - vm * C.Wi;
  acc_core_cal(a, x0, x1, x2, float(um), float(vm), 1.0f / Xi.z, sq, make_float4(C.fxi, C.fyi, C.cxi, C.cyi),
               make_float2(float(C.Wi) - 0.5f, float(C.Hi) - 0.5f), k);
}

// Wave reduce-scatter of the 37 accumulators in six halvings. In each step a lane and its partner (lane
// l^32, l^16, l^8, l^7 (the mirror within eight lanes), l^2, l^1) hold the same list of partial sums; the
// lane whose bit of the step is set keeps the upper part of the list (entries h .. L-1, h = ceil(L/2)), the
// other the lower part, and each adds its partner's copy of the part it keeps. The first two exchanges are
// the gfx950 lane-half swaps, the other four DPP moves. After the last step every lane holds the wave's
// total of one accumulator (its slot) or padding (slot -1): 40 exchanges and adds instead of 37 full-wave
// sums of six DPP adds each.
__device__ inline float swap32_sum(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ inline float swap16_sum(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// keeps `hi` when `upper`, else `lo`, plus the partner's copy of the same entry (DPP control CTRL)
template <int CTRL>
__device__ inline float dpp_pair_sum(float lo, float hi, bool upper) {
  const float keep = upper ? hi : lo, send = upper ? lo : hi;
  return keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), CTRL, 0xf, 0xf, true));
}

__device__ inline float acc_reduce_scatter(const Acc& a, int lane, int& slot) {
  const float* v = reinterpret_cast<const float*>(&a);
  float w1[19], w2[10], w3[5], w4[3], w5[2];
#pragma unroll
  for (int k = 0; k < 19; ++k) w1[k] = swap32_sum(v[k], k + 19 < 37 ? v[k + 19] : 0.0f);
#pragma unroll
  for (int k = 0; k < 10; ++k) w2[k] = swap16_sum(w1[k], k + 10 < 19 ? w1[k + 10] : 0.0f);
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
#pragma unroll
  for (int k = 0; k < 5; ++k) w3[k] = dpp_pair_sum<0x128>(w2[k], k + 5 < 10 ? w2[k + 5] : 0.0f, b3);  // row_ror:8
#pragma unroll
  for (int k = 0; k < 3; ++k) w4[k] = dpp_pair_sum<0x141>(w3[k], k + 3 < 5 ? w3[k + 3] : 0.0f, b2);  // row_half_mirror
#pragma unroll
  for (int k = 0; k < 2; ++k) w5[k] = dpp_pair_sum<0x4e>(w4[k], k + 2 < 3 ? w4[k + 2] : 0.0f, b1);  // quad_perm [2,3,0,1]
  const float tot = dpp_pair_sum<0xb1>(w5[0], w5[1], b0);                                            // quad_perm [1,0,3,2]
  // the entry a lane ends with: its kept offsets, last step first; padding once a kept entry is past a list
  int s = b0 ? 1 : 0;
  bool ok = true;
  s += b1 ? 2 : 0;
  ok = ok && s < 3;
  s += b2 ? 3 : 0;
  ok = ok && s < 5;
  s += b3 ? 5 : 0;
  ok = ok && s < 10;
  s += (lane & 16) ? 10 : 0;
  ok = ok && s < 19;
  s += (lane & 32) ? 19 : 0;
  ok = ok && s < 37;
  slot = ok ? s : -1;
  return tot;
}

// Block reduction of the 37 accumulators in a fixed order; threads 0..36 write the tile partial.
__device__ inline void acc_block_store(Acc& a, float* __restrict__ out, float (*lds)[37]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  int slot;
  const float t = acc_reduce_scatter(a, lane, slot);
  if (slot >= 0) lds[wave][slot] = t;
  __syncthreads();
  if (threadIdx.x < kPartial) {
    float s = 0.0f;
    if (threadIdx.x < 37) {
#pragma unroll
      for (int w = 0; w < kReduceThreads / kWave; ++w) s += lds[w][threadIdx.x];
    }
    out[threadIdx.x] = s;
  }
}

// Per-wave queue of matched (n, m) pairs in LDS: a ring of kQueue entries that each wave fills from its
// scanned pixels and drains in rounds of 64, so that every lane of a round computes a valid match
// (the scanned tile holds holes, unmatched pixels and band edges that would otherwise idle lanes).
constexpr int kScanU = 4;    // scanned pixels per lane per refill
// One round of 64 matches per drain batch: deeper batches keep more gathers in flight per wave but cost
// registers, and the kernel gains more from occupancy (71 VGPRs, 7 waves per SIMD: 0.42 ms per launch on
// the batched graph, against 0.43 ms with two rounds, 0.45 ms with four and 0.49 ms with eight).
constexpr int kRounds = 1;   // rounds of 64 matches per drain batch (2 gathers each in flight per lane)
constexpr int kQueue = 512;  // >= 64 * (kScanU + kRounds), a power of two
static_assert(kQueue >= 64 * (kScanU + kRounds) && (kQueue & (kQueue - 1)) == 0, "queue size");

template <int DT, int MODE>
__device__ inline void drain_rounds(Acc& a, const void* __restrict__ arena, const EdgeDev& E, const int2* q,
                                    unsigned& head, unsigned avail, const float* M, const GnConst& k,
                                    const EdgeCal& C) {
  using raw_t = typename Px<DT>::raw_t;
  const int lane = threadIdx.x & (kWave - 1);
  int2 e[kRounds];
  raw_t rj[kRounds], ri[kRounds];
  bool ok[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    ok[r] = unsigned(r * kWave + lane) < avail;
    e[r] = ok[r] ? q[(head + r * kWave + lane) & (kQueue - 1)] : make_int2(0, 0);
  }
#pragma unroll
  for (int r = 0; r < kRounds; ++r)
    if (ok[r]) {
      rj[r] = Px<DT>::load_raw(arena, E.off_j + e[r].x);
      ri[r] = Px<DT>::load_raw(arena, E.off_i + e[r].y);
    }
#pragma unroll
  for (int r = 0; r < kRounds; ++r)
    if (ok[r]) {
      if constexpr (MODE == kCalibrated)
        acc_pixel_cal(a, Px<DT>::unpack(rj[r]), Px<DT>::unpack(ri[r]), e[r].x, e[r].y, M, C, k);
      else
        acc_pixel(a, Px<DT>::unpack(rj[r]), Px<DT>::unpack(ri[r]), M, k);
    }
  head += min(avail, unsigned(kRounds * kWave));
}

template <int DT, int PPT, int MODE>
__device__ inline void reduce_tile(const void* __restrict__ arena, const EdgeDev& E, int tile,
                                   const float* M, const int32_t* __restrict__ idx_arena,
                                   float* __restrict__ out, const GnConst& k, float (*lds)[37],
                                   int2* __restrict__ queue, const EdgeCal& C) {
  static_assert(PPT % kScanU == 0, "pixels per thread must be a multiple of the scan unroll");
  Acc a;
  acc_zero(a);
  const int64_t base = int64_t(tile) * (kReduceThreads * PPT);
  const int32_t* __restrict__ idx = idx_arena + E.idx_off;
  int2* q = queue + (threadIdx.x / kWave) * kQueue;
  unsigned head = 0, tail = 0;  // wave-uniform
  // the matches of the next scan unit are loaded before the current one is drained, so that their
  // latency overlaps the gathers and the arithmetic of the drain
  auto load_matches = [&](int k0, int32_t* m) {
#pragma unroll
    for (int u = 0; u < kScanU; ++u) {
      const int64_t n = base + int64_t(k0 + u) * kReduceThreads + threadIdx.x;
      m[u] = (n < E.npx_j) ? __builtin_nontemporal_load(idx + n) : -1;
    }
  };
  int32_t m[kScanU];
  load_matches(0, m);
#pragma unroll 1
  for (int k0 = 0; k0 < PPT; k0 += kScanU) {
#pragma unroll
    for (int u = 0; u < kScanU; ++u)
      if (m[u] >= E.npx_i) m[u] = -1;
#pragma unroll
    for (int u = 0; u < kScanU; ++u) {
      const bool valid = m[u] >= 0;
      const uint64_t ballot = __ballot(valid);
      if (valid) {
        const unsigned below = __builtin_amdgcn_mbcnt_hi(uint32_t(ballot >> 32),
                                                         __builtin_amdgcn_mbcnt_lo(uint32_t(ballot), 0u));
        const int n = int(base + int64_t(k0 + u) * kReduceThreads + threadIdx.x);
        q[(tail + below) & (kQueue - 1)] = make_int2(n, m[u]);
      }
      tail += unsigned(__popcll(ballot));
    }
    if (k0 + kScanU < PPT) load_matches(k0 + kScanU, m);
    __builtin_amdgcn_wave_barrier();  // the wave's queue writes are ordered before its reads
    while (tail - head >= unsigned(kRounds * kWave))
      drain_rounds<DT, MODE>(a, arena, E, q, head, kRounds * kWave, M, k, C);
  }
  while (tail != head) drain_rounds<DT, MODE>(a, arena, E, q, head, tail - head, M, k, C);
  acc_block_store(a, out, lds);
}

// Plain form: one launch per edge, one block per tile.
template <int DT, int PPT, int MODE>
__global__ __launch_bounds__(kReduceThreads) void k_edge_reduce_one(
    const void* __restrict__ arena, EdgeDev E, int edge_id, const EdgeXf* __restrict__ xf,
    const int32_t* __restrict__ idx_arena, float* __restrict__ partials, GnConst k, EdgeCal C) {
  __shared__ float lds[kReduceThreads / kWave][37];
  __shared__ int2 queue[kReduceThreads / kWave * kQueue];
  float M[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) M[q] = xf[edge_id].m[q];
  reduce_tile<DT, PPT, MODE>(arena, E, blockIdx.x, M, idx_arena,
                             partials + int64_t(E.tile0 + blockIdx.x) * kPartial, k, lds, queue, C);
}

// --------------------------------------------------------------------------------------------------
// Match stream of the batched form. The matches and the pointmaps stay fixed while the GN iterations move
// the poses, so the plan gathers, once per set of matches, each valid match's two pointmap entries into
// one contiguous record in the edge's segment of a stream; every iteration then reads the stream with
// plain coalesced loads instead of scanning the match map and gathering the reference point.
//   BF16 record (16 B): X_j (3 bf16), X_i (3 bf16), sq = (C_i C_j)^(1/4) (float32)
//   F32 record (32 B):  X_j (3 float32), X_i (3 float32), sq (float32), one pad
// The bf16 values are the arena's own bits, so the stream holds exactly the stored inputs. Segment s of
// edge e covers pixels [s*seg_px, (s+1)*seg_px) of keyframe j; its records sit at the start of slot
// range [(tile0 + s) * seg_px, ...) in increasing pixel order, and seg_count holds how many there are.
// --------------------------------------------------------------------------------------------------
template <int DT>
struct Rec;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <>
struct Rec<DS3_BF16> {
  struct raw_t {
    u32x4 w;
  };
  __device__ static inline raw_t make(uint2 rj, uint2 ri, float sq) {
    raw_t r;
    r.w = u32x4{rj.x, (rj.y & 0xffffu) | (ri.x << 16), (ri.x >> 16) | (ri.y << 16), __float_as_uint(sq)};
    return r;
  }
  __device__ static inline raw_t load(const raw_t* p) {
    raw_t r;
    r.w = __builtin_nontemporal_load(&p->w);
    return r;
  }
  __device__ static inline void unpack(const raw_t& r, float* xj, float* xi, float& sq) {
    xj[0] = bf16_lo(r.w.x); xj[1] = bf16_hi(r.w.x); xj[2] = bf16_lo(r.w.y);
    xi[0] = bf16_hi(r.w.y); xi[1] = bf16_lo(r.w.z); xi[2] = bf16_hi(r.w.z);
    sq = __uint_as_float(r.w.w);
  }
};

template <>
struct Rec<DS3_F32> {
  struct raw_t {
    f32x4 a, b;
  };
  __device__ static inline raw_t make(float4 Xj, float4 Xi, float sq) {
    raw_t r;
    r.a = f32x4{Xj.x, Xj.y, Xj.z, Xi.x};
    r.b = f32x4{Xi.y, Xi.z, sq, 0.0f};
    return r;
  }
  __device__ static inline raw_t load(const raw_t* p) {
    raw_t r;
    r.a = __builtin_nontemporal_load(&p->a);
    r.b = __builtin_nontemporal_load(&p->b);
    return r;
  }
  __device__ static inline void unpack(const raw_t& r, float* xj, float* xi, float& sq) {
    xj[0] = r.a.x; xj[1] = r.a.y; xj[2] = r.a.z;
    xi[0] = r.a.w; xi[1] = r.b.x; xi[2] = r.b.y;
    sq = r.b.z;
  }
};

template <int DT>
__device__ inline typename Rec<DT>::raw_t make_rec(typename Px<DT>::raw_t rj, typename Px<DT>::raw_t ri, float sq);
template <>
__device__ inline Rec<DS3_BF16>::raw_t make_rec<DS3_BF16>(uint2 rj, uint2 ri, float sq) {
  return Rec<DS3_BF16>::make(rj, ri, sq);
}
template <>
__device__ inline Rec<DS3_F32>::raw_t make_rec<DS3_F32>(float4 rj, float4 ri, float sq) {
  return Rec<DS3_F32>::make(rj, ri, sq);
}

constexpr int kGatherUnroll = 4;  // 256-pixel chunks whose loads are issued together

// One block per segment: scans the segment's matches in pixel order, keeps those that pass the
// pose-independent checks and writes their records compacted (order-preserving: ballot ranks within a
// wave, wave totals through LDS), then the count. Calibrated mode (MODE == kCalibrated, ecal per edge):
// float32 records of the calibrated point Xcal_j[n] and the target (u_m, v_m, 1/z_i[m]).
template <int DT, int MODE>
__global__ __launch_bounds__(kReduceThreads) void k_gather_stream(const void* __restrict__ arena,
                                                                  const EdgeDev* __restrict__ edges,
                                                                  const WorkItem* __restrict__ items,
                                                                  const int32_t* __restrict__ idx_arena,
                                                                  int seg_px, void* __restrict__ stream,
                                                                  int32_t* __restrict__ seg_count,
                                                                  const EdgeCal* __restrict__ ecal) {
  using raw_t = typename Px<DT>::raw_t;
  constexpr int RDT = MODE == kCalibrated ? int(DS3_F32) : DT;
  using rec_t = typename Rec<RDT>::raw_t;
  __shared__ int s_tot[kGatherUnroll][kReduceThreads / kWave];
  const WorkItem W = items[blockIdx.x];
  const EdgeDev E = edges[W.edge];
  const int seg = E.tile0 + W.tile;
  rec_t* __restrict__ out = static_cast<rec_t*>(stream) + int64_t(seg) * seg_px;
  const int32_t* __restrict__ idx = idx_arena + E.idx_off;
  const int64_t base = int64_t(W.tile) * seg_px;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  EdgeCal C{};
  if constexpr (MODE == kCalibrated) C = ecal[W.edge];
  int running = 0;  // block-uniform
  for (int c0 = 0; c0 < seg_px; c0 += kReduceThreads * kGatherUnroll) {
    int32_t m[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      const int64_t n = base + c0 + u * kReduceThreads + threadIdx.x;
      const bool in = (c0 + u * kReduceThreads + int(threadIdx.x) < seg_px) && n < E.npx_j;
      m[u] = in ? __builtin_nontemporal_load(idx + n) : -1;
      if (m[u] >= E.npx_i) m[u] = -1;
    }
    raw_t rj[kGatherUnroll], ri[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u)
      if (m[u] >= 0) {
        const int64_t n = base + c0 + u * kReduceThreads + threadIdx.x;
        rj[u] = Px<DT>::load_raw(arena, E.off_j + n);
        ri[u] = Px<DT>::load_raw(arena, E.off_i + m[u]);
      }
    bool ok[kGatherUnroll];
    float sq[kGatherUnroll];
    unsigned rank[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      ok[u] = false;
      sq[u] = 0.0f;
      if (m[u] >= 0) {
        if constexpr (MODE == kCalibrated) {
          ok[u] = cal_static_ok(Px<DT>::unpack(rj[u]), Px<DT>::unpack(ri[u]), sq[u]);
        } else {
          float dj2, di2;
          ok[u] = match_static_ok(Px<DT>::unpack(rj[u]), Px<DT>::unpack(ri[u]), dj2, di2, sq[u]);
        }
      }
      const uint64_t ballot = __ballot(ok[u]);
      rank[u] = __builtin_amdgcn_mbcnt_hi(uint32_t(ballot >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(ballot), 0u));
      if (lane == 0) s_tot[u][wave] = __popcll(ballot);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      int off = running;
      for (int w = 0; w < kReduceThreads / kWave; ++w) {
        const int t = s_tot[u][w];
        if (w < wave) off += t;
        running += t;
      }
      if (ok[u]) {
        if constexpr (MODE == kCalibrated) {
          const int n = int(base + c0 + u * kReduceThreads + threadIdx.x);
          const float4 Xj = Px<DT>::unpack(rj[u]), Xi = Px<DT>::unpack(ri[u]);
          float X0, X1;
          cal_point(Xj.z, n, C, X0, X1);
          const int vm = m[u] / C.Wi, um = m[u] - vm * C.Wi;
          // record: (X0, X1, z_j, u_m), (v_m, 1/z_i[m], sq, 0)
          out[off + int(rank[u])] = Rec<DS3_F32>::make(make_float4(X0, X1, Xj.z, 0.0f),
                                                       make_float4(float(um), float(vm), 1.0f / Xi.z, 0.0f), sq[u]);
        } else {
          out[off + int(rank[u])] = make_rec<DT>(rj[u], ri[u], sq[u]);
        }
      }
    }
    __syncthreads();  // s_tot is rewritten by the next chunk
  }
  if (threadIdx.x == 0) seg_count[seg] = running;
}

// E of one match in float64 (eq. (1), whitening and Huber as acc_core) from the stored values and a
// float64 T_ij; used where a decision compares two costs that differ by less than float32 resolves.
__device__ inline double rsqrt_f64(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}

__device__ inline double cost_f64(const double* T, const float* xj, const float* xi, float sq, const GnConst& k) {
  const double X0 = xj[0], X1 = xj[1], X2 = xj[2];
  const double x0 = T[0] * X0 + T[1] * X1 + T[2] * X2 + T[9];
  const double x1 = T[3] * X0 + T[4] * X1 + T[5] * X2 + T[10];
  const double x2 = T[6] * X0 + T[7] * X1 + T[8] * X2 + T[11];
  const double y0 = xi[0], y1 = xi[1], y2 = xi[2];
  // 1/|x| from the hardware estimate refined by two Newton steps (to the last bits; the accept test needs
  // ~1e-12), |x| = |x|^2 / |x|: no square root and no division per point
  const double d2 = x0 * x0 + x1 * x1 + x2 * x2, di2 = y0 * y0 + y1 * y1 + y2 * y2;
  const double rd = rsqrt_f64(d2), rdi = rsqrt_f64(di2);
  const double d = d2 * rd, di = di2 * rdi;
  const double e[4] = {x0 * rd - y0 * rdi, x1 * rd - y1 * rdi, x2 * rd - y2 * rdi, d - di};
  const double s = double(sq);
  const double kap = k.kappa_d;
  double c = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double r = fabs(s * e[q] * (q < 3 ? k.inv_sr_d : k.inv_sd_d));
    c += r <= kap ? 0.5 * r * r : kap * r - 0.5 * kap * kap;
  }
  return c;
}

// One block per segment: the segment's records with `unroll` loads in flight per thread, accumulated
// as in the plain form, reduced over the block in a fixed order into the segment's partial. Segments of
// edges flagged in skip (may be NULL) are left alone. C64: the segment's cost is also evaluated in float64
// at the float64 transform xf64[edge] (12 doubles, sR row-major then t) and written to cost64[segment].
// MODE == kCalibrated: float32 records of the calibrated mode (DT must be DS3_F32), K_i from ecal[edge].
template <int DT, int U, bool C64, int MODE>
__global__ __launch_bounds__(kReduceThreads) void k_reduce_stream(const void* __restrict__ stream,
                                                                  const int32_t* __restrict__ seg_count,
                                                                  const EdgeDev* __restrict__ edges,
                                                                  const WorkItem* __restrict__ items,
                                                                  const EdgeXf* __restrict__ xf, int seg_px,
                                                                  float* __restrict__ partials, GnConst k,
                                                                  const int32_t* __restrict__ skip,
                                                                  const double* __restrict__ xf64,
                                                                  double* __restrict__ cost64,
                                                                  const EdgeCal* __restrict__ ecal) {
  static_assert(MODE == kRayRange || (DT == DS3_F32 && !C64), "calibrated records are float32, no float64 cost");
  using rec_t = typename Rec<DT>::raw_t;
  __shared__ float lds[kReduceThreads / kWave][37];
  __shared__ double lds64[kReduceThreads / kWave];
  const WorkItem W = items[blockIdx.x];
  if (skip && skip[W.edge]) return;  // edges whose caller no longer needs their sums (block-uniform)
  const EdgeDev E = edges[W.edge];
  const int seg = E.tile0 + W.tile;
  float M[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) M[q] = xf[W.edge].m[q];
  double M64[C64 ? 12 : 1];
  if constexpr (C64) {
#pragma unroll
    for (int q = 0; q < 12; ++q) M64[q] = xf64[12 * int64_t(W.edge) + q];
  }
  float4 Ki = make_float4(0.f, 0.f, 0.f, 0.f);
  float2 lim = make_float2(0.f, 0.f);
  if constexpr (MODE == kCalibrated) {
    const EdgeCal C = ecal[W.edge];
    Ki = make_float4(C.fxi, C.fyi, C.cxi, C.cyi);
    lim = make_float2(float(C.Wi) - 0.5f, float(C.Hi) - 0.5f);
  }
  double c64 = 0.0;
  const rec_t* __restrict__ in = static_cast<const rec_t*>(stream) + int64_t(seg) * seg_px;
  const int cnt = seg_count[seg];
  Acc a;
  acc_zero(a);
  // U records in flight per thread: a ring of U registers, each refilled with the record U groups ahead as
  // soon as its current record has been taken, so that U loads are outstanding while one record is computed
  // (deeper rings cost 4 registers per record, not a second copy of the arithmetic's registers)
  rec_t buf[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = u * kReduceThreads + int(threadIdx.x);
    if (q < cnt) buf[u] = Rec<DT>::load(in + q);
  }
#pragma unroll 1
  for (int k0 = 0; k0 < cnt; k0 += kReduceThreads * U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = k0 + u * kReduceThreads + int(threadIdx.x);
      const rec_t r = buf[u];
      if (q + kReduceThreads * U < cnt) buf[u] = Rec<DT>::load(in + q + kReduceThreads * U);
      if (q < cnt) {
        float xj[3], xi[3], sq;
        Rec<DT>::unpack(r, xj, xi, sq);
        float x0, x1, x2;
        transform(M, xj[0], xj[1], xj[2], x0, x1, x2);
        if constexpr (MODE == kCalibrated) {
          // xi holds the target (u_m, v_m, 1/z_i[m])
          if (x2 > 1e-9f && x2 < __builtin_huge_valf() && isfinite(x0) && isfinite(x1))
            acc_core_cal(a, x0, x1, x2, xi[0], xi[1], xi[2], sq, Ki, lim, k);
        } else {
          const float d2 = fmaf(x0, x0, fmaf(x1, x1, x2 * x2));
          if (d2 > 1e-18f && d2 < __builtin_huge_valf()) {
            const float di2 = fmaf(xi[0], xi[0], fmaf(xi[1], xi[1], xi[2] * xi[2]));
            acc_core(a, x0, x1, x2, d2, xi[0], xi[1], xi[2], di2, sq, k);
            if constexpr (C64) c64 += cost_f64(M64, xj, xi, sq, k);
          }
        }
      }
    }
  }
  acc_block_store(a, partials + int64_t(seg) * kPartial, lds);
  if constexpr (C64) {
    const double s = wave_sum(c64);
    if ((threadIdx.x & (kWave - 1)) == 0) lds64[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kReduceThreads / kWave; ++w) t += lds64[w];
      cost64[seg] = t;
    }
  }
}

size_t stream_record_bytes(ds3_dtype dt, bool calibrated) {
  return (dt == DS3_F32 || calibrated) ? sizeof(Rec<DS3_F32>::raw_t) : sizeof(Rec<DS3_BF16>::raw_t);
}

int launch_gather_stream(ds3_dtype dt, const void* arena, const EdgeDev* edges, const WorkItem* items,
                         int n_items, const int32_t* idx_arena, int seg_px, void* stream, int32_t* seg_count,
                         hipStream_t s, const EdgeCal* ecal) {
  if (n_items <= 0) return DS3_OK;
  dim3 g(n_items), b(kReduceThreads);
  if (ecal) {
    if (dt == DS3_F32)
      hipLaunchKernelGGL((k_gather_stream<DS3_F32, kCalibrated>), g, b, 0, s, arena, edges, items, idx_arena, seg_px,
                         stream, seg_count, ecal);
    else
      hipLaunchKernelGGL((k_gather_stream<DS3_BF16, kCalibrated>), g, b, 0, s, arena, edges, items, idx_arena, seg_px,
                         stream, seg_count, ecal);
  } else {
    if (dt == DS3_F32)
      hipLaunchKernelGGL((k_gather_stream<DS3_F32, kRayRange>), g, b, 0, s, arena, edges, items, idx_arena, seg_px,
                         stream, seg_count, nullptr);
    else
      hipLaunchKernelGGL((k_gather_stream<DS3_BF16, kRayRange>), g, b, 0, s, arena, edges, items, idx_arena, seg_px,
                         stream, seg_count, nullptr);
  }
  return check_hip(hipGetLastError(), "k_gather_stream");
}

template <int DT, bool C64, int MODE>
static int launch_reduce_stream_dt(int unroll, const void* stream, const int32_t* seg_count, const EdgeDev* edges,
                                   const WorkItem* items, int n_items, const EdgeXf* xf, int seg_px,
                                   float* partials, GnConst c, const int32_t* skip, const double* xf64,
                                   double* cost64, const EdgeCal* ecal, hipStream_t s) {
  dim3 g(n_items), b(kReduceThreads);
  switch (unroll) {
    case 1: hipLaunchKernelGGL((k_reduce_stream<DT, 1, C64, MODE>), g, b, 0, s, stream, seg_count, edges, items, xf, seg_px, partials, c, skip, xf64, cost64, ecal); break;
    case 2: hipLaunchKernelGGL((k_reduce_stream<DT, 2, C64, MODE>), g, b, 0, s, stream, seg_count, edges, items, xf, seg_px, partials, c, skip, xf64, cost64, ecal); break;
    case 4: hipLaunchKernelGGL((k_reduce_stream<DT, 4, C64, MODE>), g, b, 0, s, stream, seg_count, edges, items, xf, seg_px, partials, c, skip, xf64, cost64, ecal); break;
    default: return fail(DS3_EINVAL, "unsupported stream unroll");
  }
  return check_hip(hipGetLastError(), "k_reduce_stream");
}

int launch_reduce_stream(ds3_dtype dt, int unroll, const void* stream, const int32_t* seg_count,
                         const EdgeDev* edges, const WorkItem* items, int n_items, const EdgeXf* xf, int seg_px,
                         float* partials, GnConst c, const int32_t* skip, hipStream_t s, const double* xf64,
                         double* cost64, const EdgeCal* ecal) {
  if (n_items <= 0) return DS3_OK;
  if ((xf64 == nullptr) != (cost64 == nullptr)) return fail(DS3_EINVAL, "float64 cost needs both buffers");
  if (ecal) {
    if (xf64) return fail(DS3_ENOTSUP, "calibrated mode has no float64 cost");
    return launch_reduce_stream_dt<DS3_F32, false, kCalibrated>(unroll, stream, seg_count, edges, items, n_items, xf,
                                                                seg_px, partials, c, skip, nullptr, nullptr, ecal, s);
  }
  if (dt == DS3_F32)
    return xf64 ? launch_reduce_stream_dt<DS3_F32, true, kRayRange>(unroll, stream, seg_count, edges, items, n_items,
                                                                    xf, seg_px, partials, c, skip, xf64, cost64,
                                                                    nullptr, s)
                : launch_reduce_stream_dt<DS3_F32, false, kRayRange>(unroll, stream, seg_count, edges, items, n_items,
                                                                     xf, seg_px, partials, c, skip, nullptr, nullptr,
                                                                     nullptr, s);
  return xf64 ? launch_reduce_stream_dt<DS3_BF16, true, kRayRange>(unroll, stream, seg_count, edges, items, n_items, xf,
                                                                   seg_px, partials, c, skip, xf64, cost64, nullptr, s)
              : launch_reduce_stream_dt<DS3_BF16, false, kRayRange>(unroll, stream, seg_count, edges, items, n_items,
                                                                    xf, seg_px, partials, c, skip, nullptr, nullptr,
                                                                    nullptr, s);
}

template <int DT, int MODE>
static int launch_one_dt(int ppt, const void* arena, const EdgeDev& e, int edge_id, const EdgeXf* xf,
                         const int32_t* idx, float* partials, GnConst c, const EdgeCal& C, hipStream_t s) {
  dim3 grid(e.n_tiles), block(kReduceThreads);
  switch (ppt) {
    case 4: hipLaunchKernelGGL((k_edge_reduce_one<DT, 4, MODE>), grid, block, 0, s, arena, e, edge_id, xf, idx, partials, c, C); break;
    case 8: hipLaunchKernelGGL((k_edge_reduce_one<DT, 8, MODE>), grid, block, 0, s, arena, e, edge_id, xf, idx, partials, c, C); break;
    case 16: hipLaunchKernelGGL((k_edge_reduce_one<DT, 16, MODE>), grid, block, 0, s, arena, e, edge_id, xf, idx, partials, c, C); break;
    case 32: hipLaunchKernelGGL((k_edge_reduce_one<DT, 32, MODE>), grid, block, 0, s, arena, e, edge_id, xf, idx, partials, c, C); break;
    default: return fail(DS3_EINVAL, "unsupported pixels-per-thread");
  }
  return check_hip(hipGetLastError(), "k_edge_reduce_one");
}

int launch_edge_reduce_one(ds3_dtype dt, int ppt, const void* arena, const EdgeDev& e, int edge_id,
                           const EdgeXf* xf, const int32_t* idx_arena, float* partials, GnConst c,
                           hipStream_t s, const EdgeCal* cal) {
  if (e.n_tiles <= 0) return DS3_OK;
  const EdgeCal C = cal ? *cal : EdgeCal{};
  if (cal) {
    if (dt == DS3_F32) return launch_one_dt<DS3_F32, kCalibrated>(ppt, arena, e, edge_id, xf, idx_arena, partials, c, C, s);
    return launch_one_dt<DS3_BF16, kCalibrated>(ppt, arena, e, edge_id, xf, idx_arena, partials, c, C, s);
  }
  if (dt == DS3_F32) return launch_one_dt<DS3_F32, kRayRange>(ppt, arena, e, edge_id, xf, idx_arena, partials, c, C, s);
  return launch_one_dt<DS3_BF16, kRayRange>(ppt, arena, e, edge_id, xf, idx_arena, partials, c, C, s);
}

int make_edge_cal(const double* K, int n_kf, const int32_t* kf_w, const EdgeDev* edges, int n_edges, EdgeCal* out) {
  for (int k = 0; k < n_kf; ++k) {
    const double* q = K + 4 * k;
    if (!(q[0] > 0) || !(q[1] > 0) || !std::isfinite(q[0]) || !std::isfinite(q[1]) || !std::isfinite(q[2]) ||
        !std::isfinite(q[3]))
      return fail(DS3_EINVAL, "calibrated mode: bad intrinsics of keyframe " + std::to_string(k));
  }
  for (int e = 0; e < n_edges; ++e) {
    const double* Ki = K + 4 * edges[e].i;
    const double* Kj = K + 4 * edges[e].j;
    EdgeCal C;
    C.fxi = float(Ki[0]);
    C.fyi = float(Ki[1]);
    C.cxi = float(Ki[2]);
    C.cyi = float(Ki[3]);
    C.ifxj = float(1.0 / Kj[0]);
    C.ifyj = float(1.0 / Kj[1]);
    C.cxj = float(Kj[2]);
    C.cyj = float(Kj[3]);
    C.Wi = kf_w[edges[e].i];
    C.Wj = kf_w[edges[e].j];
    C.Hi = edges[e].npx_i / C.Wi;
    C.pad = 0;
    out[e] = C;
  }
  return DS3_OK;
}

// --------------------------------------------------------------------------------------------------
// Per-edge finalize: float64 sum of the edge's tile partials (tile order), A = Ad^T H_L Ad, b = Ad^T b_L
// --------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_edge_finalize(const EdgeDev* __restrict__ edges,
                                                      const float* __restrict__ partials,
                                                      const double* __restrict__ Ad_all,
                                                      double* __restrict__ A_out, double* __restrict__ b_out,
                                                      double* __restrict__ cost_e,
                                                      int64_t* __restrict__ count_e) {
  __shared__ double S[37];
  __shared__ double HL[49];
  __shared__ double Ad[49];
  __shared__ double Mt[49];
  const int e = blockIdx.x;
  const int t = threadIdx.x;
  const EdgeDev E = edges[e];
  if (t < 37) {
    double s = 0.0;
    const float* p = partials + int64_t(E.tile0) * kPartial + t;
    // eight loads in flight, summed in tile order
    int k = 0;
    for (; k + 8 <= E.n_tiles; k += 8) {
      float v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = p[int64_t(k + q) * kPartial];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += double(v[q]);
    }
    for (; k < E.n_tiles; ++k) s += double(p[int64_t(k) * kPartial]);
    S[t] = s;
  }
  if (t < 49) Ad[t] = Ad_all[49 * int64_t(e) + t];
  __syncthreads();
  if (t < 49) {
    int r = t / 7, c = t % 7;
    int lo = r < c ? r : c, hi = r < c ? c : r;
    HL[t] = S[HIDX(lo, hi)];
  }
  __syncthreads();
  if (t < 49) {  // Mt = H_L Ad
    int a = t / 7, c = t % 7;
    double s = 0.0;
    for (int b = 0; b < 7; ++b) s += HL[7 * a + b] * Ad[7 * b + c];
    Mt[t] = s;
  }
  __syncthreads();
  if (t < 49) {  // A = Ad^T Mt; upper triangle computed, mirrored for exact symmetry
    int r = t / 7, c = t % 7;
    int lo = r < c ? r : c, hi = r < c ? c : r;
    double s = 0.0;
    for (int a = 0; a < 7; ++a) s += Ad[7 * a + lo] * Mt[7 * a + hi];
    A_out[49 * int64_t(e) + t] = s;
  }
  if (t < 7) {
    double s = 0.0;
    for (int a = 0; a < 7; ++a) s += Ad[7 * a + t] * S[28 + a];
    b_out[7 * int64_t(e) + t] = s;
  }
  if (t == 0) {
    cost_e[e] = S[35];
    count_e[e] = int64_t(S[36] + 0.5);
  }
}

int launch_edge_finalize(const EdgeDev* edges, int n_edges, const float* partials, const double* Ad,
                         double* A_out, double* b_out, double* cost_e, int64_t* count_e, hipStream_t s) {
  if (n_edges <= 0) return DS3_OK;
  hipLaunchKernelGGL(k_edge_finalize, dim3(n_edges), dim3(64), 0, s, edges, partials, Ad, A_out, b_out,
                     cost_e, count_e);
  return check_hip(hipGetLastError(), "k_edge_finalize");
}

// --------------------------------------------------------------------------------------------------
// Assembly: diagonal blocks and g per keyframe (incident edges in index order), off-diagonal blocks per
// keyframe pair (its edges in index order); anchor rows/columns are identity with g = 0.
// H must be zero outside the written blocks.
// --------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_assemble(int n_kf, const int32_t* __restrict__ node_ptr,
                                                 const int32_t* __restrict__ node_adj,
                                                 const int32_t* __restrict__ pair_ptr,
                                                 const int32_t* __restrict__ pair_edges,
                                                 const int32_t* __restrict__ pair_ij,
                                                 const double* __restrict__ A_e,
                                                 const double* __restrict__ b_e,
                                                 const uint8_t* __restrict__ anchor,
                                                 double* __restrict__ H, double* __restrict__ g,
                                                 unsigned* __restrict__ zero, int n_zero) {
  const int t = threadIdx.x;
  const int64_t n = 7 * int64_t(n_kf);
  if (blockIdx.x == 0 && t < n_zero) zero[t] = 0u;  // words the solve that follows needs cleared
  if (int(blockIdx.x) < n_kf) {
    const int k = blockIdx.x;
    const bool anc = anchor && anchor[k];
    if (t < 49) {
      double s = 0.0;
      const int p1 = node_ptr[k + 1];
      int p = node_ptr[k];
      for (; p + 4 <= p1; p += 4) {  // four loads in flight, summed in edge order
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = A_e[49 * int64_t(node_adj[p + q] >> 1) + t];
#pragma unroll
        for (int q = 0; q < 4; ++q) s += v[q];
      }
      for (; p < p1; ++p) s += A_e[49 * int64_t(node_adj[p] >> 1) + t];
      int r = t / 7, c = t % 7;
      H[(7 * int64_t(k) + r) * n + 7 * k + c] = anc ? (r == c ? 1.0 : 0.0) : s;
    } else if (t < 56) {
      const int r = t - 49;
      double s = 0.0;
      for (int p = node_ptr[k]; p < node_ptr[k + 1]; ++p) {
        const int code = node_adj[p];
        const double v = b_e[7 * int64_t(code >> 1) + r];
        s += (code & 1) ? v : -v;
      }
      g[7 * int64_t(k) + r] = anc ? 0.0 : s;
    }
  } else {
    const int p = blockIdx.x - n_kf;
    const int a = pair_ij[2 * p], b = pair_ij[2 * p + 1];
    const bool anc = anchor && (anchor[a] || anchor[b]);
    if (t < 49) {
      double s = 0.0;
      const int q1 = pair_ptr[p + 1];
      int q = pair_ptr[p];
      for (; q + 4 <= q1; q += 4) {  // four loads in flight, summed in edge order
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = A_e[49 * int64_t(pair_edges[q + u]) + t];
#pragma unroll
        for (int u = 0; u < 4; ++u) s -= v[u];
      }
      for (; q < q1; ++q) s -= A_e[49 * int64_t(pair_edges[q]) + t];
      if (anc) s = 0.0;
      const int r = t / 7, c = t % 7;
      H[(7 * int64_t(a) + r) * n + 7 * b + c] = s;
      H[(7 * int64_t(b) + c) * n + 7 * a + r] = s;
    }
  }
}

int launch_assemble(int n_kf, const int32_t* node_ptr, const int32_t* node_adj, const int32_t* pair_ptr,
                    const int32_t* pair_edges, const int32_t* pair_ij, int n_pairs, const double* A_e,
                    const double* b_e, const uint8_t* anchor_mask, double* H, double* g, hipStream_t s,
                    unsigned* zero, int n_zero) {
  if (n_zero < 0 || n_zero > 64 || (n_zero > 0 && !zero)) return fail(DS3_EINVAL, "assemble: bad zero words");
  hipLaunchKernelGGL(k_assemble, dim3(n_kf + n_pairs), dim3(64), 0, s, n_kf, node_ptr, node_adj, pair_ptr,
                     pair_edges, pair_ij, A_e, b_e, anchor_mask, H, g, zero, n_zero);
  return check_hip(hipGetLastError(), "k_assemble");
}

// Deterministic sum of per-edge costs and counts over one block of 256 threads (fixed strided split + fixed
// tree); thread 0 writes them. With ctr, the sum and *status are also appended to a history (slot *ctr,
// then ctr advances; slots past hist_len are dropped).
__device__ inline void sum_costs_block(const double* __restrict__ cost_e, const int64_t* __restrict__ count_e,
                                       int n_edges, double* __restrict__ cost_out, int64_t* __restrict__ count_out,
                                       const int32_t* __restrict__ status, unsigned* __restrict__ ctr,
                                       double* __restrict__ cost_hist, int32_t* __restrict__ status_hist,
                                       int hist_len) {
  __shared__ double sc[256];
  __shared__ long long sn[256];
  double c = 0.0;
  long long m = 0;
  for (int e = threadIdx.x; e < n_edges; e += 256) {
    c += cost_e[e];
    m += count_e[e];
  }
  sc[threadIdx.x] = c;
  sn[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      sc[threadIdx.x] += sc[threadIdx.x + w];
      sn[threadIdx.x] += sn[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (cost_out) *cost_out = sc[0];
    if (count_out) *count_out = sn[0];
    if (ctr) {
      const unsigned k = *ctr;
      if (k < unsigned(hist_len)) {
        cost_hist[k] = sc[0];
        status_hist[k] = *status;
      }
      *ctr = k + 1;
    }
  }
}

__global__ __launch_bounds__(256) void k_sum_costs(const double* __restrict__ cost_e,
                                                   const int64_t* __restrict__ count_e, int n_edges,
                                                   double* __restrict__ cost_out,
                                                   int64_t* __restrict__ count_out,
                                                   const int32_t* __restrict__ status, unsigned* __restrict__ ctr,
                                                   double* __restrict__ cost_hist,
                                                   int32_t* __restrict__ status_hist, int hist_len) {
  sum_costs_block(cost_e, count_e, n_edges, cost_out, count_out, status, ctr, cost_hist, status_hist, hist_len);
}

int launch_sum_costs(const double* cost_e, const int64_t* count_e, int n_edges, double* cost_out,
                     int64_t* count_out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_costs, dim3(1), dim3(256), 0, s, cost_e, count_e, n_edges, cost_out, count_out,
                     static_cast<const int32_t*>(nullptr), static_cast<unsigned*>(nullptr),
                     static_cast<double*>(nullptr), static_cast<int32_t*>(nullptr), 0);
  return check_hip(hipGetLastError(), "k_sum_costs");
}

// --------------------------------------------------------------------------------------------------
// Update T <- Exp(tau) T (Sec. III-D), fixed poses untouched; helpers
// --------------------------------------------------------------------------------------------------
__global__ void k_sim3_update(double* __restrict__ poses, const double* __restrict__ tau,
                              const uint8_t* __restrict__ fixed, int n) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (fixed && fixed[k]) return;
  Sim3 E = sim3_exp(tau + 7 * int64_t(k));
  Sim3 T = sim3_load(poses + 8 * int64_t(k));
  sim3_store(sim3_mul(E, T), poses + 8 * int64_t(k));
}

int launch_sim3_update(double* poses, const double* tau, const uint8_t* fixed, int n, hipStream_t s) {
  if (n <= 0) return DS3_OK;
  hipLaunchKernelGGL(k_sim3_update, dim3((n + 63) / 64), dim3(64), 0, s, poses, tau, fixed, n);
  return check_hip(hipGetLastError(), "k_sim3_update");
}

// The last step of a plan iteration in one launch: block 0 sums the edge costs and records them with the
// ladder status (as k_sum_costs), blocks 1.. apply T <- Exp(tau) T (as k_sim3_update). Both only read what the
// solve and the reduction before them wrote.
__global__ __launch_bounds__(256) void k_update_record(double* __restrict__ poses, const double* __restrict__ tau,
                                                       const uint8_t* __restrict__ fixed, int n,
                                                       const double* __restrict__ cost_e,
                                                       const int64_t* __restrict__ count_e, int n_edges,
                                                       double* __restrict__ cost_out, int64_t* __restrict__ count_out,
                                                       const int32_t* __restrict__ status, unsigned* __restrict__ ctr,
                                                       double* __restrict__ cost_hist,
                                                       int32_t* __restrict__ status_hist, int hist_len) {
  if (blockIdx.x == 0) {
    sum_costs_block(cost_e, count_e, n_edges, cost_out, count_out, status, ctr, cost_hist, status_hist, hist_len);
    return;
  }
  const int k = (blockIdx.x - 1) * 256 + threadIdx.x;
  if (k >= n) return;
  if (fixed && fixed[k]) return;
  Sim3 E = sim3_exp(tau + 7 * int64_t(k));
  Sim3 T = sim3_load(poses + 8 * int64_t(k));
  sim3_store(sim3_mul(E, T), poses + 8 * int64_t(k));
}

int launch_update_record(double* poses, const double* tau, const uint8_t* fixed, int n, const double* cost_e,
                         const int64_t* count_e, int n_edges, double* cost_out, int64_t* count_out,
                         const int32_t* status, unsigned* ctr, double* cost_hist, int32_t* status_hist, int hist_len,
                         hipStream_t s) {
  const int blocks = 1 + (std::max(n, 0) + 255) / 256;
  hipLaunchKernelGGL(k_update_record, dim3(blocks), dim3(256), 0, s, poses, tau, fixed, n, cost_e, count_e, n_edges,
                     cost_out, count_out, status, ctr, cost_hist, status_hist, hist_len);
  return check_hip(hipGetLastError(), "k_update_record");
}

__global__ void k_fill_f64(double* p, size_t n, double v) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  size_t stride = size_t(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_u32(unsigned* p, size_t n, unsigned v) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  size_t stride = size_t(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_copy_f64(const double* src, double* dst, size_t n) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  size_t stride = size_t(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

static int grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return int(b);
}

int launch_fill(double* p, size_t n, double v, hipStream_t s) {
  if (n == 0) return DS3_OK;
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return check_hip(hipGetLastError(), "k_fill_f64");
}

int launch_fill_u32(unsigned* p, size_t n, unsigned v, hipStream_t s) {
  if (n == 0) return DS3_OK;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return check_hip(hipGetLastError(), "k_fill_u32");
}

int launch_copy_f64(const double* src, double* dst, size_t n, hipStream_t s) {
  if (n == 0) return DS3_OK;
  hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
  return check_hip(hipGetLastError(), "k_copy_f64");
}

// Valid matches per tile (for ordering the work items): one block per (edge, tile).
__global__ __launch_bounds__(256) void k_count_valid(const EdgeDev* __restrict__ edges,
                                                     const int32_t* __restrict__ idx_arena, int tile_px,
                                                     int32_t* __restrict__ counts) {
  const int e = blockIdx.y;
  const EdgeDev E = edges[e];
  const int tile = blockIdx.x;
  if (tile >= E.n_tiles) return;
  int c = 0;
  const int64_t base = int64_t(tile) * tile_px;
  for (int q = threadIdx.x; q < tile_px; q += 256) {
    int64_t n = base + q;
    if (n < E.npx_j) {
      int32_t m = idx_arena[E.idx_off + n];
      c += (m >= 0 && m < E.npx_i) ? 1 : 0;
    }
  }
  c = wave_sum(c);
  __shared__ int s[4];
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) counts[E.tile0 + tile] = s[0] + s[1] + s[2] + s[3];
}

int launch_count_valid(const EdgeDev* edges, int n_edges, const int32_t* idx_arena, int tile_px,
                       int max_tiles, int32_t* counts, hipStream_t s) {
  if (n_edges <= 0 || max_tiles <= 0) return DS3_OK;
  hipLaunchKernelGGL(k_count_valid, dim3(max_tiles, n_edges), dim3(256), 0, s, edges, idx_arena, tile_px,
                     counts);
  return check_hip(hipGetLastError(), "k_count_valid");
}

}  // namespace ds3
