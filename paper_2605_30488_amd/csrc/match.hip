// Projective ray matching (Sec. III-A "Learned geometry": p* = argmin_p |psi([X_ref]_p) - psi(x)|^2)
// and bidirectional verification with the nu gate (Sec. III-B).
//
// Per query pixel: Levenberg-Marquardt over the continuous reference pixel p on the bilinear interpolant
// of the reference ray image psi(X_ref) (not renormalised), started at the query's own pixel scaled to
// the reference grid; a trial step is accepted iff it lowers |s(p) - psi(x)|^2 (damping / 10, floored),
// otherwise the damping grows x10; stop after max_iters trial steps or a trial step (accepted or not)
// below step_tol_px. idx = round(p*) (ties up). Valid iff no hole was touched, the final angular residual is
// within ang_tol_px * min(|ds/du|, |ds/dv|) and the range agrees within range_rel_tol. The mutual check
// keeps pixel n of j iff its match m in i maps back within a Chebyshev radius of n.
//
// The reference ray image is built once per keyframe (float4: psi, |X|; holes have |X| = 0) so each LM
// sample is four 16-byte reads. Batched launches walk (direction, tile) items that the host interleaves
// so that all tiles of one direction land on one XCD (block b runs on XCD b mod 8), keeping that
// reference ray image in one L2.
#include "common.hpp"
#include "internal.hpp"
#include "match_internal.hpp"

namespace ds3 {

// Ray image (psi, |X|) of every pixel and, when conf is given, its confidence as a plain float array
// (the mutual check then reads 4 B per pixel instead of a 16 B or 8 B xyzc entry).
template <int DT>
__global__ void k_raymap(const void* __restrict__ arena, int64_t n, float4* __restrict__ rays,
                         float* __restrict__ conf) {
  int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (; k < n; k += stride) {
    float4 X = Px<DT>::load(arena, k);
    if (conf) conf[k] = X.w;
    float d2 = fmaf(X.x, X.x, fmaf(X.y, X.y, X.z * X.z));
    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
    if (finite3(X.x, X.y, X.z) && d2 > 1e-18f) {
      float rd = 1.0f / sqrtf(d2);
      float d = sqrtf(d2);
      r = make_float4(X.x * rd, X.y * rd, X.z * rd, d);
    }
    rays[k] = r;
  }
}

int launch_raymap(const void* arena, int64_t n, ds3_dtype dt, float4* rays, float* conf, hipStream_t s) {
  if (n <= 0) return DS3_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (dt == DS3_F32)
    hipLaunchKernelGGL(k_raymap<DS3_F32>, dim3(blocks), dim3(256), 0, s, arena, n, rays, conf);
  else
    hipLaunchKernelGGL(k_raymap<DS3_BF16>, dim3(blocks), dim3(256), 0, s, arena, n, rays, conf);
  return check_hip(hipGetLastError(), "k_raymap");
}

struct Sample {
  float s[3], su[3], sv[3];
  bool hole;
};

// The four texels of the last cell a query sampled, each minus the query's target ray: a trial that stays
// in the same cell (the common case once the steps are sub-pixel, and for every damped retry that moves a
// little) reuses them instead of gathering again. Interpolating the differences gives the residual
// s(p) - psi(x) directly: neighbouring rays differ from the target by about a pixel's angle, so their
// differences are nearly exact in float32 and the residual keeps its relative precision down to the
// optimum, where s(p) and psi(x) agree to six digits. (Interpolating the rays first and subtracting
// afterwards loses those digits: the cost then stops decreasing at steps of about 1e-4 px.)
struct Cell {
  int u0, v0;
  float a[3], b[3], c[3], d[3];
  bool hole;
};

__device__ inline void cell_origin(int H, int W, float u, float v, int& u0, int& v0) {
  u0 = max(min(int(floorf(u)), W - 2), 0);
  v0 = max(min(int(floorf(v)), H - 2), 0);
}

__device__ inline void fetch_cell(const float4* __restrict__ R, int W, int u0, int v0, const float* t, Cell& C) {
  const int64_t i00 = int64_t(v0) * W + u0;
  const float4 a = R[i00], b = R[i00 + 1], c = R[i00 + W], d = R[i00 + W + 1];
  C.u0 = u0;
  C.v0 = v0;
  C.hole = !(a.w > 0.f) || !(b.w > 0.f) || !(c.w > 0.f) || !(d.w > 0.f);
  C.a[0] = a.x - t[0]; C.a[1] = a.y - t[1]; C.a[2] = a.z - t[2];
  C.b[0] = b.x - t[0]; C.b[1] = b.y - t[1]; C.b[2] = b.z - t[2];
  C.c[0] = c.x - t[0]; C.c[1] = c.y - t[1]; C.c[2] = c.z - t[2];
  C.d[0] = d.x - t[0]; C.d[1] = d.y - t[1]; C.d[2] = d.z - t[2];
}

// Bilinear sample of (ray image - target ray), i.e. the residual, and its in-cell derivatives at (u, v);
// gathers only when the cell differs from the cached one.
__device__ inline Sample sample_rays(const float4* __restrict__ R, int H, int W, float u, float v, const float* t,
                                     Cell& C) {
  int u0, v0;
  cell_origin(H, W, u, v, u0, v0);
  if (u0 != C.u0 || v0 != C.v0) fetch_cell(R, W, u0, v0, t, C);
  const float fu = u - float(u0), fv = v - float(v0);
  Sample S;
  S.hole = C.hole;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float top = fmaf(fu, C.b[k] - C.a[k], C.a[k]);
    const float bot = fmaf(fu, C.d[k] - C.c[k], C.c[k]);
    S.s[k] = fmaf(fv, bot - top, top);
    S.su[k] = fmaf(fv, (C.d[k] - C.c[k]) - (C.b[k] - C.a[k]), C.b[k] - C.a[k]);
    S.sv[k] = bot - top;
  }
  return S;
}

// One query: returns idx (or -1); p and iteration count through the pointers when non-null.
__device__ inline int32_t match_query(const float4* __restrict__ R, int H, int W, float4 x, int qu, int qv,
                                      int Hq, int Wq, const MatchConst& P, float* pu, float* pv,
                                      int* iters) {
  *pu = __int_as_float(0x7fc00000);
  *pv = __int_as_float(0x7fc00000);
  *iters = 0;
  const float dx2 = fmaf(x.x, x.x, fmaf(x.y, x.y, x.z * x.z));
  if (!finite3(x.x, x.y, x.z) || !(dx2 > 1e-18f)) return -1;
  const float dx = sqrtf(dx2);
  const float rdx = 1.0f / dx;
  const float t[3] = {x.x * rdx, x.y * rdx, x.z * rdx};
  float u = (Wq > 1) ? float(qu) * (float(W - 1) / float(Wq - 1)) : 0.0f;
  float v = (Hq > 1) ? float(qv) * (float(H - 1) / float(Hq - 1)) : 0.0f;
  Cell C;
  C.u0 = -1;
  C.v0 = -1;
  Sample S = sample_rays(R, H, W, u, v, t, C);
  if (S.hole) return -1;
  float r0 = S.s[0], r1 = S.s[1], r2 = S.s[2];
  float c = fmaf(r0, r0, fmaf(r1, r1, r2 * r2));
  float lam = P.lambda0;
  // normal equations at the current p; unchanged by a rejected step, so rebuilt only on acceptance
  float a = fmaf(S.su[0], S.su[0], fmaf(S.su[1], S.su[1], S.su[2] * S.su[2]));
  float b = fmaf(S.su[0], S.sv[0], fmaf(S.su[1], S.sv[1], S.su[2] * S.sv[2]));
  float dd = fmaf(S.sv[0], S.sv[0], fmaf(S.sv[1], S.sv[1], S.sv[2] * S.sv[2]));
  float gu = fmaf(S.su[0], r0, fmaf(S.su[1], r1, S.su[2] * r2));
  float gv = fmaf(S.sv[0], r0, fmaf(S.sv[1], r1, S.sv[2] * r2));
  // The trial loop is written with selects rather than branches so that a wave's divergent lanes cost
  // few exec-mask instructions: every active lane samples once per trial (at the current point when the
  // step does not move), and lanes leave through `active`.
  int it = 0;
  bool active = true, hole = false;
  for (; it < P.max_iters; ++it) {
    if (!active) break;
    const float A = a * (1.0f + lam), D = dd * (1.0f + lam);
    const float det = A * D - b * b;
    const bool det_ok = det > 0.0f;
    const float idet = __builtin_amdgcn_rcpf(det);  // hardware reciprocal (1 ulp)
    const float du = -(D * gu - b * gv) * idet;
    const float dv = -(A * gv - b * gu) * idet;
    const float un = det_ok ? fminf(fmaxf(u + du, 0.0f), float(W - 1)) : u;
    const float vn = det_ok ? fminf(fmaxf(v + dv, 0.0f), float(H - 1)) : v;
    // no movement (singular system, clamped or vanishing step): same sample, same cost, reject
    const bool moved = (un != u) || (vn != v);
    const Sample Sn = sample_rays(R, H, W, un, vn, t, C);
    if (moved && Sn.hole) {
      hole = true;
      active = false;
      continue;  // `it` advances past this trial
    }
    const float n0 = Sn.s[0], n1 = Sn.s[1], n2 = Sn.s[2];
    const float cn = fmaf(n0, n0, fmaf(n1, n1, n2 * n2));
    const bool acc = moved && (cn < c);
    const float step = fmaxf(fabsf(un - u), fabsf(vn - v));
    // A trial step shorter than the tolerance ends the search whether or not it is accepted (a
    // non-singular system: singular ones retry with a larger damping); the oracle takes the same rule.
    if (!acc && det_ok && step < P.step_tol) active = false;
    lam = acc ? fmaxf(lam * 0.1f, P.lambda_min) : lam * 10.0f;
    if (acc) {
      u = un; v = vn; S = Sn; c = cn;
      r0 = n0; r1 = n1; r2 = n2;
      a = fmaf(S.su[0], S.su[0], fmaf(S.su[1], S.su[1], S.su[2] * S.su[2]));
      b = fmaf(S.su[0], S.sv[0], fmaf(S.su[1], S.sv[1], S.su[2] * S.sv[2]));
      dd = fmaf(S.sv[0], S.sv[0], fmaf(S.sv[1], S.sv[1], S.sv[2] * S.sv[2]));
      gu = fmaf(S.su[0], r0, fmaf(S.su[1], r1, S.su[2] * r2));
      gv = fmaf(S.sv[0], r0, fmaf(S.sv[1], r1, S.sv[2] * r2));
      if (step < P.step_tol) active = false;  // converged: `it` advances past this trial
    }
  }
  if (hole) {
    *iters = it;
    return -1;
  }
  *iters = it;
  *pu = u;
  *pv = v;
  const float nsu = sqrtf(fmaf(S.su[0], S.su[0], fmaf(S.su[1], S.su[1], S.su[2] * S.su[2])));
  const float nsv = sqrtf(fmaf(S.sv[0], S.sv[0], fmaf(S.sv[1], S.sv[1], S.sv[2] * S.sv[2])));
  const float rr = sqrtf(c);
  if (!(rr <= P.ang_tol * fminf(nsu, nsv))) return -1;
  const int mu = min(max(int(floorf(u + 0.5f)), 0), W - 1);
  const int mv = min(max(int(floorf(v + 0.5f)), 0), H - 1);
  const int32_t m = mv * W + mu;
  const float4 Rm = R[m];
  if (!(Rm.w > 0.f)) return -1;
  if (!(fabsf(dx - Rm.w) <= P.range_tol * Rm.w)) return -1;
  return m;
}

// Single direction: one thread per query pixel.
template <int DT>
__global__ __launch_bounds__(256) void k_match_one(const float4* __restrict__ rays, int H, int W,
                                                   const void* __restrict__ qry, int Hq, int Wq,
                                                   MatchConst P, int32_t* __restrict__ idx_out,
                                                   float* __restrict__ p_out, int32_t* __restrict__ it_out) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= int64_t(Hq) * Wq) return;
  const float4 x = Px<DT>::load(qry, n);
  float pu, pv;
  int its;
  const int32_t m = match_query(rays, H, W, x, int(n % Wq), int(n / Wq), Hq, Wq, P, &pu, &pv, &its);
  idx_out[n] = m;
  if (p_out) {
    p_out[2 * n] = pu;
    p_out[2 * n + 1] = pv;
  }
  if (it_out) it_out[n] = its;
}

int launch_match_one(const float4* rays, int H, int W, const void* qry, int Hq, int Wq, ds3_dtype dt,
                     const MatchConst& P, int32_t* idx_out, float* p_out, int32_t* it_out, hipStream_t s) {
  const int64_t n = int64_t(Hq) * Wq;
  if (n <= 0) return DS3_OK;
  dim3 grid(unsigned((n + 255) / 256)), block(256);
  if (dt == DS3_F32)
    hipLaunchKernelGGL(k_match_one<DS3_F32>, grid, block, 0, s, rays, H, W, qry, Hq, Wq, P, idx_out, p_out, it_out);
  else
    hipLaunchKernelGGL(k_match_one<DS3_BF16>, grid, block, 0, s, rays, H, W, qry, Hq, Wq, P, idx_out, p_out, it_out);
  return check_hip(hipGetLastError(), "k_match_one");
}

// Locate the (entry, tile) of block b in the binned item map; false for padding blocks.
__device__ inline bool locate_item(const ItemMap& M, int b, int& entry, int& tile) {
  const int x = b & 7, slot = b >> 3;
  if (slot >= M.bin_tiles[x]) return false;
  int lo = M.bin_start[x], hi = M.bin_start[x + 1] - 1;
  while (lo < hi) {  // last entry with prefix <= slot
    const int mid = (lo + hi + 1) >> 1;
    if (M.prefix[mid] <= slot) lo = mid; else hi = mid - 1;
  }
  entry = lo;
  tile = slot - M.prefix[lo];
  return true;
}

// Batched: one 16x16 tile of query pixels per block; blocks of one direction share an XCD. The LM trial-step count is
// summed per block and added to one of kStepStripes counters 128 B apart (block b to stripe b mod
// kStepStripes): a single counter hit by every wave becomes a hot spot of one L2 channel that stalls the
// whole launch.
template <int DT>
__global__ __launch_bounds__(256) void k_match_batched(const float4* __restrict__ rays,
                                                       const void* __restrict__ cross,
                                                       const MatchDir* __restrict__ dirs, ItemMap map,
                                                       MatchConst P, int32_t* __restrict__ idx_tmp,
                                                       unsigned* __restrict__ step_stripes) {
  int entry, tile;
  if (!locate_item(map, blockIdx.x, entry, tile)) return;  // uniform per block
  const MatchDir D = dirs[entry];
  // a 16x16 tile of query pixels: their matches (and the LM steps towards them) cover a compact window of
  // the reference ray image, so the block's gathers share far more L2 lines than a 256-pixel row segment's
  const int tiles_x = (D.Wq + kMatchTile - 1) / kMatchTile;
  const int qu = (tile % tiles_x) * kMatchTile + int(threadIdx.x % kMatchTile);
  const int qv = (tile / tiles_x) * kMatchTile + int(threadIdx.x / kMatchTile);
  int its = 0;
  if (qu < D.Wq && qv < D.Hq) {
    const int64_t n = int64_t(qv) * D.Wq + qu;
    const float4 x = Px<DT>::load(cross, D.qry_off + n);
    float pu, pv;
    idx_tmp[D.out_off + n] = match_query(rays + D.ref_off, D.Hr, D.Wr, x, qu, qv, D.Hq, D.Wq, P, &pu, &pv, &its);
  }
  if (step_stripes) {
    __shared__ int s[4];
    its = wave_sum(its);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = its;
    __syncthreads();
    if (threadIdx.x == 0) {
      const int tot = s[0] + s[1] + s[2] + s[3];
      if (tot) atomicAdd(&step_stripes[(blockIdx.x % kStepStripes) * kStripeStride], unsigned(tot));
    }
  }
}

__global__ void k_sum_stripes(const unsigned* __restrict__ step_stripes, unsigned long long* __restrict__ out) {
  unsigned long long v = 0;
  for (int k = threadIdx.x; k < kStepStripes; k += blockDim.x) v += step_stripes[k * kStripeStride];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  __shared__ unsigned long long part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = part[0] + part[1] + part[2] + part[3];
}

int launch_match_batched(const float4* rays, const void* cross, ds3_dtype dt, const MatchDir* dirs,
                         ItemMap map, int grid, const MatchConst& P, int32_t* idx_tmp,
                         unsigned* step_stripes, hipStream_t s) {
  if (grid <= 0) return DS3_OK;
  if (dt == DS3_F32)
    hipLaunchKernelGGL(k_match_batched<DS3_F32>, dim3(grid), dim3(256), 0, s, rays, cross, dirs, map, P, idx_tmp,
                       step_stripes);
  else
    hipLaunchKernelGGL(k_match_batched<DS3_BF16>, dim3(grid), dim3(256), 0, s, rays, cross, dirs, map, P, idx_tmp,
                       step_stripes);
  return check_hip(hipGetLastError(), "k_match_batched");
}

int launch_sum_stripes(const unsigned* step_stripes, unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_stripes, dim3(1), dim3(256), 0, s, step_stripes, out);
  return check_hip(hipGetLastError(), "k_sum_stripes");
}

// --------------------------------------------------------------------------------------------------
// Mutual check + nu counts. Side J (pixels of j): final idx and valid mask; side I (pixels of i):
// count only. Every block writes its tile's count to its own slot of the partials (no atomics: the
// blocks of one side would otherwise all hit one counter), then k_side_counts sums each side in a fixed
// order: counts[2e] = i-side count, counts[2e+1] = j-side count.
// --------------------------------------------------------------------------------------------------
template <int DT>
__global__ __launch_bounds__(256) void k_mutual(const MutualDir* __restrict__ md, ItemMap map,
                                                MatchConst P, const int32_t* __restrict__ idx_tmp,
                                                int32_t* __restrict__ idx_final, uint8_t* __restrict__ valid,
                                                unsigned* __restrict__ part) {
  constexpr int kPer = kMutualPx / 256;
  int entry, tile;
  if (!locate_item(map, blockIdx.x, entry, tile)) return;  // uniform per block
  const MutualDir M = md[entry];
  const int64_t n_self = int64_t(M.H_self) * M.W_self;
  const int64_t n_other = int64_t(M.H_other) * M.W_other;
  const int32_t* fwd = idx_tmp + M.fwd_off;
  const int32_t* bwd = idx_tmp + M.bwd_off;
  // four independent pixels per thread, every load of a stage issued before its first use:
  // forward matches, then the backward matches and both confidences
  int64_t n[kPer];
  int32_t m[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    n[u] = int64_t(tile) * kMutualPx + u * 256 + threadIdx.x;
    m[u] = (n[u] < n_self) ? fwd[n[u]] : -1;
    m[u] = (m[u] < n_other) ? m[u] : -1;
  }
  int32_t n2[kPer];
  float cs[kPer], co[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const bool has = m[u] >= 0;
    n2[u] = has ? bwd[m[u]] : -1;
    co[u] = has ? M.conf_other[m[u]] : 0.0f;
    cs[u] = (n[u] < n_self) ? M.conf_self[n[u]] : 0.0f;
  }
  int hit = 0;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    if (n[u] >= n_self) continue;
    bool ok = m[u] >= 0 && n2[u] >= 0 && n2[u] < n_self;
    if (ok) {
      const int du = abs(int(n2[u] % M.W_self) - int(n[u] % M.W_self));
      const int dv = abs(int(n2[u] / M.W_self) - int(n[u] / M.W_self));
      ok = max(du, dv) <= P.radius;
    }
    if (ok) hit += (sqrt(double(co[u]) * double(cs[u])) >= P.q_min) ? 1 : 0;
    if (M.write_out) {
      idx_final[M.out_off + n[u]] = ok ? m[u] : -1;
      valid[M.out_off + n[u]] = ok ? 1 : 0;
    }
  }
  hit = wave_sum(hit);
  __shared__ int s[4];
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = hit;
  __syncthreads();
  if (threadIdx.x == 0) part[M.part_off + tile] = unsigned(s[0] + s[1] + s[2] + s[3]);
}

// One wave per side: lanes stride the side's tile partials, then a fixed-shape wave sum.
__global__ __launch_bounds__(256) void k_side_counts(const unsigned* __restrict__ part,
                                                     const int64_t* __restrict__ side, int n_slots,
                                                     unsigned* __restrict__ counts) {
  const int slot = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (slot >= n_slots) return;  // uniform per wave
  const int lane = threadIdx.x & 63;
  const int64_t off = side[2 * slot], n = side[2 * slot + 1];
  int c = 0;
  for (int64_t t = lane; t < n; t += 64) c += int(part[off + t]);
  c = wave_sum(c);
  if (lane == 0) counts[slot] = unsigned(c);
}

int launch_side_counts(const unsigned* part, const int64_t* side, int n_slots, unsigned* counts, hipStream_t s) {
  if (n_slots <= 0) return DS3_OK;
  hipLaunchKernelGGL(k_side_counts, dim3((n_slots + 3) / 4), dim3(256), 0, s, part, side, n_slots, counts);
  return check_hip(hipGetLastError(), "k_side_counts");
}

int launch_mutual(const MutualDir* md, ItemMap map, int grid, ds3_dtype dt, const MatchConst& P,
                  const int32_t* idx_tmp, int32_t* idx_final, uint8_t* valid, unsigned* part,
                  hipStream_t s) {
  if (grid <= 0) return DS3_OK;
  if (dt == DS3_F32)
    hipLaunchKernelGGL(k_mutual<DS3_F32>, dim3(grid), dim3(256), 0, s, md, map, P, idx_tmp, idx_final, valid, part);
  else
    hipLaunchKernelGGL(k_mutual<DS3_BF16>, dim3(grid), dim3(256), 0, s, md, map, P, idx_tmp, idx_final, valid, part);
  return check_hip(hipGetLastError(), "k_mutual");
}

// nu = count / pixels in double; admit = min(nu_i, nu_j) >= nu_min (same arithmetic as a double sum).
__global__ void k_nu_finalize(const unsigned* __restrict__ counts, const int64_t* __restrict__ npx,
                              int n_edges, double nu_min, float* __restrict__ nu,
                              int32_t* __restrict__ admit) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_edges) return;
  const double ni = double(counts[2 * e]) / double(npx[2 * e]);
  const double nj = double(counts[2 * e + 1]) / double(npx[2 * e + 1]);
  if (nu) {
    nu[2 * e] = float(ni);
    nu[2 * e + 1] = float(nj);
  }
  if (admit) admit[e] = (fmin(ni, nj) >= nu_min) ? 1 : 0;
}

int launch_nu_finalize(const unsigned* counts, const int64_t* npx, int n_edges, double nu_min, float* nu,
                       int32_t* admit, hipStream_t s) {
  if (n_edges <= 0) return DS3_OK;
  hipLaunchKernelGGL(k_nu_finalize, dim3((n_edges + 127) / 128), dim3(128), 0, s, counts, npx, n_edges,
                     nu_min, nu, admit);
  return check_hip(hipGetLastError(), "k_nu_finalize");
}

}  // namespace ds3
