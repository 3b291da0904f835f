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
// Two passes: the query side of every pixel is gathered over the edges that end in its keyframe and
// stored once (no atomics, which also clears the outputs); the gathered side then adds its terms with
// float atomics, since several matches of one edge can land on one pixel of i and a keyframe is the
// gathered side of several edges.
#include "common.hpp"
#include "internal.hpp"
#include "sim3.hpp"

namespace ds3 {

constexpr int kAdjThreads = 256;
constexpr int kAdjWaves = kAdjThreads / kWave;  // per-edge partials are written per wave (no block barrier)
constexpr int kAdjPPT = 2;  // 65 VGPRs, 7 waves per SIMD in the gather (4: 99 VGPRs and 15% slower; 1: block reductions dominate)

// Forward pass and cotangents of one match (n of j, m of i), scaled by dcost. Returns false for the
// pixels the cost skips (holes, zero ranges, bad confidences, non-finite values).
struct AdjPix {
  float x[3];    // T_ij X_j[n]
  float gx[3];   // dE/dx
  float gam[4];  // dE/de
  float pi[3];   // psi(X_i[m])
  float rdi;     // 1 / |X_i[m]|
  float dc;      // sum_c w_c r_c^2
  float rho;     // Huber cost of the four components (not scaled by dcost)
};

__device__ inline bool adj_pixel(const float4 Xj, const float4 Xi, const float* M, const GnConst& k, float dcost,
                                 AdjPix& o) {
  const float x0 = fmaf(M[0], Xj.x, fmaf(M[1], Xj.y, fmaf(M[2], Xj.z, M[9])));
  const float x1 = fmaf(M[3], Xj.x, fmaf(M[4], Xj.y, fmaf(M[5], Xj.z, M[10])));
  const float x2 = fmaf(M[6], Xj.x, fmaf(M[7], Xj.y, fmaf(M[8], Xj.z, M[11])));
  const float d2 = fmaf(x0, x0, fmaf(x1, x1, x2 * x2));
  const float di2 = fmaf(Xi.x, Xi.x, fmaf(Xi.y, Xi.y, Xi.z * Xi.z));
  const float dj2 = fmaf(Xj.x, Xj.x, fmaf(Xj.y, Xj.y, Xj.z * Xj.z));
  const float cc = Xi.w * Xj.w;
  const float mn = fminf(fminf(d2, di2), dj2);
  const float sum = (d2 + di2) + (dj2 + cc);
  if (!(mn > 1e-18f) || !(cc >= 0.0f) || !(sum < __builtin_huge_valf())) return false;
  const float rd = rsqrtf(d2), rdi = rsqrtf(di2);
  const float d = d2 * rd, di = di2 * rdi;
  const float p[3] = {x0 * rd, x1 * rd, x2 * rd};
  o.pi[0] = Xi.x * rdi;
  o.pi[1] = Xi.y * rdi;
  o.pi[2] = Xi.z * rdi;
  o.rdi = rdi;
  const float e4[4] = {p[0] - o.pi[0], p[1] - o.pi[1], p[2] - o.pi[2], d - di};
  const float sq = __builtin_amdgcn_sqrtf(__builtin_amdgcn_sqrtf(cc));
  const float isg[4] = {k.inv_sr, k.inv_sr, k.inv_sr, k.inv_sd};
  float dc = 0.0f, rho = 0.0f;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float r = sq * e4[c] * isg[c];
    const float a = fabsf(r);
    const float w = fminf(1.0f, k.kappa * __builtin_amdgcn_rcpf(a));
    o.gam[c] = w * r * sq * isg[c] * dcost;
    dc = fmaf(w * r, r, dc);
    const float t = w * a;  // rho = t (|r| - t/2)
    rho = fmaf(t, fmaf(-0.5f, t, a), rho);
  }
  o.rho = rho;
  o.dc = dc * dcost;
  const float pg = p[0] * o.gam[0] + p[1] * o.gam[1] + p[2] * o.gam[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) o.gx[a] = (o.gam[a] - p[a] * pg) * rd + o.gam[3] * p[a];
  o.x[0] = x0;
  o.x[1] = x1;
  o.x[2] = x2;
  return true;
}

// Query side, gathered: block (tile, k) owns 2048 pixels of keyframe k and walks the edges that end in
// k (j = k). Per pixel it sums dE/dX_k = (s_ij R_ij)^T dE/dx and the j half of dE/dC over those edges in
// registers and stores them once (zeros where nothing contributes); per (edge, tile) it leaves the
// seven pose-tangent pieces [g; x cross g; x . g] in part7 (row stride `stride` tiles).
template <int DT>
__global__ __launch_bounds__(kAdjThreads) void k_adjoint_gather_j(
    const void* __restrict__ arena, const EdgeDev* __restrict__ edges, const EdgeXf* __restrict__ xf,
    const int32_t* __restrict__ idx_arena, const int64_t* __restrict__ kf_off, const int32_t* __restrict__ kf_npx,
    const int32_t* __restrict__ node_ptr, const int32_t* __restrict__ node_adj, GnConst k, float dcost,
    float* __restrict__ grad_xyz, float* __restrict__ grad_conf, float* __restrict__ part7, int stride) {
  const int kf = blockIdx.y;
  const int tile = blockIdx.x;
  const int npx = kf_npx[kf];
  if (tile * kAdjThreads * kAdjPPT >= npx) return;  // uniform per block
  const int64_t off = kf_off[kf];
  typename Px<DT>::raw_t xr[kAdjPPT];
  float acc[kAdjPPT][4];
#pragma unroll
  for (int u = 0; u < kAdjPPT; ++u) {
    const int n = tile * kAdjThreads * kAdjPPT + u * kAdjThreads + threadIdx.x;
    xr[u] = Px<DT>::load_raw(arena, off + (n < npx ? n : 0));
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[u][c] = 0.0f;
  }
  for (int q = node_ptr[kf]; q < node_ptr[kf + 1]; ++q) {
    const int code = node_adj[q];
    if (!(code & 1)) continue;  // this keyframe is the gathered side of that edge
    const int e = code >> 1;
    const EdgeDev E = edges[e];
    float M[12];
#pragma unroll
    for (int r = 0; r < 12; ++r) M[r] = xf[e].m[r];
    const int32_t* idx = idx_arena + E.idx_off;
    float g7[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < kAdjPPT; ++u) {
      const int n = tile * kAdjThreads * kAdjPPT + u * kAdjThreads + threadIdx.x;
      const int32_t m = (n < npx) ? idx[n] : -1;
      if (m < 0 || m >= E.npx_i) continue;
      const float4 Xj = Px<DT>::unpack(xr[u]);
      const float4 Xi = Px<DT>::load(arena, E.off_i + m);
      AdjPix o;
      if (!adj_pixel(Xj, Xi, M, k, dcost, o)) continue;
      acc[u][0] += M[0] * o.gx[0] + M[3] * o.gx[1] + M[6] * o.gx[2];
      acc[u][1] += M[1] * o.gx[0] + M[4] * o.gx[1] + M[7] * o.gx[2];
      acc[u][2] += M[2] * o.gx[0] + M[5] * o.gx[1] + M[8] * o.gx[2];
      acc[u][3] += o.dc / (4.0f * Xj.w);
      g7[0] += o.gx[0];
      g7[1] += o.gx[1];
      g7[2] += o.gx[2];
      g7[3] += o.x[1] * o.gx[2] - o.x[2] * o.gx[1];
      g7[4] += o.x[2] * o.gx[0] - o.x[0] * o.gx[2];
      g7[5] += o.x[0] * o.gx[1] - o.x[1] * o.gx[0];
      g7[6] += o.x[0] * o.gx[0] + o.x[1] * o.gx[1] + o.x[2] * o.gx[2];
    }
    // one partial per wave and edge, summed in a fixed order by the edge finalize
    float* pw = part7 + ((int64_t(e) * stride + tile) * kAdjWaves + (threadIdx.x >> 6)) * 8;
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      const float v = wave_sum_to_lane63(g7[c]);
      if ((threadIdx.x & 63) == 63) pw[c] = v;
    }
  }
#pragma unroll
  for (int u = 0; u < kAdjPPT; ++u) {
    const int n = tile * kAdjThreads * kAdjPPT + u * kAdjThreads + threadIdx.x;
    if (n >= npx) continue;
    float* gj = grad_xyz + 3 * (off + n);
    gj[0] = acc[u][0];
    gj[1] = acc[u][1];
    gj[2] = acc[u][2];
    grad_conf[off + n] = acc[u][3];
  }
}

// Gathered side, scattered: the matches of one tile of an edge add dE/dX_i[m] and the i half of dE/dC
// with float atomics (several matches can land on one pixel of i, and a keyframe is the gathered side of
// several edges). Runs after k_adjoint_gather_j, whose plain stores it accumulates onto.
template <int DT>
__global__ __launch_bounds__(kAdjThreads) void k_adjoint_scatter_i(
    const void* __restrict__ arena, const EdgeDev* __restrict__ edges, const EdgeXf* __restrict__ xf,
    const int32_t* __restrict__ idx_arena, GnConst k, float dcost, float* __restrict__ grad_xyz,
    float* __restrict__ grad_conf) {
  const int e = blockIdx.y;
  const EdgeDev E = edges[e];
  const int tile = blockIdx.x;
  const int tiles_e = (E.npx_j + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  if (tile >= tiles_e) return;  // uniform per block
  float M[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) M[q] = xf[e].m[q];
  const int32_t* idx = idx_arena + E.idx_off;
#pragma unroll 2
  for (int u = 0; u < kAdjPPT; ++u) {
    const int64_t n = int64_t(tile) * kAdjThreads * kAdjPPT + int64_t(u) * kAdjThreads + threadIdx.x;
    if (n >= E.npx_j) continue;
    const int32_t m = idx[n];
    if (m < 0 || m >= E.npx_i) continue;
    const float4 Xj = Px<DT>::load(arena, E.off_j + n);
    const float4 Xi = Px<DT>::load(arena, E.off_i + m);
    AdjPix o;
    if (!adj_pixel(Xj, Xi, M, k, dcost, o)) continue;
    const float pgi = o.pi[0] * o.gam[0] + o.pi[1] * o.gam[1] + o.pi[2] * o.gam[2];
    float* gi = grad_xyz + 3 * (E.off_i + m);
#pragma unroll
    for (int a = 0; a < 3; ++a) atomicAdd(gi + a, -((o.gam[a] - o.pi[a] * pgi) * o.rdi + o.gam[3] * o.pi[a]));
    atomicAdd(grad_conf + E.off_i + m, o.dc / (4.0f * Xi.w));
  }
}

// --------------------------------------------------------------------------------------------------
// Inverse match maps for a graph whose matches stay fixed: for edge e and pixel m of keyframe i(e), the
// pixels n of j(e) with idx[n] = m, in increasing n, as CSR (offsets at obase[e], npx_i + 1 of them;
// lists at sbase[e]). Built once by count, scan, fill and a per-list sort.
// --------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_inv_count(const EdgeDev* __restrict__ edges,
                                                   const int32_t* __restrict__ idx_arena,
                                                   const int64_t* __restrict__ cbase, int32_t* __restrict__ cnt) {
  const int e = blockIdx.y;
  const EdgeDev E = edges[e];
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= E.npx_j) return;
  const int32_t m = idx_arena[E.idx_off + n];
  if (m < 0 || m >= E.npx_i) return;
  atomicAdd(cnt + cbase[e] + m, 1);
}

__global__ __launch_bounds__(1024) void k_inv_scan(const EdgeDev* __restrict__ edges,
                                                   const int64_t* __restrict__ cbase,
                                                   const int64_t* __restrict__ obase,
                                                   const int32_t* __restrict__ cnt, int32_t* __restrict__ off) {
  __shared__ int sh[2][1024];
  const int e = blockIdx.x, t = threadIdx.x;
  const int npx = edges[e].npx_i;
  const int chunk = (npx + 1023) / 1024;
  const int lo = min(npx, t * chunk), hi = min(npx, lo + chunk);
  const int32_t* c = cnt + cbase[e];
  int32_t* o = off + obase[e];
  int sum = 0;
  for (int m = lo; m < hi; ++m) sum += c[m];
  sh[0][t] = sum;
  __syncthreads();
  int src = 0;
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan of the chunk sums
    const int v = sh[src][t] + (t >= d ? sh[src][t - d] : 0);
    sh[src ^ 1][t] = v;
    src ^= 1;
    __syncthreads();
  }
  int run = sh[src][t] - sum;
  for (int m = lo; m < hi; ++m) {
    o[m] = run;
    run += c[m];
  }
  if (t == 1023) o[npx] = sh[src][t];
}

__global__ __launch_bounds__(256) void k_inv_fill(const EdgeDev* __restrict__ edges,
                                                  const int32_t* __restrict__ idx_arena,
                                                  const int64_t* __restrict__ cbase,
                                                  const int64_t* __restrict__ obase,
                                                  const int64_t* __restrict__ sbase,
                                                  const int32_t* __restrict__ off, int32_t* __restrict__ cur,
                                                  int32_t* __restrict__ src) {
  const int e = blockIdx.y;
  const EdgeDev E = edges[e];
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= E.npx_j) return;
  const int32_t m = idx_arena[E.idx_off + n];
  if (m < 0 || m >= E.npx_i) return;
  const int slot = atomicAdd(cur + cbase[e] + m, 1);
  src[sbase[e] + off[obase[e] + m] + slot] = n;
}

__global__ __launch_bounds__(256) void k_inv_sort(const EdgeDev* __restrict__ edges,
                                                  const int64_t* __restrict__ obase,
                                                  const int64_t* __restrict__ sbase,
                                                  const int32_t* __restrict__ off, int32_t* __restrict__ src) {
  const int e = blockIdx.y;
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= edges[e].npx_i) return;
  const int32_t* o = off + obase[e];
  const int a = o[m], b = o[m + 1];
  int32_t* L = src + sbase[e];
  for (int x = a + 1; x < b; ++x) {  // insertion sort, lists are short
    const int32_t v = L[x];
    int y = x - 1;
    while (y >= a && L[y] > v) {
      L[y + 1] = L[y];
      --y;
    }
    L[y + 1] = v;
  }
}

// Cost and adjoint in one gather pass over a fixed graph: block (tile, k) owns 2048 pixels of keyframe
// k. For the edges that end in k it walks the matches of its pixels (query side, as in
// k_adjoint_gather_j, plus the Huber cost in slot 7 of the tile pieces); for the edges that start in k
// it walks, per pixel m, the list of query pixels matched to m (gathered side). Both sides are summed in
// registers in a fixed order and stored once: no atomics, bitwise reproducible.
template <int DT>
__global__ __launch_bounds__(kAdjThreads) void k_adjoint_gather(
    const void* __restrict__ arena, const EdgeDev* __restrict__ edges, const EdgeXf* __restrict__ xf,
    const int32_t* __restrict__ idx_arena, const int64_t* __restrict__ kf_off, const int32_t* __restrict__ kf_npx,
    const int32_t* __restrict__ node_ptr, const int32_t* __restrict__ node_adj, const int64_t* __restrict__ obase,
    const int64_t* __restrict__ sbase, const int64_t* __restrict__ cbase, const int32_t* __restrict__ inv_off,
    const int32_t* __restrict__ inv_src, const int32_t* __restrict__ inv_head, GnConst k, float dcost,
    float* __restrict__ grad_xyz, float* __restrict__ grad_conf, float* __restrict__ part7, int stride) {
  using raw_t = typename Px<DT>::raw_t;
  const int kf = blockIdx.y;
  const int tile = blockIdx.x;
  const int npx = kf_npx[kf];
  if (tile * kAdjThreads * kAdjPPT >= npx) return;  // uniform per block
  const int64_t off = kf_off[kf];
  const int p0 = tile * kAdjThreads * kAdjPPT + threadIdx.x;
  raw_t xr[kAdjPPT];
  float acc[kAdjPPT][4];
#pragma unroll
  for (int u = 0; u < kAdjPPT; ++u) {
    const int n = p0 + u * kAdjThreads;
    xr[u] = Px<DT>::load_raw(arena, off + (n < npx ? n : 0));
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[u][c] = 0.0f;
  }
  const int q0 = node_ptr[kf], q1 = node_ptr[kf + 1];
  for (int q = q0; q < q1; ++q) {  // query side: pixel n of this keyframe, its match m in i
    const int code = node_adj[q];
    if (!(code & 1)) continue;
    const int e = code >> 1;
    const EdgeDev E = edges[e];
    float M[12];
#pragma unroll
    for (int r = 0; r < 12; ++r) M[r] = xf[e].m[r];
    const int32_t* idx = idx_arena + E.idx_off;
    // every load of the edge first: the matches, then the matched pixels
    int32_t mm[kAdjPPT];
#pragma unroll
    for (int u = 0; u < kAdjPPT; ++u) {
      const int n = p0 + u * kAdjThreads;
      mm[u] = (n < npx) ? idx[n] : -1;
      mm[u] = (mm[u] < E.npx_i) ? mm[u] : -1;
    }
    raw_t xi[kAdjPPT];
#pragma unroll
    for (int u = 0; u < kAdjPPT; ++u) xi[u] = Px<DT>::load_raw(arena, E.off_i + (mm[u] >= 0 ? mm[u] : 0));
    float g8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < kAdjPPT; ++u) {
      if (mm[u] < 0) continue;
      const float4 Xj = Px<DT>::unpack(xr[u]);
      AdjPix o;
      if (!adj_pixel(Xj, Px<DT>::unpack(xi[u]), M, k, dcost, o)) continue;
      acc[u][0] += M[0] * o.gx[0] + M[3] * o.gx[1] + M[6] * o.gx[2];
      acc[u][1] += M[1] * o.gx[0] + M[4] * o.gx[1] + M[7] * o.gx[2];
      acc[u][2] += M[2] * o.gx[0] + M[5] * o.gx[1] + M[8] * o.gx[2];
      acc[u][3] += o.dc / (4.0f * Xj.w);
      g8[0] += o.gx[0];
      g8[1] += o.gx[1];
      g8[2] += o.gx[2];
      g8[3] += o.x[1] * o.gx[2] - o.x[2] * o.gx[1];
      g8[4] += o.x[2] * o.gx[0] - o.x[0] * o.gx[2];
      g8[5] += o.x[0] * o.gx[1] - o.x[1] * o.gx[0];
      g8[6] += o.x[0] * o.gx[0] + o.x[1] * o.gx[1] + o.x[2] * o.gx[2];
      g8[7] += o.rho;
    }
    // one partial per wave and edge (the waves of the block never wait for each other), summed in a
    // fixed order by the edge finalize
    float* pw = part7 + ((int64_t(e) * stride + tile) * kAdjWaves + (threadIdx.x >> 6)) * 8;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const float v = wave_sum_to_lane63(g8[c]);
      if ((threadIdx.x & 63) == 63) pw[c] = v;
    }
  }
  for (int q = q0; q < q1; ++q) {  // gathered side: pixel m of this keyframe, the query pixels matched to it
    const int code = node_adj[q];
    if (code & 1) continue;
    const int e = code >> 1;
    const EdgeDev E = edges[e];
    float M[12];
#pragma unroll
    for (int r = 0; r < 12; ++r) M[r] = xf[e].m[r];
    const int32_t* hd = inv_head + cbase[e];
    int h[kAdjPPT], n0[kAdjPPT];
#pragma unroll
    for (int u = 0; u < kAdjPPT; ++u) {
      const int m = p0 + u * kAdjThreads;
      h[u] = (m < npx) ? hd[m] : -1;
      n0[u] = (h[u] >= 0) ? h[u] : ((h[u] <= -2) ? -2 - h[u] : -1);
    }
    raw_t xj[kAdjPPT];
#pragma unroll
    for (int u = 0; u < kAdjPPT; ++u) xj[u] = Px<DT>::load_raw(arena, E.off_j + (n0[u] >= 0 ? n0[u] : 0));
#pragma unroll
    for (int u = 0; u < kAdjPPT; ++u) {
      if (n0[u] < 0) continue;
      const float4 Xi = Px<DT>::unpack(xr[u]);
      // the first query pixel from the head word; the rest of a longer list (rare) from the CSR, in
      // increasing n as before
      int x = 0, xe = 0;
      if (h[u] <= -2) {
        const int32_t* lo = inv_off + obase[e];
        const int m = p0 + u * kAdjThreads;
        x = lo[m];
        xe = lo[m + 1];
      }
      const int32_t* lst = inv_src + sbase[e];
      for (bool first = true; first || x + 1 < xe; first = false) {
        const float4 Xj = first ? Px<DT>::unpack(xj[u]) : Px<DT>::load(arena, E.off_j + lst[++x]);
        AdjPix o;
        if (!adj_pixel(Xj, Xi, M, k, dcost, o)) continue;
        const float pgi = o.pi[0] * o.gam[0] + o.pi[1] * o.gam[1] + o.pi[2] * o.gam[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[u][c] -= (o.gam[c] - o.pi[c] * pgi) * o.rdi + o.gam[3] * o.pi[c];
        acc[u][3] += o.dc / (4.0f * Xi.w);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kAdjPPT; ++u) {
    const int n = p0 + u * kAdjThreads;
    if (n >= npx) continue;
    float* gj = grad_xyz + 3 * (off + n);
    gj[0] = acc[u][0];
    gj[1] = acc[u][1];
    gj[2] = acc[u][2];
    grad_conf[off + n] = acc[u][3];
  }
}

// E_global alone (eq. 5), in the same (tile, edge) grid as the adjoint: per pixel the Huber cost of the
// four whitened residual components, with the validity rules, square roots and weights of the GN
// reduction; per block one (cost, count) pair in the block's slot of part (stride 8).
template <int DT>
__global__ __launch_bounds__(kAdjThreads) void k_edge_cost(const void* __restrict__ arena,
                                                           const EdgeDev* __restrict__ edges,
                                                           const EdgeXf* __restrict__ xf,
                                                           const int32_t* __restrict__ idx_arena, GnConst k,
                                                           float* __restrict__ part) {
  const int e = blockIdx.y;
  const EdgeDev E = edges[e];
  const int tile = blockIdx.x;
  const int tiles_e = (E.npx_j + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  if (tile >= tiles_e) return;  // uniform per block
  float M[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) M[q] = xf[e].m[q];
  const int32_t* idx = idx_arena + E.idx_off;
  float cost = 0.0f, cnt = 0.0f;
#pragma unroll 2
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
    const float mn = fminf(fminf(d2, di2), dj2);
    const float sum = (d2 + di2) + (dj2 + cc);
    if (!(mn > 1e-18f) || !(cc >= 0.0f) || !(sum < __builtin_huge_valf())) continue;
    const float rd = rsqrtf(d2), rdi = rsqrtf(di2);
    const float e4[4] = {x0 * rd - Xi.x * rdi, x1 * rd - Xi.y * rdi, x2 * rd - Xi.z * rdi, d2 * rd - di2 * rdi};
    const float sq = __builtin_amdgcn_sqrtf(__builtin_amdgcn_sqrtf(cc));
    const float isg[4] = {k.inv_sr, k.inv_sr, k.inv_sr, k.inv_sd};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float a = fabsf(sq * isg[c] * e4[c]);
      const float t = fminf(1.0f, k.kappa * __builtin_amdgcn_rcpf(a)) * a;  // rho = t (|r| - t/2)
      cost = fmaf(t, fmaf(-0.5f, t, a), cost);
    }
    cnt += 1.0f;
  }
  __shared__ float red[kAdjThreads / kWave][2];
  cost = wave_sum(cost);
  cnt = wave_sum(cnt);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = cost;
    red[threadIdx.x >> 6][1] = cnt;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    float s = 0.0f;
    for (int w = 0; w < kAdjThreads / kWave; ++w) s += red[w][threadIdx.x];
    part[(int64_t(e) * gridDim.x + tile) * 8 + threadIdx.x] = s;
  }
}

// Per edge: cost and count from the tile pairs, float64 / int64, in tile order.
__global__ void k_cost_edge_finalize(const EdgeDev* __restrict__ edges, int tiles_stride,
                                     const float* __restrict__ part, double* __restrict__ cost_e,
                                     int64_t* __restrict__ count_e, int n_edges) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_edges) return;
  const int tiles_e = (edges[e].npx_j + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  double c = 0.0;
  int64_t n = 0;
  for (int t = 0; t < tiles_e; ++t) {
    c += double(part[(int64_t(e) * tiles_stride + t) * 8]);
    n += int64_t(part[(int64_t(e) * tiles_stride + t) * 8 + 1]);
  }
  cost_e[e] = c;
  count_e[e] = n;
}

int launch_cost_batched(ds3_dtype dt, const void* arena, const EdgeDev* edges, int n_edges, int max_npx_j,
                        const EdgeXf* xf, const int32_t* idx, GnConst c, float* part, double* cost_e,
                        int64_t* count_e, hipStream_t s) {
  const int tiles = (max_npx_j + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  if (n_edges <= 0 || tiles <= 0) return 0;
  dim3 grid(tiles, n_edges), block(kAdjThreads);
  if (dt == DS3_F32)
    hipLaunchKernelGGL(k_edge_cost<DS3_F32>, grid, block, 0, s, arena, edges, xf, idx, c, part);
  else
    hipLaunchKernelGGL(k_edge_cost<DS3_BF16>, grid, block, 0, s, arena, edges, xf, idx, c, part);
  DS3_TRY(check_hip(hipGetLastError(), "k_edge_cost"));
  hipLaunchKernelGGL(k_cost_edge_finalize, dim3((n_edges + 63) / 64), dim3(64), 0, s, edges, tiles, part, cost_e,
                     count_e, n_edges);
  return check_hip(hipGetLastError(), "k_cost_edge_finalize");
}

// Per edge: b_e = Ad^T (sum of tile pieces), float64.
// With cost_e, slot 7 of the tile pieces (the tile's Huber cost) is summed into cost_e and count_e is
// cleared.
__global__ void k_adjoint_edge_finalize(const EdgeDev* __restrict__ edges, int tiles_stride,
                                        const float* __restrict__ part7, const double* __restrict__ Ad,
                                        double* __restrict__ b_e, int n_edges, double* __restrict__ cost_e,
                                        int64_t* __restrict__ count_e) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_edges) return;
  const EdgeDev E = edges[e];
  const int tiles_e = (E.npx_j + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int t = 0; t < tiles_e; ++t)
    for (int w = 0; w < kAdjWaves; ++w)
      for (int c = 0; c < 8; ++c) s[c] += double(part7[((int64_t(e) * tiles_stride + t) * kAdjWaves + w) * 8 + c]);
  if (cost_e) {
    cost_e[e] = s[7];
    count_e[e] = 0;
  }
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
  return n_edges * tiles * kAdjWaves * 8;
}

int launch_adjoint(ds3_dtype dt, const void* arena, const EdgeDev* edges, int n_edges, int max_npx_j,
                   int max_npx_kf, const EdgeXf* xf, const double* Ad, const int32_t* idx, GnConst c,
                   float dcost, float* grad_xyz, float* grad_conf, float* part7, double* b_e, int n_kf,
                   const int64_t* kf_off, const int32_t* kf_npx, const int32_t* node_ptr,
                   const int32_t* node_adj, double* grad_tau, ds3_timer* timer, hipStream_t s) {
  const int tiles = (max_npx_j + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  const int tiles_kf = (max_npx_kf + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  DS3_TRY(timer_record(timer, true, s));
  if (tiles_kf > 0) {
    dim3 grid(tiles_kf, n_kf), block(kAdjThreads);
    if (dt == DS3_F32)
      hipLaunchKernelGGL(k_adjoint_gather_j<DS3_F32>, grid, block, 0, s, arena, edges, xf, idx, kf_off, kf_npx,
                         node_ptr, node_adj, c, dcost, grad_xyz, grad_conf, part7, tiles);
    else
      hipLaunchKernelGGL(k_adjoint_gather_j<DS3_BF16>, grid, block, 0, s, arena, edges, xf, idx, kf_off, kf_npx,
                         node_ptr, node_adj, c, dcost, grad_xyz, grad_conf, part7, tiles);
    DS3_TRY(check_hip(hipGetLastError(), "k_adjoint_gather_j"));
  }
  if (n_edges > 0 && tiles > 0) {
    dim3 grid(tiles, n_edges), block(kAdjThreads);
    if (dt == DS3_F32)
      hipLaunchKernelGGL(k_adjoint_scatter_i<DS3_F32>, grid, block, 0, s, arena, edges, xf, idx, c, dcost,
                         grad_xyz, grad_conf);
    else
      hipLaunchKernelGGL(k_adjoint_scatter_i<DS3_BF16>, grid, block, 0, s, arena, edges, xf, idx, c, dcost,
                         grad_xyz, grad_conf);
    DS3_TRY(check_hip(hipGetLastError(), "k_adjoint_scatter_i"));
  }
  DS3_TRY(timer_record(timer, false, s));
  if (n_edges > 0 && tiles > 0) {
    hipLaunchKernelGGL(k_adjoint_edge_finalize, dim3((n_edges + 63) / 64), dim3(64), 0, s, edges, tiles, part7,
                       Ad, b_e, n_edges, static_cast<double*>(nullptr), static_cast<int64_t*>(nullptr));
    DS3_TRY(check_hip(hipGetLastError(), "k_adjoint_edge_finalize"));
  }
  hipLaunchKernelGGL(k_grad_tau, dim3((7 * n_kf + 127) / 128), dim3(128), 0, s, n_kf, node_ptr, node_adj, b_e,
                     grad_tau);
  return check_hip(hipGetLastError(), "k_grad_tau");
}

// One word per pixel m of keyframe i(e) for the gather: -1 when no query pixel is matched to m, the pixel
// n when exactly one is, -2 - n (n the first of the list) when several are (the rest stay in the CSR).
__global__ __launch_bounds__(256) void k_inv_head(const EdgeDev* __restrict__ edges,
                                                  const int64_t* __restrict__ cbase,
                                                  const int64_t* __restrict__ obase,
                                                  const int64_t* __restrict__ sbase,
                                                  const int32_t* __restrict__ off, const int32_t* __restrict__ src,
                                                  int32_t* __restrict__ head) {
  const int e = blockIdx.y;
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= edges[e].npx_i) return;
  const int32_t* o = off + obase[e];
  const int a = o[m], b = o[m + 1];
  const int32_t n0 = (b > a) ? src[sbase[e] + a] : 0;
  head[cbase[e] + m] = (b == a) ? -1 : ((b == a + 1) ? n0 : -2 - n0);
}

int launch_inverse_maps(const EdgeDev* edges, int n_edges, int max_npx_j, int max_npx_i, const int32_t* idx,
                        const int64_t* cbase, const int64_t* obase, const int64_t* sbase, int32_t* cnt,
                        size_t cnt_len, int32_t* off, int32_t* src, int32_t* head, hipStream_t s) {
  if (n_edges <= 0) return 0;
  DS3_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(cnt), cnt_len, 0u, s));
  const dim3 gj((max_npx_j + 255) / 256, n_edges), gi((max_npx_i + 255) / 256, n_edges);
  hipLaunchKernelGGL(k_inv_count, gj, dim3(256), 0, s, edges, idx, cbase, cnt);
  DS3_TRY(check_hip(hipGetLastError(), "k_inv_count"));
  hipLaunchKernelGGL(k_inv_scan, dim3(n_edges), dim3(1024), 0, s, edges, cbase, obase, cnt, off);
  DS3_TRY(check_hip(hipGetLastError(), "k_inv_scan"));
  DS3_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(cnt), cnt_len, 0u, s));
  hipLaunchKernelGGL(k_inv_fill, gj, dim3(256), 0, s, edges, idx, cbase, obase, sbase, off, cnt, src);
  DS3_TRY(check_hip(hipGetLastError(), "k_inv_fill"));
  hipLaunchKernelGGL(k_inv_sort, gi, dim3(256), 0, s, edges, obase, sbase, off, src);
  DS3_TRY(check_hip(hipGetLastError(), "k_inv_sort"));
  hipLaunchKernelGGL(k_inv_head, gi, dim3(256), 0, s, edges, cbase, obase, sbase, off, src, head);
  return check_hip(hipGetLastError(), "k_inv_head");
}

int launch_adjoint_gather(ds3_dtype dt, const void* arena, const EdgeDev* edges, int n_edges, int max_npx_j,
                          int max_npx_kf, const EdgeXf* xf, const double* Ad, const int32_t* idx, GnConst c,
                          float dcost, float* grad_xyz, float* grad_conf, float* part7, double* b_e,
                          double* cost_e, int64_t* count_e, int n_kf, const int64_t* kf_off,
                          const int32_t* kf_npx, const int32_t* node_ptr, const int32_t* node_adj,
                          const int64_t* obase, const int64_t* sbase, const int64_t* cbase,
                          const int32_t* inv_off, const int32_t* inv_src, const int32_t* inv_head, double* grad_tau,
                          ds3_timer* timer, hipStream_t s) {
  const int tiles = (max_npx_j + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  const int tiles_kf = (max_npx_kf + kAdjThreads * kAdjPPT - 1) / (kAdjThreads * kAdjPPT);
  DS3_TRY(timer_record(timer, true, s));
  if (tiles_kf > 0) {
    dim3 grid(tiles_kf, n_kf), block(kAdjThreads);
    if (dt == DS3_F32)
      hipLaunchKernelGGL(k_adjoint_gather<DS3_F32>, grid, block, 0, s, arena, edges, xf, idx, kf_off, kf_npx,
                         node_ptr, node_adj, obase, sbase, cbase, inv_off, inv_src, inv_head, c, dcost, grad_xyz,
                         grad_conf, part7, tiles);
    else
      hipLaunchKernelGGL(k_adjoint_gather<DS3_BF16>, grid, block, 0, s, arena, edges, xf, idx, kf_off, kf_npx,
                         node_ptr, node_adj, obase, sbase, cbase, inv_off, inv_src, inv_head, c, dcost, grad_xyz,
                         grad_conf, part7, tiles);
    DS3_TRY(check_hip(hipGetLastError(), "k_adjoint_gather"));
  }
  DS3_TRY(timer_record(timer, false, s));
  if (n_edges > 0 && tiles > 0) {
    hipLaunchKernelGGL(k_adjoint_edge_finalize, dim3((n_edges + 63) / 64), dim3(64), 0, s, edges, tiles, part7,
                       Ad, b_e, n_edges, cost_e, count_e);
    DS3_TRY(check_hip(hipGetLastError(), "k_adjoint_edge_finalize"));
  }
  hipLaunchKernelGGL(k_grad_tau, dim3((7 * n_kf + 127) / 128), dim3(128), 0, s, n_kf, node_ptr, node_adj, b_e,
                     grad_tau);
  return check_hip(hipGetLastError(), "k_grad_tau");
}

}  // namespace ds3
