// Regularised normal equations of eq. (7) with the epsilon ladder of the text after it:
//   (H + lambda diag H + eps_r I) tau = -g,  eps_r = eps0 * mult^r,  r = 0 .. attempts-1,
// and a zero update (status -1) when every factorisation fails.
//
// Right-looking blocked Cholesky over 32x32 float64 tiles, one kernel per panel so that kernel
// boundaries order the steps (no in-kernel grid barriers, no device-wide cache maintenance):
//   init      copy + regularise the lower tiles; the owner of tile (0, 0) factors it;
//   panel k   every workgroup owns one trailing tile (i, j), k < j <= i: it forms L_ik = A_ik L_kk^-T
//             (and L_jk) from the stored inverse, updates A_ij -= L_ik L_jk^T, stores L_ik and carries
//             the forward substitution when j = k+1, and the owner of (k+1, k+1) factors it right away;
//   backsub   ceil(nt / 8) workgroups solve L^T x = y, each owning eight diagonal blocks and passing
//             the solved blocks down through flags.
// A diagonal factorisation produces the inverse of L_kk and y_k = L_kk^-1 b_k: the inverse is accumulated
// by the same column updates that form L, four columns per barrier; L_kk itself is never stored.
// Attempt 0 runs this way; only when it fails does a persistent fallback kernel run attempts 1.. with its
// own bounded grid barriers (the common case never pays for the ladder).
//
// Tile products run on the float64 MFMA; LDS tiles use row stride NB + 2.
#include "chol_tile.hpp"
#include "internal.hpp"

namespace ds3 {

constexpr int kCholThreads = 256;
constexpr long kSpinLimit = 1L << 24;
constexpr int kMaxAttempts = 16;
constexpr int kMaxN = 8192;

struct CholArgs {
  const double* H;
  const double* g;
  int n, np, nt;
  double lambda, eps0, mult;
  int attempts;
  double* tau;
  int32_t* status;
  double* Wm;   // np x np working copy (lower tiles)
  double* L;    // np x np factor (lower tiles)
  double* Inv;  // nt tiles: inverse of each diagonal factor (row-major 32x32, zero above the diagonal)
  double* b;    // np: -g after forward elimination
  double* y;    // np: L^-1 (-g) per block
  double* x;    // np: solution blocks as published by the back substitutions
  unsigned* sync;  // [0] barrier count, [1] generation, [2] error, [3] attempt-0 failed,
                   // [4 .. 4 + attempts*nt) failure of diagonal tile s in attempt r, then nt ready flags
                   // of the fallback
};

// Stores the inverse of the diagonal factor and y_i = L_ii^-1 b_i (b_i in LDS sb). S: a free LDS tile.
// (The diagonal factor itself is not needed afterwards: the panels and both substitutions use its
// inverse.)
__device__ void store_diag(const CholArgs& a, int i, const f64x4& Xq, double* S, const double* sb) {
  diag_out(a.Inv + int64_t(i) * NB * NB, a.y + i * NB, Xq, S, sb);
}

// Regularised lower tile (i, j) of H as a fragment; identity on padding, zero above the diagonal.
__device__ inline void frag_from_H(const CholArgs& a, int i, int j, double eps, f64x4& q) {
  const int cc = j * NB + fcol();
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rr = i * NB + frow(v);
    double x;
    if (rr < a.n && cc < a.n) {
      x = (cc <= rr) ? a.H[int64_t(rr) * a.n + cc] : 0.0;
      if (rr == cc) x += a.lambda * x + eps;
    } else {
      x = (rr == cc) ? 1.0 : 0.0;
    }
    q[v] = x;
  }
}

// Init of one lower tile for regularisation eps. The owner of (0, 0) factors it; returns its success
// (true for every other tile).
__device__ bool init_tile(const CholArgs& a, int i, int j, double eps, double* S, double* fb) {
  f64x4 q;
  frag_from_H(a, i, j, eps, q);
  double* sb = fb + 4 * kFw * NB;
  if (j == 0 && threadIdx.x < NB) {
    const int rr = i * NB + threadIdx.x;
    const double bv = (rr < a.n) ? -a.g[rr] : 0.0;
    a.b[rr] = bv;
    if (i == 0) sb[threadIdx.x] = bv;
  }
  if (i != 0) {
    frag_store(q, a.Wm + int64_t(i) * NB * a.np + j * NB, a.np);
    return true;
  }
  __syncthreads();
  f64x4 Xq;
  if (!factor_frag(q, fb, Xq)) return false;
  store_diag(a, 0, Xq, S, sb);
  return true;
}

// Trailing tile (i, j) of panel k. Returns false only for the next diagonal tile (i = j = k+1) when its
// factorisation fails.
__device__ bool panel_tile(const CholArgs& a, int k, int i, int j, double* S0, double* S1, double* S2,
                           double* fb) {
  const int np = a.np;
  const bool offd = (j != i);
  const bool col = (j == k + 1);  // this workgroup stores L_ik and eliminates b_i
  // the next diagonal tile is on the critical path of the whole factorisation: its waves get issue
  // priority over the other workgroups sharing their compute unit
  if (i == j && i == k + 1) __builtin_amdgcn_s_setprio(3);
  f64x4 qinv, qi, qj, qa;
  frag_load(qinv, a.Inv + int64_t(k) * NB * NB, NB);
  frag_load(qi, a.Wm + int64_t(i) * NB * np + k * NB, np);
  if (offd) frag_load(qj, a.Wm + int64_t(j) * NB * np + k * NB, np);
  frag_load(qa, a.Wm + int64_t(i) * NB * np + j * NB, np);
  double yk = 0.0, bi = 0.0;
  if (col && threadIdx.x < NB) yk = a.y[k * NB + threadIdx.x];
  if (col && (threadIdx.x & 7) == 0) bi = a.b[i * NB + (threadIdx.x >> 3)];
  __syncthreads();  // previous users of S0..S2 and fb (fallback loop) are done
  frag_to_lds(qinv, S0);
  frag_to_lds(qi, S1);
  if (offd) frag_to_lds(qj, S2);
  double* sy = fb + 2 * kFw * NB;  // y_k while the factor scratch is unused (parity-1 buffer)
  double* sb = fb + 4 * kFw * NB;
  if (col && threadIdx.x < NB) sy[threadIdx.x] = yk;
  __syncthreads();
  f64x4 li = {0.0, 0.0, 0.0, 0.0}, lj = {0.0, 0.0, 0.0, 0.0};
  frag_gemm_abt<false>(S1, S0, li);  // L_ik = A_ik Inv_k^T
  if (offd) frag_gemm_abt<false>(S2, S0, lj);
  __syncthreads();
  frag_to_lds(li, S1);
  if (offd) frag_to_lds(lj, S2);
  __syncthreads();
  frag_gemm_abt<true>(S1, offd ? S2 : S1, qa);  // A_ij -= L_ik L_jk^T
  if (col) {
    frag_store(li, a.L + int64_t(i) * NB * np + k * NB, np);
    // forward elimination b_i -= L_ik y_k on 8 threads per row, reduced with lane shuffles
    const int r = threadIdx.x >> 3, p = threadIdx.x & 7;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < NB / 8; ++q) acc = fma(S1[r * LDT + p + 8 * q], sy[p + 8 * q], acc);
    acc += __shfl_xor(acc, 1, 8);
    acc += __shfl_xor(acc, 2, 8);
    acc += __shfl_xor(acc, 4, 8);
    if (p == 0) {
      const double bv = bi - acc;
      a.b[i * NB + r] = bv;
      sb[r] = bv;
    }
  }
  if (i == j && i == k + 1) {
    __syncthreads();
    f64x4 Xq;
    if (!factor_frag(qa, fb, Xq)) return false;
    store_diag(a, i, Xq, S0, sb);
    return true;
  }
  frag_store(qa, a.Wm + int64_t(i) * NB * np + j * NB, np);
  return true;
}

// Lower-triangle tile number tt -> (i, j), j <= i, row by row.
__device__ inline void tile_index(int tt, int& i, int& j) {
  i = int((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > tt) --i;
  while ((i + 1) * (i + 2) / 2 <= tt) ++i;
  j = tt - i * (i + 1) / 2;
}

// Workgroups are dealt round-robin to the eight XCDs (block b to XCD b mod 8). Block 0 carries tile 0,
// whose diagonal factorisation is the critical path, and blocks 8 and 16 carry tiles 1 and 2, the two
// tiles the next panel's diagonal workgroup (again on XCD 0) starts from; the other blocks of XCD 0 carry
// nothing, so the critical tile has the compute units of an XCD nearly to itself, and tiles 3.. go to the
// remaining seven XCDs in block order. (The placement only affects speed.)
constexpr int kXcds = 8;
__device__ inline int tile_of_block(int b) {
  if (b % kXcds == 0) return (b / kXcds <= 2) ? b / kXcds : -1;
  return 3 + (b - b / kXcds - 1);
}

static int blocks_for_tiles(int tiles) {
  // enough blocks for tile `tiles - 1`: tiles 0..2 sit at blocks 0, 8, 16, tile t >= 3 at the
  // (t - 3)-th block that is not a multiple of 8
  if (tiles <= 3) return 8 * (tiles - 1) + 1;
  const int j = tiles - 4;  // index among the blocks that are not multiples of 8
  const int b = j + j / 7 + 1;
  return std::max(b + 1, 17);
}

// ---------------------------------------------------------------------------------------------------
// Attempt 0: init, panels, back substitution
// ---------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kCholThreads) void k_chol_init(CholArgs a) {
  __shared__ double S[NB * LDT];
  __shared__ double fb[kFactorScratch];
  const int t = tile_of_block(blockIdx.x);
  if (t < 0 || t >= a.nt * (a.nt + 1) / 2) return;  // uniform per block
  int i, j;
  tile_index(t, i, j);
  if (i == 0)  // every solution value starts as pending for the back substitution
    for (int k = threadIdx.x; k < a.np; k += blockDim.x)
      reinterpret_cast<unsigned long long*>(a.x)[k] = kXPending;
  const bool ok = init_tile(a, i, j, a.eps0, S, fb);
  if (i == 0 && threadIdx.x == 0) {
    a.sync[3] = ok ? 0u : 1u;
    *a.status = -2;  // replaced by the back substitution or the fallback
  }
}

__global__ __launch_bounds__(kCholThreads) void k_chol_panel(CholArgs a, int k) {
  if (a.sync[3] != 0u) return;  // attempt 0 already failed (uniform)
  __shared__ double S0[NB * LDT];
  __shared__ double S1[NB * LDT];
  __shared__ double S2[NB * LDT];
  __shared__ double fb[kFactorScratch];
  const int m = a.nt - k - 1;
  const int t = tile_of_block(blockIdx.x);
  if (t < 0 || t >= m * (m + 1) / 2) return;  // uniform per block
  int ii, jj;
  tile_index(t, ii, jj);
  if (!panel_tile(a, k, k + 1 + ii, k + 1 + jj, S0, S1, S2, fb) && threadIdx.x == 0) a.sync[3] = 1u;
}

__device__ inline unsigned ld_acq(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Back substitution L^T x = y over ceil(nt / 8) workgroups. Workgroup w owns the eight diagonal blocks
// [8w, 8w + 8). Its first eight waves keep, per owned column j, acc_j = sum over the rows below its block
// of L[row][j] x[row] (thread = column slot x half of the 32 rows of a block row) and keep the factor rows
// of the next two block rows in two register buffers, refilling a buffer right after its use. The ninth wave does everything on the chain: it waits for the x_i of later workgroups, solves its
// own blocks x_i = Inv_i^T (y_i - acc_i) from the Inv blocks staged in LDS at the start, and publishes
// them. A loaded value only becomes usable once every older load of its wave has returned (one in-order
// counter per wave), so the chain lives in a wave that has no loads in flight. Each published value is
// its own ready flag: x starts as a signalling-NaN pattern no arithmetic produces, the owner overwrites it
// with a relaxed agent-scope store and the readers poll the 32 values of the block, so no fence sits on
// the chain.
// Every wait is bounded; a timeout sets sync[2], zeroes the workgroup's part of tau and ends in status -2.
constexpr int kBsBlocks = 8;
constexpr int kBsCols = kBsBlocks * NB;       // 256
constexpr int kBsColThreads = 2 * kBsCols;    // 512
constexpr int kBsThreads = kBsColThreads + 64;
constexpr int kBsRows = NB / 2;               // rows of a block row per column thread

__device__ inline unsigned long long x_load(const double* p) {
  return __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kBsThreads) void k_chol_backsub(CholArgs a) {
  const int nt = a.nt, w = blockIdx.x;
  const int b0 = w * kBsBlocks, b1 = min(nt, b0 + kBsBlocks);
  if (a.sync[3] != 0u) {  // attempt 0 failed: the fallback takes over, or gives up with one attempt
    if (a.attempts == 1) {
      for (int k = b0 * NB + threadIdx.x; k < min(a.n, b1 * NB); k += kBsThreads) a.tau[k] = 0.0;
      if (w == 0 && threadIdx.x == 0) *a.status = -1;
    }
    return;
  }
  __shared__ double sinv[kBsBlocks * NB * NB];  // Inv of the eight own blocks, staged once
  __shared__ double ys[kBsCols];
  __shared__ double red[2][kBsCols];
  __shared__ double xs[NB];
  __shared__ int s_ok;
  const int t = threadIdx.x;
  const bool chain = t >= kBsColThreads;  // the ninth wave
  for (int e = t; e < kBsBlocks * NB * NB; e += kBsThreads) {
    const int blk = b0 + e / (NB * NB);
    sinv[e] = (blk < b1) ? a.Inv[int64_t(b0) * NB * NB + e] : 0.0;
  }
  const int cs = t & (kBsCols - 1), h = (t >> 8) & 1;
  const int col = b0 * NB + cs;
  const bool has_col = !chain && col < b1 * NB;
  const int64_t np = a.np;
  if (t < kBsCols) ys[t] = (col < b1 * NB) ? a.y[col] : 0.0;
  // column waves: factor rows of block row i from a clamped (always valid) address; entries outside the
  // strictly lower part are masked where they are used, so that no load is waited for before its use
  auto load_rows = [&](int i, double* buf) {
    const int ii = max(i, 0);
#pragma unroll
    for (int r = 0; r < kBsRows; ++r) buf[r] = a.L[int64_t(ii * NB + kBsRows * h + r) * np + (has_col ? col : 0)];
  };
  // chain wave: lane l solves column c = l % 32 over the half u in 16 (l / 32) .. + 15
  const int lc = t & 31, lh = (t >> 5) & 1;
  double R0[kBsRows], R1[kBsRows];
  if (!chain) {
    load_rows(nt - 1, R0);
    load_rows(nt - 2, R1);
  }
  double acc = 0.0;
  bool ok = true;
  // one block row: the column waves apply cur (rows of block row i) once x_i is in xs and then refill it
  // with block row i - 2; the chain wave either waits for x_i or solves it from Inv_i in LDS
  auto step = [&](int i, double* cur) {
    if (!chain) red[h][cs] = acc;
    __syncthreads();  // acc of block i complete in red
    if (chain) {
      if (i >= b1) {  // a later workgroup's block
        const double* px = a.x + i * NB + lc;
        long spins = 0;
        bool good = true;
        unsigned long long v = x_load(px);
        while (!__all(v != kXPending)) {
          if (++spins > kSpinLimit || ld_acq(&a.sync[2]) != 0u) {
            good = false;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          v = x_load(px);
        }
        if (t == kBsColThreads) {
          if (!good) atomicOr(&a.sync[2], 1u);
          s_ok = good;
        }
        if (lh == 0) xs[lc] = __longlong_as_double(static_cast<long long>(v));
      } else {  // own block: x_i[c] = sum_{u >= c} Inv_i[u][c] (y_i[u] - acc_i[u])
        const int base = (i - b0) * NB;
        const double* inv = sinv + (i - b0) * NB * NB;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < kBsRows; ++q) {
          const int u = 16 * lh + q;
          v = fma(inv[u * NB + lc], ys[base + u] - (red[0][base + u] + red[1][base + u]), v);
        }
        v += __shfl_xor(v, 32);
        if (lh == 0) {
          xs[lc] = v;
          if (i * NB + lc < a.n) a.tau[i * NB + lc] = v;
          __hip_atomic_store(reinterpret_cast<unsigned long long*>(a.x + i * NB + lc),
                             static_cast<unsigned long long>(__double_as_longlong(v)), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        }
        if (t == kBsColThreads) s_ok = 1;
      }
    }
    __syncthreads();  // x_i in xs
    if (!s_ok) {
      ok = false;
      return;
    }
    if (!chain) {
      if (has_col && col < i * NB) {
#pragma unroll
        for (int r = 0; r < kBsRows; ++r) acc = fma(cur[r], xs[kBsRows * h + r], acc);
      }
      load_rows(i - 2, cur);  // two buffers: this one is current again at block row i - 2
    }
  };
  for (int i = nt - 1; i >= b0 && ok; i -= 2) {
    step(i, R0);
    if (i - 1 < b0 || !ok) break;
    step(i - 1, R1);
  }
  if (!ok) {
    for (int k = b0 * NB + t; k < min(a.n, b1 * NB); k += kBsThreads) a.tau[k] = 0.0;
    if (w == 0 && t == 0) *a.status = -2;
    return;
  }
  if (w == 0 && t == 0) *a.status = (ld_acq(&a.sync[2]) != 0u) ? -2 : 0;
}

// ---------------------------------------------------------------------------------------------------
// Fallback: attempts 1 .. attempts-1 in one persistent launch with bounded grid barriers
// ---------------------------------------------------------------------------------------------------

// Grid-wide barrier; false when the wait timed out or another workgroup reported an error.
__device__ bool grid_barrier(unsigned* sync, unsigned nblocks) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    __threadfence();
    const unsigned g0 = ld_acq(&sync[1]);
    const unsigned arrived = atomicAdd(&sync[0], 1u);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&sync[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      __hip_atomic_fetch_add(&sync[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long spins = 0;
      while (ld_acq(&sync[1]) == g0) {
        if (ld_acq(&sync[2]) != 0u || ++spins > kSpinLimit) {
          atomicOr(&sync[2], 1u);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __threadfence();
    s_ok = ok && (ld_acq(&sync[2]) == 0u);
  }
  __syncthreads();
  return s_ok != 0;
}

__global__ __launch_bounds__(kCholThreads) void k_chol_fallback(CholArgs a) {
  if (a.sync[3] == 0u) return;  // attempt 0 succeeded (uniform)
  __shared__ double S0[NB * LDT];
  __shared__ double S1[NB * LDT];
  __shared__ double S2[NB * LDT];
  __shared__ double fb[kFactorScratch];
  const unsigned G = gridDim.x;
  const int w = blockIdx.x;
  const int nt = a.nt, np = a.np, n = a.n;
  // fail_flag[r * nt + s]: diagonal tile s failed in attempt r; one slot per (attempt, tile) so a flag
  // read after a barrier can only have been written before that barrier.
  unsigned* fail_flag = a.sync + 4;
  unsigned* ready = a.sync + 4 + a.attempts * nt;
  if (w == 0)
    for (int k = threadIdx.x; k < (a.attempts + 1) * nt; k += kCholThreads) a.sync[4 + k] = 0u;
  if (!grid_barrier(a.sync, G)) return;
  int result = -1;
  double eps = a.eps0 * a.mult;
  for (int r = 1; r < a.attempts; ++r, eps *= a.mult) {
    const int n_lower = nt * (nt + 1) / 2;
    for (int tt = w; tt < n_lower; tt += G) {
      int i, j;
      tile_index(tt, i, j);
      __syncthreads();
      if (!init_tile(a, i, j, eps, S0, fb) && threadIdx.x == 0) atomicOr(&fail_flag[r * nt], 1u);
      __syncthreads();
    }
    if (!grid_barrier(a.sync, G)) return;
    bool failed = ld_acq(&fail_flag[r * nt]) != 0u;
    for (int k = 0; k + 1 < nt && !failed; ++k) {
      const int m = nt - k - 1;
      const int n_tiles = m * (m + 1) / 2;
      for (int tt = w; tt < n_tiles; tt += G) {
        int ii, jj;
        tile_index(tt, ii, jj);
        if (!panel_tile(a, k, k + 1 + ii, k + 1 + jj, S0, S1, S2, fb) && threadIdx.x == 0)
          atomicOr(&fail_flag[r * nt + k + 1], 1u);
        __syncthreads();
      }
      if (!grid_barrier(a.sync, G)) return;
      failed = ld_acq(&fail_flag[r * nt + k + 1]) != 0u;
    }
    if (!failed) {
      result = r;
      break;
    }
  }
  if (result < 0) {
    if (w == 0) {
      for (int k = threadIdx.x; k < n; k += kCholThreads) a.tau[k] = 0.0;
      if (threadIdx.x == 0) *a.status = -1;
    }
    return;
  }
  // back substitution as a dataflow wave: block k owned by workgroup k mod G, highest blocks first
  __shared__ double acc_s[NB];
  __shared__ int s_ok;
  const int k_first = (w < nt) ? w + ((nt - 1 - w) / int(G)) * int(G) : -1;
  for (int k = k_first; k >= 0; k -= int(G)) {
    if (threadIdx.x < NB) acc_s[threadIdx.x] = 0.0;
    __syncthreads();
    for (int i = nt - 1; i > k; --i) {
      if (threadIdx.x == 0) {
        long spins = 0;
        int ok = 1;
        while (ld_acq(&ready[i]) == 0u) {
          if (ld_acq(&a.sync[2]) != 0u || ++spins > kSpinLimit) {
            atomicOr(&a.sync[2], 1u);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        s_ok = ok;
      }
      __syncthreads();
      if (!s_ok) return;
      if (threadIdx.x < NB) {
        const int c = threadIdx.x;
        const double* Lik = a.L + int64_t(i) * NB * np + k * NB;
        double s = 0.0;
        for (int t = 0; t < NB; ++t) s += Lik[int64_t(t) * np + c] * a.x[i * NB + t];
        acc_s[c] += s;
      }
      __syncthreads();
    }
    if (threadIdx.x < NB) {
      const int c = threadIdx.x;
      const double* Inv = a.Inv + int64_t(k) * NB * NB;
      double s = 0.0;
      for (int t = c; t < NB; ++t) s += Inv[t * NB + c] * (a.y[k * NB + t] - acc_s[t]);
      a.x[k * NB + c] = s;
      const int rr = k * NB + c;
      if (rr < n) a.tau[rr] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      __hip_atomic_store(&ready[k], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (k == 0) *a.status = result;
    }
    __syncthreads();
  }
}

static void chol_dims(int n, int& nt, int& np) {
  nt = (n + NB - 1) / NB;
  if (nt < 1) nt = 1;
  np = nt * NB;
}

size_t chol_workspace_bytes(int n) {
  int nt, np;
  chol_dims(n, nt, np);
  Carver c(nullptr);
  c.take<double>(size_t(np) * np);
  c.take<double>(size_t(np) * np);
  c.take<double>(size_t(nt) * NB * NB);
  c.take<double>(np);
  c.take<double>(np);
  c.take<double>(np);
  c.take<unsigned>(4 + (kMaxAttempts + 1) * nt);
  return c.used;
}

static int launch_backsub(const CholArgs& a, hipStream_t s) {
  const int groups = (a.nt + kBsBlocks - 1) / kBsBlocks;
  hipLaunchKernelGGL(k_chol_backsub, dim3(groups), dim3(kBsThreads), 0, s, a);
  return check_hip(hipGetLastError(), "k_chol_backsub");
}

static int chol_args(CholArgs& a, const double* H, const double* g, int n, double lambda, double eps0,
                     double mult, int attempts, double* tau, int32_t* status, void* ws) {
  if (n <= 0 || !H || !g || !tau || !status || !ws) return fail(DS3_EINVAL, "chol: bad arguments");
  if (n > kMaxN) return fail(DS3_EINVAL, "chol: n above 8192");
  if (attempts < 1 || attempts > kMaxAttempts) return fail(DS3_EINVAL, "chol: attempts out of range");
  chol_dims(n, a.nt, a.np);
  Carver c(ws);
  a.Wm = c.take<double>(size_t(a.np) * a.np);
  a.L = c.take<double>(size_t(a.np) * a.np);
  a.Inv = c.take<double>(size_t(a.nt) * NB * NB);
  a.b = c.take<double>(a.np);
  a.y = c.take<double>(a.np);
  a.x = c.take<double>(a.np);
  a.sync = c.take<unsigned>(4 + (kMaxAttempts + 1) * a.nt);
  a.H = H; a.g = g; a.n = n;
  a.lambda = lambda; a.eps0 = eps0; a.mult = mult; a.attempts = attempts;
  a.tau = tau; a.status = status;
  return DS3_OK;
}

unsigned* chol_sync_words(void* ws, int n) {
  int nt, np;
  chol_dims(n, nt, np);
  Carver c(ws);
  c.take<double>(size_t(np) * np);
  c.take<double>(size_t(np) * np);
  c.take<double>(size_t(nt) * NB * NB);
  c.take<double>(np);
  c.take<double>(np);
  c.take<double>(np);
  return c.take<unsigned>(4 + (kMaxAttempts + 1) * nt);
}

static int launch_fallback(const CholArgs& a, hipStream_t s) {
  int G = (a.nt - 1) * a.nt / 2;
  if (G < 1) G = 1;
  if (G > 128) G = 128;
  hipLaunchKernelGGL(k_chol_fallback, dim3(G), dim3(kCholThreads), 0, s, a);
  return check_hip(hipGetLastError(), "k_chol_fallback");
}

int launch_chol_fallback(const double* H, const double* g, int n, double lambda, double eps0, double mult,
                         int attempts, double* tau, int32_t* status, void* ws, hipStream_t s) {
  CholArgs a;
  DS3_TRY(chol_args(a, H, g, n, lambda, eps0, mult, attempts, tau, status, ws));
  return launch_fallback(a, s);
}

int launch_chol_ladder(const double* H, const double* g, int n, double lambda, double eps0, double mult,
                       int attempts, double* tau, int32_t* status, void* ws, hipStream_t s) {
  CholArgs a;
  DS3_TRY(chol_args(a, H, g, n, lambda, eps0, mult, attempts, tau, status, ws));
  // barrier words start at zero (a fill kernel, not a memset, so the sequence can be captured)
  DS3_TRY(launch_fill_u32(a.sync, 3, 0u, s));
  hipLaunchKernelGGL(k_chol_init, dim3(blocks_for_tiles(a.nt * (a.nt + 1) / 2)), dim3(kCholThreads), 0, s, a);
  DS3_TRY(check_hip(hipGetLastError(), "k_chol_init"));
  for (int k = 0; k + 1 < a.nt; ++k) {
    const int m = a.nt - k - 1;
    hipLaunchKernelGGL(k_chol_panel, dim3(blocks_for_tiles(m * (m + 1) / 2)), dim3(kCholThreads), 0, s, a, k);
    DS3_TRY(check_hip(hipGetLastError(), "k_chol_panel"));
  }
  DS3_TRY(launch_backsub(a, s));
  if (attempts > 1) DS3_TRY(launch_fallback(a, s));
  return DS3_OK;
}

}  // namespace ds3
