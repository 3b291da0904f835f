// Regularised normal equations of eq. (7) with the epsilon ladder of the text after it:
//   (H + lambda diag H + eps_r I) tau = -g,  eps_r = eps0 * mult^r,  r = 0 .. attempts-1,
// and a zero update (status -1) when every factorisation fails.
//
// Right-looking blocked Cholesky over 32x32 float64 tiles, one kernel per panel so that kernel
// boundaries order the steps (no in-kernel grid barriers, no device-wide cache maintenance):
//   init      copy + regularise the lower tiles; the owner of tile (0, 0) factors it, inverts the factor
//             and starts the forward substitution of -g;
//   panel k   every workgroup owns one trailing tile (i, j), k < j <= i: it forms L_ik = A_ik L_kk^-T
//             (and L_jk) from the stored inverse, updates A_ij -= L_ik L_jk^T, stores L_ik and carries
//             the forward substitution when j = k+1, and the owner of (k+1, k+1) factors it right away;
//   backsub   one workgroup solves L^T x = y block by block.
// Attempt 0 runs this way; only when it fails does a persistent fallback kernel run attempts 1.. with its
// own bounded grid barriers (the common case never pays for the ladder).
#include "common.hpp"
#include "internal.hpp"

namespace ds3 {

constexpr int NB = 32;
constexpr int LDT = NB + 1;
constexpr int kCholThreads = 256;
constexpr long kSpinLimit = 1L << 24;
constexpr int kMaxAttempts = 16;

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
  double* Inv;  // nt tiles: inverse of each diagonal factor
  double* b;    // np: -g after forward elimination
  double* y;    // np: L^-1 (-g) per block
  double* x;    // np: solution blocks
  unsigned* sync;  // [0] barrier count, [1] generation, [2] error, [3] attempt-0 failed,
                   // [4 .. 4 + attempts*nt) failure of diagonal tile s in attempt r, then nt ready flags
};

// ---------------------------------------------------------------------------------------------------
// Tile helpers (32x32, lower triangular factors, LDS row stride LDT)
// ---------------------------------------------------------------------------------------------------
__device__ inline double rsqrt_full(double d) {
  double y = __builtin_amdgcn_rsq(d);  // hardware estimate, refined by two Newton steps
  y = y * fma(-0.5 * d * y, y, 1.5);
  y = y * fma(-0.5 * d * y, y, 1.5);
  return y;
}

__device__ inline void tile_load(double* T, const double* src, int ld) {
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) T[(e / NB) * LDT + e % NB] = src[int64_t(e / NB) * ld + e % NB];
}

__device__ inline void tile_store(const double* T, double* dst, int ld) {
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) dst[int64_t(e / NB) * ld + e % NB] = T[(e / NB) * LDT + e % NB];
}

// Lower Cholesky of the LDS tile in place (upper part zeroed); false on a non-positive or non-finite
// pivot. 256 threads; thread t owns column t % 32 of rows t / 32 + 8q. Two barriers per column.
__device__ bool tile_potrf(double* T) {
  const int s = threadIdx.x % NB;
  const int r0 = threadIdx.x / NB;
  for (int c = 0; c < NB; ++c) {
    __syncthreads();
    const double d = T[c * LDT + c];
    if (!(d > 0.0) || !isfinite(d)) return false;  // uniform: every thread read the same pivot
    const double y = rsqrt_full(d);
    const double ls = T[s * LDT + c] * y;
    double lr[NB * NB / kCholThreads];
#pragma unroll
    for (int q = 0; q < NB * NB / kCholThreads; ++q) lr[q] = T[(r0 + 8 * q) * LDT + c] * y;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB * NB / kCholThreads; ++q) {
      const int r = r0 + 8 * q;
      if (s == c && r >= c) T[r * LDT + c] = lr[q];  // r == c: d / sqrt(d) = sqrt(d)
      if (s > c && r >= s) T[r * LDT + s] = fma(-lr[q], ls, T[r * LDT + s]);
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NB * NB; e += kCholThreads)
    if (e % NB > e / NB) T[(e / NB) * LDT + e % NB] = 0.0;
  __syncthreads();
  return true;
}

// X = L^-1 (lower): column c solved by thread c with the column kept in registers (x_t = 0 for t < c,
// so the dot products can run over every t < r).
__device__ void tile_trinv(const double* Lt, double* X) {
  if (threadIdx.x < NB) {
    const int c = threadIdx.x;
    double x[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int t = 0; t < r; ++t) {
        if (t & 1) s1 = fma(Lt[r * LDT + t], x[t], s1);
        else s0 = fma(Lt[r * LDT + t], x[t], s0);
      }
      x[r] = (r >= c) ? (((r == c) ? 1.0 : 0.0) - (s0 + s1)) / Lt[r * LDT + r] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) X[r * LDT + c] = x[r];
  }
  __syncthreads();
}

// T <- T * Inv^T (Inv lower triangular): the panel solve L_ik = A_ik L_kk^-T.
__device__ inline void tile_mul_invT(double* T, const double* Inv) {
  double acc[NB * NB / kCholThreads];
  int q = 0;
  for (int e = threadIdx.x; e < NB * NB; e += kCholThreads, ++q) {
    const int r = e / NB, c = e % NB;
    double s = 0.0;
    for (int t = 0; t <= c; ++t) s = fma(T[r * LDT + t], Inv[c * LDT + t], s);
    acc[q] = s;
  }
  __syncthreads();
  q = 0;
  for (int e = threadIdx.x; e < NB * NB; e += kCholThreads, ++q) T[(e / NB) * LDT + e % NB] = acc[q];
  __syncthreads();
}

// ydst = Inv * bsrc (32 threads)
__device__ inline void tile_gemv_store(const double* Inv, const double* bsrc, double* ydst) {
  __syncthreads();
  if (threadIdx.x < NB) {
    const int r = threadIdx.x;
    double s = 0.0;
    for (int t = 0; t <= r; ++t) s = fma(Inv[r * LDT + t], bsrc[t], s);
    ydst[r] = s;
  }
  __syncthreads();
}

// Copy + regularise one lower tile of H into T (LDS); identity on padding.
__device__ inline void tile_from_H(const CholArgs& a, int i, int j, double eps, double* T) {
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int rr = i * NB + e / NB, cc = j * NB + e % NB;
    double v;
    if (rr < a.n && cc < a.n) {
      v = a.H[int64_t(rr) * a.n + cc];
      if (rr == cc) v += a.lambda * v + eps;
    } else {
      v = (rr == cc) ? 1.0 : 0.0;
    }
    T[(e / NB) * LDT + e % NB] = v;
  }
}

// Factor a diagonal tile in S1: L -> L buffer, inverse -> Inv buffer, y_i = Inv (b_i). False on failure.
__device__ bool factor_diag(const CholArgs& a, int i, double* S1, double* S2) {
  __syncthreads();
  if (!tile_potrf(S1)) return false;
  tile_store(S1, a.L + int64_t(i) * NB * a.np + i * NB, a.np);
  tile_trinv(S1, S2);
  tile_store(S2, a.Inv + int64_t(i) * NB * NB, NB);
  tile_gemv_store(S2, a.b + i * NB, a.y + i * NB);
  return true;
}

__device__ inline void tile_index(int tt, int& i, int& j) {
  i = 0;
  while ((i + 1) * (i + 2) / 2 <= tt) ++i;
  j = tt - i * (i + 1) / 2;
}

// ---------------------------------------------------------------------------------------------------
// Attempt 0: init, panels, back substitution
// ---------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kCholThreads) void k_chol_init(CholArgs a) {
  __shared__ double S1[NB * LDT];
  __shared__ double S2[NB * LDT];
  int i, j;
  tile_index(blockIdx.x, i, j);
  tile_from_H(a, i, j, a.eps0, S1);
  if (j == 0 && threadIdx.x < NB) {
    const int rr = i * NB + threadIdx.x;
    a.b[rr] = (rr < a.n) ? -a.g[rr] : 0.0;
  }
  __syncthreads();
  if (i == 0) {
    const bool ok = factor_diag(a, 0, S1, S2);
    if (threadIdx.x == 0) {
      a.sync[3] = ok ? 0u : 1u;
      *a.status = -2;  // replaced by the back substitution or the fallback
    }
  } else {
    tile_store(S1, a.Wm + int64_t(i) * NB * a.np + j * NB, a.np);
  }
}

__global__ __launch_bounds__(kCholThreads) void k_chol_panel(CholArgs a, int k) {
  if (a.sync[3] != 0u) return;  // attempt 0 already failed (uniform)
  __shared__ double S0[NB * LDT];
  __shared__ double S1[NB * LDT];
  __shared__ double S2[NB * LDT];
  const int np = a.np;
  int ii, jj;
  tile_index(blockIdx.x, ii, jj);
  const int i = k + 1 + ii, j = k + 1 + jj;
  tile_load(S0, a.Inv + int64_t(k) * NB * NB, NB);
  tile_load(S1, a.Wm + int64_t(i) * NB * np + k * NB, np);
  if (j != i) tile_load(S2, a.Wm + int64_t(j) * NB * np + k * NB, np);
  __syncthreads();
  tile_mul_invT(S1, S0);  // L_ik
  const double* Ljk = S1;
  if (j != i) {
    tile_mul_invT(S2, S0);  // L_jk
    Ljk = S2;
  }
  double acc[NB * NB / kCholThreads];
  int q = 0;
  double* Aij = a.Wm + int64_t(i) * NB * np + j * NB;
  for (int e = threadIdx.x; e < NB * NB; e += kCholThreads, ++q) {
    const int rr = e / NB, cc = e % NB;
    double s = Aij[int64_t(rr) * np + cc];
    for (int t = 0; t < NB; ++t) s = fma(-S1[rr * LDT + t], Ljk[cc * LDT + t], s);
    acc[q] = s;
  }
  if (j == k + 1) {
    tile_store(S1, a.L + int64_t(i) * NB * np + k * NB, np);
    if (threadIdx.x < NB) {
      const int rr = threadIdx.x;
      double s = 0.0;
      for (int t = 0; t < NB; ++t) s = fma(S1[rr * LDT + t], a.y[k * NB + t], s);
      a.b[i * NB + rr] -= s;
    }
  }
  __syncthreads();
  if (i == j && i == k + 1) {
    q = 0;
    for (int e = threadIdx.x; e < NB * NB; e += kCholThreads, ++q) S1[(e / NB) * LDT + e % NB] = acc[q];
    const bool ok = factor_diag(a, i, S1, S2);
    if (!ok && threadIdx.x == 0) a.sync[3] = 1u;
  } else {
    q = 0;
    for (int e = threadIdx.x; e < NB * NB; e += kCholThreads, ++q) Aij[int64_t(e / NB) * np + e % NB] = acc[q];
  }
}

// Back substitution L^T x = y by one workgroup of 1024 threads: for block k (last first),
// x_k = Inv_k^T (y_k - sum_{i>k} L_ik^T x_i); the sum is split over 32 row slices per column.
constexpr int kBackThreads = 1024;

__global__ __launch_bounds__(kBackThreads) void k_chol_backsub(CholArgs a) {
  if (a.sync[3] != 0u) {  // attempt 0 failed: the fallback takes over, or gives up with one attempt
    if (a.attempts == 1) {
      for (int k = threadIdx.x; k < a.n; k += kBackThreads) a.tau[k] = 0.0;
      if (threadIdx.x == 0) *a.status = -1;
    }
    return;
  }
  __shared__ double part[32][NB + 1];
  __shared__ double rhs[NB];
  const int c = threadIdx.x % NB, sl = threadIdx.x / NB;  // column within the block, row slice
  const int np = a.np;
  for (int k = a.nt - 1; k >= 0; --k) {
    const int c0 = k * NB;
    double s = 0.0;
    for (int row = c0 + NB + sl; row < np; row += 32) s = fma(a.L[int64_t(row) * np + c0 + c], a.x[row], s);
    part[sl][c] = s;
    __syncthreads();
    if (threadIdx.x < NB) {
      double t = 0.0;
      for (int q = 0; q < 32; ++q) t += part[q][threadIdx.x];
      rhs[threadIdx.x] = a.y[c0 + threadIdx.x] - t;
    }
    __syncthreads();
    if (threadIdx.x < NB) {
      const double* Inv = a.Inv + int64_t(k) * NB * NB;
      double v = 0.0;
      for (int t = threadIdx.x; t < NB; ++t) v = fma(Inv[t * NB + threadIdx.x], rhs[t], v);
      a.x[c0 + threadIdx.x] = v;
      if (c0 + threadIdx.x < a.n) a.tau[c0 + threadIdx.x] = v;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *a.status = 0;
}

// ---------------------------------------------------------------------------------------------------
// Fallback: attempts 1 .. attempts-1 in one persistent launch with bounded grid barriers
// ---------------------------------------------------------------------------------------------------
__device__ inline unsigned ld_acq(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

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
      tile_from_H(a, i, j, eps, S1);
      if (j == 0 && threadIdx.x < NB) {
        const int rr = i * NB + threadIdx.x;
        a.b[rr] = (rr < n) ? -a.g[rr] : 0.0;
      }
      __syncthreads();
      if (i == 0) {
        if (!factor_diag(a, 0, S1, S2) && threadIdx.x == 0) atomicOr(&fail_flag[r * nt], 1u);
      } else {
        tile_store(S1, a.Wm + int64_t(i) * NB * np + j * NB, np);
      }
      __syncthreads();
    }
    if (!grid_barrier(a.sync, G)) return;
    bool failed = ld_acq(&fail_flag[r * nt]) != 0u;
    for (int k = 0; k + 1 < nt && !failed; ++k) {
      const int m = nt - k - 1;
      const int n_tiles = m * (m + 1) / 2;
      bool have_inv = false;
      for (int tt = w; tt < n_tiles; tt += G) {
        int ii, jj;
        tile_index(tt, ii, jj);
        const int i = k + 1 + ii, j = k + 1 + jj;
        if (!have_inv) {
          tile_load(S0, a.Inv + int64_t(k) * NB * NB, NB);
          have_inv = true;
        }
        tile_load(S1, a.Wm + int64_t(i) * NB * np + k * NB, np);
        __syncthreads();
        tile_mul_invT(S1, S0);
        const double* Ljk = S1;
        if (j != i) {
          tile_load(S2, a.Wm + int64_t(j) * NB * np + k * NB, np);
          __syncthreads();
          tile_mul_invT(S2, S0);
          Ljk = S2;
        }
        double acc[NB * NB / kCholThreads];
        int q = 0;
        double* Aij = a.Wm + int64_t(i) * NB * np + j * NB;
        for (int e = threadIdx.x; e < NB * NB; e += kCholThreads, ++q) {
          const int rr = e / NB, cc = e % NB;
          double s = Aij[int64_t(rr) * np + cc];
          for (int t = 0; t < NB; ++t) s = fma(-S1[rr * LDT + t], Ljk[cc * LDT + t], s);
          acc[q] = s;
        }
        if (j == k + 1) {
          tile_store(S1, a.L + int64_t(i) * NB * np + k * NB, np);
          __syncthreads();
          if (threadIdx.x < NB) {
            const int rr = threadIdx.x;
            double s = 0.0;
            for (int t = 0; t < NB; ++t) s = fma(S1[rr * LDT + t], a.y[k * NB + t], s);
            a.b[i * NB + rr] -= s;
          }
        }
        __syncthreads();
        if (i == j && i == k + 1) {
          q = 0;
          for (int e = threadIdx.x; e < NB * NB; e += kCholThreads, ++q) S1[(e / NB) * LDT + e % NB] = acc[q];
          if (!factor_diag(a, i, S1, S2) && threadIdx.x == 0) atomicOr(&fail_flag[r * nt + k + 1], 1u);
        } else {
          q = 0;
          for (int e = threadIdx.x; e < NB * NB; e += kCholThreads, ++q)
            Aij[int64_t(e / NB) * np + e % NB] = acc[q];
        }
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

int launch_chol_ladder(const double* H, const double* g, int n, double lambda, double eps0, double mult,
                       int attempts, double* tau, int32_t* status, void* ws, hipStream_t s) {
  if (n <= 0 || !H || !g || !tau || !status || !ws) return fail(DS3_EINVAL, "chol: bad arguments");
  if (attempts < 1 || attempts > kMaxAttempts) return fail(DS3_EINVAL, "chol: attempts out of range");
  CholArgs a;
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
  // barrier words start at zero (a fill kernel, not a memset, so the sequence can be captured)
  DS3_TRY(launch_fill_u32(a.sync, 3, 0u, s));
  hipLaunchKernelGGL(k_chol_init, dim3(a.nt * (a.nt + 1) / 2), dim3(kCholThreads), 0, s, a);
  DS3_TRY(check_hip(hipGetLastError(), "k_chol_init"));
  for (int k = 0; k + 1 < a.nt; ++k) {
    const int m = a.nt - k - 1;
    hipLaunchKernelGGL(k_chol_panel, dim3(m * (m + 1) / 2), dim3(kCholThreads), 0, s, a, k);
    DS3_TRY(check_hip(hipGetLastError(), "k_chol_panel"));
  }
  hipLaunchKernelGGL(k_chol_backsub, dim3(1), dim3(kBackThreads), 0, s, a);
  DS3_TRY(check_hip(hipGetLastError(), "k_chol_backsub"));
  if (attempts > 1) {
    int G = (a.nt - 1) * a.nt / 2;
    if (G < 1) G = 1;
    if (G > 128) G = 128;
    hipLaunchKernelGGL(k_chol_fallback, dim3(G), dim3(kCholThreads), 0, s, a);
    DS3_TRY(check_hip(hipGetLastError(), "k_chol_fallback"));
  }
  return DS3_OK;
}

}  // namespace ds3
