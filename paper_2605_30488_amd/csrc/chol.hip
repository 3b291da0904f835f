// Regularised normal equations of eq. (7) with the epsilon ladder of the text after it:
//   (H + lambda diag H + eps_r I) tau = -g,  eps_r = eps0 * mult^r,  r = 0 .. attempts-1,
// and a zero update (status -1) when every factorisation fails.
//
// One persistent launch: a right-looking blocked Cholesky over 32x32 float64 tiles with one grid barrier
// per panel. In step k every workgroup owns trailing tiles (i, j), k < j <= i; it forms L_ik = A_ik
// L_kk^-T (and L_jk) itself from the stored inverse of the diagonal factor, so the panel solve and the
// trailing update need no separate phase. The owner of (k+1, k+1) factors it right after its update;
// the owner of each (i, k+1) stores L_ik and carries the forward substitution of -g. Back substitution
// runs as a dataflow wave over per-block ready flags. Every wait is bounded: on a spin timeout the kernel
// records an error and all workgroups leave.
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
  unsigned* sync;  // [0] barrier count, [1] generation, [2] error, [3] pad,
                   // [4 .. 4 + attempts*nt) failure of diagonal tile s in attempt r, then nt ready flags
};

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

__device__ inline void tile_load(double* T, const double* src, int ld) {
  for (int e = threadIdx.x; e < NB * NB; e += kCholThreads) {
    int r = e / NB, c = e % NB;
    T[r * LDT + c] = src[int64_t(r) * ld + c];
  }
}

__device__ inline void tile_store(const double* T, double* dst, int ld) {
  for (int e = threadIdx.x; e < NB * NB; e += kCholThreads) {
    int r = e / NB, c = e % NB;
    dst[int64_t(r) * ld + c] = T[r * LDT + c];
  }
}

// T <- T * Inv^T (Inv lower triangular): the panel solve L_ik = A_ik L_kk^-T.
__device__ inline void tile_mul_invT(double* T, const double* Inv) {
  double acc[NB * NB / kCholThreads];
  int q = 0;
  for (int e = threadIdx.x; e < NB * NB; e += kCholThreads, ++q) {
    int r = e / NB, c = e % NB;
    double s = 0.0;
    for (int t = 0; t <= c; ++t) s += T[r * LDT + t] * Inv[c * LDT + t];
    acc[q] = s;
  }
  __syncthreads();
  q = 0;
  for (int e = threadIdx.x; e < NB * NB; e += kCholThreads, ++q) T[(e / NB) * LDT + e % NB] = acc[q];
  __syncthreads();
}

// In-place lower Cholesky of the tile; false on a non-positive or non-finite pivot (uniform result).
__device__ bool tile_potrf(double* T) {
  __shared__ int s_ok;
  for (int c = 0; c < NB; ++c) {
    __syncthreads();
    if (threadIdx.x == 0) {
      double d = T[c * LDT + c];
      int ok = (d > 0.0) && isfinite(d);
      s_ok = ok;
      if (ok) T[c * LDT + c] = sqrt(d);
    }
    __syncthreads();
    if (!s_ok) return false;
    const double piv = T[c * LDT + c];
    for (int r = c + 1 + threadIdx.x; r < NB; r += kCholThreads) T[r * LDT + c] /= piv;
    __syncthreads();
    for (int e = threadIdx.x; e < NB * NB; e += kCholThreads) {
      int r = e / NB, s = e % NB;
      if (s > c && r >= s) T[r * LDT + s] -= T[r * LDT + c] * T[s * LDT + c];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NB * NB; e += kCholThreads) {
    int r = e / NB, c = e % NB;
    if (c > r) T[r * LDT + c] = 0.0;
  }
  __syncthreads();
  return true;
}

// X = L^-1 for the lower-triangular L (column c by thread c).
__device__ void tile_trinv(const double* Lt, double* X) {
  for (int e = threadIdx.x; e < NB * NB; e += kCholThreads) X[(e / NB) * LDT + e % NB] = 0.0;
  __syncthreads();
  if (threadIdx.x < NB) {
    const int c = threadIdx.x;
    for (int r = c; r < NB; ++r) {
      double s = (r == c) ? 1.0 : 0.0;
      for (int t = c; t < r; ++t) s -= Lt[r * LDT + t] * X[t * LDT + c];
      X[r * LDT + c] = s / Lt[r * LDT + r];
    }
  }
  __syncthreads();
}

// y_blk = Inv * b_blk (32 threads)
__device__ inline void tile_gemv_store(const double* Inv, const double* bsrc, double* ydst) {
  __syncthreads();
  if (threadIdx.x < NB) {
    const int r = threadIdx.x;
    double s = 0.0;
    for (int t = 0; t <= r; ++t) s += Inv[r * LDT + t] * bsrc[t];
    ydst[r] = s;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kCholThreads) void k_chol_ladder(CholArgs a) {
  __shared__ double S0[NB * LDT];  // Inv_k
  __shared__ double S1[NB * LDT];  // L_ik / diagonal work
  __shared__ double S2[NB * LDT];  // L_jk / inverse work
  const unsigned G = gridDim.x;
  const int w = blockIdx.x;
  const int nt = a.nt, np = a.np, n = a.n;
  // fail_flag[r * nt + s]: the factorisation of diagonal tile s failed in attempt r. One slot per
  // (attempt, tile) so a flag read after a barrier can only have been written before that barrier.
  unsigned* fail_flag = a.sync + 4;
  unsigned* ready = a.sync + 4 + a.attempts * nt;
  if (w == 0) {
    for (int k = threadIdx.x; k < (a.attempts + 1) * nt; k += kCholThreads) a.sync[4 + k] = 0u;
    if (threadIdx.x == 0) *a.status = -2;  // stays -2 only if the kernel leaves on a barrier timeout
  }
  int result = -1;
  double eps = a.eps0;
  for (int r = 0; r < a.attempts; ++r, eps *= a.mult) {
    // ---- copy + regularise the lower tiles; workgroup 0 factors tile (0, 0) on the way
    const int n_lower = nt * (nt + 1) / 2;
    for (int tt = w; tt < n_lower; tt += G) {
      int i = 0;
      while ((i + 1) * (i + 2) / 2 <= tt) ++i;
      const int j = tt - i * (i + 1) / 2;
      for (int e = threadIdx.x; e < NB * NB; e += kCholThreads) {
        const int rr = i * NB + e / NB, cc = j * NB + e % NB;
        double v;
        if (rr < n && cc < n) {
          v = a.H[int64_t(rr) * n + cc];
          if (rr == cc) v += a.lambda * v + eps;
        } else {
          v = (rr == cc) ? 1.0 : 0.0;
        }
        S1[(e / NB) * LDT + e % NB] = v;
      }
      if (j == 0 && threadIdx.x < NB) {
        const int rr = i * NB + threadIdx.x;
        a.b[rr] = (rr < n) ? -a.g[rr] : 0.0;
      }
      __syncthreads();
      if (i == 0) {  // tile (0, 0): factor now
        const bool ok = tile_potrf(S1);
        if (!ok) {
          if (threadIdx.x == 0) atomicOr(&fail_flag[r * nt], 1u);
        } else {
          tile_store(S1, a.L, np);
          tile_trinv(S1, S2);
          tile_store(S2, a.Inv, NB);
          __syncthreads();
          tile_gemv_store(S2, a.b, a.y);
        }
      } else {
        tile_store(S1, a.Wm + int64_t(i) * NB * np + j * NB, np);
      }
      __syncthreads();
    }
    if (!grid_barrier(a.sync, G)) return;
    bool failed = ld_acq(&fail_flag[r * nt]) != 0u;
    // ---- panel steps
    for (int k = 0; k + 1 < nt && !failed; ++k) {
      const int m = nt - k - 1;
      const int n_tiles = m * (m + 1) / 2;
      bool have_inv = false;
      for (int tt = w; tt < n_tiles; tt += G) {
        int ii = 0;
        while ((ii + 1) * (ii + 2) / 2 <= tt) ++ii;
        const int jj = tt - ii * (ii + 1) / 2;
        const int i = k + 1 + ii, j = k + 1 + jj;
        if (!have_inv) {
          tile_load(S0, a.Inv + int64_t(k) * NB * NB, NB);
          have_inv = true;
        }
        tile_load(S1, a.Wm + int64_t(i) * NB * np + k * NB, np);
        __syncthreads();
        tile_mul_invT(S1, S0);  // L_ik
        const double* Ljk = S1;
        if (j != i) {
          tile_load(S2, a.Wm + int64_t(j) * NB * np + k * NB, np);
          __syncthreads();
          tile_mul_invT(S2, S0);  // L_jk
          Ljk = S2;
        }
        // C = A_ij - L_ik L_jk^T
        double acc[NB * NB / kCholThreads];
        int q = 0;
        double* Aij = a.Wm + int64_t(i) * NB * np + j * NB;
        for (int e = threadIdx.x; e < NB * NB; e += kCholThreads, ++q) {
          const int rr = e / NB, cc = e % NB;
          double s = Aij[int64_t(rr) * np + cc];
          for (int t = 0; t < NB; ++t) s -= S1[rr * LDT + t] * Ljk[cc * LDT + t];
          acc[q] = s;
        }
        if (j == k + 1) {
          // final L_ik, and forward elimination of block i: b_i -= L_ik y_k
          tile_store(S1, a.L + int64_t(i) * NB * np + k * NB, np);
          __syncthreads();
          if (threadIdx.x < NB) {
            const int rr = threadIdx.x;
            double s = 0.0;
            for (int t = 0; t < NB; ++t) s += S1[rr * LDT + t] * a.y[k * NB + t];
            a.b[i * NB + rr] -= s;
          }
        }
        __syncthreads();
        if (i == j && i == k + 1) {
          q = 0;
          for (int e = threadIdx.x; e < NB * NB; e += kCholThreads, ++q) S1[(e / NB) * LDT + e % NB] = acc[q];
          const bool ok = tile_potrf(S1);
          if (!ok) {
            if (threadIdx.x == 0) atomicOr(&fail_flag[r * nt + k + 1], 1u);
          } else {
            tile_store(S1, a.L + int64_t(i) * NB * np + i * NB, np);
            tile_trinv(S1, S2);
            tile_store(S2, a.Inv + int64_t(i) * NB * NB, NB);
            tile_gemv_store(S2, a.b + i * NB, a.y + i * NB);
          }
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
  // ---- back substitution L^T x = y, block k owned by workgroup k mod G, highest blocks first
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
  // barrier words start at zero (a fill kernel, not a memset, so the launch sequence can be captured)
  DS3_TRY(launch_fill_u32(a.sync, 4, 0u, s));
  int max_tiles = (a.nt - 1) * a.nt / 2;
  int G = max_tiles < 1 ? 1 : max_tiles;
  if (G > 128) G = 128;
  hipLaunchKernelGGL(k_chol_ladder, dim3(G), dim3(kCholThreads), 0, s, a);
  return check_hip(hipGetLastError(), "k_chol_ladder");
}

}  // namespace ds3
