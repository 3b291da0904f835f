// Float64 32x32 tile primitives shared by the dense and the tile-sparse ladder solvers of eq. (7): the
// accumulator layout of the float64 matrix-core instruction, tile products, and the factorisation of a
// symmetric positive definite tile into the inverse of its Cholesky factor (the solvers never store the
// factor of a diagonal tile, only its inverse).
#pragma once
#include "common.hpp"

namespace ds3 {

constexpr int NB = 32;
// LDS row stride of a tile: the 16 rows a wave reads down one column of a tile product land on distinct
// banks (with NB + 4, rows eight apart shared banks: 0.65 -> 0.49 us for a product), rows stay 16-byte
// aligned
constexpr int LDT = NB + 2;

// Pending marker of the solution values read by the back substitution (a signalling-NaN bit pattern:
// arithmetic only produces quiet NaNs).
constexpr unsigned long long kXPending = 0x7ff4dead00000000ull;

// Columns per barrier of the diagonal factorisation, and its LDS scratch: double-buffered groups of kFw
// published columns of T and kFw rows of X, then the block of b, then the NB pivots.
constexpr int kFw = 4;
constexpr int kFactorScratch = 4 * kFw * NB + 2 * NB;

// ---------------------------------------------------------------------------------------------------
// Fragment helpers. The 256 threads hold a 32x32 tile in the accumulator layout of the float64 MFMA
// (16x16x4): wave w owns quadrant (w/2, w%2); lane l holds column 16 (w%2) + l%16 of rows
// 16 (w/2) + l/16 + 4 v, v = 0..3 (accumulator register v of this instruction holds rows l/16 + 4 v).
// ---------------------------------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ inline int fcol() { return 16 * ((threadIdx.x >> 6) & 1) + (threadIdx.x & 15); }
__device__ inline int frow(int v) { return 16 * (threadIdx.x >> 7) + ((threadIdx.x >> 4) & 3) + 4 * v; }

__device__ inline void frag_load(f64x4& q, const double* src, int64_t ld) {
  const int c = fcol();
#pragma unroll
  for (int v = 0; v < 4; ++v) q[v] = src[int64_t(frow(v)) * ld + c];
}

__device__ inline void frag_store(const f64x4& q, double* dst, int64_t ld) {
  const int c = fcol();
#pragma unroll
  for (int v = 0; v < 4; ++v) dst[int64_t(frow(v)) * ld + c] = q[v];
}

__device__ inline void frag_to_lds(const f64x4& q, double* S) {
  const int c = fcol();
#pragma unroll
  for (int v = 0; v < 4; ++v) S[frow(v) * LDT + c] = q[v];
}

// acc (+/-)= (A B^T) restricted to this wave's quadrant, A and B LDS tiles: eight MFMA steps over t.
template <bool SUB>
__device__ inline void frag_gemm_abt(const double* A, const double* B, f64x4& acc) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const double* a = A + (16 * (w >> 1) + (l & 15)) * LDT + (l >> 4);
  const double* b = B + (16 * (w & 1) + (l & 15)) * LDT + (l >> 4);
#pragma unroll
  for (int t0 = 0; t0 < NB; t0 += 4) {
    const double x = SUB ? -a[t0] : a[t0];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, b[t0], acc, 0, 0, 0);
  }
}

// 1/d from the hardware estimate (relative error about 2^-24) refined by one Halley step,
// y (1 + e + e^2) with e = 1 - d y: cubic convergence reaches full precision in three dependent fmas
// where two Newton steps take four (the pivot chain of the factorisation runs through this).
__device__ inline double recip(double d) {
  const double y = __builtin_amdgcn_rcp(d);
  const double e = fma(-d, y, 1.0);
  return fma(y, fma(e, e, e), y);
}

// 1/sqrt(d) from the hardware estimate refined by two Newton steps.
__device__ inline double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

__device__ inline bool pivot_ok(double d) { return (d > 0.0) && isfinite(d); }

// Cholesky of the SPD tile held as a fragment, producing the inverse of its factor, kFw columns per
// barrier (right-looking LDL^T on the full symmetric tile). Before a step, columns c .. c+kFw-1 of T and
// rows c .. c+kFw-1 of the inverse accumulator X (identity at the start) are published in LDS. Every
// thread factors the kFw x kFw pivot block D (pivots d_q, multipliers g_pq = D'[p][q] / d_q: the one
// sequential chain of the step) and brings the published entries it needs up to date within the block,
//   a_q(r) = T[r][c+q] - sum_{p<q} a_p(r) g_qp,   x_q(j) = X[c+q][j] - sum_{p<q} g_qp x_p(j).
// The rank-kFw updates
//   T[r][s] -= sum_q (a_q(r) / d_q) a_q(s),   X[r][j] -= sum_q (a_q(r) / d_q) x_q(j)   (r >= c+kFw)
// are one float64 MFMA each per wave (K = kFw): lane l feeds the A operand of row 16 (w/2) + l%16 and
// pivot q = l/16 (zero for rows above the trailing block, which leaves them untouched) and the B operand
// of column fcol() and pivot q. Entries of T outside the trailing block pick up terms that are never
// read again. The block's own rows of X take their step values x_q. At the end
// L^-1[r][j] = X[r][j] / sqrt(d_r) (the factor itself is not needed).
// Returns false (uniformly) on a non-positive or non-finite pivot.
__device__ inline bool factor_frag(f64x4& Tf, double* fb, f64x4& Xq) {
  const int s = fcol();
  const int l = threadIdx.x & 63;
  const int rbase = 16 * (threadIdx.x >> 7);  // first row of this wave's quadrant
  const int ra = rbase + (l & 15);            // A-operand row of this lane
  const int qa = l >> 4;                      // pivot of both operands; also the lane's row in a group of 4
  f64x4 X;
#pragma unroll
  for (int v = 0; v < 4; ++v) X[v] = (frow(v) == s) ? 1.0 : 0.0;
  // buffer layout per parity: kFw columns of T, then kFw rows of X, NB doubles each
  constexpr int kBuf = 2 * kFw * NB;
  double* piv = fb + 4 * kFw * NB + NB;
  if (s < kFw)
#pragma unroll
    for (int v = 0; v < 4; ++v) fb[s * NB + frow(v)] = Tf[v];
  if (rbase == 0) fb[(kFw + qa) * NB + s] = X[0];  // rows 0..3: register 0 of the top quadrants
  __syncthreads();
  bool ok = true;
  for (int c = 0; c < NB; c += kFw) {
    const double* P = fb + ((c / kFw) & 1) * kBuf;
    // every LDS read of the step first
    double D[kFw][kFw], ar[kFw], as[kFw], xs[kFw];
#pragma unroll
    for (int p = 0; p < kFw; ++p)
#pragma unroll
      for (int q = 0; q <= p; ++q) D[p][q] = P[q * NB + c + p];
#pragma unroll
    for (int q = 0; q < kFw; ++q) {
      ar[q] = P[q * NB + ra];
      as[q] = P[q * NB + s];
      xs[q] = P[(kFw + q) * NB + s];
    }
    // keep every read above the pivot chain, so that their latency overlaps it (the scheduler would
    // otherwise sink them below the chain and add the LDS round trip to every step)
    __builtin_amdgcn_sched_barrier(0);
    // pivot block (identical in every thread, so the outcome is uniform)
    // D[p][r] -= D[p][q] D[r][q] / d_q: the products are formed while the reciprocal of the pivot is
    // in flight, so the chain from one pivot to the next is the reciprocal and one fma
    double dq[kFw], iq[kFw], g[kFw][kFw];
#pragma unroll
    for (int q = 0; q < kFw; ++q) {
      double pr[kFw][kFw];
#pragma unroll
      for (int p = q + 1; p < kFw; ++p)
#pragma unroll
        for (int r = q + 1; r <= p; ++r) pr[p][r] = D[p][q] * D[r][q];
      dq[q] = D[q][q];
      ok = ok && pivot_ok(dq[q]);
      iq[q] = recip(dq[q]);
#pragma unroll
      for (int p = q + 1; p < kFw; ++p) g[p][q] = D[p][q] * iq[q];
#pragma unroll
      for (int p = q + 1; p < kFw; ++p)
#pragma unroll
        for (int r = q + 1; r <= p; ++r) D[p][r] = fma(-pr[p][r], iq[q], D[p][r]);
    }
#pragma unroll
    for (int q = 1; q < kFw; ++q)
#pragma unroll
      for (int p = 0; p < q; ++p) {
        ar[q] = fma(-ar[p], g[q][p], ar[q]);
        as[q] = fma(-as[p], g[q][p], as[q]);
        xs[q] = fma(-g[q][p], xs[p], xs[q]);
      }
    double aop = -ar[0] * iq[0], bop = as[0], xop = xs[0], dsel = dq[0];
#pragma unroll
    for (int q = 1; q < kFw; ++q) {
      aop = (qa == q) ? -ar[q] * iq[q] : aop;
      bop = (qa == q) ? as[q] : bop;
      xop = (qa == q) ? xs[q] : xop;
      dsel = (qa == q) ? dq[q] : dsel;
    }
    aop = (ra >= c + kFw) ? aop : 0.0;
    Tf = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop, Tf, 0, 0, 0);
    X = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, xop, X, 0, 0, 0);
    // rows c .. c+kFw-1 sit in register (c - rbase) / 4 of this quadrant, one per lane row qa: they take
    // x_qa at this lane's column; the pivots go to LDS (lanes 0, 16, 32, 48 of wave 0 hold q = 0..3)
    const int vin = (c - rbase) >> 2;  // wave-uniform; outside 0..3 when the rows are in the other quadrant
    if (vin == 0) X[0] = xop;
    else if (vin == 1) X[1] = xop;
    else if (vin == 2) X[2] = xop;
    else if (vin == 3) X[3] = xop;
    if (threadIdx.x < 64 && (threadIdx.x & 15) == 0) piv[c + qa] = dsel;
    if (c + kFw < NB) {
      double* Q = fb + ((c / kFw + 1) & 1) * kBuf;
      const int qs = s - c - kFw;
      if (qs >= 0 && qs < kFw)
#pragma unroll
        for (int v = 0; v < 4; ++v) Q[qs * NB + frow(v)] = Tf[v];
      const int vn = (c + kFw - rbase) >> 2;  // register of rows c+kFw .. c+2kFw-1, if in this quadrant
      if (vn == 0) Q[(kFw + qa) * NB + s] = X[0];
      else if (vn == 1) Q[(kFw + qa) * NB + s] = X[1];
      else if (vn == 2) Q[(kFw + qa) * NB + s] = X[2];
      else if (vn == 3) Q[(kFw + qa) * NB + s] = X[3];
    }
    __syncthreads();
  }
  if (!ok) return false;
#pragma unroll
  for (int v = 0; v < 4; ++v) Xq[v] = (s <= frow(v)) ? X[v] * rsqrt_nr(piv[frow(v)]) : 0.0;
  return true;
}


// Stores the inverse of a diagonal factor (Xq, as returned by factor_frag) at inv_dst (row-major 32x32)
// and y = Inv b at y_dst, b in LDS sb. S: a free LDS tile. The product runs on 8 threads per row, reduced
// with lane shuffles.
__device__ inline void diag_out(double* inv_dst, double* y_dst, const f64x4& Xq, double* S, const double* sb) {
  frag_store(Xq, inv_dst, NB);
  frag_to_lds(Xq, S);
  __syncthreads();
  const int r = threadIdx.x >> 3, p = threadIdx.x & 7;
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < NB / 8; ++q) acc = fma(S[r * LDT + p + 8 * q], sb[p + 8 * q], acc);
  acc += __shfl_xor(acc, 1, 8);
  acc += __shfl_xor(acc, 2, 8);
  acc += __shfl_xor(acc, 4, 8);
  if (p == 0) y_dst[r] = acc;
}

}  // namespace ds3
