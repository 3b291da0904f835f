// The closed-form similarity of eq. (4) (Sec. III-C) from the moments of the correspondences, shared by
// the device solve of the gauge synchronisation and the host entry point ds3_umeyama (float64):
// A = (1/N) sum (x - xb)(y - yb)^T = U Lambda V^T, S = diag(1, 1, det(U V^T)), R = U S V^T,
// s = tr(S Lambda) / ((1/N) sum |y - yb|^2), t = xb - s R yb.
#pragma once

#include <hip/hip_runtime.h>

#include "sim3.hpp"

namespace ds3 {

// One-sided Jacobi SVD of the 3x3 A (row-major): A = U diag(sig) V^T, sig descending.
__host__ __device__ inline void svd3(const double* A, double* U, double* sig, double* V) {
  double W[9];
  for (int e = 0; e < 9; ++e) W[e] = A[e];
  for (int e = 0; e < 9; ++e) V[e] = (e % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        double al = 0, be = 0, ga = 0;
        for (int r = 0; r < 3; ++r) {
          al += W[3 * r + p] * W[3 * r + p];
          be += W[3 * r + q] * W[3 * r + q];
          ga += W[3 * r + p] * W[3 * r + q];
        }
        if (fabs(ga) <= 1e-300 || fabs(ga) <= 1e-17 * sqrt(al * be)) continue;
        off = fmax(off, fabs(ga) / sqrt(al * be));
        const double zeta = (be - al) / (2.0 * ga);
        const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int r = 0; r < 3; ++r) {
          const double wp = W[3 * r + p], wq = W[3 * r + q];
          W[3 * r + p] = c * wp - s * wq;
          W[3 * r + q] = s * wp + c * wq;
          const double vp = V[3 * r + p], vq = V[3 * r + q];
          V[3 * r + p] = c * vp - s * vq;
          V[3 * r + q] = s * vp + c * vq;
        }
      }
    if (off < 1e-16) break;
  }
  double sv[3];
  for (int k = 0; k < 3; ++k) sv[k] = sqrt(W[k] * W[k] + W[3 + k] * W[3 + k] + W[6 + k] * W[6 + k]);
  int ord[3] = {0, 1, 2};
  for (int a = 0; a < 3; ++a)
    for (int b = a + 1; b < 3; ++b)
      if (sv[ord[b]] > sv[ord[a]]) { int t = ord[a]; ord[a] = ord[b]; ord[b] = t; }
  double Vs[9], Us[9];
  for (int k = 0; k < 3; ++k) {
    sig[k] = sv[ord[k]];
    for (int r = 0; r < 3; ++r) {
      Vs[3 * r + k] = V[3 * r + ord[k]];
      Us[3 * r + k] = (sig[k] > 0.0) ? W[3 * r + ord[k]] / sig[k] : 0.0;
    }
  }
  if (!(sig[2] > 1e-14 * sig[0])) {  // complete U with the cross product of its first two columns
    Us[2] = Us[3] * Us[7] - Us[6] * Us[4];
    Us[5] = Us[6] * Us[1] - Us[0] * Us[7];
    Us[8] = Us[0] * Us[4] - Us[3] * Us[1];
  }
  for (int e = 0; e < 9; ++e) { U[e] = Us[e]; V[e] = Vs[e]; }
}

__host__ __device__ inline double det3(const double* M) {
  return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
         M[2] * (M[3] * M[7] - M[4] * M[6]);
}

// Unit quaternion (x, y, z, w), w >= 0, of a rotation matrix (row-major), from its largest pivot.
__host__ __device__ inline void mat_to_quat(const double* R, double* q) {
  const double tr = R[0] + R[4] + R[8];
  if (tr > R[0] && tr > R[4] && tr > R[8]) {
    const double S = sqrt(1.0 + tr) * 2.0;
    q[3] = 0.25 * S; q[0] = (R[7] - R[5]) / S; q[1] = (R[2] - R[6]) / S; q[2] = (R[3] - R[1]) / S;
  } else if (R[0] > R[4] && R[0] > R[8]) {
    const double S = sqrt(1.0 + R[0] - R[4] - R[8]) * 2.0;
    q[3] = (R[7] - R[5]) / S; q[0] = 0.25 * S; q[1] = (R[1] + R[3]) / S; q[2] = (R[2] + R[6]) / S;
  } else if (R[4] > R[8]) {
    const double S = sqrt(1.0 + R[4] - R[0] - R[8]) * 2.0;
    q[3] = (R[2] - R[6]) / S; q[0] = (R[1] + R[3]) / S; q[1] = 0.25 * S; q[2] = (R[5] + R[7]) / S;
  } else {
    const double S = sqrt(1.0 + R[8] - R[0] - R[4]) * 2.0;
    q[3] = (R[3] - R[1]) / S; q[0] = (R[2] + R[6]) / S; q[1] = (R[5] + R[7]) / S; q[2] = 0.25 * S;
  }
  if (q[3] < 0)
    for (int k = 0; k < 4; ++k) q[k] = -q[k];
  quat_normalize(q);
}

// T* of eq. (4) from the centroids xb, yb, the cross-covariance A (row-major) and the spread sy2 of y.
// Returns false (T untouched) when the correspondences are degenerate: rank(A) < 2 (second singular
// value <= 1e-12 of the first: collinear points, whose rotation is not determined) or no spread of y.
__host__ __device__ inline bool umeyama_solve(const double* xb, const double* yb, const double* A, double sy2,
                                              Sim3& T) {
  double U[9], sig[3], V[9];
  svd3(A, U, sig, V);
  if (!(sig[1] > 1e-12 * sig[0]) || !(sy2 > 0.0)) return false;
  double UVt[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      UVt[3 * r + c] = U[3 * r] * V[3 * c] + U[3 * r + 1] * V[3 * c + 1] + U[3 * r + 2] * V[3 * c + 2];
  const double d = det3(UVt) < 0.0 ? -1.0 : 1.0;
  double R[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      R[3 * r + c] = U[3 * r] * V[3 * c] + U[3 * r + 1] * V[3 * c + 1] + d * U[3 * r + 2] * V[3 * c + 2];
  const double s = (sig[0] + sig[1] + d * sig[2]) / sy2;
  double Ry[3];
  mat3_vec(R, yb, Ry);
  for (int k = 0; k < 3; ++k) T.t[k] = xb[k] - s * Ry[k];
  T.s = s;
  mat_to_quat(R, T.q);
  return true;
}

}  // namespace ds3
