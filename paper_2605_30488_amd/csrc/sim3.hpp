// Float64 Sim(3) on the device (Sec. III-A pose model, Sec. III-D left perturbation T <- Exp(tau) T).
//
// Pose storage: [t(3), q(4) = (x, y, z, w), s], T_WC = [[sR(q), t], [0, 1]]. Tangent tau = (v, omega,
// zeta). Exp(tau) = [[e^zeta R(omega), V v], [0, 1]] with V = A I + B W + C W^2, W = [omega]x and
//   A = int_0^1 e^{s zeta} ds, B = int_0^1 e^{s zeta} sin(s theta)/theta ds,
//   C = int_0^1 e^{s zeta} (1 - cos(s theta))/theta^2 ds,  theta = |omega|.
// The closed forms of B and C cancel catastrophically near zeta = theta = 0 (and C near theta = 0), so
// three regimes are used: a double power series in (zeta, theta) for rho = |(zeta, theta)| < 0.05, a
// series in theta with exact moments int_0^1 s^k e^{s zeta} ds for theta < 0.05 <= rho, and the
// closed forms for theta >= 0.05 where their relative cancellation error stays below ~1e-13.
#pragma once

#include <hip/hip_runtime.h>

namespace ds3 {

struct Sim3 {
  double t[3];
  double q[4];
  double s;
};

__device__ __host__ inline Sim3 sim3_load(const double* p) {
  Sim3 T;
  for (int k = 0; k < 3; ++k) T.t[k] = p[k];
  for (int k = 0; k < 4; ++k) T.q[k] = p[3 + k];
  T.s = p[7];
  return T;
}

__device__ __host__ inline void sim3_store(const Sim3& T, double* p) {
  for (int k = 0; k < 3; ++k) p[k] = T.t[k];
  for (int k = 0; k < 4; ++k) p[3 + k] = T.q[k];
  p[7] = T.s;
}

__device__ __host__ inline void quat_normalize(double* q) {
  double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) q[k] /= n;
}

// Hamilton product a (x) b.
__device__ __host__ inline void quat_mul(const double* a, const double* b, double* o) {
  o[0] = a[3] * b[0] + b[3] * a[0] + (a[1] * b[2] - a[2] * b[1]);
  o[1] = a[3] * b[1] + b[3] * a[1] + (a[2] * b[0] - a[0] * b[2]);
  o[2] = a[3] * b[2] + b[3] * a[2] + (a[0] * b[1] - a[1] * b[0]);
  o[3] = a[3] * b[3] - (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
}

// Rotation matrix (row-major) of a quaternion, normalised on the fly.
__device__ __host__ inline void quat_to_mat(const double* qin, double* R) {
  double q[4] = {qin[0], qin[1], qin[2], qin[3]};
  quat_normalize(q);
  double x = q[0], y = q[1], z = q[2], w = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

__device__ __host__ inline void mat3_vec(const double* R, const double* v, double* o) {
  for (int r = 0; r < 3; ++r) o[r] = R[3 * r] * v[0] + R[3 * r + 1] * v[1] + R[3 * r + 2] * v[2];
}

__device__ __host__ inline void mat3T_vec(const double* R, const double* v, double* o) {
  for (int r = 0; r < 3; ++r) o[r] = R[r] * v[0] + R[3 + r] * v[1] + R[6 + r] * v[2];
}

// A * B
__device__ __host__ inline Sim3 sim3_mul(const Sim3& A, const Sim3& B) {
  Sim3 C;
  double R[9], Rt[3];
  quat_to_mat(A.q, R);
  mat3_vec(R, B.t, Rt);
  for (int k = 0; k < 3; ++k) C.t[k] = A.s * Rt[k] + A.t[k];
  quat_mul(A.q, B.q, C.q);
  quat_normalize(C.q);
  C.s = A.s * B.s;
  return C;
}

// A^-1 = [[R^T / s, -R^T t / s], [0, 1]]
__device__ __host__ inline Sim3 sim3_inv(const Sim3& A) {
  Sim3 I;
  double R[9], v[3];
  quat_to_mat(A.q, R);
  mat3T_vec(R, A.t, v);
  for (int k = 0; k < 3; ++k) I.t[k] = -v[k] / A.s;
  double n = sqrt(A.q[0] * A.q[0] + A.q[1] * A.q[1] + A.q[2] * A.q[2] + A.q[3] * A.q[3]);
  I.q[0] = -A.q[0] / n; I.q[1] = -A.q[1] / n; I.q[2] = -A.q[2] / n; I.q[3] = A.q[3] / n;
  I.s = 1.0 / A.s;
  return I;
}

// int_0^1 s^k e^{s z} ds for k = 0..10 into I[0..10].
__device__ __host__ inline void exp_moments(double z, double* I) {
  if (fabs(z) <= 2.0) {
    // sum_n z^n / (n! (n + k + 1)); 40 terms reach double precision for |z| <= 2
    // (fully unrolled so that every reciprocal below is a compile-time constant)
#pragma unroll
    for (int k = 0; k <= 10; ++k) I[k] = 0.0;
    double term = 1.0;  // z^n / n!
#pragma unroll
    for (int n = 0; n < 40; ++n) {
#pragma unroll
      for (int k = 0; k <= 10; ++k) I[k] = fma(term, 1.0 / double(n + k + 1), I[k]);
      term *= z * (1.0 / double(n + 1));
    }
  } else {
    double ez = exp(z);
    I[0] = expm1(z) / z;
    for (int k = 1; k <= 10; ++k) I[k] = (ez - k * I[k - 1]) / z;
  }
}

// Coefficients of V = A I + B W + C W^2 for (zeta, theta).
__device__ __host__ inline void sim3_V_coeffs(double zeta, double theta, double& A, double& B,
                                              double& C) {
  const double th2 = theta * theta;
  const double rho2 = zeta * zeta + th2;
  if (rho2 < 0.05 * 0.05) {
    // double series, total degree n + 2m <= 12
    // (fully unrolled: the factorial denominators fold into constant reciprocals)
    A = 0.0; B = 0.0; C = 0.0;
    double zn = 1.0, nfact = 1.0;
#pragma unroll
    for (int n = 0; n <= 12; ++n) {
      A += zn * (1.0 / (nfact * (n + 1)));
      double tm = 1.0, f1 = 1.0, f2 = 2.0;  // theta^{2m}, (2m+1)!, (2m+2)!
      double sgn = 1.0;
#pragma unroll
      for (int m = 0; n + 2 * m <= 12; ++m) {
        B += zn * tm * (sgn / (nfact * f1 * (n + 2 * m + 2)));
        C += zn * tm * (sgn / (nfact * f2 * (n + 2 * m + 3)));
        tm *= th2;
        f1 *= double(2 * m + 2) * double(2 * m + 3);
        f2 *= double(2 * m + 3) * double(2 * m + 4);
        sgn = -sgn;
      }
      zn *= zeta;
      nfact *= double(n + 1);
    }
    return;
  }
  A = (fabs(zeta) < 1e-6) ? 1.0 + zeta * (0.5 + zeta * (1.0 / 6.0 + zeta / 24.0)) : expm1(zeta) / zeta;
  if (theta < 0.05) {
    double I[11];
    exp_moments(zeta, I);
    B = 0.0; C = 0.0;
    double tm = 1.0, f1 = 1.0, f2 = 2.0, sgn = 1.0;
#pragma unroll
    for (int m = 0; m <= 4; ++m) {
      B += tm * (sgn / f1) * I[2 * m + 1];
      C += tm * (sgn / f2) * I[2 * m + 2];
      tm *= th2;
      f1 *= double(2 * m + 2) * double(2 * m + 3);
      f2 *= double(2 * m + 3) * double(2 * m + 4);
      sgn = -sgn;
    }
    return;
  }
  const double ez = exp(zeta), st = sin(theta), ct = cos(theta);
  B = (ez * (zeta * st - theta * ct) + theta) / (theta * rho2);
  C = (A - (ez * (zeta * ct + theta * st) - zeta) / rho2) / th2;
}

// V x for V = A I + B [w]x + C [w]x^2.
__device__ __host__ inline void sim3_V_apply(double A, double B, double C, const double* w,
                                             const double* x, double* o) {
  double wx[3] = {w[1] * x[2] - w[2] * x[1], w[2] * x[0] - w[0] * x[2], w[0] * x[1] - w[1] * x[0]};
  double wwx[3] = {w[1] * wx[2] - w[2] * wx[1], w[2] * wx[0] - w[0] * wx[2], w[0] * wx[1] - w[1] * wx[0]};
  for (int k = 0; k < 3; ++k) o[k] = A * x[k] + B * wx[k] + C * wwx[k];
}

__device__ __host__ inline Sim3 sim3_exp(const double* tau) {
  const double* v = tau;
  const double* w = tau + 3;
  const double zeta = tau[6];
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double theta = sqrt(th2);
  Sim3 T;
  // quaternion of the rotation: (sin(theta/2)/theta * w, cos(theta/2))
  double h = (theta < 1e-4) ? 0.5 - th2 / 48.0 : sin(0.5 * theta) / theta;
  T.q[0] = h * w[0]; T.q[1] = h * w[1]; T.q[2] = h * w[2]; T.q[3] = cos(0.5 * theta);
  T.s = exp(zeta);
  double A, B, C;
  sim3_V_coeffs(zeta, theta, A, B, C);
  sim3_V_apply(A, B, C, w, v, T.t);
  return T;
}

__device__ __host__ inline void sim3_log(const Sim3& T, double* tau) {
  const double zeta = log(T.s);
  double q[4] = {T.q[0], T.q[1], T.q[2], T.q[3]};
  quat_normalize(q);
  if (q[3] < 0) for (int k = 0; k < 4; ++k) q[k] = -q[k];
  const double nv = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
  double w[3] = {0.0, 0.0, 0.0};
  double theta = 0.0;
  if (nv > 0.0) {
    theta = 2.0 * atan2(nv, q[3]);
    const double f = theta / nv;
    for (int k = 0; k < 3; ++k) w[k] = f * q[k];
  }
  double A, B, C;
  sim3_V_coeffs(zeta, theta, A, B, C);
  // V as a matrix, then Cramer's rule for V v = t
  double M[9];
  const double W[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
  double W2[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      W2[3 * r + c] = W[3 * r] * W[c] + W[3 * r + 1] * W[3 + c] + W[3 * r + 2] * W[6 + c];
  for (int e = 0; e < 9; ++e) M[e] = B * W[e] + C * W2[e];
  M[0] += A; M[4] += A; M[8] += A;
  const double det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                     M[2] * (M[3] * M[7] - M[4] * M[6]);
  const double* t = T.t;
  double v[3];
  v[0] = (t[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (t[1] * M[8] - M[5] * t[2]) +
          M[2] * (t[1] * M[7] - M[4] * t[2])) / det;
  v[1] = (M[0] * (t[1] * M[8] - M[5] * t[2]) - t[0] * (M[3] * M[8] - M[5] * M[6]) +
          M[2] * (M[3] * t[2] - t[1] * M[6])) / det;
  v[2] = (M[0] * (M[4] * t[2] - t[1] * M[7]) - M[1] * (M[3] * t[2] - t[1] * M[6]) +
          t[0] * (M[3] * M[7] - M[4] * M[6])) / det;
  for (int k = 0; k < 3; ++k) { tau[k] = v[k]; tau[3 + k] = w[k]; }
  tau[6] = zeta;
}

// Adjoint of T on tau = (v, omega, zeta): v' = sR v + [t]x R omega - zeta t, omega' = R omega,
// zeta' = zeta (T Exp(tau) T^-1 = Exp(Ad_T tau)). Row-major 7x7.
__device__ __host__ inline void sim3_adjoint(const Sim3& T, double* Ad) {
  double R[9];
  quat_to_mat(T.q, R);
  for (int e = 0; e < 49; ++e) Ad[e] = 0.0;
  const double* t = T.t;
  const double tx[9] = {0, -t[2], t[1], t[2], 0, -t[0], -t[1], t[0], 0};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      Ad[7 * r + c] = T.s * R[3 * r + c];
      Ad[7 * r + 3 + c] = tx[3 * r] * R[c] + tx[3 * r + 1] * R[3 + c] + tx[3 * r + 2] * R[6 + c];
      Ad[7 * (3 + r) + 3 + c] = R[3 * r + c];
    }
  for (int r = 0; r < 3; ++r) Ad[7 * r + 6] = -t[r];
  Ad[48] = 1.0;
}

}  // namespace ds3
