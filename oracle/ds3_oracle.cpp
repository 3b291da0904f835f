// FP64 CPU oracle for the dense Sim(3) back-end of CoMo3R-SLAM (collaborative monocular dense SLAM).
//
// TEST INFRASTRUCTURE ONLY. Nothing on the product path may load this library: only the tests, the
// smoke entry and the CPU-baseline leg of the benchmark do. It shares no code, header or table with the
// HIP library; the two meet only on the seeded synthetic inputs.
//
// Everything here is plain and slow on purpose: FP64 throughout, every sum in index order, no blocking,
// no fusion. Parallel loops (OpenMP) only split independent work (pixels of one direction, edges) and
// write disjoint outputs, so results do not depend on the thread count.
//
// Paper map (CoMo3R-SLAM, Sec. III):
//   ray operator psi(X) = X/|X|, pi(X) = (psi, |X|)                   Sec. III-A, "Learned geometry"
//   projective matching p* = argmin_p |psi([X^f_f]_p) - psi(x)|^2     Sec. III-A, "Learned geometry"
//   match confidence q = sqrt(Q_m Q_n)                                 Sec. III-A / III-B
//   bidirectional gate min(nu_i, nu_j) >= nu_min                       Sec. III-B
//   Sim(3) pose, T_ij = T_i^-1 T_j                                     Sec. III-A, "Ray-range tracking"
//   residual e_mn                                                      eq. (1)
//   whitening Sigma_mn = Sigma/q, Huber kappa, IRLS w = min(1,k/|r|)   Sec. III-A, "Ray-range tracking"
//   E_global                                                           eq. (5)
//   left perturbation T <- Exp(tau) T, tau = (v, omega, zeta)         Sec. III-D
//   Jacobian blocks and the -/+ Ad_{T_i^-1} endpoint maps              eq. (6) and the text after it
//   regularised normal equations and the epsilon ladder                eq. (7) and the text after it
//   calibrated mode: pixel reprojection and log-depth residuals on      Sec. IV-C, "Calibration"
//   pointmaps constrained to the calibrated rays
//
// Readings where the paper is silent (stated in the design notes of the repository):
//   matching = Levenberg-Marquardt on the bilinear interpolant of the reference ray image, started at
//   the query's own pixel; validity = no hole, angular residual within half a pixel, range agreement;
//   mutual consistency within a Chebyshev radius; Huber rho(r) = r^2/2 inside kappa,
//   kappa|r| - kappa^2/2 outside; anchor rows and columns replaced by identity.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

typedef struct {
  int32_t max_iters;        // LM trial steps per query
  double lambda0;           // initial LM damping
  double lambda_min;        // floor of the damping after an accepted step
  double step_tol_px;       // stop after a trial step (accepted or not) with max(|du|,|dv|) below this
  double ang_tol_px;        // validity: |r| <= ang_tol_px * min(|ds/du|, |ds/dv|)
  double range_rel_tol;     // validity: ||x| - |X_ref[idx]|| <= range_rel_tol * |X_ref[idx]|
  int32_t mutual_radius_px; // mutual check: Chebyshev distance of the round trip
  double q_min;             // confidence needed to count towards nu
  double nu_min;            // admission gate on min(nu_i, nu_j)
} orc_match_params;

typedef struct {
  double sigma_ray;     // sigma_r
  double sigma_dist;    // sigma_d
  double huber_k;       // kappa
  double lambda;        // diag(H) damping of eq. (7)
  double eps0;          // first epsilon of the ladder
  double eps_mult;      // growth of epsilon per failed attempt
  int32_t max_attempts; // attempts of the ladder
} orc_gn_params;

}  // extern "C"

namespace {

// ------------------------------------------------------------------------------------------------
// Small dense helpers (row-major)
// ------------------------------------------------------------------------------------------------
using M4 = std::array<double, 16>;
using M3 = std::array<double, 9>;

M4 m4_identity() {
  M4 I{};
  I[0] = I[5] = I[10] = I[15] = 1.0;
  return I;
}

M4 m4_mul(const M4& A, const M4& B) {
  M4 C{};
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 4; ++k) acc += A[r * 4 + k] * B[k * 4 + c];
      C[r * 4 + c] = acc;
    }
  return C;
}

M3 m3_mul(const M3& A, const M3& B) {
  M3 C{};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += A[r * 3 + k] * B[k * 3 + c];
      C[r * 3 + c] = acc;
    }
  return C;
}

double m3_det(const M3& A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// Solve the 3x3 system A x = b by Gaussian elimination with partial pivoting.
bool m3_solve(M3 A, std::array<double, 3> b, std::array<double, 3>& x) {
  int piv[3] = {0, 1, 2};
  for (int col = 0; col < 3; ++col) {
    int best = col;
    for (int r = col + 1; r < 3; ++r)
      if (std::fabs(A[piv[r] * 3 + col]) > std::fabs(A[piv[best] * 3 + col])) best = r;
    std::swap(piv[col], piv[best]);
    double p = A[piv[col] * 3 + col];
    if (p == 0.0) return false;
    for (int r = col + 1; r < 3; ++r) {
      double f = A[piv[r] * 3 + col] / p;
      for (int c = col; c < 3; ++c) A[piv[r] * 3 + c] -= f * A[piv[col] * 3 + c];
      b[piv[r]] -= f * b[piv[col]];
    }
  }
  for (int col = 2; col >= 0; --col) {
    double acc = b[piv[col]];
    for (int c = col + 1; c < 3; ++c) acc -= A[piv[col] * 3 + c] * x[c];
    x[col] = acc / A[piv[col] * 3 + col];
  }
  return true;
}

// ------------------------------------------------------------------------------------------------
// Sim(3) as 4x4 matrices [[sR, t], [0, 1]] (Sec. III-A, "Ray-range tracking").
// Pose storage: [tx, ty, tz, qx, qy, qz, qw, s], unit quaternion (x, y, z, w), s > 0.
// ------------------------------------------------------------------------------------------------
M3 quat_to_rot(const double* q_in) {
  double x = q_in[0], y = q_in[1], z = q_in[2], w = q_in[3];
  double n = std::sqrt(x * x + y * y + z * z + w * w);
  x /= n; y /= n; z /= n; w /= n;
  return M3{1 - 2 * (y * y + z * z), 2 * (x * y - w * z),     2 * (x * z + w * y),
            2 * (x * y + w * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
            2 * (x * z - w * y),     2 * (y * z + w * x),     1 - 2 * (x * x + y * y)};
}

// Rotation matrix to unit quaternion (largest-pivot method), sign fixed to w >= 0.
void rot_to_quat(const M3& R, double* q) {
  double tr = R[0] + R[4] + R[8];
  double x, y, z, w;
  if (tr > R[0] && tr > R[4] && tr > R[8]) {
    double S = std::sqrt(1.0 + tr) * 2.0;
    w = 0.25 * S; x = (R[7] - R[5]) / S; y = (R[2] - R[6]) / S; z = (R[3] - R[1]) / S;
  } else if (R[0] > R[4] && R[0] > R[8]) {
    double S = std::sqrt(1.0 + R[0] - R[4] - R[8]) * 2.0;
    w = (R[7] - R[5]) / S; x = 0.25 * S; y = (R[1] + R[3]) / S; z = (R[2] + R[6]) / S;
  } else if (R[4] > R[8]) {
    double S = std::sqrt(1.0 + R[4] - R[0] - R[8]) * 2.0;
    w = (R[2] - R[6]) / S; x = (R[1] + R[3]) / S; y = 0.25 * S; z = (R[5] + R[7]) / S;
  } else {
    double S = std::sqrt(1.0 + R[8] - R[0] - R[4]) * 2.0;
    w = (R[3] - R[1]) / S; x = (R[2] + R[6]) / S; y = (R[5] + R[7]) / S; z = 0.25 * S;
  }
  if (w < 0) { x = -x; y = -y; z = -z; w = -w; }
  double n = std::sqrt(x * x + y * y + z * z + w * w);
  q[0] = x / n; q[1] = y / n; q[2] = z / n; q[3] = w / n;
}

M4 pose_to_mat(const double* p) {
  M3 R = quat_to_rot(p + 3);
  double s = p[7];
  M4 T = m4_identity();
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) T[r * 4 + c] = s * R[r * 3 + c];
    T[r * 4 + 3] = p[r];
  }
  return T;
}

void mat_to_pose(const M4& T, double* p) {
  M3 sR{T[0], T[1], T[2], T[4], T[5], T[6], T[8], T[9], T[10]};
  double s = std::cbrt(m3_det(sR));
  M3 R;
  for (int k = 0; k < 9; ++k) R[k] = sR[k] / s;
  p[0] = T[3]; p[1] = T[7]; p[2] = T[11];
  rot_to_quat(R, p + 3);
  p[7] = s;
}

// Inverse of [[sR, t], [0, 1]] is [[R^T/s, -R^T t/s], [0, 1]].
M4 sim3_inverse_mat(const M4& T) {
  M3 sR{T[0], T[1], T[2], T[4], T[5], T[6], T[8], T[9], T[10]};
  double s = std::cbrt(m3_det(sR));
  M4 I = m4_identity();
  for (int r = 0; r < 3; ++r) {
    double acc = 0.0;
    for (int c = 0; c < 3; ++c) {
      I[r * 4 + c] = sR[c * 3 + r] / (s * s);  // (sR)^T / s^2 = R^T / s
      acc += sR[c * 3 + r] * T[c * 4 + 3];
    }
    I[r * 4 + 3] = -acc / (s * s);
  }
  return I;
}

// Generator of sim(3) for tau = (v, omega, zeta): [[zeta I + [omega]x, v], [0, 0]].
M4 sim3_hat(const double* tau) {
  const double* v = tau;
  const double* w = tau + 3;
  double z = tau[6];
  return M4{z,     -w[2], w[1],  v[0],
            w[2],  z,     -w[0], v[1],
            -w[1], w[0],  z,     v[2],
            0,     0,     0,     0};
}

// Exp(tau): the matrix exponential of the generator, evaluated plainly by its power series after
// scaling the argument below 1/2 in the infinity norm, then squaring back.
M4 sim3_exp_mat(const double* tau) {
  M4 G = sim3_hat(tau);
  double nrm = 0.0;
  for (int r = 0; r < 4; ++r) {
    double row = 0.0;
    for (int c = 0; c < 4; ++c) row += std::fabs(G[r * 4 + c]);
    nrm = std::max(nrm, row);
  }
  int squarings = 0;
  while (nrm > 0.5) { nrm *= 0.5; ++squarings; }
  double scale = std::ldexp(1.0, -squarings);
  for (double& g : G) g *= scale;
  M4 E = m4_identity();
  M4 term = m4_identity();
  for (int k = 1; k <= 40; ++k) {
    term = m4_mul(term, G);
    double mx = 0.0;
    for (double& t : term) { t /= k; mx = std::max(mx, std::fabs(t)); }
    for (int e = 0; e < 16; ++e) E[e] += term[e];
    if (mx < 1e-20) break;
  }
  for (int k = 0; k < squarings; ++k) E = m4_mul(E, E);
  return E;
}

// Log(T): zeta = ln s; omega from the unit quaternion (angle 2 atan2(|q_v|, q_w)); v solves V v = t with
// V = sum_k A^k/(k+1)!, A = zeta I + [omega]x, the translation block of exp of the generator.
void sim3_log_pose(const double* p, double* tau) {
  double zeta = std::log(p[7]);
  double q[4] = {p[3], p[4], p[5], p[6]};
  double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (double& c : q) c /= qn;
  if (q[3] < 0) for (double& c : q) c = -c;
  double nv = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
  double w[3] = {0, 0, 0};
  if (nv > 0.0) {
    double theta = 2.0 * std::atan2(nv, q[3]);
    for (int k = 0; k < 3; ++k) w[k] = theta * q[k] / nv;
  }
  M3 A{zeta, -w[2], w[1], w[2], zeta, -w[0], -w[1], w[0], zeta};
  M3 V{1, 0, 0, 0, 1, 0, 0, 0, 1};
  M3 term{1, 0, 0, 0, 1, 0, 0, 0, 1};
  for (int k = 1; k <= 80; ++k) {
    term = m3_mul(term, A);
    double mx = 0.0;
    for (double& t : term) { t /= (k + 1); mx = std::max(mx, std::fabs(t)); }
    for (int e = 0; e < 9; ++e) V[e] += term[e];
    if (mx < 1e-20) break;
  }
  std::array<double, 3> t{p[0], p[1], p[2]}, v{};
  m3_solve(V, t, v);
  tau[0] = v[0]; tau[1] = v[1]; tau[2] = v[2];
  tau[3] = w[0]; tau[4] = w[1]; tau[5] = w[2];
  tau[6] = zeta;
}

// Adjoint of T = [[sR, t], [0, 1]] on tau = (v, omega, zeta), defined by T Exp(tau) T^-1 = Exp(Ad_T tau):
//   v' = sR v + [t]x R omega - zeta t,  omega' = R omega,  zeta' = zeta.
void sim3_adjoint(const M4& T, double* Ad /* 7x7 row-major */) {
  M3 sR{T[0], T[1], T[2], T[4], T[5], T[6], T[8], T[9], T[10]};
  double s = std::cbrt(m3_det(sR));
  M3 R;
  for (int k = 0; k < 9; ++k) R[k] = sR[k] / s;
  double t[3] = {T[3], T[7], T[11]};
  M3 tx{0, -t[2], t[1], t[2], 0, -t[0], -t[1], t[0], 0};
  M3 txR = m3_mul(tx, R);
  std::fill(Ad, Ad + 49, 0.0);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      Ad[r * 7 + c] = sR[r * 3 + c];
      Ad[r * 7 + 3 + c] = txR[r * 3 + c];
      Ad[(3 + r) * 7 + 3 + c] = R[r * 3 + c];
    }
  for (int r = 0; r < 3; ++r) Ad[r * 7 + 6] = -t[r];
  Ad[6 * 7 + 6] = 1.0;
}

void apply_mat(const M4& T, const double* X, double* Y) {
  for (int r = 0; r < 3; ++r)
    Y[r] = T[r * 4 + 0] * X[0] + T[r * 4 + 1] * X[1] + T[r * 4 + 2] * X[2] + T[r * 4 + 3];
}

// ------------------------------------------------------------------------------------------------
// Ray operator psi(X) = X/|X| and holes
// ------------------------------------------------------------------------------------------------
bool is_hole(const double* X) {
  if (!std::isfinite(X[0]) || !std::isfinite(X[1]) || !std::isfinite(X[2])) return true;
  return std::sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]) <= 1e-9;
}

double norm3(const double* X) { return std::sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]); }

// ------------------------------------------------------------------------------------------------
// Projective ray matching (Sec. III-A): minimise |s(p) - psi(x)|^2 over the continuous reference pixel
// p, where s is the bilinear interpolant of the reference ray image psi(X_ref).
// ------------------------------------------------------------------------------------------------
struct RaySample {
  double s[3], su[3], sv[3];
  bool hole;
};

// Bilinear interpolant of the ray image in the cell holding p (the last cell at the far border), and
// its exact partial derivatives inside that cell.
RaySample sample_rays(const std::vector<double>& rays, const std::vector<char>& holes, int H, int W,
                      double u, double v) {
  RaySample out{};
  int u0 = std::min(static_cast<int>(std::floor(u)), W - 2);
  int v0 = std::min(static_cast<int>(std::floor(v)), H - 2);
  u0 = std::max(u0, 0);
  v0 = std::max(v0, 0);
  double fu = u - u0, fv = v - v0;
  int i00 = v0 * W + u0, i10 = i00 + 1, i01 = i00 + W, i11 = i01 + 1;
  out.hole = holes[i00] || holes[i10] || holes[i01] || holes[i11];
  for (int c = 0; c < 3; ++c) {
    double r00 = rays[i00 * 3 + c], r10 = rays[i10 * 3 + c];
    double r01 = rays[i01 * 3 + c], r11 = rays[i11 * 3 + c];
    out.s[c] = (1 - fu) * (1 - fv) * r00 + fu * (1 - fv) * r10 + (1 - fu) * fv * r01 + fu * fv * r11;
    out.su[c] = (1 - fv) * (r10 - r00) + fv * (r11 - r01);
    out.sv[c] = (1 - fu) * (r01 - r00) + fu * (r11 - r10);
  }
  return out;
}

struct MatchOut {
  int32_t idx;    // v*W + u in the reference, -1 when invalid
  double pu, pv;  // continuous optimum
  double ang_ratio;    // |r| / (ang_tol * min|ds|) at the optimum (validity test ii)
  double range_ratio;  // ||x| - |X_ref|| / (range_tol |X_ref|) (validity test iii)
  int32_t iters;       // LM trial steps taken
};

MatchOut match_one(const double* x, int qu, int qv, int Hq, int Wq, const double* ref_xyz,
                   const std::vector<double>& rays, const std::vector<char>& holes, int H, int W,
                   const orc_match_params& P) {
  MatchOut o{-1, NAN, NAN, NAN, NAN, 0};
  if (is_hole(x)) return o;
  double dx = norm3(x);
  double t[3] = {x[0] / dx, x[1] / dx, x[2] / dx};
  double u = (Wq > 1) ? qu * double(W - 1) / double(Wq - 1) : 0.0;
  double v = (Hq > 1) ? qv * double(H - 1) / double(Hq - 1) : 0.0;
  RaySample S = sample_rays(rays, holes, H, W, u, v);
  if (S.hole) return o;
  auto cost_of = [&](const RaySample& R) {
    double c = 0.0;
    for (int k = 0; k < 3; ++k) c += (R.s[k] - t[k]) * (R.s[k] - t[k]);
    return c;
  };
  double c = cost_of(S);
  double lam = P.lambda0;
  int it = 0;
  for (; it < P.max_iters; ++it) {
    double a = 0, b = 0, d = 0, gu = 0, gv = 0;
    for (int k = 0; k < 3; ++k) {
      double r = S.s[k] - t[k];
      a += S.su[k] * S.su[k];
      b += S.su[k] * S.sv[k];
      d += S.sv[k] * S.sv[k];
      gu += S.su[k] * r;
      gv += S.sv[k] * r;
    }
    double A = a * (1.0 + lam), D = d * (1.0 + lam);
    double det = A * D - b * b;
    if (!(det > 0.0)) { lam *= 10.0; continue; }
    double du = -(D * gu - b * gv) / det;
    double dv = -(A * gv - b * gu) / det;
    double un = std::min(std::max(u + du, 0.0), double(W - 1));
    double vn = std::min(std::max(v + dv, 0.0), double(H - 1));
    RaySample Sn = sample_rays(rays, holes, H, W, un, vn);
    if (Sn.hole) { o.iters = it + 1; return o; }
    double cn = cost_of(Sn);
    double step = std::max(std::fabs(un - u), std::fabs(vn - v));
    if (cn < c) {
      u = un; v = vn; S = Sn; c = cn;
      lam = std::max(lam * 0.1, P.lambda_min);
    } else {
      lam *= 10.0;
    }
    // convergence: a trial step below the tolerance ends the search, accepted or not (a rejected one
    // that short means the cost no longer decreases along the damped Gauss-Newton direction, and the
    // tenfold damping would only shorten the next steps further)
    if (step < P.step_tol_px) { ++it; break; }
  }
  o.iters = it;
  o.pu = u;
  o.pv = v;
  double nsu = norm3(S.su), nsv = norm3(S.sv);
  double rr = std::sqrt(c);
  o.ang_ratio = rr / (P.ang_tol_px * std::min(nsu, nsv));
  int mu = std::min(std::max(static_cast<int>(std::floor(u + 0.5)), 0), W - 1);
  int mv = std::min(std::max(static_cast<int>(std::floor(v + 0.5)), 0), H - 1);
  int m = mv * W + mu;
  const double* Xr = ref_xyz + 3 * static_cast<int64_t>(m);
  if (is_hole(Xr)) return o;
  double dr = norm3(Xr);
  o.range_ratio = std::fabs(dx - dr) / (P.range_rel_tol * dr);
  if (o.ang_ratio <= 1.0 && o.range_ratio <= 1.0) o.idx = m;
  return o;
}

void build_rays(const double* xyz, int64_t n, std::vector<double>& rays, std::vector<char>& holes) {
  rays.assign(3 * n, 0.0);
  holes.assign(n, 0);
  for (int64_t k = 0; k < n; ++k) {
    const double* X = xyz + 3 * k;
    if (is_hole(X)) { holes[k] = 1; continue; }
    double d = norm3(X);
    for (int c = 0; c < 3; ++c) rays[3 * k + c] = X[c] / d;
  }
}

// ------------------------------------------------------------------------------------------------
// Huber kernel (Sec. III-A): rho(r) = r^2/2 for |r| <= k, k|r| - k^2/2 beyond; IRLS weight min(1, k/|r|).
// ------------------------------------------------------------------------------------------------
double huber_rho(double r, double k) {
  double a = std::fabs(r);
  return (a <= k) ? 0.5 * r * r : k * a - 0.5 * k * k;
}
double huber_w(double r, double k) {
  double a = std::fabs(r);
  return (a <= k) ? 1.0 : k / a;
}

// ------------------------------------------------------------------------------------------------
// Per-edge linearisation of E_global (eq. 5) with the chain of eq. (6):
//   x = T_ij X_j,  J_x = [Dpsi/Dx ; Dd/Dx] [I  -[x]x  x],  J_j = J_x Ad_{T_i^-1},  J_i = -J_x Ad_{T_i^-1}.
// Accumulates the edge's 14x14 block of J^T W J, its 14-vector J^T W e, the cost and the count.
// ------------------------------------------------------------------------------------------------
struct EdgeAcc {
  double H[14 * 14];
  double g[14];
  double cost;
  int64_t count;
};

struct Residual {
  double e[4];
  double x[3];
  double d;
  double q;
  bool ok;
};

// Residual of eq. (1) for one match; ok == false for holes and non-finite values.
Residual edge_residual(const M4& Tij, const double* Xj, const double* Xi, double Ci, double Cj) {
  Residual R{};
  R.ok = false;
  if (is_hole(Xj) || is_hole(Xi) || !std::isfinite(Ci) || !std::isfinite(Cj)) return R;
  apply_mat(Tij, Xj, R.x);
  R.d = norm3(R.x);
  if (!(R.d > 1e-9)) return R;
  double di = norm3(Xi);
  for (int c = 0; c < 3; ++c) R.e[c] = R.x[c] / R.d - Xi[c] / di;
  R.e[3] = R.d - di;
  R.q = std::sqrt(Ci * Cj);
  R.ok = std::isfinite(R.q);
  return R;
}

void linearize_edge(const M4& Ti, const M4& Tj, const double* xyz_j, const double* conf_j,
                    int64_t npx_j, const double* xyz_i, const double* conf_i, int64_t npx_i,
                    const int32_t* idx, const orc_gn_params& P, EdgeAcc& acc) {
  std::memset(&acc, 0, sizeof(acc));
  M4 Tiinv = sim3_inverse_mat(Ti);
  M4 Tij = m4_mul(Tiinv, Tj);
  double Ad[49];
  sim3_adjoint(Tiinv, Ad);
  const double sig[4] = {P.sigma_ray, P.sigma_ray, P.sigma_ray, P.sigma_dist};
  for (int64_t n = 0; n < npx_j; ++n) {
    int32_t m = idx[n];
    if (m < 0 || m >= npx_i) continue;
    Residual R = edge_residual(Tij, xyz_j + 3 * n, xyz_i + 3 * int64_t(m), conf_i[m], conf_j[n]);
    if (!R.ok) continue;
    double sq = std::sqrt(R.q);
    double W[4];
    for (int c = 0; c < 4; ++c) {
      double r = sq * R.e[c] / sig[c];
      acc.cost += huber_rho(r, P.huber_k);
      W[c] = huber_w(r, P.huber_k) * R.q / (sig[c] * sig[c]);
    }
    acc.count += 1;
    // [Dpsi/Dx ; Dd/Dx]: 4x3
    const double d = R.d;
    double Dpx[4][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        Dpx[a][b] = ((a == b ? 1.0 : 0.0) - R.x[a] * R.x[b] / (d * d)) / d;
    for (int b = 0; b < 3; ++b) Dpx[3][b] = R.x[b] / d;
    // Dx/Dtau = [I  -[x]x  x]: 3x7
    const double* x = R.x;
    double Dxt[3][7] = {{1, 0, 0, 0, x[2], -x[1], x[0]},
                        {0, 1, 0, -x[2], 0, x[0], x[1]},
                        {0, 0, 1, x[1], -x[0], 0, x[2]}};
    double Jx[4][7];
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 7; ++k) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b) s += Dpx[a][b] * Dxt[b][k];
        Jx[a][k] = s;
      }
    // Full 4x14 Jacobian: [J_i | J_j] = [-J_x Ad | +J_x Ad]
    double J[4][14];
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 7; ++k) {
        double s = 0.0;
        for (int l = 0; l < 7; ++l) s += Jx[a][l] * Ad[l * 7 + k];
        J[a][k] = -s;
        J[a][7 + k] = s;
      }
    for (int r = 0; r < 14; ++r) {
      for (int c = 0; c < 14; ++c) {
        double s = 0.0;
        for (int a = 0; a < 4; ++a) s += J[a][r] * W[a] * J[a][c];
        acc.H[r * 14 + c] += s;
      }
      double s = 0.0;
      for (int a = 0; a < 4; ++a) s += J[a][r] * W[a] * R.e[a];
      acc.g[r] += s;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Calibrated mode (Sec. IV-C, "Calibration": with supplied intrinsics the pointmaps are constrained to
// the calibrated rays and the pose residuals are pixel reprojection and log-depth). Readings:
//   the calibrated point of pixel n = (u, v) of keyframe k is z K_k^-1 (u, v, 1), z = the predicted
//   point's depth (its third coordinate); for a match (m, n) of edge (i, j), x = T_ij Xcal_j[n] and
//     r = ( fx_i x0/x2 + cx_i - u_m,  fy_i x1/x2 + cy_i - v_m,  ln x2 - ln z_i[m] ),
//   whitened by sqrt(q)/sigma_pix (pixel rows) and sqrt(q)/sigma_logz (depth row), q = sqrt(C_i C_j);
//   the same component-wise Huber kernel and IRLS weights; a match is used only if neither point is a
//   hole, z_j[n], z_i[m] and x2 are above 1e-9 (both points and the transformed one in front) and the
//   reprojection lands on keyframe i's image, -0.5 <= fx_i x0/x2 + cx_i < W_i - 0.5 and likewise for v
//   with H_i (a reprojection off the image is no pixel of i; it also keeps x0/x2 and x1/x2 bounded).
// The chain rule is the one of eq. (6) with this residual: J_x = (dr/dx) [I  -[x]x  x].
// ------------------------------------------------------------------------------------------------
struct CalResidual {
  double r[3];  // unwhitened: pixel, pixel, log-depth
  double x[3];
  double q;
  bool ok;
};

// K: fx, fy, cx, cy of a keyframe.
CalResidual cal_residual(const M4& Tij, const double* Xj, int64_t n, int Wj, const double* Kj, const double* Xi,
                         int64_t m, int Wi, int Hi, const double* Ki, double Ci, double Cj) {
  CalResidual R{};
  R.ok = false;
  if (is_hole(Xj) || is_hole(Xi) || !std::isfinite(Ci) || !std::isfinite(Cj)) return R;
  const double zj = Xj[2], zi = Xi[2];
  if (!(zj > 1e-9) || !(zi > 1e-9)) return R;
  const double un = double(n % Wj), vn = double(n / Wj);
  const double Xc[3] = {zj * (un - Kj[2]) / Kj[0], zj * (vn - Kj[3]) / Kj[1], zj};
  apply_mat(Tij, Xc, R.x);
  if (!(R.x[2] > 1e-9)) return R;
  const double um = double(m % Wi), vm = double(m / Wi);
  const double pu = Ki[0] * R.x[0] / R.x[2] + Ki[2], pv = Ki[1] * R.x[1] / R.x[2] + Ki[3];
  if (!(pu >= -0.5 && pu < Wi - 0.5 && pv >= -0.5 && pv < Hi - 0.5)) return R;
  R.r[0] = pu - um;
  R.r[1] = pv - vm;
  R.r[2] = std::log(R.x[2]) - std::log(zi);
  R.q = std::sqrt(Ci * Cj);
  R.ok = std::isfinite(R.q) && std::isfinite(R.r[0]) && std::isfinite(R.r[1]) && std::isfinite(R.r[2]);
  return R;
}

void linearize_edge_cal(const M4& Ti, const M4& Tj, const double* xyz_j, const double* conf_j, int64_t npx_j,
                        int Wj, const double* Kj, const double* xyz_i, const double* conf_i, int64_t npx_i, int Wi,
                        const double* Ki, const int32_t* idx, double sigma_pix, double sigma_logz,
                        const orc_gn_params& P, EdgeAcc& acc) {
  std::memset(&acc, 0, sizeof(acc));
  M4 Tiinv = sim3_inverse_mat(Ti);
  M4 Tij = m4_mul(Tiinv, Tj);
  double Ad[49];
  sim3_adjoint(Tiinv, Ad);
  const double sig[3] = {sigma_pix, sigma_pix, sigma_logz};
  for (int64_t n = 0; n < npx_j; ++n) {
    int32_t m = idx[n];
    if (m < 0 || m >= npx_i) continue;
    CalResidual R = cal_residual(Tij, xyz_j + 3 * n, n, Wj, Kj, xyz_i + 3 * int64_t(m), m, Wi, int(npx_i / Wi), Ki,
                                 conf_i[m], conf_j[n]);
    if (!R.ok) continue;
    double sq = std::sqrt(R.q);
    double W[3];
    for (int c = 0; c < 3; ++c) {
      double r = sq * R.r[c] / sig[c];
      acc.cost += huber_rho(r, P.huber_k);
      W[c] = huber_w(r, P.huber_k) * R.q / (sig[c] * sig[c]);
    }
    acc.count += 1;
    const double* x = R.x;
    const double z = x[2];
    // dr/dx: 3x3
    double Drx[3][3] = {{Ki[0] / z, 0.0, -Ki[0] * x[0] / (z * z)},
                        {0.0, Ki[1] / z, -Ki[1] * x[1] / (z * z)},
                        {0.0, 0.0, 1.0 / z}};
    // Dx/Dtau = [I  -[x]x  x]: 3x7
    double Dxt[3][7] = {{1, 0, 0, 0, x[2], -x[1], x[0]},
                        {0, 1, 0, -x[2], 0, x[0], x[1]},
                        {0, 0, 1, x[1], -x[0], 0, x[2]}};
    double Jx[3][7];
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 7; ++k) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b) s += Drx[a][b] * Dxt[b][k];
        Jx[a][k] = s;
      }
    // [J_i | J_j] = [-J_x Ad | +J_x Ad]
    double J[3][14];
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 7; ++k) {
        double s = 0.0;
        for (int l = 0; l < 7; ++l) s += Jx[a][l] * Ad[l * 7 + k];
        J[a][k] = -s;
        J[a][7 + k] = s;
      }
    for (int r = 0; r < 14; ++r) {
      for (int c = 0; c < 14; ++c) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s += J[a][r] * W[a] * J[a][c];
        acc.H[r * 14 + c] += s;
      }
      double s = 0.0;
      for (int a = 0; a < 3; ++a) s += J[a][r] * W[a] * R.r[a];
      acc.g[r] += s;
    }
  }
}

// Scatter of the per-edge 14x14 blocks and 14-vectors into H (7N x 7N) and g in edge order, then the
// anchor rows and columns replaced by identity (g = 0).
void scatter_blocks(const std::vector<EdgeAcc>& acc, int n_kf, const int32_t* ei, const int32_t* ej, int n_edges,
                    const int32_t* anchors, int n_anchors, double* H, double* g, double* cost_out,
                    int64_t* count_out, double* edge_cost, int64_t* edge_count) {
  const int64_t n = 7 * int64_t(n_kf);
  std::fill(H, H + n * n, 0.0);
  std::fill(g, g + n, 0.0);
  double cost = 0.0;
  int64_t count = 0;
  for (int e = 0; e < n_edges; ++e) {
    const int64_t base[2] = {7 * int64_t(ei[e]), 7 * int64_t(ej[e])};
    for (int r = 0; r < 14; ++r) {
      int64_t gr = base[r / 7] + r % 7;
      for (int c = 0; c < 14; ++c) H[gr * n + base[c / 7] + c % 7] += acc[e].H[r * 14 + c];
      g[gr] += acc[e].g[r];
    }
    cost += acc[e].cost;
    count += acc[e].count;
    if (edge_cost) edge_cost[e] = acc[e].cost;
    if (edge_count) edge_count[e] = acc[e].count;
  }
  for (int a = 0; a < n_anchors; ++a) {
    int64_t b0 = 7 * int64_t(anchors[a]);
    for (int64_t r = b0; r < b0 + 7; ++r) {
      for (int64_t c = 0; c < n; ++c) { H[r * n + c] = 0.0; H[c * n + r] = 0.0; }
      H[r * n + r] = 1.0;
      g[r] = 0.0;
    }
  }
  *cost_out = cost;
  if (count_out) *count_out = count;
}

// Plain Cholesky M = L L^T (lower, row by row). Fails on a non-positive or non-finite pivot.
bool cholesky(std::vector<double>& M, int n) {
  for (int j = 0; j < n; ++j) {
    double s = M[int64_t(j) * n + j];
    for (int k = 0; k < j; ++k) s -= M[int64_t(j) * n + k] * M[int64_t(j) * n + k];
    if (!(s > 0.0) || !std::isfinite(s)) return false;
    double ljj = std::sqrt(s);
    M[int64_t(j) * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = M[int64_t(i) * n + j];
      for (int k = 0; k < j; ++k) t -= M[int64_t(i) * n + k] * M[int64_t(j) * n + k];
      M[int64_t(i) * n + j] = t / ljj;
    }
  }
  return true;
}

// eq. (7) with the epsilon ladder: attempts r = 0..max_attempts-1 with eps_r = eps0 * mult^r; a zero step
// and status -1 when every attempt fails; otherwise status = r of the attempt that factorised.
int chol_ladder(const double* H, const double* g, int n, double lambda, double eps0, double mult,
                int attempts, double* tau) {
  std::vector<double> M(int64_t(n) * n);
  double eps = eps0;
  for (int r = 0; r < attempts; ++r, eps *= mult) {
    for (int64_t e = 0; e < int64_t(n) * n; ++e) M[e] = H[e];
    for (int k = 0; k < n; ++k) M[int64_t(k) * n + k] += lambda * H[int64_t(k) * n + k] + eps;
    if (!cholesky(M, n)) continue;
    std::vector<double> y(n);
    for (int i = 0; i < n; ++i) {
      double s = -g[i];
      for (int k = 0; k < i; ++k) s -= M[int64_t(i) * n + k] * y[k];
      y[i] = s / M[int64_t(i) * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < n; ++k) s -= M[int64_t(k) * n + i] * tau[k];
      tau[i] = s / M[int64_t(i) * n + i];
    }
    return r;
  }
  for (int i = 0; i < n; ++i) tau[i] = 0.0;
  return -1;
}

}  // namespace

// ================================================================================================
// C ABI of the oracle
// ================================================================================================
extern "C" {

int orc_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_sim3_exp(const double* tau, double* pose_out) { mat_to_pose(sim3_exp_mat(tau), pose_out); }

void orc_sim3_exp_mat(const double* tau, double* M_out) {
  M4 M = sim3_exp_mat(tau);
  std::memcpy(M_out, M.data(), sizeof(double) * 16);
}

void orc_sim3_log(const double* pose, double* tau) { sim3_log_pose(pose, tau); }

void orc_pose_to_mat(const double* pose, double* M_out) {
  M4 M = pose_to_mat(pose);
  std::memcpy(M_out, M.data(), sizeof(double) * 16);
}

void orc_mat_to_pose(const double* M_in, double* pose) {
  M4 M;
  std::memcpy(M.data(), M_in, sizeof(double) * 16);
  mat_to_pose(M, pose);
}

void orc_sim3_adjoint(const double* pose, double* Ad) { sim3_adjoint(pose_to_mat(pose), Ad); }

// Relative pose T_ij = T_i^-1 T_j as a pose vector.
void orc_relative(const double* pi, const double* pj, double* pij) {
  mat_to_pose(m4_mul(sim3_inverse_mat(pose_to_mat(pi)), pose_to_mat(pj)), pij);
}

// Left update T <- Exp(tau) T for n poses; entries flagged in `fixed` are left untouched.
void orc_sim3_update(double* poses, const double* tau, int n, const uint8_t* fixed) {
  for (int k = 0; k < n; ++k) {
    if (fixed && fixed[k]) continue;
    M4 T = m4_mul(sim3_exp_mat(tau + 7 * k), pose_to_mat(poses + 8 * k));
    mat_to_pose(T, poses + 8 * k);
  }
}

// One matching direction. ref: canonical pointmap of the reference view (H x W x 3); qry: the other
// view's points expressed in the reference camera (Hq x Wq x 3). Outputs per query pixel: idx (-1 invalid)
// and optional diagnostics (continuous optimum, the two validity ratios, LM trial steps).
int orc_match(const double* ref_xyz, int H, int W, const double* qry_xyz, int Hq, int Wq,
              const orc_match_params* P, int32_t* idx_out, double* p_out, double* ratios_out,
              int32_t* iters_out) {
  if (H < 2 || W < 2 || Hq < 1 || Wq < 1) return -1;
  std::vector<double> rays;
  std::vector<char> holes;
  build_rays(ref_xyz, int64_t(H) * W, rays, holes);
  const int64_t nq = int64_t(Hq) * Wq;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t n = 0; n < nq; ++n) {
    int qu = int(n % Wq), qv = int(n / Wq);
    MatchOut o = match_one(qry_xyz + 3 * n, qu, qv, Hq, Wq, ref_xyz, rays, holes, H, W, *P);
    idx_out[n] = o.idx;
    if (p_out) { p_out[2 * n] = o.pu; p_out[2 * n + 1] = o.pv; }
    if (ratios_out) { ratios_out[2 * n] = o.ang_ratio; ratios_out[2 * n + 1] = o.range_ratio; }
    if (iters_out) iters_out[n] = o.iters;
  }
  return 0;
}

// Mutual consistency (both decoded directions) and the nu gate of Sec. III-B.
// idx_ji: per pixel of j, its match in i; idx_ij: per pixel of i, its match in j.
// valid_j[n] = 1 iff idx_ji[n] = m >= 0, idx_ij[m] = n' >= 0 and Chebyshev(n', n) <= radius (grid of j);
// nu_j counts valid pixels with q = sqrt(C_i[m] C_j[n]) >= q_min over H_j W_j; nu_i symmetrically.
// idx_out = idx_ji where valid_j, else -1. Returns admit (1) or reject (0).
int orc_mutual(const int32_t* idx_ji, const int32_t* idx_ij, int Hi, int Wi, int Hj, int Wj,
               const double* conf_i, const double* conf_j, const orc_match_params* P,
               int32_t* idx_out, uint8_t* valid_j, double* nu /* [nu_i, nu_j] */) {
  const int64_t nj = int64_t(Hj) * Wj, ni = int64_t(Hi) * Wi;
  int64_t cnt_j = 0, cnt_i = 0;
  for (int64_t n = 0; n < nj; ++n) {
    int32_t m = idx_ji[n];
    uint8_t ok = 0;
    if (m >= 0 && m < ni) {
      int32_t n2 = idx_ij[m];
      if (n2 >= 0 && n2 < nj) {
        int du = std::abs(int(n2 % Wj) - int(n % Wj)), dv = std::abs(int(n2 / Wj) - int(n / Wj));
        ok = std::max(du, dv) <= P->mutual_radius_px;
      }
    }
    valid_j[n] = ok;
    idx_out[n] = ok ? m : -1;
    if (ok && std::sqrt(conf_i[m] * conf_j[n]) >= P->q_min) ++cnt_j;
  }
  for (int64_t m = 0; m < ni; ++m) {
    int32_t n = idx_ij[m];
    if (n < 0 || n >= nj) continue;
    int32_t m2 = idx_ji[n];
    if (m2 < 0 || m2 >= ni) continue;
    int du = std::abs(int(m2 % Wi) - int(m % Wi)), dv = std::abs(int(m2 / Wi) - int(m / Wi));
    if (std::max(du, dv) <= P->mutual_radius_px && std::sqrt(conf_j[n] * conf_i[m]) >= P->q_min) ++cnt_i;
  }
  nu[0] = double(cnt_i) / double(ni);
  nu[1] = double(cnt_j) / double(nj);
  return std::min(nu[0], nu[1]) >= P->nu_min ? 1 : 0;
}

// Assemble eq. (7)'s H and g over all edges (eq. 5), plus E at the given poses.
// Keyframes: xyz (3 per px) and conf arenas with per-keyframe pixel offsets and sizes.
// Edge e = (ei[e], ej[e]) reads idx[idx_off[e] ...] over the pixels of ej[e].
// Anchor blocks: rows and columns replaced by identity, g = 0.
// Outputs H (7N x 7N row-major), g (7N), cost, valid count; optional per-edge [cost, count].
int orc_gn_assemble(const double* poses, int n_kf, const int64_t* kf_off, const int64_t* kf_npx,
                    const double* xyz, const double* conf, const int32_t* ei, const int32_t* ej,
                    const int64_t* idx_off, int n_edges, const int32_t* idx, const int32_t* anchors,
                    int n_anchors, const orc_gn_params* P, double* H, double* g, double* cost_out,
                    int64_t* count_out, double* edge_cost, int64_t* edge_count) {
  std::vector<EdgeAcc> acc(n_edges);
#pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < n_edges; ++e) {
    int i = ei[e], j = ej[e];
    linearize_edge(pose_to_mat(poses + 8 * i), pose_to_mat(poses + 8 * j), xyz + 3 * kf_off[j],
                   conf + kf_off[j], kf_npx[j], xyz + 3 * kf_off[i], conf + kf_off[i], kf_npx[i],
                   idx + idx_off[e], *P, acc[e]);
  }
  scatter_blocks(acc, n_kf, ei, ej, n_edges, anchors, n_anchors, H, g, cost_out, count_out, edge_cost, edge_count);
  return 0;
}

// Solve (H + lambda diag H + eps_r I) tau = -g with the epsilon ladder. Returns the status.
int orc_chol_ladder(const double* H, const double* g, int n, double lambda, double eps0, double mult,
                    int attempts, double* tau) {
  return chol_ladder(H, g, n, lambda, eps0, mult, attempts, tau);
}

// One Gauss-Newton/IRLS step of eq. (5) via eq. (7): assemble at the input poses, solve with the
// ladder, update every non-anchor pose by T <- Exp(tau) T. cost_out = E at the input poses.
int orc_gn_step(double* poses, int n_kf, const int64_t* kf_off, const int64_t* kf_npx,
                const double* xyz, const double* conf, const int32_t* ei, const int32_t* ej,
                const int64_t* idx_off, int n_edges, const int32_t* idx, const int32_t* anchors,
                int n_anchors, const orc_gn_params* P, double* cost_out, int32_t* status_out,
                double* tau_out) {
  const int64_t n = 7 * int64_t(n_kf);
  std::vector<double> H(n * n), g(n), tau(n);
  int64_t count = 0;
  orc_gn_assemble(poses, n_kf, kf_off, kf_npx, xyz, conf, ei, ej, idx_off, n_edges, idx, anchors,
                  n_anchors, P, H.data(), g.data(), cost_out, &count, nullptr, nullptr);
  int st = chol_ladder(H.data(), g.data(), int(n), P->lambda, P->eps0, P->eps_mult, P->max_attempts,
                       tau.data());
  std::vector<uint8_t> fixed(n_kf, 0);
  for (int a = 0; a < n_anchors; ++a) fixed[anchors[a]] = 1;
  orc_sim3_update(poses, tau.data(), n_kf, fixed.data());
  if (status_out) *status_out = st;
  if (tau_out) std::memcpy(tau_out, tau.data(), sizeof(double) * n);
  return 0;
}

// E_global alone (eq. 5) at the given poses.
double orc_cost(const double* poses, int n_kf, const int64_t* kf_off, const int64_t* kf_npx,
                const double* xyz, const double* conf, const int32_t* ei, const int32_t* ej,
                const int64_t* idx_off, int n_edges, const int32_t* idx, const orc_gn_params* P) {
  std::vector<double> ec(n_edges);
  const double sig[4] = {P->sigma_ray, P->sigma_ray, P->sigma_ray, P->sigma_dist};
#pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < n_edges; ++e) {
    int i = ei[e], j = ej[e];
    M4 Tij = m4_mul(sim3_inverse_mat(pose_to_mat(poses + 8 * i)), pose_to_mat(poses + 8 * j));
    const double* xj = xyz + 3 * kf_off[j];
    const double* xi = xyz + 3 * kf_off[i];
    const double* cj = conf + kf_off[j];
    const double* ci = conf + kf_off[i];
    const int32_t* id = idx + idx_off[e];
    double c = 0.0;
    for (int64_t p = 0; p < kf_npx[j]; ++p) {
      int32_t m = id[p];
      if (m < 0 || m >= kf_npx[i]) continue;
      Residual R = edge_residual(Tij, xj + 3 * p, xi + 3 * int64_t(m), ci[m], cj[p]);
      if (!R.ok) continue;
      double sq = std::sqrt(R.q);
      for (int k = 0; k < 4; ++k) c += huber_rho(sq * R.e[k] / sig[k], P->huber_k);
    }
    ec[e] = c;
  }
  double cost = 0.0;
  for (int e = 0; e < n_edges; ++e) cost += ec[e];
  return cost;
}

// Gradient of E_global (eq. 5) with the matches held fixed, with respect to the canonical pointmaps
// (3 per px), the confidences, and a left tangent tau per pose (7 per keyframe). Uses
// d rho / d r = w r, r_c = sqrt(q) e_c / sigma_c, q = sqrt(C_i C_j), so d r_c / d C = r_c / (4 C).
// Gradients are accumulated (+=) into caller-zeroed buffers, edges in index order.
int orc_cost_grad(const double* poses, int n_kf, const int64_t* kf_off, const int64_t* kf_npx,
                  const double* xyz, const double* conf, const int32_t* ei, const int32_t* ej,
                  const int64_t* idx_off, int n_edges, const int32_t* idx, const orc_gn_params* P,
                  double* grad_xyz, double* grad_conf, double* grad_tau, double* cost_out) {
  const double sig[4] = {P->sigma_ray, P->sigma_ray, P->sigma_ray, P->sigma_dist};
  double cost = 0.0;
  for (int e = 0; e < n_edges; ++e) {
    int i = ei[e], j = ej[e];
    M4 Tiinv = sim3_inverse_mat(pose_to_mat(poses + 8 * i));
    M4 Tij = m4_mul(Tiinv, pose_to_mat(poses + 8 * j));
    double Ad[49];
    sim3_adjoint(Tiinv, Ad);
    const double* xj = xyz + 3 * kf_off[j];
    const double* xi = xyz + 3 * kf_off[i];
    const double* cj = conf + kf_off[j];
    const double* ci = conf + kf_off[i];
    const int32_t* id = idx + idx_off[e];
    double gx[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t p = 0; p < kf_npx[j]; ++p) {
      int32_t m = id[p];
      if (m < 0 || m >= kf_npx[i]) continue;
      Residual R = edge_residual(Tij, xj + 3 * p, xi + 3 * int64_t(m), ci[m], cj[p]);
      if (!R.ok) continue;
      double sq = std::sqrt(R.q);
      double gam[4], dc = 0.0;
      for (int k = 0; k < 4; ++k) {
        double r = sq * R.e[k] / sig[k];
        cost += huber_rho(r, P->huber_k);
        double drho = huber_w(r, P->huber_k) * r;  // rho'(r)
        gam[k] = drho * sq / sig[k];              // dE/de_k
        dc += drho * r;
      }
      // dE/dx through psi(x) and |x|
      const double d = R.d;
      double gxv[3];
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b)
          s += gam[b] * ((a == b ? 1.0 : 0.0) - R.x[a] * R.x[b] / (d * d)) / d;
        gxv[a] = s + gam[3] * R.x[a] / d;
      }
      // x = sR_ij X_j + t_ij  ->  dE/dX_j = (sR_ij)^T dE/dx
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b) s += Tij[b * 4 + a] * gxv[b];
        grad_xyz[3 * (kf_off[j] + p) + a] += s;
      }
      // e depends on X_i through -psi(X_i) and -|X_i|
      const double* Xi = xi + 3 * int64_t(m);
      double di = norm3(Xi);
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b)
          s += gam[b] * ((a == b ? 1.0 : 0.0) - Xi[a] * Xi[b] / (di * di)) / di;
        grad_xyz[3 * (kf_off[i] + m) + a] -= s + gam[3] * Xi[a] / di;
      }
      grad_conf[kf_off[j] + p] += dc / (4.0 * cj[p]);
      grad_conf[kf_off[i] + m] += dc / (4.0 * ci[m]);
      // pose tangent: dE/dtau_j = Ad^T [I -[x]x x]^T dE/dx, dE/dtau_i = -(same)
      const double* x = R.x;
      double Dxt[3][7] = {{1, 0, 0, 0, x[2], -x[1], x[0]},
                          {0, 1, 0, -x[2], 0, x[0], x[1]},
                          {0, 0, 1, x[1], -x[0], 0, x[2]}};
      for (int k = 0; k < 7; ++k) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b) s += Dxt[b][k] * gxv[b];
        gx[k] += s;
      }
    }
    for (int k = 0; k < 7; ++k) {
      double s = 0.0;
      for (int l = 0; l < 7; ++l) s += Ad[l * 7 + k] * gx[l];
      grad_tau[7 * j + k] += s;
      grad_tau[7 * i + k] -= s;
    }
  }
  *cost_out = cost;
  return 0;
}

// Whitened residuals r_c = sqrt(q) e_c / sigma_c of eq. (1) and their IRLS weights, per pixel of j for one
// edge (i, j); rows of invalid pixels are zero with ok = 0. Exposed so tests can differentiate them.
int orc_edge_residuals(const double* pose_i, const double* pose_j, const double* xyz_j,
                       const double* conf_j, int64_t npx_j, const double* xyz_i, const double* conf_i,
                       int64_t npx_i, const int32_t* idx, const orc_gn_params* P, double* r_out,
                       double* w_out, uint8_t* ok_out) {
  M4 Tij = m4_mul(sim3_inverse_mat(pose_to_mat(pose_i)), pose_to_mat(pose_j));
  const double sig[4] = {P->sigma_ray, P->sigma_ray, P->sigma_ray, P->sigma_dist};
  for (int64_t n = 0; n < npx_j; ++n) {
    int32_t m = idx[n];
    ok_out[n] = 0;
    for (int c = 0; c < 4; ++c) { r_out[4 * n + c] = 0.0; w_out[4 * n + c] = 0.0; }
    if (m < 0 || m >= npx_i) continue;
    Residual R = edge_residual(Tij, xyz_j + 3 * n, xyz_i + 3 * int64_t(m), conf_i[m], conf_j[n]);
    if (!R.ok) continue;
    double sq = std::sqrt(R.q);
    for (int c = 0; c < 4; ++c) {
      r_out[4 * n + c] = sq * R.e[c] / sig[c];
      w_out[4 * n + c] = huber_w(r_out[4 * n + c], P->huber_k);
    }
    ok_out[n] = 1;
  }
  return 0;
}

// ---- calibrated mode (Sec. IV-C) ----------------------------------------------------------------
// As orc_gn_assemble with the calibrated residual: K (n_kf x 4: fx, fy, cx, cy) and kf_w (image width per
// keyframe) are the supplied intrinsics; sigma_pix and sigma_logz whiten the pixel and log-depth rows.
int orc_gn_assemble_cal(const double* poses, int n_kf, const int64_t* kf_off, const int64_t* kf_npx,
                        const int32_t* kf_w, const double* K, const double* xyz, const double* conf, const int32_t* ei,
                        const int32_t* ej, const int64_t* idx_off, int n_edges, const int32_t* idx,
                        const int32_t* anchors, int n_anchors, const orc_gn_params* P, double sigma_pix,
                        double sigma_logz, double* H, double* g, double* cost_out, int64_t* count_out,
                        double* edge_cost, int64_t* edge_count) {
  std::vector<EdgeAcc> acc(n_edges);
#pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < n_edges; ++e) {
    int i = ei[e], j = ej[e];
    linearize_edge_cal(pose_to_mat(poses + 8 * i), pose_to_mat(poses + 8 * j), xyz + 3 * kf_off[j], conf + kf_off[j],
                       kf_npx[j], kf_w[j], K + 4 * j, xyz + 3 * kf_off[i], conf + kf_off[i], kf_npx[i], kf_w[i],
                       K + 4 * i, idx + idx_off[e], sigma_pix, sigma_logz, *P, acc[e]);
  }
  scatter_blocks(acc, n_kf, ei, ej, n_edges, anchors, n_anchors, H, g, cost_out, count_out, edge_cost, edge_count);
  return 0;
}

// One Gauss-Newton/IRLS step in calibrated mode (assemble, ladder solve of eq. 7, left update).
int orc_gn_step_cal(double* poses, int n_kf, const int64_t* kf_off, const int64_t* kf_npx, const int32_t* kf_w,
                    const double* K, const double* xyz, const double* conf, const int32_t* ei, const int32_t* ej,
                    const int64_t* idx_off, int n_edges, const int32_t* idx, const int32_t* anchors, int n_anchors,
                    const orc_gn_params* P, double sigma_pix, double sigma_logz, double* cost_out,
                    int32_t* status_out, double* tau_out) {
  const int64_t n = 7 * int64_t(n_kf);
  std::vector<double> H(n * n), g(n), tau(n);
  orc_gn_assemble_cal(poses, n_kf, kf_off, kf_npx, kf_w, K, xyz, conf, ei, ej, idx_off, n_edges, idx, anchors,
                      n_anchors, P, sigma_pix, sigma_logz, H.data(), g.data(), cost_out, nullptr, nullptr, nullptr);
  int st = chol_ladder(H.data(), g.data(), int(n), P->lambda, P->eps0, P->eps_mult, P->max_attempts, tau.data());
  std::vector<uint8_t> fixed(n_kf, 0);
  for (int a = 0; a < n_anchors; ++a) fixed[anchors[a]] = 1;
  orc_sim3_update(poses, tau.data(), n_kf, fixed.data());
  if (status_out) *status_out = st;
  if (tau_out) std::memcpy(tau_out, tau.data(), sizeof(double) * n);
  return 0;
}

// Per pixel of j for one edge in calibrated mode: whitened residuals r (npx_j x 3), IRLS weights w
// (npx_j x 3) and the validity flag.
int orc_edge_residuals_cal(const double* pose_i, const double* pose_j, const double* xyz_j, const double* conf_j,
                           int64_t npx_j, int Wj, const double* Kj, const double* xyz_i, const double* conf_i,
                           int64_t npx_i, int Wi, const double* Ki, const int32_t* idx, const orc_gn_params* P,
                           double sigma_pix, double sigma_logz, double* r_out, double* w_out, uint8_t* ok_out) {
  M4 Tij = m4_mul(sim3_inverse_mat(pose_to_mat(pose_i)), pose_to_mat(pose_j));
  const double sig[3] = {sigma_pix, sigma_pix, sigma_logz};
  for (int64_t n = 0; n < npx_j; ++n) {
    int32_t m = idx[n];
    ok_out[n] = 0;
    for (int c = 0; c < 3; ++c) { r_out[3 * n + c] = 0.0; w_out[3 * n + c] = 0.0; }
    if (m < 0 || m >= npx_i) continue;
    CalResidual R = cal_residual(Tij, xyz_j + 3 * n, n, Wj, Kj, xyz_i + 3 * int64_t(m), m, Wi, int(npx_i / Wi), Ki,
                                 conf_i[m], conf_j[n]);
    if (!R.ok) continue;
    double sq = std::sqrt(R.q);
    for (int c = 0; c < 3; ++c) {
      r_out[3 * n + c] = sq * R.r[c] / sig[c];
      w_out[3 * n + c] = huber_w(r_out[3 * n + c], P->huber_k);
    }
    ok_out[n] = 1;
  }
  return 0;
}

// E in calibrated mode at the given poses.
double orc_cost_cal(const double* poses, int n_kf, const int64_t* kf_off, const int64_t* kf_npx, const int32_t* kf_w,
                    const double* K, const double* xyz, const double* conf, const int32_t* ei, const int32_t* ej,
                    const int64_t* idx_off, int n_edges, const int32_t* idx, const orc_gn_params* P, double sigma_pix,
                    double sigma_logz) {
  std::vector<double> ec(n_edges);
  const double sig[3] = {sigma_pix, sigma_pix, sigma_logz};
#pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < n_edges; ++e) {
    int i = ei[e], j = ej[e];
    M4 Tij = m4_mul(sim3_inverse_mat(pose_to_mat(poses + 8 * i)), pose_to_mat(poses + 8 * j));
    const int32_t* id = idx + idx_off[e];
    double c = 0.0;
    for (int64_t p = 0; p < kf_npx[j]; ++p) {
      int32_t m = id[p];
      if (m < 0 || m >= kf_npx[i]) continue;
      CalResidual R = cal_residual(Tij, xyz + 3 * (kf_off[j] + p), p, kf_w[j], K + 4 * j,
                                   xyz + 3 * (kf_off[i] + int64_t(m)), m, kf_w[i], int(kf_npx[i] / kf_w[i]), K + 4 * i,
                                   conf[kf_off[i] + m], conf[kf_off[j] + p]);
      if (!R.ok) continue;
      double sq = std::sqrt(R.q);
      for (int k = 0; k < 3; ++k) c += huber_rho(sq * R.r[k] / sig[k], P->huber_k);
    }
    ec[e] = c;
  }
  double cost = 0.0;
  for (int e = 0; e < n_edges; ++e) cost += ec[e];
  return cost;
}

}  // extern "C"
