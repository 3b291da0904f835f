"""FP64 CPU oracle of the dense Sim(3) back-end (CoMo3R-SLAM, Sec. III).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the product library never does. It shares no code with the HIP path.

The heavy loops (matching, per-pixel linearisation, Cholesky) live in ``ds3_oracle.cpp`` (plain FP64
C++, compiled by :func:`build`); this module marshals numpy arrays into it and holds the parts that are
plain numpy: Umeyama's closed form (eq. 4), the component tracker of Sec. III-C, the canonical pointmap
fusion of eq. (2), BF16 rounding and the pose-error measure.

Pose layout everywhere: ``[tx, ty, tz, qx, qy, qz, qw, s]`` (float64), ``T_WC = [[sR, t], [0, 1]]``.
Tangent layout: ``tau = (v, omega, zeta)`` (Sec. III-D).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ds3_oracle.cpp")
# DS3_ORACLE_LIB names another build of ds3_oracle.cpp to load (the sanitizer test's instrumented copy)
_LIB_PATH = os.environ.get("DS3_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, OpenMP, no FMA contraction so sums round as written)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["g++", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
               "-std=c++17", _SRC, "-o", _LIB_PATH + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class MatchParams(C.Structure):
    """Matching constants. nu_min = 0.1 is the paper's gate (Sec. III-B); the LM schedule, the
    validity tolerances, the mutual radius and q_min = 1.5 (the paper's only confidence threshold,
    Sec. III-E) are readings where the paper is silent."""
    _fields_ = [("max_iters", C.c_int32), ("lambda0", C.c_double), ("lambda_min", C.c_double),
                ("step_tol_px", C.c_double), ("ang_tol_px", C.c_double),
                ("range_rel_tol", C.c_double), ("mutual_radius_px", C.c_int32),
                ("q_min", C.c_double), ("nu_min", C.c_double)]

    @classmethod
    def default(cls) -> "MatchParams":
        return cls(10, 1e-4, 1e-9, 1e-4, 0.5, 0.10, 1, 1.5, 0.1)


class GNParams(C.Structure):
    """sigma_r = 0.003, sigma_d = 10, kappa = 1.345 (Sec. IV-A, Implementation); lambda = 0 for the
    back-end and eps_r = 1e-6 * 100^r over six attempts (text after eq. 7)."""
    _fields_ = [("sigma_ray", C.c_double), ("sigma_dist", C.c_double), ("huber_k", C.c_double),
                ("lam", C.c_double), ("eps0", C.c_double), ("eps_mult", C.c_double),
                ("max_attempts", C.c_int32)]

    @classmethod
    def default(cls) -> "GNParams":
        return cls(0.003, 10.0, 1.345, 0.0, 1e-6, 100.0, 6)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        d, i32, i64, u8 = (C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                           C.POINTER(C.c_uint8))
        L.orc_num_threads.restype = C.c_int
        for name in ("orc_sim3_exp", "orc_sim3_exp_mat", "orc_sim3_log", "orc_pose_to_mat",
                     "orc_mat_to_pose", "orc_sim3_adjoint"):
            getattr(L, name).argtypes = [d, d]
            getattr(L, name).restype = None
        L.orc_relative.argtypes = [d, d, d]
        L.orc_sim3_update.argtypes = [d, d, C.c_int, u8]
        L.orc_match.argtypes = [d, C.c_int, C.c_int, d, C.c_int, C.c_int, C.POINTER(MatchParams),
                                i32, d, d, i32]
        L.orc_mutual.argtypes = [i32, i32, C.c_int, C.c_int, C.c_int, C.c_int, d, d,
                                 C.POINTER(MatchParams), i32, u8, d]
        L.orc_gn_assemble.argtypes = [d, C.c_int, i64, i64, d, d, i32, i32, i64, C.c_int, i32, i32,
                                      C.c_int, C.POINTER(GNParams), d, d, d, i64, d, i64]
        L.orc_chol_ladder.argtypes = [d, d, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, d]
        L.orc_gn_step.argtypes = [d, C.c_int, i64, i64, d, d, i32, i32, i64, C.c_int, i32, i32,
                                  C.c_int, C.POINTER(GNParams), d, i32, d]
        L.orc_cost.argtypes = [d, C.c_int, i64, i64, d, d, i32, i32, i64, C.c_int, i32,
                               C.POINTER(GNParams)]
        L.orc_cost.restype = C.c_double
        L.orc_cost_grad.argtypes = [d, C.c_int, i64, i64, d, d, i32, i32, i64, C.c_int, i32,
                                    C.POINTER(GNParams), d, d, d, d]
        L.orc_edge_residuals.argtypes = [d, d, d, d, C.c_int64, d, d, C.c_int64, i32,
                                         C.POINTER(GNParams), d, d, u8]
        dd = C.c_double
        L.orc_gn_assemble_cal.argtypes = [d, C.c_int, i64, i64, i32, d, d, d, i32, i32, i64, C.c_int, i32, i32,
                                          C.c_int, C.POINTER(GNParams), dd, dd, d, d, d, i64, d, i64]
        L.orc_gn_step_cal.argtypes = [d, C.c_int, i64, i64, i32, d, d, d, i32, i32, i64, C.c_int, i32, i32,
                                      C.c_int, C.POINTER(GNParams), dd, dd, d, i32, d]
        L.orc_cost_cal.argtypes = [d, C.c_int, i64, i64, i32, d, d, d, i32, i32, i64, C.c_int, i32,
                                   C.POINTER(GNParams), dd, dd]
        L.orc_cost_cal.restype = C.c_double
        L.orc_edge_residuals_cal.argtypes = [d, d, d, d, C.c_int64, C.c_int, d, d, d, C.c_int64, C.c_int, d, i32,
                                             C.POINTER(GNParams), dd, dd, d, d, u8]
        _lib = L
    return _lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().orc_num_threads()


# ---------------------------------------------------------------------------------------------
# Sim(3) (Sec. III-A, III-D)
# ---------------------------------------------------------------------------------------------
def sim3_exp(tau) -> np.ndarray:
    """Exp(tau) as a pose vector: the matrix exponential of [[zeta I + [omega]x, v], [0, 0]]."""
    tau = _f64(tau).reshape(-1, 7)
    out = np.empty((tau.shape[0], 8))
    for k in range(tau.shape[0]):
        lib().orc_sim3_exp(_p(tau[k], C.c_double), _p(out[k], C.c_double))
    return out


def sim3_exp_mat(tau) -> np.ndarray:
    tau = _f64(tau).reshape(7)
    out = np.empty(16)
    lib().orc_sim3_exp_mat(_p(tau, C.c_double), _p(out, C.c_double))
    return out.reshape(4, 4)


def sim3_log(pose) -> np.ndarray:
    pose = _f64(pose).reshape(-1, 8)
    out = np.empty((pose.shape[0], 7))
    for k in range(pose.shape[0]):
        lib().orc_sim3_log(_p(pose[k], C.c_double), _p(out[k], C.c_double))
    return out


def pose_to_mat(pose) -> np.ndarray:
    pose = _f64(pose).reshape(8)
    out = np.empty(16)
    lib().orc_pose_to_mat(_p(pose, C.c_double), _p(out, C.c_double))
    return out.reshape(4, 4)


def mat_to_pose(M) -> np.ndarray:
    M = _f64(M).reshape(16)
    out = np.empty(8)
    lib().orc_mat_to_pose(_p(M, C.c_double), _p(out, C.c_double))
    return out


def sim3_adjoint(pose) -> np.ndarray:
    pose = _f64(pose).reshape(8)
    out = np.empty(49)
    lib().orc_sim3_adjoint(_p(pose, C.c_double), _p(out, C.c_double))
    return out.reshape(7, 7)


def relative(pi, pj) -> np.ndarray:
    """T_ij = T_i^-1 T_j (Sec. III-A)."""
    pi, pj, out = _f64(pi).reshape(8), _f64(pj).reshape(8), np.empty(8)
    lib().orc_relative(_p(pi, C.c_double), _p(pj, C.c_double), _p(out, C.c_double))
    return out


def sim3_update(poses, tau, fixed=None) -> np.ndarray:
    """T_k <- Exp(tau_k) T_k for every k not flagged in ``fixed`` (returns a new array)."""
    poses = _f64(poses).reshape(-1, 8).copy()
    tau = _f64(tau).reshape(-1, 7)
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    lib().orc_sim3_update(_p(poses, C.c_double), _p(tau, C.c_double), poses.shape[0],
                          None if fx is None else _p(fx, C.c_uint8))
    return poses


# ---------------------------------------------------------------------------------------------
# Matching (Sec. III-A "Learned geometry", Sec. III-B)
# ---------------------------------------------------------------------------------------------
@dataclass
class MatchResult:
    idx: np.ndarray          # int32, -1 invalid
    p: np.ndarray            # (n, 2) continuous optimum (u, v), NaN for queries with no optimum
    ratios: np.ndarray       # (n, 2) validity ratios (angular, range); valid iff both <= 1
    iters: np.ndarray        # int32 LM trial steps


def match(ref_xyz, qry_xyz, params: MatchParams | None = None) -> MatchResult:
    """One direction: queries (the other view's points in the reference camera) against the
    reference's canonical pointmap. Shapes (H, W, 3) and (Hq, Wq, 3)."""
    P = params or MatchParams.default()
    ref = _f64(ref_xyz)
    qry = _f64(qry_xyz)
    H, W = ref.shape[:2]
    Hq, Wq = qry.shape[:2]
    n = Hq * Wq
    idx = np.empty(n, np.int32)
    p = np.empty((n, 2))
    ratios = np.empty((n, 2))
    iters = np.empty(n, np.int32)
    rc = lib().orc_match(_p(ref, C.c_double), H, W, _p(qry, C.c_double), Hq, Wq, C.byref(P),
                         _p(idx, C.c_int32), _p(p, C.c_double), _p(ratios, C.c_double),
                         _p(iters, C.c_int32))
    if rc != 0:
        raise ValueError("oracle match: bad shapes")
    return MatchResult(idx, p, ratios, iters)


@dataclass
class BidirResult:
    idx_j2i: np.ndarray      # int32 per pixel of j, -1 where not mutually valid
    valid_j: np.ndarray      # uint8
    nu: np.ndarray           # [nu_i, nu_j]
    admit: bool
    fwd: MatchResult         # j -> i direction (queries = pixels of j)
    bwd: MatchResult         # i -> j direction (queries = pixels of i)


def mutual(idx_ji, idx_ij, shape_i, shape_j, conf_i, conf_j, params: MatchParams | None = None):
    P = params or MatchParams.default()
    Hi, Wi = shape_i
    Hj, Wj = shape_j
    a = np.ascontiguousarray(idx_ji, np.int32)
    b = np.ascontiguousarray(idx_ij, np.int32)
    ci, cj = _f64(conf_i).reshape(-1), _f64(conf_j).reshape(-1)
    out = np.empty(Hj * Wj, np.int32)
    valid = np.empty(Hj * Wj, np.uint8)
    nu = np.empty(2)
    admit = lib().orc_mutual(_p(a, C.c_int32), _p(b, C.c_int32), Hi, Wi, Hj, Wj,
                             _p(ci, C.c_double), _p(cj, C.c_double), C.byref(P),
                             _p(out, C.c_int32), _p(valid, C.c_uint8), _p(nu, C.c_double))
    return out, valid, nu, bool(admit)


def match_bidir(X_ii, X_ji, X_jj, X_ij, C_i, C_j, params: MatchParams | None = None) -> BidirResult:
    """Both decoded directions + mutual check + nu gate. X_ii, X_jj: canonical pointmaps;
    X_ji: j's points in camera i (H_j, W_j, 3); X_ij: i's points in camera j (H_i, W_i, 3)."""
    P = params or MatchParams.default()
    fwd = match(X_ii, X_ji, P)
    bwd = match(X_jj, X_ij, P)
    Hi, Wi = np.shape(X_ii)[:2]
    Hj, Wj = np.shape(X_jj)[:2]
    idx, valid, nu, admit = mutual(fwd.idx, bwd.idx, (Hi, Wi), (Hj, Wj), C_i, C_j, P)
    return BidirResult(idx, valid, nu, admit, fwd, bwd)


# ---------------------------------------------------------------------------------------------
# Graph step (eqs. 1, 5, 6, 7)
# ---------------------------------------------------------------------------------------------
class Graph:
    """Flat arrays the oracle's C entry points take: keyframe arenas (xyz, conf) with offsets,
    edges (i, j) with their idx offsets (idx has H_j*W_j entries per edge)."""

    def __init__(self, xyz_list, conf_list, edges, idx_list, anchors=(0,)):
        self.n_kf = len(xyz_list)
        npx = np.array([int(np.prod(np.shape(x)[:2])) for x in xyz_list], np.int64)
        # image width per keyframe (calibrated mode splits pixel indices into (u, v)); flat inputs: 0
        self.kf_w = np.array([int(np.shape(x)[1]) if np.ndim(x) == 3 else 0 for x in xyz_list], np.int32)
        self.kf_npx = npx
        self.kf_off = np.concatenate([[0], np.cumsum(npx)[:-1]]).astype(np.int64)
        self.xyz = np.ascontiguousarray(
            np.concatenate([_f64(x).reshape(-1, 3) for x in xyz_list]), np.float64)
        self.conf = np.ascontiguousarray(
            np.concatenate([_f64(c).reshape(-1) for c in conf_list]), np.float64)
        edges = np.asarray(edges, np.int64).reshape(-1, 2)
        self.ei = np.ascontiguousarray(edges[:, 0], np.int32)
        self.ej = np.ascontiguousarray(edges[:, 1], np.int32)
        self.n_edges = edges.shape[0]
        lens = np.array([np.size(a) for a in idx_list], np.int64)
        for e in range(self.n_edges):
            if lens[e] != npx[self.ej[e]]:
                raise ValueError(f"edge {e}: idx has {lens[e]} entries, keyframe j has {npx[self.ej[e]]}")
        self.idx_off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
        self.idx = np.ascontiguousarray(np.concatenate([np.asarray(a).reshape(-1) for a in idx_list]),
                                        np.int32) if self.n_edges else np.zeros(0, np.int32)
        self.anchors = np.ascontiguousarray(anchors, np.int32)

    def _common(self, poses):
        poses = _f64(poses).reshape(self.n_kf, 8)
        return (poses, self.n_kf, _p(self.kf_off, C.c_int64), _p(self.kf_npx, C.c_int64),
                _p(self.xyz, C.c_double), _p(self.conf, C.c_double), _p(self.ei, C.c_int32),
                _p(self.ej, C.c_int32), _p(self.idx_off, C.c_int64), self.n_edges,
                _p(self.idx, C.c_int32))


def gn_assemble(graph: Graph, poses, params: GNParams | None = None):
    """H (7N x 7N), g (7N), E at `poses`, valid count, per-edge cost and count."""
    P = params or GNParams.default()
    poses = _f64(poses).reshape(graph.n_kf, 8)
    n = 7 * graph.n_kf
    H = np.empty((n, n))
    g = np.empty(n)
    cost = C.c_double()
    count = C.c_int64()
    ec = np.empty(graph.n_edges)
    en = np.empty(graph.n_edges, np.int64)
    args = graph._common(poses)
    lib().orc_gn_assemble(_p(poses, C.c_double), *args[1:], _p(graph.anchors, C.c_int32),
                          len(graph.anchors), C.byref(P), _p(H, C.c_double), _p(g, C.c_double),
                          C.byref(cost), C.byref(count), _p(ec, C.c_double), _p(en, C.c_int64))
    return H, g, cost.value, count.value, ec, en


def chol_ladder(H, g, lam=0.0, eps0=1e-6, mult=100.0, attempts=6):
    """eq. (7) with the epsilon ladder: returns (tau, status); status = attempt used, -1 = zero step."""
    H = _f64(H)
    g = _f64(g).reshape(-1)
    n = g.shape[0]
    tau = np.empty(n)
    st = lib().orc_chol_ladder(_p(H, C.c_double), _p(g, C.c_double), n, lam, eps0, mult, attempts,
                               _p(tau, C.c_double))
    return tau, st


def gn_step(graph: Graph, poses, params: GNParams | None = None):
    """One GN/IRLS step; returns (new poses, cost at the input poses, status, tau)."""
    P = params or GNParams.default()
    poses = _f64(poses).reshape(graph.n_kf, 8).copy()
    cost = C.c_double()
    st = C.c_int32()
    tau = np.empty(7 * graph.n_kf)
    args = graph._common(poses)
    lib().orc_gn_step(_p(poses, C.c_double), *args[1:], _p(graph.anchors, C.c_int32),
                      len(graph.anchors), C.byref(P), C.byref(cost), C.byref(st),
                      _p(tau, C.c_double))
    return poses, cost.value, st.value, tau


def gn_solve(graph: Graph, poses, iters: int, params: GNParams | None = None):
    costs = []
    for _ in range(iters):
        poses, c, _, _ = gn_step(graph, poses, params)
        costs.append(c)
    return poses, costs


def cost(graph: Graph, poses, params: GNParams | None = None) -> float:
    P = params or GNParams.default()
    poses = _f64(poses).reshape(graph.n_kf, 8)
    args = graph._common(poses)
    return lib().orc_cost(_p(poses, C.c_double), *args[1:], C.byref(P))


def edge_residuals(graph: Graph, poses, e: int, params: GNParams | None = None):
    """Per pixel of j for edge e: whitened residuals r (npx_j, 4), IRLS weights w (npx_j, 4), ok mask."""
    P = params or GNParams.default()
    poses = _f64(poses).reshape(graph.n_kf, 8)
    i, j = int(graph.ei[e]), int(graph.ej[e])
    nj, ni = int(graph.kf_npx[j]), int(graph.kf_npx[i])
    r = np.empty((nj, 4))
    w = np.empty((nj, 4))
    ok = np.empty(nj, np.uint8)
    xj = graph.xyz[graph.kf_off[j]:graph.kf_off[j] + nj]
    xi = graph.xyz[graph.kf_off[i]:graph.kf_off[i] + ni]
    cj = graph.conf[graph.kf_off[j]:graph.kf_off[j] + nj]
    ci = graph.conf[graph.kf_off[i]:graph.kf_off[i] + ni]
    idx = graph.idx[graph.idx_off[e]:graph.idx_off[e] + nj]
    pi, pj = np.ascontiguousarray(poses[i]), np.ascontiguousarray(poses[j])
    lib().orc_edge_residuals(_p(pi, C.c_double), _p(pj, C.c_double), _p(xj, C.c_double),
                             _p(cj, C.c_double), nj, _p(xi, C.c_double), _p(ci, C.c_double), ni,
                             _p(idx, C.c_int32), C.byref(P), _p(r, C.c_double), _p(w, C.c_double),
                             _p(ok, C.c_uint8))
    return r, w, ok.astype(bool)


def cost_grad(graph: Graph, poses, params: GNParams | None = None):
    """(E, dE/dxyz (npx,3), dE/dconf (npx,), dE/dtau (N,7)) with matches held fixed."""
    P = params or GNParams.default()
    poses = _f64(poses).reshape(graph.n_kf, 8)
    gx = np.zeros_like(graph.xyz)
    gc = np.zeros_like(graph.conf)
    gt = np.zeros((graph.n_kf, 7))
    c = C.c_double()
    args = graph._common(poses)
    lib().orc_cost_grad(_p(poses, C.c_double), *args[1:], C.byref(P), _p(gx, C.c_double),
                        _p(gc, C.c_double), _p(gt, C.c_double), C.byref(c))
    return c.value, gx, gc, gt


# ---------------------------------------------------------------------------------------------
# Calibrated mode (Sec. IV-C, "Calibration"): pixel reprojection and log-depth residuals on the
# pointmaps constrained to the calibrated rays. See ds3_oracle.cpp for the readings.
# ---------------------------------------------------------------------------------------------
@dataclass
class Calib:
    """Supplied intrinsics K (n_kf x 4: fx, fy, cx, cy) and the whitening of the residual rows (the paper
    states no constants for this mode; readings: one pixel for the reprojection rows, 0.1 for log-depth)."""
    K: np.ndarray
    sigma_pix: float = 1.0
    sigma_logz: float = 0.1


def _cal_args(graph: Graph, calib: Calib):
    K = np.ascontiguousarray(np.asarray(calib.K, np.float64).reshape(graph.n_kf, 4))
    if np.any(graph.kf_w <= 0):
        raise ValueError("calibrated mode needs (H, W, 3) pointmaps (image widths)")
    return K


def gn_assemble_cal(graph: Graph, poses, calib: Calib, params: GNParams | None = None):
    """H (7N x 7N), g (7N), E, valid count, per-edge cost and count at `poses` in calibrated mode."""
    P = params or GNParams.default()
    poses = _f64(poses).reshape(graph.n_kf, 8)
    K = _cal_args(graph, calib)
    n = 7 * graph.n_kf
    H, g = np.empty((n, n)), np.empty(n)
    cost, count = C.c_double(), C.c_int64()
    ec, en = np.empty(graph.n_edges), np.empty(graph.n_edges, np.int64)
    lib().orc_gn_assemble_cal(_p(poses, C.c_double), graph.n_kf, _p(graph.kf_off, C.c_int64),
                              _p(graph.kf_npx, C.c_int64), _p(graph.kf_w, C.c_int32), _p(K, C.c_double),
                              _p(graph.xyz, C.c_double), _p(graph.conf, C.c_double), _p(graph.ei, C.c_int32),
                              _p(graph.ej, C.c_int32), _p(graph.idx_off, C.c_int64), graph.n_edges,
                              _p(graph.idx, C.c_int32), _p(graph.anchors, C.c_int32), len(graph.anchors),
                              C.byref(P), calib.sigma_pix, calib.sigma_logz, _p(H, C.c_double), _p(g, C.c_double),
                              C.byref(cost), C.byref(count), _p(ec, C.c_double), _p(en, C.c_int64))
    return H, g, cost.value, count.value, ec, en


def gn_step_cal(graph: Graph, poses, calib: Calib, params: GNParams | None = None):
    """One GN/IRLS step in calibrated mode; returns (new poses, cost at the input poses, status, tau)."""
    P = params or GNParams.default()
    poses = _f64(poses).reshape(graph.n_kf, 8).copy()
    K = _cal_args(graph, calib)
    cost, st = C.c_double(), C.c_int32()
    tau = np.empty(7 * graph.n_kf)
    lib().orc_gn_step_cal(_p(poses, C.c_double), graph.n_kf, _p(graph.kf_off, C.c_int64),
                          _p(graph.kf_npx, C.c_int64), _p(graph.kf_w, C.c_int32), _p(K, C.c_double),
                          _p(graph.xyz, C.c_double), _p(graph.conf, C.c_double), _p(graph.ei, C.c_int32),
                          _p(graph.ej, C.c_int32), _p(graph.idx_off, C.c_int64), graph.n_edges,
                          _p(graph.idx, C.c_int32), _p(graph.anchors, C.c_int32), len(graph.anchors), C.byref(P),
                          calib.sigma_pix, calib.sigma_logz, C.byref(cost), C.byref(st), _p(tau, C.c_double))
    return poses, cost.value, st.value, tau


def cost_cal(graph: Graph, poses, calib: Calib, params: GNParams | None = None) -> float:
    P = params or GNParams.default()
    poses = _f64(poses).reshape(graph.n_kf, 8)
    K = _cal_args(graph, calib)
    return lib().orc_cost_cal(_p(poses, C.c_double), graph.n_kf, _p(graph.kf_off, C.c_int64),
                              _p(graph.kf_npx, C.c_int64), _p(graph.kf_w, C.c_int32), _p(K, C.c_double),
                              _p(graph.xyz, C.c_double), _p(graph.conf, C.c_double), _p(graph.ei, C.c_int32),
                              _p(graph.ej, C.c_int32), _p(graph.idx_off, C.c_int64), graph.n_edges,
                              _p(graph.idx, C.c_int32), C.byref(P), calib.sigma_pix, calib.sigma_logz)


def edge_residuals_cal(graph: Graph, poses, e: int, calib: Calib, params: GNParams | None = None):
    """Per pixel of j for edge e in calibrated mode: whitened residuals r (npx_j, 3), IRLS weights w
    (npx_j, 3), ok mask."""
    P = params or GNParams.default()
    poses = _f64(poses).reshape(graph.n_kf, 8)
    K = _cal_args(graph, calib)
    i, j = int(graph.ei[e]), int(graph.ej[e])
    nj, ni = int(graph.kf_npx[j]), int(graph.kf_npx[i])
    r, w, ok = np.empty((nj, 3)), np.empty((nj, 3)), np.empty(nj, np.uint8)
    sl = lambda a, k, n, c=1: np.ascontiguousarray(a[graph.kf_off[k] * c:(graph.kf_off[k] + n) * c])
    xj, xi = sl(graph.xyz.reshape(-1), j, nj, 3), sl(graph.xyz.reshape(-1), i, ni, 3)
    cj, ci = sl(graph.conf, j, nj), sl(graph.conf, i, ni)
    idx = np.ascontiguousarray(graph.idx[graph.idx_off[e]:graph.idx_off[e] + nj])
    pi, pj = np.ascontiguousarray(poses[i]), np.ascontiguousarray(poses[j])
    Kj, Ki = np.ascontiguousarray(K[j]), np.ascontiguousarray(K[i])
    lib().orc_edge_residuals_cal(_p(pi, C.c_double), _p(pj, C.c_double), _p(xj, C.c_double), _p(cj, C.c_double), nj,
                                 int(graph.kf_w[j]), _p(Kj, C.c_double), _p(xi, C.c_double), _p(ci, C.c_double), ni,
                                 int(graph.kf_w[i]), _p(Ki, C.c_double), _p(idx, C.c_int32), C.byref(P),
                                 calib.sigma_pix, calib.sigma_logz, _p(r, C.c_double), _p(w, C.c_double),
                                 _p(ok, C.c_uint8))
    return r, w, ok.astype(bool)


# ---------------------------------------------------------------------------------------------
# Gauge synchronisation (Sec. III-C, eqs. 3-4)
# ---------------------------------------------------------------------------------------------
def umeyama(x, y):
    """Closed form of eq. (4): (s, R, t) minimising sum |x - (s R y + t)|^2. Returns a pose vector,
    or None when the cross-covariance has rank < 2 (collinear or coincident points)."""
    x = _f64(x).reshape(-1, 3)
    y = _f64(y).reshape(-1, 3)
    n = x.shape[0]
    xb, yb = x.mean(0), y.mean(0)
    xt, yt = x - xb, y - yb
    A = xt.T @ yt / n
    U, lam, Vt = np.linalg.svd(A)
    if lam[1] <= 1e-12 * max(lam[0], 1e-300):
        return None
    S = np.diag([1.0, 1.0, np.sign(np.linalg.det(U @ Vt)) or 1.0])
    R = U @ S @ Vt
    s = np.trace(np.diag(lam) @ S) / ((yt * yt).sum() / n)
    t = xb - s * R @ yb
    M = np.eye(4)
    M[:3, :3] = s * R
    M[:3, 3] = t
    return mat_to_pose(M)


def compose(pa, pb) -> np.ndarray:
    return mat_to_pose(pose_to_mat(pa) @ pose_to_mat(pb))


def invert(p) -> np.ndarray:
    return mat_to_pose(np.linalg.inv(pose_to_mat(p)))


def transform_points(pose, X) -> np.ndarray:
    M = pose_to_mat(pose)
    X = _f64(X).reshape(-1, 3)
    return X @ M[:3, :3].T + M[:3, 3]


def fuse(canon, pred, pairs, poses) -> np.ndarray:
    """Confidence-weighted running average of eq. (2) (Sec. III-A), applied pair by pair in order.

    canon: (N, 4) xyz + confidence of the canonical keyframe pointmaps (X-hat, C-hat); pred: (M, 4) the
    registered predictions, pixel-aligned with their keyframe and expressed in the frame's camera, with
    their confidence C; pairs: rows (canon_off, pred_off, n_px); poses: one pose per pair, T_kf mapping
    the frame into the keyframe. For pixel m of a pair, with y = T_kf x:
        X-hat <- (C-hat X-hat + C y) / (C-hat + C),   C-hat <- C-hat + C.
    A pixel whose prediction is not finite, or whose summed confidence is not positive, is left as it
    is. Returns the updated copy of canon (float64)."""
    out = _f64(canon).reshape(-1, 4).copy()
    P = _f64(pred).reshape(-1, 4)
    for (co, po, n), pose in zip(np.asarray(pairs, dtype=np.int64).reshape(-1, 3), np.asarray(poses).reshape(-1, 8)):
        x = P[po:po + n]
        c_new = x[:, 3]
        c_old = out[co:co + n, 3]
        tot = c_old + c_new
        ok = np.isfinite(x).all(axis=1) & (tot > 0)
        with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
            y = transform_points(pose, x[:, :3])
            avg = (c_old[:, None] * out[co:co + n, :3] + c_new[:, None] * y) / tot[:, None]
        out[co:co + n, :3] = np.where(ok[:, None], avg, out[co:co + n, :3])
        out[co:co + n, 3] = np.where(ok, tot, c_old)
    return out


@dataclass
class GaugeLink:
    edge: int
    ref_agent_comp: int
    moved_agents: list
    T_star: np.ndarray
    n_corr: int
    used_umeyama: bool


def gauge_sync(poses, agent_of_kf, edges, admitted, matches, xyz_list, nc_min=64):
    """Component tracker of Sec. III-C. Walks admitted inter-agent edges in order; each edge that joins
    two components moves one of them by T* (Umeyama on its matches lifted to world frames, or the
    endpoint transform T_ref T_mov^-1 below nc_min correspondences). Reference: the component holding
    agent 0, otherwise the one whose smallest agent id is smallest. `matches[e]` is (idx_j2i, valid_j).
    Returns (new poses, list of GaugeLink)."""
    poses = _f64(poses).reshape(-1, 8).copy()
    agent_of_kf = np.asarray(agent_of_kf)
    n_agents = int(agent_of_kf.max()) + 1
    comp = list(range(n_agents))  # component label of each agent = smallest agent id in it
    links = []
    for e, (i, j) in enumerate(np.asarray(edges).reshape(-1, 2)):
        i, j = int(i), int(j)
        ai, aj = int(agent_of_kf[i]), int(agent_of_kf[j])
        if ai == aj or not admitted[e] or comp[ai] == comp[aj]:
            continue
        ref_is_i = comp[ai] < comp[aj]
        ref_c, mov_c = (comp[ai], comp[aj]) if ref_is_i else (comp[aj], comp[ai])
        idx_j2i, valid_j = matches[e]
        sel = np.nonzero(np.asarray(valid_j).reshape(-1) != 0)[0]
        m = np.asarray(idx_j2i).reshape(-1)[sel]
        wi = transform_points(poses[i], _f64(xyz_list[i]).reshape(-1, 3)[m])
        wj = transform_points(poses[j], _f64(xyz_list[j]).reshape(-1, 3)[sel])
        ref_kf, mov_kf = (i, j) if ref_is_i else (j, i)
        x, y = (wi, wj) if ref_is_i else (wj, wi)
        T = umeyama(x, y) if len(sel) >= nc_min else None
        used = T is not None
        if T is None:
            T = compose(poses[ref_kf], invert(poses[mov_kf]))
        moved = [a for a in range(n_agents) if comp[a] == mov_c]
        for k in np.nonzero(np.isin(agent_of_kf, moved))[0]:
            poses[k] = compose(T, poses[k])
        for a in moved:
            comp[a] = ref_c
        links.append(GaugeLink(e, ref_c, moved, T, int(len(sel)), used))
    return poses, links


# ---------------------------------------------------------------------------------------------
# Ray-range tracking (Sec. III-A): one free pose T_kf under the residual of eq. (1) and LM damping
# ---------------------------------------------------------------------------------------------
@dataclass
class TrackParams:
    """LM schedule of the tracker. The paper states only that the tracker uses LM damping (text after
    eq. 7, the lambda diag(H) term); the schedule is a reading: lambda0 = 1e-4, divided by 10 after an
    accepted trial (floor lambda_min) and multiplied by 10 after a rejected one, at most max_trials
    trial steps, stop after an accepted step whose largest tangent component is below step_tol."""
    lambda0: float = 1e-4
    lambda_min: float = 1e-9
    lambda_up: float = 10.0
    lambda_down: float = 0.1
    max_trials: int = 20
    step_tol: float = 1e-7


@dataclass
class TrackResult:
    pose: np.ndarray       # T_kf after the search (8)
    cost: float            # E_track at that pose
    trials: int            # trial steps taken
    costs: list = field(default_factory=list)    # E_track after each trial step (the kept pose's)
    lambdas: list = field(default_factory=list)  # damping used by each trial step
    accepted: list = field(default_factory=list)


def track(xyz_kf, conf_kf, xyz_fr, conf_fr, idx, T0, params: GNParams | None = None,
          tp: TrackParams | None = None) -> TrackResult:
    """E_track(T_kf) = sum over the matches (m, n) of sum_c rho([Sigma_mn^-1/2 e_mn(T_kf)]_c) with e of
    eq. (1) between the keyframe's canonical point X_k[m] and the frame's point X_f[n] (idx[n] = m, -1 =
    no match), minimised over T_kf (frame -> keyframe) by LM: at the kept pose T with normal equations
    H, g (the IRLS linearisation of eqs. 5-6 restricted to one edge with the keyframe fixed at the
    identity), a trial step solves (H + lambda diag H + eps_r I) tau = -g (eq. 7 with the epsilon ladder)
    and T' = Exp(tau) T (left update, Sec. III-D); the trial is accepted iff E_track(T') < E_track(T)."""
    P = params or GNParams.default()
    tp = tp or TrackParams()
    ident = np.array([0, 0, 0, 0, 0, 0, 1, 1.0])
    g = Graph([xyz_kf, xyz_fr], [conf_kf, conf_fr], [(0, 1)], [np.asarray(idx).reshape(-1)], anchors=(0,))

    def linearise(T):
        H, gv, E, *_ = gn_assemble(g, np.stack([ident, T]), P)
        return H[7:, 7:].copy(), gv[7:].copy(), E

    T = _f64(T0).reshape(8).copy()
    H, b, E = linearise(T)
    lam = tp.lambda0
    res = TrackResult(T, E, 0)
    for _ in range(tp.max_trials):
        res.trials += 1
        res.lambdas.append(lam)
        tau, _ = chol_ladder(H, b, lam, P.eps0, P.eps_mult, P.max_attempts)
        T1 = sim3_update(T[None], tau[None])[0]
        H1, b1, E1 = linearise(T1)
        if E1 < E:
            T, H, b, E = T1, H1, b1, E1
            lam = max(lam * tp.lambda_down, tp.lambda_min)
            res.accepted.append(True)
            res.costs.append(E)
            if np.abs(tau).max() < tp.step_tol:
                break
        else:
            lam = lam * tp.lambda_up
            res.accepted.append(False)
            res.costs.append(E)
    res.pose, res.cost = T, E
    return res


# ---------------------------------------------------------------------------------------------
# Precision helpers and metrics
# ---------------------------------------------------------------------------------------------
def bf16_round(a) -> np.ndarray:
    """FP32 -> BF16 with round-to-nearest, ties to even (plain bit definition), returned as uint16.
    NaN inputs map to a quiet NaN."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(a)
    r[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return r


def bf16_to_f32(b) -> np.ndarray:
    b = np.ascontiguousarray(b, np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)


def pose_error(p, p_ref) -> np.ndarray:
    """Per keyframe: max(rotation angle of R R_ref^T, |t - t_ref| / max(|t_ref|, 1 m), |s/s_ref - 1|)."""
    p = _f64(p).reshape(-1, 8)
    p_ref = _f64(p_ref).reshape(-1, 8)
    out = np.empty(p.shape[0])
    for k in range(p.shape[0]):
        q = p[k, 3:7] / np.linalg.norm(p[k, 3:7])
        r = p_ref[k, 3:7] / np.linalg.norm(p_ref[k, 3:7])
        # relative rotation q * conj(r): angle = 2 atan2(|vec|, |w|)
        w = q[3] * r[3] + q[:3] @ r[:3]
        v = r[3] * q[:3] - q[3] * r[:3] - np.cross(q[:3], r[:3])
        ang = 2.0 * np.arctan2(np.linalg.norm(v), abs(w))
        dt = np.linalg.norm(p[k, :3] - p_ref[k, :3]) / max(np.linalg.norm(p_ref[k, :3]), 1.0)
        ds = abs(p[k, 7] / p_ref[k, 7] - 1)
        out[k] = max(ang, dt, ds)
    return out
