"""FP64 oracle of the terminal segment-level depth refinement (CoMo3R-SLAM, Sec. III-E, eqs. (8)-(10)).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): plain numpy, FP64 for the real-valued parts and
exact int64 arithmetic for the segmentation. It shares no code with the HIP path.

What it computes, in the paper's order:
  1. per keyframe, SLIC over canonical surface normals and normalised log-range (about M_k = 200 segments),
     pixels with confidence below C_min = 1.5 excluded, segments with fewer than 16 valid pixels excluded;
  2. the parameterisation of eq. (8): the corrected point of pixel p in segment g is its pristine point
     scaled by exp(eta_g) (|X_init| exp(eta_g) psi(X_init) = X_init exp(eta_g));
  3. the point residual of eq. (9) over the graph's matches, whitened by sqrt(q)/sigma_point, Huber rho;
  4. the boundary and prior terms of eq. (10);
  5. Jacobi-style damped Newton steps: each segment's 1x1 normal equation from the diagonal blocks of the
     data term (J_g = -X_i(eta), J_h = s_ij R_ij X_j(eta), both whitened) and of the boundary term, the
     prior's lambda_prior, the full gradient, damping lambda_lm and a clip at eta_max; anchor-keyframe
     segments stay fixed.

Readings where the paper is silent (listed in the design notes):
  * normals: cross product of central differences along u and v (one-sided at the border), unit length,
    oriented towards the camera (n . X <= 0); zero if any pixel used is a hole or the product vanishes;
  * normalised log-range: (ln|X| - min) / (max - min) over the keyframe's valid pixels;
  * SLIC in exact integer arithmetic so that labels are reproducible: features quantised as
    round(1024 (n + 1)) (three channels) and round(1024 l); grid interval S = round(sqrt(HW / M_k)); one
    centre per grid cell at (min(c_x S + S // 2, W - 1), min(c_y S + S // 2, H - 1)) with that pixel's
    features; distance D = S^2 |F_p - F_c|^2 + 512^2 |xy_p - xy_c|^2 (compactness: a spatial offset of S
    weighs like half a unit of feature); each valid pixel compares the centres of the 3x3 grid cells around
    its own (ties: lowest centre index); centres move to the floor of their members' mean position and
    features; 10 iterations; no connectivity enforcement;
  * boundary pairs: 4-adjacent pixels of two valid segments; Delta_gh = mean over those pixel pairs of
    ln|X(p)| - ln|X(p')| with p in g, p' in h;
  * objective minimised: E' = sum rho(r) + (lambda_smooth/2) sum_B r_b^2 + (lambda_prior/2) sum eta^2
    (the normal-equation convention under which H_prior = lambda_prior I, as printed); damping
    (1 + lambda_lm) H (Marquardt, as eq. (7)'s lambda diag H); every call runs `iters` iterations; the
    Huber kappa is the pose cost's 1.345.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

Q = 1024          # feature quantisation
SPATIAL_W = 512   # compactness: quantised feature units per grid interval


@dataclass
class DepthParams:
    segments_per_kf: int = 200   # M_k
    conf_min: float = 1.5        # C_min^SLIC
    min_seg_px: int = 16
    slic_iters: int = 10
    sigma_point: float = 0.05
    huber_k: float = 1.345
    lambda_smooth: float = 1.0
    lambda_prior: float = 1.0
    lambda_lm: float = 0.05
    eta_max: float = 0.5


# ------------------------------------------------------------------------------------------------
# Features (Sec. III-E: canonical surface normals and normalised log-range)
# ------------------------------------------------------------------------------------------------
def valid_mask(X, C, conf_min):
    X = np.asarray(X, np.float64)
    n = np.sqrt((X * X).sum(-1))
    return np.isfinite(X).all(-1) & (n > 1e-9) & (np.asarray(C, np.float64) >= conf_min)


def normals(X):
    """(H, W, 3) FP64 unit normals, oriented towards the camera; zero where undefined."""
    X = np.asarray(X, np.float64)
    H, W, _ = X.shape
    hole = ~(np.isfinite(X).all(-1) & (np.sqrt((X * X).sum(-1)) > 1e-9))
    Xs = np.where(hole[..., None], 0.0, X)
    iu0 = np.clip(np.arange(W) - 1, 0, W - 1)
    iu1 = np.clip(np.arange(W) + 1, 0, W - 1)
    iv0 = np.clip(np.arange(H) - 1, 0, H - 1)
    iv1 = np.clip(np.arange(H) + 1, 0, H - 1)
    du = Xs[:, iu1] - Xs[:, iu0]
    dv = Xs[iv1] - Xs[iv0]
    bad = hole[:, iu1] | hole[:, iu0] | hole[iv1] | hole[iv0] | hole
    c = np.stack([du[..., 1] * dv[..., 2] - du[..., 2] * dv[..., 1],
                  du[..., 2] * dv[..., 0] - du[..., 0] * dv[..., 2],
                  du[..., 0] * dv[..., 1] - du[..., 1] * dv[..., 0]], -1)
    ln = np.sqrt((c[..., 0] * c[..., 0] + c[..., 1] * c[..., 1]) + c[..., 2] * c[..., 2])
    ok = ~bad & (ln > 0) & np.isfinite(ln)
    n = np.where(ok[..., None], c / np.where(ok, ln, 1.0)[..., None], 0.0)
    facing = (n * Xs).sum(-1) > 0
    return np.where(facing[..., None], -n, n)


def features(X, C, conf_min=1.5):
    """Quantised SLIC features (H, W, 4) int64 and the valid mask: round(Q (n + 1)), round(Q l)."""
    X = np.asarray(X, np.float64)
    valid = valid_mask(X, C, conf_min)
    n = normals(X)
    L = np.log(np.sqrt((np.where(np.isfinite(X), X, 0.0) ** 2).sum(-1)).clip(1e-300))
    if valid.any():
        lo, hi = L[valid].min(), L[valid].max()
        ell = (L - lo) / (hi - lo) if hi > lo else np.zeros_like(L)
    else:
        ell = np.zeros_like(L)
    F = np.empty(X.shape[:2] + (4,), np.int64)
    F[..., :3] = np.floor(Q * (n + 1.0) + 0.5).astype(np.int64)
    F[..., 3] = np.floor(Q * ell + 0.5).astype(np.int64)
    F[~valid] = 0
    return F, valid


# ------------------------------------------------------------------------------------------------
# SLIC in integer arithmetic
# ------------------------------------------------------------------------------------------------
def grid(H, W, M):
    S = max(1, int(np.floor(np.sqrt(H * W / M) + 0.5)))
    return S, -(-W // S), -(-H // S)


def slic(F, valid, M, iters=10):
    """Labels (H, W) int64 in [0, nx ny) or -1 for invalid pixels, and the centres after the last
    update ((nx ny, 6) int64: x, y, F0..F3)."""
    H, W, _ = F.shape
    S, nx, ny = grid(H, W, M)
    cy, cx = np.divmod(np.arange(nx * ny), nx)
    px = np.minimum(cx * S + S // 2, W - 1)
    py = np.minimum(cy * S + S // 2, H - 1)
    cen = np.concatenate([px[:, None], py[:, None], F[py, px]], 1).astype(np.int64)
    v, u = np.mgrid[0:H, 0:W]
    gx = np.minimum(u // S, nx - 1)
    gy = np.minimum(v // S, ny - 1)
    big = np.iinfo(np.int64).max
    labels = np.full((H, W), -1, np.int64)
    for _ in range(iters):
        best = np.full((H, W), big, np.int64)
        lab = np.full((H, W), -1, np.int64)
        for dy in (-1, 0, 1):                 # candidate order = increasing centre index
            for dx in (-1, 0, 1):
                ccx, ccy = gx + dx, gy + dy
                inside = (ccx >= 0) & (ccx < nx) & (ccy >= 0) & (ccy < ny)
                c = np.where(inside, ccy * nx + ccx, 0)
                dF = F - cen[c][..., 2:]
                d = S * S * (dF * dF).sum(-1) + SPATIAL_W ** 2 * ((u - cen[c][..., 0]) ** 2 +
                                                                  (v - cen[c][..., 1]) ** 2)
                take = inside & valid & (d < best)
                best = np.where(take, d, best)
                lab = np.where(take, c, lab)
        labels = lab
        m = labels >= 0
        cnt = np.bincount(labels[m], minlength=nx * ny)
        sums = np.zeros((nx * ny, 6), np.int64)
        vals = [u[m], v[m]] + [F[..., k][m] for k in range(4)]
        for k, a in enumerate(vals):
            np.add.at(sums[:, k], labels[m], a.astype(np.int64))   # exact integer sums
        upd = cnt > 0
        cen[upd] = sums[upd] // cnt[upd, None]
    return labels, cen


def segment(X, C, params: DepthParams | None = None):
    """Labels of one keyframe after excluding segments with fewer than min_seg_px pixels, and the
    number of grid centres (segment slots) of the keyframe."""
    P = params or DepthParams()
    F, valid = features(X, C, P.conf_min)
    H, W = F.shape[:2]
    labels, _ = slic(F, valid, P.segments_per_kf, P.slic_iters)
    S, nx, ny = grid(H, W, P.segments_per_kf)
    cnt = np.bincount(labels[labels >= 0], minlength=nx * ny)
    small = cnt < P.min_seg_px
    labels = np.where((labels >= 0) & small[np.maximum(labels, 0)], -1, labels)
    return labels, nx * ny


# ------------------------------------------------------------------------------------------------
# Boundary pairs and Delta_gh (eq. 10)
# ------------------------------------------------------------------------------------------------
def boundary(X, labels):
    """{(g, h): (sum of ln|X(p)| - ln|X(p')| over 4-adjacent pixel pairs p in g, p' in h, count)} over
    ordered pairs (both orientations), local segment ids; sums in pixel order (rows, then columns)."""
    X = np.asarray(X, np.float64)
    L = np.log(np.sqrt((np.where(np.isfinite(X), X, 0.0) ** 2).sum(-1)).clip(1e-300))
    H, W = labels.shape
    gs, hs, ds = [], [], []
    for (a, b) in (((slice(None), slice(0, W - 1)), (slice(None), slice(1, W))),
                   ((slice(0, H - 1), slice(None)), (slice(1, H), slice(None)))):
        g, h = labels[a].ravel(), labels[b].ravel()
        d = (L[a] - L[b]).ravel()
        sel = (g >= 0) & (h >= 0) & (g != h)
        gs += [g[sel], h[sel]]
        hs += [h[sel], g[sel]]
        ds += [d[sel], -d[sel]]
    g, h, d = np.concatenate(gs), np.concatenate(hs), np.concatenate(ds)
    M = int(labels.max()) + 1 if labels.size else 1
    key = g * M + h
    uk, inv = np.unique(key, return_inverse=True)
    s = np.bincount(inv, weights=d, minlength=len(uk))
    c = np.bincount(inv, minlength=len(uk))
    return {(int(k // M), int(k % M)): (float(sv), int(cv)) for k, sv, cv in zip(uk, s, c)}


# ------------------------------------------------------------------------------------------------
# The refinement (eqs. 8-10) over a graph
# ------------------------------------------------------------------------------------------------
class DepthProblem:
    """Keyframes (pristine pointmaps, confidences), edges (i, j) with their matches (idx over j's pixels),
    anchor keyframes; segmentation and boundary tables built at construction."""

    def __init__(self, xyz_list, conf_list, edges, idx_list, anchors=(0,), params: DepthParams | None = None,
                 labels=None):
        """labels (tests only): per keyframe (labels (H, W) with -1 for excluded pixels, number of segment
        slots) used instead of segmenting the given pointmaps."""
        self.P = params or DepthParams()
        self.X = [np.asarray(x, np.float64) for x in xyz_list]
        self.C = [np.asarray(c, np.float64) for c in conf_list]
        self.edges = [(int(i), int(j)) for i, j in edges]
        self.idx = [np.asarray(v, np.int64).reshape(-1) for v in idx_list]
        self.anchors = set(int(a) for a in anchors)
        self.labels, self.base = [], []
        off = 0
        for k, (X, C) in enumerate(zip(self.X, self.C)):
            lab, m = segment(X, C, self.P) if labels is None else (np.asarray(labels[k][0], np.int64), labels[k][1])
            self.labels.append(lab)
            self.base.append(off)
            off += m
        self.n_seg = off
        self.seg_valid = np.zeros(off, bool)
        self.seg_kf = np.zeros(off, np.int64)
        for k, lab in enumerate(self.labels):
            self.seg_valid[self.base[k] + lab[lab >= 0]] = True
            m = (self.base[k + 1] if k + 1 < len(self.base) else off) - self.base[k]
            self.seg_kf[self.base[k]:self.base[k] + m] = k
        self.free = self.seg_valid & ~np.isin(self.seg_kf, list(self.anchors))
        # boundary pairs with global ids: {(g, h): Delta_gh}, both orientations
        self.pairs = {}
        for k, (X, lab) in enumerate(zip(self.X, self.labels)):
            for (g, h), (s, c) in boundary(X, lab).items():
                self.pairs[(self.base[k] + g, self.base[k] + h)] = s / c

    def glabel(self, k):
        lab = self.labels[k].reshape(-1)
        return np.where(lab >= 0, self.base[k] + lab, -1)

    def residuals(self, poses, eta):
        """Per edge, over its usable matches: whitened residuals r (n, 3) of eq. (9) at eta, the segment of
        each endpoint (global id, -1 if excluded), and the Jacobians d r / d eta_h, d r / d eta_g."""
        P = self.P
        import oracle as O
        out = []
        for e, (i, j) in enumerate(self.edges):
            T = O.pose_to_mat(O.relative(poses[i], poses[j]))
            sR, t = T[:3, :3], T[:3, 3]
            idx = self.idx[e]
            n = np.flatnonzero((idx >= 0) & (idx < self.X[i].shape[0] * self.X[i].shape[1]))
            m = idx[n]
            Xj = self.X[j].reshape(-1, 3)[n]
            Xi = self.X[i].reshape(-1, 3)[m]
            Cj = self.C[j].reshape(-1)[n]
            Ci = self.C[i].reshape(-1)[m]
            ok = (np.isfinite(Xj).all(1) & np.isfinite(Xi).all(1) & (np.sqrt((Xj * Xj).sum(1)) > 1e-9) &
                  (np.sqrt((Xi * Xi).sum(1)) > 1e-9) & np.isfinite(Ci) & np.isfinite(Cj))
            n, m, Xj, Xi, Cj, Ci = n[ok], m[ok], Xj[ok], Xi[ok], Cj[ok], Ci[ok]
            h = self.glabel(j)[n]
            g = self.glabel(i)[m]
            eh = np.where(h >= 0, eta[np.maximum(h, 0)], 0.0)
            eg = np.where(g >= 0, eta[np.maximum(g, 0)], 0.0)
            Xj_e = Xj * np.exp(eh)[:, None]                     # eq. (8)
            Xi_e = Xi * np.exp(eg)[:, None]
            s = np.sqrt(np.sqrt(Ci * Cj)) / P.sigma_point       # sqrt(q) / sigma_point
            x = Xj_e @ sR.T + t
            r = s[:, None] * (x - Xi_e)                         # eq. (9) residual, whitened
            Jh = s[:, None] * (Xj_e @ sR.T)                     # d r / d eta_h
            Jg = -s[:, None] * Xi_e                             # d r / d eta_g
            out.append((r, h, g, Jh, Jg))
        return out

    def linearise(self, poses, eta):
        """E' at eta and, per segment, the diagonal H and the gradient g of the Jacobi step."""
        P = self.P
        Hd = np.zeros(self.n_seg)
        gd = np.zeros(self.n_seg)
        E = 0.0
        for r, h, g, Jh, Jg in self.residuals(poses, eta):
            a = np.abs(r)
            E += np.where(a <= P.huber_k, 0.5 * r * r, P.huber_k * a - 0.5 * P.huber_k ** 2).sum()
            w = np.where(a <= P.huber_k, 1.0, P.huber_k / np.where(a > 0, a, 1.0))
            for seg, J in ((h, Jh), (g, Jg)):
                sel = seg >= 0
                np.add.at(Hd, seg[sel], (w * J * J).sum(1)[sel])
                np.add.at(gd, seg[sel], (w * J * r).sum(1)[sel])
        H = Hd + P.lambda_prior
        grad = gd + P.lambda_prior * eta
        E += 0.5 * P.lambda_prior * (eta[self.seg_valid] ** 2).sum()
        for (g, h), dlt in self.pairs.items():
            rb = eta[g] - eta[h] + dlt
            H[g] += P.lambda_smooth
            grad[g] += P.lambda_smooth * rb
            if g < h:
                E += 0.5 * P.lambda_smooth * rb * rb
        return E, H, grad

    def step(self, poses, eta):
        """One Jacobi damped Newton step; returns (new eta, E' at the input eta)."""
        P = self.P
        E, H, grad = self.linearise(poses, eta)
        d = np.clip(-grad / ((1.0 + P.lambda_lm) * H), -P.eta_max, P.eta_max)
        return np.where(self.free, eta + d, eta), E

    def run(self, poses, eta=None, iters=10):
        eta = np.zeros(self.n_seg) if eta is None else np.asarray(eta, np.float64).copy()
        costs = []
        for _ in range(iters):
            eta, E = self.step(poses, eta)
            costs.append(E)
        return eta, costs

    def apply(self, eta):
        """The corrected pointmaps X_init exp(eta_g) (excluded pixels unchanged)."""
        out = []
        for k, X in enumerate(self.X):
            gl = self.glabel(k).reshape(X.shape[:2])
            f = np.where(gl >= 0, np.exp(eta[np.maximum(gl, 0)]), 1.0)
            out.append(X * f[..., None])
        return out
