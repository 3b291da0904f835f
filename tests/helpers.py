"""Shared test-side constructions (inputs only; no method arithmetic)."""
import math

import numpy as np

import synth


def exact_graph(n_kf=3, H=12, W=16, seed=0, edges=None, frac_valid=0.8):
    """Keyframes whose pointmaps are permuted views of ONE set of world points, so that every match
    is exact: keyframe k holds T_k^-1 P[p] at pixel pi_k(p). Edge (i, j) maps pixel n of j to
    pi_i(pi_j^-1(n)); a random subset is dropped. Residuals of eq. (1) vanish at the true poses."""
    rng = np.random.default_rng(seed)
    npx = H * W
    P = rng.uniform(-4, 4, size=(npx, 3)) + np.array([0.0, 0.0, 10.0])
    poses = []
    for k in range(n_kf):
        if k == 0:
            R, t, s = np.eye(3), np.zeros(3), 1.0
        else:
            R = synth.axis_angle(rng.normal(size=3), rng.uniform(0.05, 0.4))
            t = rng.normal(size=3) * 0.7
            s = math.exp(rng.uniform(-0.3, 0.3))
        poses.append(synth.pose_vec(R, t, s))
    poses = np.stack(poses)
    perms = [rng.permutation(npx) for _ in range(n_kf)]
    xyz = []
    for k in range(n_kf):
        R, t, s = synth.pose_parts(poses[k])
        Xc = (P - t) @ R / s
        X = np.empty_like(Xc)
        X[perms[k]] = Xc
        xyz.append(X.reshape(H, W, 3))
    conf = [rng.uniform(1, 5, size=(H, W)) for _ in range(n_kf)]
    if edges is None:
        edges = [(k, k + 1) for k in range(n_kf - 1)] + ([(0, n_kf - 1)] if n_kf > 2 else [])
    idx = []
    for i, j in edges:
        inv_j = np.empty(npx, np.int64)
        inv_j[perms[j]] = np.arange(npx)
        m = perms[i][inv_j]
        keep = rng.uniform(size=npx) < frac_valid
        idx.append(np.where(keep, m, -1).astype(np.int32))
    return xyz, conf, np.array(edges, np.int64), idx, poses


def perturb(poses, rng, rot=0.02, trans=0.05, scale=0.02, fixed=(0,)):
    out = poses.copy()
    for k in range(len(poses)):
        if k in fixed:
            continue
        R, t, s = synth.pose_parts(poses[k])
        w = rng.normal(size=3) * rot
        Rn = synth.axis_angle(w, np.linalg.norm(w))
        out[k] = synth.pose_vec(Rn @ R, t + rng.normal(size=3) * trans, s * math.exp(rng.normal() * scale))
    return out


# ------------------------------------------------------------------------------------------------
# Scale-aware comparisons: the entries of H, g and the gradients span many orders of magnitude (the ray
# rows are weighted by 1/sigma_r^2 = 1.1e5, the range row by 1/sigma_d^2 = 0.01), so each part is
# compared against its own magnitude, never against the largest entry of the whole array.
# ------------------------------------------------------------------------------------------------
def jacobi_scaled_err(H, H_ref):
    """max_ab |H - H_ref|_ab / sqrt(H_ref_aa H_ref_bb): the difference of D^-1/2 H D^-1/2 with
    D = diag(H_ref), so that every row and column (ray, range, scale) is measured in its own units."""
    H, H_ref = np.asarray(H, np.float64), np.asarray(H_ref, np.float64)
    d = np.sqrt(np.abs(np.diag(H_ref)))
    s = np.outer(d, d)
    ok = s > 0
    return float((np.abs(H - H_ref)[ok] / s[ok]).max())


def block_rel_err(H, H_ref, b=7):
    """Largest relative difference over the nonzero b x b blocks, each against its own largest entry."""
    H, H_ref = np.asarray(H, np.float64), np.asarray(H_ref, np.float64)
    n = H.shape[0] // b
    worst = 0.0
    for r in range(n):
        for c in range(n):
            B = H_ref[r * b:(r + 1) * b, c * b:(c + 1) * b]
            m = np.abs(B).max()
            if m > 0:
                worst = max(worst, float(np.abs(H[r * b:(r + 1) * b, c * b:(c + 1) * b] - B).max() / m))
    return worst


TANGENT_GROUPS = ((0, 3), (3, 6), (6, 7))  # v, omega, zeta


def tangent_group_err(g, g_ref, floor=1e-3):
    """Per keyframe and per tangent group (translation, rotation, scale) of (N, 7) gradients: the largest
    relative difference, each group against its own largest entry (groups that are exactly zero in the
    reference, such as an anchor's, must be zero).

    A keyframe's group can be a cancellation residue: the pose gradients of a graph sum to zero (gauge
    invariance of E), so one keyframe's scale entry can be the difference of entries 1e5 times larger on
    its neighbours, and float32 accumulation resolves it only to the rounding of those. Each group is
    therefore measured against max(its own largest entry, floor x the largest entry of that group over
    all keyframes): a wrong scale column still shows up in full, since the scale group is never compared
    against the translation or rotation groups."""
    g = np.asarray(g, np.float64).reshape(-1, 7)
    g_ref = np.asarray(g_ref, np.float64).reshape(-1, 7)
    worst = 0.0
    for a, b in TANGENT_GROUPS:
        group_max = np.abs(g_ref[:, a:b]).max()
        for k in range(g.shape[0]):
            m = max(np.abs(g_ref[k, a:b]).max(), floor * group_max)
            d = np.abs(g[k, a:b] - g_ref[k, a:b]).max()
            worst = max(worst, d / m if m > 0 else (0.0 if d == 0 else np.inf))
    return float(worst)


def pixel_channel_err(gx, gx_ref, px_off):
    """Per keyframe (pixel ranges px_off[k]:px_off[k+1]) and per channel of a per-pixel gradient ((P, C)
    or (P,)): the largest difference against that keyframe's channel's own largest entry."""
    gx = np.asarray(gx, np.float64)
    gx_ref = np.asarray(gx_ref, np.float64)
    if gx.ndim == 1:
        gx, gx_ref = gx[:, None], gx_ref[:, None]
    worst = 0.0
    for k in range(len(px_off) - 1):
        a, b = px_off[k], px_off[k + 1]
        for c in range(gx.shape[1]):
            m = np.abs(gx_ref[a:b, c]).max()
            d = np.abs(gx[a:b, c] - gx_ref[a:b, c]).max()
            worst = max(worst, d / m if m > 0 else (0.0 if d == 0 else np.inf))
    return float(worst)
