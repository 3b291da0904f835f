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
