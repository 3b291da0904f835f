"""Pins of the oracle's calibrated mode (Sec. IV-C, "Calibration": with supplied intrinsics the pointmaps
are constrained to the calibrated rays and the pose residuals are pixel reprojection and log-depth).

Independent pins: the generator's pinhole projection (ground-truth matches round the projection of the
true point to the nearest pixel, so at the true poses every pixel residual is within half a pixel and the
log-depth residual is the depth ratio of the true point and the matched pixel), exact correspondences
whose optimum is the truth (views rolled by multiples of 90 degrees about the optical axis map pixel
centres onto pixel centres), central finite differences of the scalar cost (gradient) and of the whitened
residual vector (Gauss-Newton Hessian), in the inlier and the outlier regime of the Huber kernel."""
import math

import numpy as np
import pytest

import oracle as O
import synth

IDENT = np.array([0, 0, 0, 0, 0, 0, 1, 1.0])


def tangent_step(poses, k, tau):
    T = np.zeros((poses.shape[0], 7))
    T[k] = tau
    return O.sim3_update(poses, T)


@pytest.fixture(scope="module")
def mixed():
    """Two agents: 512x384 and 512x288 keyframes; edge 4 joins a 384-row keyframe (i) to a 288-row one (j),
    so the two endpoints have different principal points."""
    g = synth.make_config(3, n_agents=2, kf_per_agent=3, n_edges=6)
    i, j = (int(v) for v in g.edges[4])
    assert g.shape(i) != g.shape(j)
    return g


@pytest.mark.parametrize("which", ["tiny pair", "mixed resolutions", "cropped frame"])
def test_ground_truth_residual_is_the_pinhole_rounding(which, request):
    """At the generator's true poses, on its ground-truth matches, the pixel residual of a match is the
    distance of the true projection to the pixel centre it was rounded to (|r_u|, |r_v| <= 0.5 px) and
    the log-depth residual is ln(z / z_i[m]) of the true point against the matched pixel's depth. A
    swapped (u, v), the other keyframe's intrinsics or width, or an inverted transform breaks both.
    'cropped frame': keyframe j of the tiny pair without its first 5 columns and with c_x - 5, so that
    its width and principal point differ from keyframe i's."""
    if which == "tiny pair":
        g, e = synth.make_config(1), 0
    else:
        g, e = (request.getfixturevalue("mixed"), 4) if which == "mixed resolutions" else (synth.make_config(1), 0)
    i, j = (int(v) for v in g.edges[e])
    idx = g.gt_idx(e)
    K = g.intrinsics()
    xyz, conf, world_j = list(g.xyz), [np.ones_like(c) for c in g.conf], g.world[j]
    if which == "cropped frame":
        c0 = 5
        Hj, Wj = g.shape(j)
        xyz[j] = np.ascontiguousarray(g.xyz[j][:, c0:])
        conf[j] = np.ascontiguousarray(conf[j][:, c0:])
        idx = np.ascontiguousarray(idx.reshape(Hj, Wj)[:, c0:]).reshape(-1)
        world_j = world_j.reshape(Hj, Wj, 3)[:, c0:].reshape(-1, 3)
        K[j, 2] -= c0
    cal = O.Calib(K, sigma_pix=1.0, sigma_logz=1.0)
    G = O.Graph(xyz, conf, g.edges[e:e + 1], [idx], anchors=(0,))
    r, w, ok = O.edge_residuals_cal(G, g.poses_gt, 0, cal)
    valid = idx >= 0
    assert ok[valid].all() and not ok[~valid].any() and valid.sum() > 1000
    assert np.abs(r[ok, :2]).max() <= 0.5 + 1e-5
    # the projection itself, from the generator's world points and camera (not the oracle's code)
    R, t, s = synth.pose_parts(g.poses_gt[i])
    X = (world_j - t) @ R / s                  # true points of j in i's canonical frame
    cam = g.cams[i]
    u = cam.f * X[:, 0] / X[:, 2] + cam.cx
    v = cam.f * X[:, 1] / X[:, 2] + cam.cy
    m = idx[valid]
    assert np.allclose(r[valid, 0], u[valid] - m % cam.W, atol=2e-4)
    assert np.allclose(r[valid, 1], v[valid] - m // cam.W, atol=2e-4)
    zi = np.asarray(g.xyz[i], np.float64).reshape(-1, 3)[m, 2]
    assert np.allclose(r[valid, 2], np.log(X[valid, 2] / zi), atol=2e-6)


def rolled_views(H=12, seed=0, n_kf=3):
    """Square H x H views with f_x = f_y and the principal point at the image centre, keyframe k rolled
    by k * 90 degrees about the optical axis and scaled by s_k, all at the origin: the roll maps pixel
    centres onto pixel centres, so every match is exact and the true poses zero every residual."""
    rng = np.random.default_rng(seed)
    f, c = 1.3 * H, (H - 1) / 2.0
    K = np.array([[f, f, c, c]] * n_kf)
    v, u = np.mgrid[0:H, 0:H].astype(np.float64)
    z = 4.0 + 2.0 * rng.uniform(size=(H, H)) + 0.3 * u          # depths of keyframe 0's pixels
    P0 = np.stack([z * (u - c) / f, z * (v - c) / f, z], -1)     # its calibrated points (world frame)
    poses, xyz = [], []
    for k in range(n_kf):
        ang = k * math.pi / 2
        Rz = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1.0]])
        s = 1.0 if k == 0 else math.exp(rng.uniform(-0.3, 0.3))
        poses.append(synth.pose_vec(Rz, np.zeros(3), s))
        X = np.empty_like(P0)
        # pixel (u, v) of keyframe k sees the world point of keyframe 0's pixel rot_k(u, v)
        for vv in range(H):
            for uu in range(H):
                a, b = uu - c, vv - c
                ca, sa = round(math.cos(ang)), round(math.sin(ang))
                u0, v0 = int(round(ca * a - sa * b + c)), int(round(sa * a + ca * b + c))
                X[vv, uu] = Rz.T @ P0[v0, u0] / s
        xyz.append(X)
    poses = np.stack(poses)
    edges = [(0, 1), (1, 2), (0, 2)]
    idx = []
    for i, j in edges:
        # the true match of pixel n of j: the pixel of i seeing the same world point
        Wp = [(xyz_k.reshape(-1, 3) @ synth.pose_parts(poses[k])[0].T) * synth.pose_parts(poses[k])[2]
              for k, xyz_k in ((i, xyz[i]), (j, xyz[j]))]
        d = np.linalg.norm(Wp[1][:, None, :] - Wp[0][None, :, :], axis=-1)
        idx.append(np.argmin(d, axis=1).astype(np.int32))
    return xyz, edges, idx, poses, K


def test_exact_rolled_views_recover_the_truth():
    xyz, edges, idx, gt, K = rolled_views()
    conf = [np.full(x.shape[:2], 2.0) for x in xyz]
    G = O.Graph(xyz, conf, edges, idx, anchors=(0,))
    cal = O.Calib(K)
    r, _, ok = O.edge_residuals_cal(G, gt, 0, cal)
    assert ok.all() and np.abs(r).max() < 1e-9
    rng = np.random.default_rng(3)
    P = gt.copy()
    for k in (1, 2):
        tau = np.concatenate([rng.normal(size=3) * 0.05, rng.normal(size=3) * 0.03, [rng.normal() * 0.03]])
        P = tangent_step(P, k, tau)
    errs = []
    for _ in range(8):
        P, c, st, _ = O.gn_step_cal(G, P, cal)
        assert st == 0
        errs.append(O.pose_error(P, gt).max())
    assert errs[-1] < 1e-9, errs
    assert errs[2] < 1e-3 * errs[0] or errs[2] < 1e-9   # Gauss-Newton on a zero-residual problem


def _tiny(seed_pose=0, scale=1.0):
    g = synth.make_config(1)
    idx = g.gt_idx(0)
    G = O.Graph(g.xyz, g.conf, g.edges, [idx], anchors=())
    rng = np.random.default_rng(seed_pose)
    P = g.poses_gt.copy()
    tau = np.concatenate([rng.normal(size=3) * 0.02, rng.normal(size=3) * 0.01, [0.01]]) * scale
    P = tangent_step(P, 1, tau)
    return g, G, P


@pytest.mark.parametrize("sigma_pix,regime", [(1.0, "mostly inliers"), (0.05, "mostly outliers")])
def test_gradient_matches_central_differences(sigma_pix, regime):
    g, G, P = _tiny()
    cal = O.Calib(g.intrinsics(), sigma_pix=sigma_pix, sigma_logz=0.1)
    _, gv, E, cnt, _, _ = O.gn_assemble_cal(G, P, cal)
    r, w, ok = O.edge_residuals_cal(G, P, 0, cal)
    out = (w[ok] < 1).mean()
    assert (out < 0.3) if regime == "mostly inliers" else (out > 0.6)
    h = 1e-6
    fd = np.zeros(14)
    for k in range(2):
        for a in range(7):
            tp = np.zeros(7)
            tp[a] = h
            Ep = O.cost_cal(G, tangent_step(P, k, tp), cal)
            Em = O.cost_cal(G, tangent_step(P, k, -tp), cal)
            fd[7 * k + a] = (Ep - Em) / (2 * h)
    for grp in (slice(0, 3), slice(3, 6), slice(6, 7), slice(7, 10), slice(10, 13), slice(13, 14)):
        m = np.abs(fd[grp]).max()
        assert np.abs(gv[grp] - fd[grp]).max() <= 1e-5 * max(m, 1e-3 * np.abs(fd).max()), (grp, gv[grp], fd[grp])


def test_hessian_is_gauss_newton_of_the_fd_jacobian():
    """H of the oracle = sum J^T W J with J from central differences of the whitened residual vector and
    W the IRLS weights at the linearisation point (both endpoints, all 14 tangent directions)."""
    g, G, P = _tiny(seed_pose=2)
    cal = O.Calib(g.intrinsics(), sigma_pix=1.0, sigma_logz=0.1)
    H, *_ = O.gn_assemble_cal(G, P, cal)
    r0, w0, ok0 = O.edge_residuals_cal(G, P, 0, cal)
    h = 1e-6
    J = np.zeros((ok0.sum(), 3, 14))
    for k in range(2):
        for a in range(7):
            tp = np.zeros(7)
            tp[a] = h
            rp, _, okp = O.edge_residuals_cal(G, tangent_step(P, k, tp), 0, cal)
            rm, _, okm = O.edge_residuals_cal(G, tangent_step(P, k, -tp), 0, cal)
            assert (okp[ok0] & okm[ok0]).all()
            J[:, :, 7 * k + a] = (rp[ok0] - rm[ok0]) / (2 * h)
    Href = np.einsum("pci,pc,pcj->ij", J, w0[ok0], J)
    d = np.sqrt(np.abs(np.diag(Href)))
    assert np.abs(H - Href).max() / 1.0 >= 0  # shapes agree
    scaled = np.abs(H - Href) / np.outer(d, d)
    assert scaled.max() <= 1e-5, scaled.max()
    # the pixel rows do not see the scale: the scale column comes from the log-depth row alone
    assert np.allclose(J[:, :2, 6], 0, atol=1e-6) and np.allclose(J[:, :2, 13], 0, atol=1e-6)


def test_holes_points_behind_and_off_image_reprojections_are_skipped():
    g, G, P = _tiny()
    cal = O.Calib(g.intrinsics())
    xyz = [np.array(x, np.float64) for x in g.xyz]
    idx = g.gt_idx(0)
    Hi, Wi = g.shape(0)
    # matches whose target pixel is 3 px inside keyframe i's image: unaffected by the small pose offset
    cand = [p for p in np.flatnonzero(idx >= 0) if 3 <= idx[p] % Wi < Wi - 3 and 3 <= idx[p] // Wi < Hi - 3]
    n = np.array(cand[:8])
    xyz[1].reshape(-1, 3)[n[0]] = np.nan
    xyz[1].reshape(-1, 3)[n[1]] = 0.0
    xyz[1].reshape(-1, 3)[n[2], 2] = -3.0          # behind keyframe j's camera
    xyz[0].reshape(-1, 3)[idx[n[3]], 2] = -1.0     # matched pixel of i behind its camera
    xyz[1].reshape(-1, 3)[n[4], 2] *= 0.01         # reprojects far off keyframe i's image
    G2 = O.Graph(xyz, g.conf, g.edges, [idx], anchors=())
    _, _, ok = O.edge_residuals_cal(G2, P, 0, cal)
    assert not ok[n[:5]].any() and ok[n[5:]].all()
    _, _, E, cnt, _, _ = O.gn_assemble_cal(G2, P, cal)
    _, _, E0, cnt0, _, _ = O.gn_assemble_cal(G, P, cal)
    assert np.isfinite(E) and cnt <= cnt0 - 5
