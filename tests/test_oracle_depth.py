"""Pins of the oracle's terminal segment-level depth refinement (Sec. III-E, eqs. (8)-(10)).

Independent pins: closed-form normals of a plane; the normalised log-range's end points; SLIC on uniform
features reducing to the grid partition, and respecting a feature edge that is not on the grid; boundary
differences on hand-made stripes; the gradient of E' against central differences (data, boundary and prior
terms together), the Jacobi diagonal against the finite-difference Jacobian of the whitened residuals;
exact recovery of per-segment log-scales on exact correspondences; the closed form of prior-only damped
steps, the clip, and fixed anchor segments."""
import numpy as np
import pytest

import oracle as O
from oracle import depth as D
from tests.helpers import exact_graph


def plane_view(H=24, W=32, n=(0.3, -0.2, -0.93), c=-6.0, f=30.0):
    """Pinhole view of the plane n . X = c: each pixel's ray hits it at X = (c / (n . r)) r."""
    n = np.asarray(n, float)
    n /= np.linalg.norm(n)
    v, u = np.mgrid[0:H, 0:W].astype(float)
    r = np.stack([(u - (W - 1) / 2) / f, (v - (H - 1) / 2) / f, np.ones_like(u)], -1)
    return (c / (r @ n))[..., None] * r, n


def test_normals_of_a_plane():
    X, n = plane_view()
    N = D.normals(X)
    want = n if (n @ X[0, 0]) < 0 else -n           # oriented towards the camera
    assert np.abs(N - want).max() < 1e-12          # central and one-sided differences lie in the plane
    X[5, 7] = np.nan
    N = D.normals(X)
    assert np.all(N[5, 7] == 0) and np.all(N[5, 6] == 0) and np.all(N[4, 7] == 0) and np.all(N[6, 8] != 0)


def test_features_quantise_and_normalise_log_range():
    X, n = plane_view()
    C = np.full(X.shape[:2], 3.0)
    C[0, 0] = 1.0                                  # below C_min = 1.5: excluded
    F, valid = D.features(X, C)
    assert not valid[0, 0] and valid.sum() == valid.size - 1 and np.all(F[0, 0] == 0)
    L = np.log(np.linalg.norm(X, axis=-1))
    Lv = L[valid]
    assert F[..., 3][valid].min() == 0 and F[..., 3][valid].max() == D.Q
    k = np.unravel_index(np.argmax(np.where(valid, L, -np.inf)), L.shape)
    assert F[k][3] == D.Q
    want = np.floor(D.Q * ((L - Lv.min()) / (Lv.max() - Lv.min())) + 0.5)
    assert np.array_equal(F[..., 3][valid], want[valid].astype(np.int64))
    nq = n if (n @ X[1, 1]) < 0 else -n
    assert np.array_equal(F[1, 1, :3], np.floor(D.Q * (nq + 1) + 0.5).astype(np.int64))


def test_slic_uniform_features_give_the_grid():
    """Uniform features: only the spatial term matters, every pixel is closest to the centre of its own
    grid cell (odd S: no ties) and the centres stay at the cell centres."""
    S, n = 7, 4
    H = W = S * n
    F = np.full((H, W, 4), 500, np.int64)
    valid = np.ones((H, W), bool)
    M = n * n
    assert D.grid(H, W, M) == (S, n, n)
    lab, cen = D.slic(F, valid, M, iters=10)
    v, u = np.mgrid[0:H, 0:W]
    assert np.array_equal(lab, (v // S) * n + u // S)
    assert np.array_equal(cen[:, 0], (np.arange(M) % n) * S + S // 2)


def test_slic_ties_go_to_the_lowest_centre_index():
    """Even S: a pixel on a cell boundary is equidistant from two (or four) centres and takes the lowest
    index, so cell k holds the pixels x in ((k - 1) S + S/2 .. k S + S/2] along each axis."""
    S, n = 8, 4
    H = W = S * n
    F = np.full((H, W, 4), 77, np.int64)
    lab, _ = D.slic(F, np.ones((H, W), bool), n * n, iters=10)
    v, u = np.mgrid[0:H, 0:W]
    ax = lambda x: np.where(x == 0, 0, (x - 1) // S)
    assert np.array_equal(lab, ax(v) * n + ax(u))


def test_small_segments_are_excluded():
    X, _ = plane_view(H=32, W=32)
    C = np.full((32, 32), 3.0)
    C[:8, :8] = 1.0                                # grid cell 0 (S = 8): 10 valid pixels around its centre
    C[3:5, 0:5] = 3.0
    F, valid = D.features(X, C)
    raw, _ = D.slic(F, valid, 16)
    assert np.array_equal(raw[3:5, 0:5], np.zeros((2, 5), np.int64)) and (raw == 0).sum() == 10
    lab, M = D.segment(X, C, D.DepthParams(segments_per_kf=16))
    assert M == 16
    assert np.all(lab[3:5, 0:5] == -1)             # fewer than 16 valid pixels: excluded
    assert np.array_equal(lab[raw != 0], raw[raw != 0])


def test_slic_respects_a_feature_edge_off_the_grid():
    S, n = 9, 5
    H = W = S * n
    F = np.zeros((H, W, 4), np.int64)
    edge = 2 * S + 4                                # not a grid line
    F[:, :edge, :3] = (1024, 1024, 0)              # two surface orientations
    F[:, edge:, :3] = (1024, 0, 1024)
    F[..., 3] = 300
    valid = np.ones((H, W), bool)
    valid[3, 3] = False
    lab, _ = D.slic(F, valid, n * n, iters=10)
    assert lab[3, 3] == -1
    u = np.mgrid[0:H, 0:W][1]
    for s in np.unique(lab[lab >= 0]):
        side = u[lab == s] < edge
        assert side.all() or (~side).all(), s


def test_boundary_differences_on_stripes():
    H, W = 6, 9
    lab = np.zeros((H, W), np.int64)
    lab[:, 3:6] = 1
    lab[:, 6:] = 2
    lab[0, 0] = -1                                 # excluded pixel: no pairs
    rng = np.random.default_rng(0)
    d = rng.uniform(2, 20, size=(H, W))
    X = d[..., None] * np.array([0.0, 0.0, 1.0])
    L = np.log(d)
    b = D.boundary(X, lab)
    assert set(b) == {(0, 1), (1, 0), (1, 2), (2, 1)}
    s01, c01 = b[(0, 1)]
    assert c01 == H and abs(s01 - (L[:, 2] - L[:, 3]).sum()) < 1e-12
    s10, c10 = b[(1, 0)]
    assert c10 == H and abs(s10 + s01) < 1e-12
    s12, c12 = b[(1, 2)]
    assert c12 == H and abs(s12 - (L[:, 5] - L[:, 6]).sum()) < 1e-12


def _tiny_problem(seed=7, lam_s=1.0, lam_p=1.0):
    """The 64x48 pair, 12 segments per keyframe, ground-truth matches, perturbed relative pose."""
    import synth
    g = synth.make_config(1)
    idx = [g.gt_idx(0)]
    P = D.DepthParams(segments_per_kf=12, lambda_smooth=lam_s, lambda_prior=lam_p)
    prob = D.DepthProblem(g.xyz, g.conf, g.edges, idx, anchors=(0,), params=P)
    rng = np.random.default_rng(seed)
    eta = np.where(prob.seg_valid, rng.normal(size=prob.n_seg) * 0.05, 0.0)
    return g, prob, eta


def test_gradient_against_central_differences():
    g, prob, eta = _tiny_problem()
    poses = g.poses_gt.copy()
    E, H, grad = prob.linearise(poses, eta)
    h = 1e-6
    for s in np.flatnonzero(prob.seg_valid):
        e1, e2 = eta.copy(), eta.copy()
        e1[s] += h
        e2[s] -= h
        fd = (prob.linearise(poses, e1)[0] - prob.linearise(poses, e2)[0]) / (2 * h)
        assert abs(grad[s] - fd) <= 1e-5 * max(abs(fd), 1.0), (s, grad[s], fd)


def test_jacobi_diagonal_is_the_fd_jacobian():
    """H_gg = sum w (dr/deta_g)^2 over the data term + lambda_smooth x (boundary pairs of g) + lambda_prior,
    with dr/deta_g from central differences of the whitened residual vector."""
    g, prob, eta = _tiny_problem(lam_s=0.7, lam_p=0.3)
    poses = g.poses_gt.copy()
    E, H, grad = prob.linearise(poses, eta)
    (r0, hs, gs, _, _), = prob.residuals(poses, eta)
    a = np.abs(r0)
    w = np.where(a <= prob.P.huber_k, 1.0, prob.P.huber_k / np.where(a > 0, a, 1.0))
    npairs = np.zeros(prob.n_seg)
    for (s1, _s2) in prob.pairs:
        npairs[s1] += 1
    step = 1e-6
    for s in np.flatnonzero(prob.seg_valid)[::3]:
        e1, e2 = eta.copy(), eta.copy()
        e1[s] += step
        e2[s] -= step
        (r1, *_), = prob.residuals(poses, e1)
        (r2, *_), = prob.residuals(poses, e2)
        J = (r1 - r2) / (2 * step)
        want = (w * J * J).sum() + 0.7 * npairs[s] + 0.3
        assert abs(H[s] - want) <= 1e-6 * want, (s, H[s], want)


def test_exact_log_scales_are_recovered():
    """Exact correspondences with keyframe j's segments shrunk by exp(-eta*): with the data term alone the
    Jacobi damped Newton steps recover eta* (each of j's segments is a 1-D problem: keyframe i is the anchor)."""
    xyz, conf, edges, idx, gt = exact_graph(n_kf=2, H=24, W=32, seed=4, edges=[(0, 1)], frac_valid=1.0)
    conf = [np.full(c.shape, 3.0) for c in conf]
    P = D.DepthParams(segments_per_kf=12, lambda_smooth=0.0, lambda_prior=0.0)
    base = D.DepthProblem(xyz, conf, edges, idx, anchors=(0,), params=P)
    labels = [(base.labels[k], (base.base[1] if k == 0 else base.n_seg - base.base[1])) for k in range(2)]
    rng = np.random.default_rng(1)
    eta_true = np.where(base.seg_valid & (base.seg_kf == 1), rng.uniform(-0.1, 0.1, base.n_seg), 0.0)
    gl = base.glabel(1).reshape(xyz[1].shape[:2])
    shrunk = [xyz[0], xyz[1] * np.where(gl >= 0, np.exp(-eta_true[np.maximum(gl, 0)]), 1.0)[..., None]]
    prob = D.DepthProblem(shrunk, conf, edges, idx, anchors=(0,), params=P, labels=labels)
    eta, costs = prob.run(gt, iters=10)
    assert np.abs(eta - eta_true).max() < 1e-9, np.abs(eta - eta_true).max()
    assert costs[-1] < 1e-12 * costs[0]
    assert np.all(eta[base.seg_kf == 0] == 0)       # anchor segments never move


def test_prior_only_steps_and_clip():
    """Without matches and boundary pairs, a damped step is -eta / (1 + lambda_lm): eta_k = eta_0 q^k with
    q = lambda_lm / (1 + lambda_lm); a step larger than eta_max is clipped."""
    g, prob, _ = _tiny_problem(lam_s=0.0, lam_p=0.3)
    prob.edges, prob.idx = [], []
    eta0 = np.where(prob.free, 0.2, 0.0)
    eta, _ = prob.run(g.poses_gt, eta0, iters=3)
    q = prob.P.lambda_lm / (1 + prob.P.lambda_lm)
    assert np.allclose(eta[prob.free], 0.2 * q ** 3, rtol=1e-12, atol=0)
    eta, _ = prob.run(g.poses_gt, np.where(prob.free, 5.0, 0.0), iters=1)
    assert np.allclose(eta[prob.free], 4.5, rtol=0, atol=1e-15)
