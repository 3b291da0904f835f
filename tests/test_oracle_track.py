"""Pins of the oracle's ray-range tracker (Sec. III-A, E_track with LM damping; eq. 7 with lambda > 0):
exact recovery on exact correspondences, the undamped first trial against one Gauss-Newton step of the
two-keyframe graph computed by the independent C step (its own Cholesky ladder and Exp update), the
gradient against central differences of E_track, and the LM bookkeeping (kept costs never increase,
the damping follows its schedule, a pose without matches stays put)."""
import numpy as np

import oracle as O
import synth
from tests.helpers import exact_graph, perturb

IDENT = np.array([0, 0, 0, 0, 0, 0, 1, 1.0])


def _exact(seed=3):
    xyz, conf, edges, idx, gt = exact_graph(n_kf=2, H=24, W=32, seed=seed, frac_valid=0.9)
    return xyz, conf, idx[0], gt[1]


def test_exact_correspondences_recover_the_pose():
    xyz, conf, idx, T_gt = _exact()
    rng = np.random.default_rng(1)
    for k in range(4):
        tau = np.concatenate([rng.normal(size=3) * 0.2, rng.normal(size=3) * 0.15, [rng.normal() * 0.1]])
        T0 = O.sim3_update(T_gt[None], tau[None])[0]
        r = O.track(xyz[0], conf[0], xyz[1], conf[1], idx, T0)
        assert O.pose_error(r.pose[None], T_gt[None])[0] < 1e-9, k
        assert r.cost < 1e-12 and r.trials < 20


def test_undamped_first_trial_is_one_gauss_newton_step():
    """lambda0 = 0: the first trial solves the same normal equations as one GN step of the graph
    {keyframe (anchor, identity), frame} with the frame's pose T_kf, which the C oracle computes with its
    own assembly, Cholesky ladder and update."""
    g = synth.make_config(1)
    idx = g.gt_idx(0)
    T0 = O.relative(g.poses_init[0], g.poses_init[1])
    r = O.track(g.xyz[0], g.conf[0], g.xyz[1], g.conf[1], idx, T0, tp=O.TrackParams(lambda0=0.0, max_trials=1))
    og = O.Graph(g.xyz, g.conf, [(0, 1)], [idx], anchors=(0,))
    p, c, st, _ = O.gn_step(og, np.stack([IDENT, T0]))
    assert st == 0 and r.accepted == [True]
    assert O.pose_error(r.pose[None], p[1][None])[0] < 1e-12


def test_gradient_matches_finite_differences():
    """The g of the tracker's normal equations is dE_track/dtau for T <- Exp(tau) T (central FD, FP64)."""
    g = synth.make_config(1)
    idx = g.gt_idx(0)
    T = O.relative(g.poses_init[0], g.poses_init[1])
    og = O.Graph(g.xyz, g.conf, [(0, 1)], [idx], anchors=(0,))
    _, gv, E, *_ = O.gn_assemble(og, np.stack([IDENT, T]))
    b = gv[7:]
    h = 1e-6
    for c in range(7):
        d = np.zeros(7)
        d[c] = h
        Ep = O.cost(og, np.stack([IDENT, O.sim3_update(T[None], d[None])[0]]))
        Em = O.cost(og, np.stack([IDENT, O.sim3_update(T[None], -d[None])[0]]))
        fd = (Ep - Em) / (2 * h)
        assert abs(fd - b[c]) <= 1e-5 * np.abs(b).max() + 1e-7 * E, c


def test_lm_bookkeeping_with_rejections():
    """A start about 3 rad away with no damping: the first steps overshoot and are rejected. Kept costs
    never increase; each rejection multiplies the damping by 10, each acceptance divides it by 10 down to
    its floor; the search still reaches the optimum the tracker finds from a near start."""
    g = synth.make_config(1)
    idx = g.gt_idx(0)
    T_gt = O.relative(g.poses_gt[0], g.poses_gt[1])
    rng = np.random.default_rng(0)
    tau = np.concatenate([rng.normal(size=3) * 3, rng.normal(size=3) * 1.2, [rng.normal() * 1.0]])
    T0 = O.sim3_update(T_gt[None], tau[None])[0]
    tp = O.TrackParams(lambda0=0.0, max_trials=30)
    r = O.track(g.xyz[0], g.conf[0], g.xyz[1], g.conf[1], idx, T0, tp=tp)
    assert not all(r.accepted) and any(r.accepted)
    assert all(b <= a for a, b in zip(r.costs, r.costs[1:]))
    for k in range(len(r.lambdas) - 1):
        want = max(r.lambdas[k] * tp.lambda_down, tp.lambda_min) if r.accepted[k] else r.lambdas[k] * tp.lambda_up
        assert r.lambdas[k + 1] == want
    near = O.track(g.xyz[0], g.conf[0], g.xyz[1], g.conf[1], idx, T_gt, tp=O.TrackParams(max_trials=40))
    assert O.pose_error(r.pose[None], near.pose[None])[0] < 1e-6


def test_no_matches_leaves_the_pose():
    xyz, conf, idx, T_gt = _exact(seed=4)
    T0 = perturb(np.stack([IDENT, T_gt]), np.random.default_rng(2))[1]
    r = O.track(xyz[0], conf[0], xyz[1], conf[1], np.full_like(idx, -1), T0)
    assert np.array_equal(r.pose, T0) and r.cost == 0.0 and not any(r.accepted)
