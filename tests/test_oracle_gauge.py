"""Pins of gauge synchronisation (Sec. III-C, eqs. 3-4): Umeyama's closed form and the component
tracker with its endpoint fallback."""
import numpy as np
import pytest

import oracle as O
import synth
from tests.helpers import exact_graph


def _sim(rng):
    return O.sim3_exp(rng.normal(size=7) * np.array([2, 2, 2, 1, 1, 1, 0.4]))[0]


def test_umeyama_recovers_exact_similarity():
    rng = np.random.default_rng(0)
    for _ in range(20):
        y = rng.normal(size=(200, 3)) * 3
        T = _sim(rng)
        x = O.transform_points(T, y)
        est = O.umeyama(x, y)
        assert np.allclose(O.pose_to_mat(est), O.pose_to_mat(T), atol=1e-10)


def test_umeyama_planar_points_keep_a_rotation():
    """Coplanar correspondences (rank-2 covariance): det(UV^T) can be -1; S flips it to a rotation."""
    rng = np.random.default_rng(1)
    y = np.c_[rng.normal(size=(100, 2)), np.zeros(100)]
    T = _sim(rng)
    x = O.transform_points(T, y)
    est = O.umeyama(x, y)
    R = O.pose_to_mat(est)[:3, :3] / est[7]
    assert abs(np.linalg.det(R) - 1) < 1e-12
    assert np.allclose(O.transform_points(est, y), x, atol=1e-9)


def test_umeyama_is_optimal_under_noise():
    """First-order optimality of eq. (3): the objective grows under any small similarity perturbation."""
    rng = np.random.default_rng(2)
    y = rng.normal(size=(500, 3)) * 2
    x = O.transform_points(_sim(rng), y) + rng.normal(size=(500, 3)) * 0.05
    est = O.umeyama(x, y)
    f0 = ((x - O.transform_points(est, y)) ** 2).sum()
    for _ in range(50):
        d = rng.normal(size=7) * 1e-4
        moved = O.mat_to_pose(O.sim3_exp_mat(d) @ O.pose_to_mat(est))
        assert ((x - O.transform_points(moved, y)) ** 2).sum() >= f0 - 1e-12


def test_umeyama_rejects_collinear():
    y = np.outer(np.linspace(-1, 1, 50), [1.0, 2.0, 3.0])
    assert O.umeyama(y * 2 + 1, y) is None


def test_gauge_sync_recovers_component_gauge():
    """Two agents (keyframes 0-1 and 2-3) with exact matches; agent 1's map sits in a foreign gauge G.
    Synchronisation through the inter-agent edge (1, 2) undoes G exactly."""
    xyz, conf, edges, idx, gt = exact_graph(n_kf=4, H=12, W=16, seed=3,
                                            edges=[(0, 1), (2, 3), (1, 2)], frac_valid=0.9)
    agent = np.array([0, 0, 1, 1])
    G = _sim(np.random.default_rng(4))
    init = gt.copy()
    for k in (2, 3):
        init[k] = O.compose(G, gt[k])
    matches = [(idx[e], (idx[e] >= 0).astype(np.uint8)) for e in range(3)]
    out, links = O.gauge_sync(init, agent, edges, [True] * 3, matches, xyz)
    assert len(links) == 1 and links[0].edge == 2 and links[0].used_umeyama
    assert links[0].moved_agents == [1]
    assert O.pose_error(out, gt).max() < 1e-9


def test_gauge_sync_endpoint_fallback_and_reference_choice():
    xyz, conf, edges, idx, gt = exact_graph(n_kf=4, H=6, W=8, seed=5,
                                            edges=[(0, 1), (2, 3), (2, 1)], frac_valid=0.9)
    agent = np.array([0, 0, 1, 1])
    G = _sim(np.random.default_rng(6))
    init = gt.copy()
    for k in (2, 3):
        init[k] = O.compose(G, gt[k])
    matches = [(idx[e], (idx[e] >= 0).astype(np.uint8)) for e in range(3)]
    # fewer than N_c^min correspondences -> T* = T_ref T_mov^-1 (agent 0 is the reference even though
    # the edge is written (2, 1)); the moving endpoint lands on the reference endpoint's pose
    out, links = O.gauge_sync(init, agent, edges, [True] * 3, matches, xyz, nc_min=10 ** 6)
    assert not links[0].used_umeyama and links[0].moved_agents == [1]
    assert np.allclose(O.pose_to_mat(out[2]), O.pose_to_mat(init[1]), atol=1e-12)
    rel_before = O.relative(init[2], init[3])
    rel_after = O.relative(out[2], out[3])
    assert np.allclose(O.pose_to_mat(rel_before), O.pose_to_mat(rel_after), atol=1e-10)
    assert np.array_equal(out[:2], init[:2])


def test_gauge_sync_skips_connected_and_rejected():
    xyz, conf, edges, idx, gt = exact_graph(n_kf=4, H=6, W=8, seed=7,
                                            edges=[(0, 2), (1, 3), (0, 1)], frac_valid=0.9)
    agent = np.array([0, 0, 1, 1])
    matches = [(idx[e], (idx[e] >= 0).astype(np.uint8)) for e in range(3)]
    out, links = O.gauge_sync(gt, agent, edges, [False, True, True], matches, xyz)
    assert [l.edge for l in links] == [1]  # edge 0 rejected by the gate, edge 2 intra-agent
