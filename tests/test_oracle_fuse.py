"""Pins of the oracle's canonical pointmap fusion (eq. 2, Sec. III-A): a hand-worked example, the fixed
point of a geometrically consistent prediction (transform built with SciPy's rotation routine, not the
oracle's), sequential fusion equal to the one-shot confidence-weighted average over all predictions,
the pixels the reading leaves unchanged (non-finite prediction, non-positive summed confidence) and the
routing of pairs through their offsets."""
import numpy as np
from scipy.spatial.transform import Rotation

import oracle as O


def _pose(rng):
    q = Rotation.random(random_state=int(rng.integers(1 << 30))).as_quat()  # x, y, z, w
    return np.concatenate([rng.normal(size=3), q, [np.exp(rng.uniform(-0.7, 0.7))]])


def _apply(pose, X):  # s R x + t with SciPy's rotation
    return pose[7] * Rotation.from_quat(pose[3:7]).apply(X) + pose[:3]


def _apply_inv(pose, Y):  # R^T (y - t) / s
    return Rotation.from_quat(pose[3:7]).inv().apply(Y - pose[:3]) / pose[7]


IDENT = np.array([0, 0, 0, 0, 0, 0, 1, 1.0])


def test_hand_worked_identity_example():
    """(1, 2, 3) with confidence 1 fused with (3, 2, 1) with confidence 3 under the identity:
    ((1, 2, 3) + 3 (3, 2, 1)) / 4 = (2.5, 2, 1.5), confidence 4."""
    out = O.fuse([[1, 2, 3, 1]], [[3, 2, 1, 3]], [(0, 0, 1)], [IDENT])
    assert np.array_equal(out, [[2.5, 2.0, 1.5, 4.0]])


def test_consistent_prediction_is_a_fixed_point():
    """A prediction that is exactly the canonical points seen from the frame (x = T^-1 X-hat) leaves
    X-hat in place and adds its confidence: pins the direction of T and the pose layout."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        pose = _pose(rng)
        X = rng.normal(size=(50, 3)) * 3
        c0, c1 = rng.uniform(1, 5, 50), rng.uniform(1, 5, 50)
        x = _apply_inv(pose, X)
        out = O.fuse(np.c_[X, c0], np.c_[x, c1], [(0, 0, 50)], [pose])
        assert np.allclose(out[:, :3], X, rtol=1e-12, atol=1e-12)
        assert np.allclose(out[:, 3], c0 + c1, rtol=0, atol=1e-12)


def test_sequential_fusion_is_the_weighted_average_of_all():
    """Fusing K predictions one after another equals sum_k C_k y_k / sum_k C_k (k = 0 the canonical
    map), each y_k = T_k x_k built with SciPy."""
    rng = np.random.default_rng(4)
    n, K = 40, 4
    X0, C0 = rng.normal(size=(n, 3)), rng.uniform(1, 5, n)
    poses = [_pose(rng) for _ in range(K)]
    xs = [rng.normal(size=(n, 3)) for _ in range(K)]
    cs = [rng.uniform(1, 5, n) for _ in range(K)]
    canon = np.c_[X0, C0]
    for k in range(K):
        canon = O.fuse(canon, np.c_[xs[k], cs[k]], [(0, 0, n)], [poses[k]])
    num = C0[:, None] * X0 + sum(cs[k][:, None] * _apply(poses[k], xs[k]) for k in range(K))
    den = C0 + sum(cs)
    assert np.allclose(canon[:, :3], num / den[:, None], rtol=1e-12, atol=1e-12)
    assert np.allclose(canon[:, 3], den, rtol=1e-14)


def test_unchanged_pixels():
    """Non-finite prediction entries and a non-positive summed confidence leave the pixel as it is."""
    canon = np.array([[1, 1, 1, 2.0], [2, 2, 2, 2.0], [3, 3, 3, 0.0], [4, 4, 4, 1.0]])
    pred = np.array([[np.nan, 0, 0, 1.0], [0, np.inf, 0, 1.0], [9, 9, 9, 0.0], [0, 0, 0, 1.0]])
    out = O.fuse(canon, pred, [(0, 0, 4)], [IDENT])
    assert np.array_equal(out[:3], canon[:3])
    assert np.array_equal(out[3], [2.0, 2.0, 2.0, 2.0])


def test_pairs_route_through_offsets():
    """Three pairs at scattered offsets, against a per-pixel loop written from eq. (2)."""
    rng = np.random.default_rng(5)
    canon = np.c_[rng.normal(size=(100, 3)), rng.uniform(1, 5, 100)]
    pred = np.c_[rng.normal(size=(90, 3)), rng.uniform(1, 5, 90)]
    pairs = [(10, 50, 20), (60, 0, 30), (0, 30, 7)]
    poses = [_pose(rng) for _ in pairs]
    out = O.fuse(canon, pred, pairs, poses)
    ref = canon.copy()
    for (co, po, n), pose in zip(pairs, poses):
        for m in range(n):
            y = _apply(pose, pred[po + m, :3][None])[0]
            c_old, c_new = ref[co + m, 3], pred[po + m, 3]
            ref[co + m, :3] = (c_old * ref[co + m, :3] + c_new * y) / (c_old + c_new)
            ref[co + m, 3] = c_old + c_new
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-12)
