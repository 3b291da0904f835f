"""Pins of the oracle's Sim(3) algebra (Sec. III-A pose model, Sec. III-D left perturbation).

Exp is pinned to SciPy's Pade-based matrix exponential (an independent routine) and to textbook closed
forms (Rodrigues for pure rotation, e^zeta for pure scale); Log by round trips; Ad by its defining
identity T Exp(tau) T^-1 = Exp(Ad_T tau)."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O


def hat(t):
    v, w, z = t[:3], t[3:6], t[6]
    return np.array([[z, -w[2], w[1], v[0]], [w[2], z, -w[0], v[1]], [-w[1], w[0], z, v[2]],
                     [0, 0, 0, 0.0]])


@pytest.mark.parametrize("scale", [1e-9, 1e-5, 1e-2, 0.3, 1.0, 2.0])
def test_exp_matches_scipy_expm(scale):
    rng = np.random.default_rng(int(scale * 1e9) % 997)
    for _ in range(100):
        t = rng.normal(size=7) * scale
        nw = np.linalg.norm(t[3:6])
        if nw > 3.0:
            t[3:6] *= 3.0 / nw
        E = sl.expm(hat(t))
        M = O.sim3_exp_mat(t)
        assert np.abs(M - E).max() <= 1e-12 * max(1.0, np.abs(E).max())


def test_exp_special_cases():
    # pure rotation: Rodrigues' formula
    axis = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    ang = 1.1
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    Rr = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K
    M = O.sim3_exp_mat(np.concatenate([[0, 0, 0], axis * ang, [0]]))
    assert np.allclose(M[:3, :3], Rr, atol=1e-14) and np.allclose(M[:3, 3], 0, atol=1e-15)
    # pure scale: s = e^zeta
    M = O.sim3_exp_mat([0, 0, 0, 0, 0, 0, 0.7])
    assert np.allclose(M[:3, :3], math.exp(0.7) * np.eye(3), atol=1e-14)
    # pure translation
    M = O.sim3_exp_mat([1.5, -2.0, 0.25, 0, 0, 0, 0])
    assert np.allclose(M[:3, 3], [1.5, -2.0, 0.25], atol=1e-15)
    # scale with translation: t = (e^zeta - 1)/zeta v
    z = 0.4
    M = O.sim3_exp_mat([1.0, 0, 0, 0, 0, 0, z])
    assert abs(M[0, 3] - (math.exp(z) - 1) / z) < 1e-14
    # identity
    p = O.sim3_exp(np.zeros(7))[0]
    assert np.array_equal(p, np.array([0, 0, 0, 0, 0, 0, 1, 1.0]))


@pytest.mark.parametrize("scale", [1e-8, 1e-4, 1e-2, 0.5, 1.5])
def test_log_exp_round_trip(scale):
    rng = np.random.default_rng(7)
    for _ in range(100):
        t = rng.normal(size=7) * scale
        nw = np.linalg.norm(t[3:6])
        if nw > 3.0:
            t[3:6] *= 3.0 / nw
        back = O.sim3_log(O.sim3_exp(t)[0])[0]
        # absolute error: the pose vector itself carries ~1e-16 absolute precision
        assert np.abs(back - t).max() <= 1e-13 * max(1.0, np.abs(t).max())


def test_exp_log_round_trip_poses():
    rng = np.random.default_rng(3)
    for _ in range(50):
        p = O.sim3_exp(rng.normal(size=7))[0]
        q = O.sim3_exp(O.sim3_log(p)[0])[0]
        assert np.allclose(O.pose_to_mat(p), O.pose_to_mat(q), atol=1e-12)


def test_adjoint_identity():
    rng = np.random.default_rng(11)
    for _ in range(30):
        p = O.sim3_exp(rng.normal(size=7))[0]
        t = rng.normal(size=7) * 0.3
        T = O.pose_to_mat(p)
        lhs = T @ O.sim3_exp_mat(t) @ np.linalg.inv(T)
        rhs = O.sim3_exp_mat(O.sim3_adjoint(p) @ t)
        assert np.abs(lhs - rhs).max() < 1e-12


def test_group_one_parameter():
    rng = np.random.default_rng(5)
    t = rng.normal(size=7) * 0.4
    A = O.sim3_exp_mat(0.3 * t) @ O.sim3_exp_mat(0.7 * t)
    assert np.abs(A - O.sim3_exp_mat(t)).max() < 1e-13


def test_relative_and_update():
    rng = np.random.default_rng(9)
    pi = O.sim3_exp(rng.normal(size=7))[0]
    pj = O.sim3_exp(rng.normal(size=7))[0]
    pij = O.relative(pi, pj)
    assert np.allclose(O.pose_to_mat(pi) @ O.pose_to_mat(pij), O.pose_to_mat(pj), atol=1e-12)
    tau = rng.normal(size=(2, 7)) * 0.1
    up = O.sim3_update(np.stack([pi, pj]), tau, fixed=[1, 0])
    assert np.array_equal(up[0], pi)  # fixed pose untouched, bit for bit
    assert np.allclose(O.pose_to_mat(up[1]), O.sim3_exp_mat(tau[1]) @ O.pose_to_mat(pj), atol=1e-12)
    assert abs(np.linalg.norm(up[1, 3:7]) - 1) < 1e-15


def test_pose_error_measure():
    p = np.array([0, 0, 0, 0, 0, 0, 1, 1.0])
    q = p.copy()
    q[:3] = [0.5, 0, 0]
    assert abs(O.pose_error(q, p)[0] - 0.5) < 1e-15          # |t_ref| < 1 m -> divide by 1 m
    q = p.copy()
    q[7] = 1.01
    assert abs(O.pose_error(q, p)[0] - 0.01) < 1e-12
    ang = 1e-4
    q = p.copy()
    q[3:7] = [math.sin(ang / 2), 0, 0, math.cos(ang / 2)]
    assert abs(O.pose_error(q, p)[0] - ang) < 1e-15
