"""GPU parity of the block-sparse ladder solve (ds3_spchol_*) with the FP64 oracle's dense ladder, numpy's
dense solve and the library's dense solver, on pose-graph patterns of 7x7 blocks: chains, stars, random
graphs, chains with cross links (the batched graph's structure) and a fully dense pattern; the epsilon
ladder (a later attempt, every attempt failing), lambda > 0, blocks outside the pattern and the upper
triangle left unread, isolated keyframes, repeated calls on one object, and the GN plan with the sparse
and the dense solver."""
import numpy as np
import pytest
import torch

import oracle as O
from tests.test_spchol_host import PATTERNS, _chains_and_links

pytestmark = pytest.mark.gpu

ds3 = pytest.importorskip("paper_2605_30488_amd.api")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dev)


def _gn_like(n, pairs, seed, ridge=1e-3):
    """Sum of per-pair Gauss-Newton terms [J_a J_b]^T [J_a J_b] (10 residual rows each) plus a small ridge:
    symmetric positive definite with exactly the pair pattern."""
    rng = np.random.default_rng(seed)
    H = ridge * np.eye(7 * n)
    for a, b in pairs:
        J = rng.normal(size=(10, 14)) * rng.uniform(0.5, 2.0)
        M = J.T @ J
        ia, ib = slice(7 * a, 7 * a + 7), slice(7 * b, 7 * b + 7)
        H[ia, ia] += M[:7, :7]
        H[ib, ib] += M[7:, 7:]
        H[ia, ib] += M[:7, 7:]
        H[ib, ia] += M[7:, :7]
    for k in range(n):  # keyframes without pairs still get a well-conditioned block
        H[7 * k:7 * k + 7, 7 * k:7 * k + 7] += np.eye(7)
    return H, rng.normal(size=7 * n)


def _pattern_mask(n, pairs):
    m = np.eye(n, dtype=bool)
    for a, b in pairs:
        m[a, b] = m[b, a] = True
    return np.kron(m, np.ones((7, 7), dtype=bool))


@pytest.mark.parametrize("name", sorted(PATTERNS))
def test_spchol_matches_oracle_and_dense(dev, name):
    n, pairs = PATTERNS[name]
    H, g = _gn_like(n, pairs, seed=len(name))
    S = ds3.SpChol(n, pairs)
    tau, st = S.solve(_t(H, dev), _t(g, dev), lam=0.0)
    ref, st_ref = O.chol_ladder(H, g, lam=0.0)
    tau_d, st_d = ds3.chol_ladder_solve(_t(H, dev), _t(g, dev), lam=0.0)
    t = tau.cpu().numpy()
    assert int(st.item()) == st_ref == int(st_d.item()) == 0
    assert np.allclose(t, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())
    assert np.allclose(t, tau_d.cpu().numpy(), rtol=1e-9, atol=1e-11 * np.abs(ref).max())
    S.close()


def test_spchol_lambda_and_batched_structure(dev):
    """Four chains of 50 keyframes with cross links (n = 1400), lambda = 0.1: against numpy's dense solve of
    (H + lambda diag H + eps I) and the library's dense solver."""
    n, pairs = _chains_and_links(per=50, links=3, seed=11)
    H, g = _gn_like(n, pairs, seed=5)
    S = ds3.SpChol(n, pairs)
    info = S.info()
    assert info["blocks"] < 0.25 * n * (n + 1) / 2
    tau, st = S.solve(_t(H, dev), _t(g, dev), lam=0.1)
    A = H + 0.1 * np.diag(np.diag(H)) + 1e-6 * np.eye(7 * n)
    ref = np.linalg.solve(A, -g)
    tau_d, _ = ds3.chol_ladder_solve(_t(H, dev), _t(g, dev), lam=0.1)
    t = tau.cpu().numpy()
    assert int(st.item()) == 0
    assert np.allclose(t, ref, rtol=1e-9, atol=1e-10 * np.abs(ref).max())
    assert np.allclose(t, tau_d.cpu().numpy(), rtol=1e-9, atol=1e-10 * np.abs(ref).max())
    S.close()


def test_spchol_reads_only_the_lower_pattern(dev):
    """NaN in every entry outside the pattern's blocks and in the strict upper triangle: the result is
    bitwise the one of the clean matrix."""
    n, pairs = PATTERNS["random"]
    H, g = _gn_like(n, pairs, seed=21)
    S = ds3.SpChol(n, pairs)
    tau0, _ = S.solve(_t(H, dev), _t(g, dev))
    Hd = H.copy()
    Hd[~_pattern_mask(n, pairs)] = np.nan
    Hd[np.triu_indices(7 * n, 1)] = np.nan
    tau1, st1 = S.solve(_t(Hd, dev), _t(g, dev))
    assert int(st1.item()) == 0
    assert np.array_equal(tau0.cpu().numpy(), tau1.cpu().numpy())
    S.close()


@pytest.mark.parametrize("p", [3, 60, 139])
def test_spchol_ladder_later_attempt(dev, p):
    """A negative diagonal entry at row p on top of a weakly coupled positive definite part: attempt 0 fails
    wherever p sits in the elimination order, a later attempt succeeds, and status and solution equal the
    oracle's dense ladder."""
    n, pairs = PATTERNS["chains_and_links"]
    rng = np.random.default_rng(p)
    Hc, g = _gn_like(n, pairs, seed=p)
    H = 0.002 * Hc + np.diag(rng.uniform(1.5, 2.5, size=7 * n))
    H[p, p] = -0.5
    S = ds3.SpChol(n, pairs)
    tau, st = S.solve(_t(H, dev), _t(g, dev))
    ref, st_ref = O.chol_ladder(H, g)
    assert st_ref == 3
    assert int(st.item()) == st_ref
    assert np.allclose(tau.cpu().numpy(), ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())
    H[p, p] = -1e5
    tau, st = S.solve(_t(H, dev), _t(g, dev))
    assert int(st.item()) == -1 and np.all(tau.cpu().numpy() == 0)
    S.close()


@pytest.mark.parametrize("n", [1, 5])
def test_spchol_without_pairs(dev, n):
    """No pairs: block-diagonal H, every keyframe its own column at level 0."""
    H, g = _gn_like(n, [], seed=n)
    S = ds3.SpChol(n, [])
    assert S.info()["levels"] == 1
    tau, st = S.solve(_t(H, dev), _t(g, dev))
    ref, st_ref = O.chol_ladder(H, g)
    assert int(st.item()) == st_ref == 0
    assert np.allclose(tau.cpu().numpy(), ref, rtol=1e-10)
    S.close()


def test_spchol_dense_pattern(dev):
    """Every pair of 40 keyframes (a dense factor, 280 x 280): its tables still fit, and the solve equals
    the dense ones."""
    n = 40
    pairs = [(a, b) for a in range(n) for b in range(a)]
    _, _, info = ds3.spchol_analyse(n, pairs)
    assert info["blocks"] == n * (n + 1) // 2 and info["table_words"] <= 28 * 1024
    H, g = _gn_like(n, pairs, seed=40)
    S = ds3.SpChol(n, pairs)
    tau, st = S.solve(_t(H, dev), _t(g, dev), lam=0.05)
    ref, st_ref = O.chol_ladder(H, g, lam=0.05)
    assert int(st.item()) == st_ref == 0
    assert np.allclose(tau.cpu().numpy(), ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())
    S.close()


def test_spchol_repeated_calls(dev):
    """Two different systems on one object, one after the other, and the first again."""
    n, pairs = PATTERNS["chains_and_links"]
    S = ds3.SpChol(n, pairs)
    out = []
    for seed in (1, 2, 1):
        H, g = _gn_like(n, pairs, seed=seed)
        tau, st = S.solve(_t(H, dev), _t(g, dev))
        ref, _ = O.chol_ladder(H, g)
        assert int(st.item()) == 0
        assert np.allclose(tau.cpu().numpy(), ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())
        out.append(tau.cpu().numpy())
    assert np.array_equal(out[0], out[2])
    S.close()
