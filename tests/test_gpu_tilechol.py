"""GPU parity of the tile-sparse ladder solve (ds3_tilechol_*) with the FP64 oracle's dense ladder, numpy's
dense solve and the library's dense solver, on pose-graph patterns of 7x7 blocks: chains, stars, random
graphs, chains with cross links (the batched graph's structure) and a fully dense pattern; the epsilon
ladder (a later attempt through the dense fallback, every attempt failing, a single attempt), lambda > 0,
blocks outside the pattern and the upper triangle left unread, isolated keyframes, repeated calls on one
object, and the GN plan with the tile-sparse, the dense and the default solver."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2605_30488_amd._lib import DS3Error
from tests.test_gpu_spchol import _gn_like, _pattern_mask
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


@pytest.mark.parametrize("name", sorted(PATTERNS))
def test_tilechol_matches_oracle_and_dense(dev, name):
    n, pairs = PATTERNS[name]
    H, g = _gn_like(n, pairs, seed=len(name) + 1)
    S = ds3.TileChol(n, pairs)
    tau, st = S.solve(_t(H, dev), _t(g, dev), lam=0.0)
    ref, st_ref = O.chol_ladder(H, g, lam=0.0)
    tau_d, st_d = ds3.chol_ladder_solve(_t(H, dev), _t(g, dev), lam=0.0)
    t = tau.cpu().numpy()
    assert int(st.item()) == st_ref == int(st_d.item()) == 0
    assert np.allclose(t, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())
    assert np.allclose(t, tau_d.cpu().numpy(), rtol=1e-9, atol=1e-11 * np.abs(ref).max())
    S.close()


def test_tilechol_lambda_and_batched_structure(dev):
    """Four chains of 50 keyframes with cross links (n = 1400), lambda = 0.1: against numpy's dense solve of
    (H + lambda diag H + eps I) and the library's dense solver."""
    n, pairs = _chains_and_links(per=50, links=3, seed=11)
    H, g = _gn_like(n, pairs, seed=5)
    S = ds3.TileChol(n, pairs)
    info = S.info()
    assert info["levels"] < (7 * n + 31) // 32
    tau, st = S.solve(_t(H, dev), _t(g, dev), lam=0.1)
    A = H + 0.1 * np.diag(np.diag(H)) + 1e-6 * np.eye(7 * n)
    ref = np.linalg.solve(A, -g)
    tau_d, _ = ds3.chol_ladder_solve(_t(H, dev), _t(g, dev), lam=0.1)
    t = tau.cpu().numpy()
    assert int(st.item()) == 0
    assert np.allclose(t, ref, rtol=1e-9, atol=1e-10 * np.abs(ref).max())
    assert np.allclose(t, tau_d.cpu().numpy(), rtol=1e-9, atol=1e-10 * np.abs(ref).max())
    S.close()


def test_tilechol_reads_only_the_lower_pattern(dev):
    """NaN in every entry outside the pattern's blocks and in the strict upper triangle: the result is
    bitwise the one of the clean matrix."""
    n, pairs = PATTERNS["chains_and_links"]
    H, g = _gn_like(n, pairs, seed=21)
    S = ds3.TileChol(n, pairs)
    tau0, _ = S.solve(_t(H, dev), _t(g, dev))
    Hd = H.copy()
    Hd[~_pattern_mask(n, pairs)] = np.nan
    Hd[np.triu_indices(7 * n, 1)] = np.nan
    tau1, st1 = S.solve(_t(Hd, dev), _t(g, dev), attempts=1)
    assert int(st1.item()) == 0
    assert np.array_equal(tau0.cpu().numpy(), tau1.cpu().numpy())
    S.close()


@pytest.mark.parametrize("p", [3, 60, 139, 700])
def test_tilechol_ladder_later_attempt(dev, p):
    """A negative diagonal entry at row p on top of a weakly coupled positive definite part: attempt 0 fails
    wherever p sits in the tile layout, the dense fallback's later attempt succeeds, and status and solution
    equal the oracle's dense ladder. With a pivot no epsilon can fix, every attempt fails (status -1, tau
    0), with one attempt and with six."""
    n, pairs = PATTERNS["chains_and_links"]
    rng = np.random.default_rng(p)
    Hc, g = _gn_like(n, pairs, seed=p)
    H = 0.002 * Hc + np.diag(rng.uniform(1.5, 2.5, size=7 * n))
    H[p, p] = -0.5
    S = ds3.TileChol(n, pairs)
    tau, st = S.solve(_t(H, dev), _t(g, dev))
    ref, st_ref = O.chol_ladder(H, g)
    assert st_ref == 3
    assert int(st.item()) == st_ref
    assert np.allclose(tau.cpu().numpy(), ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())
    tau1, st1 = S.solve(_t(H, dev), _t(g, dev), attempts=1)
    assert int(st1.item()) == -1 and np.all(tau1.cpu().numpy() == 0)
    H[p, p] = -1e5
    tau, st = S.solve(_t(H, dev), _t(g, dev))
    assert int(st.item()) == -1 and np.all(tau.cpu().numpy() == 0)
    S.close()


@pytest.mark.parametrize("n", [1, 5, 13])
def test_tilechol_without_pairs(dev, n):
    """No pairs: block-diagonal H. No keyframe subtree reaches the smallest alignment threshold, so the layout
    is packed and the keyframes that straddle tile boundaries chain the tiles: one level per tile."""
    H, g = _gn_like(n, [], seed=n)
    S = ds3.TileChol(n, [])
    assert S.info()["levels"] == S.info()["tiles"] == -(-7 * n // 32)
    tau, st = S.solve(_t(H, dev), _t(g, dev))
    ref, st_ref = O.chol_ladder(H, g)
    assert int(st.item()) == st_ref == 0
    assert np.allclose(tau.cpu().numpy(), ref, rtol=1e-10)
    S.close()


def test_tilechol_dense_pattern(dev):
    """Every pair of 40 keyframes (a dense factor, 280 x 280): the solve equals the dense ones."""
    n = 40
    pairs = [(a, b) for a in range(n) for b in range(a)]
    H, g = _gn_like(n, pairs, seed=40)
    S = ds3.TileChol(n, pairs)
    tau, st = S.solve(_t(H, dev), _t(g, dev), lam=0.05)
    ref, st_ref = O.chol_ladder(H, g, lam=0.05)
    assert int(st.item()) == st_ref == 0
    assert np.allclose(tau.cpu().numpy(), ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())
    S.close()


def test_tilechol_repeated_calls(dev):
    """Two different systems on one object, one after the other, and the first again (bitwise)."""
    n, pairs = PATTERNS["random"]
    S = ds3.TileChol(n, pairs)
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


def test_tilechol_small_workspace_is_refused(dev):
    n, pairs = PATTERNS["path"]
    H, g = _gn_like(n, pairs, seed=3)
    S = ds3.TileChol(n, pairs)
    ws = torch.empty(1024, dtype=torch.uint8, device=dev)
    with pytest.raises(DS3Error) as e:
        S.solve(_t(H, dev), _t(g, dev), ws=ws)
    assert e.value.code == -4
    S.close()
