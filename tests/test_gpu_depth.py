"""GPU parity of the terminal segment-level depth refinement (Sec. III-E, eqs. 8-10; ds3_depth_plan_*)
against the FP64 oracle (oracle.depth): the segmentation bit for bit (integer SLIC on features computed in
float64 in the reference's operation order), the boundary table, ten Jacobi damped Newton iterations of the
segment log-scales (eta and E' per iteration), the refined pointmaps, BF16 storage, anchors, excluded
keyframes and edges without matches."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from oracle import depth as D

pytestmark = pytest.mark.gpu

ds3 = pytest.importorskip("paper_2605_30488_amd.api")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dev, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(dev)


def _bf16(arrs):
    return [O.bf16_to_f32(O.bf16_round(a)).reshape(np.shape(a)).astype(np.float64) for a in arrs]


def _setup(dev, xyz, conf, edges, idx, M, dtype="f32", anchors=(0,), **kw):
    a = ds3.build_arena(xyz, conf, dtype, dev)
    flat = _t(np.concatenate([np.asarray(v).reshape(-1) for v in idx]) if len(idx) else np.zeros(0, np.int32), dev,
              torch.int32)
    G = ds3.Graph(a, edges, flat, anchors=anchors)
    p = ds3.default_depth_params()
    p.segments_per_kf = M
    for k, v in kw.items():
        setattr(p, k, v)
    plan = ds3.DepthPlan(G, p)
    xo, co = (_bf16(xyz), _bf16(conf)) if dtype == "bf16" else (xyz, conf)
    P = D.DepthParams(segments_per_kf=M, **kw)
    prob = D.DepthProblem(xo, co, edges, idx, anchors=anchors, params=P)
    return a, plan, prob


def _check_segmentation(plan, prob, arena):
    lab = plan.labels().cpu().numpy()
    for k, (H, W, off) in enumerate(arena.images):
        want = prob.glabel(k)
        got = lab[off:off + H * W]
        assert np.array_equal(got, want), (k, int((got != want).sum()))
    assert plan.info["segments"] == prob.n_seg
    assert plan.info["valid_segments"] == int(prob.seg_valid.sum())
    assert plan.info["boundary_slots"] == len(prob.pairs)


def _check_refinement(dev, plan, prob, poses, iters=10, tol_eta=2e-6, tol_cost=1e-5):
    P = _t(poses, dev)
    costs = plan.run(P, iters).cpu().numpy()
    eta = plan.eta().cpu().numpy()
    eta_ref, costs_ref = prob.run(poses, iters=iters)
    err = np.abs(eta - eta_ref).max()
    cerr = np.max(np.abs(costs - costs_ref) / np.abs(costs_ref))
    print(f"{prob.n_seg} segment slots ({int(prob.seg_valid.sum())} valid): max |eta - eta_ref| {err:.2e} "
          f"(max |eta| {np.abs(eta_ref).max():.3f}), cost rel {cerr:.2e}; costs {costs[0]:.6e} -> {costs[-1]:.6e}")
    assert err <= tol_eta and cerr <= tol_cost
    return eta, eta_ref


def test_tiny_pair(dev):
    g = synth.make_config(1)
    idx = [g.gt_idx(0)]
    a, plan, prob = _setup(dev, g.xyz, g.conf, g.edges, idx, M=12)
    _check_segmentation(plan, prob, a)
    eta, eta_ref = _check_refinement(dev, plan, prob, g.poses_init)
    base1 = prob.base[1]
    assert np.all(eta[:base1] == 0)                 # keyframe 0 is the anchor
    assert np.abs(eta_ref[base1:]).max() > 1e-3    # the refinement moved the other keyframe's segments
    X = plan.apply().cpu().numpy()
    want = np.concatenate([x.reshape(-1, 3) for x in prob.apply(eta_ref)])
    assert np.allclose(X[:, :3], want, rtol=2e-6, atol=0)
    plan.close()


@pytest.fixture(scope="module")
def single():
    g = synth.make_config(2)
    kfs = [0, 1, 2, 3]
    sub = [e for e, (i, j) in enumerate(g.edges) if i in kfs and j in kfs]
    return g, kfs, sub


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_four_keyframes_512x384(dev, single, dtype):
    """Keyframes 0-3 of the single-agent graph and the edges among them, 200 segments per keyframe."""
    g, kfs, sub = single
    remap = {k: n for n, k in enumerate(kfs)}
    edges = [(remap[int(g.edges[e][0])], remap[int(g.edges[e][1])]) for e in sub]
    idx = [g.gt_idx(e) for e in sub]
    xyz, conf = [g.xyz[k] for k in kfs], [g.conf[k] for k in kfs]
    a, plan, prob = _setup(dev, xyz, conf, edges, idx, M=200, dtype=dtype)
    _check_segmentation(plan, prob, a)
    _check_refinement(dev, plan, prob, g.poses_gt[kfs])
    plan.close()


def test_excluded_keyframe_and_edge_without_matches(dev):
    """Keyframe 2's confidences are all below C_min (no segment), and one edge has no valid match: the
    segmentation and the refinement still agree with the oracle."""
    g = synth.make_config(3, n_agents=1, kf_per_agent=3, n_edges=3)
    xyz = list(g.xyz)
    conf = [np.array(c) for c in g.conf]
    conf[2][:] = 1.2
    idx = g.gt_idx_all()
    idx[1] = np.full_like(idx[1], -1)
    a, plan, prob = _setup(dev, xyz, conf, g.edges, idx, M=150, anchors=(1,))
    _check_segmentation(plan, prob, a)
    assert not prob.seg_valid[prob.seg_kf == 2].any()
    eta, _ = _check_refinement(dev, plan, prob, g.poses_gt, iters=5)
    assert np.all(eta[prob.seg_kf == 1] == 0) and np.all(eta[prob.seg_kf == 2] == 0)
    plan.close()


def test_set_eta_and_continue(dev):
    """A run from a given eta (set_eta) equals the oracle from the same eta; two calls of 3 iterations
    equal one of 6."""
    g = synth.make_config(1)
    idx = [g.gt_idx(0)]
    a, plan, prob = _setup(dev, g.xyz, g.conf, g.edges, idx, M=12)
    rng = np.random.default_rng(3)
    eta0 = np.where(prob.seg_valid, rng.normal(size=prob.n_seg) * 0.05, 0.0)
    plan.set_eta(_t(eta0, dev))
    P = _t(g.poses_init, dev)
    plan.run(P, 3)
    plan.run(P, 3)
    eta = plan.eta().cpu().numpy()
    ref, _ = prob.run(g.poses_init, eta=eta0, iters=6)
    ref[prob.seg_kf == 0] = eta0[prob.seg_kf == 0]
    assert np.abs(eta - ref).max() <= 2e-6
    plan.close()
