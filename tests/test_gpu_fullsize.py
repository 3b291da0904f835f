"""GPU parity at the benchmark's full size and launch configuration: the batched multi-agent graph
(4 agents x 50 keyframes at 512x384 / 512x288, 800 edges), matched by one ds3_match_batch call on FP32
pointmaps and refined on BF16 pointmaps by an autotuned GN plan (persistent residual launch under a
hipGraph), exactly as bench.py times it. The oracle cannot redo the whole graph in seconds, so it
checks sampled outputs: the matches of sampled edges, and two full GN steps on ground-truth matches
(every edge, FP64, on the same BF16-rounded inputs)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

ds3 = pytest.importorskip("paper_2605_30488_amd.api")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def batched(dev):
    import bench
    g = synth.make_config(3)
    W = bench.build_workload(g, "bf16", dev)
    return g, W


def _bf16(a):
    return O.bf16_to_f32(O.bf16_round(a)).reshape(np.shape(a)).astype(np.float64)


def test_match_batch_fullsize_sampled_edges(dev, batched):
    """One batched launch set over all 800 edges (FP32 pointmaps, as the benchmark matches); 12 seeded
    sampled edges (both resolutions, intra- and inter-agent) agree with the oracle on >= 99.9% of the
    pixels either side calls valid, nu within 2e-3 and the same admission."""
    import bench
    g, W = batched
    idx, valid, nu, admit = bench.match_all(W)
    idx, valid, nu, admit = idx.cpu().numpy(), valid.cpu().numpy(), nu.cpu().numpy(), admit.cpu().numpy()
    rng = np.random.default_rng(2024)
    sample = sorted(rng.choice(len(W.edges), size=12, replace=False).tolist())
    worst = 1.0
    for e in sample:
        i, j = W.edges[e]
        Xji, Xij = g.cross_view(e)
        Hj, Wj = g.shape(j)
        sl = slice(W.idx_offsets[e], W.idx_offsets[e] + Hj * Wj)
        r = O.match_bidir(g.xyz[i], Xji, g.xyz[j], Xij, g.conf[i], g.conf[j])
        either = (r.idx_j2i >= 0) | (idx[sl] >= 0)
        agree = (r.idx_j2i == idx[sl])[either].mean()
        worst = min(worst, agree)
        print(f"edge {e} ({i}->{j}, {Hj}x{Wj}): agreement {agree:.5f} over {either.sum()} px; "
              f"nu {nu[e]} vs {r.nu}")
        assert agree >= 0.999
        assert np.allclose(nu[e], r.nu, atol=2e-3)
        assert bool(admit[e]) == r.admit
    print(f"worst agreement over sampled edges: {worst:.5f}")


def test_match_bf16_inputs_are_not_a_parity_target(dev, batched):
    """Why matching reads FP32: on BF16-rounded pointmaps (2^-9 relative, about a pixel of ray angle) the
    FP32 kernel and the FP64 oracle, given identical inputs, land in different local minima of the rough
    cost for several percent of the pixels. Recorded, with a loose floor."""
    g, W = batched
    e = 62
    i, j = W.edges[e]
    Xji, Xij = g.cross_view(e)
    (Hi, Wi), (Hj, Wj) = g.shape(i), g.shape(j)
    b = [_bf16(a) for a in (g.xyz[i], Xji, g.xyz[j], Xij, g.conf[i], g.conf[j])]
    ones = [np.concatenate([np.asarray(x, np.float32).reshape(-1, 3), np.asarray(c, np.float32).reshape(-1, 1)],
                           axis=1) for x, c in ((b[0], b[4]), (b[1], b[5]), (b[2], b[5]), (b[3], b[4]))]
    t = [torch.as_tensor(a).to(dev) for a in ones]
    got = ds3.match_bidir(t[0], t[1], t[2], t[3], (Hi, Wi), (Hj, Wj), "f32")[0].cpu().numpy()
    r = O.match_bidir(*b)
    either = (r.idx_j2i >= 0) | (got >= 0)
    agree = (r.idx_j2i == got)[either].mean()
    print(f"edge {e} on BF16-rounded inputs: agreement {agree:.5f} over {either.sum()} px")
    assert agree >= 0.9


def test_plan_fullsize_bf16_two_steps(dev, batched):
    """The autotuned batched plan on all 800 edges (BF16 storage, FP32 accumulation, FP64 solve) against
    two FP64 oracle GN steps on the same BF16-rounded inputs and ground-truth matches: poses within 1e-5
    (arithmetic-only error) and the costs within 1e-5 relative."""
    g, W = batched
    idx = g.gt_idx_all()
    flat = torch.as_tensor(np.concatenate([np.asarray(v).reshape(-1) for v in idx]), dtype=torch.int32).to(dev)
    G = ds3.Graph(W.arena, W.edges, flat, W.idx_offsets, anchors=(0,))
    start = g.poses_gt.copy()
    rng = np.random.default_rng(7)
    for k in range(1, g.n_kf):  # moderate noise around the truth, common gauge
        start[k] = O.compose(O.sim3_exp(rng.normal(size=7) * np.array([.02, .02, .02, .01, .01, .01, .01]))[0],
                             start[k])
    P = torch.as_tensor(start).to(dev)
    plan = ds3.GNPlan(G, P, autotune=True)
    cost, st = plan.run(2)
    torch.cuda.synchronize()
    og = O.Graph([_bf16(x) for x in g.xyz], [_bf16(c) for c in g.conf], g.edges, idx, anchors=(0,))
    ref = start.copy()
    ref_costs = []
    for _ in range(2):
        ref, c, s, _ = O.gn_step(og, ref)
        ref_costs.append(c)
        assert s == 0
    err = O.pose_error(P.cpu().numpy(), ref).max()
    rel = np.abs(cost.cpu().numpy() - np.array(ref_costs)) / np.array(ref_costs)
    print(f"full-size plan: {plan.info()}; pose error {err:.2e}; cost rel err {rel}")
    assert st.cpu().numpy().tolist() == [0, 0]
    assert err <= 1e-5
    assert rel.max() <= 1e-5
    plan.close()


def test_plan_fullsize_bf16_pose_error_per_agent(dev, batched):
    """The precision configuration: the batched plan on all 800 edges with BF16 pointmaps and
    confidences, FP32 accumulation and the FP64 solve, 20 iterations from the tracker-synchronised start
    on ground-truth matches, against the FP64 oracle's 20 iterations stored by
    tests/golden/make_pose_ref.py. Pose error (max over each agent's keyframes) against the oracle on the
    same BF16-rounded inputs (arithmetic only) is asserted <= 1e-5; against the oracle on the original
    FP32 inputs (total) it is printed with the oracle's own rounded-vs-unrounded distance: the rounding of
    the inputs to BF16 alone moves the FP64 solution by 1.1e-4 to 3.9e-4 per agent, above the 1e-4 that
    was aimed at, whatever the arithmetic."""
    import json
    import os
    import sys
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, here)
    from make_pose_ref import fingerprint
    ref = json.load(open(os.path.join(here, "pose_ref_batched.json")))
    g, W = batched
    idx = g.gt_idx_all()
    assert fingerprint(g, idx) == ref["fingerprint"], "the generator no longer produces the stored graph"
    flat = torch.as_tensor(np.concatenate([np.asarray(v).reshape(-1) for v in idx]), dtype=torch.int32).to(dev)
    G = ds3.Graph(W.arena, W.edges, flat, W.idx_offsets, anchors=(0,))
    P = torch.as_tensor(np.array(ref["start"])).to(dev)
    plan = ds3.GNPlan(G, P, autotune=True)
    cost, st = plan.run(ref["iters"])
    torch.cuda.synchronize()
    got = P.cpu().numpy()
    e_arith = O.pose_error(got, np.array(ref["poses_bf16"]))
    e_total = O.pose_error(got, np.array(ref["poses_f32"]))
    e_quant = O.pose_error(np.array(ref["poses_bf16"]), np.array(ref["poses_f32"]))
    agents = range(int(g.agent.max()) + 1)
    per = {name: [float(e[g.agent == a].max()) for a in agents]
           for name, e in (("arithmetic", e_arith), ("total", e_total), ("oracle_quantisation", e_quant))}
    rel = np.abs(cost.cpu().numpy() - np.array(ref["costs_bf16"])) / np.array(ref["costs_bf16"])
    print(f"pose error per agent after {ref['iters']} iterations: {per}; cost rel err max {rel.max():.2e}")
    assert st.cpu().numpy().tolist() == ref["status_bf16"]
    assert max(per["arithmetic"]) <= 1e-5
    assert rel.max() <= 1e-5
    plan.close()
