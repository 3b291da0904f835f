"""GPU parity of the ray-range tracker (ds3_track: E_track of Sec. III-A with LM damping) against the
oracle's tracker (oracle.track, FP64) on the same inputs: exact correspondences, the tiny synthetic pair
from the identity and from a far start that forces rejected trials, a batch of 40 problems over the
single-agent graph's keyframe pairs (512x384, FP32 and BF16 storage), mixed resolutions, and problems
without matches."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.helpers import exact_graph

pytestmark = pytest.mark.gpu

ds3 = pytest.importorskip("paper_2605_30488_amd.api")

IDENT = np.array([0, 0, 0, 0, 0, 0, 1, 1.0])


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dev, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(dev)


def _bf16(a):
    return O.bf16_to_f32(O.bf16_round(a)).reshape(np.shape(a)).astype(np.float64)


def _run(dev, xyz, conf, problems, idx_list, T0, dtype="f32", tp=None):
    a = ds3.build_arena(xyz, conf, dtype, dev)
    idx = _t(np.concatenate([np.asarray(v).reshape(-1) for v in idx_list]), dev, torch.int32)
    T = _t(np.asarray(T0).reshape(-1, 8), dev)
    trk = ds3.Tracker(a, problems, track_params=tp)
    cost, trials, status = trk.run(idx, T)
    torch.cuda.synchronize()
    return T.cpu().numpy(), cost.cpu().numpy(), trials.cpu().numpy(), status.cpu().numpy()


def test_exact_correspondences(dev):
    xyz, conf, edges, idx, gt = exact_graph(n_kf=2, H=40, W=120, seed=81, frac_valid=0.9)  # 2 segments
    xyz = [np.asarray(x, np.float32) for x in xyz]
    conf = [np.asarray(c, np.float32) for c in conf]
    rng = np.random.default_rng(2)
    tau = np.concatenate([rng.normal(size=3) * 0.2, rng.normal(size=3) * 0.1, [0.05]])
    T0 = O.sim3_update(gt[1][None], tau[None])[0]
    T, cost, trials, st = _run(dev, xyz, conf, [(0, 1)], [idx[0]], T0)
    r = O.track(xyz[0], conf[0], xyz[1], conf[1], idx[0], T0)
    err_gt = O.pose_error(T, gt[1][None])[0]
    print(f"exact: gpu trials {trials[0]} oracle {r.trials}; pose error vs truth {err_gt:.2e}")
    assert err_gt <= 1e-5 and O.pose_error(T, r.pose[None])[0] <= 1e-5
    assert st[0] >= 0


@pytest.mark.parametrize("start", ["identity", "far"])
def test_tiny_pair_against_oracle(dev, start):
    """The 64x48 pair with ground-truth matches. 'far': about 3 rad from the truth with no initial
    damping, where the oracle rejects five trials in a row before it converges."""
    g = synth.make_config(1)
    idx = g.gt_idx(0)
    T_gt = O.relative(g.poses_gt[0], g.poses_gt[1])
    tp_o = O.TrackParams()
    if start == "identity":
        T0 = IDENT.copy()
    else:
        rng = np.random.default_rng(0)
        tau = np.concatenate([rng.normal(size=3) * 3, rng.normal(size=3) * 1.2, [rng.normal() * 1.0]])
        T0 = O.sim3_update(T_gt[None], tau[None])[0]
        tp_o = O.TrackParams(lambda0=0.0, max_trials=30)
    tp = ds3.default_track_params()
    tp.lambda0, tp.max_trials = tp_o.lambda0, tp_o.max_trials
    T, cost, trials, st = _run(dev, g.xyz, g.conf, [(0, 1)], [idx], T0, tp=tp)
    r = O.track(g.xyz[0], g.conf[0], g.xyz[1], g.conf[1], idx, T0, tp=tp_o)
    err = O.pose_error(T, r.pose[None])[0]
    print(f"{start}: trials gpu {trials[0]} oracle {r.trials} ({''.join('A' if a else 'r' for a in r.accepted)}); "
          f"pose error {err:.2e}; cost {cost[0]:.6e} vs {r.cost:.6e}")
    assert err <= 1e-5
    assert abs(cost[0] - r.cost) <= 1e-4 * r.cost


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batch_of_keyframe_pairs(dev, dtype):
    """40 problems in one call: each edge (i, j) of the single-agent graph (20 keyframes 512x384) tracks
    keyframe j against keyframe i on its ground-truth matches from the noisy relative pose. Every pose
    within 1e-5 of the oracle's tracker on the same (for bf16: the same rounded) inputs."""
    g = synth.make_config(2)
    idx = g.gt_idx_all()
    problems = [(int(i), int(j)) for i, j in g.edges]
    T0 = np.stack([O.relative(g.poses_init[i], g.poses_init[j]) for i, j in problems])
    T, cost, trials, st = _run(dev, g.xyz, g.conf, problems, idx, T0, dtype=dtype)
    xyz = [_bf16(x) for x in g.xyz] if dtype == "bf16" else g.xyz
    conf = [_bf16(c) for c in g.conf] if dtype == "bf16" else g.conf
    worst, worst_c = 0.0, 0.0
    for p, (i, j) in enumerate(problems[::4]):
        q = 4 * p
        r = O.track(xyz[i], conf[i], xyz[j], conf[j], idx[q], T0[q])
        worst = max(worst, O.pose_error(T[q][None], r.pose[None])[0])
        worst_c = max(worst_c, abs(cost[q] - r.cost) / r.cost)
    print(f"{dtype}: 10 of 40 problems checked; worst pose error {worst:.2e}, cost {worst_c:.2e}; "
          f"trials {trials.tolist()}")
    assert worst <= 1e-5 and worst_c <= 1e-4
    assert np.all(st >= 0)


def test_mixed_resolution_and_empty_problems(dev):
    """Two 288x512 frames against 384x512 keyframes in one call, next to a problem whose matches are all
    -1 (pose unchanged, cost 0, every trial rejected); then the same call with zero trials."""
    g = synth.make_config(3, n_agents=2, kf_per_agent=3, n_edges=6)
    idx_all = g.gt_idx_all()
    cand = [(e, int(i), int(j)) for e, (i, j) in enumerate(g.edges) if g.shape(i) != g.shape(j)][:2]
    assert len(cand) == 2
    problems = [(i, j) for _, i, j in cand] + [(0, 1)]
    idx = [idx_all[e] for e, _, _ in cand] + [np.full(g.shape(1)[0] * g.shape(1)[1], -1, np.int32)]
    rng = np.random.default_rng(5)
    T0 = []
    for i, j in problems:
        T = O.relative(g.poses_gt[i], g.poses_gt[j])
        tau = np.concatenate([rng.normal(size=3) * 0.05, rng.normal(size=3) * 0.02, [0.02]])
        T0.append(O.sim3_update(T[None], tau[None])[0])
    T0 = np.stack(T0)
    T, cost, trials, _ = _run(dev, g.xyz, g.conf, problems, idx, T0)
    for p, (i, j) in enumerate(problems[:2]):
        r = O.track(g.xyz[i], g.conf[i], g.xyz[j], g.conf[j], idx[p], T0[p])
        assert O.pose_error(T[p][None], r.pose[None])[0] <= 1e-5, p
    assert np.array_equal(T[2], T0[2]) and cost[2] == 0.0 and trials[2] == 20
    tp = ds3.default_track_params()
    tp.max_trials = 0
    T2, cost2, trials2, _ = _run(dev, g.xyz, g.conf, problems, idx, T0, tp=tp)
    assert np.array_equal(T2, T0) and np.all(trials2 == 0)
