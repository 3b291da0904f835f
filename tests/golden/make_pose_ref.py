"""Writes pose_ref_batched.json: the FP64 oracle's Gauss-Newton solution of the batched multi-agent
graph (4 agents x 50 keyframes, 512x384 / 512x288, 800 edges) on its original FP32 inputs and on the
same inputs rounded to BF16 (round to nearest even), 20 iterations each, from one common start.

The start is the generator's initial poses (noisy ground truth under independent per-agent gauges)
after the oracle's component tracker (Sec. III-C, eq. 4) on the ground-truth matches; every edge whose
ground-truth matches cover at least 10% of keyframe j counts as admitted. The matches are the
generator's projections (never the GPU's). The GPU tests and the benchmark run their BF16 plan from the
stored start on the same matches and compare with the stored solutions: the distance to the FP32
solution is the total error, the distance to the BF16 one the arithmetic-only error.

It calls only ``oracle`` and ``synth``. A fingerprint of the inputs is stored with the result so that a
reader can tell whether the generator still produces the same graph. Run: python tests/golden/make_pose_ref.py
(a few minutes on 8 cores).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

ITERS = 20
OUT = os.path.join(HERE, "pose_ref_batched.json")


def fingerprint(g, idx) -> str:
    h = hashlib.sha256()
    for a in g.xyz + g.conf + list(idx):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(np.ascontiguousarray(g.poses_init).tobytes())
    h.update(np.ascontiguousarray(g.edges).tobytes())
    return h.hexdigest()[:16]


def bf16_inputs(g):
    xyz = [O.bf16_to_f32(O.bf16_round(x)).reshape(x.shape).astype(np.float64) for x in g.xyz]
    conf = [O.bf16_to_f32(O.bf16_round(c)).reshape(c.shape).astype(np.float64) for c in g.conf]
    return xyz, conf


def start_poses(g, idx):
    admitted = [bool((i >= 0).mean() >= 0.1) for i in idx]
    matches = [(i, (i >= 0).astype(np.uint8)) for i in idx]
    p0, links = O.gauge_sync(g.poses_init, g.agent, g.edges, admitted, matches, g.xyz)
    return p0, admitted, links


def main():
    t0 = time.time()
    g = synth.make_config(3)
    idx = g.gt_idx_all()
    p0, admitted, links = start_poses(g, idx)
    print(f"graph + tracker in {time.time() - t0:.1f}s ({len(links)} merges)", flush=True)
    res = {"what": "FP64 oracle GN solutions of the batched graph (config seed 1003), FP32 and BF16 inputs",
           "cite": "eqs. (1), (5)-(7); Sec. III-C tracker for the start; BF16 round to nearest even",
           "iters": ITERS, "fingerprint": fingerprint(g, idx), "admitted": admitted,
           "start": p0.tolist()}
    xb, cb = bf16_inputs(g)
    for name, (xyz, conf) in {"f32": (g.xyz, g.conf), "bf16": (xb, cb)}.items():
        og = O.Graph(xyz, conf, g.edges, idx, anchors=(0,))
        p = p0.copy()
        costs, status = [], []
        for it in range(ITERS):
            t1 = time.time()
            p, c, st, _ = O.gn_step(og, p)
            costs.append(c)
            status.append(int(st))
            print(f"{name} iteration {it}: cost {c:.9e} status {st} ({time.time() - t1:.1f}s)", flush=True)
        res[f"poses_{name}"] = p.tolist()
        res[f"costs_{name}"] = costs
        res[f"status_{name}"] = status
    e = O.pose_error(np.array(res["poses_bf16"]), np.array(res["poses_f32"]))
    res["quantisation_error_max"] = float(e.max())
    res["quantisation_error_per_agent"] = [float(e[g.agent == a].max()) for a in range(int(g.agent.max()) + 1)]
    print("oracle quantisation error (bf16 vs f32 inputs) per agent:", res["quantisation_error_per_agent"])
    with open(OUT, "w") as f:
        json.dump(res, f)
    print(f"wrote {OUT} in {time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
