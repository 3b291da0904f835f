"""Pins of the oracle's projective ray matching (Sec. III-A "Learned geometry") and its bidirectional
verification (Sec. III-B).

Independent pins: identity views; brute-force nearest reference ray; a brute-force sub-pixel grid search
of the same bilinear cost; the pinhole closed form of the generator's camera (which the method never
sees); constructed invalid cases; hand-made mutual-check tables."""
import numpy as np
import pytest

import oracle as O
import synth


@pytest.fixture(scope="module")
def pair():
    g = synth.make_config(1)
    Xji, Xij = g.cross_view(0)
    return g, Xji, Xij


def test_identity_view_matches_itself(pair):
    g, _, _ = pair
    r = O.match(g.xyz[0], g.xyz[0])
    assert np.array_equal(r.idx, np.arange(r.idx.size, dtype=np.int32))


def test_brute_force_nearest_ray(pair):
    """round(p*) equals the discrete nearest reference ray for every valid query more than 0.1 px from
    a rounding boundary (closer than that the angular Voronoi cells of the reference grid are sheared
    away from the pixel squares); a transposed or shifted index fails almost every pixel."""
    g, Xji, _ = pair
    r = O.match(g.xyz[0], Xji)
    ref = g.xyz[0].reshape(-1, 3).astype(np.float64)
    rays = ref / np.linalg.norm(ref, axis=1, keepdims=True)
    q = Xji.reshape(-1, 3).astype(np.float64)
    ok = r.idx >= 0
    t = q[ok] / np.linalg.norm(q[ok], axis=1, keepdims=True)
    bf = np.argmin(((rays[None] - t[:, None]) ** 2).sum(-1), axis=1)
    p = r.p[ok]
    marg = np.minimum(np.abs(p[:, 0] - np.floor(p[:, 0]) - 0.5), np.abs(p[:, 1] - np.floor(p[:, 1]) - 0.5))
    far = marg > 0.1
    assert far.sum() > 1000
    assert np.array_equal(bf[far], r.idx[ok][far])
    assert (bf != r.idx[ok]).mean() < 0.03


def _bilinear_cost(rays, H, W, t, u, v):
    u0 = np.clip(np.floor(u).astype(int), 0, W - 2)
    v0 = np.clip(np.floor(v).astype(int), 0, H - 2)
    fu, fv = u - u0, v - v0
    R = rays.reshape(H, W, 3)
    s = ((1 - fu) * (1 - fv))[..., None] * R[v0, u0] + (fu * (1 - fv))[..., None] * R[v0, u0 + 1] + \
        ((1 - fu) * fv)[..., None] * R[v0 + 1, u0] + (fu * fv)[..., None] * R[v0 + 1, u0 + 1]
    return ((s - t) ** 2).sum(-1)


def test_lm_reaches_the_continuous_minimum(pair):
    """The LM optimum is the minimiser of the bilinear cost: no point of a 1/64-px grid (+-1.5 px around
    it) has a lower cost by more than rounding. Optima clamped onto the image border are excluded: there
    the step is a clamped unconstrained step, not a projection onto the border."""
    g, Xji, _ = pair
    r = O.match(g.xyz[0], Xji)
    H, W = g.xyz[0].shape[:2]
    ref = g.xyz[0].reshape(-1, 3).astype(np.float64)
    rays = ref / np.linalg.norm(ref, axis=1, keepdims=True)
    q = Xji.reshape(-1, 3).astype(np.float64)
    rng = np.random.default_rng(0)
    interior = (r.p[:, 0] > 0) & (r.p[:, 0] < W - 1) & (r.p[:, 1] > 0) & (r.p[:, 1] < H - 1)
    valid = np.nonzero((r.idx >= 0) & interior)[0]
    off = np.arange(-96, 97) / 64.0
    for n in rng.choice(valid, 60, replace=False):
        t = q[n] / np.linalg.norm(q[n])
        uu, vv = np.meshgrid(np.clip(r.p[n, 0] + off, 0, W - 1), np.clip(r.p[n, 1] + off, 0, H - 1))
        c = _bilinear_cost(rays, H, W, t, uu, vv)
        c_star = _bilinear_cost(rays, H, W, t, np.array([r.p[n, 0]]), np.array([r.p[n, 1]]))[0]
        assert c_star <= c.min() + 1e-12


@pytest.mark.parametrize("cfg", [1, 2])
def test_pinhole_closed_form(cfg):
    """For a pinhole-generated reference the optimum is the projection K x / x_z up to the bias of
    bilinearly interpolating unit rays (about 2e-3 px at 64x48, 3e-4 px at 512x384)."""
    g = synth.make_config(cfg)
    e = 0
    i, j = g.edges[e]
    Xji, _ = g.cross_view(e)
    if cfg == 2:  # a sampled block of queries keeps this fast
        Xji = Xji[100:160, 150:250]
    r = O.match(g.xyz[i], Xji)
    cam = g.cams[i]
    x = Xji.reshape(-1, 3).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = cam.f * x[:, 0] / x[:, 2] + cam.cx
        v = cam.f * x[:, 1] / x[:, 2] + cam.cy
    inside = (u > 0.01) & (u < cam.W - 1.01) & (v > 0.01) & (v < cam.H - 1.01)
    sel = (r.idx >= 0) & inside
    assert sel.sum() > 0.5 * sel.size
    dev = np.maximum(np.abs(r.p[sel, 0] - u[sel]), np.abs(r.p[sel, 1] - v[sel]))
    assert dev.max() < (2.5e-3 if cfg == 1 else 4e-4)


def test_invalid_cases(pair):
    g, Xji, _ = pair
    # wrong range: every surface of the reference is 20x farther than the queries, test (iii) fails
    r = O.match(g.xyz[0], Xji * 0.05)
    assert np.all(r.idx < 0)
    # behind the camera: the ray cannot be matched
    r = O.match(g.xyz[0], -Xji)
    assert np.all(r.idx < 0)
    # query holes
    q = Xji.copy()
    q[:, :5] = 0.0
    q[:, 5] = np.nan
    r = O.match(g.xyz[0], q)
    assert np.all(r.idx.reshape(q.shape[:2])[:, :6] < 0)
    # a hole in the reference invalidates queries whose final cell touches it
    r0 = O.match(g.xyz[0], Xji)
    n = int(np.nonzero(r0.idx >= 0)[0][len(r0.idx) // 3])
    ref = g.xyz[0].copy().reshape(-1, 3)
    ref[r0.idx[n]] = 0.0
    r1 = O.match(ref.reshape(g.xyz[0].shape), Xji)
    assert r1.idx[n] == -1


def test_mutual_table():
    """Hand-made 2x3 (i) and 2x2 (j) grids."""
    P = O.MatchParams.default()
    P.q_min = 1.5
    # j -> i: n=0->m=0, n=1->m=2, n=2->m=5 (round trip lands 2 px away), n=3 invalid
    idx_ji = np.array([0, 2, 5, -1], np.int32)
    # i -> j over the 6 pixels of i (2 rows x 3 cols)
    idx_ij = np.array([0, -1, 1, 3, -1, 0], np.int32)
    ci = np.array([1.0, 1.0, 4.0, 1.0, 1.0, 1.0])
    cj = np.array([4.0, 1.0, 1.0, 1.0])
    out, valid, nu, admit = O.mutual(idx_ji, idx_ij, (2, 3), (2, 2), ci, cj, P)
    # n=2: m=5 -> n'=0; Chebyshev((0,0),(0,1)) = 1 -> valid with radius 1
    assert valid.tolist() == [1, 1, 1, 0]
    assert out.tolist() == [0, 2, 5, -1]
    # q: n0: sqrt(1*4)=2 >= 1.5; n1: sqrt(4*1)=2; n2: sqrt(1*1)=1 < 1.5
    assert nu[1] == pytest.approx(2 / 4)
    # i side: m0 -> n0 -> m0 ok q=2; m2 -> n1 -> m2 ok q=2; m3 -> n3 -> invalid; m5 -> n0 -> m0:
    # Chebyshev((2,1),(0,0)) = 2 > 1 -> not counted
    assert nu[0] == pytest.approx(2 / 6)
    assert admit
    P.mutual_radius_px = 0
    out, valid, nu, admit = O.mutual(idx_ji, idx_ij, (2, 3), (2, 2), ci, cj, P)
    assert valid.tolist() == [1, 1, 0, 0]


def test_bidirectional_symmetry(pair):
    g, Xji, Xij = pair
    a = O.match_bidir(g.xyz[0], Xji, g.xyz[1], Xij, g.conf[0], g.conf[1])
    b = O.match_bidir(g.xyz[1], Xij, g.xyz[0], Xji, g.conf[1], g.conf[0])
    assert np.allclose(a.nu, b.nu[::-1])
    assert a.admit == b.admit
    assert 0.3 < a.nu.min() and a.admit


def test_matches_agree_with_ground_truth(pair):
    """Noise-free prior: the verified matches are the generator's projective ground truth except at
    rounding ties and at the occlusion tolerance boundary."""
    g, Xji, Xij = pair
    a = O.match_bidir(g.xyz[0], Xji, g.xyz[1], Xij, g.conf[0], g.conf[1])
    gt = g.gt_idx(0)
    both = (gt >= 0) & (a.idx_j2i >= 0)
    assert both.sum() > 0.6 * gt.size
    assert (a.idx_j2i[both] == gt[both]).mean() > 0.995


def test_bf16_round_to_nearest_even():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.0, np.inf,
                  3.4028234e38, 0.0, -0.0, 1e-40], np.float32)
    b = O.bf16_round(x)
    # 1e-40 is the subnormal 0x000116C2: its low half is below the halfway point -> 0x0001
    assert b.tolist() == [0x3F80, 0x3F80, 0x3F82, 0x3F81, 0xC000, 0x7F80, 0x7F80, 0x0000, 0x8000, 0x0001]
    nan = O.bf16_round(np.array([np.nan], np.float32))[0]
    assert (nan & 0x7F80) == 0x7F80 and (nan & 0x7F) != 0
    assert np.array_equal(O.bf16_to_f32(np.array([0x3F80, 0xC000], np.uint16)), [1.0, -2.0])
