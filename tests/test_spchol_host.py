"""Host-side symbolic analysis of the block-sparse solver (ds3_spchol_analyse; no GPU): the elimination
order, the filled factor pattern, the elimination-tree levels and the product counts are recomputed here
from their definitions (minimum degree on the elimination graph with ties to the lowest id; fill = the
cliques elimination leaves; a column's level = one more than its deepest child's) and must agree exactly.
Argument errors and patterns too large for the solver's tables are refused before any device use."""
import numpy as np
import pytest

from paper_2605_30488_amd import api
from paper_2605_30488_amd._lib import DS3Error


def _adjacency(n, pairs):
    adj = [set() for _ in range(n)]
    for a, b in pairs:
        adj[a].add(b)
        adj[b].add(a)
    return adj


def _reference(n, pairs):
    """Minimum-degree order, levels and the factor's row sets, written out plainly."""
    adj = _adjacency(n, pairs)
    alive = set(range(n))
    order, rows = [], {}
    while alive:
        v = min(alive, key=lambda u: (len(adj[u]), u))
        nb = set(adj[v])
        rows[v] = nb
        for a in nb:
            adj[a] |= nb - {a}
            adj[a].discard(v)
        alive.remove(v)
        order.append(v)
    pos = {v: k for k, v in enumerate(order)}
    level = [0] * n
    for v in order:
        if rows[v]:
            p = min(rows[v], key=lambda u: pos[u])
            level[p] = max(level[p], level[v] + 1)
    perm = sorted(order, key=lambda v: level[v])  # stable: elimination position within a level
    return perm, level, rows


def _counts(n, pairs, perm):
    """Blocks, fill blocks and left-looking block products of the factor in the column order perm."""
    col = {v: c for c, v in enumerate(perm)}
    adj = _adjacency(n, pairs)
    struct = [set() for _ in range(n)]
    cur = [set(col[u] for u in adj[perm[c]]) for c in range(n)]
    for c in range(n):
        s = {x for x in cur[c] if x > c}
        struct[c] = s
        for x in s:
            cur[x] |= s - {x}
    orig = {(min(col[a], col[b]), max(col[a], col[b])) for a, b in pairs}
    blocks = n + sum(len(s) for s in struct)
    fill = sum(1 for c in range(n) for x in struct[c] if (c, x) not in orig)
    contrib = [[j for j in range(n) if k in struct[j]] for k in range(n)]
    products = 0
    for k in range(n):
        for x in [k] + sorted(struct[k]):
            products += sum(1 for j in contrib[k] if x == k or x in struct[j])
    return blocks, fill, products


def _chains_and_links(n_agents=4, per=30, links=2, seed=3):
    rng = np.random.default_rng(seed)
    n = n_agents * per
    pairs = [(a * per + k, a * per + k + 1) for a in range(n_agents) for k in range(per - 1)]
    for a in range(n_agents):
        for k in range(per):
            for _ in range(links):
                b = int(rng.integers(n_agents))
                if b == a:
                    continue
                kk = int(np.clip(k + rng.integers(-3, 4), 0, per - 1))
                pairs.append((a * per + k, b * per + kk))
    return n, pairs


PATTERNS = {
    "path": (12, [(k, k + 1) for k in range(11)]),
    "star": (9, [(0, k) for k in range(1, 9)]),
    "isolated_and_repeats": (7, [(1, 3), (3, 1), (1, 3), (5, 6)]),
    "random": (40, [tuple(p) for p in np.random.default_rng(7).integers(0, 40, size=(90, 2)) if p[0] != p[1]]),
    "chains_and_links": _chains_and_links(),
}


@pytest.mark.parametrize("name", sorted(PATTERNS))
def test_analysis_matches_definitions(name):
    n, pairs = PATTERNS[name]
    perm, level, info = api.spchol_analyse(n, pairs)
    ref_perm, ref_level, _ = _reference(n, pairs)
    assert list(perm) == ref_perm
    assert list(level) == ref_level
    blocks, fill, products = _counts(n, pairs, ref_perm)
    assert info["n_kf"] == n
    assert info["blocks"] == blocks
    assert info["fill_blocks"] == fill
    assert info["products"] == products
    assert info["levels"] == max(ref_level) + 1
    # the column order is a topological order of the elimination tree: levels never decrease
    assert all(level[perm[c]] <= level[perm[c + 1]] for c in range(n - 1))


def test_minimum_degree_cuts_the_fill_of_a_batched_pattern():
    """On four keyframe chains with cross links, the block factor keeps a small fraction of the dense
    lower triangle's n (n + 1) / 2 blocks."""
    n, pairs = _chains_and_links(per=50, links=3)
    _, _, info = api.spchol_analyse(n, pairs)
    assert info["blocks"] < 0.25 * n * (n + 1) / 2


@pytest.mark.parametrize("n,pairs", [(0, []), (1171, []), (4, [(1, 1)]), (4, [(0, 4)]), (4, [(-1, 2)])])
def test_argument_errors(n, pairs):
    with pytest.raises(DS3Error) as e:
        api.spchol_analyse(n, pairs)
    assert e.value.code == -1


def test_pattern_too_large_for_the_tables_is_refused_before_device_use():
    """A dense pattern of 120 keyframes needs far more index words than the solver keeps in LDS:
    ds3_spchol_create reports DS3_ENOSPACE from the analysis alone (no device memory is touched)."""
    n = 120
    pairs = [(a, b) for a in range(n) for b in range(a)]
    _, _, info = api.spchol_analyse(n, pairs)
    assert info["table_words"] > 28 * 1024
    with pytest.raises(DS3Error) as e:
        api.SpChol(n, pairs)
    assert e.value.code == -4
