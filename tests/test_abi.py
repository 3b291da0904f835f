"""The C-ABI library loads on the CPU and exports every entry point include/ds3.h declares (no compute
calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ds3.h")
LIB = os.path.join(ROOT, "paper_2605_30488_amd", "libds3.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ds3_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2605_30488_amd import _build
        _build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_2605_30488_amd import _lib
    assert sorted(_lib.exported_names()) == declared()


def test_pure_host_entry_points(lib):
    """Calls that touch no device: parameter defaults, status strings, workspace sizing, argument
    checks that fail before any HIP call."""
    from paper_2605_30488_amd import _lib as L
    ds3 = L.load()
    p = L.MatchParams()
    ds3.ds3_default_match_params(ctypes.byref(p))
    assert (p.max_iters, p.lambda0, p.ang_tol_px, p.range_rel_tol, p.mutual_radius_px, p.q_min, p.nu_min) == \
        (10, 1e-4, 0.5, 0.10, 1, 1.5, 0.1)
    q = L.GNParams()
    ds3.ds3_default_gn_params(ctypes.byref(q))
    assert (q.sigma_ray, q.sigma_dist, q.huber_k, q.lam, q.eps0, q.eps_mult, q.max_attempts) == \
        (0.003, 10.0, 1.345, 0.0, 1e-6, 100.0, 6)
    assert ds3.ds3_version() >= 100
    assert b"invalid" in ds3.ds3_status_string(-1)
    assert ds3.ds3_match_workspace_bytes(384, 512) >= 384 * 512 * 16
    assert ds3.ds3_match_workspace_bytes(0, 512) == 0
    assert ds3.ds3_chol_workspace_bytes(1400) > 2 * 1400 * 1400 * 8
    kf = (L.Image * 2)(L.Image(48, 64, 0), L.Image(48, 64, 3072))
    ed = (L.Edge * 1)(L.Edge(0, 1, 0))
    assert ds3.ds3_gn_workspace_bytes(2, kf, 1, ed, 0) > 0
    bad = (L.Edge * 1)(L.Edge(0, 0, 0))  # self loop
    assert ds3.ds3_gn_workspace_bytes(2, kf, 1, bad, 0) == 0
    # null pointers are rejected before any device call
    assert ds3.ds3_match(None, L.Image(2, 2, 0), None, L.Image(2, 2, 0), 0, ctypes.byref(p), None, None,
                         None, None, 0, None) == -1
    assert ds3.ds3_pack_xyzc(None, None, 5, 0, None, None) == -1


def test_fuse_argument_checks_on_the_host(lib):
    """ds3_fuse rejects bad pair tables before any HIP call: negative sizes, two pairs sharing canonical
    pixels, pairs reaching past either arena, fewer poses than pairs, overlapping canonical and
    prediction arenas, misaligned arenas, a short workspace; an empty call is a no-op. (Pointers are
    never dereferenced on these paths.)"""
    from paper_2605_30488_amd import _lib as L
    ds3 = L.load()
    canon = ctypes.c_void_p(1 << 20)  # 16-byte aligned, never touched
    pred = ctypes.c_void_p(1 << 24)
    T = ctypes.c_void_p(1 << 21)
    ws_n = ds3.ds3_fuse_workspace_bytes(2)
    assert ws_n >= 2 * 32 and ds3.ds3_fuse_workspace_bytes(0) == 0
    ws = ctypes.c_void_p(1 << 22)
    nc, npd = 150, 150
    ok = (L.FusePair * 2)(L.FusePair(0, 0, 100), L.FusePair(100, 100, 50))
    overlap = (L.FusePair * 2)(L.FusePair(0, 0, 100), L.FusePair(99, 100, 50))
    neg = (L.FusePair * 1)(L.FusePair(0, 0, -1))
    past_canon = (L.FusePair * 2)(L.FusePair(0, 0, 100), L.FusePair(101, 100, 50))
    past_pred = (L.FusePair * 2)(L.FusePair(0, 0, 100), L.FusePair(100, 101, 50))
    assert ds3.ds3_fuse(canon, nc, pred, npd, overlap, 2, T, 2, ws, ws_n, None) == -1
    assert ds3.ds3_fuse(canon, nc, pred, npd, neg, 1, T, 2, ws, ws_n, None) == -1
    assert ds3.ds3_fuse(canon, nc, pred, npd, past_canon, 2, T, 2, ws, ws_n, None) == -1
    assert ds3.ds3_fuse(canon, nc, pred, npd, past_pred, 2, T, 2, ws, ws_n, None) == -1
    assert ds3.ds3_fuse(canon, nc, pred, npd, ok, 2, T, 1, ws, ws_n, None) == -1   # one pose for two pairs
    assert ds3.ds3_fuse(canon, nc, pred, 149, ok, 2, T, 2, ws, ws_n, None) == -1  # prediction arena short
    # aliasing: the prediction arena starts inside the canonical one, or is the same memory
    assert ds3.ds3_fuse(canon, nc, ctypes.c_void_p((1 << 20) + 16 * 149), npd, ok, 2, T, 2, ws, ws_n,
                        None) == -1
    assert ds3.ds3_fuse(canon, nc, canon, npd, ok, 2, T, 2, ws, ws_n, None) == -1
    assert ds3.ds3_fuse(ctypes.c_void_p((1 << 20) + 4), nc, pred, npd, ok, 2, T, 2, ws, ws_n, None) == -1
    assert ds3.ds3_fuse(canon, nc, pred, npd, ok, 2, T, 2, ws, 8, None) == -4
    assert ds3.ds3_fuse(canon, nc, pred, npd, ok, 0, T, 2, ws, ws_n, None) == 0
    assert ds3.ds3_fuse(canon, nc, pred, npd, ok, -1, T, 2, ws, ws_n, None) == -1


def test_tune_cache_directory_is_created_without_a_child_process(lib, tmp_path, monkeypatch):
    """ds3_tune_cache_reset creates the autotuner cache's missing directories (mkdir, host only) and
    removes a stale cache file."""
    from paper_2605_30488_amd import _lib as L
    ds3 = L.load()
    path = tmp_path / "a" / "b" / "c" / "tune.txt"
    monkeypatch.setenv("DS3_TUNE_CACHE", str(path))
    assert not path.parent.exists()
    assert ds3.ds3_tune_cache_reset() == 0
    assert path.parent.is_dir() and not path.exists()
    path.write_text("gfx950|bf16|cu256|196608x196608\t16 2\n")
    assert ds3.ds3_tune_cache_reset() == 0
    assert not path.exists()


def test_library_sources_start_no_child_process():
    """The library never forks or runs a shell: no system/popen/fork/exec call in its sources."""
    csrc = os.path.join(ROOT, "paper_2605_30488_amd", "csrc")
    pat = re.compile(r"\b(std::system|system|popen|fork|vfork|execl|execlp|execle|execv|execvp|execve|posix_spawn)\s*\(")
    for name in os.listdir(csrc):
        text = open(os.path.join(csrc, name)).read()
        code = re.sub(r"//[^\n]*", "", re.sub(r"/\*.*?\*/", "", text, flags=re.S))
        assert not pat.search(code), name


def test_umeyama_host_entry_point(lib):
    """ds3_umeyama (host, FP64, eq. 4) against the oracle's closed form: exact recovery of a known
    similarity, the optimum under noise, the reflection case of planar points (det(UV^T) = -1 must not
    give a reflection), and rejection of collinear points and bad arguments. No GPU involved."""
    import numpy as np
    import oracle as O
    from paper_2605_30488_amd import DS3Error, api
    rng = np.random.default_rng(12)
    y = rng.normal(size=(200, 3)) * 3.0
    T = O.sim3_exp(np.concatenate([rng.normal(size=3), rng.normal(size=3) * 0.7, [0.4]]))[0]
    x = O.transform_points(T, y)
    got = api.umeyama(x, y)
    assert np.allclose(O.pose_to_mat(got), O.pose_to_mat(T), atol=1e-12)
    xn = x + rng.normal(size=x.shape) * 0.05
    assert np.allclose(O.pose_to_mat(api.umeyama(xn, y)), O.pose_to_mat(O.umeyama(xn, y)), atol=1e-12)
    # planar y and a mirrored x: the proper rotation with S = diag(1, 1, -1)
    yp = y.copy()
    yp[:, 2] = 0.0
    xp = yp * np.array([1.0, 1.0, 1.0]) @ O.pose_to_mat(T)[:3, :3].T
    xp[:, 2] *= -1.0
    Tp = api.umeyama(xp, yp)
    R = O.pose_to_mat(Tp)[:3, :3] / Tp[7]
    assert abs(np.linalg.det(R) - 1.0) < 1e-12
    assert np.allclose(O.pose_to_mat(Tp), O.pose_to_mat(O.umeyama(xp, yp)), atol=1e-10)
    # collinear: degenerate, reported with its own code
    yl = np.outer(np.linspace(-1, 1, 50), [1.0, 2.0, 3.0])
    with pytest.raises(DS3Error) as e:
        api.umeyama(yl, yl)
    assert e.value.code == -5
    dp = ctypes.POINTER(ctypes.c_double)
    buf = np.zeros(8)
    assert lib.ds3_umeyama(None, None, 3, buf.ctypes.data_as(dp)) == -1
    one = np.zeros(3)
    assert lib.ds3_umeyama(one.ctypes.data_as(dp), one.ctypes.data_as(dp), 0, buf.ctypes.data_as(dp)) == -1


def test_track_noalloc_refuses_oversized_problems_on_the_host(lib):
    """ds3_track_noalloc sizes its scratch on the host and refuses, before any HIP call, problems that do not
    fit the static array (12 frames of 512x384 in f32 need about 72 MiB of the 64 MiB)."""
    from paper_2605_30488_amd import _lib as L
    ds3 = L.load()
    n = 12
    table = (L.TrackProblem * n)()
    for p in range(n):
        table[p] = L.TrackProblem(L.Image(384, 512, 0), L.Image(384, 512, 196608 * (p + 1)), 196608 * p)
    need = ds3.ds3_track_workspace_bytes(n, table, 0)
    assert need > 64 << 20 and ds3.ds3_track_workspace_bytes(6, table, 0) <= 64 << 20
    gp, tp = L.GNParams(), L.TrackParams()
    ds3.ds3_default_gn_params(ctypes.byref(gp))
    ds3.ds3_default_track_params(ctypes.byref(tp))
    with pytest.raises(L.DS3Error, match=f"need {need} bytes of scratch"):
        L.call("ds3_track_noalloc", None, 0, table, n, None, ctypes.byref(gp), ctypes.byref(tp), None, None, None,
               None, None)
