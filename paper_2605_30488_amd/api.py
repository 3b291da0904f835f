"""Python binding of libds3: argument marshalling only. Every step runs in the library's HIP kernels;
torch provides device memory and the current stream.

Conventions (see include/ds3.h): poses are float64 (N, 8) [t, q(xyzw), s]; tangents float64 (N, 7)
(v, omega, zeta); keyframes live in an xyzc arena (float32 (P, 4) or bfloat16-as-int16 (P, 4)).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from ._lib import call

DTYPES = {"f32": L.F32, "bf16": L.BF16}


def _dt(dtype) -> int:
    if isinstance(dtype, int):
        return dtype
    return DTYPES[dtype]


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _need_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("libds3 takes device tensors")
        if t is not None and not t.is_contiguous():
            raise ValueError("libds3 takes contiguous tensors")


def default_match_params() -> L.MatchParams:
    p = L.MatchParams()
    L.load().ds3_default_match_params(C.byref(p))
    return p


def default_gn_params() -> L.GNParams:
    p = L.GNParams()
    L.load().ds3_default_gn_params(C.byref(p))
    return p


def calibrated_gn_params(K, sigma_pix=1.0, sigma_logz=0.1, base: L.GNParams | None = None) -> L.GNParams:
    """Graph-step constants of the calibrated mode (Sec. IV-C): K is (n_kf, 4) [fx, fy, cx, cy] per keyframe in
    the arena's order. The returned struct keeps its own host copy of K alive."""
    p = L.GNParams()
    if base is None:
        L.load().ds3_default_gn_params(C.byref(p))
    else:
        C.pointer(p)[0] = base
    k = (C.c_double * (4 * len(K)))(*[float(v) for row in K for v in row])
    p._K_keep = k
    p.K = C.cast(k, C.POINTER(C.c_double))
    p.sigma_pix, p.sigma_logz = float(sigma_pix), float(sigma_logz)
    return p


def version() -> int:
    return L.load().ds3_version()


# ------------------------------------------------------------------------------------------------
# Keyframe layout
# ------------------------------------------------------------------------------------------------
def pack_xyzc(xyz: torch.Tensor, conf: torch.Tensor, dtype="f32", out: torch.Tensor | None = None):
    """(P, 3) float32 + (P,) float32 -> xyzc arena: (P, 4) float32, or (P, 4) int16 holding bfloat16."""
    xyz = xyz.reshape(-1, 3).contiguous()
    conf = conf.reshape(-1).contiguous()
    _need_cuda(xyz, conf)
    n = xyz.shape[0]
    if out is None:
        out = torch.empty((n, 4), dtype=torch.float32 if _dt(dtype) == L.F32 else torch.int16,
                          device=xyz.device)
    call("ds3_pack_xyzc", _ptr(xyz), _ptr(conf), n, _dt(dtype), _ptr(out), _stream())
    return out


@dataclass
class Arena:
    """Keyframe pointmaps packed back to back, plus their image table."""
    data: torch.Tensor           # (P, 4) float32 or int16 (bfloat16 bits)
    images: list                 # [(H, W, px_offset)]
    dtype: str

    def table(self):
        arr = (L.Image * len(self.images))()
        for k, (H, W, off) in enumerate(self.images):
            arr[k] = L.Image(H, W, off)
        return arr

    def image(self, k) -> L.Image:
        H, W, off = self.images[k]
        return L.Image(H, W, off)

    def view(self, k) -> torch.Tensor:
        H, W, off = self.images[k]
        return self.data[off:off + H * W]


def build_arena(xyz_list, conf_list, dtype="f32", device="cuda") -> Arena:
    """Pack per-keyframe (H, W, 3) pointmaps and (H, W) confidences into one arena."""
    images, off = [], 0
    for x in xyz_list:
        H, W = int(x.shape[0]), int(x.shape[1])
        images.append((H, W, off))
        off += H * W
    xyz = torch.cat([torch.as_tensor(x, dtype=torch.float32).reshape(-1, 3) for x in xyz_list]).to(device)
    conf = torch.cat([torch.as_tensor(c, dtype=torch.float32).reshape(-1) for c in conf_list]).to(device)
    return Arena(pack_xyzc(xyz, conf, dtype), images, dtype)


def edge_table(edges, idx_offsets):
    arr = (L.Edge * len(edges))()
    for e, ((i, j), off) in enumerate(zip(edges, idx_offsets)):
        arr[e] = L.Edge(int(i), int(j), int(off))
    return arr


# ------------------------------------------------------------------------------------------------
# Matching
# ------------------------------------------------------------------------------------------------
def match(ref: torch.Tensor, ref_hw, qry: torch.Tensor, qry_hw, dtype="f32", params=None,
          diagnostics=False):
    """One direction (ds3_match): queries (the other view's points in the reference camera) against
    the reference's canonical pointmap; both as xyzc arenas. Returns idx (int32 Hq*Wq) and, with
    diagnostics, (p (Hq*Wq, 2) float32, iters int32)."""
    _need_cuda(ref, qry)
    P = params or default_match_params()
    Hr, Wr = ref_hw
    Hq, Wq = qry_hw
    dev = ref.device
    idx = torch.empty(Hq * Wq, dtype=torch.int32, device=dev)
    p = torch.empty((Hq * Wq, 2), dtype=torch.float32, device=dev) if diagnostics else None
    it = torch.empty(Hq * Wq, dtype=torch.int32, device=dev) if diagnostics else None
    nb = L.load().ds3_match_workspace_bytes(Hr, Wr)
    ws = _ws(nb, dev)
    call("ds3_match", _ptr(ref), L.Image(Hr, Wr, 0), _ptr(qry), L.Image(Hq, Wq, 0), _dt(dtype), C.byref(P),
         _ptr(idx), _ptr(p), _ptr(it), _ptr(ws), ws.numel(), _stream())
    return (idx, p, it) if diagnostics else idx


def match_bidir(X_ii, X_ji, X_jj, X_ij, hw_i, hw_j, dtype="f32", params=None):
    """Both directions + mutual check + nu gate (ds3_match_bidir). Returns (idx_j2i int32, valid_j uint8,
    nu float32[2] = (nu_i, nu_j), admit int32[1]) on the device."""
    _need_cuda(X_ii, X_ji, X_jj, X_ij)
    P = params or default_match_params()
    Hi, Wi = hw_i
    Hj, Wj = hw_j
    dev = X_ii.device
    idx = torch.empty(Hj * Wj, dtype=torch.int32, device=dev)
    valid = torch.empty(Hj * Wj, dtype=torch.uint8, device=dev)
    nu = torch.empty(2, dtype=torch.float32, device=dev)
    admit = torch.empty(1, dtype=torch.int32, device=dev)
    ws = _ws(L.load().ds3_match_bidir_workspace_bytes(Hi, Wi, Hj, Wj), dev)
    call("ds3_match_bidir", _ptr(X_ii), _ptr(X_ji), _ptr(X_jj), _ptr(X_ij), L.Image(Hi, Wi, 0),
         L.Image(Hj, Wj, 0), _dt(dtype), C.byref(P), _ptr(idx), _ptr(valid), _ptr(nu), _ptr(admit),
         _ptr(ws), ws.numel(), _stream())
    return idx, valid, nu, admit


def match_batch(arena: Arena, cross: torch.Tensor, cross_off, edges, idx_offsets, idx_total, params=None,
                idx_out=None, valid_out=None, ws=None, lm_steps=None, timer=None):
    """Batched bidirectional matching of every edge (ds3_match_batch). cross: xyzc arena of the
    cross-view pointmaps; cross_off[2e], cross_off[2e+1] their pixel offsets (X^j_i, X^i_j).
    Returns (idx arena int32, valid arena uint8, nu (E, 2) float32, admit (E,) int32); lm_steps, a
    device int64 tensor of one element, receives the number of LM trial steps when given; timer (a
    KernelTimer) is recorded around the launch that runs the LM queries."""
    _need_cuda(arena.data, cross)
    P = params or default_match_params()
    dev = arena.data.device
    kf = arena.table()
    et = edge_table(edges, idx_offsets)
    ne = len(edges)
    off = (C.c_int64 * (2 * ne))(*[int(v) for v in cross_off])
    idx = idx_out if idx_out is not None else torch.empty(idx_total, dtype=torch.int32, device=dev)
    valid = valid_out if valid_out is not None else torch.empty(idx_total, dtype=torch.uint8, device=dev)
    nu = torch.empty((ne, 2), dtype=torch.float32, device=dev)
    admit = torch.empty(ne, dtype=torch.int32, device=dev)
    nb = L.load().ds3_match_batch_workspace_bytes(len(arena.images), kf, ne, et)
    if ws is None or ws.numel() < nb:
        ws = _ws(nb, dev)
    call("ds3_match_batch", _ptr(arena.data), kf, len(arena.images), _ptr(cross), off, et, ne,
         _dt(arena.dtype), C.byref(P), _ptr(idx), _ptr(valid), _ptr(nu), _ptr(admit), _ptr(lm_steps),
         timer.handle if timer is not None else None, _ptr(ws), ws.numel(), _stream())
    return idx, valid, nu, admit


def match_batch_workspace(arena: Arena, edges, idx_offsets) -> torch.Tensor:
    kf = arena.table()
    et = edge_table(edges, idx_offsets)
    nb = L.load().ds3_match_batch_workspace_bytes(len(arena.images), kf, len(edges), et)
    return _ws(nb, arena.data.device)


# ------------------------------------------------------------------------------------------------
# Gauge synchronisation
# ------------------------------------------------------------------------------------------------
def gauge_align(arena: Arena, i: int, j: int, idx_j2i, valid_j, poses, ref_is_i=True, nc_min=64):
    """T* of eq. (4) for one edge (ds3_gauge_align). Returns (T (8,) float64, used_umeyama int32[1])."""
    dev = arena.data.device
    T = torch.empty(8, dtype=torch.float64, device=dev)
    used = torch.empty(1, dtype=torch.int32, device=dev)
    ws = _ws(L.load().ds3_gauge_workspace_bytes(len(arena.images)), dev)
    call("ds3_gauge_align", _ptr(arena.data), arena.image(i), _ptr(arena.data), arena.image(j),
         _dt(arena.dtype), _ptr(idx_j2i), _ptr(valid_j), _ptr(poses), i, j, int(bool(ref_is_i)), nc_min,
         _ptr(T), _ptr(used), _ptr(ws), ws.numel(), _stream())
    return T, used


def umeyama(x, y):
    """eq. (4) on the host (ds3_umeyama, float64): the pose of T* mapping the (n, 3) points y onto x.
    Raises DS3Error (code DS3_EDEGENERATE = -5) for collinear correspondences."""
    import numpy as np
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    y = np.ascontiguousarray(y, np.float64).reshape(-1, 3)
    if x.shape != y.shape:
        raise ValueError("umeyama takes two (n, 3) arrays of the same shape")
    T = np.empty(8)
    dp = C.POINTER(C.c_double)
    call("ds3_umeyama", x.ctypes.data_as(dp), y.ctypes.data_as(dp), x.shape[0], T.ctypes.data_as(dp))
    return T


def apply_gauge(poses, mask, T):
    call("ds3_apply_gauge", _ptr(poses), poses.shape[0], _ptr(mask), _ptr(T), _stream())
    return poses


def gauge_sync(poses, agent_of_kf, arena: Arena, edges, idx_offsets, idx_arena, valid_arena, admit,
               nc_min=64):
    """Component tracker of Sec. III-C over the whole graph (ds3_gauge_sync); poses updated in place.
    Returns the number of merges."""
    n = poses.shape[0]
    ag = (C.c_int32 * n)(*[int(a) for a in agent_of_kf])
    et = edge_table(edges, idx_offsets)
    links = C.c_int32(0)
    ws = _ws(L.load().ds3_gauge_workspace_bytes(n), poses.device)
    call("ds3_gauge_sync", _ptr(poses), n, ag, _ptr(arena.data), arena.table(), _dt(arena.dtype), et,
         len(edges), _ptr(idx_arena), _ptr(valid_arena), _ptr(admit), nc_min, C.byref(links), _ptr(ws),
         ws.numel(), _stream())
    return links.value


# ------------------------------------------------------------------------------------------------
# Sim(3)
# ------------------------------------------------------------------------------------------------
def sim3_exp(tau: torch.Tensor) -> torch.Tensor:
    tau = tau.reshape(-1, 7).contiguous()
    out = torch.empty((tau.shape[0], 8), dtype=torch.float64, device=tau.device)
    call("ds3_sim3_exp", _ptr(tau), _ptr(out), tau.shape[0], _stream())
    return out


def sim3_log(poses: torch.Tensor) -> torch.Tensor:
    poses = poses.reshape(-1, 8).contiguous()
    out = torch.empty((poses.shape[0], 7), dtype=torch.float64, device=poses.device)
    call("ds3_sim3_log", _ptr(poses), _ptr(out), poses.shape[0], _stream())
    return out


def sim3_update(poses: torch.Tensor, tau: torch.Tensor, fixed: torch.Tensor | None = None):
    """In place: poses[k] <- Exp(tau[k]) poses[k] except where fixed."""
    call("ds3_sim3_update", _ptr(poses), _ptr(tau), _ptr(fixed), poses.shape[0], _stream())
    return poses


# ------------------------------------------------------------------------------------------------
# Graph step
# ------------------------------------------------------------------------------------------------
class Graph:
    """A keyframe graph on the device: arena, edges (i, j) with idx offsets and the idx arena."""

    def __init__(self, arena: Arena, edges, idx_arena: torch.Tensor, idx_offsets=None, anchors=(0,)):
        self.arena = arena
        self.edges = [(int(i), int(j)) for i, j in edges]
        if idx_offsets is None:
            idx_offsets, off = [], 0
            for i, j in self.edges:
                idx_offsets.append(off)
                H, W, _ = arena.images[j]
                off += H * W
        self.idx_offsets = [int(o) for o in idx_offsets]
        self.idx = idx_arena
        self.anchors = list(anchors)
        self.kf = arena.table()
        self.et = edge_table(self.edges, self.idx_offsets)
        self.n_kf = len(arena.images)
        self.an = (C.c_int32 * max(len(self.anchors), 1))(*self.anchors)
        self._ws = None

    @property
    def dtype(self):
        return _dt(self.arena.dtype)

    def workspace(self):
        nb = L.load().ds3_gn_workspace_bytes(self.n_kf, self.kf, len(self.edges), self.et, self.dtype)
        if nb == 0:
            raise ValueError("invalid graph topology")
        if self._ws is None or self._ws.numel() < nb:
            self._ws = _ws(nb, self.arena.data.device)
        return self._ws


def gn_linearize(graph: Graph, poses, params=None):
    """Normal equations of eq. (7) at poses: (H (7N, 7N), g (7N), cost (1,), count (1,)) float64/int64."""
    P = params or default_gn_params()
    dev = poses.device
    n = 7 * graph.n_kf
    H = torch.empty((n, n), dtype=torch.float64, device=dev)
    g = torch.empty(n, dtype=torch.float64, device=dev)
    cost = torch.empty(1, dtype=torch.float64, device=dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    ws = graph.workspace()
    call("ds3_gn_linearize", _ptr(poses), graph.n_kf, graph.kf, _ptr(graph.arena.data), graph.dtype, graph.et,
         len(graph.edges), _ptr(graph.idx), C.byref(P), graph.an, len(graph.anchors), _ptr(H), _ptr(g),
         _ptr(cost), _ptr(cnt), _ptr(ws), ws.numel(), _stream())
    return H, g, cost, cnt


def sim3_gn_step(graph: Graph, poses, params=None, want_tau=False):
    """One plain-form GN step (ds3_sim3_gn_step); poses updated in place. Returns (cost at the input
    poses (1,), ladder status (1,) int32[, tau (7N,)])."""
    P = params or default_gn_params()
    dev = poses.device
    cost = torch.empty(1, dtype=torch.float64, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    tau = torch.empty(7 * graph.n_kf, dtype=torch.float64, device=dev) if want_tau else None
    ws = graph.workspace()
    call("ds3_sim3_gn_step", _ptr(poses), graph.n_kf, graph.kf, _ptr(graph.arena.data), graph.dtype, graph.et,
         len(graph.edges), _ptr(graph.idx), C.byref(P), graph.an, len(graph.anchors), _ptr(cost), _ptr(st),
         _ptr(tau), _ptr(ws), ws.numel(), _stream())
    return (cost, st, tau) if want_tau else (cost, st)


def chol_ladder_solve(H, g, lam=0.0, eps0=1e-6, mult=100.0, attempts=6):
    """(H + lam diag H + eps_r I) tau = -g with the epsilon ladder. Returns (tau, status int32[1])."""
    H = H.contiguous()
    g = g.contiguous()
    n = g.numel()
    tau = torch.empty(n, dtype=torch.float64, device=H.device)
    st = torch.empty(1, dtype=torch.int32, device=H.device)
    ws = _ws(L.load().ds3_chol_workspace_bytes(n), H.device)
    call("ds3_chol_ladder_solve", _ptr(H), _ptr(g), n, float(lam), float(eps0), float(mult), int(attempts),
         _ptr(tau), _ptr(st), _ptr(ws), ws.numel(), _stream())
    return tau, st


def _pair_array(pairs):
    p = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    return p, p.ctypes.data_as(C.POINTER(C.c_int32))


_SP_INFO = ("n_kf", "blocks", "fill_blocks", "levels", "products", "table_words")


def spchol_analyse(n_kf: int, pairs):
    """Host symbolic analysis of the keyframe-pair pattern (ds3_spchol_analyse): (perm, level, info)."""
    p, pp = _pair_array(pairs)
    perm = np.empty(max(n_kf, 1), dtype=np.int32)
    level = np.empty(max(n_kf, 1), dtype=np.int32)
    info = (C.c_int64 * 6)()
    call("ds3_spchol_analyse", int(n_kf), len(p), pp, perm.ctypes.data_as(C.POINTER(C.c_int32)),
         level.ctypes.data_as(C.POINTER(C.c_int32)), info)
    return perm[:n_kf], level[:n_kf], dict(zip(_SP_INFO, list(info)))


class SpChol:
    """Block-sparse ladder solve (ds3_spchol_*) for a fixed keyframe-pair pattern of 7x7 blocks."""

    def __init__(self, n_kf: int, pairs):
        self.n_kf = int(n_kf)
        p, pp = _pair_array(pairs)
        h = C.c_void_p()
        call("ds3_spchol_create", self.n_kf, len(p), pp, C.byref(h))
        self.handle = h

    def info(self) -> dict:
        a = (C.c_int64 * 6)()
        call("ds3_spchol_info", self.handle, a)
        return dict(zip(_SP_INFO, list(a)))

    def solve(self, H, g, lam=0.0, eps0=1e-6, mult=100.0, attempts=6, tau=None, status=None):
        """(H + lam diag H + eps_r I) tau = -g on the pattern. Returns (tau, status int32[1])."""
        n = 7 * self.n_kf
        if H.shape != (n, n) or g.numel() != n or H.dtype != torch.float64 or g.dtype != torch.float64:
            raise ValueError("H must be (7 n_kf)^2 float64 and g 7 n_kf float64")
        H = H.contiguous()
        g = g.contiguous()
        _need_cuda(H, g)
        tau = torch.empty(n, dtype=torch.float64, device=H.device) if tau is None else tau
        st = torch.empty(1, dtype=torch.int32, device=H.device) if status is None else status
        call("ds3_spchol_solve", self.handle, _ptr(H), _ptr(g), float(lam), float(eps0), float(mult),
             int(attempts), _ptr(tau), _ptr(st), _stream())
        return tau, st

    def close(self):
        if self.handle:
            L.load().ds3_spchol_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_TC_INFO = ("n_kf", "tiles", "factor_tiles", "levels", "updates", "pad_rows", "threshold")


def tilechol_analyse(n_kf: int, pairs):
    """Host analysis of the tile-sparse solver (ds3_tilechol_analyse): (kf_row0, info)."""
    p, pp = _pair_array(pairs)
    row0 = np.empty(max(n_kf, 1), dtype=np.int32)
    info = (C.c_int64 * 7)()
    call("ds3_tilechol_analyse", int(n_kf), len(p), pp, row0.ctypes.data_as(C.POINTER(C.c_int32)), info)
    return row0[:n_kf], dict(zip(_TC_INFO, list(info)))


class TileChol:
    """Tile-sparse ladder solve (ds3_tilechol_*) for a fixed keyframe-pair pattern of 7x7 blocks."""

    def __init__(self, n_kf: int, pairs):
        self.n_kf = int(n_kf)
        p, pp = _pair_array(pairs)
        h = C.c_void_p()
        call("ds3_tilechol_create", self.n_kf, len(p), pp, C.byref(h))
        self.handle = h
        self._ws = None

    def info(self) -> dict:
        a = (C.c_int64 * 7)()
        call("ds3_tilechol_info", self.handle, a)
        return dict(zip(_TC_INFO, list(a)))

    def solve(self, H, g, lam=0.0, eps0=1e-6, mult=100.0, attempts=6, tau=None, status=None, ws=None):
        """(H + lam diag H + eps_r I) tau = -g on the pattern. Returns (tau, status int32[1]). ws: the dense
        workspace (uint8 device tensor of ds3_chol_workspace_bytes(7 n_kf) bytes), kept per object if None."""
        n = 7 * self.n_kf
        if H.shape != (n, n) or g.numel() != n or H.dtype != torch.float64 or g.dtype != torch.float64:
            raise ValueError("H must be (7 n_kf)^2 float64 and g 7 n_kf float64")
        H = H.contiguous()
        g = g.contiguous()
        _need_cuda(H, g)
        if ws is None:
            if self._ws is None or self._ws.device != H.device:
                self._ws = _ws(L.load().ds3_chol_workspace_bytes(n), H.device)
            ws = self._ws
        tau = torch.empty(n, dtype=torch.float64, device=H.device) if tau is None else tau
        st = torch.empty(1, dtype=torch.int32, device=H.device) if status is None else status
        call("ds3_tilechol_solve", self.handle, _ptr(H), _ptr(g), float(lam), float(eps0), float(mult),
             int(attempts), _ptr(tau), _ptr(st), _ptr(ws), ws.numel(), _stream())
        return tau, st

    def close(self):
        if self.handle:
            L.load().ds3_tilechol_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class KernelTimer:
    """ds3_timer: HIP events that a library call records around one kernel launch on its stream."""

    def __init__(self):
        h = C.c_void_p()
        call("ds3_timer_create", C.byref(h))
        self.handle = h

    def ms(self) -> float:
        """Duration of the last recorded launch (waits for it)."""
        v = C.c_float()
        call("ds3_timer_elapsed_ms", self.handle, C.byref(v))
        return v.value

    def close(self):
        if self.handle:
            L.load().ds3_timer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GNPlan:
    """Batched form (ds3_gn_plan_*): the valid matches gathered once into a match stream, one residual
    launch over it per iteration, captured with the rest of the iteration in a hipGraph. Binds to
    `poses`, which every run updates in place. After the graph's idx (or arena) contents change, call
    refresh(). reduce_timer (a KernelTimer, kept alive by the plan) is recorded around the residual
    launch. solver: 1 the dense solve of eq. (7), 2 the block-sparse one (ds3_spchol_*), 3 the tile-sparse
    one (ds3_tilechol_*), 0 the tile-sparse one when its tree has fewer levels than the dense panels."""

    def __init__(self, graph: Graph, poses, params=None, autotune=False, px_per_thread=0, use_graph=True,
                 reduce_timer=None, unroll=0, solver=0):
        self.graph = graph
        self.poses = poses
        self.reduce_timer = reduce_timer
        P = params or default_gn_params()
        opts = L.PlanOpts(int(autotune), int(px_per_thread), int(use_graph),
                          reduce_timer.handle if reduce_timer is not None else None, int(unroll), int(solver))
        h = C.c_void_p()
        call("ds3_gn_plan_create", graph.n_kf, graph.kf, _ptr(graph.arena.data), graph.dtype, graph.et,
             len(graph.edges), _ptr(graph.idx), C.byref(P), graph.an, len(graph.anchors), C.byref(opts),
             _ptr(poses), C.byref(h), _stream())
        self.handle = h

    def run(self, iters: int):
        """Returns (cost per iteration (iters,) float64, ladder status (iters,) int32) on the device."""
        dev = self.poses.device
        cost = torch.empty(max(iters, 1), dtype=torch.float64, device=dev)
        st = torch.empty(max(iters, 1), dtype=torch.int32, device=dev)
        call("ds3_gn_plan_run", self.handle, iters, _ptr(cost), _ptr(st), _stream())
        return cost[:iters], st[:iters]

    def refresh(self):
        """Re-gather the match stream from the graph's current idx and arena contents."""
        call("ds3_gn_plan_refresh", self.handle, _stream())

    def set_timer(self, timer):
        """Record `timer` (a KernelTimer, or None) around the residual launch of each later run."""
        call("ds3_gn_plan_set_timer", self.handle, timer.handle if timer is not None else None)
        self.reduce_timer = timer

    def time_reduce(self, reps: int = 10) -> float:
        ms = C.c_float()
        call("ds3_gn_plan_time_reduce", self.handle, reps, C.byref(ms), _stream())
        return ms.value

    def info(self) -> dict:
        a = (C.c_int64 * 11)()
        call("ds3_gn_plan_info", self.handle, a, 11)
        return {"items": a[0], "px_per_thread": a[1], "px_scanned": a[2], "px_valid": a[3],
                "bytes_streaming": a[4], "bytes_stream_per_iter": a[5], "bytes_refresh": a[6], "unroll": a[7],
                "solver": {2: "sparse", 3: "tile"}.get(a[8], "dense"), "factor_blocks": a[9], "factor_levels": a[10]}

    def close(self):
        if self.handle:
            L.load().ds3_gn_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------------
# Cost and adjoint
# ------------------------------------------------------------------------------------------------
def gn_cost(graph: Graph, poses, params=None):
    P = params or default_gn_params()
    cost = torch.empty(1, dtype=torch.float64, device=poses.device)
    ws = graph.workspace()
    call("ds3_gn_cost", _ptr(poses), graph.n_kf, graph.kf, _ptr(graph.arena.data), graph.dtype, graph.et,
         len(graph.edges), _ptr(graph.idx), C.byref(P), _ptr(cost), _ptr(ws), ws.numel(), _stream())
    return cost


def gn_cost_adjoint(graph: Graph, poses, dcost=1.0, params=None, timer=None):
    """(dE/dxyz (P, 3) float32, dE/dconf (P,) float32, dE/dtau (N, 7) float64), scaled by dcost; timer (a
    KernelTimer) is recorded around the two per-pixel adjoint launches. The arena is assumed to hold only
    the graph's keyframes (every pixel is written)."""
    P = params or default_gn_params()
    dev = poses.device
    npx = graph.arena.data.shape[0]
    gx = torch.empty((npx, 3), dtype=torch.float32, device=dev)
    gc = torch.empty(npx, dtype=torch.float32, device=dev)
    gt = torch.empty((graph.n_kf, 7), dtype=torch.float64, device=dev)
    ws = graph.workspace()
    call("ds3_gn_cost_adjoint", _ptr(poses), graph.n_kf, graph.kf, _ptr(graph.arena.data), graph.dtype,
         graph.et, len(graph.edges), _ptr(graph.idx), C.byref(P), float(dcost), _ptr(gx), _ptr(gc), _ptr(gt),
         timer.handle if timer is not None else None, _ptr(ws), ws.numel(), _stream())
    return gx, gc, gt


class AdjointPlan:
    """Cost + adjoint over a graph whose matches stay fixed (ds3_adjoint_plan_*): the inverse match maps
    are built once; each run gathers both sides of every pixel (no atomics, reproducible)."""

    def __init__(self, graph: Graph, params=None):
        self.graph = graph
        self.params = params or default_gn_params()
        h = C.c_void_p()
        call("ds3_adjoint_plan_create", graph.n_kf, graph.kf, _ptr(graph.arena.data), graph.dtype, graph.et,
             len(graph.edges), _ptr(graph.idx), C.byref(self.params), C.byref(h), _stream())
        self.handle = h

    def run(self, poses, dcost=1.0, timer=None, out=None):
        """(cost (1,) float64, dE/dxyz (P, 3) float32, dE/dconf (P,) float32, dE/dtau (N, 7) float64);
        `out` may pass those four tensors to be overwritten."""
        dev = poses.device
        npx = self.graph.arena.data.shape[0]
        if out is None:
            out = (torch.empty(1, dtype=torch.float64, device=dev),
                   torch.empty((npx, 3), dtype=torch.float32, device=dev),
                   torch.empty(npx, dtype=torch.float32, device=dev),
                   torch.empty((self.graph.n_kf, 7), dtype=torch.float64, device=dev))
        cost, gx, gc, gt = out
        call("ds3_adjoint_plan_run", self.handle, _ptr(poses), float(dcost), _ptr(gx), _ptr(gc), _ptr(gt),
             _ptr(cost), timer.handle if timer is not None else None, _stream())
        return cost, gx, gc, gt

    def close(self):
        if self.handle:
            L.load().ds3_adjoint_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DenseSim3Cost(torch.autograd.Function):
    """E_global (eq. 5) as an autograd function of (xyz (P, 3), conf (P,), tau (N, 7)) at poses
    Exp(tau) T0 with tau = 0 at the evaluation point: forward packs the pointmaps into a float32 arena
    and evaluates the cost; backward runs the hand-written adjoint (per-edge recomputation)."""

    @staticmethod
    def forward(ctx, xyz, conf, tau, graph: Graph, poses0, params=None):
        arena = Arena(pack_xyzc(xyz.detach().float().contiguous(), conf.detach().float().contiguous(), "f32"),
                      graph.arena.images, "f32")
        g = Graph(arena, graph.edges, graph.idx, graph.idx_offsets, graph.anchors)
        poses = poses0.clone()
        sim3_update(poses, tau.detach().to(torch.float64).contiguous())
        cost = gn_cost(g, poses, params)
        ctx.save_for_backward(xyz, conf, tau)
        ctx.graph, ctx.poses, ctx.params = g, poses, params
        return cost.reshape(())

    @staticmethod
    def backward(ctx, dE):
        xyz, conf, tau = ctx.saved_tensors
        d = float(dE.item())
        gx, gc, gt = gn_cost_adjoint(ctx.graph, ctx.poses, d, ctx.params)
        return (gx.to(xyz.dtype).reshape(xyz.shape), gc.to(conf.dtype).reshape(conf.shape),
                gt.to(tau.dtype), None, None, None)


# ------------------------------------------------------------------------------------------------
# Ray-range tracking (Sec. III-A)
# ------------------------------------------------------------------------------------------------
def default_track_params() -> L.TrackParams:
    p = L.TrackParams()
    L.load().ds3_default_track_params(C.byref(p))
    return p


class Tracker:
    """ds3_track over a fixed problem table: problems are (keyframe, frame) image indices of `arena` with
    the frame-to-keyframe matches of problem p at idx_offsets[p] of an idx arena (H_f * W_f int32 each;
    consecutive by default). The workspace is allocated once, at the first run that uses it (runs with
    noalloc=True call ds3_track_noalloc, which takes its scratch from the library's static device array)."""

    def __init__(self, arena: Arena, problems, idx_offsets=None, params=None, track_params=None):
        self.arena = arena
        self.problems = [(int(k), int(f)) for k, f in problems]
        if idx_offsets is None:
            idx_offsets, off = [], 0
            for _, f in self.problems:
                idx_offsets.append(off)
                H, W, _ = arena.images[f]
                off += H * W
        self.idx_offsets = [int(o) for o in idx_offsets]
        self.n = len(self.problems)
        self.table = (L.TrackProblem * max(self.n, 1))()
        for p, ((k, f), off) in enumerate(zip(self.problems, self.idx_offsets)):
            self.table[p] = L.TrackProblem(arena.image(k), arena.image(f), off)
        self.params = params or default_gn_params()
        self.track_params = track_params or default_track_params()
        self.ws = None

    def workspace_bytes(self) -> int:
        return int(L.load().ds3_track_workspace_bytes(self.n, self.table, _dt(self.arena.dtype)))

    def run(self, idx: torch.Tensor, T: torch.Tensor, timer=None, noalloc=False):
        """T: (n, 8) float64 starting poses, updated in place. Returns (E_track (n,) float64, trial steps
        (n,) int32, ladder status (n,) int32) on the device."""
        _need_cuda(idx, T)
        if idx.dtype != torch.int32 or T.dtype != torch.float64 or tuple(T.shape) != (self.n, 8):
            raise ValueError("track takes int32 matches and (n, 8) float64 poses")
        need = max((o + self.arena.images[f][0] * self.arena.images[f][1]
                    for o, (_, f) in zip(self.idx_offsets, self.problems)), default=0)
        if idx.numel() < need:
            raise ValueError("the idx arena is shorter than the problem table needs")
        dev = T.device
        cost = torch.empty(max(self.n, 1), dtype=torch.float64, device=dev)
        trials = torch.empty(max(self.n, 1), dtype=torch.int32, device=dev)
        status = torch.empty(max(self.n, 1), dtype=torch.int32, device=dev)
        if noalloc:
            if timer is not None:
                raise ValueError("ds3_track_noalloc records no timer")
            call("ds3_track_noalloc", _ptr(self.arena.data), _dt(self.arena.dtype), self.table, self.n, _ptr(idx),
                 C.byref(self.params), C.byref(self.track_params), _ptr(T), _ptr(cost), _ptr(trials),
                 _ptr(status), _stream())
            return cost[:self.n], trials[:self.n], status[:self.n]
        if self.ws is None:
            self.ws = _ws(self.workspace_bytes(), self.arena.data.device)
        call("ds3_track", _ptr(self.arena.data), _dt(self.arena.dtype), self.table, self.n, _ptr(idx),
             C.byref(self.params), C.byref(self.track_params), _ptr(T), _ptr(cost), _ptr(trials), _ptr(status),
             timer.handle if timer is not None else None, _ptr(self.ws), self.ws.numel(), _stream())
        return cost[:self.n], trials[:self.n], status[:self.n]


def track(arena: Arena, problems, idx: torch.Tensor, T: torch.Tensor, idx_offsets=None, params=None,
          track_params=None):
    """One ds3_track call (see Tracker.run)."""
    return Tracker(arena, problems, idx_offsets, params, track_params).run(idx, T)


# ------------------------------------------------------------------------------------------------
# Terminal segment-level depth refinement (Sec. III-E, eqs. 8-10)
# ------------------------------------------------------------------------------------------------
def default_depth_params() -> L.DepthParams:
    p = L.DepthParams()
    L.load().ds3_default_depth_params(C.byref(p))
    return p


class DepthPlan:
    """ds3_depth_plan_*: segments the pristine keyframes of `graph.arena` at creation (labels, boundary
    table, eta = 0), then run(poses, iters) takes Jacobi damped Newton steps of the segment log-scales."""

    def __init__(self, graph: Graph, params=None):
        self.graph = graph
        self.params = params or default_depth_params()
        h = C.c_void_p()
        call("ds3_depth_plan_create", graph.n_kf, graph.kf, _ptr(graph.arena.data), graph.dtype, graph.et,
             len(graph.edges), _ptr(graph.idx), graph.an, len(graph.anchors), C.byref(self.params), C.byref(h),
             _stream())
        self.handle = h
        self.info = self._info()

    def _info(self) -> dict:
        a = (C.c_int64 * 6)()
        call("ds3_depth_plan_info", self.handle, a, 6)
        return {"segments": a[0], "valid_segments": a[1], "boundary_slots": a[2], "tiles": a[3],
                "px_scanned": a[4], "arena_px": a[5]}

    def run(self, poses: torch.Tensor, iters: int, timer=None):
        """Returns E' at each iteration's input eta ((iters,) float64, device)."""
        _need_cuda(poses)
        cost = torch.empty(max(iters, 1), dtype=torch.float64, device=poses.device)
        call("ds3_depth_plan_run", self.handle, _ptr(poses), iters, _ptr(cost),
             timer.handle if timer is not None else None, _stream())
        return cost[:iters]

    def labels(self) -> torch.Tensor:
        out = torch.empty(self.info["arena_px"], dtype=torch.int32, device=self.graph.arena.data.device)
        call("ds3_depth_plan_get", self.handle, _ptr(out), None, _stream())
        return out

    def eta(self) -> torch.Tensor:
        out = torch.empty(self.info["segments"], dtype=torch.float64, device=self.graph.arena.data.device)
        call("ds3_depth_plan_get", self.handle, None, _ptr(out), _stream())
        return out

    def set_eta(self, eta: torch.Tensor):
        _need_cuda(eta)
        if eta.dtype != torch.float64 or eta.numel() != self.info["segments"]:
            raise ValueError("eta: float64, one entry per segment slot")
        call("ds3_depth_plan_set_eta", self.handle, _ptr(eta), _stream())

    def apply(self) -> torch.Tensor:
        """The refined pointmaps X_init exp(eta) as a float32 (P, 4) xyzc arena."""
        out = torch.empty((self.info["arena_px"], 4), dtype=torch.float32, device=self.graph.arena.data.device)
        call("ds3_depth_plan_apply", self.handle, _ptr(out), _stream())
        return out

    def close(self):
        if self.handle:
            L.load().ds3_depth_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------------
# Canonical pointmap fusion (eq. 2)
# ------------------------------------------------------------------------------------------------
class FusePlan:
    """A fixed pair table for ds3_fuse, uploaded through a workspace owned by the plan. pairs: rows
    (canon_off, pred_off, n_px) in pixels."""

    def __init__(self, pairs, device):
        rows = [tuple(int(v) for v in p) for p in pairs]
        self.n = len(rows)
        self.table = (L.FusePair * max(self.n, 1))(*[L.FusePair(*r) for r in rows])
        self.ws = _ws(L.load().ds3_fuse_workspace_bytes(self.n), device)

    def run(self, canon: torch.Tensor, pred: torch.Tensor, T: torch.Tensor):
        """In place on canon ((N, 4) float32 xyzc): X-hat <- (C-hat X-hat + C T x) / (C-hat + C),
        C-hat <- C-hat + C per pixel of every pair; pred (M, 4) float32 xyzc in the frames' cameras; T
        (n_pairs, 8) float64 poses mapping each frame into its keyframe."""
        _need_cuda(canon, pred, T)
        if canon.dtype != torch.float32 or pred.dtype != torch.float32 or T.dtype != torch.float64:
            raise ValueError("fuse takes float32 xyzc arenas and float64 poses")
        if canon.dim() != 2 or canon.shape[1] != 4 or pred.dim() != 2 or pred.shape[1] != 4:
            raise ValueError("fuse takes (N, 4) xyzc arenas")
        if not (canon.is_contiguous() and pred.is_contiguous() and T.is_contiguous()):
            raise ValueError("fuse takes contiguous tensors")
        if T.dim() != 2 or T.shape[1] != 8:
            raise ValueError("fuse takes (n_pairs, 8) poses")
        call("ds3_fuse", _ptr(canon), canon.shape[0], _ptr(pred), pred.shape[0], self.table, self.n, _ptr(T),
             T.shape[0], _ptr(self.ws), self.ws.numel(), _stream())
        return canon


def fuse(canon: torch.Tensor, pred: torch.Tensor, pairs, T: torch.Tensor):
    """One ds3_fuse call (eq. 2) with a fresh pair table; see FusePlan.run."""
    return FusePlan(pairs, canon.device).run(canon, pred, T)
