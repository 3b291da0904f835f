"""Seeded synthetic keyframe graphs shaped like the paper's workloads (CoMo3R-SLAM, Sec. IV).

This module only MAKES INPUTS. It holds none of the method's arithmetic: it ray-casts a scene with a
pinhole camera that the method never sees, expresses hit points in camera frames with plain rotation
matrices, and picks edges by ground-truth visibility. Both the FP64 oracle and the HIP library are fed
from here; neither is imported.

Scene: a ground plane and two walls (random orientation), five boxes (sides 0.5-3 m, yawed) around the
origin, inside a background sphere, so every pixel hits something at 2-20 m and no pixel is a hole.
Keyframe k: pose (R_k, t_k, s_k), T_WC = [s_k R_k, t_k]; canonical pointmap X_k = metric hits / s_k
(monocular scale); confidence ~ U(1, 5) i.i.d. The learned prior's cross-view pointmap X^j_i is the
noise-free stand-in T_i^-1 T_j X_j, computed from the world hit points.

Configurations (seed = 1000 + number unless given):
  1  tiny: 2 keyframes 64x48, GT offset (rot <= 15 deg, trans <= 1 m, scale 0.8-1.25), 1 edge
  2  single agent: 20 keyframes 512x384 on a loop, 40 edges (19 sequential + 21 loop), pose noise
  3  batched: 4 agents x 50 keyframes, agents 0/2 at 512x384 and 1/3 at 512x288, 800 edges
     (196 sequential + 604 inter-agent by overlap), per-edge valid band U(0.3, 1), per-agent gauges
  4  = 3 (the BF16 rounding is applied by the consumer)
  5  long horizon: 4 agents x 250 keyframes 512x384, 4000 edges (996 sequential + 3004 by overlap)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

try:  # ray casting runs on torch when present (multi-threaded CPU or a GPU); numpy otherwise
    import torch
except ImportError:  # pragma: no cover
    torch = None

_DEVICE = None


def set_device(dev):
    """Device for the bulk ray casting ('cpu', 'cuda', ...); None picks cuda when available."""
    global _DEVICE
    _DEVICE = dev


def _device():
    if torch is None:
        return None
    if _DEVICE is not None:
        return torch.device(_DEVICE)
    return torch.device("cuda") if torch.cuda.is_available() else torch.device("cpu")

__all__ = ["SynthGraph", "make_config", "make_pair", "rot_to_quat", "quat_to_rot"]


# ---------------------------------------------------------------------------------------------
# Plain rotation helpers (generator-side only)
# ---------------------------------------------------------------------------------------------
def axis_angle(axis, angle) -> np.ndarray:
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def quat_to_rot(q) -> np.ndarray:
    x, y, z, w = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def rot_to_quat(R) -> np.ndarray:
    R = np.asarray(R, np.float64)
    m = np.array([1 + R[0, 0] + R[1, 1] + R[2, 2], 1 + R[0, 0] - R[1, 1] - R[2, 2],
                  1 - R[0, 0] + R[1, 1] - R[2, 2], 1 - R[0, 0] - R[1, 1] + R[2, 2]])
    k = int(np.argmax(m))
    s = 2.0 * math.sqrt(max(m[k], 1e-300))
    if k == 0:
        q = [(R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s, s / 4]
    elif k == 1:
        q = [s / 4, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s, (R[2, 1] - R[1, 2]) / s]
    elif k == 2:
        q = [(R[0, 1] + R[1, 0]) / s, s / 4, (R[1, 2] + R[2, 1]) / s, (R[0, 2] - R[2, 0]) / s]
    else:
        q = [(R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, s / 4, (R[1, 0] - R[0, 1]) / s]
    q = np.array(q)
    if q[3] < 0:
        q = -q
    return q / np.linalg.norm(q)


def pose_vec(R, t, s) -> np.ndarray:
    return np.concatenate([np.asarray(t, np.float64), rot_to_quat(R), [float(s)]])


def pose_parts(p):
    p = np.asarray(p, np.float64)
    return quat_to_rot(p[3:7]), p[:3].copy(), float(p[7])


def look_at(center, target, down=(0.0, 1.0, 0.0)) -> np.ndarray:
    """Camera-to-world rotation of an x-right, y-down, z-forward camera at `center` facing `target`."""
    z = np.asarray(target, np.float64) - np.asarray(center, np.float64)
    z /= np.linalg.norm(z)
    x = np.cross(np.asarray(down, np.float64), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    return np.stack([x, y, z], axis=1)


# ---------------------------------------------------------------------------------------------
# Scene and ray casting
# ---------------------------------------------------------------------------------------------
@dataclass
class Scene:
    planes: list       # (n, d): n.X = d
    boxes: list        # (center, half, yaw)
    sphere: tuple      # (center, radius)

    @staticmethod
    def random(rng: np.random.Generator, center=(0.0, 0.0, 0.0), ground_y=1.6, wall_dist=(8.0, 11.0),
               sphere_r=12.5, box_r=2.5) -> "Scene":
        c = np.asarray(center, np.float64)
        tilt = axis_angle(rng.normal(size=3), rng.uniform(0, math.radians(3)))
        n_g = tilt @ np.array([0.0, 1.0, 0.0])
        planes = [(n_g, float(n_g @ (c + np.array([0, ground_y, 0]))))]
        for _ in range(2):
            ang = rng.uniform(0, 2 * math.pi)
            n = np.array([math.cos(ang), 0.0, math.sin(ang)])
            planes.append((n, float(n @ c + rng.uniform(*wall_dist))))
        boxes = []
        for _ in range(5):
            half = rng.uniform(0.25, 1.5, size=3)
            r, a = box_r * math.sqrt(rng.uniform(0, 1)), rng.uniform(0, 2 * math.pi)
            bc = c + np.array([r * math.cos(a), ground_y - half[1], r * math.sin(a)])
            boxes.append((bc, half, rng.uniform(0, math.pi)))
        return Scene(planes, boxes, (c, sphere_r))

    def cast(self, o: np.ndarray, d: np.ndarray) -> np.ndarray:
        """Distance along unit directions d (n, 3) from origin o (3,) to the nearest surface."""
        dev = _device()
        if dev is not None:
            return self._cast_torch(o, d, dev)
        return self._cast_np(o, d)

    def _cast_torch(self, o, d, dev) -> np.ndarray:
        D = torch.as_tensor(d, dtype=torch.float64, device=dev)
        O = torch.as_tensor(np.asarray(o, np.float64), device=dev)
        best = torch.full((D.shape[0],), float("inf"), dtype=torch.float64, device=dev)
        inf = torch.tensor(float("inf"), dtype=torch.float64, device=dev)
        for nrm, off in self.planes:
            n = torch.as_tensor(nrm, dtype=torch.float64, device=dev)
            den = D @ n
            t = (off - O @ n) / den
            t = torch.where(torch.isfinite(t) & (t > 1e-6), t, inf)
            best = torch.minimum(best, t)
        for bc, half, yaw in self.boxes:
            Ry = torch.tensor([[math.cos(yaw), 0, math.sin(yaw)], [0, 1, 0], [-math.sin(yaw), 0, math.cos(yaw)]],
                              dtype=torch.float64, device=dev)
            ol = Ry.T @ (O - torch.as_tensor(bc, dtype=torch.float64, device=dev))
            dl = D @ Ry
            h = torch.as_tensor(half, dtype=torch.float64, device=dev)
            inv = 1.0 / dl
            t1 = (-h - ol) * inv
            t2 = (h - ol) * inv
            tmin = torch.nan_to_num(torch.minimum(t1, t2), nan=-float("inf")).max(dim=1).values
            tmax = torch.nan_to_num(torch.maximum(t1, t2), nan=float("inf")).min(dim=1).values
            hit = (tmax >= tmin) & (tmax > 1e-6)
            t = torch.where(tmin > 1e-6, tmin, tmax)
            best = torch.minimum(best, torch.where(hit, t, inf))
        sc, sr = self.sphere
        oc = O - torch.as_tensor(sc, dtype=torch.float64, device=dev)
        b = D @ oc
        cc = oc @ oc - sr * sr
        disc = b * b - cc
        t = -b + torch.sqrt(torch.clamp(disc, min=0.0))
        best = torch.minimum(best, torch.where(disc < 0, inf, t))
        return best.cpu().numpy()

    def _cast_np(self, o: np.ndarray, d: np.ndarray) -> np.ndarray:
        n = d.shape[0]
        best = np.full(n, np.inf)
        for nrm, off in self.planes:
            den = d @ nrm
            with np.errstate(divide="ignore", invalid="ignore"):
                t = (off - o @ nrm) / den
            t[~np.isfinite(t) | (t <= 1e-6)] = np.inf
            best = np.minimum(best, t)
        for bc, half, yaw in self.boxes:
            Ry = np.array([[math.cos(yaw), 0, math.sin(yaw)], [0, 1, 0], [-math.sin(yaw), 0, math.cos(yaw)]])
            ol = Ry.T @ (o - bc)
            dl = d @ Ry
            with np.errstate(divide="ignore", invalid="ignore"):
                inv = 1.0 / dl
                t1 = (-half - ol) * inv
                t2 = (half - ol) * inv
            tmin = np.nanmax(np.minimum(t1, t2), axis=1)
            tmax = np.nanmin(np.maximum(t1, t2), axis=1)
            hit = (tmax >= tmin) & (tmax > 1e-6)
            t = np.where(tmin > 1e-6, tmin, tmax)
            t[~hit] = np.inf
            best = np.minimum(best, t)
        sc, sr = self.sphere
        oc = o - sc
        b = d @ oc
        cc = oc @ oc - sr * sr
        disc = b * b - cc
        t = -b + np.sqrt(np.maximum(disc, 0.0))
        t[disc < 0] = np.inf
        return np.minimum(best, t)


@dataclass
class Camera:
    H: int
    W: int
    f: float
    cx: float
    cy: float

    @staticmethod
    def of(H, W) -> "Camera":
        return Camera(H, W, 0.9 * W, (W - 1) / 2.0, (H - 1) / 2.0)

    def unit_rays(self) -> np.ndarray:
        v, u = np.mgrid[0:self.H, 0:self.W].astype(np.float64)
        d = np.stack([(u - self.cx) / self.f, (v - self.cy) / self.f, np.ones_like(u)], -1)
        return (d / np.linalg.norm(d, axis=-1, keepdims=True)).reshape(-1, 3)


# ---------------------------------------------------------------------------------------------
# Graph container
# ---------------------------------------------------------------------------------------------
@dataclass
class SynthGraph:
    name: str
    cams: list                 # Camera per keyframe (generator-only)
    agent: np.ndarray          # (N,) agent id per keyframe
    poses_gt: np.ndarray       # (N, 8)
    poses_init: np.ndarray     # (N, 8)
    xyz: list                  # (H, W, 3) float32 canonical pointmaps
    conf: list                 # (H, W) float32 confidences
    world: list                # (H*W, 3) float64 world hit points (generator-only)
    dist: list                 # (H*W,) metric hit distance (generator-only)
    edges: np.ndarray          # (E, 2) int64, (i, j): matches of j's pixels into i
    band: np.ndarray           # (E, 2) int64 [u_lo, u_hi) on j's columns
    gn_iters: int = 10
    meta: dict = field(default_factory=dict)

    @property
    def n_kf(self) -> int:
        return len(self.xyz)

    def shape(self, k):
        return self.xyz[k].shape[:2]

    def intrinsics(self) -> np.ndarray:
        """(N, 4) float64 [fx, fy, cx, cy] per keyframe: the generator's pinhole cameras, the intrinsics a
        caller supplies in calibrated mode."""
        return np.array([[c.f, c.f, c.cx, c.cy] for c in self.cams], np.float64)

    def _in_cam(self, k, P):
        R, t, s = pose_parts(self.poses_gt[k])
        return (P - t) @ R / s          # canonical coordinates of camera k

    def cross_view(self, e):
        """Prior stand-ins for edge e = (i, j): X^j_i (j's pixels in camera i, (Hj, Wj, 3), zero outside
        the edge's column band, i.e. holes) and X^i_j (i's pixels in camera j, (Hi, Wi, 3)); float32."""
        i, j = (int(v) for v in self.edges[e])
        Hj, Wj = self.shape(j)
        Hi, Wi = self.shape(i)
        Xji = self._in_cam(i, self.world[j]).reshape(Hj, Wj, 3).astype(np.float32)
        lo, hi = self.band[e]
        Xji[:, :lo] = 0.0
        Xji[:, hi:] = 0.0
        Xij = self._in_cam(j, self.world[i]).reshape(Hi, Wi, 3).astype(np.float32)
        return Xji, Xij

    def gt_idx(self, e, rel_tol=0.05) -> np.ndarray:
        """Ground-truth matches of edge e: each pixel of j inside the band whose world point projects
        into i and is the surface i sees there (distance within rel_tol); -1 elsewhere. int32."""
        i, j = (int(v) for v in self.edges[e])
        cam = self.cams[i]
        R, t, _ = pose_parts(self.poses_gt[i])
        X = (self.world[j] - t) @ R          # metric camera-i coordinates
        z = X[:, 2]
        with np.errstate(divide="ignore", invalid="ignore"):
            u = cam.f * X[:, 0] / z + cam.cx
            v = cam.f * X[:, 1] / z + cam.cy
        ok = (z > 0.05) & (u > -0.5) & (u < cam.W - 0.5) & (v > -0.5) & (v < cam.H - 0.5)
        mu = np.clip(np.floor(u + 0.5), 0, cam.W - 1).astype(np.int64)
        mv = np.clip(np.floor(v + 0.5), 0, cam.H - 1).astype(np.int64)
        m = mv * cam.W + mu
        m[~ok] = 0
        dist = np.linalg.norm(X, axis=1)
        ok &= np.abs(self.dist[i][m] - dist) <= rel_tol * self.dist[i][m]
        Wj = self.cams[j].W
        col = np.arange(self.world[j].shape[0]) % Wj
        lo, hi = self.band[e]
        ok &= (col >= lo) & (col < hi)
        return np.where(ok, m, -1).astype(np.int32)

    def gt_idx_all(self):
        return [self.gt_idx(e) for e in range(len(self.edges))]

    def gt_idx_all_torch(self, dev, rel_tol=0.05):
        """gt_idx of every edge computed with torch on `dev` (for the long-horizon graph, where the
        per-edge numpy version takes a minute), concatenated in edge order as one int32 tensor. The
        projection is written element by element in the same order as gt_idx."""
        out = []
        world, dist_i = {}, {}
        for e in range(len(self.edges)):
            i, j = (int(v) for v in self.edges[e])
            if j not in world:
                world[j] = torch.as_tensor(self.world[j], dtype=torch.float64, device=dev)
            if i not in dist_i:
                dist_i[i] = torch.as_tensor(self.dist[i], dtype=torch.float64, device=dev)
            cam = self.cams[i]
            R, t, _ = pose_parts(self.poses_gt[i])
            A = world[j] - torch.as_tensor(t, dtype=torch.float64, device=dev)
            X = [A[:, 0] * float(R[0, c]) + A[:, 1] * float(R[1, c]) + A[:, 2] * float(R[2, c]) for c in range(3)]
            z = X[2]
            u = cam.f * X[0] / z + cam.cx
            v = cam.f * X[1] / z + cam.cy
            ok = (z > 0.05) & (u > -0.5) & (u < cam.W - 0.5) & (v > -0.5) & (v < cam.H - 0.5)
            mu = torch.clamp(torch.floor(u + 0.5), 0, cam.W - 1).to(torch.int64)
            mv = torch.clamp(torch.floor(v + 0.5), 0, cam.H - 1).to(torch.int64)
            m = torch.where(ok, mv * cam.W + mu, torch.zeros_like(mu))
            dist = torch.sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2])
            di = dist_i[i][m]
            ok = ok & (torch.abs(di - dist) <= rel_tol * di)
            col = torch.arange(A.shape[0], device=dev) % self.cams[j].W
            lo, hi = self.band[e]
            ok = ok & (col >= lo) & (col < hi)
            out.append(torch.where(ok, m, torch.full_like(m, -1)).to(torch.int32))
        return torch.cat(out)


# ---------------------------------------------------------------------------------------------
# Construction helpers
# ---------------------------------------------------------------------------------------------
def _render(scene: Scene, cam: Camera, R, t, s, rng: np.random.Generator):
    d_cam = cam.unit_rays()
    d_w = d_cam @ R.T
    dist = scene.cast(np.asarray(t, np.float64), d_w)
    if not np.all(np.isfinite(dist)):
        raise RuntimeError("ray escaped the scene")
    world = t + d_w * dist[:, None]
    xyz = (d_cam * dist[:, None] / s).reshape(cam.H, cam.W, 3).astype(np.float32)
    conf = rng.uniform(1.0, 5.0, size=(cam.H, cam.W)).astype(np.float32)
    return xyz, conf, world, dist


def _overlap(cam_i: Camera, pose_i, world_j_sub, dist_i):
    R, t, _ = pose_parts(pose_i)
    X = (world_j_sub - t) @ R
    z = X[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = cam_i.f * X[:, 0] / z + cam_i.cx
        v = cam_i.f * X[:, 1] / z + cam_i.cy
    ok = (z > 0.05) & (u > -0.5) & (u < cam_i.W - 0.5) & (v > -0.5) & (v < cam_i.H - 0.5)
    mu = np.clip(np.floor(u + 0.5), 0, cam_i.W - 1).astype(np.int64)
    mv = np.clip(np.floor(v + 0.5), 0, cam_i.H - 1).astype(np.int64)
    m = mv * cam_i.W + mu
    m[~ok] = 0
    ok &= np.abs(dist_i[m] - np.linalg.norm(X, axis=1)) <= 0.05 * dist_i[m]
    return float(ok.mean())


def _perturb(p, rng, sig_rot, sig_t, sig_s):
    R, t, s = pose_parts(p)
    w = rng.normal(size=3) * sig_rot
    ang = np.linalg.norm(w)
    Rn = axis_angle(w, ang) if ang > 0 else np.eye(3)
    return pose_vec(Rn @ R, t + rng.normal(size=3) * sig_t, s * math.exp(rng.normal() * sig_s))


def _apply_gauge(G, p):
    Rg, tg, sg = pose_parts(G)
    R, t, s = pose_parts(p)
    return pose_vec(Rg @ R, sg * (Rg @ t) + tg, sg * s)


def _random_gauge(rng):
    axis = rng.normal(size=3)
    return pose_vec(axis_angle(axis, rng.uniform(0, math.pi)),
                    rng.normal(size=3) / math.sqrt(3) * rng.uniform(0, 10) / 1.0,
                    math.exp(rng.uniform(math.log(0.5), math.log(2.0))))


def _bands(rng, shapes_j, lo=0.3, hi=1.0):
    out = []
    for (_, W) in shapes_j:
        rho = rng.uniform(lo, hi)
        width = max(1, int(round(rho * W)))
        u0 = int(rng.integers(0, W - width + 1))
        out.append((u0, u0 + width))
    return np.array(out, np.int64)


def make_pair(H=48, W=64, seed=1001, max_rot_deg=15.0, max_trans=1.0, scale_range=(0.8, 1.25)):
    """Two keyframes; keyframe 0 at the identity (the anchor), keyframe 1 at a random offset."""
    rng = np.random.default_rng(seed)
    scene = Scene.random(rng, center=(0.0, 0.0, 8.0), ground_y=1.6, wall_dist=(9.0, 12.0),
                         sphere_r=11.5, box_r=2.5)
    cam = Camera.of(H, W)
    p0 = pose_vec(np.eye(3), np.zeros(3), 1.0)
    Rr = axis_angle(rng.normal(size=3), math.radians(rng.uniform(0, max_rot_deg)))
    dirn = rng.normal(size=3)
    tr = dirn / np.linalg.norm(dirn) * rng.uniform(0, max_trans)
    s1 = math.exp(rng.uniform(math.log(scale_range[0]), math.log(scale_range[1])))
    p1 = pose_vec(Rr, tr, s1)
    xyz, conf, world, dist = [], [], [], []
    for p in (p0, p1):
        R, t, s = pose_parts(p)
        a, b, c, d = _render(scene, cam, R, t, s, rng)
        xyz.append(a); conf.append(b); world.append(c); dist.append(d)
    edges = np.array([[0, 1]], np.int64)
    band = np.array([[0, W]], np.int64)
    poses_gt = np.stack([p0, p1])
    poses_init = np.stack([p0, p0])  # start of keyframe 1 at the identity relative pose
    return SynthGraph("pair", [cam, cam], np.zeros(2, np.int64), poses_gt, poses_init, xyz, conf,
                      world, dist, edges, band, gn_iters=10, meta={"seed": seed})


def _ring_path(n, radius_xz, phase0, sweep, rng, height=0.0, wobble_deg=4.0, center=(0.0, 0.0, 0.0)):
    c = np.asarray(center, np.float64)
    out = []
    ph_yaw, ph_pitch = rng.uniform(0, 2 * math.pi, size=2)
    for k in range(n):
        a = phase0 + sweep * k / max(n - 1, 1)
        pos = c + np.array([radius_xz[0] * math.cos(a), height, radius_xz[1] * math.sin(a)])
        R = look_at(pos, c + np.array([0.0, 0.3, 0.0]))
        yaw = math.radians(wobble_deg) * math.sin(2 * math.pi * k / 13.0 + ph_yaw)
        pitch = math.radians(wobble_deg * 0.5) * math.sin(2 * math.pi * k / 17.0 + ph_pitch)
        R = R @ axis_angle([0, 1, 0], yaw) @ axis_angle([1, 0, 0], pitch)
        out.append((R, pos))
    return out


def _build(name, scene, cams, agent, path, rng, scales):
    xyz, conf, world, dist, gt = [], [], [], [], []
    for k, ((R, t), cam) in enumerate(zip(path, cams)):
        a, b, c, d = _render(scene, cam, R, t, scales[k], rng)
        xyz.append(a); conf.append(b); world.append(c); dist.append(d)
        gt.append(pose_vec(R, t, scales[k]))
    return xyz, conf, world, dist, np.stack(gt)


def _overlap_matrix(cams, poses, world, dist, stride=16):
    """O[i, j]: fraction of a subsampled grid of j's pixels that i sees (projection inside i's image and
    i's own surface at that pixel within 5%)."""
    n = len(cams)
    subs = []
    for k in range(n):
        H, W = cams[k].H, cams[k].W
        v, u = np.mgrid[0:H:stride, 0:W:stride]
        subs.append(world[k][(v * W + u).reshape(-1)])
    counts = np.array([s.shape[0] for s in subs])
    allp = np.concatenate(subs)
    owner = np.repeat(np.arange(n), counts)
    O = np.zeros((n, n))
    for i in range(n):
        cam = cams[i]
        R, t, _ = pose_parts(poses[i])
        X = (allp - t) @ R
        z = X[:, 2]
        with np.errstate(divide="ignore", invalid="ignore"):
            u = cam.f * X[:, 0] / z + cam.cx
            v = cam.f * X[:, 1] / z + cam.cy
        ok = (z > 0.05) & (u > -0.5) & (u < cam.W - 0.5) & (v > -0.5) & (v < cam.H - 0.5)
        mu = np.clip(np.floor(np.nan_to_num(u) + 0.5), 0, cam.W - 1).astype(np.int64)
        mv = np.clip(np.floor(np.nan_to_num(v) + 0.5), 0, cam.H - 1).astype(np.int64)
        m = mv * cam.W + mu
        ok &= np.abs(dist[i][m] - np.linalg.norm(X, axis=1)) <= 0.05 * dist[i][m]
        O[i] = np.bincount(owner, weights=ok, minlength=n) / counts
        O[i, i] = 0.0
    return O


def make_config(k: int, seed: int | None = None, n_agents=None, kf_per_agent=None, n_edges=None):
    """Build configuration k (1..5) of the workload table; sizes may be shrunk for tests."""
    seed = 1000 + k if seed is None else seed
    if k == 1:
        return make_pair(seed=seed)
    rng = np.random.default_rng(seed)
    scene = Scene.random(rng)
    if k == 2:
        n = kf_per_agent or 20
        cams = [Camera.of(384, 512)] * n
        path = _ring_path(n, (7.0, 6.0), 0.0, 2 * math.pi * (n - 1) / n, rng)
        scales = np.exp(rng.uniform(-0.2, 0.2, size=n))
        scales[0] = 1.0
        agent = np.zeros(n, np.int64)
        xyz, conf, world, dist, gt = _build("single", scene, cams, agent, path, rng, scales)
        O = _overlap_matrix(cams, gt, world, dist)
        seq = [(i, i + 1) for i in range(n - 1)]
        n_loop = (n_edges or 40) - len(seq)
        cand = sorted(((min(O[i, j], O[j, i]), i, j) for i in range(n) for j in range(i + 2, n)),
                      reverse=True)
        loops = [(i, j) for _, i, j in cand[:n_loop]]
        edges = np.array(seq + loops, np.int64)
        band = np.array([[0, cams[j].W] for _, j in edges], np.int64)
        init = np.stack([gt[0]] + [_perturb(p, rng, math.radians(2.0), 0.1, 0.05) for p in gt[1:]])
        return SynthGraph("single_agent", cams, agent, gt, init, xyz, conf, world, dist, edges, band,
                          gn_iters=20, meta={"seed": seed})
    if k in (3, 4, 5):
        na = n_agents or 4
        nk = kf_per_agent or (50 if k in (3, 4) else 250)
        n_e = n_edges or (800 if k in (3, 4) else 4000)
        cams, path, agent = [], [], []
        for a in range(na):
            res = (384, 512) if (k == 5 or a % 2 == 0) else (288, 512)
            radius = (7.0 + 0.4 * a, 6.0 + 0.4 * a)
            direction = 1.0 if a % 2 == 0 else -1.0
            sweep = direction * 2 * math.pi * (0.75 if k in (3, 4) else 3.0)
            p = _ring_path(nk, radius, a * math.pi / 2, sweep, rng, height=0.2 * (a - 1.5))
            path += p
            cams += [Camera.of(*res)] * nk
            agent += [a] * nk
        agent = np.array(agent, np.int64)
        n = len(path)
        scales = np.exp(rng.uniform(-0.2, 0.2, size=n))
        scales[0] = 1.0
        xyz, conf, world, dist, gt = _build("multi", scene, cams, agent, path, rng, scales)
        seq = [(q, q + 1) for q in range(n - 1) if agent[q] == agent[q + 1]]
        O = _overlap_matrix(cams, gt, world, dist, stride=32 if k == 5 else 16)
        n_inter = n_e - len(seq)
        # retrieval stand-in: each keyframe keeps its top-k overlapping keyframes of other agents
        cand = {}
        for q in range(n):
            others = [o for o in np.argsort(-O[q]) if agent[o] != agent[q]][:8]
            for o in others:
                key = (min(q, o), max(q, o))
                cand[key] = max(cand.get(key, 0.0), min(O[q, o], O[o, q]))
        if k == 5:  # long horizon: intra-agent loop edges by overlap as well
            for q in range(n):
                for o in np.argsort(-O[q])[:6]:
                    if agent[o] == agent[q] and abs(int(o) - q) >= 2:
                        key = (min(q, int(o)), max(q, int(o)))
                        cand[key] = max(cand.get(key, 0.0), min(O[q, o], O[o, q]))
        inter = sorted(cand.items(), key=lambda kv: -kv[1])[:n_inter]
        edges = np.array(seq + [kv[0] for kv in inter], np.int64)
        band = _bands(rng, [(cams[j].H, cams[j].W) for _, j in edges])
        gauges = [pose_vec(np.eye(3), np.zeros(3), 1.0)] + [_random_gauge(rng) for _ in range(na - 1)]
        init = []
        for q in range(n):
            p = gt[q] if q == 0 else _perturb(gt[q], rng, math.radians(2.0), 0.1, 0.05)
            init.append(_apply_gauge(gauges[agent[q]], p))
        return SynthGraph({3: "batched", 4: "batched_bf16", 5: "long_horizon"}[k], cams, agent, gt,
                          np.stack(init), xyz, conf, world, dist, edges, band,
                          gn_iters=20, meta={"seed": seed, "gauges": np.stack(gauges)})
    raise ValueError(f"unknown configuration {k}")
