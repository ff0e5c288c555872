"""Seeded synthetic terrains, scans and poses.

This module is shared by the tests, the benchmark and the CPU oracle's
callers. It holds only the *inputs*: ground-truth terrain heights, point
positions, noise draws, sensor poses and center layouts. None of the
terrain-model arithmetic (kernel, regression, filter, evaluation) lives here,
so the GPU path and the oracle never share an implementation of the method.

The workloads follow the experiment setup (Section "Experiments"; the RBF
parameters are given in the subsection on the terrain-approximation result)
scaled to the five workloads used for parity and timing:

* ``small``   -- 10x10 m patch, 400 jittered centers, 2000 ground points,
                 10k queries (one recursive update, then evaluation).
* ``odometry``-- 50x50 m map, 100 frames of 20k ground points on a
                 boustrophedon path, 200k scan points per frame in the
                 sensor frame with the true pose.
* ``diff``    -- ``odometry`` terrain at frame 50 with a perturbed pose.
* ``large``   -- 100x100 m, 40,000 centers on a 0.5 m grid.
* ``patches`` -- 256 independent patches of uneven size.

Every stream is drawn from ``numpy.random.SeedSequence(seed)`` spawned in a
fixed order: centers, terrain, points, noise, queries, poses.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# --------------------------------------------------------------------------
# Terrain primitives (ground truth, not the model being fitted)
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Terrain:
    """Sum of Gaussian bumps, half-plane steps and stair segments."""

    bump_mu: np.ndarray  # (nb, 2)
    bump_a: np.ndarray  # (nb,)
    bump_s: np.ndarray  # (nb,)
    step_q: np.ndarray  # (ns, 2) point on the step edge
    step_n: np.ndarray  # (ns, 2) unit normal of the raised side
    step_h: np.ndarray  # (ns,)
    stair_o: np.ndarray  # (nt, 2) origin of a stair segment
    stair_dir: np.ndarray  # (nt, 2) unit direction of the flight
    stair_n: np.ndarray  # (nt,) steps per flight

    TREAD = 0.30
    RISER = 0.17
    WIDTH = 2.0
    LANDING = 2.0

    def height(self, xy: np.ndarray, chunk: int = 65536) -> np.ndarray:
        xy = np.asarray(xy, dtype=np.float64)
        out = np.empty(xy.shape[0], dtype=np.float64)
        for s in range(0, xy.shape[0], chunk):
            out[s:s + chunk] = self._height(xy[s:s + chunk])
        return out

    def _height(self, xy: np.ndarray) -> np.ndarray:
        h = np.zeros(xy.shape[0], dtype=np.float64)
        if self.bump_a.size:
            h += self._bump_sum(xy)
        for q, n, hh in zip(self.step_q, self.step_n, self.step_h):
            h += np.where((xy - q) @ n >= 0.0, hh, 0.0)
        for o, d, n in zip(self.stair_o, self.stair_dir, self.stair_n):
            h += self._stair(xy, o, d, int(n))
        return h

    CELL = 4.0
    REACH = 8.0  # bumps are dropped beyond 8 widths (relative size < 1e-13)

    def _bump_sum(self, xy):
        """Sum of bumps, culled per CELL-sized square of query points."""
        import torch  # CPU tensors: vectorised exp over (points x bumps)
        out = np.zeros(xy.shape[0])
        key = np.floor(xy / self.CELL).astype(np.int64)
        key = key[:, 0] * 1_000_003 + key[:, 1]
        order = np.argsort(key, kind="stable")
        uk, start = np.unique(key[order], return_index=True)
        stop = np.append(start[1:], order.size)
        mu = self.bump_mu
        reach = self.REACH * self.bump_s + self.CELL
        for s0, s1 in zip(start, stop):
            idx = order[s0:s1]
            p = xy[idx]
            ctr = p.mean(axis=0)
            span = np.abs(p - ctr).max()
            sel = np.flatnonzero(
                np.abs(mu - ctr).max(axis=1) <= reach + span)
            if sel.size == 0:
                continue
            P = torch.from_numpy(np.ascontiguousarray(p))
            M = torch.from_numpy(np.ascontiguousarray(mu[sel]))
            A = torch.from_numpy(self.bump_a[sel])
            S2 = torch.from_numpy(self.bump_s[sel] ** 2)
            d2 = ((P[:, None, :] - M[None, :, :]) ** 2).sum(-1)
            out[idx] = (A * torch.exp(-d2 / (2.0 * S2))).sum(1).numpy()
        return out

    def _stair(self, xy, o, d, n):
        perp = np.array([-d[1], d[0]])
        rel = xy - o
        along = rel @ d
        across = rel @ perp
        inside = np.abs(across) <= 0.5 * self.WIDTH
        up_len = n * self.TREAD
        total = 2.0 * up_len + self.LANDING
        h = np.zeros(xy.shape[0])
        # up-flight: step k occupies [k*tread, (k+1)*tread), height (k+1)*riser
        k_up = np.floor(along / self.TREAD)
        up = (along >= 0.0) & (along < up_len)
        h = np.where(up, (k_up + 1.0) * self.RISER, h)
        land = (along >= up_len) & (along < up_len + self.LANDING)
        h = np.where(land, n * self.RISER, h)
        # mirrored down-flight
        dn_along = total - along
        k_dn = np.floor(dn_along / self.TREAD)
        down = (along >= up_len + self.LANDING) & (along < total)
        h = np.where(down, (k_dn + 1.0) * self.RISER, h)
        return np.where(inside, h, 0.0)


def _bumps(rng, n, lo, hi):
    mu = rng.uniform(lo, hi, size=(n, 2))
    a = rng.uniform(-0.2, 0.2, size=n)
    s = rng.uniform(0.3, 1.5, size=n)
    return mu, a, s


def _empty2():
    return np.zeros((0, 2))


def _stairs(rng, count, lo, hi, inset=5.0):
    o = rng.uniform(lo + inset, hi - inset, size=(count, 2))
    th = rng.uniform(0.0, 2.0 * math.pi, size=count)
    d = np.stack([np.cos(th), np.sin(th)], axis=1)
    n = rng.integers(3, 9, size=count)
    return o, d, n


# --------------------------------------------------------------------------
# Model / filter parameters shared by every workload (sigma, cutoff, ...)
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Params:
    sigma: float = 0.5
    cutoff: float = 3.0
    sigma_eps: float = 0.0
    lam: float = 1e-3
    R: float = 0.02 ** 2


def grid_centers(rng, nx, ny, spacing, x0=0.0, y0=0.0, jitter=0.1, first=None):
    """Jittered centers at cell centers of an nx*ny mesh, row-major (y outer)."""
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    c = np.stack([x0 + (ii.ravel() + 0.5) * spacing,
                  y0 + (jj.ravel() + 0.5) * spacing], axis=1)
    if first is not None:
        c = c[:first]
    if jitter > 0.0:
        c = c + rng.uniform(-jitter, jitter, size=c.shape)
    return np.ascontiguousarray(c)


def _uniform_xy(rng, n, lo, hi):
    return rng.uniform(lo, hi, size=(n, 2))


def _disc_xy(rng, n, center, radius, lo, hi):
    """Uniform points in a disc, rejection-clipped to the square [lo, hi]^2."""
    out = np.empty((0, 2))
    while out.shape[0] < n:
        k = int((n - out.shape[0]) * 1.6) + 64
        r = radius * np.sqrt(rng.uniform(0.0, 1.0, size=k))
        t = rng.uniform(0.0, 2.0 * math.pi, size=k)
        p = np.stack([center[0] + r * np.cos(t), center[1] + r * np.sin(t)], 1)
        ok = (p[:, 0] >= lo) & (p[:, 0] < hi) & (p[:, 1] >= lo) & (p[:, 1] < hi)
        out = np.concatenate([out, p[ok]], 0)
    return np.ascontiguousarray(out[:n])


def rot_zyx(yaw, pitch, roll):
    cy, sy = math.cos(yaw), math.sin(yaw)
    cp, sp = math.cos(pitch), math.sin(pitch)
    cr, sr = math.cos(roll), math.sin(roll)
    Rz = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1.0]])
    Ry = np.array([[cp, 0, sp], [0, 1.0, 0], [-sp, 0, cp]])
    Rx = np.array([[1.0, 0, 0], [0, cr, -sr], [0, sr, cr]])
    return Rz @ Ry @ Rx


def so3_exp(v):
    """Rodrigues' formula for Exp: so(3) -> SO(3) (pose perturbations only)."""
    v = np.asarray(v, dtype=np.float64)
    th = float(np.linalg.norm(v))
    K = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0.0]])
    if th < 1e-12:
        return np.eye(3) + K
    return (np.eye(3) + math.sin(th) / th * K
            + (1.0 - math.cos(th)) / th ** 2 * (K @ K))


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------


@dataclasses.dataclass
class SmallCase:
    params: Params
    centers: np.ndarray  # (N, 2)
    terrain: Terrain
    xy: np.ndarray  # (M, 2) ground points
    z: np.ndarray  # (M,) noisy heights
    queries: np.ndarray  # (Q, 2)
    roi: tuple


def small_case(seed: int = 0, n_points: int = 2000, n_queries: int = 10000,
               side: float = 10.0, spacing: float = 0.5) -> SmallCase:
    """10x10 m patch: 400 jittered centers, 20 bumps + one 0.15 m step."""
    ss = np.random.SeedSequence(seed).spawn(6)
    r_c, r_t, r_p, r_n, r_q, _ = [np.random.default_rng(s) for s in ss]
    n = int(round(side / spacing))
    centers = grid_centers(r_c, n, n, spacing, jitter=0.1)
    mu, a, s = _bumps(r_t, 20, 0.0, side)
    th = r_t.uniform(0.0, 2.0 * math.pi)
    q = r_t.uniform(0.3 * side, 0.7 * side, size=(1, 2))
    terrain = Terrain(mu, a, s, q, np.array([[math.cos(th), math.sin(th)]]),
                      np.array([0.15]), _empty2(), _empty2(),
                      np.zeros(0, dtype=np.int64))
    xy = _uniform_xy(r_p, n_points, 0.0, side)
    z = terrain.height(xy) + r_n.normal(0.0, 0.02, size=n_points)
    queries = _uniform_xy(r_q, n_queries, 0.0, side)
    return SmallCase(Params(), centers, terrain, xy, z, queries,
                     (0.0, 0.0, side, side))


class OdometryCase:
    """50x50 m map, 100 frames along a 3-pass boustrophedon path.

    Frames are generated lazily and independently (each frame has its own
    spawned stream), so a benchmark can draw only the frames it times.
    """

    SIDE = 50.0
    N_FRAMES = 100
    GROUND_PER_FRAME = 20000
    SCAN_PER_FRAME = 200000
    DISC = 20.0
    SENSOR_HEIGHT = 0.6

    def __init__(self, seed: int = 1, side: float = 50.0, n_bumps: int = 400,
                 n_stairs: int = 8, n_frames: int = 100,
                 ground_per_frame: int = 20000, scan_per_frame: int = 200000):
        self.seed = seed
        self.SIDE = side
        self.N_FRAMES = n_frames
        self.GROUND_PER_FRAME = ground_per_frame
        self.SCAN_PER_FRAME = scan_per_frame
        self.params = Params()
        ss = np.random.SeedSequence(seed).spawn(6)
        self._ss = ss
        r_t = np.random.default_rng(ss[1])
        mu, a, s = _bumps(r_t, n_bumps, 0.0, side)
        so, sd, sn = _stairs(r_t, n_stairs, 0.0, side)
        self.terrain = Terrain(mu, a, s, _empty2(), _empty2(), np.zeros(0),
                               so, sd, sn)
        # sensor path: 3 passes at y = 0.2, 0.5, 0.8 of the side, x 0.1..0.9
        passes = [0.2 * side, 0.5 * side, 0.8 * side]
        per = int(math.ceil(n_frames / 3))
        path = []
        for k in range(n_frames):
            p = k // per
            u = (k % per) / max(per - 1, 1)
            if p % 2 == 1:
                u = 1.0 - u
            x = 0.1 * side + 0.8 * side * u
            heading = 0.0 if p % 2 == 0 else math.pi
            path.append((x, passes[min(p, 2)], heading))
        self.path = path
        self.roi = (0.0, 0.0, side, side)

    def _frame_rngs(self, k):
        # per-frame children: points, noise, scan points, scan noise, pose
        kids = np.random.SeedSequence(
            entropy=self._ss[2].entropy,
            spawn_key=tuple(self._ss[2].spawn_key) + (k,)).spawn(5)
        return [np.random.default_rng(s) for s in kids]

    def ground_xy(self, k):
        r_p, _, _, _, _ = self._frame_rngs(k)
        x, y, _ = self.path[k]
        return _disc_xy(r_p, self.GROUND_PER_FRAME, (x, y), self.DISC,
                        0.0, self.SIDE)

    def ground(self, k):
        r_p, r_n, _, _, _ = self._frame_rngs(k)
        x, y, _ = self.path[k]
        xy = _disc_xy(r_p, self.GROUND_PER_FRAME, (x, y), self.DISC, 0.0,
                      self.SIDE)
        z = self.terrain.height(xy) + r_n.normal(0.0, 0.02, size=xy.shape[0])
        return xy, z

    def pose(self, k):
        _, _, _, _, r_o = self._frame_rngs(k)
        x, y, heading = self.path[k]
        roll, pitch = np.deg2rad(r_o.uniform(-5.0, 5.0, size=2))
        R = rot_zyx(heading, pitch, roll)
        t = np.array([x, y, float(self.terrain.height(np.array([[x, y]]))[0])
                      + self.SENSOR_HEIGHT])
        return R, t

    def scan(self, k, n=None):
        """Scan points in the sensor frame (n x 3) and the true pose."""
        _, _, r_s, r_sn, _ = self._frame_rngs(k)
        n = self.SCAN_PER_FRAME if n is None else n
        x, y, _ = self.path[k]
        xy = _disc_xy(r_s, n, (x, y), self.DISC, 0.0, self.SIDE)
        z = self.terrain.height(xy) + r_sn.normal(0.0, 0.02, size=n)
        R, t = self.pose(k)
        world = np.concatenate([xy, z[:, None]], 1)
        sensor = (world - t) @ R  # R^T (p - t), row-wise
        return np.ascontiguousarray(sensor), R, t


def perturbed_pose(R, t, seed, std=0.05):
    """Right-perturb a pose by delta ~ N(0, std^2) per so(3)/translation axis."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[5])
    d = rng.normal(0.0, std, size=6)
    return R @ so3_exp(d[:3]), t + d[3:], d


@dataclasses.dataclass
class LargeCase:
    params: Params
    centers: np.ndarray
    terrain: Terrain
    side: float


def large_case(seed: int = 3, side: float = 100.0, spacing: float = 0.5,
               jitter: float = 0.0) -> LargeCase:
    """100x100 m, 40,000 centers on a 0.5 m grid, bumps + stair segments."""
    ss = np.random.SeedSequence(seed).spawn(6)
    r_c, r_t = np.random.default_rng(ss[0]), np.random.default_rng(ss[1])
    n = int(round(side / spacing))
    centers = grid_centers(r_c, n, n, spacing, jitter=jitter)
    mu, a, s = _bumps(r_t, int(1600 * (side / 100.0) ** 2), 0.0, side)
    so, sd, sn = _stairs(r_t, max(1, int(32 * (side / 100.0) ** 2)), 0.0, side)
    terrain = Terrain(mu, a, s, _empty2(), _empty2(), np.zeros(0), so, sd, sn)
    return LargeCase(Params(), centers, terrain, side)


def large_points(case: LargeCase, n: int, seed: int = 3, stream: int = 0):
    kids = np.random.SeedSequence(seed).spawn(6)[2].spawn(stream + 1)
    rng = np.random.default_rng(kids[stream])
    rn = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[3]
                               .spawn(stream + 1)[stream])
    xy = _uniform_xy(rng, n, 0.0, case.side)
    z = case.terrain.height(xy) + rn.normal(0.0, 0.02, size=n)
    return xy, z


@dataclasses.dataclass
class Patch:
    centers: np.ndarray
    xy: np.ndarray
    z: np.ndarray
    kind: str


def patches_case(seed: int = 4, count: int = 256, n_range=(200, 8000),
                 m_range=(1000, 40000), spacing: float = 0.5, only=None):
    """Independent patches; centers on a 0.5 m grid (first N_p nodes of a
    round(sqrt(N_p))-wide row-major mesh, +/-0.1 m jitter), points uniform
    over the covered rectangle, terrain flat / bumpy / stair. With `only` (a
    set of patch indices) the heights of the other patches are not computed
    (their z is None); every random stream is drawn as without it, so the
    selected patches are the same."""
    ss = np.random.SeedSequence(seed).spawn(6)
    r_c, r_t, r_p, r_n = [np.random.default_rng(s) for s in ss[:4]]
    out = []
    for idx in range(count):
        npc = int(r_c.integers(n_range[0], n_range[1] + 1))
        mp = int(r_p.integers(m_range[0], m_range[1] + 1))
        nx = int(round(math.sqrt(npc)))
        ny = int(math.ceil(npc / nx))
        centers = grid_centers(r_c, nx, ny, spacing, jitter=0.1, first=npc)
        w_side, h_side = nx * spacing, ny * spacing
        kind = ["flat", "bumpy", "stair"][int(r_t.integers(0, 3))]
        area = w_side * h_side
        if kind == "flat":
            terr = Terrain(_empty2(), np.zeros(0), np.zeros(0), _empty2(),
                           _empty2(), np.zeros(0), _empty2(), _empty2(),
                           np.zeros(0))
        else:
            nb = max(1, int(round(0.2 * area)))
            mu = np.stack([r_t.uniform(0, w_side, nb),
                           r_t.uniform(0, h_side, nb)], 1)
            a = r_t.uniform(-0.2, 0.2, nb)
            s = r_t.uniform(0.3, 1.5, nb)
            if kind == "stair":
                th = r_t.uniform(0, 2 * math.pi)
                q = np.array([[r_t.uniform(0.3, 0.7) * w_side,
                               r_t.uniform(0.3, 0.7) * h_side]])
                terr = Terrain(mu, a, s, q,
                               np.array([[math.cos(th), math.sin(th)]]),
                               np.array([0.15]), _empty2(), _empty2(),
                               np.zeros(0))
            else:
                terr = Terrain(mu, a, s, _empty2(), _empty2(), np.zeros(0),
                               _empty2(), _empty2(), np.zeros(0))
        # points cover the rows the centers occupy
        rows = int(math.ceil(npc / nx))
        xy = np.stack([r_p.uniform(0, w_side, mp),
                       r_p.uniform(0, rows * spacing, mp)], 1)
        noise = r_n.normal(0.0, 0.02, size=mp)
        z = terr.height(xy) + noise if (only is None or idx in only) else None
        out.append(Patch(centers, xy, z, kind))
    return Params(), out
