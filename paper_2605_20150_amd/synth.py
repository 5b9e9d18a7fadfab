"""Seeded synthetic scenes, cameras and trajectories.

This module only draws inputs: Gaussian parameter tables, pinhole cameras
and camera paths.  It holds none of the rasterizer's, the loss's or the
optimizer's arithmetic, so that the FP64 oracle and the GPU path can share
it without sharing any of the method.

Parameter rows have 59 float32 columns (the degree-3 SH parameterisation of
Sec. 2, "Per-Gaussian parameter table"):

    [0:3]   mean xyz (world)
    [3:6]   log scale
    [6:10]  rotation quaternion (w, x, y, z), not necessarily unit length
    [10]    opacity logit
    [11:14] SH DC coefficient (r, g, b)
    [14:59] 15 higher SH coefficients, coefficient-major, (r, g, b) each

Cameras are dicts with world-to-camera ``R`` (3x3, row-major) and ``t``
(p_cam = R @ p_world + t, x right, y down, z forward), focal lengths,
principal point, image size and the near/far planes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

D = 59


def _attributes(rng: np.random.Generator, n: int, logscale_mu: float,
                logscale_sigma: float) -> np.ndarray:
    """Everything except the means, drawn as the tiny-scene recipe states."""
    th = np.zeros((n, D), dtype=np.float64)
    th[:, 3:6] = rng.normal(logscale_mu, logscale_sigma, size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    th[:, 6:10] = q
    th[:, 10] = rng.normal(0.0, 1.0, size=n)
    th[:, 11:14] = rng.normal(0.0, 0.3, size=(n, 3))
    th[:, 14:59] = rng.normal(0.0, 0.05, size=(n, 45))
    return th


def tiny_scene(n: int = 1000, seed: int = 0) -> np.ndarray:
    """Tiny scene: means U[-1,1]^3, log-scale N(-4, 0.5)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = rng.uniform(-1.0, 1.0, size=(n, 3))
    th = _attributes(rng, n, -4.0, 0.5)
    th[:, 0:3] = mu
    return th.astype(np.float32)


def blob_scene(n_blobs: int, per_blob: int, half_extent: float,
               height: tuple[float, float], sigma: float, seed: int,
               logscale_mu: float = -1.0, logscale_sigma: float = 0.7) -> np.ndarray:
    """Aerial-style scene: Gaussian blobs (std ``sigma``) whose centres are
    uniform over a [-half_extent, half_extent]^2 ground square with heights
    U(height); world z is up."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cx = rng.uniform(-half_extent, half_extent, size=n_blobs)
    cy = rng.uniform(-half_extent, half_extent, size=n_blobs)
    cz = rng.uniform(height[0], height[1], size=n_blobs)
    centres = np.stack([cx, cy, cz], axis=1)
    n = n_blobs * per_blob
    mu = np.repeat(centres, per_blob, axis=0) + rng.normal(0.0, sigma, size=(n, 3))
    th = _attributes(rng, n, logscale_mu, logscale_sigma)
    th[:, 0:3] = mu
    return th.astype(np.float32)


def perturbed(theta: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """theta + N(0, sigma^2) on every column (the seeded target parameters)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (theta.astype(np.float64) + rng.normal(0.0, sigma, size=theta.shape)).astype(np.float32)


@dataclass
class Camera:
    R: np.ndarray          # 3x3 world->camera
    t: np.ndarray          # 3
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = 0.2
    z_far: float = 1.0e4

    def as_row(self) -> np.ndarray:
        """Flat float64 row: R(9) t(3) fx fy cx cy W H z_near z_far."""
        return np.concatenate([
            np.asarray(self.R, np.float64).reshape(9), np.asarray(self.t, np.float64).reshape(3),
            [self.fx, self.fy, self.cx, self.cy, float(self.width), float(self.height),
             self.z_near, self.z_far]]).astype(np.float64)


def cams_array(cams: list[Camera]) -> np.ndarray:
    return np.stack([c.as_row() for c in cams], axis=0)


def look_at(eye, target, up, width: int, height: int, f: float,
            z_near: float = 0.2, z_far: float = 1.0e4,
            cx: float | None = None, cy: float | None = None) -> Camera:
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd], axis=0)
    t = -R @ eye
    return Camera(R, t, f, f, width / 2.0 if cx is None else cx,
                  height / 2.0 if cy is None else cy, width, height, z_near, z_far)


def tiny_camera() -> Camera:
    """64x64, f = 64, principal point (32, 32), identity rotation, centre (0,0,-3)."""
    return Camera(np.eye(3), np.array([0.0, 0.0, 3.0]), 64.0, 64.0, 32.0, 32.0, 64, 64)


def focal_for_hfov(width: int, hfov_deg: float) -> float:
    return (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)


def orbit_cameras(n_views: int, radius: float, altitude: float, look: tuple,
                  width: int = 1920, height: int = 1080, hfov_deg: float = 60.0,
                  z_far: float = 1.0e4) -> list[Camera]:
    """Views evenly spaced on a circle at ``altitude`` looking at ``look``."""
    f = focal_for_hfov(width, hfov_deg)
    out = []
    for k in range(n_views):
        a = 2.0 * math.pi * k / n_views
        eye = (radius * math.cos(a), radius * math.sin(a), altitude)
        out.append(look_at(eye, look, (0.0, 0.0, 1.0), width, height, f, 0.2, z_far))
    return out


# ---------------------------------------------------------------------------
# Workloads used by tests and the benchmark
# ---------------------------------------------------------------------------

def tiny_workload():
    """Tiny scene, 1000 Gaussians, one 64x64 camera (seed 0, target seed 1)."""
    theta = tiny_scene(1000, 0)
    return theta, [tiny_camera()], perturbed(theta, 0.05, 1)


def aerial_workload(n_blobs: int = 200, per_blob: int = 5000, seed: int = 10,
                    n_views: int = 400, width: int = 1920, height: int = 1080):
    """Resident aerial training: 200 blobs x 5000 Gaussians (sigma 5 m) over a
    500 x 500 m plane, heights U(0, 40) m, log-scale N(-1, 0.7); 1920x1080
    views (60 deg horizontal fov) on a radius-250 m orbit at 150 m altitude
    looking at (0, 0, 20)."""
    theta = blob_scene(n_blobs, per_blob, 250.0, (0.0, 40.0), 5.0, seed)
    cams = orbit_cameras(n_views, 250.0, 150.0, (0.0, 0.0, 20.0), width, height)
    return theta, cams


def dense_scene(n: int, seed: int, extent: float = 1.0, logscale_mu: float = -2.5,
                logscale_sigma: float = 0.5) -> np.ndarray:
    """A denser variant of the tiny scene (larger footprints, deeper lists):
    exercises early termination and long per-tile lists at small sizes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = rng.uniform(-extent, extent, size=(n, 3))
    th = _attributes(rng, n, logscale_mu, logscale_sigma)
    th[:, 0:3] = mu
    return th.astype(np.float32)


# ---------------------------------------------------------------------------
# Street-level city and walks (out-of-core streaming and the predictor)
# ---------------------------------------------------------------------------

@dataclass
class City:
    extent: float          # the city is [-extent/2, extent/2]^2 (metres)
    pitch: float           # street spacing (street centre lines at multiples of pitch)
    street_width: float


def city_means(n: int, seed: int, extent: float = 4000.0, pitch: float = 100.0, street_width: float = 20.0,
               buildings_per_km2: float = 400.0, ground_frac: float = 0.1):
    """Centres of ``n`` Gaussians of a synthetic city (generation order, not
    spatially sorted): streets every ``pitch`` metres, ``street_width``
    wide; buildings from a Poisson process over the non-street area with
    square footprints of side U(10, 40) m and heights U(10, 100) m; each
    building gets Gaussians in proportion to its footprint area, uniform
    over its footprint x [0, h]; ``ground_frac`` of the Gaussians lie on the
    street ground (z ~ N(0, 0.1^2)).  Returns (f64 [n, 3], City)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    half = extent / 2.0
    inner = pitch - street_width
    per_row = int(round(extent / pitch))
    n_lots = per_row ** 2
    expected = buildings_per_km2 * (extent / 1000.0) ** 2 * (inner / pitch) ** 2
    n_b = max(1, int(rng.poisson(expected)))
    lot = rng.integers(0, n_lots, size=n_b)
    side = rng.uniform(10.0, 40.0, size=n_b)
    h = rng.uniform(10.0, 100.0, size=n_b)
    # footprint centre inside its lot, footprint kept off the street
    lo = street_width / 2.0 + np.minimum(side / 2.0, inner / 2.0)
    off_x = rng.uniform(lo, pitch - lo)
    off_y = rng.uniform(lo, pitch - lo)
    bx = -half + (lot % per_row) * pitch + off_x
    by = -half + (lot // per_row) * pitch + off_y
    n_ground = int(round(ground_frac * n))
    w = side * side
    counts = rng.multinomial(n - n_ground, w / w.sum())
    idx = np.repeat(np.arange(n_b), counts)
    mu = np.empty((n, 3))
    m = n - n_ground
    mu[:m, 0] = bx[idx] + (rng.uniform(-0.5, 0.5, size=m) * side[idx])
    mu[:m, 1] = by[idx] + (rng.uniform(-0.5, 0.5, size=m) * side[idx])
    mu[:m, 2] = rng.uniform(0.0, 1.0, size=m) * h[idx]
    # street ground: along a random street line, across its width
    along = rng.uniform(-half, half, size=n_ground)
    line = -half + pitch * rng.integers(0, per_row, size=n_ground)
    across = rng.uniform(-street_width / 2.0, street_width / 2.0, size=n_ground)
    horiz = rng.integers(0, 2, size=n_ground).astype(bool)
    mu[m:, 0] = np.where(horiz, along, line + across)
    mu[m:, 1] = np.where(horiz, line + across, along)
    mu[m:, 2] = rng.normal(0.0, 0.1, size=n_ground)
    return mu, City(extent, pitch, street_width)


def city_scene(n: int, seed: int, extent: float = 4000.0, pitch: float = 100.0, street_width: float = 20.0,
               buildings_per_km2: float = 400.0, ground_frac: float = 0.1,
               logscale_mu: float = -1.0, logscale_sigma: float = 0.7):
    """city_means plus the aerial-recipe attributes: (f32 [n, 59], City)."""
    mu, city = city_means(n, seed, extent, pitch, street_width, buildings_per_km2, ground_frac)
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    th = _attributes(rng, n, logscale_mu, logscale_sigma)
    th[:, 0:3] = mu
    return th.astype(np.float32), city


def block_attributes(seed: int, block: int, n: int, logscale_mu: float = -1.0,
                     logscale_sigma: float = 0.7) -> np.ndarray:
    """Attributes (every column but the means, which stay zero) of block
    ``block``'s n Gaussians, drawn in single precision from a stream keyed
    by (seed, block), so that a large scene is generated one block at a
    time: f32 [n, 59] with the aerial recipe's distributions."""
    rng = np.random.Generator(np.random.PCG64([seed, block]))
    th = np.zeros((n, D), dtype=np.float32)
    th[:, 3:6] = rng.standard_normal((n, 3), dtype=np.float32) * np.float32(logscale_sigma) + np.float32(logscale_mu)
    q = rng.standard_normal((n, 4), dtype=np.float32)
    th[:, 6:10] = q / np.linalg.norm(q, axis=1, keepdims=True)
    th[:, 10] = rng.standard_normal(n, dtype=np.float32)
    th[:, 11:14] = rng.standard_normal((n, 3), dtype=np.float32) * np.float32(0.3)
    th[:, 14:59] = rng.standard_normal((n, 45), dtype=np.float32) * np.float32(0.05)
    return th


def street_walk(city: City, n_poses: int, seed: int, step: float = 1.0, eye_height: float = 1.7,
                width: int = 1600, height: int = 900, hfov_deg: float = 60.0, z_far: float = 1000.0,
                z_near: float = 0.2) -> list[Camera]:
    """A random walk along the street centre lines: ``step`` metres per pose
    at ``eye_height``, looking along the direction of travel; at every
    intersection a uniformly chosen new direction among those that neither
    turn back nor leave the city."""
    rng = np.random.Generator(np.random.PCG64(seed))
    half = city.extent / 2.0
    p = city.pitch
    n_lines = int(round(city.extent / p))
    coords = -half + p * np.arange(n_lines + 1)     # street centre lines (incl. the border)
    dirs = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)]
    x = float(coords[rng.integers(1, n_lines)])
    y = float(coords[rng.integers(1, n_lines)])
    d = int(rng.integers(0, 4))
    f = focal_for_hfov(width, hfov_deg)
    steps_per_block = int(round(p / step))
    out = []
    k = 0
    for _ in range(n_poses):
        if k % steps_per_block == 0:
            ok = []
            for nd in range(4):
                if nd == (d + 2) % 4:
                    continue
                nx, ny = x + dirs[nd][0] * p, y + dirs[nd][1] * p
                if -half - 1e-6 <= nx <= half + 1e-6 and -half - 1e-6 <= ny <= half + 1e-6:
                    ok.append(nd)
            d = ok[int(rng.integers(0, len(ok)))] if ok else (d + 2) % 4
        eye = (x, y, eye_height)
        out.append(look_at(eye, (x + dirs[d][0], y + dirs[d][1], eye_height), (0.0, 0.0, 1.0), width, height, f,
                           z_near, z_far))
        x += dirs[d][0] * step
        y += dirs[d][1] * step
        k += 1
    return out


def blob_centres(n_blobs: int, half_extent: float, height: tuple[float, float], seed: int) -> np.ndarray:
    """Blob centres of blob_scene_parallel: x, y ~ U(-half_extent, half_extent), z ~ U(height)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cx = rng.uniform(-half_extent, half_extent, size=n_blobs)
    cy = rng.uniform(-half_extent, half_extent, size=n_blobs)
    cz = rng.uniform(height[0], height[1], size=n_blobs)
    return np.stack([cx, cy, cz], axis=1)


def blob_scene_parallel(n_blobs: int, per_blob: int, half_extent: float, height: tuple[float, float], sigma: float,
                        seed: int, order=None, logscale_mu: float = -1.0, logscale_sigma: float = 0.7,
                        workers: int = 16) -> np.ndarray:
    """The aerial blob recipe at large N, generated blob by blob on threads:
    blob b's Gaussians come from a stream keyed by (seed, b) (single
    precision draws), members N(centre_b, sigma^2 I).  ``order`` lists the
    blobs in the order their rows are laid out (default: blob id order).
    Returns f32 [n_blobs * per_blob, 59]."""
    import concurrent.futures as cf
    centres = blob_centres(n_blobs, half_extent, height, seed)
    order = np.arange(n_blobs) if order is None else np.asarray(order)
    out = np.empty((n_blobs * per_blob, D), dtype=np.float32)

    def fill(j):
        b = int(order[j])
        rng = np.random.Generator(np.random.PCG64([seed, b]))
        th = out[j * per_blob:(j + 1) * per_blob]
        th[:, 0:3] = (rng.standard_normal((per_blob, 3), dtype=np.float32) * np.float32(sigma) +
                      centres[b].astype(np.float32))
        th[:, 3:6] = (rng.standard_normal((per_blob, 3), dtype=np.float32) * np.float32(logscale_sigma) +
                      np.float32(logscale_mu))
        q = rng.standard_normal((per_blob, 4), dtype=np.float32)
        th[:, 6:10] = q / np.linalg.norm(q, axis=1, keepdims=True)
        th[:, 10] = rng.standard_normal(per_blob, dtype=np.float32)
        th[:, 11:14] = rng.standard_normal((per_blob, 3), dtype=np.float32) * np.float32(0.3)
        th[:, 14:59] = rng.standard_normal((per_blob, 45), dtype=np.float32) * np.float32(0.05)

    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(fill, range(n_blobs)))
    return out
