"""Seeded scene, camera and request generators.

Every workload here is synthetic: the paper measures on trained scenes of the
Mip-NeRF360, Tanks&Temples and Blender datasets (Methodology section), which
are not available, so scenes with the Gaussian counts, scale ranges, opacity
distribution and SH degree of the benchmark configurations stand in for them.

Layout (structure of arrays, float32, component-major so that a GPU thread per
Gaussian reads each component coalesced):
  means      [3][n]
  scales     [3][n]   activated (exp of the log-scales)
  quats      [4][n]   (w, x, y, z), unit norm as drawn
  opacities  [n]      activated (sigmoid of the logits)
  sh         [K][3][n] with K = (degree+1)^2 coefficients, coefficient-major
The raw draws (log-scales, opacity logits) are kept as well for autograd tests.

Draw order for one scene (numpy PCG64, ``default_rng(seed)``):
  cluster centres [64,3] ~ U(-3,3); cluster id ~ integers(0,64);
  means = clip(centre + N(0, 0.3^2), -3, 3)     (config 1: U(-1,1)^3 instead)
  log-scales [n,3] ~ U(ln lo, ln hi)
  quats = normalise(N(0, I4))
  opacity logits ~ N(0, sigma_o)
  SH: DC [n,3] ~ U(0,1), higher orders [n,K-1,3] ~ N(0, 0.05^2)
      (config 1: rgb ~ U(0,1) and the DC coefficient is chosen so the
       degree-0 colour equals rgb).
Cameras come from their own stream ``default_rng(seed + 1)``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# The degree-0 real spherical harmonic is the constant 1/(2*sqrt(pi)); it is
# only used here to encode a wanted RGB colour as an SH DC coefficient.
_Y00 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Scene:
    means: np.ndarray      # [3][n] f32
    scales: np.ndarray     # [3][n] f32
    quats: np.ndarray      # [4][n] f32
    opacities: np.ndarray  # [n] f32
    sh: np.ndarray         # [K][3][n] f32
    log_scales: np.ndarray  # [3][n] f32
    logits: np.ndarray     # [n] f32
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.opacities.shape[0])

    @property
    def sh_coeffs(self) -> int:
        return int(self.sh.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(
            means=np.ascontiguousarray(self.means[:, idx]),
            scales=np.ascontiguousarray(self.scales[:, idx]),
            quats=np.ascontiguousarray(self.quats[:, idx]),
            opacities=np.ascontiguousarray(self.opacities[idx]),
            sh=np.ascontiguousarray(self.sh[:, :, idx]),
            log_scales=np.ascontiguousarray(self.log_scales[:, idx]),
            logits=np.ascontiguousarray(self.logits[idx]),
            sh_degree=self.sh_degree,
        )

    def nbytes(self) -> int:
        return sum(a.nbytes for a in (self.means, self.scales, self.quats,
                                      self.opacities, self.sh))


@dataclasses.dataclass
class Camera:
    """World-to-camera pinhole camera (x right, y down, z forward).

    R is a row-major rotation, t a translation: x_cam = R @ x_world + t.
    (cx, cy) is the principal point in continuous pixel coordinates, where
    pixel (i, j) covers [i, i+1) x [j, j+1).
    """
    R: np.ndarray   # [3,3] f64
    t: np.ndarray   # [3] f64
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def position(self) -> np.ndarray:
        return -self.R.T @ self.t


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _finish(rng, means, n, lo, hi, sigma_o, sh_degree, rgb_dc):
    log_s = rng.uniform(math.log(lo), math.log(hi), size=(n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logits = rng.normal(0.0, sigma_o, size=n)
    K = (sh_degree + 1) ** 2
    sh = np.zeros((n, K, 3))
    if rgb_dc:
        rgb = rng.uniform(0.0, 1.0, size=(n, 3))
        sh[:, 0, :] = (rgb - 0.5) / _Y00
    else:
        sh[:, 0, :] = rng.uniform(0.0, 1.0, size=(n, 3))
        if K > 1:
            sh[:, 1:, :] = rng.normal(0.0, 0.05, size=(n, K - 1, 3))
    f32 = np.float32
    log_s32 = log_s.astype(f32)
    logits32 = logits.astype(f32)
    return Scene(
        means=np.ascontiguousarray(means.T.astype(f32)),
        scales=np.ascontiguousarray(np.exp(log_s32.astype(np.float64)).astype(f32).T),
        quats=np.ascontiguousarray(q.T.astype(f32)),
        opacities=_sigmoid(logits32.astype(np.float64)).astype(f32),
        sh=np.ascontiguousarray(np.transpose(sh, (1, 2, 0)).astype(f32)),
        log_scales=np.ascontiguousarray(log_s32.T),
        logits=logits32,
        sh_degree=sh_degree,
    )


def scene_uniform_cube(n: int = 10_000, seed: int = 0) -> Scene:
    """Means U[-1,1]^3, log-scales U[ln .005, ln .05], opacity sigmoid(N(0,1)),
    RGB U[0,1] as SH degree 0."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(n, 3))
    return _finish(rng, means, n, 0.005, 0.05, 1.0, 0, rgb_dc=True)


def scene_clusters(n: int, seed: int = 0, sh_degree: int = 3,
                   lo: float = 0.002, hi: float = 0.1, sigma_o: float = 1.5,
                   n_clusters: int = 64, box: float = 3.0,
                   cluster_sigma: float = 0.3) -> Scene:
    """Means from a mixture of isotropic normal clusters inside [-box, box]^3."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-box, box, size=(n_clusters, 3))
    cid = rng.integers(0, n_clusters, size=n)
    means = np.clip(centres[cid] + rng.normal(0.0, cluster_sigma, size=(n, 3)),
                    -box, box)
    return _finish(rng, means, n, lo, hi, sigma_o, sh_degree, rgb_dc=False)


def _focal(width: int, fov_deg: float) -> float:
    return width / (2.0 * math.tan(math.radians(fov_deg) / 2.0))


def camera_look_at(pos, width: int, height: int, fov_deg: float = 60.0,
                   target=(0.0, 0.0, 0.0)) -> Camera:
    """Pinhole camera at ``pos`` looking at ``target``; ``fov_deg`` is the
    horizontal field of view and pixels are square."""
    pos = np.asarray(pos, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - pos
    f /= np.linalg.norm(f)
    up = np.array([0.0, 1.0, 0.0])
    if abs(f @ up) > 0.99:
        up = np.array([0.0, 0.0, 1.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f])
    t = -R @ pos
    fx = _focal(width, fov_deg)
    return Camera(R=R, t=t, fx=fx, fy=fx, cx=width / 2.0, cy=height / 2.0,
                  width=int(width), height=int(height))


def camera_front(width: int = 256, height: int = 256) -> Camera:
    return camera_look_at((0.0, 0.0, -4.0), width, height)


def random_cameras(k: int, seed: int, resolutions, radius: float = 6.0,
                   rng=None):
    """k cameras on a sphere of ``radius`` looking at the origin.

    ``resolutions`` is either one (W, H) pair or a list to draw from
    uniformly (one draw per camera, after the position draw)."""
    rng = np.random.default_rng(seed + 1) if rng is None else rng
    cams = []
    for _ in range(k):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        if isinstance(resolutions[0], (tuple, list)):
            W, H = resolutions[int(rng.integers(0, len(resolutions)))]
        else:
            W, H = resolutions
        cams.append(camera_look_at(radius * u, W, H))
    return cams


def request_stream(n_requests: int, rate_hz: float, n_scenes: int,
                   resolutions, seed: int = 7):
    """Poisson view requests: (arrival_s, scene_id, camera)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        sid = int(rng.integers(0, n_scenes))
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        W, H = resolutions[int(rng.integers(0, len(resolutions)))]
        out.append((t, sid, camera_look_at(6.0 * u, W, H)))
    return out


# The benchmark configurations (sizes only; see the generators above).
CONFIGS = {
    "cube_10k_256": dict(n=10_000, res=(256, 256), sh_degree=0, tile=16),
    "clusters_1M_1297x840": dict(n=1_000_000, res=(1297, 840), sh_degree=3, tile=16),
    "clusters_3M_1600x1064": dict(n=3_000_000, res=(1600, 1064), sh_degree=3, tile=16, cameras=8),
    "batched_2M_16views": dict(n=2_000_000, sh_degree=3, cameras=16,
               res_set=[(256, 256), (640, 480), (1297, 840), (1600, 1064),
                        (1920, 1080)]),
    "serving_4scenes": dict(scenes=[100_000, 500_000, 1_500_000, 3_000_000], sh_degree=3,
               rate_hz=200.0,
               res_set=[(512, 512), (1280, 720), (1920, 1080)]),
}
