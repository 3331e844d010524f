"""Seeded synthetic scenes and cameras (input generators only).

This module builds the inputs that both the HIP path and the FP64 CPU oracle
consume: Gaussian parameters as component-major float32 arrays (the
rasteriser's front end moves the colour arrays Gaussian-major for the
C-ABI), pinhole cameras and target images.  It holds none of the
rasteriser's arithmetic: no projection, no colour model, no blending.

The paper trains on photographic datasets (Mip-NeRF360, Tanks&Temples,
DeepBlending; Experiments section) that are not available here.  The scenes
below stand in for them with the shapes the paper's workloads have: millions
of small anisotropic Gaussians grouped in spatial clusters, seen by a pinhole
camera at 1.6K width.

Layouts (N Gaussians, L = SH degree, K = number of SG lobes):
  means (3,N), log_scales (3,N), quats (4,N) as (w,x,y,z), opacity_logits (N,),
  sh ((L+1)^2, 3, N), sg_axes (K,3,N), sg_log_sharpness (K,N),
  sg_amplitudes (K,3,N).  All float32, C-contiguous.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh",
          "sg_axes", "sg_log_sharpness", "sg_amplitudes")

# How the lobe axes are given (the values of the C-ABI's lobe_axes field):
#   LOBES_FREE  every lobe has its own axis, sg_axes (K, 3, N)
#   LOBES_WORLD three lobes on the fixed world axes (1,0,0), (0,1,0), (0,0,1);
#               sg_axes is empty (0, 3, N)
#   LOBES_FRAME three mutually orthogonal lobes on the columns of a rotation
#               given by 3 parameters per Gaussian, sg_axes (1, 3, N)
LOBES_FREE, LOBES_WORLD, LOBES_FRAME = 0, 1, 2


def axis_vectors(lobe_mode: int, n_lobes: int) -> int:
    """Rows of sg_axes (3-vectors per Gaussian) for a lobe mode."""
    return {LOBES_FREE: n_lobes, LOBES_WORLD: 0, LOBES_FRAME: 1}[lobe_mode]


@dataclass
class Scene:
    sh_degree: int
    n_lobes: int
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sg_axes: np.ndarray
    sg_log_sharpness: np.ndarray
    sg_amplitudes: np.ndarray
    lobe_mode: int = LOBES_FREE
    # adaptive SH degree by projected radius r (pixels): degree 0 where
    # r <= sh_adaptive[0], at most 1 where r <= sh_adaptive[1], else
    # sh_degree; (0, 0) = every Gaussian uses sh_degree
    sh_adaptive: tuple = (0, 0)

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @property
    def n_axis_vectors(self) -> int:
        return axis_vectors(self.lobe_mode, self.n_lobes)

    def arrays(self) -> dict:
        return {k: getattr(self, k) for k in FIELDS}

    def floats_per_gaussian(self) -> int:
        return (3 + 3 + 4 + 1 + 3 * (self.sh_degree + 1) ** 2 + 3 * self.n_axis_vectors
                + 4 * self.n_lobes)

    def form(self) -> dict:
        """The colour form (everything but the arrays)."""
        return {"sh_degree": self.sh_degree, "n_lobes": self.n_lobes,
                "lobe_mode": self.lobe_mode, "sh_adaptive": tuple(self.sh_adaptive)}

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        out = {}
        for k in FIELDS:
            a = getattr(self, k)
            out[k] = np.ascontiguousarray(a[..., idx])
        return Scene(self.sh_degree, self.n_lobes, **out, lobe_mode=self.lobe_mode,
                     sh_adaptive=tuple(self.sh_adaptive))

    def copy(self) -> "Scene":
        return Scene(self.sh_degree, self.n_lobes,
                     **{k: getattr(self, k).copy() for k in FIELDS}, lobe_mode=self.lobe_mode,
                     sh_adaptive=tuple(self.sh_adaptive))


@dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).

    A world point X maps to camera space as R @ X + t; pixel (i, j) is
    sampled at integer coordinates (i, j).
    """
    width: int
    height: int
    R: np.ndarray            # (3,3) float32, world -> camera, row-major
    t: np.ndarray            # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    znear: float = 0.2
    bg: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))

    def __post_init__(self):
        self.R = np.asarray(self.R, np.float32).reshape(3, 3)
        self.t = np.asarray(self.t, np.float32).reshape(3)
        self.bg = np.asarray(self.bg, np.float32).reshape(3)
        self.fx = float(np.float32(self.fx))
        self.fy = float(np.float32(self.fy))
        self.cx = float(np.float32(self.cx))
        self.cy = float(np.float32(self.cy))
        self.znear = float(np.float32(self.znear))


@dataclass
class Options:
    """Rasteriser options.  Every float is a float32 value, as at the C-ABI."""
    tile_w: int = 16
    tile_h: int = 16
    batch: int = 0              # LDS batch depth, 0 = library default
    ppt: int = 0                # pixels per thread, forward blend (0 = library default)
    ppt_bwd: int = 0            # pixels per thread, backward blend
    schedule: int = 0           # blend tile schedule: 1 grid, 2 heavy-first queue, 3 heavy-first
                                # one-wave slices of tiles, 0 = library
                                # default (queue for several cameras)
    dilation: float = 0.3
    guard: float = 1.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4

    def __post_init__(self):
        for k in ("dilation", "guard", "alpha_min", "alpha_max", "t_min"):
            setattr(self, k, float(np.float32(getattr(self, k))))


def pinhole(width: int, height: int, R, t, hfov_deg: float = 60.0,
            znear: float = 0.2, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Camera with the given horizontal field of view and a centred principal
    point ((W-1)/2, (H-1)/2); square pixels (fy = fx)."""
    fx = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return Camera(width, height, R, t, fx, fx, (width - 1) / 2.0,
                  (height - 1) / 2.0, znear, np.asarray(bg, np.float32))


def look_at(eye, target, up=(0.0, -1.0, 0.0)):
    """World->camera (R, t) for a camera at `eye` looking at `target`
    (OpenCV axes: camera y points down, so `up` is the world's down-screen
    direction negated)."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    f = target - eye
    f /= np.linalg.norm(f)
    down = -np.asarray(up, np.float64)
    r = np.cross(down, f)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])          # rows: camera x, y, z axes in world
    t = -R @ eye
    return R.astype(np.float32), t.astype(np.float32)


def _unit_rows(rng, n, dim):
    v = rng.standard_normal((n, dim))
    nv = np.linalg.norm(v, axis=1, keepdims=True)
    nv[nv == 0] = 1.0
    return v / nv


def _colour_params(rng, n, sh_degree, n_lobes, dc_sigma, hi_sigma):
    nc = (sh_degree + 1) ** 2
    sh = np.empty((nc, 3, n), np.float32)
    sh[0] = rng.normal(0.0, dc_sigma, (3, n))
    if nc > 1:
        sh[1:] = rng.normal(0.0, hi_sigma, (nc - 1, 3, n))
    axes = np.empty((n_lobes, 3, n), np.float32)
    for k in range(n_lobes):
        axes[k] = _unit_rows(rng, n, 3).T
    lsharp = rng.normal(1.0, 0.5, (n_lobes, n)).astype(np.float32)
    amp = rng.normal(0.0, 0.2, (n_lobes, 3, n)).astype(np.float32)
    return sh, axes, lsharp, amp


def _shape_params(rng, n):
    log_scales = rng.normal(-3.0, 0.5, (3, n)).astype(np.float32)
    quats = _unit_rows(rng, n, 4).T.astype(np.float32)
    opacity = rng.standard_normal(n).astype(np.float32)
    return log_scales, quats, opacity


def config0_scene(seed: int = 0, n: int = 1000) -> Scene:
    """1,000 Gaussians, means uniform in [-1,1]^3, SH degree 0 + 3 lobes."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (3, n)).astype(np.float32)
    ls, q, op = _shape_params(rng, n)
    sh, axes, lsh, amp = _colour_params(rng, n, 0, 3, 0.3, 0.1)
    return Scene(0, 3, np.ascontiguousarray(means), ls, q, op, sh, axes, lsh, amp)


def config0_camera(width: int = 128, height: int = 128) -> Camera:
    """Camera at distance 4 on the -z axis looking at the origin, 60 deg FOV."""
    return pinhole(width, height, np.eye(3), (0.0, 0.0, 4.0))


def clustered_means(rng, n, n_clusters, log_sigma_mu, centre_radius=8.0,
                    ball_radius=10.0):
    """Mixture of anisotropic Gaussian clusters inside a ball.

    Cluster centres are uniform in a ball of radius `centre_radius`; each
    cluster has per-axis spread exp(N(log_sigma_mu, 0.5)) under a random
    rotation; cluster weights are proportional to exp(N(0,1)); points that
    land outside `ball_radius` are drawn again from their cluster.
    """
    u = rng.uniform(0.0, 1.0, n_clusters) ** (1.0 / 3.0)
    centres = _unit_rows(rng, n_clusters, 3) * (centre_radius * u)[:, None]
    sig = np.exp(rng.normal(log_sigma_mu, 0.5, (n_clusters, 3)))
    rots = np.empty((n_clusters, 3, 3))
    for c in range(n_clusters):
        qm, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        rots[c] = qm
    w = np.exp(rng.standard_normal(n_clusters))
    w /= w.sum()
    assign = rng.choice(n_clusters, size=n, p=w)
    pts = np.empty((n, 3))
    todo = np.arange(n)
    while todo.size:
        c = assign[todo]
        z = rng.standard_normal((todo.size, 3)) * sig[c]
        p = centres[c] + np.einsum("nij,nj->ni", rots[c], z)
        ok = np.einsum("ni,ni->n", p, p) <= ball_radius ** 2
        pts[todo[ok]] = p[ok]
        todo = todo[~ok]
    return np.ascontiguousarray(pts.T.astype(np.float32))


def clustered_scene(n: int, seed: int, sh_degree: int = 1, n_lobes: int = 4,
                    n_clusters: int = 500, log_sigma_mu: float = math.log(0.5),
                    sh_dc_sigma: float = 0.3, sh_hi_sigma: float = 0.1) -> Scene:
    """Clustered scene; colour = SH of `sh_degree` + `n_lobes` SG lobes.

    The geometry draws come first from the generator so that two calls with
    the same seed and different colour forms share identical geometry.
    """
    rng = np.random.default_rng(seed)
    means = clustered_means(rng, n, n_clusters, log_sigma_mu)
    ls, q, op = _shape_params(rng, n)
    crng = np.random.default_rng([seed, sh_degree, n_lobes])
    sh, axes, lsh, amp = _colour_params(crng, n, sh_degree, n_lobes,
                                        sh_dc_sigma, sh_hi_sigma)
    return Scene(sh_degree, n_lobes, means, ls, q, op, sh, axes, lsh, amp)


def sh3_scene(n: int, seed: int, **kw) -> Scene:
    """Same geometry as `clustered_scene(n, seed)`, colour = degree-3 SH with
    all 48 coefficients N(0, 0.1) and no lobes."""
    rng = np.random.default_rng(seed)
    means = clustered_means(rng, n, kw.get("n_clusters", 500),
                            kw.get("log_sigma_mu", math.log(0.5)))
    ls, q, op = _shape_params(rng, n)
    crng = np.random.default_rng([seed, 3, 0])
    sh = crng.normal(0.0, 0.1, (16, 3, n)).astype(np.float32)
    z3 = np.zeros((0, 3, n), np.float32)
    return Scene(3, 0, means, ls, q, op, sh, z3, np.zeros((0, n), np.float32), z3.copy())


def orthogonal_scene(n: int, seed: int, lobe_mode: int, sh_degree: int = 0,
                     sh_adaptive=(0, 0), n_clusters: int = 500,
                     log_sigma_mu: float = math.log(0.5)) -> Scene:
    """Same geometry as `clustered_scene(n, seed)` with three mutually
    orthogonal lobes: on the world axes (LOBES_WORLD) or on the columns of a
    per-Gaussian rotation whose 3 parameters are N(0, 1) (LOBES_FRAME).
    SH: degree-0 coefficients N(0, 0.3), higher degrees N(0, 0.1); lobe
    log-sharpness N(1, 0.5), amplitudes N(0, 0.2)."""
    rng = np.random.default_rng(seed)
    means = clustered_means(rng, n, n_clusters, log_sigma_mu)
    ls, q, op = _shape_params(rng, n)
    crng = np.random.default_rng([seed, sh_degree, 3, 100 + lobe_mode])
    nc = (sh_degree + 1) ** 2
    sh = np.empty((nc, 3, n), np.float32)
    sh[0] = crng.normal(0.0, 0.3, (3, n))
    if nc > 1:
        sh[1:] = crng.normal(0.0, 0.1, (nc - 1, 3, n))
    A = axis_vectors(lobe_mode, 3)
    axes = crng.normal(0.0, 1.0, (A, 3, n)).astype(np.float32)
    lsh = crng.normal(1.0, 0.5, (3, n)).astype(np.float32)
    amp = crng.normal(0.0, 0.2, (3, 3, n)).astype(np.float32)
    return Scene(sh_degree, 3, means, ls, q, op, sh, axes, lsh, amp, lobe_mode=lobe_mode,
                 sh_adaptive=tuple(sh_adaptive))


# adaptive SH thresholds used by the "full" form (projected radius, pixels):
# the smallest splats (radius 2, the floor the dilation sets) take degree 0,
# radius up to 8 degree 1, larger ones degree 2
ADAPTIVE_SH_RADII = (2, 8)


def config1_camera(width: int = 1600, height: int = 1060) -> Camera:
    """Camera inside the scene ball at (0,0,-5), looking at the centre."""
    return pinhole(width, height, np.eye(3), (0.0, 0.0, 5.0))


def ring_cameras(n_cams: int = 64, radius: float = 6.0, seed: int = 3,
                 sizes=((640, 480), (800, 800), (1280, 720))):
    """Cameras on a horizontal circle looking at the origin; each camera's
    resolution is drawn uniformly from `sizes`."""
    rng = np.random.default_rng(seed)
    pick = rng.integers(0, len(sizes), n_cams)
    cams = []
    for k in range(n_cams):
        th = 2.0 * math.pi * k / n_cams
        eye = (radius * math.cos(th), 0.0, radius * math.sin(th))
        R, t = look_at(eye, (0.0, 0.0, 0.0))
        w, h = sizes[pick[k]]
        cams.append(pinhole(w, h, R, t))
    return cams


def target_image(width: int, height: int, seed: int) -> np.ndarray:
    """Seeded target image, uniform in [0,1], layout (3, H, W) float32."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, (3, height, width)).astype(np.float32)


# Named workloads ------------------------------------------------------------

def workload(name: str):
    """Return (scene, cameras, options) for a named workload.

    sg-1k-128      : 1,000 Gaussians, SH0 + 3 lobes, 128x128 (seed 0)
    sg-3m-1600     : 3M clustered Gaussians, SH1 + 4 lobes, 1600x1060 (seed 1)
    sh3-3m-1600    : same geometry, degree-3 SH colour
    orthw-3m-1600  : same geometry, SH0 + 3 lobes on the world axes
    full-3m-1600   : same geometry, adaptive SH (0-2) + 3 lobes on a
                     per-Gaussian orthonormal frame
    sg-1m-1297     : 1M clustered, SH1 + 4 lobes, 1297x840 (seed 2), L1 target
    sg-2m-64cam    : 2M clustered, 64 ring cameras of mixed size (seed 3)
    sg-6m-1920     : 6M Gaussians in 2,000 tight clusters, 1920x1080 (seed 4)
    """
    if name == "sg-1k-128":
        return config0_scene(0), [config0_camera()], Options()
    if name == "sg-3m-1600":
        return clustered_scene(3_000_000, 1), [config1_camera()], Options()
    if name == "sh3-3m-1600":
        return sh3_scene(3_000_000, 1), [config1_camera()], Options()
    if name == "orthw-3m-1600":
        return orthogonal_scene(3_000_000, 1, LOBES_WORLD), [config1_camera()], Options()
    if name == "full-3m-1600":
        return (orthogonal_scene(3_000_000, 1, LOBES_FRAME, sh_degree=2,
                                 sh_adaptive=ADAPTIVE_SH_RADII), [config1_camera()], Options())
    if name == "sg-1m-1297":
        return clustered_scene(1_000_000, 2), [config1_camera(1297, 840)], Options()
    if name == "sg-2m-64cam":
        return clustered_scene(2_000_000, 3), ring_cameras(), Options()
    if name == "sg-6m-1920":
        sc = clustered_scene(6_000_000, 4, n_clusters=2000,
                             log_sigma_mu=math.log(0.05))
        return sc, [config1_camera(1920, 1080)], Options()
    raise KeyError(name)


def small_clustered(n: int, seed: int, width: int, height: int,
                    sh_degree: int = 1, n_lobes: int = 4, n_clusters: int = 20):
    """A reduced clustered scene for parity tests: the same laws as the
    large scenes at a size the oracle finishes in seconds."""
    sc = clustered_scene(n, seed, sh_degree, n_lobes, n_clusters=n_clusters)
    return sc, config1_camera(width, height)
