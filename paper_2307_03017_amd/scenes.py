"""Seeded synthetic forward-facing scenes: the inputs of an HSGD refinement.

This module only draws and rasterises inputs. It holds none of the method's
arithmetic (no homography, no compositing, no loss, no resampling of an MPI or
an image); the FP64 oracle and the HIP path both consume what it produces and
each computes everything else on its own.

The paper evaluates on real forward-facing captures (a handful of posed views,
tens of fronto-parallel planes, one dominant surface per pixel, Sec. 3.3 and
Sec. 5.1). Those datasets are not available here, so seeded procedural scenes
with the same structure stand in for them:

* planes: inverse depth uniform on [0.01, 1], plane 0 the nearest (depth 1);
* depth: a 6x5 grid of uniform inverse depths, bilinearly interpolated over the
  image; every pixel puts alpha = 1 on the plane nearest in inverse depth
  (ties to the nearer plane) and alpha = 0 elsewhere;
* colour: per plane, a Voronoi partition of 24 seeds, each cell a uniform RGB
  colour (ties to the lower seed index);
* cameras: pinhole, principal point at the image centre, identity rotation,
  translation (U(-a, a), U(-a, a), 0) per source view; the reference camera is
  the identity pose;
* initial MPI (stand-in for the paper's initial-MPI network, Sec. 3.2): the
  ground truth rasterised at the coarsest level with Gaussian noise on the alpha
  logits (sigma 0.5, alpha clipped to [0.01, 0.99] first) and on colour
  (sigma 0.1, clipped to [0, 1]).

The scene is resolution independent: ``rasterise`` evaluates it at pixel centres
of any (h, w) grid, so the coarse initial MPI and the full-resolution ground
truth are two samplings of one procedural scene.
"""

from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

# Workloads. Sizes, views, focal lengths, translation ranges, hierarchy and k
# follow the synthetic stand-ins for the paper's forward-facing setting
# (Sec. 4 uses 40 planes, k = 5, 3 iterations on 378x512 frames).
CONFIGS = {
    # tiny case: the oracle runs it in well under a second
    "c1": dict(W=64, H=48, D=8, N=3, f=60.0, a=0.05, levels=2, iters=(2, 1), k=2, seed=1),
    # the benchmark frame: 512x384, 32 planes, 4 views, 3 levels, 1 iteration each
    "c2": dict(W=512, H=384, D=32, N=4, f=400.0, a=0.1, levels=3, iters=(1, 1, 1), k=4, seed=2),
    # serving-mix frame sizes (resolution, planes, k); views and seeds vary per scene
    "s256": dict(W=256, H=192, D=16, N=3, f=200.0, a=0.1, levels=3, iters=(1, 1, 1), k=2, seed=100),
    "s512": dict(W=512, H=384, D=32, N=4, f=400.0, a=0.1, levels=3, iters=(1, 1, 1), k=4, seed=103),
    "s1008": dict(W=1008, H=756, D=32, N=5, f=787.5, a=0.1, levels=3, iters=(1, 1, 1), k=4, seed=106),
    # large XR frame: 1920x1080, 64 planes, 8 views, 4 levels (coarsest holds only the initial MPI)
    "c5": dict(W=1920, H=1080, D=64, N=8, f=1500.0, a=0.15, levels=4, iters=(0, 1, 1, 1), k=3, seed=5),
    # the benchmark frame with tilted cameras: every view also rotated (Euler angles with a
    # 0.01 rad standard deviation) and moved along z (within +-0.02), as hand-held
    # forward-facing captures are, so its plane maps are general homographies
    "c2g": dict(W=512, H=384, D=32, N=4, f=400.0, a=0.1, levels=3, iters=(1, 1, 1), k=4, seed=2,
                tilt=0.01, tz=0.02),
}

ALPHA_EPS = 0.01
ALPHA_LOGIT_SIGMA = 0.5
COLOUR_SIGMA = 0.1
N_VORONOI = 24
GRID_COLS, GRID_ROWS = 6, 5


def plane_depths(D: int) -> np.ndarray:
    """Plane depths, plane 0 nearest: inverse depth linear from 1 down to 0.01."""
    z = np.arange(D, dtype=np.float64)
    inv = 1.0 - z * (1.0 - 0.01) / max(D - 1, 1)
    return 1.0 / inv


def level_shapes(W: int, H: int, levels: int):
    """(w, h) of each hierarchy level, coarsest first; each level halves the next."""
    out = []
    for l in range(levels):
        s = 2 ** (levels - 1 - l)
        if W % s or H % s:
            raise ValueError(f"{W}x{H} is not divisible by {s} for {levels} levels")
        out.append((W // s, H // s))
    return out


@dataclass
class Scene:
    W: int
    H: int
    D: int
    N: int
    f: float
    a: float
    levels: int
    iters: tuple
    k: int
    seed: int
    depths: np.ndarray = field(repr=False, default=None)
    grid: np.ndarray = field(repr=False, default=None)        # [ROWS][COLS] inverse depths
    seeds_xy: np.ndarray = field(repr=False, default=None)    # [D][24][2] in [0,1]^2
    seeds_rgb: np.ndarray = field(repr=False, default=None)   # [D][24][3]
    t: np.ndarray = field(repr=False, default=None)           # [N][3] camera translations
    R: np.ndarray = field(repr=False, default=None)           # [N][3][3] camera rotations (identity unless tilted)
    init_noise_a: np.ndarray = field(repr=False, default=None)
    init_noise_c: np.ndarray = field(repr=False, default=None)

    # --- cameras (full resolution) -------------------------------------------------------
    def K_ref(self) -> np.ndarray:
        return np.array([[self.f, 0.0, (self.W - 1) / 2.0],
                         [0.0, self.f, (self.H - 1) / 2.0],
                         [0.0, 0.0, 1.0]])

    def K_views(self) -> np.ndarray:
        return np.repeat(self.K_ref()[None], self.N, axis=0)

    def R_views(self) -> np.ndarray:
        if self.R is not None:
            return self.R.copy()
        return np.repeat(np.eye(3)[None], self.N, axis=0)

    def t_views(self) -> np.ndarray:
        return self.t.copy()

    def shapes(self):
        return level_shapes(self.W, self.H, self.levels)

    # --- rasterisation ---------------------------------------------------------------------
    def rasterise(self, w: int, h: int, dtype=np.float64) -> np.ndarray:
        """Ground-truth MPI sampled at the pixel centres of a w x h grid: [D][h][w][4].
        Every value is computed in float64 (rows in chunks to bound memory) and stored in
        ``dtype``: alpha is 0 or 1, colours are the seeds' uniform draws."""
        D = self.D
        u = (np.arange(w) + 0.5) / w
        v = (np.arange(h) + 0.5) / h
        # inverse-depth field: bilinear interpolation of the control grid (its corners at the
        # image corners)
        gx = u * (GRID_COLS - 1)
        gy = v * (GRID_ROWS - 1)
        x0 = np.minimum(np.floor(gx).astype(int), GRID_COLS - 2)
        y0 = np.minimum(np.floor(gy).astype(int), GRID_ROWS - 2)
        fx = gx - x0
        fy = gy - y0
        g = self.grid
        plane_inv = 1.0 / self.depths
        aspect = self.W / self.H
        px = (u * aspect)[None, :, None]
        mpi = np.zeros((D, h, w, 4), dtype=dtype)
        zz = np.arange(D)[:, None, None]
        rows = max(1, (1 << 20) // max(w, 1))
        # planes are independent: large frames colour them on a few threads (NumPy releases
        # the interpreter lock inside its array operations)
        pool = ThreadPoolExecutor(min(8, os.cpu_count() or 1)) if w * h >= (1 << 20) else None
        for r0 in range(0, h, rows):
            r1 = min(h, r0 + rows)
            ys = slice(r0, r1)
            top = g[y0[ys]][:, x0] * (1 - fx)[None, :] + g[y0[ys]][:, x0 + 1] * fx[None, :]
            bot = g[y0[ys] + 1][:, x0] * (1 - fx)[None, :] + g[y0[ys] + 1][:, x0 + 1] * fx[None, :]
            inv_depth = top * (1 - fy[ys])[:, None] + bot * fy[ys][:, None]
            dist = np.abs(inv_depth[None] - plane_inv[:, None, None])   # [D][rows][w]
            nearest = np.argmin(dist, axis=0)                            # first index wins ties
            mpi[:, ys, :, 3] = (zz == nearest[None])
            dx2 = px[..., 0]                                             # [1][w]
            dy2 = v[ys][:, None]                                         # [rows][1]

            def colour_plane(z, ys=ys, nrows=r1 - r0, dx2=dx2, dy2=dy2):
                # nearest seed; a strict comparison keeps the lower index on ties
                best = None
                cell = np.zeros((nrows, w), dtype=np.intp)
                for j in range(N_VORONOI):
                    sx = self.seeds_xy[z, j, 0] * aspect
                    sy = self.seeds_xy[z, j, 1]
                    d2 = (dx2 - sx) ** 2 + (dy2 - sy) ** 2
                    if best is None:
                        best = d2
                    else:
                        closer = d2 < best
                        best = np.where(closer, d2, best)
                        cell[closer] = j
                mpi[z, ys, :, :3] = self.seeds_rgb[z][cell]

            if pool is None:
                for z in range(D):
                    colour_plane(z)
            else:
                list(pool.map(colour_plane, range(D)))
        if pool is not None:
            pool.shutdown()
        return mpi

    def gt_mpi(self, dtype=np.float64) -> np.ndarray:
        """Ground-truth MPI at full resolution, [D][H][W][4]."""
        return self.rasterise(self.W, self.H, dtype)

    def initial_mpi(self) -> np.ndarray:
        """Noisy ground truth at the coarsest level, [D][h0][w0][4] float64 in [0, 1]."""
        w0, h0 = self.shapes()[0]
        gt = self.rasterise(w0, h0)
        a = np.clip(gt[..., 3], ALPHA_EPS, 1.0 - ALPHA_EPS)
        logit = np.log(a) - np.log1p(-a)
        a0 = 1.0 / (1.0 + np.exp(-(logit + ALPHA_LOGIT_SIGMA * self.init_noise_a)))
        c0 = np.clip(gt[..., :3] + COLOUR_SIGMA * self.init_noise_c, 0.0, 1.0)
        out = np.empty_like(gt)
        out[..., :3] = c0
        out[..., 3] = a0
        return out

    def noisy_mpi(self, w: int, h: int, seed: int, dtype=np.float32) -> np.ndarray:
        """The ground truth rasterised at w x h with the initial MPI's noise model, drawn from
        its own generator (seed): an MPI state of the kind a refinement works on, at any
        level. Computed in ``dtype`` (float32 keeps full-frame states small)."""
        gt = self.rasterise(w, h, dtype)
        rng = np.random.default_rng(seed)
        one = dtype(1.0)
        a = np.clip(gt[..., 3], dtype(ALPHA_EPS), one - dtype(ALPHA_EPS))
        logit = np.log(a) - np.log1p(-a)
        logit += dtype(ALPHA_LOGIT_SIGMA) * rng.standard_normal(a.shape, dtype=dtype)
        gt[..., 3] = one / (one + np.exp(-logit))
        del a, logit
        for c in range(3):
            noise = rng.standard_normal(gt.shape[:3], dtype=dtype)
            gt[..., c] = np.clip(gt[..., c] + dtype(COLOUR_SIGMA) * noise, 0.0, 1.0)
        return gt


def make_scene(name: str = "c1", seed: int | None = None, **overrides) -> Scene:
    """Draw a scene. Draw order: control grid, Voronoi seeds and colours per plane,
    view translations, initial-MPI noise (alpha, then colour), then (tilted configs only)
    view rotations and z translations."""
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    if seed is not None:
        cfg["seed"] = seed
    sc = Scene(**{k: cfg[k] for k in ("W", "H", "D", "N", "f", "a", "levels", "k", "seed")},
               iters=tuple(cfg["iters"]))
    rng = np.random.default_rng(sc.seed)
    sc.depths = plane_depths(sc.D)
    sc.grid = rng.uniform(0.01, 1.0, size=(GRID_ROWS, GRID_COLS))
    sc.seeds_xy = np.empty((sc.D, N_VORONOI, 2))
    sc.seeds_rgb = np.empty((sc.D, N_VORONOI, 3))
    for z in range(sc.D):
        sc.seeds_xy[z] = rng.uniform(0.0, 1.0, size=(N_VORONOI, 2))
        sc.seeds_rgb[z] = rng.uniform(0.0, 1.0, size=(N_VORONOI, 3))
    txy = rng.uniform(-sc.a, sc.a, size=(sc.N, 2))
    sc.t = np.concatenate([txy, np.zeros((sc.N, 1))], axis=1)
    w0, h0 = sc.shapes()[0]
    sc.init_noise_a = rng.standard_normal((sc.D, h0, w0))
    sc.init_noise_c = rng.standard_normal((sc.D, h0, w0, 3))
    if cfg.get("tilt", 0.0) > 0.0:
        # drawn last, so a tilted scene shares everything else with its untilted config
        ang = rng.normal(0.0, cfg["tilt"], size=(sc.N, 3))
        sc.R = np.stack([_euler(*a) for a in ang])
        sc.t[:, 2] = rng.uniform(-cfg["tz"], cfg["tz"], size=sc.N)
    return sc


def _euler(ax: float, ay: float, az: float) -> np.ndarray:
    """Rotation Rz Ry Rx from Euler angles (radians)."""
    cx, sx, cy, sy, cz, sz = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def random_mpi(rng: np.random.Generator, D: int, H: int, W: int, lo: float = 0.0,
               hi: float = 1.0) -> np.ndarray:
    """Uniform random straight-RGBA MPI [D][H][W][4] (float64) for parity cases."""
    return rng.uniform(lo, hi, size=(D, H, W, 4))


def random_images(rng: np.random.Generator, N: int, H: int, W: int) -> np.ndarray:
    """Uniform random target images [N][H][W][3] (float64)."""
    return rng.uniform(0.0, 1.0, size=(N, H, W, 3))
