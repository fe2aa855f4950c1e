"""Shared builders for parity cases: seeded camera rigs, FP32-rounded inputs, mask decoding.

Inputs are drawn in FP64, rounded once to FP32 for the device, and the oracle receives the
same FP32 values widened back to FP64, so both sides start from identical numbers.
"""

import numpy as np

from paper_2307_03017_amd import scenes


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def rot(ax, ay, az):
    cx, sx, cy, sy, cz, sz = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def rig(seed, N, D, W, H, f, a, general=False):
    """A camera rig: identity reference, N views. Pure translations in x/y unless general
    (then small rotations and a z translation as well)."""
    rng = np.random.default_rng(seed)
    K_ref = np.array([[f, 0.0, (W - 1) / 2.0], [0.0, f, (H - 1) / 2.0], [0, 0, 1.0]])
    K = np.repeat(K_ref[None], N, axis=0)
    t = np.zeros((N, 3))
    t[:, :2] = rng.uniform(-a, a, size=(N, 2))
    if general:
        R = np.stack([rot(*(rng.normal(size=3) * 0.02)) for _ in range(N)])
        t[:, 2] = rng.uniform(-0.05, 0.05, size=N)
    else:
        R = np.repeat(np.eye(3)[None], N, axis=0)
    return dict(K_ref=K_ref, K=K, R=R, t=t, depths=scenes.plane_depths(D), W=W, H=H)


def oracle_maps(O, rg, Wl=None, Hl=None):
    W, H = rg["W"], rg["H"]
    Wl = W if Wl is None else Wl
    Hl = H if Hl is None else Hl
    Kr = O.level_intrinsics(rg["K_ref"], W, H, Wl, Hl)
    K = np.stack([O.level_intrinsics(k, W, H, Wl, Hl) for k in rg["K"]])
    return O.view_to_ref_maps(Kr, K, rg["R"], rg["t"], rg["depths"])


def device_warps(hsgd, rg, Wl=None, Hl=None, device="cuda"):
    W, H = rg["W"], rg["H"]
    Wl = W if Wl is None else Wl
    Hl = H if Hl is None else Hl
    return hsgd.level_warps(rg["K_ref"], rg["K"], rg["R"], rg["t"], rg["depths"], W, H, Wl, Hl, device)


def mask_bits(mask_i64, D):
    """int64 [H][W] plane bitmask -> bool [D][H][W]."""
    m = np.asarray(mask_i64).view(np.uint64)
    z = np.arange(D, dtype=np.uint64)[:, None, None]
    return ((m[None] >> z) & np.uint64(1)).astype(bool)


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def grad_close(g, g_ref, rtol, what=""):
    """The gradient parity bound at relative tolerance rtol: over the compared set
    ||g - g_ref|| / ||g_ref|| <= rtol, and for every element
    |g - g_ref| <= rtol |g_ref| + 0.01 rtol max|g_ref| (rtol 1e-4: 1e-4 |g_ref| + 1e-6 max|g_ref|).
    The elementwise form catches an error confined to a few cells (a tile seam, a frame
    border) that the global norm would dilute. Returns (norm ratio, worst elementwise ratio)
    and prints both."""
    a = np.asarray(g, np.float64).ravel()
    b = np.asarray(g_ref, np.float64).ravel()
    assert a.shape == b.shape, (a.shape, b.shape)
    rel = rel_err(a, b)
    bound = rtol * np.abs(b) + 0.01 * rtol * (np.abs(b).max() if b.size else 0.0)
    d = np.abs(a - b)
    worst = float((d / np.where(bound > 0, bound, 1.0)).max()) if b.size else 0.0
    print(f"{what} gradient: norm ratio {rel:.2e} (tol {rtol:.0e}), worst elementwise {worst:.3f} of the bound",
          flush=True)
    assert rel <= rtol, (what, rel)
    if not np.all(d <= bound):
        i = int(np.argmax(d - bound))
        raise AssertionError(f"{what}: element {i} differs by {d[i]:.3e} > bound {bound[i]:.3e} "
                             f"(g {a[i]:.6e}, ref {b[i]:.6e}); {int(np.sum(d > bound))} of {d.size} beyond")
    return rel, worst
