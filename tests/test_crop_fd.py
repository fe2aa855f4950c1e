"""The crop-based finite differences, the mosaic gradients and the patch renders used by the
full-size checks agree with the oracle's full-frame analytic gradient (L is quadratic in any
single MPI scalar) and full-frame render, for small and for large per-plane shifts, at
frame borders and corners included."""

import numpy as np
import pytest

from oracle import hsgd_oracle as O
from tests._crop_fd import fd_scalar, grad_voxels, patch_render
from tests._problems import f32, oracle_maps, rig


@pytest.mark.parametrize("focal", [100.0, 600.0])          # shifts up to ~10 / ~60 px
def test_crop_fd_equals_full_frame_gradient(focal):
    rng = np.random.default_rng(5)
    N, D, W, H = 3, 8, 96, 72
    rg = rig(5, N, D, W, H, focal, 0.1)
    M = f32(rng.uniform(0.05, 0.95, size=(D, H, W, 4)))
    I = f32(rng.uniform(size=(N, H, W, 3)))
    G = oracle_maps(O, rg)
    _, g = O.loss_and_grad(M, G, I)
    picks = [(int(rng.integers(D)), int(rng.integers(H)), int(rng.integers(W)), int(rng.integers(4)))
             for _ in range(40)]
    picks += [(0, 0, 0, 3), (D - 1, H - 1, W - 1, 0), (3, 0, W - 1, 1)]   # frame corners
    for idx in picks:
        fd = fd_scalar(O, M, G, I, idx)
        assert abs(fd - g[idx]) <= 1e-8 * max(1.0, abs(g[idx])), (idx, fd, g[idx])


def test_patch_render_equals_full_frame_render():
    rng = np.random.default_rng(6)
    N, D, W, H = 2, 8, 96, 72
    rg = rig(6, N, D, W, H, 600.0, 0.1)
    M = f32(rng.uniform(0.05, 0.95, size=(D, H, W, 4)))
    G = oracle_maps(O, rg)
    full = O.render(M, G)
    for i in range(N):
        for rows, cols in [((0, 7), (0, 9)), ((30, 41), (50, 95)), ((64, 71), (88, 95))]:
            p = patch_render(O, M, G, i, rows, cols)
            ref = full[i, rows[0]:rows[1] + 1, cols[0]:cols[1] + 1]
            assert np.max(np.abs(p - ref)) <= 1e-12


@pytest.mark.parametrize("focal", [100.0, 600.0])          # shifts up to ~10 / ~60 px
def test_mosaic_gradient_equals_full_frame_gradient(focal):
    """Every voxel of a 6-plane frame's border rows and columns, and random interior ones,
    including voxels that some view cannot see (shifted out of its frame)."""
    rng = np.random.default_rng(7)
    N, D, W, H = 3, 6, 80, 56
    rg = rig(7, N, D, W, H, focal, 0.1)
    M = f32(rng.uniform(0.05, 0.95, size=(D, H, W, 4)))
    I = f32(rng.uniform(size=(N, H, W, 3)))
    G = oracle_maps(O, rg)
    _, g = O.loss_and_grad(M, G, I)
    vox = [(z, y, x) for z in range(D) for y in (0, H - 1) for x in range(0, W, 3)]
    vox += [(z, y, x) for z in range(D) for y in range(0, H, 3) for x in (0, W - 1)]
    vox += [(int(rng.integers(D)), int(rng.integers(H)), int(rng.integers(W))) for _ in range(100)]
    got = grad_voxels(O, M, G, I, vox)
    ref = np.array([g[z, y, x] for z, y, x in vox])
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())
    assert np.count_nonzero(ref) > 0.5 * ref.size
