"""The crop-based finite differences used by the full-size gradient checks agree with the
oracle's full-frame analytic gradient (L is quadratic in any single MPI scalar)."""

import numpy as np

from oracle import hsgd_oracle as O
from tests._crop_fd import fd_scalar
from tests._problems import f32, oracle_maps, rig


def test_crop_fd_equals_full_frame_gradient():
    rng = np.random.default_rng(5)
    N, D, W, H = 3, 8, 96, 72
    rg = rig(5, N, D, W, H, 100.0, 0.1)            # shifts up to 10 px
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
