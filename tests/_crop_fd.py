"""Central finite differences of the FP64 oracle's photometric loss for single MPI scalars at
full frame size, evaluated on crops.

With translation warps a voxel (z, Y, X) is read only by the rays of a 2x2 pixel patch per
view, so the loss difference between M + h e and M - h e is confined to those pixels. Each
view's patch is rendered by the oracle from an MPI crop that holds every tap of the patch's
rays (all planes); a translation map renders a crop exactly like the full frame. Taps outside
the real frame fall outside the crop as well, so zero padding agrees.
"""

import numpy as np


def _patch_loss(O, Mc, G_i, tgt, r0, c0, rows, cols, N):
    C = O.render_view(Mc, G_i)[0]
    d = C[rows[0] - r0:rows[1] - r0 + 1, cols[0] - c0:cols[1] - c0 + 1] - tgt
    return float(np.sum(d * d) / (2.0 * N))


def fd_scalar(O, M, G, targets, idx, h=1e-3):
    """Central difference of the oracle loss w.r.t. M[idx] (idx = (z, Y, X, ch))."""
    D, H, W, _ = M.shape
    N = len(G)
    z, Y, X, ch = idx
    total = 0.0
    for i in range(N):
        sx = G[i, :, 0, 2]
        sy = G[i, :, 1, 2]
        fx, fy = int(np.floor(sx[z])), int(np.floor(sy[z]))
        # view pixels whose taps at plane z can include (X, Y), with one pixel of margin
        rows = (max(Y - fy - 2, 0), min(Y - fy + 1, H - 1))
        cols = (max(X - fx - 2, 0), min(X - fx + 1, W - 1))
        if rows[0] > rows[1] or cols[0] > cols[1]:
            continue
        # MPI crop holding every tap of those rays on every plane (the crop is also the
        # rendered view window, with the same origin)
        r0 = max(rows[0] + int(np.floor(sy.min())) - 1, 0)
        r1 = min(rows[1] + int(np.floor(sy.max())) + 2, H - 1)
        c0 = max(cols[0] + int(np.floor(sx.min())) - 1, 0)
        c1 = min(cols[1] + int(np.floor(sx.max())) + 2, W - 1)
        r0, c0 = min(r0, rows[0]), min(c0, cols[0])
        r1, c1 = max(r1, rows[1]), max(c1, cols[1])
        Mc = M[:, r0:r1 + 1, c0:c1 + 1].copy()
        tgt = targets[i, rows[0]:rows[1] + 1, cols[0]:cols[1] + 1]
        Mc[z, Y - r0, X - c0, ch] += h
        lp = _patch_loss(O, Mc, G[i], tgt, r0, c0, rows, cols, N)
        Mc[z, Y - r0, X - c0, ch] -= 2 * h
        lm = _patch_loss(O, Mc, G[i], tgt, r0, c0, rows, cols, N)
        total += (lp - lm) / (2 * h)
    return total
