"""Exact evaluations of the FP64 oracle's photometric loss for one MPI scalar at full frame
size, on per-plane crops.

With translation warps a voxel (z, Y, X) is read only by the rays of a 2x2 pixel patch per
view, so the loss difference between M + h e and M - h e is confined to those pixels. Each
view's patch (with a one-pixel margin) is rendered by the oracle from a small MPI whose plane
z' is the patch's tap window on plane z' of the full MPI (zero outside the frame, matching
zero padding); every plane gets its own translation so that the crop renders exactly like
the full frame. A crop render is therefore only patch-sized, whatever the shifts.
"""

import numpy as np

MARGIN = 2          # view pixels around the 2x2 patch
PAD = 2             # MPI pixels around each plane's tap window


def _crop_problem(M, Gi, rows, cols):
    D, H, W, _ = M.shape
    h = rows[1] - rows[0] + 1
    w = cols[1] - cols[0] + 1
    ch_, cw_ = h + 2 * PAD, w + 2 * PAD
    Mc = np.zeros((D, ch_, cw_, 4))
    Gc = np.zeros((D, 3, 3))
    origins = []
    for z in range(D):
        sx, sy = Gi[z, 0, 2], Gi[z, 1, 2]
        ox = cols[0] + int(np.floor(sx)) - PAD
        oy = rows[0] + int(np.floor(sy)) - PAD
        ys, xs = slice(max(oy, 0), min(oy + ch_, H)), slice(max(ox, 0), min(ox + cw_, W))
        if ys.start < ys.stop and xs.start < xs.stop:
            Mc[z, ys.start - oy:ys.stop - oy, xs.start - ox:xs.stop - ox] = M[z, ys, xs]
        # crop-view pixel (a, b) = view pixel (cols[0] + a, rows[0] + b); its tap in the
        # plane crop sits at (cols[0] + a + sx - ox, ...)
        Gc[z] = np.eye(3)
        Gc[z, 0, 2] = (cols[0] - ox) + sx
        Gc[z, 1, 2] = (rows[0] - oy) + sy
        origins.append((oy, ox))
    return Mc, Gc, origins


def _patch_loss(O, Mc, Gc, tgt, h, w, N):
    C = O.render_view(Mc, Gc)[0][:h, :w]
    d = C - tgt
    return float(np.sum(d * d) / (2.0 * N))


def fd_scalar(O, M, G, targets, idx, h=1e-3):
    """Central difference of the oracle loss w.r.t. M[idx] (idx = (z, Y, X, ch)); G holds
    the oracle's view-to-reference maps, which must be pure translations."""
    D, H, W, _ = M.shape
    N = len(G)
    z, Y, X, ch = idx
    total = 0.0
    for i in range(N):
        fx, fy = int(np.floor(G[i, z, 0, 2])), int(np.floor(G[i, z, 1, 2]))
        rows = (max(Y - fy - MARGIN, 0), min(Y - fy + MARGIN - 1, H - 1))
        cols = (max(X - fx - MARGIN, 0), min(X - fx + MARGIN - 1, W - 1))
        if rows[0] > rows[1] or cols[0] > cols[1]:
            continue
        hh, ww = rows[1] - rows[0] + 1, cols[1] - cols[0] + 1
        Mc, Gc, origins = _crop_problem(M, G[i], rows, cols)
        oy, ox = origins[z]
        cy, cx = Y - oy, X - ox
        if not (0 <= cy < Mc.shape[1] and 0 <= cx < Mc.shape[2]):
            continue
        tgt = targets[i, rows[0]:rows[1] + 1, cols[0]:cols[1] + 1]
        Mc[z, cy, cx, ch] += h
        lp = _patch_loss(O, Mc, Gc, tgt, hh, ww, N)
        Mc[z, cy, cx, ch] -= 2 * h
        lm = _patch_loss(O, Mc, Gc, tgt, hh, ww, N)
        total += (lp - lm) / (2 * h)
    return total


def patch_render(O, M, G, i, rows, cols):
    """Oracle render of view i's pixels rows x cols (inclusive ranges) of the full frame."""
    Mc, Gc, _ = _crop_problem(M, G[i], rows, cols)
    return O.render_view(Mc, Gc)[0][:rows[1] - rows[0] + 1, :cols[1] - cols[0] + 1]


def grad_voxels(O, M, G, targets, vox):
    """The oracle's dL/dM (all 4 channels) at the voxels vox = [(z, Y, X), ...] of a full
    frame with translation maps, as an array [len(vox)][4].

    For view i, voxel (z, Y, X) is read only by the view rays of the 2x2 patch whose taps on
    plane z cover it. Every voxel gets a slot in one mosaic MPI: the 4x4 view pixels around
    its patch and, on every plane, their tap window (zero outside the frame). All crops of
    view i share one map per plane (same fractional shift, the integer part absorbed into
    the crop origin), so the oracle renders the mosaic once and back-propagates the
    photometric residual (C - I) / N of the slots' in-frame pixels with its own render_vjp
    (the residual is 0 on every other mosaic pixel). A voxel's value is the mosaic gradient
    at its slot position, summed over the views."""
    M = np.asarray(M)
    D, H, W, _ = M.shape
    N = len(G)
    hw = 2 * MARGIN                  # patch side (view pixels)
    cs = hw + 2 * PAD                # crop side (MPI pixels); crop pixel (MARGIN + PAD)^2 is the voxel
    slot = cs                        # slots side by side (their other rays carry no residual)
    n = len(vox)
    out = np.zeros((n, 4))
    for i in range(N):
        sx, sy = G[i, :, 0, 2], G[i, :, 1, 2]
        ix, iy = np.floor(sx).astype(int), np.floor(sy).astype(int)
        Gc = np.repeat(np.eye(3)[None], D, axis=0)
        Gc[:, 0, 2] = sx - ix + PAD
        Gc[:, 1, 2] = sy - iy + PAD
        zv = np.array([v[0] for v in vox])
        Yv = np.array([v[1] for v in vox])
        Xv = np.array([v[2] for v in vox])
        r0, c0 = Yv - iy[zv] - MARGIN, Xv - ix[zv] - MARGIN     # patch origins (view pixels)
        Mc = np.zeros((D, cs, n, slot, 4))
        j = np.arange(cs)
        for z in range(D):
            ry = (r0 + iy[z] - PAD)[:, None] + j[None]          # [n][cs] plane rows of the crops
            rx = (c0 + ix[z] - PAD)[:, None] + j[None]
            ok = ((ry >= 0) & (ry < H))[:, :, None] & ((rx >= 0) & (rx < W))[:, None, :]
            blk = M[z][np.clip(ry, 0, H - 1)[:, :, None], np.clip(rx, 0, W - 1)[:, None, :]]
            Mc[z, :, :, :cs] = np.where(ok[..., None], blk, 0.0).transpose(1, 0, 2, 3)
        Mc = Mc.reshape(D, cs, n * slot, 4)
        T = np.zeros((cs, n, slot, 3))
        valid = np.zeros((cs, n, slot), bool)
        j = np.arange(hw)
        py = r0[:, None] + j[None]                               # [n][hw] view rows / columns
        px = c0[:, None] + j[None]
        inside = ((py >= 0) & (py < H))[:, :, None] & ((px >= 0) & (px < W))[:, None, :]
        tv = targets[i][np.clip(py, 0, H - 1)[:, :, None], np.clip(px, 0, W - 1)[:, None, :]]
        valid[:hw, :, :hw] = inside.transpose(1, 0, 2)
        T[:hw, :, :hw] = np.where(inside[..., None], tv, 0.0).transpose(1, 0, 2, 3)
        T = T.reshape(cs, n * slot, 3)
        valid = valid.reshape(cs, n * slot)
        C = O.render(Mc, Gc[None])[0]
        r = np.where(valid[..., None], (C - T) / N, 0.0)
        g = O.render_vjp(Mc, Gc[None], r[None])
        for k, (z0, Y, X) in enumerate(vox):
            out[k] += g[z0, MARGIN + PAD, k * slot + MARGIN + PAD]
    return out
