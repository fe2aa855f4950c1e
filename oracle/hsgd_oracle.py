"""FP64 CPU oracle for Hierarchical Sparse Gradient Descent (HSGD) on a multi-plane image.

TEST INFRASTRUCTURE ONLY. This is the plain, slow, obviously-correct reference that the
HIP path is checked against. Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path never does, and this module shares
no code with the product (it imports nothing from it).

Everything follows the paper (RealLiFe, arXiv 2307.03017) in its own order and notation:

* MPI (Sec. 3.1): D fronto-parallel straight-RGBA planes, stored [D][H][W][4] with
  plane z = 0 the nearest. The paper counts d = 1..D with d = D the front plane, so
  z = D - d.
* Rendering (Eq. render / Eq. over): warp every plane into the view, then composite.
  Front to back with transmittance T_z = prod_{j<z}(1 - a_j) this is the over operator
  sum_d c_d a_d prod_{i>d}(1 - a_i).
* Plane homography (Eq. homo): H_i^{-1}(d) maps a reference pixel on the plane at depth
  d to source view i; rendering view i gathers with its inverse.
* Compositing weight / "alpha gradient" (Eq. gradient, Eq. overA):
  A_z = a_z * T_z = dO/dc_z, the selection score on the reference view.
* Sparsification (Sec. 3.3, Gradient Sparsification): per pixel keep the k planes with
  the largest A along depth, in their original order.
* Update (Eq. 4 with phi = 0, Eq. for M_{n+1}): analytic descent restricted to the kept
  voxels, M <- clip(M - lambda * dL/dM, 0, 1) on S, unchanged elsewhere.
* Hierarchy (Sec. 3.2 / 3.3): levels at H/2^l x W/2^l, coarse to fine, the MPI upsampled
  between levels.
* Plane-sweep volume (Sec. 3.2, Hierarchical PSV Construction): every source image
  sampled on every reference plane through H_i^{-1}(d), then box-downsampled level by level.

Readings where the paper is silent (each listed in the design notes):
  bilinear sampling in pixel-index coordinates with zero padding, colour and alpha
  interpolated separately, black background; world-to-camera poses, plane normal
  (0, 0, 1); photometric loss L = 1/(2N) sum (C - I)^2 in place of the trained VGG loss;
  descent sign M - lambda*grad; equal scores go to the nearer plane; the selection score
  is evaluated in IEEE float32 with the exact operation order below (so indices can be
  compared bit for bit); 2x upsampling is bilinear with half-pixel centres and edge clamp;
  the image pyramid is a 2x2 box mean; a sample whose homogeneous coordinate is <= 0 is
  transparent.

Parity pins for every function live in tests/test_oracle_*.py.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "plane_homography", "view_to_ref_maps", "level_intrinsics", "sample_bilinear",
    "render_view", "render", "photometric_loss", "loss_and_grad", "render_vjp",
    "select_scores_f32", "select_active", "select_ids", "apply_update", "bf16_round",
    "upsample2x", "downsample2x", "target_pyramid", "psnr", "refine",
    "plane_sweep", "psv_pyramid",
]


# --------------------------------------------------------------------------------------
# Geometry: Sec. 3.2, Eq. (homo)
# --------------------------------------------------------------------------------------
def plane_homography(K_r, K_i, R_i, t_i, d, R_r=None, t_r=None, n=(0.0, 0.0, 1.0)):
    """H_i^{-1}(d) of Eq. (homo): reference pixel (u, v, 1) on the plane n^T X = d of the
    reference camera frame -> homogeneous pixel of source view i.

    H_i^{-1}(d) = K_i R_i (I + (R_i^{-1} t_i - R_r^{-1} t_r) n^T R_r / d) R_r^{-1} K_r^{-1}
    """
    R_r = np.eye(3) if R_r is None else np.asarray(R_r, float)
    t_r = np.zeros(3) if t_r is None else np.asarray(t_r, float)
    K_r = np.asarray(K_r, float)
    K_i = np.asarray(K_i, float)
    R_i = np.asarray(R_i, float)
    t_i = np.asarray(t_i, float)
    n = np.asarray(n, float)
    inner = np.eye(3) + np.outer(np.linalg.inv(R_i) @ t_i - np.linalg.inv(R_r) @ t_r, n) @ R_r / d
    return K_i @ R_i @ inner @ np.linalg.inv(R_r) @ np.linalg.inv(K_r)


def view_to_ref_maps(K_r, K, R, t, depths):
    """G[i][z]: pixel of view i -> reference pixel on plane z (inverse of Eq. homo)."""
    N, D = len(K), len(depths)
    G = np.empty((N, D, 3, 3))
    for i in range(N):
        for z in range(D):
            G[i, z] = np.linalg.inv(plane_homography(K_r, K[i], R[i], t[i], depths[z]))
    return G


def level_intrinsics(K, W, H, Wl, Hl):
    """Intrinsics of a W x H camera resampled to Wl x Hl (pixel-index coordinates: the
    centre of pixel x sits at x, so a principal point c maps to (c + 0.5) * s - 0.5)."""
    K = np.asarray(K, float)
    sx, sy = Wl / W, Hl / H
    out = K.copy()
    out[0, 0] = K[0, 0] * sx
    out[0, 1] = K[0, 1] * sx
    out[1, 1] = K[1, 1] * sy
    out[0, 2] = (K[0, 2] + 0.5) * sx - 0.5
    out[1, 2] = (K[1, 2] + 0.5) * sy - 0.5
    return out


# --------------------------------------------------------------------------------------
# Warp: grid_sample of an MPI plane (Sec. 3.2, Eq. for I^{w^-1}; warp omega_t of Eq. render)
# --------------------------------------------------------------------------------------
def _warp_points(G, H, W):
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    q0 = G[0, 0] * xs + G[0, 1] * ys + G[0, 2]
    q1 = G[1, 0] * xs + G[1, 1] * ys + G[1, 2]
    q2 = G[2, 0] * xs + G[2, 1] * ys + G[2, 2]
    front = q2 > 0
    safe = np.where(front, q2, 1.0)
    return q0 / safe, q1 / safe, front


def _bilinear_taps(u, v, front, H, W):
    """The 4 bilinear taps of positions (u, v): list of (flat index, weight); weights of
    taps outside the plane (zero padding) or of samples behind the camera are 0."""
    x0 = np.floor(u)
    y0 = np.floor(v)
    fx = u - x0
    fy = v - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    taps = []
    for dx, dy, w in ((0, 0, (1 - fx) * (1 - fy)), (1, 0, fx * (1 - fy)),
                      (0, 1, (1 - fx) * fy), (1, 1, fx * fy)):
        xx = x0 + dx
        yy = y0 + dy
        ok = (xx >= 0) & (xx < W) & (yy >= 0) & (yy < H) & front
        flat = np.clip(yy, 0, H - 1) * W + np.clip(xx, 0, W - 1)
        taps.append((flat, np.where(ok, w, 0.0)))
    return taps


def sample_bilinear(plane, G):
    """Sample one plane [H][W][C] at q = G (x, y, 1) for every pixel of an H x W view."""
    H, W, C = plane.shape
    u, v, front = _warp_points(G, H, W)
    flatp = plane.reshape(H * W, C)
    out = np.zeros((H, W, C))
    for flat, w in _bilinear_taps(u, v, front, H, W):
        out += flatp[flat] * w[..., None]
    return out


def sample_bilinear_T(grad_samples, G, H, W):
    """Exact transpose of sample_bilinear: scatter per-pixel values [H][W][C] back onto
    the plane's taps with the same weights."""
    C = grad_samples.shape[-1]
    u, v, front = _warp_points(G, H, W)
    out = np.zeros((H * W, C))
    for flat, w in _bilinear_taps(u, v, front, H, W):
        for ch in range(C):
            out[:, ch] += np.bincount(flat.ravel(), weights=(w * grad_samples[..., ch]).ravel(),
                                      minlength=H * W)
    return out.reshape(H, W, C)


# --------------------------------------------------------------------------------------
# Rendering: Eq. (render), Eq. (over)
# --------------------------------------------------------------------------------------
def render_view(M, G_i):
    """Render one view: C = sum_z c~_z a~_z T_z with T_z = prod_{j<z} (1 - a~_j).

    Returns the image [H][W][3], the warped samples [D][H][W][4] and T [D][H][W]."""
    D, H, W, _ = M.shape
    T = np.ones((H, W))
    C = np.zeros((H, W, 3))
    samples = np.empty((D, H, W, 4))
    Ts = np.empty((D, H, W))
    for z in range(D):
        s = sample_bilinear(M[z], G_i[z])
        samples[z] = s
        Ts[z] = T
        C += (T * s[..., 3])[..., None] * s[..., :3]
        T = T * (1.0 - s[..., 3])
    return C, samples, Ts


def render(M, G):
    """Render every view: [N][H][W][3]."""
    return np.stack([render_view(M, G[i])[0] for i in range(len(G))])


def photometric_loss(C, targets):
    """L = 1/(2N) sum_i sum_p sum_ch (C - I)^2 (stands in for the trained VGG loss)."""
    N = len(targets)
    return float(np.sum((C - targets) ** 2) / (2.0 * N))


def psnr(C, targets):
    mse = float(np.mean((C - targets) ** 2))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(1.0 / mse)


def _view_adjoint(M_shape, G_i, samples, Ts, g):
    """Adjoint of render_view at upstream gradient g = dL/dC [H][W][3] -> dL/dM.

    Colour: dL/dc~_z = g a~_z T_z (the weight of Eq. gradient). Alpha:
    dL/da~_z = T_z <g, c~_z - B_z>, with B_z the composite of the planes behind z, built by
    the back-to-front recursion B <- a~_z c~_z + (1 - a~_z) B. Then the transpose of the
    bilinear warp carries both to the MPI voxels."""
    D, H, W, _ = M_shape
    grad = np.zeros(M_shape)
    B = np.zeros((H, W, 3))
    for z in range(D - 1, -1, -1):
        c = samples[z][..., :3]
        a = samples[z][..., 3]
        T = Ts[z]
        gs = np.empty((H, W, 4))
        gs[..., :3] = g * (a * T)[..., None]
        gs[..., 3] = T * np.sum(g * (c - B), axis=-1)
        B = a[..., None] * c + (1.0 - a)[..., None] * B
        grad[z] += sample_bilinear_T(gs, G_i[z], H, W)
    return grad


def loss_and_grad(M, G, targets):
    """Photometric loss and its exact dense gradient dL/dM [D][H][W][4]."""
    N = len(G)
    grad = np.zeros(M.shape)
    loss = 0.0
    for i in range(N):
        C, samples, Ts = render_view(M, G[i])
        r = (C - targets[i]) / N                          # dL/dC_i
        loss += float(np.sum((C - targets[i]) ** 2) / (2.0 * N))
        grad += _view_adjoint(M.shape, G[i], samples, Ts, r)
    return loss, grad


def render_vjp(M, G, g_img):
    """Vector-Jacobian product of render(): sum_i J_i^T g_img[i], dense [D][H][W][4]."""
    grad = np.zeros(M.shape)
    for i in range(len(G)):
        _, samples, Ts = render_view(M, G[i])
        grad += _view_adjoint(M.shape, G[i], samples, Ts, g_img[i])
    return grad


# --------------------------------------------------------------------------------------
# Gradient sparsification: Sec. 3.3, Eq. (gradient), Eq. (overA)
# --------------------------------------------------------------------------------------
def select_scores_f32(alpha):
    """A_z = a_z T_z on the un-warped reference MPI, in IEEE float32 with the operation
    order A_z = fl(a_z * T_z), T_{z+1} = fl(T_z * fl(1 - a_z)), T_0 = 1."""
    a = np.asarray(alpha, dtype=np.float32)
    one = np.float32(1.0)
    T = np.ones(a.shape[1:], dtype=np.float32)
    A = np.empty_like(a)
    for z in range(a.shape[0]):
        A[z] = a[z] * T
        T = T * (one - a[z])
    return A


def select_active(alpha, k, tau=-1.0, rule="topk"):
    """Per pixel, the planes kept by the sparsification rule (Sec. 3.3), as a bool mask
    [D][H][W]. "topk" (the paper's rule): the k planes with the largest A (equal A: the
    nearer plane first). "mvs" (the MVS-sampling alternative the paper ablates): the plane
    with the largest A (equal A: the nearer) and its neighbours, floor((k-1)/2) nearer
    planes and the rest farther, the window moved inside [0, D). With tau >= 0, kept planes
    whose A <= tau are dropped too."""
    A = select_scores_f32(alpha)
    D = A.shape[0]
    k = min(int(k), D)
    mask = np.zeros(A.shape, dtype=bool)
    if rule == "topk":
        order = np.argsort(-A, axis=0, kind="stable")       # ties keep ascending z
        np.put_along_axis(mask, order[:k], True, axis=0)
    elif rule == "mvs":
        best = np.argmax(A, axis=0)                         # first (nearest) maximum
        lo = np.clip(best - (k - 1) // 2, 0, D - k)
        z = np.arange(D)[:, None, None]
        mask = (z >= lo[None]) & (z < lo[None] + k)
    else:
        raise ValueError(rule)
    if tau >= 0:
        mask &= A > np.float32(tau)
    return mask


def select_ids(mask):
    """Sparse indices S in original spatial order: ascending linear ids z*H*W + y*W + x,
    with per-plane offsets [D+1]."""
    D = mask.shape[0]
    ids = np.flatnonzero(mask.reshape(-1)).astype(np.int64)
    counts = mask.reshape(D, -1).sum(axis=1)
    plane_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return ids, plane_off


# --------------------------------------------------------------------------------------
# Sparse update: Eq. 4 (phi = 0, descent) restored onto S as in the M_{n+1} update
# --------------------------------------------------------------------------------------
def bf16_round(x):
    """Round float values to bfloat16 (round to nearest, ties to even) and back."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def sparsity_loss(alpha):
    """L_s of Sec. 3.4: the mean over the level's voxels of log(1.5 - |0.5 - alpha|)."""
    a = np.asarray(alpha, float)
    return float(np.mean(np.log(1.5 - np.abs(0.5 - a))))


def sparsity_grad(alpha):
    """dL_s/dalpha per voxel: sign(0.5 - alpha) / (1.5 - |0.5 - alpha|) / (D H W), taking the
    subgradient 0 at alpha = 0.5 (descent moves alpha towards 0 below 0.5, towards 1 above)."""
    a = np.asarray(alpha, float)
    d = 0.5 - a
    return np.sign(d) / (1.5 - np.abs(d)) / a.size


def apply_update(M, grad, mask, lr_rgb, lr_alpha, bf16=False):
    """M <- clip(M - lambda * grad, 0, 1) on the active voxels, unchanged elsewhere."""
    lam = np.array([lr_rgb, lr_rgb, lr_rgb, lr_alpha])
    new = np.clip(M - lam * grad, 0.0, 1.0)
    if bf16:
        new = bf16_round(new)
    return np.where(mask[..., None], new, M)


# --------------------------------------------------------------------------------------
# Hierarchy: Sec. 3.2 (H/2^l pyramid), Sec. 3.3 (refine the upsampled MPI)
# --------------------------------------------------------------------------------------
def _upsample_axis(n_in):
    s = (np.arange(2 * n_in) + 0.5) / 2.0 - 0.5
    s = np.clip(s, 0.0, n_in - 1.0)
    i0 = np.floor(s).astype(np.int64)
    i1 = np.minimum(i0 + 1, n_in - 1)
    return i0, i1, s - i0


def upsample2x(M, bf16=False):
    """2x bilinear upsampling of every plane: source coordinate (x + 0.5)/2 - 0.5, clamped
    to the edge; colour and alpha interpolated independently."""
    D, h, w, C = M.shape
    y0, y1, fy = _upsample_axis(h)
    x0, x1, fx = _upsample_axis(w)
    fy = fy[:, None, None]
    fx = fx[None, :, None]
    out = np.empty((D, 2 * h, 2 * w, C))
    for z in range(D):
        P = M[z]
        out[z] = ((1 - fy) * (1 - fx) * P[y0][:, x0] + (1 - fy) * fx * P[y0][:, x1]
                  + fy * (1 - fx) * P[y1][:, x0] + fy * fx * P[y1][:, x1])
    return bf16_round(out) if bf16 else out


def downsample2x(img):
    """2x2 box mean of images [..., H, W, C]."""
    *lead, H, W, C = img.shape
    r = img.reshape(*lead, H // 2, 2, W // 2, 2, C)
    return r.mean(axis=(-4, -2))


def target_pyramid(targets, levels):
    """Targets at every level, coarsest first."""
    pyr = [np.asarray(targets, float)]
    for _ in range(levels - 1):
        pyr.append(downsample2x(pyr[-1]))
    return pyr[::-1]


# --------------------------------------------------------------------------------------
# Plane-sweep volume: Sec. 3.2 (Hierarchical PSV Construction)
# --------------------------------------------------------------------------------------
def plane_sweep(images, K_r, K, R, t, depths):
    """P[i][z] = I_i^{w^-1}(., ., d_z): source image i grid-sampled at the reference meshgrid
    carried by H_i^{-1}(d_z) of Eq. (homo), for every view i and plane z. images [N][H][W][3];
    the reference grid has the images' size. Returns [N][D][H][W][3] (the paper's
    N x D x H x W x 3)."""
    images = np.asarray(images, float)
    N, H, W, _ = images.shape
    P = np.empty((N, len(depths), H, W, 3))
    for i in range(N):
        for z, d in enumerate(depths):
            P[i, z] = sample_bilinear(images[i], plane_homography(K_r, K[i], R[i], t[i], d))
    return P


def psv_pyramid(P, levels):
    """The hierarchy of plane-sweep volumes: level 0 is P itself, level l the 2x2 box mean of
    level l - 1 over the spatial axes (H/2^l x W/2^l), finest first."""
    pyr = [np.asarray(P, float)]
    for _ in range(levels - 1):
        pyr.append(downsample2x(pyr[-1]))
    return pyr


def refine(M0, targets, K_r, K, R, t, depths, iters, k, lr_rgb, lr_alpha, tau=-1.0,
           bf16=False, rule="topk", lambda_s=0.0):
    """Coarse-to-fine HSGD with analytic descent. M0 is the initial MPI at the coarsest
    level, targets the full-resolution views. Per level: upsample (l > 0), then iters[l]
    times: select S on the current MPI, loss and dense gradient, sparse update on S.

    Returns the final MPI and a list of per-iteration dicts (level, loss, psnr, active)."""
    L = len(iters)
    N, H, W, _ = np.shape(targets)
    pyr = target_pyramid(targets, L)
    M = bf16_round(M0) if bf16 else np.asarray(M0, float).copy()
    log = []
    for l in range(L):
        if l > 0:
            M = upsample2x(M, bf16=bf16)
        Hl, Wl = pyr[l].shape[1:3]
        if M.shape[1:3] != (Hl, Wl):
            raise ValueError("initial MPI does not match the coarsest level")
        Kr_l = level_intrinsics(K_r, W, H, Wl, Hl)
        K_l = np.stack([level_intrinsics(K[i], W, H, Wl, Hl) for i in range(N)])
        G = view_to_ref_maps(Kr_l, K_l, R, t, depths)
        for _ in range(iters[l]):
            mask = select_active(M[..., 3], k, tau, rule)
            loss, grad = loss_and_grad(M, G, pyr[l])
            if lambda_s:
                grad[..., 3] += lambda_s * sparsity_grad(M[..., 3])     # the prior phi of Eq. 4
            mse = 2.0 * loss / (3.0 * Hl * Wl)          # sum of squares = 2 N L
            log.append(dict(level=l, loss=loss, active=int(mask.sum()),
                            psnr=float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)))
            M = apply_update(M, grad, mask, lr_rgb, lr_alpha, bf16=bf16)
    return M, log
