"""Degenerate cases of the method on the GPU, each against the FP64 oracle: one plane and one
view on the smallest frame, a view whose planes all land outside the frame, a mask that
keeps every plane, the maximum view and plane counts, a single-level refine, a refine with
no iterations, the smallest plane-sweep volumes, and the selection fused into the level
transition against the stand-alone selection."""

import numpy as np
import pytest
import torch

from oracle import hsgd_oracle as O
from paper_2307_03017_amd import hsgd, scenes
from tests._problems import device_warps, f32, grad_close, mask_bits, oracle_maps, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda"


def to_dev(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV).to(dtype)


def shift_rig(W, H, D, f, t_xy):
    """Identity-rotation rig with the given per-view (t_x, t_y)."""
    N = len(t_xy)
    K_ref = np.array([[f, 0.0, (W - 1) / 2.0], [0.0, f, (H - 1) / 2.0], [0, 0, 1.0]])
    t = np.zeros((N, 3))
    t[:, :2] = t_xy
    return dict(K_ref=K_ref, K=np.repeat(K_ref[None], N, axis=0), R=np.repeat(np.eye(3)[None], N, axis=0),
                t=t, depths=scenes.plane_depths(D), W=W, H=H)


def test_one_plane_one_view_smallest_frame():
    rg = shift_rig(2, 2, 1, 3.0, [(0.13, -0.21)])          # fractional shift on a 2 x 2 frame
    rng = np.random.default_rng(70)
    M = f32(rng.uniform(0.05, 0.95, size=(1, 2, 2, 4)))
    I = f32(rng.uniform(size=(1, 2, 2, 3)))
    G = oracle_maps(O, rg)
    table = device_warps(hsgd, rg)
    assert table.shift_only
    out, loss = hsgd.hsgd_render(to_dev(M), table, 1, images=to_dev(I), want_loss=True)
    assert np.abs(out.cpu().numpy() - O.render(M, G)).max() <= 1e-6
    L_ref, g_ref = O.loss_and_grad(M, G, I)
    assert abs(loss.item() - L_ref) <= 1e-6 * L_ref
    g, _ = hsgd.hsgd_grad_step(to_dev(M), table, 1, images=to_dev(I), want_grad=True)
    grad_close(g.cpu().numpy(), g_ref, 1e-5, "2x2 frame")
    mask, ids, off, n = hsgd.hsgd_select_active(to_dev(M), 1)
    assert np.array_equal(mask_bits(mask.cpu().numpy(), 1), np.ones((1, 2, 2), bool))
    assert int(n.item()) == 4 and np.array_equal(ids[:4].cpu().numpy(), np.arange(4))


def test_view_with_every_plane_outside_the_frame():
    # view 1 moves by more than twice the frame on every plane: it sees only the black
    # background, its render is exactly 0, and its residual -I contributes no gradient
    W, H, D, f = 40, 24, 6, 30.0
    far = 3.0 * W * scenes.plane_depths(D).max() / f
    rg = shift_rig(W, H, D, f, [(0.05, 0.02), (far, 0.0)])
    rng = np.random.default_rng(71)
    M = f32(rng.uniform(0.05, 0.95, size=(D, H, W, 4)))
    I = f32(rng.uniform(size=(2, H, W, 3)))
    G = oracle_maps(O, rg)
    table = device_warps(hsgd, rg)
    out, loss = hsgd.hsgd_render(to_dev(M), table, 2, images=to_dev(I), want_loss=True)
    C = out.cpu().numpy()
    assert np.all(C[1] == 0.0)
    assert np.abs(C - O.render(M, G)).max() <= 1e-5
    L_ref, g_ref = O.loss_and_grad(M, G, I)
    assert abs(loss.item() - L_ref) <= 1e-5 * L_ref
    g, _ = hsgd.hsgd_grad_step(to_dev(M), table, 2, images=to_dev(I), want_grad=True)
    grad_close(g.cpu().numpy(), g_ref, 1e-4, "view outside")
    g0, _ = hsgd.hsgd_grad_step(to_dev(M), device_warps(hsgd, shift_rig(W, H, D, f, [(0.05, 0.02)])), 1,
                                images=to_dev(I[:1]), want_grad=True)
    # the dense gradient of the two-view loss is the first view's alone (halved: L is a mean over views)
    assert rel_err(g.cpu().numpy(), 0.5 * g0.cpu().numpy()) <= 1e-5


def test_mask_of_every_plane_equals_the_dense_gradient():
    W, H, D, f = 70, 30, 8, 60.0
    rg = shift_rig(W, H, D, f, [(0.04, -0.03), (-0.05, 0.01), (0.02, 0.05)])
    rng = np.random.default_rng(72)
    M = f32(rng.uniform(0.05, 0.95, size=(D, H, W, 4)))
    I = f32(rng.uniform(size=(3, H, W, 3)))
    table = device_warps(hsgd, rg)
    Md = to_dev(M)
    mask = hsgd.hsgd_select_active(Md, D, with_ids=False)
    assert np.all(mask_bits(mask.cpu().numpy(), D))
    gs, ls = hsgd.hsgd_grad_step(Md, table, 3, images=to_dev(I), mask=mask, kcap=D, want_grad=True, want_loss=True)
    gd, ld = hsgd.hsgd_grad_step(Md, table, 3, images=to_dev(I), want_grad=True, want_loss=True)
    assert rel_err(gs.cpu().numpy(), gd.cpu().numpy()) <= 1e-6
    assert abs(ls.item() - ld.item()) <= 1e-6 * ld.item()
    _, g_ref = O.loss_and_grad(M, oracle_maps(O, rg), I)
    grad_close(gs.cpu().numpy(), g_ref, 1e-4, "mask of every plane")


def test_single_level_refine_matches_oracle():
    sc = scenes.make_scene("c1")
    G = O.view_to_ref_maps(sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(), sc.depths)
    targets = O.render(sc.gt_mpi(), G)
    M0 = f32(sc.noisy_mpi(sc.W, sc.H, seed=73))
    ref, log = O.refine(M0, targets, sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(), sc.depths, (2,),
                        sc.k, 1.0, 1.0)
    out, losses = hsgd.hsgd_refine(to_dev(M0), to_dev(targets), sc.K_ref(), sc.K_views(), sc.R_views(),
                                   sc.t_views(), sc.depths, (2,), sc.k)
    np.testing.assert_allclose(losses.cpu().numpy(), [e["loss"] for e in log], rtol=1e-4)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-4


def test_smallest_plane_sweeps():
    rng = np.random.default_rng(74)
    # one view, one plane, a 3 x 2 image (a ragged tile with W % 4 != 0)
    rg = shift_rig(3, 2, 1, 4.0, [(0.3, -0.2)])
    I = f32(rng.uniform(size=(1, 2, 3, 3)))
    P = hsgd.hsgd_plane_sweep(to_dev(I), hsgd.psv_warps(rg["K_ref"], rg["K"], rg["R"], rg["t"], rg["depths"], DEV),
                              1, 1)[0]
    ref = O.plane_sweep(I, rg["K_ref"], rg["K"], rg["R"], rg["t"], rg["depths"])
    assert np.abs(P.cpu().numpy() - ref).max() <= 1e-6
    # a view that moves out of the image on every plane sweeps to zeros
    W, H, D, f = 20, 8, 3, 10.0
    far = 3.0 * W * scenes.plane_depths(D).max() / f
    rg = shift_rig(W, H, D, f, [(far, 0.0)])
    I = f32(rng.uniform(size=(1, H, W, 3)))
    P = hsgd.hsgd_plane_sweep(to_dev(I), hsgd.psv_warps(rg["K_ref"], rg["K"], rg["R"], rg["t"], rg["depths"], DEV),
                              D, 2)
    assert all(torch.count_nonzero(p).item() == 0 for p in P)


def test_maximum_views_and_planes():
    # 64 views and 64 planes (every bit of the plane mask word), k = 64 and a sparse k
    W, H, D, N, f = 16, 8, 64, 64, 10.0
    rng = np.random.default_rng(75)
    t = rng.uniform(-0.05, 0.05, size=(N, 2))
    rg = shift_rig(W, H, D, f, t)
    M = f32(rng.uniform(0.05, 0.95, size=(D, H, W, 4)))
    I = f32(rng.uniform(size=(N, H, W, 3)))
    G = oracle_maps(O, rg)
    table = device_warps(hsgd, rg)
    Md = to_dev(M)
    out, loss = hsgd.hsgd_render(Md, table, N, images=to_dev(I), want_loss=True)
    assert np.abs(out.cpu().numpy() - O.render(M, G)).max() <= 1e-5
    L_ref, g_ref = O.loss_and_grad(M, G, I)
    assert abs(loss.item() - L_ref) <= 1e-5 * L_ref
    for k in (64, 5):
        mask = hsgd.hsgd_select_active(Md, k, with_ids=False)
        S = mask_bits(mask.cpu().numpy(), D)
        assert np.array_equal(S, O.select_active(M[..., 3], k))
        g, _ = hsgd.hsgd_grad_step(Md, table, N, images=to_dev(I), mask=mask, kcap=k, want_grad=True)
        g = g.cpu().numpy()
        assert np.all(g[~S] == 0.0)
        grad_close(g[S], g_ref[S], 1e-4, f"64 views, k {k}")
    # the update with every view's slice summed (the update kernel's largest view table)
    M2 = Md.clone()
    mask = hsgd.hsgd_select_active(Md, 5, with_ids=False)
    hsgd.hsgd_grad_step(M2, table, N, images=to_dev(I), mask=mask, kcap=5, lr_rgb=0.5, lr_alpha=0.5)
    S = mask_bits(mask.cpu().numpy(), D)
    exp = O.apply_update(M, g_ref, S, 0.5, 0.5)
    assert np.abs(M2.cpu().numpy() - exp).max() <= 1e-5


def test_refine_with_no_iterations_only_upsamples():
    sc = scenes.make_scene("c1")
    M0 = f32(sc.initial_mpi())
    G = O.view_to_ref_maps(sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(), sc.depths)
    targets = O.render(sc.gt_mpi(), G)
    out, losses = hsgd.hsgd_refine(to_dev(M0), to_dev(targets), sc.K_ref(), sc.K_views(), sc.R_views(),
                                   sc.t_views(), sc.depths, (0, 0), sc.k)
    assert losses.numel() == 0
    assert np.abs(out.cpu().numpy() - O.upsample2x(M0)).max() <= 1e-6


@pytest.mark.parametrize("D, k, rule, quant, dtype, W, H", [
    (32, 4, "topk", False, torch.float32, 64, 32),
    (13, 5, "topk", True, torch.float32, 64, 32),       # exact ties in the scores
    (8, 6, "topk", True, torch.float32, 64, 32),        # k > D/2: the passes that drop the worst
    (32, 4, "mvs", True, torch.bfloat16, 64, 32),
    (64, 3, "topk", False, torch.bfloat16, 64, 32),     # every bit of the mask word
    (16, 3, "topk", True, torch.float32, 260, 42),      # three column tiles, the last ragged
    (32, 4, "topk", False, torch.bfloat16, 250, 6),     # ragged tiles, a 3-row source level
    (7, 2, "topk", False, torch.float32, 4, 4),         # a 2 x 2 source level: every column a border
    # source levels of >= 2048 workgroups of 62 columns x 1 row: the 2 x 2 kernel
    (8, 3, "topk", True, torch.float32, 2010, 260),     # ragged last column tile
    (16, 4, "mvs", False, torch.bfloat16, 2048, 256),
], ids=lambda v: str(v).replace("torch.", ""))
def test_level_transition_selects_like_select_active(D, k, rule, quant, dtype, W, H):
    """The level transition fuses the 2x upsampling with the new level's first selection. A
    two-level refine that spends its only iteration on the finer level must equal, bit for
    bit, the upsampling, hsgd_select_active on the stored level and one hsgd_grad_step on
    that mask with the same rates (quantised alphas put exact ties into the scores)."""
    _level_transition_case(D, k, rule, quant, dtype, W, H)


@pytest.mark.parametrize("W, H", [(64, 32), (2048, 256)], ids=["per_pixel", "blocks"])
def test_level_transition_with_threshold(W, H):
    """The same with the score threshold tau on, through both level-transition kernels."""
    _level_transition_case(16, 5, "topk", False, torch.float32, W, H, tau=0.02)


def _level_transition_case(D, k, rule, quant, dtype, W, H, tau=-1.0):
    N, f = 3, 40.0
    rng = np.random.default_rng(80 + D)
    rg = shift_rig(W, H, D, f, rng.uniform(-0.05, 0.05, size=(N, 2)))
    M0 = rng.uniform(0.05, 0.95, size=(D, H // 2, W // 2, 4))
    if quant:
        M0[..., 3] = rng.integers(0, 5, size=(D, H // 2, W // 2)) / 4.0
    M0d = to_dev(M0, dtype)
    I = to_dev(rng.uniform(size=(N, H, W, 3)))
    lr_rgb, lr_a = 0.7, 0.9
    print(f"level transition D={D} k={k} rule={rule} tau={tau} {dtype} {W}x{H}", flush=True)
    out, losses = hsgd.hsgd_refine(M0d, I, rg["K_ref"], rg["K"], rg["R"], rg["t"], rg["depths"], (0, 1), k,
                                   tau=tau, lr_rgb=lr_rgb, lr_alpha=lr_a, rule=rule)
    up = hsgd.hsgd_upsample2x(M0d)
    mask = hsgd.hsgd_select_active(up, k, tau=tau, rule=rule, with_ids=False)
    if tau >= 0:                                   # the threshold drops some selected planes
        S = mask_bits(mask.cpu().numpy(), D)
        assert 0 < S.sum() < k * (H * W)
    _, loss = hsgd.hsgd_grad_step(up, device_warps(hsgd, rg), N, images=I, mask=mask, kcap=k, lr_rgb=lr_rgb,
                                  lr_alpha=lr_a, want_loss=True)
    torch.cuda.synchronize()
    assert torch.equal(out, up)
    assert losses.numel() == 1 and abs(losses.item() - loss.item()) <= 1e-6 * loss.item()


def test_refine_target_pyramid_equals_chained_downsampling():
    """The refine builds the missing coarser targets with one fused launch per run of up to
    three levels. Given every level (each the 2x2 box means of the one above, from
    hsgd_downsample2x), none, or only some of them, the refine must come out the same, bit
    for bit: the fused pyramid computes what chained downsampling does."""
    sc = scenes.make_scene("c2", levels=4, iters=(1, 1, 1, 1))
    rng = np.random.default_rng(91)
    targets = to_dev(rng.uniform(size=(sc.N, sc.H, sc.W, 3)))
    chain = [targets]
    for _ in range(3):
        chain.insert(0, hsgd.hsgd_downsample2x(chain[0]))
    init = to_dev(sc.initial_mpi())
    plan = hsgd.RefinePlan(sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(), sc.depths, sc.W, sc.H,
                           sc.iters, sc.k)
    results = []
    for given in ([None, None, None], chain[:3], [None, chain[1], None], [chain[0], None, None]):
        plan.levels[0].copy_(init)
        plan.run(targets, descriptors=plan.descriptors(targets, given))
        torch.cuda.synchronize()
        results.append((plan.levels[-1].clone(), plan.loss_log[:4].clone()))
    for out, losses in results[1:]:
        assert torch.equal(out, results[0][0])
        assert torch.equal(losses, results[0][1])
