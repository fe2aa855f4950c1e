// extern "C" entry points of libhsgd: validate every argument, then enqueue the kernels
// on the caller's stream. Nothing is enqueued when validation fails.
#include <hip/hip_runtime_api.h>

#include <cmath>

#include "hsgd_internal.h"

using namespace hsgd;

namespace hsgd {
hsgd_status hip_status(int err, const char* what) {
    if (err == hipSuccess) return HSGD_OK;
    return fail(HSGD_E_HIP, "%s: %s", what, hipGetErrorString((hipError_t)err));
}
}  // namespace hsgd

extern "C" {

hsgd_status hsgd_select_active(const hsgd_mpi* m, hsgd_select_params p, uint64_t* mask,
                               int32_t* ids, int32_t cap, int32_t* plane_off,
                               int32_t* n_active, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
    clear_error();
    const char* fn = "hsgd_select_active";
    hsgd_status st = check_mpi(m, fn);
    if (st) return st;
    if (!mask) return fail(HSGD_E_ARG, "%s: mask is NULL", fn);
    if (p.k < 1 || p.k > m->D) return fail(HSGD_E_ARG, "%s: k=%d outside [1, D=%d]", fn, p.k, m->D);
    if (std::isnan(p.tau)) return fail(HSGD_E_ARG, "%s: tau is NaN", fn);
    if (p.rule != HSGD_SELECT_TOPK && p.rule != HSGD_SELECT_MVS)
        return fail(HSGD_E_ARG, "%s: unknown selection rule %d", fn, p.rule);
    const bool any = ids || plane_off || n_active;
    if (any && !(ids && plane_off && n_active))
        return fail(HSGD_E_ARG, "%s: ids, plane_off and n_active must all be given or all NULL", fn);
    if (ids && (int64_t)cap < (int64_t)p.k * m->H * m->W)
        return fail(HSGD_E_CAPACITY, "%s: cap=%d < k*H*W=%lld", fn, cap,
                    (long long)p.k * m->H * m->W);
    if (!ids) return hip_status(launch_select(*m, p.k, p.tau, p.rule, mask, nullptr, nullptr, stream), fn);
    const ActiveLayout L = active_ws(m->D, m->H, m->W, cap, false);
    st = check_ws(ws, ws_bytes, L.bytes);
    if (st) return st;
    const ActiveSet as = active_at(ws, L, ids, n_active);
    return hip_status(launch_select(*m, p.k, p.tau, p.rule, mask, &as, plane_off, stream), fn);
}

hsgd_status hsgd_render(const hsgd_mpi* m, const hsgd_views* v, float* out_rgb,
                        float* out_loss, void* ws, size_t ws_bytes, hipStream_t stream) {
    clear_error();
    const char* fn = "hsgd_render";
    hsgd_status st = check_mpi(m, fn);
    if (st) return st;
    st = check_views(v, m, out_loss != nullptr, fn);
    if (st) return st;
    if (!out_rgb && !out_loss) return fail(HSGD_E_ARG, "%s: no output requested", fn);
    if (out_loss) {
        st = check_ws(ws, ws_bytes, render_ws(m->H, m->W, v->N).bytes);
        if (st) return st;
    }
    return hip_status(launch_render(*m, *v, out_rgb, out_loss, ws, stream), fn);
}

hsgd_status hsgd_grad_step(hsgd_mpi* m, const hsgd_views* v, const uint64_t* mask,
                           int32_t kcap, const float* dimg, float lr_rgb, float lr_alpha,
                           float lambda_s, float* grad_out, float* out_loss, void* ws,
                           size_t ws_bytes, hipStream_t stream) {
    clear_error();
    const char* fn = "hsgd_grad_step";
    hsgd_status st = check_mpi(m, fn);
    if (st) return st;
    st = check_views(v, m, dimg == nullptr || out_loss != nullptr, fn);
    if (st) return st;
    if (!mask) kcap = m->D;
    if (kcap < 1 || kcap > m->D) return fail(HSGD_E_ARG, "%s: kcap=%d outside [1, D=%d]", fn, kcap, m->D);
    if ((int64_t)kcap * m->H * m->W >= ((int64_t)1 << 28))
        return fail(HSGD_E_SHAPE, "%s: kcap*H*W must stay below 2^28 gradient slots per view", fn);
    if (!std::isfinite(lr_rgb) || !std::isfinite(lr_alpha) || !std::isfinite(lambda_s))
        return fail(HSGD_E_ARG, "%s: learning rates and lambda_s must be finite", fn);
    const GradWs L = grad_ws(m->D, m->H, m->W, v->N, kcap);
    st = check_ws(ws, ws_bytes, L.bytes);
    if (st) return st;
    float4* slots = reinterpret_cast<float4*>((char*)ws + L.slots_off);
    float* partials = reinterpret_cast<float*>((char*)ws + L.partial_off);
    return hip_status(launch_grad_step(*m, *v, mask, kcap, dimg, lr_rgb, lr_alpha, lambda_s, grad_out, out_loss,
                                       slots, partials, stream), fn);
}

hsgd_status hsgd_upsample2x(const hsgd_mpi* coarse, hsgd_mpi* fine, hipStream_t stream) {
    clear_error();
    const char* fn = "hsgd_upsample2x";
    hsgd_status st = check_mpi(coarse, fn);
    if (st) return st;
    st = check_mpi(fine, fn);
    if (st) return st;
    if (fine->D != coarse->D || fine->H != 2 * coarse->H || fine->W != 2 * coarse->W)
        return fail(HSGD_E_SHAPE, "%s: fine must be D x 2H x 2W of the coarse MPI", fn);
    if (fine->dtype != coarse->dtype) return fail(HSGD_E_DTYPE, "%s: dtypes differ", fn);
    if (fine->rgba == coarse->rgba) return fail(HSGD_E_ARG, "%s: in-place upsampling", fn);
    return hip_status(launch_upsample(*coarse, *fine, stream), fn);
}

hsgd_status hsgd_downsample2x(const float* images, int32_t N, int32_t H, int32_t W,
                              float* out, hipStream_t stream) {
    clear_error();
    const char* fn = "hsgd_downsample2x";
    if (!images || !out) return fail(HSGD_E_ARG, "%s: NULL pointer", fn);
    if (N < 1 || N > kMaxN || H < 2 || W < 2 || H % 2 || W % 2)
        return fail(HSGD_E_SHAPE, "%s: N=%d H=%d W=%d (H, W must be even)", fn, N, H, W);
    return hip_status(launch_downsample(images, N, H, W, out, stream), fn);
}

hsgd_status hsgd_plane_sweep(const hsgd_views* src, int32_t D, int32_t L, int32_t out_dtype, void* const* out,
                             hipStream_t stream) {
    clear_error();
    const char* fn = "hsgd_plane_sweep";
    if (!src || !out) return fail(HSGD_E_ARG, "%s: NULL pointer", fn);
    if (!src->images || !src->warps) return fail(HSGD_E_ARG, "%s: images or warps are NULL", fn);
    if (src->N < 1 || src->N > kMaxN || D < 1 || D > kMaxD)
        return fail(HSGD_E_SHAPE, "%s: N=%d or D=%d out of range", fn, src->N, D);
    if (L < 1 || L > kPsvMaxL) return fail(HSGD_E_SHAPE, "%s: L=%d outside [1, %d]", fn, L, kPsvMaxL);
    if (out_dtype != HSGD_FP32 && out_dtype != HSGD_BF16) return fail(HSGD_E_DTYPE, "%s: unknown dtype %d", fn, out_dtype);
    const int s = 1 << (L - 1);
    if (src->H < 1 || src->W < 1 || src->H % s || src->W % s)
        return fail(HSGD_E_SHAPE, "%s: %dx%d is not a positive multiple of 2^(L-1) = %d", fn, src->W, src->H, s);
    if ((int64_t)src->N * D * ((src->W + 63) / 64) * ((src->H + 15) / 16) > INT32_MAX ||
        (int64_t)src->H * src->W * 12 > INT32_MAX)
        return fail(HSGD_E_SHAPE, "%s: volume or image too large for one launch", fn);
    bool any = false;
    for (int l = 0; l < L; ++l) {
        if ((uintptr_t)out[l] % 16) return fail(HSGD_E_ARG, "%s: out[%d] is not 16-byte aligned", fn, l);
        any = any || out[l];
    }
    if (!any) return fail(HSGD_E_ARG, "%s: every output level is NULL", fn);
    return hip_status(launch_plane_sweep(*src, D, L, out_dtype, out, stream), fn);
}

hsgd_status hsgd_convert(const void* src, int32_t src_dtype, void* dst, int32_t dst_dtype,
                         size_t n, hipStream_t stream) {
    clear_error();
    const char* fn = "hsgd_convert";
    if (!src || !dst) return fail(HSGD_E_ARG, "%s: NULL pointer", fn);
    if (dtype_bytes(src_dtype) == 0 || dtype_bytes(dst_dtype) == 0)
        return fail(HSGD_E_DTYPE, "%s: unknown dtype", fn);
    if (n == 0) return HSGD_OK;
    return hip_status(launch_convert(src, src_dtype, dst, dst_dtype, n, stream), fn);
}

hsgd_status hsgd_refine(hsgd_mpi* levels, const hsgd_views* views, int32_t L,
                        const int32_t* iters, hsgd_select_params sel, float lr_rgb,
                        float lr_alpha, float lambda_s, float* loss_log, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
    clear_error();
    const char* fn = "hsgd_refine";
    size_t need = 0;
    hsgd_status st = refine_check(fn, levels, views, L, iters, sel, lr_rgb, lr_alpha, lambda_s, &need);
    if (st) return st;
    st = check_ws(ws, ws_bytes, need);
    if (st) return st;
    return refine_run(fn, levels, views, L, iters, sel, lr_rgb, lr_alpha, lambda_s, loss_log, ws, stream);
}

}  // extern "C"

namespace hsgd {

hsgd_status refine_check(const char* fn, const hsgd_mpi* levels, const hsgd_views* views, int32_t L,
                         const int32_t* iters, hsgd_select_params sel, float lr_rgb, float lr_alpha,
                         float lambda_s, size_t* ws_need) {
    if (!levels || !views || !iters) return fail(HSGD_E_ARG, "%s: NULL pointer", fn);
    if (L < 1 || L > 16) return fail(HSGD_E_ARG, "%s: L=%d outside [1, 16]", fn, L);
    hsgd_status st;
    for (int l = 0; l < L; ++l) {
        st = check_mpi(&levels[l], fn);
        if (st) return st;
        st = check_views(&views[l], &levels[l], l == L - 1, fn);
        if (st) return st;
        if (iters[l] < 0) return fail(HSGD_E_ARG, "%s: iters[%d] < 0", fn, l);
        if (l > 0) {
            const hsgd_mpi& c = levels[l - 1];
            const hsgd_mpi& f = levels[l];
            if (f.D != c.D || f.H != 2 * c.H || f.W != 2 * c.W)
                return fail(HSGD_E_SHAPE, "%s: level %d is not 2x level %d", fn, l, l - 1);
            if (f.dtype != c.dtype) return fail(HSGD_E_DTYPE, "%s: levels differ in dtype", fn);
            if (views[l].N != views[0].N) return fail(HSGD_E_SHAPE, "%s: view count differs by level", fn);
            if (f.rgba == c.rgba) return fail(HSGD_E_ARG, "%s: levels %d and %d alias", fn, l - 1, l);
        }
    }
    const hsgd_mpi& top = levels[L - 1];
    if (sel.k < 1 || sel.k > top.D) return fail(HSGD_E_ARG, "%s: k=%d outside [1, D]", fn, sel.k);
    if ((int64_t)sel.k * top.H * top.W >= ((int64_t)1 << 28))
        return fail(HSGD_E_SHAPE, "%s: k*H*W must stay below 2^28 gradient slots per view", fn);
    if (std::isnan(sel.tau)) return fail(HSGD_E_ARG, "%s: tau is NaN", fn);
    if (sel.rule != HSGD_SELECT_TOPK && sel.rule != HSGD_SELECT_MVS)
        return fail(HSGD_E_ARG, "%s: unknown selection rule %d", fn, sel.rule);
    if (!std::isfinite(lr_rgb) || !std::isfinite(lr_alpha) || !std::isfinite(lambda_s))
        return fail(HSGD_E_ARG, "%s: learning rates and lambda_s must be finite", fn);
    *ws_need = refine_ws(top.D, top.H, top.W, views[0].N, sel.k, L).bytes;
    return HSGD_OK;
}

hsgd_status refine_run(const char* fn, hsgd_mpi* levels, const hsgd_views* views, int32_t L, const int32_t* iters,
                       hsgd_select_params sel, float lr_rgb, float lr_alpha, float lambda_s, float* loss_log,
                       void* ws, hipStream_t stream) {
    const hsgd_mpi& top = levels[L - 1];
    const int N = views[0].N;
    const RefineWs R = refine_ws(top.D, top.H, top.W, N, sel.k, L);

    // one mask and one workspace region sized for the finest level serve every level
    uint64_t* mask = reinterpret_cast<uint64_t*>((char*)ws + R.mask_off);
    // target pyramid: coarser images that were not given are box means of the finer ones,
    // up to three consecutive missing levels from one launch; the first such launch also
    // makes the coarsest level's first selection when that level iterates
    bool first_selected = false;
    const float* img[16];
    img[L - 1] = views[L - 1].images;
    for (int l = L - 2; l >= 0;) {
        if (views[l].images) {
            img[l] = views[l].images;
            --l;
            continue;
        }
        int nl = 0;
        float* dst[3] = {nullptr, nullptr, nullptr};
        while (nl < 3 && l - nl >= 0 && !views[l - nl].images) {
            dst[nl] = reinterpret_cast<float*>((char*)ws + R.pyr_off[l - nl]);
            ++nl;
        }
        int e;
        if (!first_selected && iters[0] > 0) {
            e = launch_select_pyramid(levels[0], sel.k, sel.tau, sel.rule, mask, img[l + 1], N, levels[l + 1].H,
                                      levels[l + 1].W, nl, dst, stream);
            first_selected = true;
        } else {
            e = launch_pyramid(img[l + 1], N, levels[l + 1].H, levels[l + 1].W, nl, dst, stream);
        }
        if (e) return hip_status(e, fn);
        for (int j = 0; j < nl; ++j) img[l - j] = dst[j];
        l -= nl;
    }
    char* inner = (char*)ws + R.inner_off;
    int it_global = 0;
    for (int l = 0; l < L; ++l) {
        // a level's first selection comes out of the upsampling kernel that fills it
        const bool fused = l > 0 && iters[l] > 0;
        if (l > 0) {
            int e = fused ? launch_upsample_select(levels[l - 1], levels[l], sel.k, sel.tau, sel.rule, mask, stream)
                          : launch_upsample(levels[l - 1], levels[l], stream);
            if (e) return hip_status(e, fn);
        }
        hsgd_views v = views[l];
        v.images = img[l];
        const GradWs G = grad_ws(levels[l].D, levels[l].H, levels[l].W, N, sel.k);
        float4* slots = reinterpret_cast<float4*>(inner + G.slots_off);
        float* partials = reinterpret_cast<float*>(inner + G.partial_off);
        for (int it = 0; it < iters[l]; ++it, ++it_global) {
            const bool selected = (fused || (l == 0 && first_selected)) && it == 0;
            int e = selected ? 0 : launch_select(levels[l], sel.k, sel.tau, sel.rule, mask, nullptr, nullptr, stream);
            if (e) return hip_status(e, fn);
            e = launch_grad_step(levels[l], v, mask, sel.k, nullptr, lr_rgb, lr_alpha, lambda_s, nullptr,
                                 loss_log ? loss_log + it_global : nullptr, slots, partials, stream);
            if (e) return hip_status(e, fn);
        }
    }
    return HSGD_OK;
}

}  // namespace hsgd
