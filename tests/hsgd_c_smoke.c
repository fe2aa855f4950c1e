/*
 * libhsgd used from plain C: device buffers from the HIP runtime, every step through the C
 * ABI of include/hsgd.h (no Python, no PyTorch). Built next to the library by the package's
 * build step; tests/test_gpu_c_abi.py runs it.
 *
 * A tiny scene: D = 4 planes of 16 x 8 pixels, plane 1 opaque and of one colour, the other
 * planes transparent; view 0 sits at the reference pose, view 1 is translated. Checked:
 * status codes; the reference-pose render reproduces the colour; the active set keeps k
 * planes of every pixel; against the views' own renders the loss and the gradient
 * vanish; a two-level refine runs and logs finite losses; a NULL argument is refused with a
 * message. Prints "ok" and exits 0 when everything holds.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "hsgd.h"

#define CHECK_HIP(x)                                                                  \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) {                                                       \
            fprintf(stderr, "%s:%d: HIP error %d\n", __FILE__, __LINE__, (int)e_);   \
            return 1;                                                                 \
        }                                                                             \
    } while (0)
#define CHECK(x)                                                                      \
    do {                                                                              \
        hsgd_status s_ = (x);                                                         \
        if (s_ != HSGD_OK) {                                                          \
            fprintf(stderr, "%s:%d: %s: %s\n", __FILE__, __LINE__,                  \
                    hsgd_status_string(s_), hsgd_last_error());                       \
            return 1;                                                                 \
        }                                                                             \
    } while (0)
#define EXPECT(c, msg)                                                                \
    do {                                                                              \
        if (!(c)) {                                                                   \
            fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, msg);                 \
            return 1;                                                                 \
        }                                                                             \
    } while (0)

enum { D = 4, H = 8, W = 16, N = 2, K = 2, L = 2 };

static const float kColour[3] = {0.2f, 0.4f, 0.6f};

/* pinhole intrinsics of a w x h camera with focal f, principal point at the centre */
static void intrinsics(double f, int w, int h, double* k) {
    const double v[9] = {f, 0.0, (w - 1) / 2.0, 0.0, f, (h - 1) / 2.0, 0.0, 0.0, 1.0};
    memcpy(k, v, sizeof v);
}

int main(void) {
    /* ---- host inputs ---- */
    static float mpi_h[D][H][W][4];
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                float* p = mpi_h[z][y][x];
                if (z == 1) {
                    p[0] = kColour[0], p[1] = kColour[1], p[2] = kColour[2], p[3] = 1.0f;
                } else {
                    p[0] = p[1] = p[2] = 0.5f, p[3] = 0.0f;
                }
            }
    double Kr[9], Kv[N * 9], Rv[N * 9], tv[N * 3], depth[D];
    intrinsics(12.0, W, H, Kr);
    for (int i = 0; i < N; ++i) {
        memcpy(Kv + 9 * i, Kr, sizeof Kr);
        for (int j = 0; j < 9; ++j) Rv[9 * i + j] = (j % 4 == 0) ? 1.0 : 0.0;
        tv[3 * i + 0] = i == 0 ? 0.0 : 0.05;
        tv[3 * i + 1] = 0.0;
        tv[3 * i + 2] = 0.0;
    }
    for (int z = 0; z < D; ++z) depth[z] = 1.0 / (1.0 - z * 0.99 / (D - 1));
    hsgd_warp warps_h[N * D];
    CHECK(hsgd_build_warps(Kr, Kv, Rv, tv, depth, N, D, warps_h));
    EXPECT(hsgd_warps_shift_only(warps_h, N * D) == 1, "expected pure translations");

    /* ---- device buffers ---- */
    const size_t mpi_bytes = sizeof mpi_h, img_bytes = sizeof(float) * N * H * W * 3;
    size_t ws_bytes = 0;
    const int32_t ops[4] = {HSGD_OP_SELECT, HSGD_OP_RENDER, HSGD_OP_GRAD_STEP, HSGD_OP_REFINE};
    for (int o = 0; o < 4; ++o) {
        const size_t b = hsgd_workspace_bytes(ops[o], D, H, W, N, K, L);
        EXPECT(b > 0, "workspace query refused valid sizes");
        if (b > ws_bytes) ws_bytes = b;
    }
    void *mpi_d, *ws_d, *coarse_d;
    hsgd_warp *warps_d, *warps_l_d[L];
    float *rgb_d, *loss_d, *grad_d, *log_d;
    uint64_t* mask_d;
    int32_t *ids_d, *off_d, *nact_d;
    CHECK_HIP(hipMalloc(&mpi_d, mpi_bytes));
    CHECK_HIP(hipMalloc(&coarse_d, mpi_bytes / 4));
    CHECK_HIP(hipMalloc((void**)&warps_d, sizeof warps_h));
    for (int l = 0; l < L; ++l) CHECK_HIP(hipMalloc((void**)&warps_l_d[l], sizeof warps_h));
    CHECK_HIP(hipMalloc((void**)&rgb_d, img_bytes));
    CHECK_HIP(hipMalloc((void**)&loss_d, sizeof(float)));
    CHECK_HIP(hipMalloc((void**)&grad_d, mpi_bytes));
    CHECK_HIP(hipMalloc((void**)&log_d, sizeof(float) * L));
    CHECK_HIP(hipMalloc((void**)&mask_d, sizeof(uint64_t) * H * W));
    CHECK_HIP(hipMalloc((void**)&ids_d, sizeof(int32_t) * K * H * W));
    CHECK_HIP(hipMalloc((void**)&off_d, sizeof(int32_t) * (D + 1)));
    CHECK_HIP(hipMalloc((void**)&nact_d, sizeof(int32_t)));
    CHECK_HIP(hipMalloc(&ws_d, ws_bytes));
    CHECK_HIP(hipMemcpy(mpi_d, mpi_h, mpi_bytes, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(warps_d, warps_h, sizeof warps_h, hipMemcpyHostToDevice));

    hsgd_mpi m = {mpi_d, D, H, W, HSGD_FP32};
    hsgd_views v = {NULL, warps_d, N, H, W, HSGD_VIEWS_SHIFT_ONLY};

    /* ---- render: view 0 (reference pose) sees the opaque plane everywhere ---- */
    CHECK(hsgd_render(&m, &v, rgb_d, NULL, ws_d, ws_bytes, NULL));
    CHECK_HIP(hipDeviceSynchronize());
    static float rgb_h[N][H][W][3];
    CHECK_HIP(hipMemcpy(rgb_h, rgb_d, img_bytes, hipMemcpyDeviceToHost));
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < 3; ++c)
                EXPECT(fabsf(rgb_h[0][y][x][c] - kColour[c]) <= 1e-6f, "reference-pose render is not the colour");

    /* ---- select: k planes per pixel, plane-major ids ---- */
    const hsgd_select_params sp = {K, -1.0f, HSGD_SELECT_TOPK};
    CHECK(hsgd_select_active(&m, sp, mask_d, ids_d, K * H * W, off_d, nact_d, ws_d, ws_bytes, NULL));
    CHECK_HIP(hipDeviceSynchronize());
    int32_t nact = 0;
    static uint64_t mask_h[H * W];
    CHECK_HIP(hipMemcpy(&nact, nact_d, sizeof nact, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(mask_h, mask_d, sizeof mask_h, hipMemcpyDeviceToHost));
    EXPECT(nact == K * H * W, "active set size is not k H W");
    for (int p = 0; p < H * W; ++p) EXPECT(__builtin_popcountll(mask_h[p]) == K, "a pixel does not keep k planes");

    /* ---- gradient against the views' own renders: zero residual ---- */
    v.images = rgb_d;
    CHECK(hsgd_grad_step(&m, &v, mask_d, K, NULL, 0.0f, 0.0f, 0.0f, grad_d, loss_d, ws_d, ws_bytes, NULL));
    CHECK_HIP(hipDeviceSynchronize());
    float loss = -1.0f;
    static float grad_h[D][H][W][4];
    CHECK_HIP(hipMemcpy(&loss, loss_d, sizeof loss, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(grad_h, grad_d, mpi_bytes, hipMemcpyDeviceToHost));
    /* (render and gradient kernels may order the bilinear sums differently: last-bit slack) */
    EXPECT(loss >= 0.0f && loss <= 1e-9f, "loss against the own renders is not zero");
    for (size_t i = 0; i < sizeof grad_h / sizeof(float); ++i)
        EXPECT(fabsf(((const float*)grad_h)[i]) <= 1e-6f, "gradient at zero residual is not zero");

    /* ---- two-level refine (8 x 4, then 16 x 8) from a grey, half-transparent start ---- */
    static float coarse_h[D][H / 2][W / 2][4];
    for (size_t i = 0; i < sizeof coarse_h / sizeof(float); ++i) ((float*)coarse_h)[i] = 0.5f;
    CHECK_HIP(hipMemcpy(coarse_d, coarse_h, sizeof coarse_h, hipMemcpyHostToDevice));
    hsgd_mpi levels[L] = {{coarse_d, D, H / 2, W / 2, HSGD_FP32}, {mpi_d, D, H, W, HSGD_FP32}};
    hsgd_views views[L];
    for (int l = 0; l < L; ++l) {
        const int wl = W >> (L - 1 - l), hl = H >> (L - 1 - l);
        double Krl[9], Kvl[N * 9];
        CHECK(hsgd_level_intrinsics(Kr, W, H, wl, hl, Krl));
        for (int i = 0; i < N; ++i) CHECK(hsgd_level_intrinsics(Kv + 9 * i, W, H, wl, hl, Kvl + 9 * i));
        hsgd_warp wl_h[N * D];
        CHECK(hsgd_build_warps(Krl, Kvl, Rv, tv, depth, N, D, wl_h));
        CHECK_HIP(hipMemcpy(warps_l_d[l], wl_h, sizeof wl_h, hipMemcpyHostToDevice));
        const hsgd_views vl = {l == L - 1 ? rgb_d : NULL, warps_l_d[l], N, hl, wl,
                               hsgd_warps_shift_only(wl_h, N * D) ? HSGD_VIEWS_SHIFT_ONLY : 0};
        views[l] = vl;
    }
    const int32_t iters[L] = {1, 1};
    CHECK(hsgd_refine(levels, views, L, iters, sp, 1.0f, 1.0f, 0.0f, log_d, ws_d, ws_bytes, NULL));
    CHECK_HIP(hipDeviceSynchronize());
    float log_h[L];
    CHECK_HIP(hipMemcpy(log_h, log_d, sizeof log_h, hipMemcpyDeviceToHost));
    for (int l = 0; l < L; ++l) EXPECT(isfinite(log_h[l]) && log_h[l] >= 0.0f, "refine logged a bad loss");

    /* ---- a refused call: nothing enqueued, a message set ---- */
    EXPECT(hsgd_render(NULL, &v, rgb_d, NULL, ws_d, ws_bytes, NULL) == HSGD_E_ARG, "NULL MPI accepted");
    EXPECT(strlen(hsgd_last_error()) > 0, "no message for a refused call");

    hipFree(mpi_d);
    hipFree(coarse_d);
    hipFree(warps_d);
    for (int l = 0; l < L; ++l) hipFree(warps_l_d[l]);
    hipFree(rgb_d);
    hipFree(loss_d);
    hipFree(grad_d);
    hipFree(log_d);
    hipFree(mask_d);
    hipFree(ids_d);
    hipFree(off_d);
    hipFree(nact_d);
    hipFree(ws_d);
    printf("ok\n");
    return 0;
}
