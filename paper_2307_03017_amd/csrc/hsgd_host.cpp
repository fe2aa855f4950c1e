// Host-side part of libhsgd: FP64 plane homographies (Sec. 3.2, Eq. homo), level
// intrinsics, argument validation, workspace layouts and error reporting. No HIP calls:
// this file also builds with g++ alone for host-only tests.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "hsgd_internal.h"

namespace hsgd {

static thread_local char g_err[512] = "";

hsgd_status fail(hsgd_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

void clear_error() { g_err[0] = 0; }

size_t dtype_bytes(int dtype) {
    switch (dtype) {
        case HSGD_FP32: return 16;
        case HSGD_BF16: return 8;
        default: return 0;
    }
}

hsgd_status check_mpi(const hsgd_mpi* m, const char* what) {
    if (!m) return fail(HSGD_E_ARG, "%s: MPI descriptor is NULL", what);
    if (!m->rgba) return fail(HSGD_E_ARG, "%s: MPI data pointer is NULL", what);
    if (dtype_bytes(m->dtype) == 0) return fail(HSGD_E_DTYPE, "%s: unknown dtype %d", what, m->dtype);
    if (m->D < 1 || m->D > kMaxD)
        return fail(HSGD_E_SHAPE, "%s: D=%d outside [1, %d]", what, m->D, kMaxD);
    if (m->H < 2 || m->W < 2 || (int64_t)m->H * m->W > (int64_t)1 << 26)
        return fail(HSGD_E_SHAPE, "%s: H=%d W=%d out of range", what, m->H, m->W);
    if ((int64_t)m->D * m->H * m->W > ((int64_t)1 << 31) - 1)
        return fail(HSGD_E_SHAPE, "%s: D*H*W exceeds 2^31-1 voxels", what);
    return HSGD_OK;
}

hsgd_status check_views(const hsgd_views* v, const hsgd_mpi* m, bool need_images,
                        const char* what) {
    if (!v) return fail(HSGD_E_ARG, "%s: views descriptor is NULL", what);
    if (!v->warps) return fail(HSGD_E_ARG, "%s: warps pointer is NULL", what);
    if (need_images && !v->images) return fail(HSGD_E_ARG, "%s: target images are NULL", what);
    if (v->N < 1 || v->N > kMaxN) return fail(HSGD_E_SHAPE, "%s: N=%d outside [1, %d]", what, v->N, kMaxN);
    if (v->H != m->H || v->W != m->W)
        return fail(HSGD_E_SHAPE, "%s: views are %dx%d but the MPI is %dx%d", what, v->W, v->H,
                    m->W, m->H);
    return HSGD_OK;
}

hsgd_status check_ws(void* ws, size_t ws_bytes, size_t need) {
    if (need && !ws) return fail(HSGD_E_WORKSPACE, "workspace is NULL, %zu bytes needed", need);
    if (ws_bytes < need)
        return fail(HSGD_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
    if ((uintptr_t)ws % kAlign)
        return fail(HSGD_E_WORKSPACE, "workspace must be %zu-byte aligned", (size_t)kAlign);
    return HSGD_OK;
}

ActiveLayout active_ws(int D, int H, int W, int64_t cap, bool with_ids) {
    ActiveLayout L{};
    L.nblk = ceil_div((int64_t)H * W, 64);
    L.nseg = ceil_div((int64_t)D * L.nblk, kScanSeg);
    L.cap = cap;
    size_t o = 0;
    L.bal_off = o;
    o += align_up(sizeof(uint64_t) * (size_t)D * L.nblk);
    L.off_off = o;
    o += align_up(sizeof(int32_t) * (size_t)D * L.nblk);
    L.seg_off = o;
    o += align_up(sizeof(int32_t) * (size_t)L.nseg);
    L.ids_off = L.nact_off = 0;
    if (with_ids) {
        L.ids_off = o;
        o += align_up(sizeof(int32_t) * (size_t)cap);
        L.nact_off = o;
        o += align_up(sizeof(int32_t));
    }
    L.bytes = o;
    return L;
}

ActiveSet active_at(void* ws, const ActiveLayout& L, int* ids, int* nact) {
    char* b = static_cast<char*>(ws);
    ActiveSet a;
    a.bal = reinterpret_cast<uint64_t*>(b + L.bal_off);
    a.off = reinterpret_cast<int*>(b + L.off_off);
    a.seg = reinterpret_cast<int*>(b + L.seg_off);
    a.ids = ids ? ids : reinterpret_cast<int*>(b + L.ids_off);
    a.nact = nact ? nact : reinterpret_cast<int*>(b + L.nact_off);
    a.nblk = L.nblk;
    a.nseg = L.nseg;
    a.cap = L.cap;
    return a;
}

RenderWs render_ws(int H, int W, int N) {
    RenderWs w{};
    // loss partials of either render kernel: general (64 x 4 rays) or translation (63 x 8)
    const int64_t general = ceil_div(W, kTileW) * ceil_div(H, kTileH) * N;
    const int64_t shift = ceil_div(W, kShiftRX) * ceil_div(H, kShiftRY) * N;
    w.nparts = general > shift ? general : shift;
    w.partial_off = 0;
    w.bytes = align_up(sizeof(float) * w.nparts);
    return w;
}

GradWs grad_ws(int D, int H, int W, int N, int kcap) {
    (void)D;
    GradWs w{};
    const int64_t cap = (int64_t)kcap * H * W;
    w.slots_off = 0;
    w.partial_off = align_up(sizeof(float) * 4 * (size_t)N * cap);
    const int64_t general = ceil_div(W, kTileW) * ceil_div(H, kTileH) * N;
    const int64_t shift = ceil_div(W + 1, kShiftOX) * ceil_div(H + 1, kShiftOY) * N;
    w.nparts = general > shift ? general : shift;
    w.bytes = w.partial_off + align_up(sizeof(float) * w.nparts);
    return w;
}

RefineWs refine_ws(int D, int H, int W, int N, int k, int L) {
    RefineWs w{};
    size_t off = 0;
    for (int l = 0; l < L - 1 && l < 16; ++l) {
        int s = 1 << (L - 1 - l);
        w.pyr_off[l] = off;
        off += align_up(sizeof(float) * 3 * (size_t)N * (H / s) * (W / s));
    }
    w.mask_off = off;
    off += align_up(sizeof(uint64_t) * (size_t)H * W);
    w.inner_off = off;
    off += grad_ws(D, H, W, N, k).bytes;
    w.bytes = off;
    return w;
}

}  // namespace hsgd

using namespace hsgd;

// ---------------------------------------------------------------------------------------
// 3x3 helpers in FP64
// ---------------------------------------------------------------------------------------
static void mat3_mul(const double* a, const double* b, double* c) {
    double r[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            r[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
    memcpy(c, r, sizeof r);
}

// Inverse by the adjugate; returns false when the matrix is singular.
static bool mat3_inv(const double* m, double* out) {
    double c00 = m[4] * m[8] - m[5] * m[7];
    double c01 = m[5] * m[6] - m[3] * m[8];
    double c02 = m[3] * m[7] - m[4] * m[6];
    double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
    double scale = 0.0;
    for (int i = 0; i < 9; ++i) scale = std::fmax(scale, std::fabs(m[i]));
    if (!(std::fabs(det) > 1e-300) || !(std::fabs(det) > 1e-14 * scale * scale * scale)) return false;
    double inv = 1.0 / det;
    out[0] = c00 * inv;
    out[1] = (m[2] * m[7] - m[1] * m[8]) * inv;
    out[2] = (m[1] * m[5] - m[2] * m[4]) * inv;
    out[3] = c01 * inv;
    out[4] = (m[0] * m[8] - m[2] * m[6]) * inv;
    out[5] = (m[2] * m[3] - m[0] * m[5]) * inv;
    out[6] = c02 * inv;
    out[7] = (m[1] * m[6] - m[0] * m[7]) * inv;
    out[8] = (m[0] * m[4] - m[1] * m[3]) * inv;
    return true;
}

extern "C" {

const char* hsgd_status_string(int32_t s) {
    switch (s) {
        case HSGD_OK: return "HSGD_OK";
        case HSGD_E_ARG: return "HSGD_E_ARG: invalid argument";
        case HSGD_E_SHAPE: return "HSGD_E_SHAPE: invalid or inconsistent shape";
        case HSGD_E_DTYPE: return "HSGD_E_DTYPE: unknown storage type";
        case HSGD_E_CAPACITY: return "HSGD_E_CAPACITY: output capacity too small";
        case HSGD_E_WORKSPACE: return "HSGD_E_WORKSPACE: workspace missing or too small";
        case HSGD_E_HIP: return "HSGD_E_HIP: HIP runtime error";
        case HSGD_E_BUDGET: return "HSGD_E_BUDGET: over the serving HBM budget";
        default: return "unknown hsgd_status";
    }
}

const char* hsgd_last_error(void) { return g_err; }

int32_t hsgd_version(void) { return 1 * 10000 + 0 * 100 + 0; }

hsgd_status hsgd_level_intrinsics(const double* K, int32_t W, int32_t H, int32_t Wl,
                                  int32_t Hl, double* out) {
    clear_error();
    if (!K || !out) return fail(HSGD_E_ARG, "hsgd_level_intrinsics: NULL pointer");
    if (W < 1 || H < 1 || Wl < 1 || Hl < 1)
        return fail(HSGD_E_SHAPE, "hsgd_level_intrinsics: sizes must be positive");
    double sx = (double)Wl / W, sy = (double)Hl / H;
    double r[9];
    memcpy(r, K, sizeof r);
    r[0] = K[0] * sx;
    r[1] = K[1] * sx;
    r[2] = (K[2] + 0.5) * sx - 0.5;
    r[4] = K[4] * sy;
    r[5] = (K[5] + 0.5) * sy - 0.5;
    memcpy(out, r, sizeof r);
    return HSGD_OK;
}

// Per (view, plane) maps of Eq. (homo): view pixel -> reference pixel (to_reference, the
// direction rendering gathers in) or reference pixel -> view pixel (the plane-sweep
// direction), as hsgd_warp records with the exact integer + fraction split of translations.
static hsgd_status build_maps(const double* K_ref, const double* K, const double* R, const double* t,
                              const double* depth, int32_t N, int32_t D, hsgd_warp* out, bool to_reference,
                              const char* fn) {
    clear_error();
    if (!K_ref || !K || !R || !t || !depth || !out)
        return fail(HSGD_E_ARG, "%s: NULL pointer", fn);
    if (N < 1 || N > kMaxN || D < 1 || D > kMaxD)
        return fail(HSGD_E_SHAPE, "%s: N=%d or D=%d out of range", fn, N, D);
    double Kr_inv[9];
    if (!mat3_inv(K_ref, Kr_inv)) return fail(HSGD_E_ARG, "%s: K_ref is singular", fn);
    for (int z = 0; z < D; ++z)
        if (!(depth[z] > 0.0) || !std::isfinite(depth[z]))
            return fail(HSGD_E_ARG, "%s: depth[%d] = %g is not positive", fn, z, depth[z]);
    hsgd_warp* tmp = new hsgd_warp[(size_t)N * D];
    for (int i = 0; i < N; ++i) {
        const double* Ki = K + 9 * i;
        const double* Ri = R + 9 * i;
        const double* ti = t + 3 * i;
        for (int z = 0; z < D; ++z) {
            // Eq. (homo) with the reference pose at the identity and n = (0, 0, 1):
            // K_i R_i (I + R_i^{-1} t_i n^T / d) K_ref^{-1} = K_i (R_i + t_i n^T / d) K_ref^{-1}
            double A[9];
            memcpy(A, Ri, sizeof A);
            for (int r = 0; r < 3; ++r) A[3 * r + 2] += ti[r] / depth[z];
            double Hm[9], G[9];
            mat3_mul(Ki, A, Hm);
            mat3_mul(Hm, Kr_inv, Hm);
            // a singular map is refused in either direction
            const bool ok = mat3_inv(Hm, G);
            if (!to_reference) memcpy(G, Hm, sizeof G);
            if (!ok || !(std::fabs(G[8]) > 0.0)) {
                delete[] tmp;
                return fail(HSGD_E_ARG, "%s: view %d plane %d map is singular", fn, i, z);
            }
            // normalise by |G[8]|: positions unchanged, the sign of the homogeneous
            // coordinate (in front of / behind the view) kept
            double s = 1.0 / std::fabs(G[8]);
            for (double& g : G) g *= s;
            hsgd_warp& w = tmp[(size_t)i * D + z];
            memset(&w, 0, sizeof w);
            for (int j = 0; j < 9; ++j) w.G[j] = G[j];
            const double eps = 1e-12;
            bool shift = std::fabs(G[0] - 1) <= eps && std::fabs(G[4] - 1) <= eps &&
                         std::fabs(G[1]) <= eps && std::fabs(G[3]) <= eps &&
                         std::fabs(G[6]) <= eps && std::fabs(G[7]) <= eps && G[8] > 0;
            if (shift && std::fabs(G[2]) < 1e6 && std::fabs(G[5]) < 1e6) {
                // exact integer + fraction split of the translation
                double fx0 = std::floor(G[2]), fy0 = std::floor(G[5]);
                double fx = G[2] - fx0, fy = G[5] - fy0;
                int ix = (int)fx0, iy = (int)fy0;
                if (fx < 1e-9) fx = 0.0;
                if (fy < 1e-9) fy = 0.0;
                float fxf = (float)fx, fyf = (float)fy;
                if (fxf >= 1.0f) { ix += 1; fxf = 0.0f; }
                if (fyf >= 1.0f) { iy += 1; fyf = 0.0f; }
                w.is_shift = 1;
                w.ix = ix;
                w.iy = iy;
                w.fx = fxf;
                w.fy = fyf;
            }
        }
    }
    memcpy(out, tmp, sizeof(hsgd_warp) * (size_t)N * D);
    delete[] tmp;
    return HSGD_OK;
}

hsgd_status hsgd_build_warps(const double* K_ref, const double* K, const double* R,
                             const double* t, const double* depth, int32_t N, int32_t D,
                             hsgd_warp* out) {
    return build_maps(K_ref, K, R, t, depth, N, D, out, true, "hsgd_build_warps");
}

hsgd_status hsgd_build_psv_warps(const double* K_ref, const double* K, const double* R,
                                 const double* t, const double* depth, int32_t N, int32_t D,
                                 hsgd_warp* out) {
    return build_maps(K_ref, K, R, t, depth, N, D, out, false, "hsgd_build_psv_warps");
}

int32_t hsgd_warps_shift_only(const hsgd_warp* warps, int32_t n) {
    if (!warps || n < 1) return 0;
    for (int32_t i = 0; i < n; ++i)
        if (warps[i].is_shift != 1) return 0;
    return 1;
}

size_t hsgd_workspace_bytes(int32_t op, int32_t D, int32_t H, int32_t W, int32_t N,
                            int32_t k, int32_t L) {
    if (D < 1 || D > kMaxD || H < 2 || W < 2 || N < 1 || N > kMaxN) return 0;
    switch (op) {
        case HSGD_OP_SELECT: return active_ws(D, H, W, 0, false).bytes;
        case HSGD_OP_RENDER: return render_ws(H, W, N).bytes;
        case HSGD_OP_GRAD_STEP:
            if (k < 1 || k > D) return 0;
            return grad_ws(D, H, W, N, k).bytes;
        case HSGD_OP_REFINE: {
            if (k < 1 || k > D || L < 1 || L > 16) return 0;
            int s = 1 << (L - 1);
            if (H % s || W % s || H / s < 2 || W / s < 2) return 0;
            return refine_ws(D, H, W, N, k, L).bytes;
        }
        default: return 0;
    }
}

}  // extern "C"
