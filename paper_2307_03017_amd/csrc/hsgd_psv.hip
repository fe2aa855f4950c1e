// Plane-sweep volume of libhsgd for gfx950 (wave64).
//
//  k_plane_sweep  the source images inverse-warped onto every reference plane and box-
//                 downsampled level by level (Sec. 3.2, Hierarchical PSV Construction)
#include <hip/hip_runtime.h>

#include "hsgd_device.h"
#include "hsgd_internal.h"

namespace hsgd {
namespace {

// ------------------------------------------------------------------------------------
// plane-sweep volume and its pyramid (Sec. 3.2, Hierarchical PSV Construction): a
// workgroup samples one 64 x 16 reference tile of one (view, plane) from the source image
// (4 consecutive pixels of a row per thread), stores it, then reduces it 2x2 level by level
// in LDS and stores each level from there: no level is read back from memory.
// ------------------------------------------------------------------------------------
constexpr int kPsvTW = 64, kPsvTH = 16;
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct PsvOut {
    void* p[kPsvMaxL];
};
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ void st_stream(T v, T* p) {
    __builtin_nontemporal_store(v, p);
}

// Store the valid vh x vw pixels of a TH x TW tile, row-major in LDS (FP32), to rows of Wl
// pixels at dst (the tile's first pixel) in the output type OT. 16-byte runs when every row
// start is 16-byte aligned (FP32: Wl % 4 == 0; BF16: Wl % 8 == 0 and 16-byte tile rows; vw
// is then a multiple of the run's pixels too), else one pixel per lane; consecutive lanes
// write consecutive addresses either way. BF16 rounds to nearest even.
template <int TH, int TW, int OT>
__device__ __forceinline__ void psv_store_tile(const float* __restrict__ s, int vh, int vw, void* __restrict__ dst,
                                               int Wl, int t) {
    if (OT == HSGD_FP32 && (Wl & 3) == 0) {
        float* o = reinterpret_cast<float*>(dst);
        constexpr int RQ = TW * 3 / 4;                      // float4 per tile row
        const int vq = vw * 3 / 4;
#pragma unroll
        for (int e0 = 0; e0 < TH * RQ; e0 += 256) {
            const int e = e0 + t, r = e / RQ, c = e - r * RQ;
            if ((TH * RQ % 256 == 0 || e < TH * RQ) && r < vh && c < vq) {
                const float4 q = reinterpret_cast<const float4*>(s)[e];
                st_stream(f32x4{q.x, q.y, q.z, q.w}, reinterpret_cast<f32x4*>(o + (size_t)r * Wl * 3) + c);
            }
        }
    } else if (OT == HSGD_BF16 && TW * 6 % 16 == 0 && (Wl & 7) == 0) {
        uint16_t* o = reinterpret_cast<uint16_t*>(dst);
        constexpr int RQ = TW * 3 / 8;                      // 8 values (16 bytes) per run
        const int vq = vw * 3 / 8;
#pragma unroll
        for (int e0 = 0; e0 < TH * RQ; e0 += 256) {
            const int e = e0 + t, r = e / RQ, c = e - r * RQ;
            if ((TH * RQ % 256 == 0 || e < TH * RQ) && r < vh && c < vq) {
                const float4 a = reinterpret_cast<const float4*>(s)[2 * e];
                const float4 b = reinterpret_cast<const float4*>(s)[2 * e + 1];
                const u32x4 q{f32_to_bf16_bits(a.x) | (f32_to_bf16_bits(a.y) << 16),
                              f32_to_bf16_bits(a.z) | (f32_to_bf16_bits(a.w) << 16),
                              f32_to_bf16_bits(b.x) | (f32_to_bf16_bits(b.y) << 16),
                              f32_to_bf16_bits(b.z) | (f32_to_bf16_bits(b.w) << 16)};
                st_stream(q, reinterpret_cast<u32x4*>(o + (size_t)r * Wl * 3) + c);
            }
        }
    } else {
#pragma unroll
        for (int e0 = 0; e0 < TH * TW; e0 += 256) {
            const int e = e0 + t, r = e / TW, c = e - r * TW;
            if ((TH * TW % 256 == 0 || e < TH * TW) && r < vh && c < vw) {
                const size_t at = ((size_t)r * Wl + c) * 3;
                if (OT == HSGD_FP32) {
                    float* o = reinterpret_cast<float*>(dst) + at;
                    st_stream(s[3 * e], o);
                    st_stream(s[3 * e + 1], o + 1);
                    st_stream(s[3 * e + 2], o + 2);
                } else {
                    uint16_t* o = reinterpret_cast<uint16_t*>(dst) + at;
                    st_stream((uint16_t)f32_to_bf16_bits(s[3 * e]), o);
                    st_stream((uint16_t)f32_to_bf16_bits(s[3 * e + 1]), o + 1);
                    st_stream((uint16_t)f32_to_bf16_bits(s[3 * e + 2]), o + 2);
                }
            }
        }
    }
}

__device__ __forceinline__ float3 bilerp(float w00, float w10, float w01, float w11, float3 a, float3 b,
                                         float3 c, float3 d) {
    return make_float3(w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x,
                       w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y,
                       w00 * a.z + w10 * b.z + w01 * c.z + w11 * d.z);
}

__device__ __forceinline__ float3 lds_rgb(const float* p) { return make_float3(p[0], p[1], p[2]); }

// The source patch of a tile under a translation map: source rows sy0 .. sy0 + 16 and
// pixels sx0 .. sx0 + 64 (the taps of 16 x 64 reference pixels), staged in LDS by coalesced
// dword loads (consecutive lanes, consecutive dwords of a row) through one buffer resource
// over the image: positions outside the image read 0, the zero padding.
constexpr int kPsvSrcRow = (kPsvTW + 1) * 3;                // dwords per patch row
constexpr int kPsvSrcN = (kPsvTH + 1) * kPsvSrcRow;         // dwords per patch
__device__ __forceinline__ void psv_stage_patch(const float* __restrict__ im, int H, int W, int sx0, int sy0,
                                                float* __restrict__ sp, int t) {
    const auto rs = row_rsrc(reinterpret_cast<const char*>(im), H * W * 12);
#pragma unroll
    for (int k = 0; k < (kPsvSrcN + 255) / 256; ++k) {
        const int e = t + 256 * k;
        const int r = e / kPsvSrcRow, c = e - r * kPsvSrcRow;
        const int row = sy0 + r, col = sx0 * 3 + c;
        const bool in = (unsigned)row < (unsigned)H && (unsigned)col < (unsigned)(3 * W);
        const float v = __uint_as_float(
            __builtin_amdgcn_raw_buffer_load_b32(rs, in ? (unsigned)(row * W * 3 + col) * 4u : 0x80000000u, 0, 0));
        if (k < kPsvSrcN / 256 || e < kPsvSrcN) sp[e] = v;
    }
}

// Bilinear samples of a thread's 4 consecutive reference pixels from the staged patch: its
// patch row ly (and ly + 1), patch pixels 4 gx .. 4 gx + 4.
__device__ __forceinline__ void psv_blend_patch(const hsgd_warp& wp, const float* __restrict__ sp, int gx, int ly,
                                                float3 (&v)[4]) {
    const float fx = wp.fx, fy = wp.fy, gxw = 1.0f - fx, gyw = 1.0f - fy;
    const float w00 = gxw * gyw, w10 = fx * gyw, w01 = gxw * fy, w11 = fx * fy;
    const float* r0 = sp + ly * kPsvSrcRow + 12 * gx;
    const float* r1 = r0 + kPsvSrcRow;
    float3 a[5], c[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        a[j] = lds_rgb(r0 + 3 * j);
        c[j] = lds_rgb(r1 + 3 * j);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = bilerp(w00, w10, w01, w11, a[j], a[j + 1], c[j], c[j + 1]);
}

__device__ __forceinline__ void psv_sample_general(const float* __restrict__ im, const hsgd_warp& wp, int x, int y,
                                                   int H, int W, float3 (&v)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const Taps tp = make_taps(wp, x + j, y, H, W);
        const float* p00 = im + 3 * tp.i00;
        const float* p10 = im + 3 * tp.i10;
        const float* p01 = im + 3 * tp.i01;
        const float* p11 = im + 3 * tp.i11;
        v[j] = bilerp(tp.w00, tp.w10, tp.w01, tp.w11, make_float3(p00[0], p00[1], p00[2]),
                      make_float3(p10[0], p10[1], p10[2]), make_float3(p01[0], p01[1], p01[2]),
                      make_float3(p11[0], p11[1], p11[2]));
    }
}

// Level l of a plane's tile (TH x TW pixels at LDS offset OFF) to memory, then level l + 1
// reduced from it into LDS (2x2 means), recursively up to level L - 1.
template <int L, int l, int OFF, int OT>
__device__ __forceinline__ void psv_level(float* __restrict__ s_lv, const PsvOut& out, int iz, int tx, int ty,
                                          int H, int W, int vh0, int vw0, int t) {
    constexpr int TH = kPsvTH >> l, TW = kPsvTW >> l;
    __syncthreads();                                        // level l complete in LDS
    const int Hl = H >> l, Wl = W >> l;
    if (out.p[l]) {
        const size_t at = (((size_t)iz * Hl + ty * TH) * Wl + tx * TW) * 3;
        void* dst = OT == HSGD_FP32 ? (void*)(reinterpret_cast<float*>(out.p[l]) + at)
                                    : (void*)(reinterpret_cast<uint16_t*>(out.p[l]) + at);
        psv_store_tile<TH, TW, OT>(s_lv + OFF, vh0 >> l, vw0 >> l, dst, Wl, t);
    }
    if constexpr (l + 1 < L) {
        constexpr int NH = TH / 2, NW = TW / 2, DST = OFF + TH * TW * 3;
#pragma unroll
        for (int e0 = 0; e0 < NH * NW; e0 += 256) {
            const int e = e0 + t;
            if (NH * NW % 256 == 0 || e < NH * NW) {
                const int ey = e / NW, ex = e - ey * NW;
                const float* a = s_lv + OFF + ((2 * ey) * TW + 2 * ex) * 3;
                const float3 p0 = lds_rgb(a), p1 = lds_rgb(a + 3), p2 = lds_rgb(a + TW * 3), p3 = lds_rgb(a + TW * 3 + 3);
                float* d = s_lv + DST + e * 3;
                d[0] = ((p0.x + p1.x) + (p2.x + p3.x)) * 0.25f;
                d[1] = ((p0.y + p1.y) + (p2.y + p3.y)) * 0.25f;
                d[2] = ((p0.z + p1.z) + (p2.z + p3.z)) * 0.25f;
            }
        }
        psv_level<L, l + 1, DST, OT>(s_lv, out, iz, tx, ty, H, W, vh0, vw0, t);
    }
}

// One plane's tile from the threads' samples v to every level in memory: level l of the
// tile ((16 >> l) x (64 >> l) pixels) is packed after level l - 1 in s_lv.
template <int L, int OT>
__device__ __forceinline__ void psv_tile_levels(const float3 (&v)[4], float* __restrict__ s_lv,
                                                const PsvOut& out, int iz, int tx, int ty, int H, int W,
                                                int vh0, int vw0, int t) {
    {
        const int gx = t & 15, ly = t >> 4;
        float4* s4 = reinterpret_cast<float4*>(s_lv + (ly * kPsvTW + 4 * gx) * 3);
        s4[0] = make_float4(v[0].x, v[0].y, v[0].z, v[1].x);
        s4[1] = make_float4(v[1].y, v[1].z, v[2].x, v[2].y);
        s4[2] = make_float4(v[2].z, v[3].x, v[3].y, v[3].z);
    }
    psv_level<L, 0, 0, OT>(s_lv, out, iz, tx, ty, H, W, vh0, vw0, t);
}

// A workgroup takes one 64 x 16 reference tile of one (view, plane), 4 consecutive pixels
// of a row per thread. Blocks run tile column fastest, then plane, then tile row: the
// workgroups resident on an XCD write whole 16-row bands of a plane (long contiguous runs
// per image row) and sweep the planes of one band, whose source rows stay in its L2.
template <bool SHIFT, int L, int OT>
__global__ __launch_bounds__(256) void k_plane_sweep(const float* __restrict__ img,
                                                     const hsgd_warp* __restrict__ warps, int D, int H, int W,
                                                     PsvOut out, int ntx, int nty) {
    // levels 0.. of the tile, packed one after another: 3 * (1024 + 256 + 64 + 16 + 4)
    // floats; before them, the source patch of a translation map (3315 floats)
    __shared__ __align__(16) float s_lv[3 * (1024 + 256 + 64 + 16 + 4)];
    static_assert(kPsvSrcN <= 3 * (1024 + 256 + 64 + 16 + 4), "source patch exceeds the LDS tile");
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = b % ntx, r = b / ntx;
    const int z = r % D, r2 = r / D;
    const int ty = r2 % nty, i = r2 / nty;
    const int iz = i * D + z;
    const hsgd_warp& wp = warps[iz];
    const int t = threadIdx.x, gx = t & 15, ly = t >> 4;
    const float* im = img + (size_t)i * H * W * 3;
    float3 v[4];
    if (SHIFT) {
        psv_stage_patch(im, H, W, tx * kPsvTW + wp.ix, ty * kPsvTH + wp.iy, s_lv, t);
        __syncthreads();
        psv_blend_patch(wp, s_lv, gx, ly, v);
        __syncthreads();                                    // the patch is overwritten below
    } else {
        psv_sample_general(im, wp, tx * kPsvTW + 4 * gx, ty * kPsvTH + ly, H, W, v);
    }
    // valid part of the tile; H and W are multiples of 2^(L-1), so every coarse pixel of it
    // has its whole 2x2 block inside the image
    const int vh0 = min(kPsvTH, H - ty * kPsvTH), vw0 = min(kPsvTW, W - tx * kPsvTW);
    psv_tile_levels<L, OT>(v, s_lv, out, iz, tx, ty, H, W, vh0, vw0, t);
}

}  // namespace

int launch_plane_sweep(const hsgd_views& src, int D, int L, int out_dtype, void* const* out, hipStream_t s) {
    const int ntx = (int)ceil_div(src.W, kPsvTW), nty = (int)ceil_div(src.H, kPsvTH);
    const int64_t nb = (int64_t)ntx * nty * src.N * D;
    PsvOut o{};
    for (int l = 0; l < L; ++l) o.p[l] = out[l];
    ProfScope ps(HSGD_K_PSV, s);
    const bool shift = (src.flags & HSGD_VIEWS_SHIFT_ONLY) != 0;
#define HSGD_PSV_LAUNCH(SH, LV)                                                                               \
    if (out_dtype == HSGD_FP32)                                                                               \
        hipLaunchKernelGGL((k_plane_sweep<SH, LV, HSGD_FP32>), dim3((unsigned)nb), dim3(256), 0, s, src.images, \
                           src.warps, D, src.H, src.W, o, ntx, nty);                                          \
    else                                                                                                      \
        hipLaunchKernelGGL((k_plane_sweep<SH, LV, HSGD_BF16>), dim3((unsigned)nb), dim3(256), 0, s, src.images, \
                           src.warps, D, src.H, src.W, o, ntx, nty)
    switch (L * 2 + (shift ? 1 : 0)) {
        case 2: HSGD_PSV_LAUNCH(false, 1); break;
        case 3: HSGD_PSV_LAUNCH(true, 1); break;
        case 4: HSGD_PSV_LAUNCH(false, 2); break;
        case 5: HSGD_PSV_LAUNCH(true, 2); break;
        case 6: HSGD_PSV_LAUNCH(false, 3); break;
        case 7: HSGD_PSV_LAUNCH(true, 3); break;
        case 8: HSGD_PSV_LAUNCH(false, 4); break;
        case 9: HSGD_PSV_LAUNCH(true, 4); break;
        case 10: HSGD_PSV_LAUNCH(false, 5); break;
        default: HSGD_PSV_LAUNCH(true, 5); break;
    }
#undef HSGD_PSV_LAUNCH
    return (int)hipGetLastError();
}

}  // namespace hsgd
