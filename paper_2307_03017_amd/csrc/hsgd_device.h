// Device helpers shared by the kernel sources of libhsgd (gfx950, wave64). Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include "hsgd.h"

namespace hsgd {
namespace {

// FP32 -> BF16 bits, round to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// Raw (untyped, stride 0) buffer resource over one MPI row of n_bytes bytes: loads at
// offsets outside [0, n_bytes) return 0, which is the zero padding of a plane outside the
// image; n_bytes = 0 makes a whole row read as padding. Word 3 selects the 32-bit data
// format that untyped loads require on this architecture family.
constexpr int kBufWord3 = 4 << 15;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const char* row, int n_bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(row), (short)0, n_bytes, kBufWord3);
}

// ------------------------------------------------------------------------------------
// bilinear taps of one (view pixel, plane): zero padding, pixel-index coordinates
// ------------------------------------------------------------------------------------
struct Taps {
    int i00, i10, i01, i11;        // flat pixel index y*W + x (clamped; weight 0 if outside)
    float w00, w10, w01, w11;
};

__device__ __forceinline__ Taps make_taps(const hsgd_warp& wp, int x, int y, int H, int W) {
    int x0, y0;
    float fx, fy;
    bool front = true;
    if (wp.is_shift) {
        x0 = x + wp.ix;
        y0 = y + wp.iy;
        fx = wp.fx;
        fy = wp.fy;
    } else {
        // The position in FP64 from the FP64 map: its error (~1e-12 px) is far below the
        // FP32 rounding of the fractions, so the taps and weights are those of the exact
        // position, as for a translation.
        const double xd = (double)x, yd = (double)y;
        const double q0 = __builtin_fma(wp.G[0], xd, __builtin_fma(wp.G[1], yd, wp.G[2]));
        const double q1 = __builtin_fma(wp.G[3], xd, __builtin_fma(wp.G[4], yd, wp.G[5]));
        const double q2 = __builtin_fma(wp.G[6], xd, __builtin_fma(wp.G[7], yd, wp.G[8]));
        front = q2 > 0.0;
        double u = -8.0, v = -8.0;
        if (front) {
            const double r = 1.0 / q2;
            u = q0 * r;
            v = q1 * r;
        }
        u = fmin(fmax(u, -8.0), (double)W + 8.0);   // NaN -> -8 (outside)
        v = fmin(fmax(v, -8.0), (double)H + 8.0);
        const double fu = floor(u), fv = floor(v);
        x0 = (int)fu;
        y0 = (int)fv;
        fx = (float)(u - fu);
        fy = (float)(v - fv);
    }
    const bool bx0 = (unsigned)x0 < (unsigned)W, bx1 = (unsigned)(x0 + 1) < (unsigned)W;
    const bool by0 = (unsigned)y0 < (unsigned)H, by1 = (unsigned)(y0 + 1) < (unsigned)H;
    const int cx0 = min(max(x0, 0), W - 1), cx1 = min(max(x0 + 1, 0), W - 1);
    const int cy0 = min(max(y0, 0), H - 1), cy1 = min(max(y0 + 1, 0), H - 1);
    Taps t;
    t.i00 = cy0 * W + cx0;
    t.i10 = cy0 * W + cx1;
    t.i01 = cy1 * W + cx0;
    t.i11 = cy1 * W + cx1;
    const float gx = 1.0f - fx, gy = 1.0f - fy;
    t.w00 = (front && bx0 && by0) ? gx * gy : 0.0f;
    t.w10 = (front && bx1 && by0) ? fx * gy : 0.0f;
    t.w01 = (front && bx0 && by1) ? gx * fy : 0.0f;
    t.w11 = (front && bx1 && by1) ? fx * fy : 0.0f;
    return t;
}

// Block index -> tile index so that each XCD (workgroups are dealt round-robin to the 8
// XCDs) works on a contiguous run of tiles: the views of one tile and neighbouring tiles
// share MPI lines in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

}  // namespace
}  // namespace hsgd
