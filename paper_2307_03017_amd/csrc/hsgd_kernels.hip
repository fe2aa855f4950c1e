// HIP kernels of libhsgd for gfx950 (wave64).
//
//  k_select     scores A_z = a_z T_z of the un-warped MPI in exact FP32 order, top-k per
//               pixel -> uint64 plane mask; per-(plane, wave) ballot counts
//               (Sec. 3.3 Gradient Sparsification, Eq. gradient / Eq. overA)
//  k_scan_*     exclusive scan of those counts in plane-major order
//  k_compact    wavefront ballot/popcount compaction -> ascending linear ids (S)
//  k_render     warp + front-to-back over per view ray (Eq. render, Eq. over, Eq. homo)
//  k_grad       forward scan, residual, back-to-front adjoint scan, transposed bilinear
//               scatter restricted to S (Sec. 3.3; Eq. 4 gradient)
//  k_update     restore the sparse step onto S with clamp (the M_{n+1} update)
//  k_upsample   2x bilinear MPI upsampling between hierarchy levels
//  k_downsample 2x2 box mean of target images (the H/2^l pyramid, Sec. 3.2)
#include <hip/hip_runtime.h>

#include "hsgd_internal.h"

namespace hsgd {
namespace {

// ------------------------------------------------------------------------------------
// storage: FP32 float4 or BF16 (4 x 16 bit, round to nearest even on store)
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

template <int DT>
struct Vox;

template <>
struct Vox<HSGD_FP32> {
    static __device__ __forceinline__ float4 load(const void* base, int i) {
        return reinterpret_cast<const float4*>(base)[i];
    }
    static __device__ __forceinline__ float alpha(const void* base, int i) {
        return reinterpret_cast<const float*>(base)[4 * (size_t)i + 3];
    }
    static __device__ __forceinline__ void store(void* base, int i, float4 v) {
        reinterpret_cast<float4*>(base)[i] = v;
    }
};

template <>
struct Vox<HSGD_BF16> {
    static __device__ __forceinline__ float4 load(const void* base, int i) {
        uint2 r = reinterpret_cast<const uint2*>(base)[i];
        return make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u),
                           __uint_as_float(r.y << 16), __uint_as_float(r.y & 0xffff0000u));
    }
    static __device__ __forceinline__ float alpha(const void* base, int i) {
        return __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(base)[4 * (size_t)i + 3] << 16);
    }
    static __device__ __forceinline__ void store(void* base, int i, float4 v) {
        uint2 r;
        r.x = f32_to_bf16_bits(v.x) | (f32_to_bf16_bits(v.y) << 16);
        r.y = f32_to_bf16_bits(v.z) | (f32_to_bf16_bits(v.w) << 16);
        reinterpret_cast<uint2*>(base)[i] = r;
    }
};

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
        const float xf = (float)x, yf = (float)y;
        float q0 = wp.G[0] * xf + wp.G[1] * yf + wp.G[2];
        float q1 = wp.G[3] * xf + wp.G[4] * yf + wp.G[5];
        float q2 = wp.G[6] * xf + wp.G[7] * yf + wp.G[8];
        front = q2 > 0.0f;
        float u = front ? q0 / q2 : -8.0f;
        float v = front ? q1 / q2 : -8.0f;
        u = fminf(fmaxf(u, -8.0f), (float)W + 8.0f);   // NaN -> -8 (outside)
        v = fminf(fmaxf(v, -8.0f), (float)H + 8.0f);
        float fu = floorf(u), fv = floorf(v);
        x0 = (int)fu;
        y0 = (int)fv;
        fx = u - fu;
        fy = v - fv;
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

template <int DT>
__device__ __forceinline__ float4 sample(const void* mpi, int plane_base, const Taps& t) {
    const float4 a = Vox<DT>::load(mpi, plane_base + t.i00);
    const float4 b = Vox<DT>::load(mpi, plane_base + t.i10);
    const float4 c = Vox<DT>::load(mpi, plane_base + t.i01);
    const float4 d = Vox<DT>::load(mpi, plane_base + t.i11);
    float4 s;
    s.x = t.w00 * a.x + t.w10 * b.x + t.w01 * c.x + t.w11 * d.x;
    s.y = t.w00 * a.y + t.w10 * b.y + t.w01 * c.y + t.w11 * d.y;
    s.z = t.w00 * a.z + t.w10 * b.z + t.w01 * c.z + t.w11 * d.z;
    s.w = t.w00 * a.w + t.w10 * b.w + t.w01 * c.w + t.w11 * d.w;
    return s;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over a 256-thread block; the result is valid on thread 0.
__device__ __forceinline__ float block_sum(float v, float* sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    float r = 0.0f;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    return r;
}

__device__ __forceinline__ void load_warps(hsgd_warp* sw, const hsgd_warp* warps, int view, int D) {
    const int* src = reinterpret_cast<const int*>(warps + (size_t)view * D);
    int* dst = reinterpret_cast<int*>(sw);
    for (int i = threadIdx.x; i < D * 16; i += blockDim.x) dst[i] = src[i];
}

// ------------------------------------------------------------------------------------
// select
// ------------------------------------------------------------------------------------
template <int DT, int MAXD>
__global__ __launch_bounds__(256) void k_select(const void* __restrict__ mpi, int D, int HW,
                                                int k, float tau, uint64_t* __restrict__ mask,
                                                int* __restrict__ counts, int64_t nblk) {
#pragma clang fp contract(off)
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t sel = 0;
    if (p < HW) {
        float A[MAXD];
        float T = 1.0f;
#pragma unroll
        for (int z = 0; z < MAXD; ++z) {
            if (z < D) {
                const float a = Vox<DT>::alpha(mpi, z * HW + p);
                const float s = a * T;                  // A_z = fl(a_z * T_z)
                A[z] = (s == s) ? s : -INFINITY;        // NaN ranks last
                T = T * (1.0f - a);                     // T_{z+1} = fl(T_z * fl(1 - a_z))
            }
        }
        const int kk = min(k, D);
        if (kk == D) {
            sel = D == 64 ? ~0ull : ((1ull << D) - 1);
        } else if (2 * kk <= D) {
            // kk passes: best remaining score, the nearer plane on equal scores
            for (int j = 0; j < kk; ++j) {
                int best = -1;
                float bestA = 0.0f;
#pragma unroll
                for (int z = 0; z < MAXD; ++z)
                    if (z < D && !((sel >> z) & 1) && (best < 0 || A[z] > bestA)) {
                        best = z;
                        bestA = A[z];
                    }
                sel |= 1ull << best;
            }
        } else {
            // D - kk passes removing the worst: lowest score, the farther plane on ties
            uint64_t out = 0;
            for (int j = 0; j < D - kk; ++j) {
                int worst = -1;
                float worstA = 0.0f;
#pragma unroll
                for (int z = 0; z < MAXD; ++z)
                    if (z < D && !((out >> z) & 1) && (worst < 0 || A[z] <= worstA)) {
                        worst = z;
                        worstA = A[z];
                    }
                out |= 1ull << worst;
            }
            sel = (D == 64 ? ~0ull : ((1ull << D) - 1)) & ~out;
        }
        if (tau >= 0.0f) {
#pragma unroll
            for (int z = 0; z < MAXD; ++z)
                if (z < D && !(A[z] > tau)) sel &= ~(1ull << z);
        }
        mask[p] = sel;
    }
    if (counts) {
        const int64_t wblk = (int64_t)p >> 6;
        for (int z = 0; z < D; ++z) {
            const uint64_t bal = __ballot((sel >> z) & 1);
            if ((threadIdx.x & 63) == 0 && wblk < nblk) counts[z * nblk + wblk] = __popcll(bal);
        }
    }
}

// Segmented exclusive scan, phase 1: each block scans 4096 consecutive counts in place
// and writes its total.
constexpr int kSeg = kScanSeg;
__global__ __launch_bounds__(256) void k_scan_seg(int* __restrict__ v, int64_t n,
                                                  int* __restrict__ seg_total) {
    __shared__ int sv[kSeg];
    __shared__ int ssum[256];
    const int64_t base = (int64_t)blockIdx.x * kSeg;
    for (int i = threadIdx.x; i < kSeg; i += 256) sv[i] = base + i < n ? v[base + i] : 0;
    __syncthreads();
    int s = 0;
    for (int j = 0; j < 16; ++j) s += sv[threadIdx.x * 16 + j];
    ssum[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        int t = threadIdx.x >= o ? ssum[threadIdx.x - o] : 0;
        __syncthreads();
        ssum[threadIdx.x] += t;
        __syncthreads();
    }
    int run = ssum[threadIdx.x] - s;
    for (int j = 0; j < 16; ++j) {
        int c = sv[threadIdx.x * 16 + j];
        sv[threadIdx.x * 16 + j] = run;
        run += c;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSeg; i += 256)
        if (base + i < n) v[base + i] = sv[i];
    if (threadIdx.x == 255) seg_total[blockIdx.x] = ssum[255];
}

// Phase 2 (one block): exclusive scan of the segment totals, plane offsets, |S|.
__global__ __launch_bounds__(1024) void k_scan_top(const int* __restrict__ v, int64_t nblk, int D,
                                                   int* __restrict__ seg, int nseg,
                                                   int* __restrict__ plane_off,
                                                   int* __restrict__ n_active) {
    __shared__ int sh[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b = 0; b < nseg; b += 1024) {
        const int i = b + threadIdx.x;
        const int x = i < nseg ? seg[i] : 0;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nseg) seg[i] = carry + sh[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
    for (int z = threadIdx.x; z < D; z += 1024) {
        const int64_t e = (int64_t)z * nblk;
        plane_off[z] = v[e] + seg[e / kSeg];
    }
    if (threadIdx.x == 0) {
        plane_off[D] = carry;
        *n_active = carry;
    }
}

__global__ __launch_bounds__(256) void k_compact(const uint64_t* __restrict__ mask, int D, int HW,
                                                 const int* __restrict__ off,
                                                 const int* __restrict__ seg, int64_t nblk,
                                                 int* __restrict__ ids, int cap) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t bits = p < HW ? mask[p] : 0;
    const int64_t wblk = (int64_t)p >> 6;
    const uint64_t lt = __lanemask_lt();
    for (int z = 0; z < D; ++z) {
        const uint64_t bal = __ballot((bits >> z) & 1);
        if ((bits >> z) & 1) {
            const int64_t e = (int64_t)z * nblk + wblk;
            const int pos = off[e] + seg[e / kSeg] + __popcll(bal & lt);
            if (pos < cap) ids[pos] = z * HW + p;
        }
    }
}

// ------------------------------------------------------------------------------------
// render
// ------------------------------------------------------------------------------------
template <int DT>
__global__ __launch_bounds__(kBlock) void k_render(const void* __restrict__ mpi, int D, int H, int W,
                                                   const hsgd_warp* __restrict__ warps,
                                                   const float* __restrict__ images,
                                                   float* __restrict__ out_rgb,
                                                   float* __restrict__ partials) {
    __shared__ hsgd_warp sw[kMaxD];
    __shared__ float sred[kBlock / 64];
    const int view = blockIdx.z;
    load_warps(sw, warps, view, D);
    __syncthreads();
    const int x = blockIdx.x * kTileW + (threadIdx.x & 63);
    const int y = blockIdx.y * kTileH + (threadIdx.x >> 6);
    const int HW = H * W;
    float sq = 0.0f;
    if (x < W && y < H) {
        float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
        for (int z = 0; z < D; ++z) {
            const Taps tp = make_taps(sw[z], x, y, H, W);
            const float4 s = sample<DT>(mpi, z * HW, tp);
            const float wgt = T * s.w;
            c0 += wgt * s.x;
            c1 += wgt * s.y;
            c2 += wgt * s.z;
            T *= 1.0f - s.w;
        }
        const size_t pix = ((size_t)view * H + y) * W + x;
        if (out_rgb) {
            out_rgb[3 * pix + 0] = c0;
            out_rgb[3 * pix + 1] = c1;
            out_rgb[3 * pix + 2] = c2;
        }
        if (partials) {
            const float d0 = c0 - images[3 * pix + 0];
            const float d1 = c1 - images[3 * pix + 1];
            const float d2 = c2 - images[3 * pix + 2];
            sq = d0 * d0 + d1 * d1 + d2 * d2;
        }
    }
    if (partials) {
        const float tot = block_sum(sq, sred);
        if (threadIdx.x == 0)
            partials[((size_t)view * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
    }
}

// Deterministic final reduction of per-block partials (FP64 accumulation).
__global__ __launch_bounds__(256) void k_reduce(const float* __restrict__ partials, int64_t n,
                                                double scale, float* __restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)partials[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (float)(sh[0] * scale);
}

// ------------------------------------------------------------------------------------
// gradient: forward scan, residual, back-to-front adjoint scan, restricted scatter
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void scatter_tap(float4* __restrict__ slots, const uint64_t* __restrict__ mask,
                                            int kcap, int HW, uint64_t full, int z, int p, float w,
                                            const float4& g) {
    if (w == 0.0f) return;
    const uint64_t m = mask ? mask[p] : full;
    if (!((m >> z) & 1)) return;
    const int r = __popcll(m & ((1ull << z) - 1));
    if (r >= kcap) return;
    float* dst = reinterpret_cast<float*>(slots + (size_t)r * HW + p);
    atomicAdd(dst + 0, w * g.x);
    atomicAdd(dst + 1, w * g.y);
    atomicAdd(dst + 2, w * g.z);
    atomicAdd(dst + 3, w * g.w);
}

template <int DT, int MAXD>
__global__ __launch_bounds__(kBlock) void k_grad(const void* __restrict__ mpi, int D, int H, int W,
                                                 const hsgd_warp* __restrict__ warps,
                                                 const float* __restrict__ images,
                                                 const float* __restrict__ dimg,
                                                 const uint64_t* __restrict__ mask, int kcap,
                                                 float inv_n, float4* __restrict__ slots,
                                                 float* __restrict__ partials) {
    __shared__ hsgd_warp sw[MAXD];
    __shared__ float sred[kBlock / 64];
    const int view = blockIdx.z;
    load_warps(sw, warps, view, D);
    __syncthreads();
    const int x = blockIdx.x * kTileW + (threadIdx.x & 63);
    const int y = blockIdx.y * kTileH + (threadIdx.x >> 6);
    const int HW = H * W;
    const uint64_t full = D == 64 ? ~0ull : ((1ull << D) - 1);
    float sq = 0.0f;
    if (x < W && y < H) {
        float Ts[MAXD];
        float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
        for (int z = 0; z < MAXD; ++z) {
            if (z < D) {
                const Taps tp = make_taps(sw[z], x, y, H, W);
                const float4 s = sample<DT>(mpi, z * HW, tp);
                Ts[z] = T;
                const float wgt = T * s.w;
                c0 += wgt * s.x;
                c1 += wgt * s.y;
                c2 += wgt * s.z;
                T *= 1.0f - s.w;
            }
        }
        const size_t pix = ((size_t)view * H + y) * W + x;
        float g0, g1, g2;
        if (images) {
            const float d0 = c0 - images[3 * pix + 0];
            const float d1 = c1 - images[3 * pix + 1];
            const float d2 = c2 - images[3 * pix + 2];
            sq = d0 * d0 + d1 * d1 + d2 * d2;
            g0 = d0 * inv_n;
            g1 = d1 * inv_n;
            g2 = d2 * inv_n;
        }
        if (dimg) {
            g0 = dimg[3 * pix + 0];
            g1 = dimg[3 * pix + 1];
            g2 = dimg[3 * pix + 2];
        }
        float b0 = 0.0f, b1 = 0.0f, b2 = 0.0f;   // composite behind plane z
#pragma unroll
        for (int zz = 0; zz < MAXD; ++zz) {
            const int z = MAXD - 1 - zz;
            if (z < D) {
                const Taps tp = make_taps(sw[z], x, y, H, W);
                const float4 s = sample<DT>(mpi, z * HW, tp);
                const float Tz = Ts[z];
                const float ca = s.w * Tz;
                float4 gs;
                gs.x = g0 * ca;
                gs.y = g1 * ca;
                gs.z = g2 * ca;
                gs.w = Tz * (g0 * (s.x - b0) + g1 * (s.y - b1) + g2 * (s.z - b2));
                const float oa = 1.0f - s.w;
                b0 = s.w * s.x + oa * b0;
                b1 = s.w * s.y + oa * b1;
                b2 = s.w * s.z + oa * b2;
                scatter_tap(slots, mask, kcap, HW, full, z, tp.i00, tp.w00, gs);
                scatter_tap(slots, mask, kcap, HW, full, z, tp.i10, tp.w10, gs);
                scatter_tap(slots, mask, kcap, HW, full, z, tp.i01, tp.w01, gs);
                scatter_tap(slots, mask, kcap, HW, full, z, tp.i11, tp.w11, gs);
            }
        }
    }
    if (partials) {
        const float tot = block_sum(sq, sred);
        if (threadIdx.x == 0)
            partials[((size_t)view * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
    }
}

// ------------------------------------------------------------------------------------
// gradient for pure-translation warps: owner-computes, no atomics, deterministic
//
// A workgroup takes a 64 x 8 block of view rays: 63 x 7 "owner" rays plus one halo column
// on the left and one halo row on top. For plane z every owner (x, y) also owns the
// reference cell (x + ix_z, y + iy_z): with a translation the four rays whose bilinear
// footprint covers that cell are the owner and its left, upper and upper-left neighbours,
// all in the block. The per-ray adjoints are combined horizontally across lanes with DPP
// and vertically across waves through LDS, and each owner writes its cell's gradient once
// into the view's slice of the slot buffer (rank-major [view][kcap][H*W]).
// ------------------------------------------------------------------------------------
constexpr int kSX = kShiftOX + 1, kSY = kShiftOY + 1;  // rays per block (with halo)
constexpr int kOX = kShiftOX, kOY = kShiftOY;          // owner rays (= owned cells) per block and plane
static_assert(kSX == 64, "one wave per row of rays");

__device__ __forceinline__ float lane_from_next(float v) {   // lane i <- lane i+1 (63 <- 0)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_from_prev(float v) {   // lane i <- lane i-1 (0 <- 0)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float4 lane_from_next4(float4 v) {
    return make_float4(lane_from_next(v.x), lane_from_next(v.y), lane_from_next(v.z), lane_from_next(v.w));
}
__device__ __forceinline__ float4 lane_from_prev4(float4 v) {
    return make_float4(lane_from_prev(v.x), lane_from_prev(v.y), lane_from_prev(v.z), lane_from_prev(v.w));
}

// Block index -> tile index so that each XCD (blocks are dealt round-robin to the 8 XCDs)
// works on a contiguous run of tiles: neighbouring tiles and the views of one tile share
// MPI lines in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

struct ShiftRec {
    int ix, iy;
    float fx, fy;
};

// Sample plane z at the ray (x, y) of this lane for a shift warp. All 64 lanes must call it
// together (the right-hand taps come from the next lane through DPP).
template <int DT>
__device__ __forceinline__ float4 shift_sample(const void* __restrict__ mpi, int zbase, int H, int W,
                                               int x, int y, const ShiftRec& sh, int lane) {
    const int X0 = x + sh.ix, Y0 = y + sh.iy;
    const bool y0ok = (unsigned)Y0 < (unsigned)H, y1ok = (unsigned)(Y0 + 1) < (unsigned)H;
    const bool x0ok = (unsigned)X0 < (unsigned)W, x1ok = (unsigned)(X0 + 1) < (unsigned)W;
    const int cx0 = min(max(X0, 0), W - 1);
    const int r0 = zbase + min(max(Y0, 0), H - 1) * W;
    const int r1 = zbase + min(max(Y0 + 1, 0), H - 1) * W;
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 t00 = (y0ok && x0ok) ? Vox<DT>::load(mpi, r0 + cx0) : zero;
    float4 t01 = (y1ok && x0ok) ? Vox<DT>::load(mpi, r1 + cx0) : zero;
    float4 t10 = lane_from_next4(t00);
    float4 t11 = lane_from_next4(t01);
    if (lane == kSX - 1) {
        const int cx1 = min(max(X0 + 1, 0), W - 1);
        t10 = (y0ok && x1ok) ? Vox<DT>::load(mpi, r0 + cx1) : zero;
        t11 = (y1ok && x1ok) ? Vox<DT>::load(mpi, r1 + cx1) : zero;
    }
    const float gx = 1.0f - sh.fx, gy = 1.0f - sh.fy;
    float4 s;
    s.x = (t00.x * gx + t10.x * sh.fx) * gy + (t01.x * gx + t11.x * sh.fx) * sh.fy;
    s.y = (t00.y * gx + t10.y * sh.fx) * gy + (t01.y * gx + t11.y * sh.fx) * sh.fy;
    s.z = (t00.z * gx + t10.z * sh.fx) * gy + (t01.z * gx + t11.z * sh.fx) * sh.fy;
    s.w = (t00.w * gx + t10.w * sh.fx) * gy + (t01.w * gx + t11.w * sh.fx) * sh.fy;
    return s;
}

// REGS: keep every plane's sample in registers between the two scans (D <= 32); otherwise
// sample again in the back-to-front scan.
template <int DT, int MAXD, bool REGS>
__global__ __launch_bounds__(kSX * kSY) void k_grad_shift(
    const void* __restrict__ mpi, int D, int H, int W, int N, const hsgd_warp* __restrict__ warps,
    const float* __restrict__ images, const float* __restrict__ dimg, const uint64_t* __restrict__ mask,
    int kcap, float inv_n, float4* __restrict__ slots, float* __restrict__ partials, int ntx, int nty) {
    __shared__ ShiftRec s_sh[MAXD];
    __shared__ float4 s_h[2][kSX * kSY];
    __shared__ float sred[kSX * kSY / 64];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int view = tile % N;
    const int t2 = tile / N;
    const int tx = t2 % ntx, ty = t2 / ntx;
    for (int z = threadIdx.x; z < D; z += blockDim.x) {
        const hsgd_warp& w = warps[(size_t)view * D + z];
        s_sh[z] = ShiftRec{w.ix, w.iy, w.fx, w.fy};
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x = tx * kOX - 1 + lane, y = ty * kOY - 1 + wv;
    const bool valid = (unsigned)x < (unsigned)W && (unsigned)y < (unsigned)H;
    const bool owner = lane >= 1 && wv >= 1;
    const int HW = H * W;
    const uint64_t full = D == 64 ? ~0ull : ((1ull << D) - 1);

    float4 smp[REGS ? MAXD : 1];
    float Ts[MAXD];
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
    for (int z = 0; z < MAXD; ++z) {
        if (z < D) {
            const float4 s = shift_sample<DT>(mpi, z * HW, H, W, x, y, s_sh[z], lane);
            if (REGS) smp[z] = s;
            Ts[z] = T;
            const float wgt = T * s.w;
            c0 += wgt * s.x;
            c1 += wgt * s.y;
            c2 += wgt * s.z;
            T *= 1.0f - s.w;
        }
    }
    float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, sq = 0.0f;
    if (valid) {
        const size_t pix = ((size_t)view * H + y) * W + x;
        if (images) {
            const float d0 = c0 - images[3 * pix + 0];
            const float d1 = c1 - images[3 * pix + 1];
            const float d2 = c2 - images[3 * pix + 2];
            if (owner) sq = d0 * d0 + d1 * d1 + d2 * d2;
            g0 = d0 * inv_n;
            g1 = d1 * inv_n;
            g2 = d2 * inv_n;
        }
        if (dimg) {
            g0 = dimg[3 * pix + 0];
            g1 = dimg[3 * pix + 1];
            g2 = dimg[3 * pix + 2];
        }
    }
    float b0 = 0.0f, b1 = 0.0f, b2 = 0.0f;   // composite behind plane z
    float4* vslots = slots + (size_t)view * kcap * HW;
#pragma unroll
    for (int zz = 0; zz < MAXD; ++zz) {
        const int z = MAXD - 1 - zz;
        if (z < D) {
            const ShiftRec sh = s_sh[z];
            const float4 s = REGS ? smp[REGS ? z : 0] : shift_sample<DT>(mpi, z * HW, H, W, x, y, sh, lane);
            const float Tz = Ts[z];
            const float ca = s.w * Tz;
            float4 a;
            a.x = g0 * ca;
            a.y = g1 * ca;
            a.z = g2 * ca;
            a.w = Tz * (g0 * (s.x - b0) + g1 * (s.y - b1) + g2 * (s.z - b2));
            const float oa = 1.0f - s.w;
            b0 = s.w * s.x + oa * b0;
            b1 = s.w * s.y + oa * b1;
            b2 = s.w * s.z + oa * b2;
            // horizontal half of the transposed bilinear: this ray (weight 1 - fx) and the
            // ray to its left (weight fx) both touch the owned cell's row
            const float4 ap = lane_from_prev4(a);
            const float gx = 1.0f - sh.fx;
            float4 h;
            h.x = a.x * gx + ap.x * sh.fx;
            h.y = a.y * gx + ap.y * sh.fx;
            h.z = a.z * gx + ap.z * sh.fx;
            h.w = a.w * gx + ap.w * sh.fx;
            float4* buf = s_h[z & 1];
            buf[threadIdx.x] = h;
            __syncthreads();
            if (owner) {
                const int X = x + sh.ix, Y = y + sh.iy;
                if ((unsigned)X < (unsigned)W && (unsigned)Y < (unsigned)H) {
                    const int p = Y * W + X;
                    const uint64_t m = mask ? mask[p] : full;
                    if ((m >> z) & 1) {
                        const int r = __popcll(m & ((1ull << z) - 1));
                        if (r < kcap) {
                            const float4 hu = buf[threadIdx.x - 64];   // the row above
                            const float gy = 1.0f - sh.fy;
                            float4 c;
                            c.x = h.x * gy + hu.x * sh.fy;
                            c.y = h.y * gy + hu.y * sh.fy;
                            c.z = h.z * gy + hu.z * sh.fy;
                            c.w = h.w * gy + hu.w * sh.fy;
                            vslots[(size_t)r * HW + p] = c;
                        }
                    }
                }
            }
        }
    }
    if (partials) {
        const float tot = block_sum(sq, sred);
        if (threadIdx.x == 0) partials[tile] = tot;
    }
}

__global__ __launch_bounds__(256) void k_fill_zero(float4* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = i; j < n; j += stride) p[j] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Sum the per-view gradient slices of every selected voxel, then apply the clamped descent
// step in place and/or write the dense-masked gradient. With shift warps, a view's slice
// holds a voxel only if the voxel lies in that view's owner coverage; outside it the view
// contributes nothing (no ray of the view reaches the voxel) and the slot is not read.
template <int DT, bool SHIFT>
__global__ __launch_bounds__(256) void k_update(void* __restrict__ mpi, int D, int H, int W,
                                                const uint64_t* __restrict__ mask, int kcap,
                                                const float4* __restrict__ slots, int nslices,
                                                const hsgd_warp* __restrict__ warps, int cover_w,
                                                int cover_h, float lr_rgb, float lr_a, int do_update,
                                                float4* __restrict__ grad_out) {
    extern __shared__ int2 s_off[];   // [nslices][D] (ix, iy) when SHIFT
    if (SHIFT) {
        for (int i = threadIdx.x; i < nslices * D; i += blockDim.x) s_off[i] = make_int2(warps[i].ix, warps[i].iy);
        __syncthreads();
    }
    const int HW = H * W;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= HW) return;
    const int X = p % W, Y = p / W;
    const uint64_t full = D == 64 ? ~0ull : ((1ull << D) - 1);
    const uint64_t m = mask ? mask[p] : full;
    auto grad_of = [&](int z, int r) {
        float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int v = 0; v < nslices; ++v) {
            if (SHIFT) {
                const int2 o = s_off[v * D + z];
                const int cx = X - o.x, cy = Y - o.y;
                if ((unsigned)cx >= (unsigned)cover_w || (unsigned)cy >= (unsigned)cover_h) continue;
            }
            const float4 t = slots[((size_t)v * kcap + r) * HW + p];
            g.x += t.x;
            g.y += t.y;
            g.z += t.z;
            g.w += t.w;
        }
        return g;
    };
    if (grad_out) {
        int r = 0;
        for (int z = 0; z < D; ++z) {
            float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
            if ((m >> z) & 1) {
                if (r < kcap) g = grad_of(z, r);
                ++r;
            }
            grad_out[(size_t)z * HW + p] = g;
        }
    }
    if (do_update) {
        uint64_t b = m;
        int r = 0;
        while (b && r < kcap) {
            const int z = __ffsll((unsigned long long)b) - 1;
            b &= b - 1;
            const float4 g = grad_of(z, r++);
            float4 v = Vox<DT>::load(mpi, z * HW + p);
            v.x = fminf(fmaxf(v.x - lr_rgb * g.x, 0.0f), 1.0f);
            v.y = fminf(fmaxf(v.y - lr_rgb * g.y, 0.0f), 1.0f);
            v.z = fminf(fmaxf(v.z - lr_rgb * g.z, 0.0f), 1.0f);
            v.w = fminf(fmaxf(v.w - lr_a * g.w, 0.0f), 1.0f);
            Vox<DT>::store(mpi, z * HW + p, v);
        }
    }
}

// ------------------------------------------------------------------------------------
// hierarchy
// ------------------------------------------------------------------------------------
template <int DT>
__global__ __launch_bounds__(256) void k_upsample(const void* __restrict__ src, int h, int w,
                                                  void* __restrict__ dst) {
    const int W2 = 2 * w, H2 = 2 * h;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.y;
    if (i >= W2 * H2) return;
    const int x = i % W2, y = i / W2;
    const float sx = fminf(fmaxf((x + 0.5f) * 0.5f - 0.5f, 0.0f), (float)(w - 1));
    const float sy = fminf(fmaxf((y + 0.5f) * 0.5f - 0.5f, 0.0f), (float)(h - 1));
    const int x0 = (int)sx, y0 = (int)sy;
    const int x1 = min(x0 + 1, w - 1), y1 = min(y0 + 1, h - 1);
    const float fx = sx - x0, fy = sy - y0;
    const int base = z * h * w;
    const float4 a = Vox<DT>::load(src, base + y0 * w + x0);
    const float4 b = Vox<DT>::load(src, base + y0 * w + x1);
    const float4 c = Vox<DT>::load(src, base + y1 * w + x0);
    const float4 d = Vox<DT>::load(src, base + y1 * w + x1);
    const float w00 = (1 - fx) * (1 - fy), w10 = fx * (1 - fy), w01 = (1 - fx) * fy, w11 = fx * fy;
    float4 o;
    o.x = w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x;
    o.y = w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y;
    o.z = w00 * a.z + w10 * b.z + w01 * c.z + w11 * d.z;
    o.w = w00 * a.w + w10 * b.w + w01 * c.w + w11 * d.w;
    Vox<DT>::store(dst, z * H2 * W2 + i, o);
}

__global__ __launch_bounds__(256) void k_downsample(const float* __restrict__ img, int H, int W,
                                                    float* __restrict__ out) {
    const int h = H / 2, w = W / 2;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y;
    if (i >= h * w) return;
    const int x = i % w, y = i / w;
    const float* s = img + ((size_t)n * H + 2 * y) * W * 3 + 6 * x;
    float* o = out + ((size_t)n * h * w + i) * 3;
    for (int c = 0; c < 3; ++c)
        o[c] = ((s[c] + s[3 + c]) + (s[3 * W + c] + s[3 * W + 3 + c])) * 0.25f;
}

template <int SDT, int DDT>
__global__ __launch_bounds__(256) void k_convert(const void* __restrict__ src, void* __restrict__ dst,
                                                 int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v;
    if (SDT == HSGD_FP32) v = reinterpret_cast<const float*>(src)[i];
    else v = __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(src)[i] << 16);
    if (DDT == HSGD_FP32) reinterpret_cast<float*>(dst)[i] = v;
    else reinterpret_cast<uint16_t*>(dst)[i] = (uint16_t)f32_to_bf16_bits(v);
}

int maxd_class(int D) { return D <= 8 ? 8 : D <= 16 ? 16 : D <= 32 ? 32 : 64; }

#define HSGD_DISPATCH_D(D, BODY)                 \
    switch (maxd_class(D)) {                     \
        case 8: { constexpr int MD = 8; BODY; } break;   \
        case 16: { constexpr int MD = 16; BODY; } break; \
        case 32: { constexpr int MD = 32; BODY; } break; \
        default: { constexpr int MD = 64; BODY; } break; \
    }

#define HSGD_DISPATCH_T(dt, BODY)                                            \
    if ((dt) == HSGD_FP32) { constexpr int DT = HSGD_FP32; BODY; }            \
    else { constexpr int DT = HSGD_BF16; BODY; }

}  // namespace

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
int launch_select(const hsgd_mpi& m, int k, float tau, uint64_t* mask, int32_t* ids, int cap,
                  int32_t* plane_off, int32_t* n_active, void* ws, hipStream_t s) {
    const int HW = m.H * m.W;
    const SelectWs L = select_ws(m.D, m.H, m.W);
    int* counts = ids ? reinterpret_cast<int*>((char*)ws + L.counts_off) : nullptr;
    const dim3 grid((unsigned)ceil_div(HW, 256));
    {
        ProfScope ps(HSGD_K_SELECT, s);
        HSGD_DISPATCH_T(m.dtype, HSGD_DISPATCH_D(m.D, hipLaunchKernelGGL((k_select<DT, MD>), grid, dim3(256), 0, s,
                                                                        m.rgba, m.D, HW, k, tau, mask, counts, L.nblk)));
    }
    if (ids) {
        const int64_t n = (int64_t)m.D * L.nblk;
        const int nseg = (int)L.nseg;
        int* seg = reinterpret_cast<int*>((char*)ws + L.seg_off);
        {
            ProfScope ps(HSGD_K_SCAN, s);
            hipLaunchKernelGGL(k_scan_seg, dim3(nseg), dim3(256), 0, s, counts, n, seg);
            hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, counts, L.nblk, m.D, seg, nseg,
                               plane_off, n_active);
        }
        ProfScope ps(HSGD_K_COMPACT, s);
        hipLaunchKernelGGL(k_compact, grid, dim3(256), 0, s, mask, m.D, HW, counts, seg, L.nblk, ids, cap);
    }
    return (int)hipGetLastError();
}

int launch_render(const hsgd_mpi& m, const hsgd_views& v, float* out_rgb, float* out_loss,
                  void* ws, hipStream_t s) {
    const RenderWs L = render_ws(m.H, m.W, v.N);
    float* partials = out_loss ? reinterpret_cast<float*>((char*)ws + L.partial_off) : nullptr;
    const dim3 grid((unsigned)ceil_div(m.W, kTileW), (unsigned)ceil_div(m.H, kTileH), (unsigned)v.N);
    {
        ProfScope ps(HSGD_K_RENDER, s);
        HSGD_DISPATCH_T(m.dtype, hipLaunchKernelGGL((k_render<DT>), grid, dim3(kBlock), 0, s, m.rgba, m.D,
                                                    m.H, m.W, v.warps, v.images, out_rgb, partials));
    }
    if (out_loss) {
        ProfScope ps(HSGD_K_REDUCE, s);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, L.nparts, 0.5 / v.N, out_loss);
    }
    return (int)hipGetLastError();
}

int launch_grad_step(const hsgd_mpi& m, const hsgd_views& v, const uint64_t* mask, int kcap,
                     const float* dimg, float lr_rgb, float lr_alpha, float* grad_out,
                     float* out_loss, void* ws, hipStream_t s) {
    const int HW = m.H * m.W;
    const GradWs L = grad_ws(m.D, m.H, m.W, v.N, kcap);
    float4* slots = reinterpret_cast<float4*>((char*)ws + L.slots_off);
    float* partials = reinterpret_cast<float*>((char*)ws + L.partial_off);
    const float inv_n = 1.0f / (float)v.N;
    const bool shift = (v.flags & HSGD_VIEWS_SHIFT_ONLY) != 0;
    int64_t nparts;
    int cover_w = 0, cover_h = 0;
    if (shift) {
        const int ntx = (int)ceil_div(m.W + 1, kOX), nty = (int)ceil_div(m.H + 1, kOY);
        cover_w = ntx * kOX;
        cover_h = nty * kOY;
        nparts = (int64_t)ntx * nty * v.N;
        const dim3 grid((unsigned)nparts);
        ProfScope ps(HSGD_K_GRAD, s);
        HSGD_DISPATCH_T(m.dtype, switch (maxd_class(m.D)) {
            case 8: hipLaunchKernelGGL((k_grad_shift<DT, 8, true>), grid, dim3(kSX * kSY), 0, s, m.rgba, m.D, m.H, m.W,
                                       v.N, v.warps, v.images, dimg, mask, kcap, inv_n, slots,
                                       out_loss ? partials : nullptr, ntx, nty); break;
            case 16: hipLaunchKernelGGL((k_grad_shift<DT, 16, true>), grid, dim3(kSX * kSY), 0, s, m.rgba, m.D, m.H, m.W,
                                        v.N, v.warps, v.images, dimg, mask, kcap, inv_n, slots,
                                        out_loss ? partials : nullptr, ntx, nty); break;
            case 32: hipLaunchKernelGGL((k_grad_shift<DT, 32, true>), grid, dim3(kSX * kSY), 0, s, m.rgba, m.D, m.H, m.W,
                                        v.N, v.warps, v.images, dimg, mask, kcap, inv_n, slots,
                                        out_loss ? partials : nullptr, ntx, nty); break;
            default: hipLaunchKernelGGL((k_grad_shift<DT, 64, false>), grid, dim3(kSX * kSY), 0, s, m.rgba, m.D, m.H, m.W,
                                        v.N, v.warps, v.images, dimg, mask, kcap, inv_n, slots,
                                        out_loss ? partials : nullptr, ntx, nty); break;
        });
    } else {
        const int64_t nslots = (int64_t)kcap * HW;
        const int fill_blocks = (int)std::min<int64_t>(ceil_div(nslots, 256), 4096);
        {
            ProfScope ps(HSGD_K_FILL, s);
            hipLaunchKernelGGL(k_fill_zero, dim3(fill_blocks), dim3(256), 0, s, slots, nslots);
        }
        const dim3 grid((unsigned)ceil_div(m.W, kTileW), (unsigned)ceil_div(m.H, kTileH), (unsigned)v.N);
        nparts = (int64_t)grid.x * grid.y * grid.z;
        ProfScope ps(HSGD_K_GRAD, s);
        HSGD_DISPATCH_T(m.dtype, HSGD_DISPATCH_D(m.D, hipLaunchKernelGGL((k_grad<DT, MD>), grid, dim3(kBlock), 0, s,
                                                                        m.rgba, m.D, m.H, m.W, v.warps, v.images, dimg,
                                                                        mask, kcap, inv_n, slots,
                                                                        out_loss ? partials : nullptr)));
    }
    const int do_update = (lr_rgb != 0.0f || lr_alpha != 0.0f) ? 1 : 0;
    {
        ProfScope ps(HSGD_K_UPDATE, s);
        const dim3 grid((unsigned)ceil_div(HW, 256));
        if (shift) {
            const size_t lds = sizeof(int2) * (size_t)v.N * m.D;
            HSGD_DISPATCH_T(m.dtype, hipLaunchKernelGGL((k_update<DT, true>), grid, dim3(256), lds, s, m.rgba, m.D, m.H,
                                                        m.W, mask, kcap, slots, v.N, v.warps, cover_w, cover_h, lr_rgb,
                                                        lr_alpha, do_update, reinterpret_cast<float4*>(grad_out)));
        } else {
            HSGD_DISPATCH_T(m.dtype, hipLaunchKernelGGL((k_update<DT, false>), grid, dim3(256), 0, s, m.rgba, m.D, m.H,
                                                        m.W, mask, kcap, slots, 1, v.warps, 0, 0, lr_rgb, lr_alpha,
                                                        do_update, reinterpret_cast<float4*>(grad_out)));
        }
    }
    if (out_loss) {
        ProfScope ps(HSGD_K_REDUCE, s);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, nparts, 0.5 / v.N, out_loss);
    }
    return (int)hipGetLastError();
}

int launch_upsample(const hsgd_mpi& c, const hsgd_mpi& f, hipStream_t s) {
    const dim3 grid((unsigned)ceil_div((int64_t)f.H * f.W, 256), (unsigned)c.D);
    ProfScope ps(HSGD_K_UPSAMPLE, s);
    HSGD_DISPATCH_T(c.dtype, hipLaunchKernelGGL((k_upsample<DT>), grid, dim3(256), 0, s, c.rgba, c.H, c.W, f.rgba));
    return (int)hipGetLastError();
}

int launch_downsample(const float* img, int N, int H, int W, float* out, hipStream_t s) {
    const dim3 grid((unsigned)ceil_div((int64_t)(H / 2) * (W / 2), 256), (unsigned)N);
    ProfScope ps(HSGD_K_DOWNSAMPLE, s);
    hipLaunchKernelGGL(k_downsample, grid, dim3(256), 0, s, img, H, W, out);
    return (int)hipGetLastError();
}

int launch_convert(const void* src, int sdt, void* dst, int ddt, size_t n, hipStream_t s) {
    const dim3 grid((unsigned)ceil_div((int64_t)n, 256));
    ProfScope ps(HSGD_K_CONVERT, s);
    if (sdt == HSGD_FP32 && ddt == HSGD_FP32)
        hipLaunchKernelGGL((k_convert<HSGD_FP32, HSGD_FP32>), grid, dim3(256), 0, s, src, dst, (int64_t)n);
    else if (sdt == HSGD_FP32)
        hipLaunchKernelGGL((k_convert<HSGD_FP32, HSGD_BF16>), grid, dim3(256), 0, s, src, dst, (int64_t)n);
    else if (ddt == HSGD_FP32)
        hipLaunchKernelGGL((k_convert<HSGD_BF16, HSGD_FP32>), grid, dim3(256), 0, s, src, dst, (int64_t)n);
    else
        hipLaunchKernelGGL((k_convert<HSGD_BF16, HSGD_BF16>), grid, dim3(256), 0, s, src, dst, (int64_t)n);
    return (int)hipGetLastError();
}

}  // namespace hsgd
