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
                                            int kcap, uint64_t full, int z, int p, float w,
                                            const float4& g) {
    if (w == 0.0f) return;
    const uint64_t m = mask ? mask[p] : full;
    if (!((m >> z) & 1)) return;
    const int r = __popcll(m & ((1ull << z) - 1));
    if (r >= kcap) return;
    float* dst = reinterpret_cast<float*>(slots + (size_t)p * kcap + r);
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
                scatter_tap(slots, mask, kcap, full, z, tp.i00, tp.w00, gs);
                scatter_tap(slots, mask, kcap, full, z, tp.i10, tp.w10, gs);
                scatter_tap(slots, mask, kcap, full, z, tp.i01, tp.w01, gs);
                scatter_tap(slots, mask, kcap, full, z, tp.i11, tp.w11, gs);
            }
        }
    }
    if (partials) {
        const float tot = block_sum(sq, sred);
        if (threadIdx.x == 0)
            partials[((size_t)view * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
    }
}

__global__ __launch_bounds__(256) void k_fill_zero(float4* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = i; j < n; j += stride) p[j] = make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int DT>
__global__ __launch_bounds__(256) void k_update(void* __restrict__ mpi, int D, int HW,
                                                const uint64_t* __restrict__ mask, int kcap,
                                                const float4* __restrict__ slots, float lr_rgb,
                                                float lr_a, int do_update,
                                                float4* __restrict__ grad_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= HW) return;
    const uint64_t full = D == 64 ? ~0ull : ((1ull << D) - 1);
    const uint64_t m = mask ? mask[p] : full;
    const float4* sp = slots + (size_t)p * kcap;
    if (grad_out) {
        int r = 0;
        for (int z = 0; z < D; ++z) {
            float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
            if ((m >> z) & 1) {
                if (r < kcap) g = sp[r];
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
            const float4 g = sp[r++];
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
    HSGD_DISPATCH_T(m.dtype, HSGD_DISPATCH_D(m.D, hipLaunchKernelGGL((k_select<DT, MD>), grid, dim3(256), 0, s,
                                                                    m.rgba, m.D, HW, k, tau, mask, counts, L.nblk)));
    if (ids) {
        const int64_t n = (int64_t)m.D * L.nblk;
        const int nseg = (int)L.nseg;
        int* seg = reinterpret_cast<int*>((char*)ws + L.seg_off);
        hipLaunchKernelGGL(k_scan_seg, dim3(nseg), dim3(256), 0, s, counts, n, seg);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, counts, L.nblk, m.D, seg, nseg,
                           plane_off, n_active);
        hipLaunchKernelGGL(k_compact, grid, dim3(256), 0, s, mask, m.D, HW, counts, seg, L.nblk, ids, cap);
    }
    return (int)hipGetLastError();
}

int launch_render(const hsgd_mpi& m, const hsgd_views& v, float* out_rgb, float* out_loss,
                  void* ws, hipStream_t s) {
    const RenderWs L = render_ws(m.H, m.W, v.N);
    float* partials = out_loss ? reinterpret_cast<float*>((char*)ws + L.partial_off) : nullptr;
    const dim3 grid((unsigned)ceil_div(m.W, kTileW), (unsigned)ceil_div(m.H, kTileH), (unsigned)v.N);
    HSGD_DISPATCH_T(m.dtype, hipLaunchKernelGGL((k_render<DT>), grid, dim3(kBlock), 0, s, m.rgba, m.D,
                                                m.H, m.W, v.warps, v.images, out_rgb, partials));
    if (out_loss)
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, L.nparts, 0.5 / v.N, out_loss);
    return (int)hipGetLastError();
}

int launch_grad_step(const hsgd_mpi& m, const hsgd_views& v, const uint64_t* mask, int kcap,
                     const float* dimg, float lr_rgb, float lr_alpha, float* grad_out,
                     float* out_loss, void* ws, hipStream_t s) {
    const int HW = m.H * m.W;
    const GradWs L = grad_ws(m.D, m.H, m.W, v.N, kcap);
    float4* slots = reinterpret_cast<float4*>((char*)ws + L.slots_off);
    float* partials = reinterpret_cast<float*>((char*)ws + L.partial_off);
    const int fill_blocks = (int)std::min<int64_t>(ceil_div(L.nslots, 256), 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3(fill_blocks), dim3(256), 0, s, slots, L.nslots);
    const dim3 grid((unsigned)ceil_div(m.W, kTileW), (unsigned)ceil_div(m.H, kTileH), (unsigned)v.N);
    const float inv_n = 1.0f / (float)v.N;
    HSGD_DISPATCH_T(m.dtype, HSGD_DISPATCH_D(m.D, hipLaunchKernelGGL((k_grad<DT, MD>), grid, dim3(kBlock), 0, s,
                                                                    m.rgba, m.D, m.H, m.W, v.warps, v.images, dimg,
                                                                    mask, kcap, inv_n, slots,
                                                                    out_loss ? partials : nullptr)));
    const int do_update = (lr_rgb != 0.0f || lr_alpha != 0.0f) ? 1 : 0;
    HSGD_DISPATCH_T(m.dtype, hipLaunchKernelGGL((k_update<DT>), dim3((unsigned)ceil_div(HW, 256)), dim3(256), 0, s,
                                                m.rgba, m.D, HW, mask, kcap, slots, lr_rgb, lr_alpha, do_update,
                                                reinterpret_cast<float4*>(grad_out)));
    if (out_loss)
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, L.nparts, 0.5 / v.N, out_loss);
    return (int)hipGetLastError();
}

int launch_upsample(const hsgd_mpi& c, const hsgd_mpi& f, hipStream_t s) {
    const dim3 grid((unsigned)ceil_div((int64_t)f.H * f.W, 256), (unsigned)c.D);
    HSGD_DISPATCH_T(c.dtype, hipLaunchKernelGGL((k_upsample<DT>), grid, dim3(256), 0, s, c.rgba, c.H, c.W, f.rgba));
    return (int)hipGetLastError();
}

int launch_downsample(const float* img, int N, int H, int W, float* out, hipStream_t s) {
    const dim3 grid((unsigned)ceil_div((int64_t)(H / 2) * (W / 2), 256), (unsigned)N);
    hipLaunchKernelGGL(k_downsample, grid, dim3(256), 0, s, img, H, W, out);
    return (int)hipGetLastError();
}

int launch_convert(const void* src, int sdt, void* dst, int ddt, size_t n, hipStream_t s) {
    const dim3 grid((unsigned)ceil_div((int64_t)n, 256));
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
