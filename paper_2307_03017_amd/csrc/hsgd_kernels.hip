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
//  k_upsample   2x bilinear MPI upsampling between hierarchy levels; k_upsample_select(_blk)
//               fuse it with the new level's first selection (per output pixel on small
//               levels, per 2 x 2 output block from three source rows on large ones)
//  k_downsample 2x2 box mean of target images (the H/2^l pyramid, Sec. 3.2); k_pyramid
//               computes up to three such levels from one read of the finer images
#include <hip/hip_runtime.h>

#include "hsgd_device.h"
#include "hsgd_internal.h"

namespace hsgd {
namespace {

// ------------------------------------------------------------------------------------
// storage: FP32 float4 or BF16 (4 x 16 bit, round to nearest even on store)
// ------------------------------------------------------------------------------------

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
    // voxels i and i + 1 (i even)
    static __device__ __forceinline__ void store2(void* base, int i, float4 a, float4 b) {
        reinterpret_cast<float4*>(base)[i] = a;
        reinterpret_cast<float4*>(base)[i + 1] = b;
    }
    // voxel `col` of the row starting at `row` (row uniform across the wave)
    static __device__ __forceinline__ float4 load_row(const char* row, unsigned col) {
        return *reinterpret_cast<const float4*>(row + (col << 4));
    }
    static __device__ __forceinline__ const char* row_ptr(const void* base, int i) {
        return reinterpret_cast<const char*>(base) + (size_t)(unsigned)i * 16;
    }
    // voxel at byte offset `off` of a buffer resource (0 outside the resource's range)
    static __device__ __forceinline__ float4 load_buf(__amdgpu_buffer_rsrc_t r, unsigned off) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                           __uint_as_float(v[3]));
    }
    static constexpr int kBytes = 16;
    static __device__ __forceinline__ float4 stored(float4 v) { return v; }
    using Raw = float4;                                     // a voxel as stored
    static __device__ __forceinline__ Raw load_raw(__amdgpu_buffer_rsrc_t r, unsigned off) { return load_buf(r, off); }
    static __device__ __forceinline__ float4 decode(const Raw& v) { return v; }
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
    // voxels i and i + 1 (i even: one 16-byte store)
    static __device__ __forceinline__ void store2(void* base, int i, float4 a, float4 b) {
        uint4 r;
        r.x = f32_to_bf16_bits(a.x) | (f32_to_bf16_bits(a.y) << 16);
        r.y = f32_to_bf16_bits(a.z) | (f32_to_bf16_bits(a.w) << 16);
        r.z = f32_to_bf16_bits(b.x) | (f32_to_bf16_bits(b.y) << 16);
        r.w = f32_to_bf16_bits(b.z) | (f32_to_bf16_bits(b.w) << 16);
        reinterpret_cast<uint4*>(base)[i >> 1] = r;
    }
    static __device__ __forceinline__ float4 load_row(const char* row, unsigned col) {
        const uint2 r = *reinterpret_cast<const uint2*>(row + (col << 3));
        return make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u),
                           __uint_as_float(r.y << 16), __uint_as_float(r.y & 0xffff0000u));
    }
    static __device__ __forceinline__ const char* row_ptr(const void* base, int i) {
        return reinterpret_cast<const char*>(base) + (size_t)(unsigned)i * 8;
    }
    static __device__ __forceinline__ float4 load_buf(__amdgpu_buffer_rsrc_t r, unsigned off) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        return make_float4(__uint_as_float(v[0] << 16), __uint_as_float(v[0] & 0xffff0000u),
                           __uint_as_float(v[1] << 16), __uint_as_float(v[1] & 0xffff0000u));
    }
    static constexpr int kBytes = 8;
    using Raw = uint2;                                      // a voxel as stored
    static __device__ __forceinline__ Raw load_raw(__amdgpu_buffer_rsrc_t r, unsigned off) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        return make_uint2(v[0], v[1]);
    }
    static __device__ __forceinline__ float4 decode(const Raw& v) {
        return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u),
                           __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xffff0000u));
    }
    // the value a store followed by a load returns (round to nearest even, NaN quieted)
    static __device__ __forceinline__ float4 stored(float4 v) {
        return make_float4(__uint_as_float(f32_to_bf16_bits(v.x) << 16), __uint_as_float(f32_to_bf16_bits(v.y) << 16),
                           __uint_as_float(f32_to_bf16_bits(v.z) << 16), __uint_as_float(f32_to_bf16_bits(v.w) << 16));
    }
};

// The four taps of a sample, loaded, and their bilinear blend (explicit FMAs: every scan
// that samples a plane gets the same bits).
struct Tap4 {
    float4 a, b, c, d;
};
template <int DT>
__device__ __forceinline__ Tap4 load_taps(const void* mpi, int plane_base, const Taps& t) {
    return Tap4{Vox<DT>::load(mpi, plane_base + t.i00), Vox<DT>::load(mpi, plane_base + t.i10),
                Vox<DT>::load(mpi, plane_base + t.i01), Vox<DT>::load(mpi, plane_base + t.i11)};
}
__device__ __forceinline__ float4 blend_taps(const Taps& t, const Tap4& v) {
    auto f = [&](float a, float b, float c, float d) {
        return __builtin_fmaf(t.w11, d, __builtin_fmaf(t.w01, c, __builtin_fmaf(t.w10, b, t.w00 * a)));
    };
    return make_float4(f(v.a.x, v.b.x, v.c.x, v.d.x), f(v.a.y, v.b.y, v.c.y, v.d.y), f(v.a.z, v.b.z, v.c.z, v.d.z),
                       f(v.a.w, v.b.w, v.c.w, v.d.w));
}
template <int DT>
__device__ __forceinline__ float4 sample(const void* mpi, int plane_base, const Taps& t) {
    return blend_taps(t, load_taps<DT>(mpi, plane_base, t));
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
    constexpr int kWords = (int)(sizeof(hsgd_warp) / sizeof(int));
    const int* src = reinterpret_cast<const int*>(warps + (size_t)view * D);
    int* dst = reinterpret_cast<int*>(sw);
    for (int i = threadIdx.x; i < D * kWords; i += blockDim.x) dst[i] = src[i];
}

// ------------------------------------------------------------------------------------
// select: scores, top-k, and the active-set structures
// ------------------------------------------------------------------------------------
// Per pixel p: A_z = fl(a_z T_z), T_{z+1} = fl(T_z fl(1 - a_z)) front to back on the
// un-warped MPI, then the k largest A_z (equal scores: the nearer plane), then the optional
// threshold. Returns the plane bitmask of p. FP32 contraction is off for this function.
// One front-to-back step of the score recursion for plane alpha a: A = fl(a T) (NaN ranks
// last), T <- fl(T fl(1 - a)).
__device__ __forceinline__ float score_step(float a, float& T) {
#pragma clang fp contract(off)
    const float s = a * T;
    T = T * (1.0f - a);
    return (s == s) ? s : -INFINITY;
}

// The plane mask of the selection rule on the scores A[0..D), then the optional threshold.
// Top-k: the k largest scores (equal scores: the nearer plane). MVS window: the largest
// score (equal: the nearer plane) with (k-1)/2 planes before it (rounded down) and the
// rest after, moved inside [0, D).
// Every pass below is branch-free: the conditions are combined with bitwise operators
// and the running best is kept by selects (with short-circuit operators the unrolled
// passes compiled to a branch per plane).
template <int MAXD>
__device__ __forceinline__ uint64_t topk_bits(const float (&A)[MAXD], int D, int k, float tau, int rule) {
    const uint64_t full = D == 64 ? ~0ull : ((1ull << D) - 1);
    const int kk = min(k, D);
    uint64_t sel = 0;
    if (kk == D) {
        sel = full;
    } else if (rule == HSGD_SELECT_MVS) {
        int best = 0;
        float bestA = A[0];
#pragma unroll
        for (int z = 1; z < MAXD; ++z) {
            const bool b = (z < D) & (A[z] > bestA);
            best = b ? z : best;
            bestA = b ? A[z] : bestA;
        }
        const int lo = min(max(best - (kk - 1) / 2, 0), D - kk);
        sel = (kk == 64 ? ~0ull : ((1ull << kk) - 1)) << lo;
    } else if (2 * kk <= D) {
        // kk passes: the best remaining score, the nearer plane on equal scores
        for (int j = 0; j < kk; ++j) {
            int best = -1;
            float bestA = 0.0f;
#pragma unroll
            for (int z = 0; z < MAXD; ++z) {
                const bool b = (z < D) & (((sel >> z) & 1ull) == 0ull) & ((best < 0) | (A[z] > bestA));
                best = b ? z : best;
                bestA = b ? A[z] : bestA;
            }
            sel |= 1ull << best;
        }
    } else {
        // D - kk passes removing the worst: the lowest score, the farther plane on ties
        uint64_t out = 0;
        for (int j = 0; j < D - kk; ++j) {
            int worst = -1;
            float worstA = 0.0f;
#pragma unroll
            for (int z = 0; z < MAXD; ++z) {
                const bool b = (z < D) & (((out >> z) & 1ull) == 0ull) & ((worst < 0) | (A[z] <= worstA));
                worst = b ? z : worst;
                worstA = b ? A[z] : worstA;
            }
            out |= 1ull << worst;
        }
        sel = full & ~out;
    }
    if (tau >= 0.0f) {
#pragma unroll
        for (int z = 0; z < MAXD; ++z)
            sel &= ~((uint64_t)((z < D) & !(A[z] > tau)) << z);
    }
    return sel;
}

// All D alpha loads are issued before the first is used (plane index clamped, so the loads
// need no guard): one memory latency per pixel rather than one per plane.
template <int DT, int MAXD>
__device__ __forceinline__ uint64_t select_bits(const void* __restrict__ mpi, int D, int HW, int p,
                                                int k, float tau, int rule) {
    float a[MAXD];
#pragma unroll
    for (int z = 0; z < MAXD; ++z) a[z] = Vox<DT>::alpha(mpi, min(z, D - 1) * HW + p);
    float A[MAXD];
    float T = 1.0f;
#pragma unroll
    for (int z = 0; z < MAXD; ++z)
        if (z < D) A[z] = score_step(a[z], T);
    return topk_bits<MAXD>(A, D, k, tau, rule);
}

// The transposed view of a 64-pixel block's masks: for every plane the wave ballot (bit
// = pixel of the block) and its population count. Every lane of the wave must call it.
__device__ __forceinline__ void emit_ballots(uint64_t sel, int D, int64_t wblk, int64_t nblk,
                                             uint64_t* __restrict__ bal, int* __restrict__ cnt) {
    for (int z = 0; z < D; ++z) {
        const uint64_t b = __ballot((sel >> z) & 1);
        if ((threadIdx.x & 63) == 0 && wblk < nblk) {
            bal[z * nblk + wblk] = b;
            cnt[z * nblk + wblk] = __popcll(b);
        }
    }
}

template <int DT, int MAXD>
__global__ __launch_bounds__(256) void k_select(const void* __restrict__ mpi, int D, int HW, int k,
                                                float tau, int rule, uint64_t* __restrict__ mask,
                                                uint64_t* __restrict__ bal, int* __restrict__ cnt,
                                                int64_t nblk) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t sel = 0;
    if (p < HW) {
        sel = select_bits<DT, MAXD>(mpi, D, HW, p, k, tau, rule);
        if (mask) mask[p] = sel;
    }
    if (bal) emit_ballots(sel, D, (int64_t)p >> 6, nblk, bal, cnt);
}

// Active-set structures from a caller's mask (NULL: every voxel); bits of a pixel beyond
// its first kcap set bits are dropped.
__global__ __launch_bounds__(256) void k_mask_ballot(const uint64_t* __restrict__ mask, int D, int HW,
                                                     int kcap, uint64_t* __restrict__ bal,
                                                     int* __restrict__ cnt, int64_t nblk) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t full = D == 64 ? ~0ull : ((1ull << D) - 1);
    uint64_t sel = 0;
    if (p < HW) {
        sel = (mask ? mask[p] : full) & full;
        if (__popcll(sel) > kcap) {
            uint64_t kept = 0;
            for (int j = 0; j < kcap; ++j) {
                const uint64_t low = sel & (~sel + 1);
                kept |= low;
                sel &= sel - 1;
            }
            sel = kept;
        }
    }
    emit_ballots(sel, D, (int64_t)p >> 6, nblk, bal, cnt);
}

// Segmented exclusive scan of the counts (plane-major), phase 1: each workgroup scans
// kSeg consecutive entries in place and writes its total.
constexpr int kSeg = kScanSeg;
__global__ __launch_bounds__(256) void k_scan_seg(int* __restrict__ v, int64_t n,
                                                  int* __restrict__ seg_total) {
    __shared__ int sv[kSeg];
    __shared__ int ssum[256];
    const int64_t base = (int64_t)blockIdx.x * kSeg;
    for (int i = threadIdx.x; i < kSeg; i += 256) sv[i] = base + i < n ? v[base + i] : 0;
    __syncthreads();
    int s = 0;
    for (int j = 0; j < kSeg / 256; ++j) s += sv[threadIdx.x * (kSeg / 256) + j];
    ssum[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        int t = threadIdx.x >= o ? ssum[threadIdx.x - o] : 0;
        __syncthreads();
        ssum[threadIdx.x] += t;
        __syncthreads();
    }
    int run = ssum[threadIdx.x] - s;
    for (int j = 0; j < kSeg / 256; ++j) {
        int c = sv[threadIdx.x * (kSeg / 256) + j];
        sv[threadIdx.x * (kSeg / 256) + j] = run;
        run += c;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSeg; i += 256)
        if (base + i < n) v[base + i] = sv[i];
    if (threadIdx.x == 255) seg_total[blockIdx.x] = ssum[255];
}

// Phase 2 (one workgroup): exclusive scan of the segment totals; plane offsets and |S|.
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
    if (plane_off) {
        for (int z = threadIdx.x; z < D; z += 1024) {
            const int64_t e = (int64_t)z * nblk;
            plane_off[z] = v[e] + seg[e / kSeg];
        }
    }
    if (threadIdx.x == 0) {
        if (plane_off) plane_off[D] = carry;
        *n_active = carry;
    }
}

// Wavefront compaction: each wave owns one 64-pixel block; for every plane its ballot
// word gives the selected lanes and their rank (popcount below the lane), its scanned
// offset the position of the block in the plane-major list. Also turns the offsets into
// global positions in place, for the gradient kernels.
__global__ __launch_bounds__(256) void k_compact(const uint64_t* __restrict__ bal, int* __restrict__ off,
                                                 const int* __restrict__ seg, int D, int HW,
                                                 int64_t nblk, int* __restrict__ ids, int64_t cap) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t wblk = (int64_t)p >> 6;
    if (wblk >= nblk) return;   // whole waves only
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (1ull << lane) - 1;
    for (int z = 0; z < D; ++z) {
        const int64_t e = (int64_t)z * nblk + wblk;
        const uint64_t b = bal[e];
        const int base = off[e] + seg[e / kSeg];
        if ((b >> lane) & 1) {
            const int64_t pos = (int64_t)base + __popcll(b & lt);
            if (pos < cap) ids[pos] = z * HW + p;
        }
        if (lane == 0) off[e] = base;
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
            c0 = __builtin_fmaf(wgt, s.x, c0);
            c1 = __builtin_fmaf(wgt, s.y, c1);
            c2 = __builtin_fmaf(wgt, s.z, c2);
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
            sq = __builtin_fmaf(d2, d2, __builtin_fmaf(d1, d1, d0 * d0));
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
// Gradient slots. A selected voxel (z, p) whose pixel has r selected planes nearer than z
// ("rank" r, r < kcap) owns slot (r, p) of a rank-major slice [kcap][H*W] of float4; the
// gradient kernels write per-view slices [N][kcap][H*W] (or one slice for general warps)
// and the update kernel sums them.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t plane_bits(int D) { return D == 64 ? ~0ull : ((1ull << D) - 1); }

// rank of plane z in mask word m, or -1 when (z, p) is not selected or beyond kcap
__device__ __forceinline__ int slot_rank(uint64_t m, int z, int kcap) {
    if (!((m >> z) & 1)) return -1;
    const int r = __popcll(m & ((1ull << z) - 1));
    return r < kcap ? r : -1;
}

// ------------------------------------------------------------------------------------
// gradient, general warps: per-ray scans, atomic transposed-bilinear scatter
// ------------------------------------------------------------------------------------
// Whole-wave lane shifts for the general-warp scatter: lane i <- lane i-1 / lane i+1; a lane
// without a source gets `none`.
__device__ __forceinline__ int lane_prev_i(int v, int none) {
    return __builtin_amdgcn_update_dpp(none, v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ int lane_next_i(int v, int none) {
    return __builtin_amdgcn_update_dpp(none, v, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ float4 lane_prev_f4(float4 v) {
    auto f = [](float a) { return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), 0x138, 0xF, 0xF, false)); };
    return make_float4(f(v.x), f(v.y), f(v.z), f(v.w));
}

// One tap's contribution to the slots: cell c (-1: none) of plane z, value g.
__device__ __forceinline__ void scatter_cell(float4* __restrict__ slots, const uint64_t* __restrict__ mask,
                                             uint64_t full, int kcap, int HW, int z, int c, const float4& g) {
    if (c < 0) return;
    const int r = slot_rank(mask ? mask[c] : full, z, kcap);
    if (r < 0) return;
    float* dst = reinterpret_cast<float*>(slots + (size_t)r * HW + c);
    atomicAdd(dst + 0, g.x);
    atomicAdd(dst + 1, g.y);
    atomicAdd(dst + 2, g.z);
    atomicAdd(dst + 3, g.w);
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
    // per plane parity: every lane's left-column tap cells (top, bottom) and its bottom-left
    // contribution, for the row merge between neighbouring waves
    __shared__ int s_cell[2][2][kBlock];
    __shared__ float4 s_low[2][kBlock];
    const int view = blockIdx.z;
    load_warps(sw, warps, view, D);
    __syncthreads();
    const int x = blockIdx.x * kTileW + (threadIdx.x & 63);
    const int y = blockIdx.y * kTileH + (threadIdx.x >> 6);
    const int HW = H * W;
    const uint64_t full = plane_bits(D);
    // every lane runs both scans (a lane past the frame samples clamped taps and carries a
    // zero residual), so that neighbouring lanes can merge their shared taps below
    const bool ray = x < W && y < H;
    float sq = 0.0f;
    float Ts[MAXD];
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
    for (int z = 0; z < MAXD; ++z) {
        if (z < D) {
            const Taps tp = make_taps(sw[z], x, y, H, W);
            const float4 s = sample<DT>(mpi, z * HW, tp);
            Ts[z] = T;
            const float wgt = T * s.w;
            c0 = __builtin_fmaf(wgt, s.x, c0);
            c1 = __builtin_fmaf(wgt, s.y, c1);
            c2 = __builtin_fmaf(wgt, s.z, c2);
            T *= 1.0f - s.w;
        }
    }
    float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
    if (ray) {
        const size_t pix = ((size_t)view * H + y) * W + x;
        if (images) {
            const float d0 = c0 - images[3 * pix + 0];
            const float d1 = c1 - images[3 * pix + 1];
            const float d2 = c2 - images[3 * pix + 2];
            sq = __builtin_fmaf(d2, d2, __builtin_fmaf(d1, d1, d0 * d0));
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
            // the four taps (cell -1: no contribution): left column 00 / 01, right 10 / 11
            int e00 = ray && tp.w00 != 0.0f ? tp.i00 : -1, e10 = ray && tp.w10 != 0.0f ? tp.i10 : -1;
            int e01 = ray && tp.w01 != 0.0f ? tp.i01 : -1, e11 = ray && tp.w11 != 0.0f ? tp.i11 : -1;
            float4 v00 = make_float4(tp.w00 * gs.x, tp.w00 * gs.y, tp.w00 * gs.z, tp.w00 * gs.w);
            const float4 v10 = make_float4(tp.w10 * gs.x, tp.w10 * gs.y, tp.w10 * gs.z, tp.w10 * gs.w);
            float4 v01 = make_float4(tp.w01 * gs.x, tp.w01 * gs.y, tp.w01 * gs.z, tp.w01 * gs.w);
            const float4 v11 = make_float4(tp.w11 * gs.x, tp.w11 * gs.y, tp.w11 * gs.z, tp.w11 * gs.w);
            // a right-column cell of lane i-1 that is lane i's left-column cell is added by
            // lane i, once (the same equality on both sides: lane i merges exactly what lane
            // i-1 drops), so neighbouring lanes of one atomic instruction rarely share a cell
            const int p10 = lane_prev_i(e10, -1), p11 = lane_prev_i(e11, -1);
            const float4 q10 = lane_prev_f4(v10), q11 = lane_prev_f4(v11);
            const int n00 = lane_next_i(e00, -1), n01 = lane_next_i(e01, -1);
            if (e00 >= 0 && p10 == e00) v00 = make_float4(v00.x + q10.x, v00.y + q10.y, v00.z + q10.z, v00.w + q10.w);
            if (e01 >= 0 && p11 == e01) v01 = make_float4(v01.x + q11.x, v01.y + q11.y, v01.z + q11.z, v01.w + q11.w);
            if (e10 >= 0 && n00 == e10) e10 = -1;
            if (e11 >= 0 && n01 == e11) e11 = -1;
            // the same between rows: a bottom-left cell of the wave above (same lane) that is
            // this lane's top-left cell is added here, and dropped there
            const int par = z & 1, t = threadIdx.x, wv = t >> 6;
            s_cell[par][0][t] = e00;
            s_cell[par][1][t] = e01;
            s_low[par][t] = v01;
            __syncthreads();   // (buffers alternate by plane: the next plane's writes go to the other)
            if (wv > 0 && e00 >= 0 && s_cell[par][1][t - 64] == e00) {
                const float4 a = s_low[par][t - 64];
                v00 = make_float4(v00.x + a.x, v00.y + a.y, v00.z + a.z, v00.w + a.w);
            }
            if (wv + 1 < kTileH && e01 >= 0 && s_cell[par][0][t + 64] == e01) e01 = -1;
            scatter_cell(slots, mask, full, kcap, HW, z, e00, v00);
            scatter_cell(slots, mask, full, kcap, HW, z, e10, v10);
            scatter_cell(slots, mask, full, kcap, HW, z, e01, v01);
            scatter_cell(slots, mask, full, kcap, HW, z, e11, v11);
        }
    }
    if (partials) {
        const float tot = block_sum(sq, sred);
        if (threadIdx.x == 0)
            partials[((size_t)view * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
    }
}

// ------------------------------------------------------------------------------------
// gradient, pure-translation warps: owner-computes, no atomics, deterministic
//
// A workgroup takes a 64 x 8 block of view rays: lane 0 and wave 0 are a halo column and
// row, lane 63 only supplies the right-hand bilinear taps of lane 62, and the 62 x 7 rays
// in between are "owners". For plane z every owner (x, y) also owns the reference cell
// (x + ix_z, y + iy_z): with a translation, the four rays whose bilinear footprint covers
// that cell are the owner and its left, upper and upper-left neighbours, all in the block.
// Per-ray adjoints are combined across lanes with DPP and across waves through LDS, and
// each owner writes its cell's gradient once, into its view's slice of the slots.
// The front-to-back scan also fetches every owned cell's mask word and keeps one byte per
// plane (rank + 1, or 0 if the cell is not selected), so the back-to-front scan needs no
// memory access besides LDS, and skips the adjoint of planes no cell of the rows needs.
// ------------------------------------------------------------------------------------
constexpr int kSX = 64, kSY = kShiftOY + 1;
constexpr int kOX = kShiftOX, kOY = kShiftOY;
static_assert(kOX == kSX - 2, "lanes: halo, owners, tap supplier");

// DPP wave shifts (bound_ctrl: a lane without a source reads 0)
// Lane i <- lane i+1 (lane 63 <- 0) and lane i <- lane i-1 (lane 0 <- 0), written so that
// the shift folds into the consuming add or multiply as a DPP operand.
__device__ __forceinline__ float lane_from_next(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_from_prev(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}

__device__ __forceinline__ int rl(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ float rlf(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Bilinear sample of a translation warp, one channel: this lane holds its column of the
// two tap rows (a0 above, a1 below), the next lane the column to the right. Vertical lerp
// of the own column, then the horizontal lerp with the next lane's (4 instructions, the
// lane shift folded into a multiply). wt = (upper row weight, lower row weight, 1 - fx,
// fx), a row outside the plane weighted 0.
__device__ __forceinline__ float lerp_taps(float a0, float a1, const float4& wt) {
    const float v = __builtin_fmaf(a1, wt.y, a0 * wt.x);
    return __builtin_fmaf(v, wt.z, lane_from_next(v) * wt.w);
}

// One 64 x 8 tile of one view (tile = view + N * (tx + ntx * ty)); every thread of the
// workgroup calls it.
// Planes whose front-to-back samples the gradient tile keeps for its back-to-front scan,
// and the waves per SIMD the kernel is compiled for: up to 32 planes 6 (3 workgroups per CU,
// within 80 registers), except FP32 at 32 planes, which keeps the samples of its last 16
// planes in the registers of 4 waves per SIMD (2 workgroups per CU) and measured faster.
// 64 planes run at 4 waves per SIMD (their LDS allows 2 workgroups per CU); BF16 there
// keeps 4 planes within that register budget.
template <int DT, int MAXD>
constexpr int grad_shift_keep() {
    return DT == HSGD_FP32 && MAXD == 32 ? 16 : (DT == HSGD_BF16 && MAXD == 64 ? 4 : 0);
}
template <int DT, int MAXD>
constexpr int grad_shift_waves() {
    return grad_shift_keep<DT, MAXD>() > 0 ? 4 : (MAXD > 32 ? 1 : 6);
}
// The batched kernel's persistent loop needs registers of its own: it keeps 8 planes at FP32
// and 32 planes, none elsewhere (the results do not depend on how many are kept).
template <int DT, int MAXD>
constexpr int batch_grad_keep() {
    return DT == HSGD_FP32 && MAXD == 32 ? 8 : 0;
}

template <int DT, int MAXD, bool MASKED, int KEEP = grad_shift_keep<DT, MAXD>()>
__device__ __forceinline__ void grad_shift_tile(
    const void* __restrict__ mpi, int D, int H, int W, int N, const hsgd_warp* __restrict__ warps,
    const float* __restrict__ images, const float* __restrict__ dimg, const uint64_t* __restrict__ mask,
    int kcap, float inv_n, float4* __restrict__ slots, float* __restrict__ partials, int ntx, int tile,
    unsigned tid) {
    __shared__ float4 s_h[2][kSX * kSY];
    __shared__ uint64_t s_bits[kSY];
    __shared__ float sred[kSX * kSY / 64];
    __shared__ float4 s_w[kSY][MAXD];                       // per wave row and plane: tap weights
    __shared__ float2 s_f[MAXD];                            // per plane: the shift's fraction
    __shared__ uint32_t s_code[(MAXD + 3) / 4][kSX * kSY];  // rank bytes of 4 planes per thread
    // Transmittance in front of the first kTL planes: these live longest (from the start of
    // the front-to-back scan to the end of the back-to-front one), so at 6 waves per SIMD
    // they go to LDS instead of registers, which would otherwise spill to scratch memory
    // (whose reloads wait for every load in flight, the look-ahead included). Six planes
    // keep 32 planes within 80 registers at 6 waves per SIMD; with 49.5 KB of LDS three
    // workgroups fit a CU. The 4-wave form that keeps 16 planes' samples has 80 KB per
    // workgroup (two per CU): 18 planes of transmittance there (74 KB) make the registers
    // for the kept samples.
    constexpr int kTL = MAXD <= 32 ? (KEEP > 8 ? 18 : 6) : 0;
    __shared__ float s_T[kTL > 0 ? kTL : 1][kSX * kSY];
    const int view = tile % N;
    const int t2 = tile / N;
    const int tx = t2 % ntx, ty = t2 / ntx;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int xl = tx * kOX - 1;                 // x of lane 0
    const int x = xl + lane, y = ty * kOY - 1 + wv;
    const bool ray = lane < kSX - 1 && (unsigned)x < (unsigned)W && (unsigned)y < (unsigned)H;
    const bool owner = lane >= 1 && lane < kSX - 1 && wv >= 1;
    const int HW = H * W;
    const uint64_t full = plane_bits(D);

    // Plane tables, one entry per lane z < MAXD (read per plane with v_readlane, feeding
    // scalar address arithmetic):
    //   lrow  byte offset, within plane z, of this wave's upper tap row y + iy clamped into
    //         the plane, | 1 if that row lies in the plane, | 2 if the row below it does,
    //         | 4 if the row below is the plane's first row (the upper one lies above it);
    //   lcol  the integer column shift times the voxel size (ix * s).
    // A wave's tap columns are then x + ix for its lanes' x.
    // The bilinear weights of each plane for this wave's row (lerp_taps' four; a tap row
    // outside the plane weighted 0) and the shift's fraction go to LDS, read per plane as
    // broadcasts. Planes z >= D repeat plane D - 1 with zero weights.
    constexpr int S = Vox<DT>::kBytes;
    const int rowbytes = W * S;
    const int dlast = __builtin_amdgcn_readfirstlane(D - 1);    // last plane, wave-uniform
    int lrow = 0, lcol = 0;
    if (lane < MAXD) {
        float4 wt = make_float4(0.f, 0.f, 0.f, 0.f);
        float2 fr = make_float2(0.f, 0.f);
        const hsgd_warp& w = warps[(size_t)view * D + min(lane, dlast)];
        const int Y0 = y + w.iy;
        const bool in0 = (unsigned)Y0 < (unsigned)H, in1 = (unsigned)(Y0 + 1) < (unsigned)H;
        lrow = min(max(Y0, 0), H - 1) * rowbytes | (in0 ? 1 : 0) | (in1 ? 2 : 0) | (Y0 == -1 ? 4 : 0);
        // (a shift beyond the frame and its halo only ever reads padding; clamping it there
        // keeps every lane's byte offset from wrapping into the row)
        lcol = min(max(w.ix, -(W + 64)), W + 64) * S;
        if (lane < D) {
            fr = make_float2(w.fx, w.fy);
            wt = make_float4(in0 ? 1.0f - fr.y : 0.0f, in1 ? fr.y : 0.0f, 1.0f - fr.x, fr.x);
        }
        s_w[wv][lane] = wt;
        if (wv == 0) s_f[lane] = fr;
    }
    const unsigned xs = (unsigned)x * (unsigned)S;                // wraps when x < 0: outside
    __syncthreads();

    // Both scans run over MAXD planes; planes z >= D sample plane D-1 with zero weights (a
    // transparent plane) and select nothing. The taps of plane z +- kAhead are loaded while
    // plane z is processed (see the end of each scan), and a scheduling fence per plane
    // keeps that look-ahead (and the register footprint) fixed. The second scan samples the
    // planes again (all but the last kKeep, below) instead of keeping them in registers: that
    // keeps the kernel small enough for several workgroups per CU, which hides the per-plane
    // barrier.
    struct Taps2 {
        typename Vox<DT>::Raw t00, t01;   // taps of rows y0 and y0 + 1, as stored (right-hand taps come from lane + 1)
        unsigned row;      // in-plane byte offset of the upper tap row, with lrow's flags
        unsigned col;      // the column shift in bytes (ix * s), wave-uniform
        // byte offset of this lane's tap column in a row: (x + ix) * s
        __device__ unsigned off(unsigned xs_) const { return xs_ + col; }
    };
    // zstride: the plane stride in voxels (H W), passed laundered to the second scan so that
    // the compiler cannot prove its loads equal the first scan's and keep those alive instead.
    // Taps come through buffer resources over the two tap rows: a column outside the
    // plane, or a whole row outside it, reads as 0 -- the zero padding -- so neither the
    // addresses nor the weights need per-lane range checks.
    auto fetch = [&](int z, int zstride) {
        Taps2 f;
        f.row = (unsigned)rl(lrow, z);
        f.col = (unsigned)rl(lcol, z);
        const char* plane = reinterpret_cast<const char*>(mpi) + (size_t)((unsigned)min(z, dlast) * (unsigned)zstride) * S;
        const char* row0 = plane + (f.row & ~7u);
        const char* row1 = row0 + ((f.row & 4u) ? 0u : (unsigned)rowbytes);
        const unsigned off = f.off(xs);
        f.t00 = Vox<DT>::load_raw(row_rsrc(row0, (f.row & 1u) ? rowbytes : 0), off);
        f.t01 = Vox<DT>::load_raw(row_rsrc(row1, (f.row & 2u) ? rowbytes : 0), off);
        return f;
    };
    // the owned cell's mask word (the cell is the upper tap row's voxel of this lane's
    // column), through a buffer resource over the cell's mask row: a cell outside the
    // plane reads 0, i.e. unselected
    auto fetch_mask = [&](const Taps2& f) -> uint64_t {
        if (!MASKED) return full;
        const char* row = reinterpret_cast<const char*>(mask) + (f.row & ~7u) / (unsigned)(S / 8);
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(row_rsrc(row, (f.row & 1u) ? W * 8 : 0),
                                                            f.off(xs) / (unsigned)(S / 8), 0, 0);
        return ((uint64_t)v[1] << 32) | v[0];
    };
    auto sample = [&](int z, const Taps2& f) {
        const float4 wt = s_w[wv][z];
        const float4 a0 = Vox<DT>::decode(f.t00), a1 = Vox<DT>::decode(f.t01);
        float4 s;
        s.x = lerp_taps(a0.x, a1.x, wt);
        s.y = lerp_taps(a0.y, a1.y, wt);
        s.z = lerp_taps(a0.z, a1.z, wt);
        s.w = lerp_taps(a0.w, a1.w, wt);
        return s;
    };
    // planes of taps in flight: BF16 taps stay as stored (half the registers) until used,
    // which leaves room for a third plane; FP32 taps fill the same registers with two
    constexpr int kAhead = DT == HSGD_BF16 ? 3 : 2;
    // The samples of the last kKeep planes of the front-to-back scan stay in registers for
    // the back-to-front scan, which starts with them: 2 kKeep fewer row loads per wave (FP32
    // at 32 planes; the kernel then runs at 4 waves per SIMD, see grad_shift_waves).
    constexpr int kKeep = KEEP;
    float4 Sk[kKeep > 0 ? kKeep : 1];
    // Every plane iteration starts with a branch on an opaque, always-true value: the block
    // boundaries keep the compiler from moving each plane's setup code across planes (which
    // would keep all of it alive at once).
    int go = 1;

    float Ts[MAXD];
    uint32_t code = 0;                           // rank + 1 of the owned cell (or 0) per plane,
                                                 // 4 planes per word, flushed to s_code
    uint64_t own_bits = 0;                       // planes where an owned cell of this wave is selected
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    {
        Taps2 q[kAhead];
        uint64_t qm[kAhead];
#pragma unroll
        for (int i = 0; i < kAhead; ++i)
            if (i < MAXD) {
                q[i] = fetch(i, HW);
                qm[i] = fetch_mask(q[i]);
            }
#pragma unroll
        for (int z = 0; z < MAXD; ++z) {
            asm volatile("" : "+v"(go));
            if (!__builtin_amdgcn_readfirstlane(go)) break;
            const Taps2 cur = q[z % kAhead];
            const uint64_t m = qm[z % kAhead];
            if (z + kAhead < MAXD) {
                q[z % kAhead] = fetch(z + kAhead, HW);
                qm[z % kAhead] = fetch_mask(q[z % kAhead]);
            }
            const float4 s = sample(z, cur);
            if (kKeep > 0 && z >= MAXD - kKeep) Sk[z >= MAXD - kKeep ? z - (MAXD - kKeep) : 0] = s;
            if (z < kTL)
                s_T[z < kTL ? z : 0][tid] = T;
            else
                Ts[z] = T;
            const float wgt = T * s.w;
            c0 = __builtin_fmaf(wgt, s.x, c0);
            c1 = __builtin_fmaf(wgt, s.y, c1);
            c2 = __builtin_fmaf(wgt, s.z, c2);
            T *= 1.0f - s.w;
            // (a cell outside the plane has a zero mask word; without a mask, check the range)
            const bool cell = owner && z < D && (MASKED || ((cur.row & 1u) && cur.off(xs) < (unsigned)rowbytes));
            // branch-free: rank + 1 of the owned cell's plane z if selected, else 0
            const uint32_t sel = cell ? (uint32_t)((m >> z) & 1) : 0u;
            const uint32_t rank = (uint32_t)__popcll(m & ((1ull << z) - 1));
            const uint32_t rc = (sel && rank < (uint32_t)kcap) ? rank + 1 : 0u;
            code |= rc << ((z & 3) * 8);
            if ((z & 3) == 3 || z == MAXD - 1) {
                s_code[z >> 2][tid] = code;
                code = 0;
            }
            if (__ballot(rc != 0)) own_bits |= 1ull << z;
            __builtin_amdgcn_sched_barrier(0);
        }
        // The look-ahead loads are consumed on the path out of the loop as well, so that
        // each is issued before its plane's branch rather than sunk to its use planes later.
#pragma unroll
        for (int i = 0; i < kAhead; ++i)
            asm volatile("" ::"v"(q[i].t00.x), "v"(q[i].t01.x), "v"((uint32_t)qm[i]));
    }
    // planes where the wave below has selected cells: it needs this wave's adjoints
    if (lane == 0) s_bits[wv] = own_bits;
    __syncthreads();
    uint64_t below_bits = 0;
    if (wv + 1 < kSY) {
        const uint64_t b = s_bits[wv + 1];
        below_bits = ((uint64_t)__builtin_amdgcn_readfirstlane((int)(b >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    }
    const uint64_t need_bits = own_bits | below_bits;

    float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, sq = 0.0f;
    if (ray) {
        // (x again from the lane's tap offset, so that x itself need not stay live)
        const size_t pix = ((size_t)view * H + y) * W + (int)xs / S;
        if (images) {
            const float d0 = c0 - images[3 * pix + 0];
            const float d1 = c1 - images[3 * pix + 1];
            const float d2 = c2 - images[3 * pix + 2];
            if (owner) sq = __builtin_fmaf(d2, d2, __builtin_fmaf(d1, d1, d0 * d0));
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
    float4* __restrict__ vslots = slots + (size_t)view * kcap * HW;
    // launder what the second scan derives its taps from, so that nothing computed per
    // plane in the first scan is kept alive for it
    int HW2 = HW;
    asm volatile("" : "+s"(HW2), "+v"(lrow), "+v"(lcol));
    uint32_t rcode = 0;
    {
        // (the first planes sampled are those below the kept ones: their loads run while the
        // kept planes are processed)
        Taps2 q[kAhead];
#pragma unroll
        for (int i = 0; i < kAhead; ++i)
            if (i + kKeep < MAXD) q[i] = fetch(MAXD - 1 - kKeep - i, HW2);
#pragma unroll
        for (int zz = 0; zz < MAXD; ++zz) {
            const int z = MAXD - 1 - zz;
            asm volatile("" : "+v"(go));
            if (!__builtin_amdgcn_readfirstlane(go)) break;
            Taps2 cur;
            float4 s;
            if (zz < kKeep) {
                cur.row = (unsigned)rl(lrow, z);
                cur.col = (unsigned)rl(lcol, z);
                s = Sk[zz < kKeep ? kKeep - 1 - zz : 0];
            } else {
                const int zk = zz - kKeep;
                cur = q[zk % kAhead];
                if (zz + kAhead < MAXD) q[zk % kAhead] = fetch(z - kAhead, HW2);
                s = sample(z, cur);
            }
            const float2 fr = s_f[z];
            const float fx = fr.x, fy = fr.y;
            if ((z & 3) == 3 || z == MAXD - 1) rcode = s_code[z >> 2][tid];
            float4* buf = s_h[z & 1];
            // the colour of plane z against the composite behind it: the alpha adjoint's
            // factor and the step of the behind composite, B <- B + a (c - B)
            const float d0 = s.x - b0, d1 = s.y - b1, d2 = s.z - b2;
            if ((need_bits >> z) & 1) {
                const float Tz = z < kTL ? s_T[z < kTL ? z : 0][tid] : Ts[z];
                const float ca = s.w * Tz;
                float4 a;
                a.x = g0 * ca;
                a.y = g1 * ca;
                a.z = g2 * ca;
                a.w = Tz * __builtin_fmaf(g2, d2, __builtin_fmaf(g1, d1, g0 * d0));
                // horizontal half of the transposed bilinear: this ray (1 - fx) and the
                // ray to the left (fx) both touch the owned cell's row
                const float gx = 1.0f - fx;
                float4 h;
                h.x = __builtin_fmaf(a.x, gx, lane_from_prev(a.x) * fx);
                h.y = __builtin_fmaf(a.y, gx, lane_from_prev(a.y) * fx);
                h.z = __builtin_fmaf(a.z, gx, lane_from_prev(a.z) * fx);
                h.w = __builtin_fmaf(a.w, gx, lane_from_prev(a.w) * fx);
                buf[tid] = h;
            }
            b0 = __builtin_fmaf(s.w, d0, b0);
            b1 = __builtin_fmaf(s.w, d1, b1);
            b2 = __builtin_fmaf(s.w, d2, b2);
            __syncthreads();
            if ((own_bits >> z) & 1) {
                const int rc = (int)((rcode >> ((z & 3) * 8)) & 0xffu);
                if (rc) {
                    // this row's and the row above's horizontal halves, both from LDS (the
                    // own half is not kept in registers across the barrier)
                    const float4 h = buf[tid];
                    const float4 hu = buf[tid - 64];
                    const float gy = 1.0f - fy;
                    float4 c;
                    c.x = __builtin_fmaf(hu.x, fy, h.x * gy);
                    c.y = __builtin_fmaf(hu.y, fy, h.y * gy);
                    c.z = __builtin_fmaf(hu.z, fy, h.z * gy);
                    c.w = __builtin_fmaf(hu.w, fy, h.w * gy);
                    // slot (rank, cell): the cell's byte offset in an FP32 RGBA plane is its
                    // tap offsets scaled from the storage's voxel size to 16 bytes
                    const unsigned cell16 = ((cur.row & ~7u) + cur.off(xs)) * (unsigned)(16 / S);
                    const unsigned idx = (unsigned)(rc - 1) * (unsigned)HW * 16u + cell16;
                    *reinterpret_cast<float4*>(reinterpret_cast<char*>(vslots) + idx) = c;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int i = 0; i < kAhead; ++i)
            if (i + kKeep < MAXD) asm volatile("" ::"v"(q[i].t00.x), "v"(q[i].t01.x));
    }
    if (partials) {
        const float tot = block_sum(sq, sred);
        if (threadIdx.x == 0) partials[tile] = tot;
    }
}

// Waves per SIMD as grad_shift_waves gives them, without spills (the first planes'
// transmittance is kept in LDS).
template <int DT, int MAXD, bool MASKED>
__global__ __launch_bounds__(kSX * kSY) __attribute__((amdgpu_waves_per_eu(grad_shift_waves<DT, MAXD>()))) void k_grad_shift(
    const void* __restrict__ mpi, int D, int H, int W, int N, const hsgd_warp* __restrict__ warps,
    const float* __restrict__ images, const float* __restrict__ dimg, const uint64_t* __restrict__ mask,
    int kcap, float inv_n, float4* __restrict__ slots, float* __restrict__ partials, int ntx) {
    grad_shift_tile<DT, MAXD, MASKED>(mpi, D, H, W, N, warps, images, dimg, mask, kcap, inv_n, slots, partials,
                                      ntx, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x);
}

// ------------------------------------------------------------------------------------
// render, translation warps: the gradient kernel's front-to-back scan on its own
// ------------------------------------------------------------------------------------
// One workgroup = 63 x 8 rays of one view (lane 63 of each wave only supplies the right-
// hand taps of lane 62): per plane two row loads through buffer resources (hardware zero
// padding), per-wave tap weights from an LDS table, the right column through DPP, two
// planes of loads in flight.
template <int DT, int MAXD>
__global__ __launch_bounds__(kSX * kSY) void k_render_shift(const void* __restrict__ mpi, int D, int H, int W,
                                                            int N, const hsgd_warp* __restrict__ warps,
                                                            const float* __restrict__ images,
                                                            float* __restrict__ out_rgb,
                                                            float* __restrict__ partials, int ntx) {
    __shared__ float4 s_w[kSY][MAXD];
    __shared__ float sred[kSX * kSY / 64];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int view = tile % N;
    const int t2 = tile / N;
    const int tx = t2 % ntx, ty = t2 / ntx;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xl = tx * kShiftRX;
    const int x = xl + lane, y = ty * kShiftRY + wv;
    const bool ray = lane < kShiftRX && x < W && y < H;
    int lx = 0, ly = 0;
    if (lane < MAXD) {
        float4 wt = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane < D) {
            const hsgd_warp& w = warps[(size_t)view * D + lane];
            lx = w.ix;
            ly = w.iy;
            const int Y0 = y + ly;
            const float gy = (unsigned)Y0 < (unsigned)H ? 1.0f - w.fy : 0.0f;
            const float hy = (unsigned)(Y0 + 1) < (unsigned)H ? w.fy : 0.0f;
            wt = make_float4(gy, hy, 1.0f - w.fx, w.fx);
        }
        s_w[wv][lane] = wt;
    }
    __syncthreads();
    const int HW = H * W;
    const int rb = W * Vox<DT>::kBytes;
    struct Taps2 {
        float4 t00, t01;
    };
    auto fetch = [&](int z) {
        Taps2 f;
        const int ix = rl(lx, z), iy = rl(ly, z);
        const int zb = min(z, D - 1) * HW;
        const int Y0 = y + iy;
        const unsigned off = (unsigned)(x + ix) * (unsigned)Vox<DT>::kBytes;
        const bool r0 = (unsigned)Y0 < (unsigned)H, r1 = (unsigned)(Y0 + 1) < (unsigned)H;
        f.t00 = Vox<DT>::load_buf(row_rsrc(Vox<DT>::row_ptr(mpi, zb + (r0 ? Y0 : 0) * W), r0 ? rb : 0), off);
        f.t01 = Vox<DT>::load_buf(row_rsrc(Vox<DT>::row_ptr(mpi, zb + (r1 ? Y0 + 1 : 0) * W), r1 ? rb : 0), off);
        return f;
    };
    constexpr int kAhead = 2;
    int go = 1;
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    {
        Taps2 q[kAhead];
#pragma unroll
        for (int i = 0; i < kAhead; ++i)
            if (i < MAXD) q[i] = fetch(i);
#pragma unroll
        for (int z = 0; z < MAXD; ++z) {
            asm volatile("" : "+v"(go));
            if (!__builtin_amdgcn_readfirstlane(go)) break;
            const Taps2 f = q[z % kAhead];
            if (z + kAhead < MAXD) q[z % kAhead] = fetch(z + kAhead);
            const float4 wt = s_w[wv][z];
            float4 s;
            s.x = lerp_taps(f.t00.x, f.t01.x, wt);
            s.y = lerp_taps(f.t00.y, f.t01.y, wt);
            s.z = lerp_taps(f.t00.z, f.t01.z, wt);
            s.w = lerp_taps(f.t00.w, f.t01.w, wt);
            const float wgt = T * s.w;
            c0 = __builtin_fmaf(wgt, s.x, c0);
            c1 = __builtin_fmaf(wgt, s.y, c1);
            c2 = __builtin_fmaf(wgt, s.z, c2);
            T *= 1.0f - s.w;
            __builtin_amdgcn_sched_barrier(0);
        }
        // keep the look-ahead loads ahead of each plane's branch (see the gradient kernel)
        asm volatile("" ::"v"(q[0].t00.x), "v"(q[0].t01.x), "v"(q[1].t00.x), "v"(q[1].t01.x));
    }
    float sq = 0.0f;
    if (ray) {
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
            sq = __builtin_fmaf(d2, d2, __builtin_fmaf(d1, d1, d0 * d0));
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

// One thread per pixel: for each selected plane (rank r < kcap) sum the view slices, then
// apply the clamped descent step in place and/or write the gradient out. With shift
// warps, view v wrote voxel (z, p) only if p lies in v's owner coverage for plane z;
// outside it no ray of v reaches the voxel and the slot is not read. Workgroup 0 also
// reduces the loss partials of the gradient kernel (fixed order, FP64).
// Workgroup blk of the update over one MPI level (256 / RS pixels: with RS > 1 the RS
// groups of 256 / RS threads take the selected planes of rank r = group (mod RS) of the
// same pixels, so the ranks of a pixel are updated in parallel); s_off is LDS for the
// [nslices][D] shifts. Every thread of the 256-thread workgroup calls it.
template <int DT, bool SHIFT, int RS = 1>
__device__ __forceinline__ void update_block(void* __restrict__ mpi, int D, int H, int W,
                                             const uint64_t* __restrict__ mask, int kcap,
                                             const float4* __restrict__ slots, int nslices,
                                             const hsgd_warp* __restrict__ warps, int cover_w,
                                             int cover_h, float lr_rgb, float lr_a, int do_update,
                                             float4* __restrict__ grad_out,
                                             const float* __restrict__ partials, int64_t nparts,
                                             double loss_scale, float* __restrict__ out_loss, float prior,
                                             int blk, int2* __restrict__ s_off) {
    if (SHIFT) {
        for (int i = threadIdx.x; i < nslices * D; i += blockDim.x) s_off[i] = make_int2(warps[i].ix, warps[i].iy);
        __syncthreads();
    }
    if (out_loss && blk == 0) {
        __shared__ double sh[256];
        double acc = 0.0;
        for (int64_t i = threadIdx.x; i < nparts; i += 256) acc += (double)partials[i];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) *out_loss = (float)(sh[0] * loss_scale);
    }
    static_assert(256 % RS == 0, "whole pixel groups");
    constexpr int kPix = 256 / RS;
    const int HW = H * W;
    const int p = blk * kPix + (int)(threadIdx.x % kPix);
    const int q = (int)(threadIdx.x / kPix);
    if (p >= HW) return;
    const int Y = p / W, X = p - Y * W;
    const uint64_t m = (mask ? mask[p] : ~0ull) & plane_bits(D);
    // Sum of the view slices of rank r (plane z), in view order. The loads of 8 views are
    // issued together through one buffer resource per view slice: a view whose owners do
    // not cover the cell (its slot holds stale data), or past the last view, gets an offset
    // outside the resource and reads 0 without touching memory.
    const unsigned slice_bytes = (unsigned)kcap * (unsigned)HW * 16u;
    auto grad_of = [&](int z, int r) {
        float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
        const unsigned off = ((unsigned)r * (unsigned)HW + (unsigned)p) * 16u;
        for (int v0 = 0; v0 < nslices; v0 += 8) {
            float4 t[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int v = min(v0 + j, nslices - 1);
                bool ok = v0 + j < nslices;
                if (SHIFT) {
                    const int2 o = s_off[v * D + z];
                    ok = ok && (unsigned)(X - o.x) < (unsigned)cover_w && (unsigned)(Y - o.y) < (unsigned)cover_h;
                }
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<float4*>(slots + (size_t)v * kcap * HW), (short)0, (int)slice_bytes, kBufWord3);
                const auto u = __builtin_amdgcn_raw_buffer_load_b128(rs, ok ? off : 0xfffffff0u, 0, 0);
                t[j] = make_float4(__uint_as_float(u[0]), __uint_as_float(u[1]), __uint_as_float(u[2]),
                                   __uint_as_float(u[3]));
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                g.x += t[j].x;
                g.y += t[j].y;
                g.z += t[j].z;
                g.w += t[j].w;
            }
        }
        return g;
    };
    uint64_t b = m;
    int r = 0;
    while (b && r < kcap) {
        const int z = __ffsll((unsigned long long)b) - 1;
        b &= b - 1;
        const int rank = r++;
        if (RS > 1 && rank % RS != q) continue;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (do_update || prior != 0.0f) v = Vox<DT>::load(mpi, z * HW + p);   // in flight with the slices
        float4 g = grad_of(z, rank);
        if (prior != 0.0f) {
            // sparsity prior: d/da log(1.5 - |0.5 - a|) = sign(0.5 - a) / (1.5 - |0.5 - a|)
            const float d = 0.5f - v.w;
            const float sg = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
            g.w = __builtin_fmaf(prior, sg / (1.5f - fabsf(d)), g.w);
        }
        if (grad_out) grad_out[(size_t)z * HW + p] = g;
        if (do_update) {
            v.x = fminf(fmaxf(__builtin_fmaf(-lr_rgb, g.x, v.x), 0.0f), 1.0f);
            v.y = fminf(fmaxf(__builtin_fmaf(-lr_rgb, g.y, v.y), 0.0f), 1.0f);
            v.z = fminf(fmaxf(__builtin_fmaf(-lr_rgb, g.z, v.z), 0.0f), 1.0f);
            v.w = fminf(fmaxf(__builtin_fmaf(-lr_a, g.w, v.w), 0.0f), 1.0f);
            Vox<DT>::store(mpi, z * HW + p, v);
        }
    }
}

// the selected planes of a pixel split over 4 thread groups (64 pixels per workgroup)
constexpr int kUpdateRS = 4;
template <int DT, bool SHIFT>
__global__ __launch_bounds__(256) void k_update(void* __restrict__ mpi, int D, int H, int W,
                                                const uint64_t* __restrict__ mask, int kcap,
                                                const float4* __restrict__ slots, int nslices,
                                                const hsgd_warp* __restrict__ warps, int cover_w,
                                                int cover_h, float lr_rgb, float lr_a, int do_update,
                                                float4* __restrict__ grad_out,
                                                const float* __restrict__ partials, int64_t nparts,
                                                double loss_scale, float* __restrict__ out_loss, float prior) {
    extern __shared__ int2 s_off[];   // [nslices][D] (ix, iy) when SHIFT
    update_block<DT, SHIFT, kUpdateRS>(mpi, D, H, W, mask, kcap, slots, nslices, warps, cover_w, cover_h, lr_rgb, lr_a,
                            do_update, grad_out, partials, nparts, loss_scale, out_loss, prior, blockIdx.x, s_off);
}

// ------------------------------------------------------------------------------------
// hierarchy
// ------------------------------------------------------------------------------------
// Source pair and fraction of output coordinate x of a 2x upsampling along an axis of n
// source samples: the sample point (x + 1/2) / 2 - 1/2, clamped to [0, n - 1].
__device__ __forceinline__ void up_axis(int x, int n, int& i0, int& i1, float& f) {
    const float sx = fminf(fmaxf((x + 0.5f) * 0.5f - 0.5f, 0.0f), (float)(n - 1));
    i0 = (int)sx;
    i1 = min(i0 + 1, n - 1);
    f = sx - i0;
}

struct UpW {
    float w00, w10, w01, w11;
};
__device__ __forceinline__ UpW up_weights(float fx, float fy) {
    return UpW{(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
}
// The bilinear blend of taps a (x0, y0), b (x1, y0), c (x0, y1), d (x1, y1): the one
// expression every upsampling path evaluates, so that they agree bit for bit.
__device__ __forceinline__ float4 up_blend(const UpW& w, const float4& a, const float4& b, const float4& c,
                                           const float4& d) {
    auto f = [&](float a_, float b_, float c_, float d_) {
        return __builtin_fmaf(w.w11, d_, __builtin_fmaf(w.w01, c_, __builtin_fmaf(w.w10, b_, w.w00 * a_)));
    };
    return make_float4(f(a.x, b.x, c.x, d.x), f(a.y, b.y, c.y, d.y), f(a.z, b.z, c.z, d.z), f(a.w, b.w, c.w, d.w));
}

// The four source taps of output voxel i of plane z of the 2x upsampling of a [D][h][w]
// level, and their weights.
template <int DT>
struct UpTaps {
    float4 a, b, c, d;
    UpW w;
};
template <int DT>
__device__ __forceinline__ UpTaps<DT> upsample_taps(const void* __restrict__ src, int h, int w, int z, int i) {
    const int W2 = 2 * w;
    const int x = i % W2, y = i / W2;
    int x0, x1, y0, y1;
    float fx, fy;
    up_axis(x, w, x0, x1, fx);
    up_axis(y, h, y0, y1, fy);
    const int base = z * h * w;
    UpTaps<DT> t;
    t.a = Vox<DT>::load(src, base + y0 * w + x0);
    t.b = Vox<DT>::load(src, base + y0 * w + x1);
    t.c = Vox<DT>::load(src, base + y1 * w + x0);
    t.d = Vox<DT>::load(src, base + y1 * w + x1);
    t.w = up_weights(fx, fy);
    return t;
}

// Blends the taps, stores output voxel i of plane z and returns the value as stored (BF16:
// rounded).
template <int DT>
__device__ __forceinline__ float4 upsample_store(const UpTaps<DT>& t, void* __restrict__ dst, int H2W2, int z,
                                                 int i) {
    const float4 o = up_blend(t.w, t.a, t.b, t.c, t.d);
    Vox<DT>::store(dst, z * H2W2 + i, o);
    return Vox<DT>::stored(o);
}

// Output voxel i of plane z of the 2x upsampling of a [D][h][w] level; returns the value
// as stored, or 0 past the level's end.
template <int DT>
__device__ __forceinline__ float4 upsample_voxel(const void* __restrict__ src, int h, int w,
                                                 void* __restrict__ dst, int z, int i) {
    if (i >= 4 * w * h) return make_float4(0.f, 0.f, 0.f, 0.f);
    return upsample_store<DT>(upsample_taps<DT>(src, h, w, z, i), dst, 4 * w * h, z, i);
}

template <int DT>
__global__ __launch_bounds__(256) void k_upsample(const void* __restrict__ src, int h, int w,
                                                  void* __restrict__ dst) {
    upsample_voxel<DT>(src, h, w, dst, blockIdx.y, blockIdx.x * blockDim.x + threadIdx.x);
}

constexpr int kUpWaves = 4;

// Upsampling fused with the first selection at the new level, for levels of few
// workgroups. A block covers 64 output pixels (lane = pixel) and its four waves split the
// planes: each upsamples and stores a
// quarter of them and puts the alpha it stored (the storage-rounded value) in LDS; the
// first wave then scores every plane of its pixel front to back and writes the mask, which
// equals what k_select computes from the stored level. Splitting the planes shortens each
// thread's chain of dependent tap loads and gives the small levels four times the waves.
template <int DT, int MAXD>
__global__ __launch_bounds__(64 * kUpWaves) void k_upsample_select(const void* __restrict__ src, int D, int h,
                                                                   int w, void* __restrict__ dst, int k,
                                                                   float tau, int rule,
                                                                   uint64_t* __restrict__ mask) {
    constexpr int kPW = (MAXD + kUpWaves - 1) / kUpWaves;   // planes per wave
    constexpr int kG = kPW < 4 ? kPW : 4;                    // tap loads of kG planes in flight together
    static_assert(kPW % kG == 0, "whole load groups");
    __shared__ float s_a[kUpWaves * kPW][64];
    const int n = 4 * w * h;
    const int lane = threadIdx.x & 63;
    const int q = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int i = blockIdx.x * 64 + lane;
    if (i < n) {
#pragma unroll
        for (int j0 = 0; j0 < kPW; j0 += kG) {
            // plane index clamped, so the loads need no guard
            UpTaps<DT> t[kG];
#pragma unroll
            for (int j = 0; j < kG; ++j) t[j] = upsample_taps<DT>(src, h, w, min(q * kPW + j0 + j, D - 1), i);
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                const int z = q * kPW + j0 + j;
                if (z < D) s_a[z][lane] = upsample_store<DT>(t[j], dst, n, z, i).w;
            }
        }
    }
    __syncthreads();
    if (q == 0 && i < n) {
        float A[MAXD];
        float T = 1.0f;
#pragma unroll
        for (int z = 0; z < MAXD; ++z)
            if (z < D) A[z] = score_step(s_a[z][lane], T);
        mask[i] = topk_bits<MAXD>(A, D, k, tau, rule);
    }
}

// Upsampling fused with the first selection at the new level, for large levels. A
// workgroup takes one source row Y and 62 source columns (lane = source column X = X0 - 1 + lane; lanes 0 and 63 only
// supply taps to their neighbours) and writes the 2 x 2 output voxels of each of its owner
// columns: per plane it loads source rows Y - 1, Y and Y + 1 (clamped) of its column and
// takes the columns X - 1 and X + 1 from the neighbouring lanes, so a loaded voxel serves
// four outputs. The taps, weights and blend of every output are those of upsample_taps
// (the same source voxels, the same expression). The four waves split the planes and put
// the alpha they stored (storage-rounded) in LDS; then each wave scores and selects a
// quarter of the 248 output pixels front to back, as k_select does on the stored level.
constexpr int kUpCols = 62;               // owner source columns per workgroup
// Below this many workgroups (8 per CU) the 2 x 2 kernel has too few waves to hide its
// longer per-wave work, and the per-pixel kernel is the faster one.
constexpr int64_t kUpBlkMinGroups = 2048;
constexpr int kUpPix = 4 * kUpCols;       // output pixels per workgroup (2 rows x 124)

// alpha as the selection reads it back from LDS: FP32, or the stored BF16 bits (exact)
template <int DT>
struct UpAlpha {
    using T = float;
    static __device__ __forceinline__ T put(float a) { return a; }
    static __device__ __forceinline__ float get(T v) { return v; }
};
template <>
struct UpAlpha<HSGD_BF16> {
    using T = uint16_t;
    static __device__ __forceinline__ T put(float a) { return (uint16_t)(__float_as_uint(a) >> 16); }
    static __device__ __forceinline__ float get(T v) { return __uint_as_float((uint32_t)v << 16); }
};

__device__ __forceinline__ float4 lane_prev4(const float4& v) {
    return make_float4(lane_from_prev(v.x), lane_from_prev(v.y), lane_from_prev(v.z), lane_from_prev(v.w));
}
__device__ __forceinline__ float4 lane_next4(const float4& v) {
    return make_float4(lane_from_next(v.x), lane_from_next(v.y), lane_from_next(v.z), lane_from_next(v.w));
}
__device__ __forceinline__ float4 pick4(bool c, const float4& a, const float4& b) {
    return make_float4(c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z, c ? a.w : b.w);
}

template <int DT, int MAXD>
__global__ __launch_bounds__(64 * kUpWaves) void k_upsample_select_blk(const void* __restrict__ src, int D, int h,
                                                                       int w, void* __restrict__ dst, int k,
                                                                       float tau, int rule,
                                                                       uint64_t* __restrict__ mask) {
    constexpr int kPW = (MAXD + kUpWaves - 1) / kUpWaves;   // planes per wave
    constexpr int kG = kPW < 4 ? kPW : 4;                    // planes of loads in flight
    static_assert(kPW % kG == 0, "whole load groups");
    using AT = typename UpAlpha<DT>::T;
    __shared__ AT s_a[MAXD][kUpPix];
    const int lane = threadIdx.x & 63;
    const int q = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int Y = blockIdx.y;
    const int X = (int)blockIdx.x * kUpCols - 1 + lane;
    const int Xc = min(max(X, 0), w - 1);
    const bool own = lane >= 1 && lane <= kUpCols && X < w;
    const int hw = h * w, W2 = 2 * w, n = 4 * hw;
    const int row0 = max(Y - 1, 0) * w + Xc, row1 = Y * w + Xc, row2 = min(Y + 1, h - 1) * w + Xc;
    // Output column 2X + a and row 2Y + b take source columns / rows x0, x1 / y0, y1 (up_axis).
    // For an owner column these are X - 1 or X (x0, a = 0), X or X + 1 (x1, a = 0), X
    // (x0, a = 1), X + 1 or X (x1, a = 1), and likewise for the rows: the flags below say
    // which, and a neighbour's column is always inside the level when it is used.
    bool xl0, xr0, xr1, yu0, yd0, yd1;
    UpW wt[2][2];
    {
        int i0, i1, j0, j1;
        float fx[2], fy[2];
        up_axis(2 * X, w, i0, i1, fx[0]);
        xl0 = i0 < X;
        xr0 = i1 > X;
        up_axis(2 * X + 1, w, i0, i1, fx[1]);
        xr1 = i1 > X;
        up_axis(2 * Y, h, j0, j1, fy[0]);
        yu0 = j0 < Y;
        yd0 = j1 > Y;
        up_axis(2 * Y + 1, h, j0, j1, fy[1]);
        yd1 = j1 > Y;
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) wt[b][a] = up_weights(fx[a], fy[b]);
    }
    // a wave whose owner columns and row are all inside the level (taps X - 1, X, X + 1 and
    // Y - 1, Y, Y + 1, as for every column and row but the first and last) skips the picks
    const bool inner = __builtin_amdgcn_ballot_w64(own && !(xl0 && !xr0 && xr1)) == 0 && yu0 && !yd0 && yd1;
    const int out0 = 2 * Y * W2 + 2 * X;    // output voxel (2Y, 2X) of plane 0
    const int pix = 2 * (lane - 1);         // LDS column of output pixel (2Y, 2X)
#pragma unroll
    for (int j0 = 0; j0 < kPW; j0 += kG) {
        float4 m[kG][3];
#pragma unroll
        for (int j = 0; j < kG; ++j) {
            // plane index clamped, so the loads need no guard
            const int base = min(q * kPW + j0 + j, D - 1) * hw;
            m[j][0] = Vox<DT>::load(src, base + row0);
            m[j][1] = Vox<DT>::load(src, base + row1);
            m[j][2] = Vox<DT>::load(src, base + row2);
        }
#pragma unroll
        for (int j = 0; j < kG; ++j) {
            const int z = q * kPW + j0 + j;
            float4 L[3], R[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                L[r] = lane_prev4(m[j][r]);
                R[r] = lane_next4(m[j][r]);
            }
            float4 o00, o01, o10, o11;
            if (inner) {
                o00 = up_blend(wt[0][0], L[0], m[j][0], L[1], m[j][1]);
                o01 = up_blend(wt[0][1], m[j][0], R[0], m[j][1], R[1]);
                o10 = up_blend(wt[1][0], L[1], m[j][1], L[2], m[j][2]);
                o11 = up_blend(wt[1][1], m[j][1], R[1], m[j][2], R[2]);
            } else {
                // per source row r: the taps of columns x0 / x1 for a = 0 and x1 for a = 1
                float4 c00[3], c01[3], c11[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    c00[r] = pick4(xl0, L[r], m[j][r]);
                    c01[r] = pick4(xr0, R[r], m[j][r]);
                    c11[r] = pick4(xr1, R[r], m[j][r]);
                }
                // rows y0 / y1: b = 0 takes rows (0 or 1) and (1 or 2), b = 1 rows 1 and (2 or 1)
                o00 = up_blend(wt[0][0], yu0 ? c00[0] : c00[1], yu0 ? c01[0] : c01[1], yd0 ? c00[2] : c00[1],
                               yd0 ? c01[2] : c01[1]);
                o01 = up_blend(wt[0][1], yu0 ? m[j][0] : m[j][1], yu0 ? c11[0] : c11[1], yd0 ? m[j][2] : m[j][1],
                               yd0 ? c11[2] : c11[1]);
                o10 = up_blend(wt[1][0], c00[1], c01[1], yd1 ? c00[2] : c00[1], yd1 ? c01[2] : c01[1]);
                o11 = up_blend(wt[1][1], m[j][1], c11[1], yd1 ? m[j][2] : m[j][1], yd1 ? c11[2] : c11[1]);
            }
            if (own && z < D) {
                Vox<DT>::store2(dst, z * n + out0, o00, o01);
                Vox<DT>::store2(dst, z * n + out0 + W2, o10, o11);
                s_a[z][pix] = UpAlpha<DT>::put(Vox<DT>::stored(o00).w);
                s_a[z][pix + 1] = UpAlpha<DT>::put(Vox<DT>::stored(o01).w);
                s_a[z][kUpPix / 2 + pix] = UpAlpha<DT>::put(Vox<DT>::stored(o10).w);
                s_a[z][kUpPix / 2 + pix + 1] = UpAlpha<DT>::put(Vox<DT>::stored(o11).w);
            }
        }
    }
    __syncthreads();
    // selection: output pixel e of the workgroup (row 2Y + e / 124, column 2 X0 + e % 124)
    const int e = q * 64 + lane;
    const int ox = 2 * (int)blockIdx.x * kUpCols + e % (kUpPix / 2);
    if (e < kUpPix && ox < W2) {
        const int oy = 2 * Y + e / (kUpPix / 2);
        float A[MAXD];
        float T = 1.0f;
#pragma unroll
        for (int z = 0; z < MAXD; ++z)
            if (z < D) A[z] = score_step(UpAlpha<DT>::get(s_a[z][e]), T);
        mask[oy * W2 + ox] = topk_bits<MAXD>(A, D, k, tau, rule);
    }
}

// The 2x2 box mean of a (x, y), b (x + 1, y), c (x, y + 1), d (x + 1, y + 1): the one
// expression every downsampling path evaluates.
__device__ __forceinline__ float box4(float a, float b, float c, float d) { return ((a + b) + (c + d)) * 0.25f; }

// Output pixel i of view n of the 2x2 box mean of [N][H][W][3] images.
__device__ __forceinline__ void downsample_pixel(const float* __restrict__ img, int H, int W,
                                                 float* __restrict__ out, int n, int i) {
    const int h = H / 2, w = W / 2;
    if (i >= h * w) return;
    const int x = i % w, y = i / w;
    const float* s = img + ((size_t)n * H + 2 * y) * W * 3 + 6 * x;
    float* o = out + ((size_t)n * h * w + i) * 3;
    for (int c = 0; c < 3; ++c) o[c] = box4(s[c], s[3 + c], s[3 * W + c], s[3 * W + 3 + c]);
}

// NL successive 2x2 box means of [N][H][W][3] images (H and W multiples of 2^NL) in one
// launch: a thread takes one pixel of the coarsest result, reads its 2^NL x 2^NL block once
// and writes its share of every level (out[j]: level j + 1), each level the box means of
// the one above as downsample_pixel computes them.
template <int NL>
__device__ __forceinline__ void pyramid_block(const float* __restrict__ img, int H, int W, float* __restrict__ out0,
                                              float* __restrict__ out1, float* __restrict__ out2, int n, int bx) {
    constexpr int S = 1 << NL;
    const int hc = H >> NL, wc = W >> NL;
    const int i = bx * 256 + threadIdx.x;
    if (i >= hc * wc) return;
    const int x = i % wc, y = i / wc;
    float cur[S / 2][S / 2][3];
#pragma unroll
    for (int r = 0; r < S / 2; ++r) {
        const float* s0 = img + (((size_t)n * H + y * S + 2 * r) * W + (size_t)x * S) * 3;
        const float* s1 = s0 + (size_t)W * 3;
#pragma unroll
        for (int c = 0; c < S / 2; ++c)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                cur[r][c][ch] = box4(s0[6 * c + ch], s0[6 * c + 3 + ch], s1[6 * c + ch], s1[6 * c + 3 + ch]);
    }
    float* const outs[3] = {out0, out1, out2};
#pragma unroll
    for (int l = 1; l <= NL; ++l) {
        const int E = S >> l;                       // this thread's block edge at level l
        const int Hl = H >> l, Wl = W >> l;
        float* o = outs[l - 1];
#pragma unroll
        for (int r = 0; r < E; ++r)
#pragma unroll
            for (int c = 0; c < E; ++c)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch)
                    o[(((size_t)n * Hl + y * E + r) * Wl + (size_t)x * E + c) * 3 + ch] = cur[r][c][ch];
        if (l < NL) {
#pragma unroll
            for (int r = 0; r < E / 2; ++r)
#pragma unroll
                for (int c = 0; c < E / 2; ++c)
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch)
                        cur[r][c][ch] = box4(cur[2 * r][2 * c][ch], cur[2 * r][2 * c + 1][ch],
                                             cur[2 * r + 1][2 * c][ch], cur[2 * r + 1][2 * c + 1][ch]);
        }
    }
}

template <int NL>
__global__ __launch_bounds__(256) void k_pyramid(const float* __restrict__ img, int H, int W,
                                                 float* __restrict__ out0, float* __restrict__ out1,
                                                 float* __restrict__ out2) {
    pyramid_block<NL>(img, H, W, out0, out1, out2, blockIdx.y, blockIdx.x);
}

// The first selection of the coarsest level and the target pyramid are independent: one
// launch runs both, its first nsel blocks selecting (as k_select) and the others reducing
// (as k_pyramid, block b of view n at nsel + n * nbx + b), so neither waits for the other.
template <int DT, int MAXD, int NL>
__global__ __launch_bounds__(256) void k_select_pyramid(const void* __restrict__ mpi, int D, int HW, int k,
                                                        float tau, int rule, uint64_t* __restrict__ mask,
                                                        int nsel, const float* __restrict__ img, int H, int W,
                                                        float* __restrict__ out0, float* __restrict__ out1,
                                                        float* __restrict__ out2, int nbx) {
    const int b = blockIdx.x;
    if (b < nsel) {
        const int p = b * 256 + threadIdx.x;
        if (p < HW) mask[p] = select_bits<DT, MAXD>(mpi, D, HW, p, k, tau, rule);
    } else {
        const int j = b - nsel;
        pyramid_block<NL>(img, H, W, out0, out1, out2, j / nbx, j % nbx);
    }
}

__global__ __launch_bounds__(256) void k_downsample(const float* __restrict__ img, int H, int W,
                                                    float* __restrict__ out) {
    downsample_pixel(img, H, W, out, blockIdx.y, blockIdx.x * blockDim.x + threadIdx.x);
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

// ------------------------------------------------------------------------------------
// batched serving step: persistent kernels over the work items of every in-flight request
// ------------------------------------------------------------------------------------
// Slot of flat work item g of kernel kk (prefix counts are non-decreasing; uniform result).
__device__ __forceinline__ int batch_slot_of(const BatchTable* __restrict__ t, int kk, int g) {
    int s = 0;
    for (int j = 1; j < t->nslot; ++j) s += g >= t->pre[kk][j] ? 1 : 0;
    return __builtin_amdgcn_readfirstlane(s);
}

__global__ __launch_bounds__(256) void k_batch_down(const BatchTable* __restrict__ t, int stage) {
    const int kk = BK_DOWN0 + stage;
    const int total = t->total[kk];
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        const int sl = batch_slot_of(t, kk, g);
        const BatchSlot& b = t->slot[sl];
        const int j = g - t->pre[kk][sl];
        const int H = b.pyr_h[stage], W = b.pyr_w[stage];
        const int nb = ((H / 2) * (W / 2) + 255) / 256;
        const int n = j / nb;
        downsample_pixel(b.pyr_src[stage], H, W, b.pyr_dst[stage], n, (j - n * nb) * 256 + threadIdx.x);
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_batch_up(const BatchTable* __restrict__ t) {
    const int total = t->total[BK_UP];
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        const int sl = batch_slot_of(t, BK_UP, g);
        const BatchSlot& b = t->slot[sl];
        const int j = g - t->pre[BK_UP][sl];
        const int nb = (4 * b.uh * b.uw + 255) / 256;
        const int z = j / nb;
        upsample_voxel<DT>(b.up_src, b.uh, b.uw, b.mpi, z, (j - z * nb) * 256 + threadIdx.x);
    }
}

template <int DT, int MAXD>
__global__ __launch_bounds__(256) void k_batch_select(const BatchTable* __restrict__ t) {
    const int total = t->total[BK_SELECT];
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        const int sl = batch_slot_of(t, BK_SELECT, g);
        const BatchSlot& b = t->slot[sl];
        const int p = (g - t->pre[BK_SELECT][sl]) * 256 + threadIdx.x;
        const int HW = b.H * b.W;
        if (p < HW) b.mask[p] = select_bits<DT, MAXD>(b.mpi, b.D, HW, p, b.k, b.tau, b.rule);
    }
}

// Tiles are taken in the XCD-grouped order of the flat item list (the grid is a multiple
// of 8 workgroups), so neighbouring tiles of one request share an XCD's L2. Register
// budget as for k_grad_shift where the tile keeps samples.
template <int DT, int MAXD>
__global__ __launch_bounds__(kSX * kSY) __attribute__((amdgpu_waves_per_eu(
    batch_grad_keep<DT, MAXD>() > 0 ? grad_shift_waves<DT, MAXD>() : 1))) void k_batch_grad(const BatchTable* __restrict__ t,
                                                                                          int kk) {
    const int total = t->total[kk];
    for (int i = blockIdx.x; i < total; i += gridDim.x) {
        const int g = xcd_tile(i, total);
        const int sl = batch_slot_of(t, kk, g);
        const BatchSlot& b = t->slot[sl];
        __syncthreads();                     // the previous tile's LDS reads are done
        // a fresh copy of the thread index per tile: nothing the tile derives from it is
        // kept live across tiles
        unsigned tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        grad_shift_tile<DT, MAXD, true, batch_grad_keep<DT, MAXD>()>(b.mpi, b.D, b.H, b.W, b.N, b.warps, b.images, nullptr, b.mask, b.kcap,
                                        1.0f / (float)b.N, b.slots, b.partials, b.ntx,
                                        g - t->pre[kk][sl], tid);
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_batch_update(const BatchTable* __restrict__ t) {
    extern __shared__ int2 s_off[];
    const int total = t->total[BK_UPDATE];
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        const int sl = batch_slot_of(t, BK_UPDATE, g);
        const BatchSlot& b = t->slot[sl];
        __syncthreads();                     // the previous item's shift table is no longer read
        update_block<DT, true>(b.mpi, b.D, b.H, b.W, b.mask, b.kcap, b.slots, b.N, b.warps, b.ntx * kOX,
                               b.nty * kOY, b.lr_rgb, b.lr_alpha, 1, nullptr, b.partials,
                               (int64_t)b.ntx * b.nty * b.N, 0.5 / b.N, b.loss_out, b.prior,
                               g - t->pre[BK_UPDATE][sl], s_off);
    }
}

int maxd_class(int D) { return D <= 8 ? 8 : D <= 16 ? 16 : D <= 32 ? 32 : 64; }

#define HSGD_DISPATCH_D(D, BODY)                         \
    switch (maxd_class(D)) {                             \
        case 8: { constexpr int MD = 8; BODY; } break;   \
        case 16: { constexpr int MD = 16; BODY; } break; \
        case 32: { constexpr int MD = 32; BODY; } break; \
        default: { constexpr int MD = 64; BODY; } break; \
    }

#define HSGD_DISPATCH_T(dt, BODY)                                  \
    if ((dt) == HSGD_FP32) { constexpr int DT = HSGD_FP32; BODY; } \
    else { constexpr int DT = HSGD_BF16; BODY; }

}  // namespace

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
static int launch_scan_compact(const ActiveSet& as, int D, int HW, int* plane_off, hipStream_t s) {
    const int64_t n = (int64_t)D * as.nblk;
    {
        ProfScope ps(HSGD_K_SCAN, s);
        hipLaunchKernelGGL(k_scan_seg, dim3((unsigned)as.nseg), dim3(256), 0, s, as.off, n, as.seg);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, as.off, as.nblk, D, as.seg, (int)as.nseg,
                           plane_off, as.nact);
    }
    ProfScope ps(HSGD_K_COMPACT, s);
    hipLaunchKernelGGL(k_compact, dim3((unsigned)ceil_div(as.nblk * 64, 256)), dim3(256), 0, s, as.bal, as.off,
                       as.seg, D, HW, as.nblk, as.ids, as.cap);
    return (int)hipGetLastError();
}

int launch_select(const hsgd_mpi& m, int k, float tau, int rule, uint64_t* mask, const ActiveSet* as,
                  int32_t* plane_off, hipStream_t s) {
    const int HW = m.H * m.W;
    const dim3 grid((unsigned)ceil_div(HW, 256));
    {
        ProfScope ps(HSGD_K_SELECT, s);
        HSGD_DISPATCH_T(m.dtype, HSGD_DISPATCH_D(m.D, hipLaunchKernelGGL((k_select<DT, MD>), grid, dim3(256), 0, s,
                                                                        m.rgba, m.D, HW, k, tau, rule, mask,
                                                                        as ? as->bal : nullptr,
                                                                        as ? as->off : nullptr,
                                                                        as ? as->nblk : (int64_t)0)));
    }
    if (!as) return (int)hipGetLastError();
    return launch_scan_compact(*as, m.D, HW, plane_off, s);
}

int launch_render(const hsgd_mpi& m, const hsgd_views& v, float* out_rgb, float* out_loss,
                  void* ws, hipStream_t s) {
    const RenderWs L = render_ws(m.H, m.W, v.N);
    float* partials = out_loss ? reinterpret_cast<float*>((char*)ws + L.partial_off) : nullptr;
    int64_t nparts;
    if (v.flags & HSGD_VIEWS_SHIFT_ONLY) {
        const int ntx = (int)ceil_div(m.W, kShiftRX), nty = (int)ceil_div(m.H, kShiftRY);
        nparts = (int64_t)ntx * nty * v.N;
        ProfScope ps(HSGD_K_RENDER, s);
        HSGD_DISPATCH_T(m.dtype, HSGD_DISPATCH_D(m.D, hipLaunchKernelGGL((k_render_shift<DT, MD>), dim3((unsigned)nparts),
                                                                        dim3(kSX * kSY), 0, s, m.rgba, m.D, m.H, m.W,
                                                                        v.N, v.warps, v.images, out_rgb, partials,
                                                                        ntx)));
    } else {
        const dim3 grid((unsigned)ceil_div(m.W, kTileW), (unsigned)ceil_div(m.H, kTileH), (unsigned)v.N);
        nparts = (int64_t)grid.x * grid.y * grid.z;
        ProfScope ps(HSGD_K_RENDER, s);
        HSGD_DISPATCH_T(m.dtype, hipLaunchKernelGGL((k_render<DT>), grid, dim3(kBlock), 0, s, m.rgba, m.D,
                                                    m.H, m.W, v.warps, v.images, out_rgb, partials));
    }
    if (out_loss) {
        ProfScope ps(HSGD_K_REDUCE, s);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, nparts, 0.5 / v.N, out_loss);
    }
    return (int)hipGetLastError();
}

int launch_grad_step(const hsgd_mpi& m, const hsgd_views& v, const uint64_t* mask, int kcap,
                     const float* dimg, float lr_rgb, float lr_alpha, float lambda_s, float* grad_out,
                     float* out_loss, float4* slots, float* partials, hipStream_t s) {
    const float prior = (float)((double)lambda_s / ((double)m.D * m.H * m.W));
    const int HW = m.H * m.W;
    const float inv_n = 1.0f / (float)v.N;
    const bool shift = (v.flags & HSGD_VIEWS_SHIFT_ONLY) != 0;
    int64_t nparts;
    int cover_w = 0, cover_h = 0;
    if (grad_out) {
        ProfScope ps(HSGD_K_FILL, s);
        const int64_t n = (int64_t)m.D * HW;
        hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 8192)), dim3(256), 0, s,
                           reinterpret_cast<float4*>(grad_out), n);
    }
    if (shift) {
        const int ntx = (int)ceil_div(m.W + 1, kOX), nty = (int)ceil_div(m.H + 1, kOY);
        cover_w = ntx * kOX;
        cover_h = nty * kOY;
        nparts = (int64_t)ntx * nty * v.N;
        const dim3 grid((unsigned)nparts);
        ProfScope ps(HSGD_K_GRAD, s);
        if (mask) {
            HSGD_DISPATCH_T(m.dtype, HSGD_DISPATCH_D(m.D, hipLaunchKernelGGL((k_grad_shift<DT, MD, true>), grid,
                                                                            dim3(kSX * kSY), 0, s, m.rgba, m.D, m.H, m.W,
                                                                            v.N, v.warps, v.images, dimg, mask, kcap,
                                                                            inv_n, slots, out_loss ? partials : nullptr,
                                                                            ntx)));
        } else {
            HSGD_DISPATCH_T(m.dtype, HSGD_DISPATCH_D(m.D, hipLaunchKernelGGL((k_grad_shift<DT, MD, false>), grid,
                                                                            dim3(kSX * kSY), 0, s, m.rgba, m.D, m.H, m.W,
                                                                            v.N, v.warps, v.images, dimg, mask, kcap,
                                                                            inv_n, slots, out_loss ? partials : nullptr,
                                                                            ntx)));
        }
    } else {
        {
            ProfScope ps(HSGD_K_FILL, s);
            const int64_t n = (int64_t)kcap * HW;
            hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 8192)), dim3(256), 0, s,
                               slots, n);
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
    if (do_update || grad_out || out_loss) {
        ProfScope ps(HSGD_K_UPDATE, s);
        const dim3 grid((unsigned)ceil_div(HW, 256 / kUpdateRS));
        const size_t lds = shift ? sizeof(int2) * (size_t)v.N * m.D : 0;
        HSGD_DISPATCH_T(m.dtype, if (shift) {
            hipLaunchKernelGGL((k_update<DT, true>), grid, dim3(256), lds, s, m.rgba, m.D, m.H, m.W, mask, kcap,
                               slots, v.N, v.warps, cover_w, cover_h, lr_rgb, lr_alpha, do_update,
                               reinterpret_cast<float4*>(grad_out), partials, nparts, 0.5 / v.N, out_loss, prior);
        } else {
            hipLaunchKernelGGL((k_update<DT, false>), grid, dim3(256), 0, s, m.rgba, m.D, m.H, m.W, mask, kcap,
                               slots, 1, v.warps, 0, 0, lr_rgb, lr_alpha, do_update,
                               reinterpret_cast<float4*>(grad_out), partials, nparts, 0.5 / v.N, out_loss, prior);
        });
    }
    return (int)hipGetLastError();
}

int launch_upsample(const hsgd_mpi& c, const hsgd_mpi& f, hipStream_t s) {
    const dim3 grid((unsigned)ceil_div((int64_t)f.H * f.W, 256), (unsigned)c.D);
    ProfScope ps(HSGD_K_UPSAMPLE, s);
    HSGD_DISPATCH_T(c.dtype, hipLaunchKernelGGL((k_upsample<DT>), grid, dim3(256), 0, s, c.rgba, c.H, c.W, f.rgba));
    return (int)hipGetLastError();
}

int launch_upsample_select(const hsgd_mpi& c, const hsgd_mpi& f, int k, float tau, int rule, uint64_t* mask,
                           hipStream_t s) {
    ProfScope ps(HSGD_K_UPSAMPLE, s);
    const dim3 blk((unsigned)ceil_div(c.W, kUpCols), (unsigned)c.H);
    if ((int64_t)blk.x * blk.y >= kUpBlkMinGroups) {
        HSGD_DISPATCH_T(c.dtype, HSGD_DISPATCH_D(c.D, hipLaunchKernelGGL((k_upsample_select_blk<DT, MD>), blk,
                                                                        dim3(64 * kUpWaves), 0, s, c.rgba, c.D, c.H,
                                                                        c.W, f.rgba, k, tau, rule, mask)));
    } else {
        const dim3 grid((unsigned)ceil_div((int64_t)f.H * f.W, 64));
        HSGD_DISPATCH_T(c.dtype, HSGD_DISPATCH_D(c.D, hipLaunchKernelGGL((k_upsample_select<DT, MD>), grid,
                                                                        dim3(64 * kUpWaves), 0, s, c.rgba, c.D, c.H,
                                                                        c.W, f.rgba, k, tau, rule, mask)));
    }
    return (int)hipGetLastError();
}

int launch_pyramid(const float* img, int N, int H, int W, int nl, float* const* out, hipStream_t s) {
    const int hc = H >> nl, wc = W >> nl;
    const dim3 grid((unsigned)ceil_div((int64_t)hc * wc, 256), (unsigned)N);
    ProfScope ps(HSGD_K_DOWNSAMPLE, s);
    if (nl == 1)
        hipLaunchKernelGGL(k_pyramid<1>, grid, dim3(256), 0, s, img, H, W, out[0], nullptr, nullptr);
    else if (nl == 2)
        hipLaunchKernelGGL(k_pyramid<2>, grid, dim3(256), 0, s, img, H, W, out[0], out[1], nullptr);
    else
        hipLaunchKernelGGL(k_pyramid<3>, grid, dim3(256), 0, s, img, H, W, out[0], out[1], out[2]);
    return (int)hipGetLastError();
}

int launch_select_pyramid(const hsgd_mpi& m, int k, float tau, int rule, uint64_t* mask, const float* img, int N,
                          int H, int W, int nl, float* const* out, hipStream_t s) {
    const int HW = m.H * m.W;
    const int nsel = (int)ceil_div(HW, 256);
    const int nbx = (int)ceil_div((int64_t)(H >> nl) * (W >> nl), 256);
    const dim3 grid((unsigned)(nsel + nbx * N));
    ProfScope ps(HSGD_K_SELECT, s);
    HSGD_DISPATCH_T(m.dtype, HSGD_DISPATCH_D(m.D, {
        if (nl == 1)
            hipLaunchKernelGGL((k_select_pyramid<DT, MD, 1>), grid, dim3(256), 0, s, m.rgba, m.D, HW, k, tau, rule,
                               mask, nsel, img, H, W, out[0], nullptr, nullptr, nbx);
        else if (nl == 2)
            hipLaunchKernelGGL((k_select_pyramid<DT, MD, 2>), grid, dim3(256), 0, s, m.rgba, m.D, HW, k, tau, rule,
                               mask, nsel, img, H, W, out[0], out[1], nullptr, nbx);
        else
            hipLaunchKernelGGL((k_select_pyramid<DT, MD, 3>), grid, dim3(256), 0, s, m.rgba, m.D, HW, k, tau, rule,
                               mask, nsel, img, H, W, out[0], out[1], out[2], nbx);
    }));
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

int batch_grad_occupancy(int dtype, int cls) {
    int n = 0;
    hipError_t e = hipSuccess;
    HSGD_DISPATCH_T(dtype, HSGD_DISPATCH_D(cls, e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                                    &n, reinterpret_cast<const void*>(&k_batch_grad<DT, MD>),
                                                    kSX * kSY, 0)));
    return e == hipSuccess ? n : 0;
}

template <int DT>
static void enqueue_batch(const BatchTable* t, const BatchLaunch& c, hipStream_t s) {
    const dim3 small((unsigned)c.grid_small), grad(kSX * kSY);
    for (int stage = 0; stage < kMaxBatchLevels - 1; ++stage)
        hipLaunchKernelGGL(k_batch_down, small, dim3(256), 0, s, t, stage);
    hipLaunchKernelGGL((k_batch_up<DT>), small, dim3(256), 0, s, t);
    HSGD_DISPATCH_D(c.max_d, hipLaunchKernelGGL((k_batch_select<DT, MD>), small, dim3(256), 0, s, t));
    if (c.max_class >= 8)
        hipLaunchKernelGGL((k_batch_grad<DT, 8>), dim3((unsigned)c.grid_grad[0]), grad, 0, s, t, (int)BK_GRAD8);
    if (c.max_class >= 16)
        hipLaunchKernelGGL((k_batch_grad<DT, 16>), dim3((unsigned)c.grid_grad[1]), grad, 0, s, t, (int)BK_GRAD16);
    if (c.max_class >= 32)
        hipLaunchKernelGGL((k_batch_grad<DT, 32>), dim3((unsigned)c.grid_grad[2]), grad, 0, s, t, (int)BK_GRAD32);
    if (c.max_class >= 64)
        hipLaunchKernelGGL((k_batch_grad<DT, 64>), dim3((unsigned)c.grid_grad[3]), grad, 0, s, t, (int)BK_GRAD64);
    const size_t lds = sizeof(int2) * (size_t)c.max_n * c.max_d;
    hipLaunchKernelGGL((k_batch_update<DT>), small, dim3(256), lds, s, t);
}

int launch_batch_step(const BatchTable* t, const BatchLaunch& c, hipStream_t s) {
    if (c.dtype == HSGD_FP32) enqueue_batch<HSGD_FP32>(t, c, s);
    else enqueue_batch<HSGD_BF16>(t, c, s);
    return (int)hipGetLastError();
}
}  // namespace hsgd
