// Internal declarations shared by the host C++ (hsgd_host.cpp), the ABI layer
// (hsgd_api.hip) and the kernels (hsgd_kernels.hip). Not installed.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "hsgd.h"

namespace hsgd {

constexpr int kMaxD = 64;
constexpr int kMaxN = 64;
constexpr size_t kAlign = 256;

// Tile of one render/gradient workgroup: a 64-wide row per wave, 4 waves.
constexpr int kTileW = 64;
constexpr int kTileH = 4;
constexpr int kBlock = kTileW * kTileH;
// Shift-warp gradient blocks: 64 x 8 lanes of which 62 x 7 own a reference cell per plane.
constexpr int kShiftOX = 62;
constexpr int kShiftOY = 7;
// Translation-warp render workgroups: 64 x 8 lanes of which 63 x 8 are rays (lane 63 only
// supplies the right-hand taps of lane 62).
constexpr int kShiftRX = 63;
constexpr int kShiftRY = 8;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---- thread-local error reporting (hsgd_host.cpp) ----
hsgd_status fail(hsgd_status s, const char* fmt, ...);
void clear_error();

// ---- validation helpers (hsgd_host.cpp); each sets the error message on failure ----
hsgd_status check_mpi(const hsgd_mpi* m, const char* what);
hsgd_status check_views(const hsgd_views* v, const hsgd_mpi* m, bool need_images,
                        const char* what);
hsgd_status check_ws(void* ws, size_t ws_bytes, size_t need);

// ---- workspace layouts (hsgd_host.cpp) ----
constexpr int kScanSeg = 4096;  // counts scanned per workgroup

// The active set S as the kernels use it: for every (plane, 64-pixel block) the ballot
// word of selected pixels and the offset of the block in the plane-major compact order,
// the segment totals of the offset scan, the compact linear ids and |S|.
struct ActiveLayout {
    size_t bal_off, off_off, seg_off, ids_off, nact_off, bytes;
    int64_t nblk, nseg, cap;
};
// with_ids = false: the caller provides ids and |S| (hsgd_select_active).
ActiveLayout active_ws(int D, int H, int W, int64_t cap, bool with_ids);

struct ActiveSet {
    uint64_t* bal;
    int* off;
    int* seg;
    int* ids;
    int* nact;
    int64_t nblk, nseg, cap;
};
ActiveSet active_at(void* ws, const ActiveLayout& L, int* ids = nullptr, int* nact = nullptr);

// render: one FP32 loss partial per workgroup.
struct RenderWs {
    size_t partial_off, bytes;
    int64_t nparts;
};
RenderWs render_ws(int H, int W, int N);

// grad_step: FP32 gradient slots, one rank-major slice [kcap][H*W] of float4 per view,
// and the loss partials.
struct GradWs {
    size_t slots_off, partial_off, bytes;
    int64_t nparts;
};
GradWs grad_ws(int D, int H, int W, int N, int kcap);

// refine: the target pyramid below the finest level, the plane mask, then the finest
// level's grad_step workspace (reused by every level).
struct RefineWs {
    size_t pyr_off[16];
    size_t mask_off, inner_off, bytes;
};
RefineWs refine_ws(int D, int H, int W, int N, int k, int L);

size_t dtype_bytes(int dtype);  // bytes per RGBA voxel, 0 for unknown

// ---- refine (hsgd_api.cpp), shared by hsgd_refine and hsgd_refine_noalloc ----
// HSGD_E_HIP with the HIP error text, or HSGD_OK for hipSuccess.
hsgd_status hip_status(int err, const char* what);
// Validates a refine call and reports the workspace bytes it needs; enqueues nothing.
hsgd_status refine_check(const char* fn, const hsgd_mpi* levels, const hsgd_views* views, int32_t L,
                         const int32_t* iters, hsgd_select_params sel, float lr_rgb, float lr_alpha,
                         float lambda_s, size_t* ws_need);
// Enqueues a validated refine with its workspace at ws (refine_ws bytes).
hsgd_status refine_run(const char* fn, hsgd_mpi* levels, const hsgd_views* views, int32_t L, const int32_t* iters,
                       hsgd_select_params sel, float lr_rgb, float lr_alpha, float lambda_s, float* loss_log,
                       void* ws, hipStream_t stream);

// ---- kernel timing (hsgd_profile.cpp) ----
constexpr int kNumKinds = HSGD_K_COUNT;
const char* kind_name(int kind);
// Brackets the launches made during its lifetime with events when profiling is on.
class ProfScope {
  public:
    ProfScope(int kind, hipStream_t s);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

  private:
    int kind_;
    hipStream_t s_;
    void* a_ = nullptr;
    void* b_ = nullptr;
};

// ---- kernel launchers (hsgd_kernels.hip); return hipSuccess or the launch error ----
// select: mask (nullable) and, when as != NULL, the active set (plane_off nullable).
int launch_select(const hsgd_mpi& m, int k, float tau, int rule, uint64_t* mask, const ActiveSet* as,
                  int32_t* plane_off, hipStream_t s);
int launch_render(const hsgd_mpi& m, const hsgd_views& v, float* out_rgb, float* out_loss,
                  void* ws, hipStream_t s);
// mask NULL: every voxel selected (kcap = D); otherwise the first kcap planes of each pixel.
int launch_grad_step(const hsgd_mpi& m, const hsgd_views& v, const uint64_t* mask, int kcap,
                     const float* dimg, float lr_rgb, float lr_alpha, float lambda_s, float* grad_out,
                     float* out_loss, float4* slots, float* partials, hipStream_t s);
int launch_upsample(const hsgd_mpi& coarse, const hsgd_mpi& fine, hipStream_t s);
// upsampling into `fine` fused with the selection on the stored result (mask [H][W])
int launch_upsample_select(const hsgd_mpi& coarse, const hsgd_mpi& fine, int k, float tau, int rule, uint64_t* mask,
                           hipStream_t s);
// nl (1..3) successive 2x2 box means of [N][H][W][3] images in one launch: out[j] receives
// level j + 1 below the input (H and W multiples of 2^nl).
int launch_pyramid(const float* img, int N, int H, int W, int nl, float* const* out, hipStream_t s);
// launch_pyramid and launch_select (mask only, no id list) of an independent level in one launch.
int launch_select_pyramid(const hsgd_mpi& m, int k, float tau, int rule, uint64_t* mask, const float* img, int N,
                          int H, int W, int nl, float* const* out, hipStream_t s);
int launch_downsample(const float* img, int N, int H, int W, float* out, hipStream_t s);
// plane-sweep volume levels 0..L-1 ([N][D][H>>l][W>>l][3] FP32 or BF16; out[l] NULL: not stored)
constexpr int kPsvMaxL = 5;
int launch_plane_sweep(const hsgd_views& src, int D, int L, int out_dtype, void* const* out, hipStream_t s);
int launch_convert(const void* src, int sdt, void* dst, int ddt, size_t n, hipStream_t s);

// ---- batched serving step (hsgd_batch.cpp builds the table, hsgd_kernels.hip runs it) ----
constexpr int kMaxSlots = 16;
constexpr int kMaxBatchLevels = 4;
// The fixed kernel sequence of one batched step; each kernel walks a flat list of work
// items (workgroup-sized pieces) concatenated over the slots it applies to.
enum BatchKernel {
    BK_DOWN0 = 0, BK_DOWN1, BK_DOWN2,            // target pyramid, finest level downwards
    BK_UP,                                        // MPI upsampling into the current level
    BK_SELECT,                                    // plane mask of the current level
    BK_GRAD8, BK_GRAD16, BK_GRAD32, BK_GRAD64,    // gradient tiles, by plane-count class
    BK_UPDATE,                                    // sparse update + loss of the iteration
    BK_COUNT
};

// One in-flight request's work in this step (device-resident, read with scalar loads).
struct BatchSlot {
    void* mpi;                        // current level [D][H][W][4] (updated in place)
    const void* up_src;               // previous level when this step upsamples into mpi
    const float* images;              // current level targets [N][H][W][3]
    const hsgd_warp* warps;           // current level [N][D], shift-only
    uint64_t* mask;                   // [H][W]
    float4* slots;                    // gradient slots [N][kcap][H][W]
    float* partials;                  // loss partials [ntx * nty * N]
    float* loss_out;                  // loss of this iteration (or null)
    const float* pyr_src[kMaxBatchLevels - 1];   // pyramid stages of the first step
    float* pyr_dst[kMaxBatchLevels - 1];
    int pyr_h[kMaxBatchLevels - 1], pyr_w[kMaxBatchLevels - 1];   // source shapes
    int D, H, W, N;
    int uh, uw;                       // upsampling source shape
    int k, kcap, ntx, nty;
    float tau, lr_rgb, lr_alpha;
    int rule;                         // selection rule (HSGD_SELECT_*)
    float prior;                      // sparsity prior weight over D H W of the level
    int pad_[3];
};

struct BatchTable {
    int nslot;
    int pad_[3];
    int total[BK_COUNT];                       // work items per kernel
    int pre[BK_COUNT][kMaxSlots + 1];          // per kernel: items before slot i
    BatchSlot slot[kMaxSlots];
};

struct BatchLaunch {
    int dtype;
    int max_class;                 // largest plane-count class admitted (8, 16, 32 or 64)
    int max_n, max_d;              // bound the update kernel's LDS table
    int grid_small;                // workgroups of the 256-thread kernels
    int grid_grad[4];              // workgroups of the gradient kernels per class
};
// Enqueue the fixed sequence of batched kernels reading `table` (device memory).
int launch_batch_step(const BatchTable* table, const BatchLaunch& cfg, hipStream_t s);
// Workgroups per CU the batched gradient kernel of a class can keep resident.
int batch_grad_occupancy(int dtype, int cls);

}  // namespace hsgd
