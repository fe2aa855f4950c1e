// Internal declarations shared by the host C++ (hsgd_host.cpp), the ABI layer
// (hsgd_api.hip) and the kernels (hsgd_kernels.hip). Not installed.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/hsgd.h"

namespace hsgd {

constexpr int kMaxD = 64;
constexpr int kMaxN = 64;
constexpr size_t kAlign = 256;

// Tile of one render/gradient workgroup: a 64-wide row per wave, 4 waves.
constexpr int kTileW = 64;
constexpr int kTileH = 4;
constexpr int kBlock = kTileW * kTileH;
// Shift-warp gradient blocks: 64 x 8 rays of which 63 x 7 own a reference cell per plane.
constexpr int kShiftOX = 63;
constexpr int kShiftOY = 7;

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
// select: per (plane, 64-pixel block) counts, plane-major.
struct SelectWs {
    size_t counts_off, seg_off, bytes;
    int64_t nblk, nseg;
};
constexpr int kScanSeg = 4096;  // counts scanned per workgroup
SelectWs select_ws(int D, int H, int W);

// render: one FP32 loss partial per workgroup.
struct RenderWs {
    size_t partial_off, bytes;
    int64_t nparts;
};
RenderWs render_ws(int H, int W, int N);

// grad_step: FP32 gradient slots [H*W][kcap][4] + loss partials.
struct GradWs {
    size_t slots_off, partial_off, bytes;
    int64_t nslots, nparts;
};
GradWs grad_ws(int D, int H, int W, int N, int kcap);

// refine: target pyramid below the finest level, the mask, and the largest select /
// grad_step workspaces (shared region).
struct RefineWs {
    size_t pyr_off[16];
    size_t mask_off, inner_off, bytes;
};
RefineWs refine_ws(int D, int H, int W, int N, int k, int L);

size_t dtype_bytes(int dtype);  // bytes per RGBA voxel, 0 for unknown

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
int launch_select(const hsgd_mpi& m, int k, float tau, uint64_t* mask, int32_t* ids, int cap,
                  int32_t* plane_off, int32_t* n_active, void* ws, hipStream_t s);
int launch_render(const hsgd_mpi& m, const hsgd_views& v, float* out_rgb, float* out_loss,
                  void* ws, hipStream_t s);
int launch_grad_step(const hsgd_mpi& m, const hsgd_views& v, const uint64_t* mask,
                     int kcap, const float* dimg, float lr_rgb, float lr_alpha,
                     float* grad_out, float* out_loss, void* ws, hipStream_t s);
int launch_upsample(const hsgd_mpi& coarse, const hsgd_mpi& fine, hipStream_t s);
int launch_downsample(const float* img, int N, int H, int W, float* out, hipStream_t s);
int launch_convert(const void* src, int sdt, void* dst, int ddt, size_t n, hipStream_t s);

}  // namespace hsgd
