// Serving core: continuous batching of HSGD refinements (hsgd_batch_* of hsgd.h).
//
// A request (one frame of a stream) runs the same coarse-to-fine schedule as hsgd_refine:
// its j-th step is iteration t of level l, preceded by the upsampling into level l when
// t == 0 and l > 0, and, at j == 0, by the target pyramid. Each hsgd_batch_step advances
// every request in flight by one such step. The host writes one BatchTable per step (the
// per-request descriptors and, per kernel, the prefix counts of work items), uploads it
// with one copy, and launches the captured graph of the fixed kernel sequence; each
// persistent kernel walks the flat item list, so one graph serves any mix of requests.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "hsgd_internal.h"

using namespace hsgd;

namespace {

constexpr int kRing = 256;        // step events kept for completion queries

struct Slot {
    bool busy = false;
    int64_t ticket = -1;
    hsgd_request req{};
    int step = 0;                  // next step of the request (0 .. total - 1)
    int total = 0;                 // steps of the request = sum(iters)
};

struct Ticket {
    int64_t done_step = -1;        // batch step holding the request's last iteration
};

struct Stream {
    int64_t bytes = 0;
    bool in_flight = false;        // a frame with iterations not yet stepped
};

int maxd_class_host(int D) { return D <= 8 ? 8 : D <= 16 ? 16 : D <= 32 ? 32 : 64; }

struct SlotWs {
    size_t mask_off, slots_off, partial_off, bytes;
};

SlotWs slot_ws(const hsgd_batch_config& c) {
    SlotWs s{};
    const int64_t HW = (int64_t)c.max_H * c.max_W;
    const int64_t ntx = ceil_div(c.max_W + 1, kShiftOX), nty = ceil_div(c.max_H + 1, kShiftOY);
    s.mask_off = 0;
    s.slots_off = align_up(s.mask_off + sizeof(uint64_t) * HW);
    s.partial_off = align_up(s.slots_off + 16 * (size_t)c.max_N * c.max_k * HW);
    s.bytes = align_up(s.partial_off + sizeof(float) * (size_t)ntx * nty * c.max_N);
    return s;
}

size_t table_bytes() { return align_up(sizeof(BatchTable)); }

hsgd_status check_config(const hsgd_batch_config* c) {
    if (!c) return fail(HSGD_E_ARG, "hsgd_batch: config is NULL");
    if (c->max_slots < 1 || c->max_slots > kMaxSlots)
        return fail(HSGD_E_ARG, "hsgd_batch: max_slots=%d outside [1, %d]", c->max_slots, kMaxSlots);
    if (c->max_D < 1 || c->max_D > kMaxD) return fail(HSGD_E_SHAPE, "hsgd_batch: max_D=%d", c->max_D);
    if (c->max_N < 1 || c->max_N > kMaxN) return fail(HSGD_E_SHAPE, "hsgd_batch: max_N=%d", c->max_N);
    if (c->max_H < 2 || c->max_W < 2) return fail(HSGD_E_SHAPE, "hsgd_batch: max_H/max_W below 2");
    if (c->max_k < 1 || c->max_k > c->max_D) return fail(HSGD_E_ARG, "hsgd_batch: max_k=%d", c->max_k);
    if ((int64_t)c->max_k * c->max_H * c->max_W >= ((int64_t)1 << 28))
        return fail(HSGD_E_SHAPE, "hsgd_batch: max_k*max_H*max_W must stay below 2^28");
    if (dtype_bytes(c->dtype) == 0) return fail(HSGD_E_DTYPE, "hsgd_batch: unknown dtype %d", c->dtype);
    if (c->hbm_budget <= 0) return fail(HSGD_E_ARG, "hsgd_batch: hbm_budget must be positive");
    return HSGD_OK;
}

size_t workspace_bytes(const hsgd_batch_config& c) {
    return table_bytes() + (size_t)c.max_slots * slot_ws(c).bytes;
}

// Resident bytes of a stream: every level's MPI, images and warps.
int64_t resident_bytes(const hsgd_request& r) {
    int64_t b = 0;
    for (int l = 0; l < r.L; ++l) {
        const hsgd_mpi& m = r.levels[l];
        b += (int64_t)m.D * m.H * m.W * (int64_t)dtype_bytes(m.dtype);
        b += (int64_t)r.views[l].N * m.H * m.W * 12;
        b += (int64_t)r.views[l].N * m.D * (int64_t)sizeof(hsgd_warp);
    }
    return b;
}

hsgd_status hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return HSGD_OK;
    return fail(HSGD_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

struct hsgd_batch {
    hsgd_batch_config cfg{};
    int device = 0;
    char* ws = nullptr;
    BatchTable* dev_table = nullptr;
    SlotWs sws{};
    BatchLaunch launch{};
    BatchTable* staging[2] = {nullptr, nullptr};     // pinned
    hipEvent_t copy_done[2] = {nullptr, nullptr};
    bool copy_used[2] = {false, false};
    hipEvent_t step_ev[kRing] = {};
    double step_ms[kRing] = {};                       // harvested completion times
    bool step_harvested[kRing] = {};
    hipEvent_t ref = nullptr;
    bool have_ref = false;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture = nullptr;                    // private stream the graph is captured on
    hipStream_t last_stream = nullptr;                // stream of the latest step (valid once steps > 0)
    int64_t steps = 0;
    std::vector<Slot> slots;
    std::vector<Ticket> tickets;
    std::map<int32_t, Stream> streams;
    int64_t used = 0;

    // completion time of step s in ms after the reference, or -1 (blocks on the event)
    double harvest(int64_t s) {
        const int i = (int)(s % kRing);
        if (!step_harvested[i]) {
            hipEventSynchronize(step_ev[i]);
            float ms = -1.0f;
            if (have_ref && hipEventElapsedTime(&ms, ref, step_ev[i]) != hipSuccess) ms = -1.0f;
            step_ms[i] = have_ref ? (double)ms : -1.0;
            step_harvested[i] = true;
        }
        return step_ms[i];
    }
};

namespace {

// (level, iteration within the level) of step j of a request.
void stage_of(const hsgd_request& r, int j, int* level, int* it) {
    int l = 0;
    while (j >= r.iters[l]) {
        j -= r.iters[l];
        ++l;
    }
    *level = l;
    *it = j;
}

void fill_table(hsgd_batch* b, BatchTable* t, std::vector<int>& order) {
    std::memset(t, 0, sizeof(BatchTable));
    const char* base = b->ws + table_bytes();
    int n = 0;
    for (int si : order) {
        const Slot& s = b->slots[si];
        const hsgd_request& r = s.req;
        int l, it;
        stage_of(r, s.step, &l, &it);
        BatchSlot& d = t->slot[n];
        const hsgd_mpi& m = r.levels[l];
        char* sw = const_cast<char*>(base) + (size_t)si * b->sws.bytes;
        d.mpi = m.rgba;
        d.D = m.D;
        d.H = m.H;
        d.W = m.W;
        d.N = r.views[l].N;
        d.images = r.views[l].images;
        d.warps = r.views[l].warps;
        d.mask = reinterpret_cast<uint64_t*>(sw + b->sws.mask_off);
        d.slots = reinterpret_cast<float4*>(sw + b->sws.slots_off);
        d.partials = reinterpret_cast<float*>(sw + b->sws.partial_off);
        d.loss_out = r.loss_log ? r.loss_log + s.step : nullptr;
        d.k = r.sel.k;
        d.kcap = r.sel.k;
        d.tau = r.sel.tau;
        d.rule = r.sel.rule;
        d.prior = (float)((double)r.lambda_s / ((double)m.D * m.H * m.W));
        d.lr_rgb = r.lr_rgb;
        d.lr_alpha = r.lr_alpha;
        d.ntx = (int)ceil_div(m.W + 1, kShiftOX);
        d.nty = (int)ceil_div(m.H + 1, kShiftOY);
        const bool up = it == 0 && l > 0;
        if (up) {
            d.up_src = r.levels[l - 1].rgba;
            d.uh = r.levels[l - 1].H;
            d.uw = r.levels[l - 1].W;
        }
        const bool pyramid = s.step == 0;
        const int64_t HW = (int64_t)m.H * m.W;
        int items[BK_COUNT] = {};
        if (pyramid) {
            for (int st = 0; st < r.L - 1; ++st) {
                const int src = r.L - 1 - st;
                const hsgd_mpi& ms = r.levels[src];
                d.pyr_src[st] = r.views[src].images;
                d.pyr_dst[st] = const_cast<float*>(r.views[src - 1].images);
                d.pyr_h[st] = ms.H;
                d.pyr_w[st] = ms.W;
                items[BK_DOWN0 + st] = r.views[src].N * (int)ceil_div((int64_t)(ms.H / 2) * (ms.W / 2), 256);
            }
        }
        if (up) items[BK_UP] = m.D * (int)ceil_div(4LL * d.uh * d.uw, 256);
        items[BK_SELECT] = (int)ceil_div(HW, 256);
        const int cls = maxd_class_host(m.D);
        const int gk = cls == 8 ? BK_GRAD8 : cls == 16 ? BK_GRAD16 : cls == 32 ? BK_GRAD32 : BK_GRAD64;
        items[gk] = d.ntx * d.nty * d.N;
        items[BK_UPDATE] = (int)ceil_div(HW, 256);
        for (int k = 0; k < BK_COUNT; ++k) {
            t->pre[k][n + 1] = t->pre[k][n] + items[k];
        }
        ++n;
    }
    t->nslot = n;
    for (int k = 0; k < BK_COUNT; ++k) {
        t->total[k] = t->pre[k][n];
        for (int j = n + 1; j <= kMaxSlots; ++j) t->pre[k][j] = t->pre[k][n];
    }
}

}  // namespace

extern "C" {

size_t hsgd_batch_workspace_bytes(const hsgd_batch_config* cfg) {
    clear_error();
    if (check_config(cfg)) return 0;
    return workspace_bytes(*cfg);
}

hsgd_status hsgd_batch_create(const hsgd_batch_config* cfg, void* ws, size_t ws_bytes, hsgd_batch** out) {
    clear_error();
    const char* fn = "hsgd_batch_create";
    if (!out) return fail(HSGD_E_ARG, "%s: out is NULL", fn);
    hsgd_status st = check_config(cfg);
    if (st) return st;
    const size_t need = workspace_bytes(*cfg);
    st = check_ws(ws, ws_bytes, need);
    if (st) return st;
    if ((int64_t)need > cfg->hbm_budget)
        return fail(HSGD_E_BUDGET, "%s: workspace (%zu bytes) exceeds the budget", fn, need);
    hsgd_batch* b = new hsgd_batch();
    b->cfg = *cfg;
    b->ws = reinterpret_cast<char*>(ws);
    b->dev_table = reinterpret_cast<BatchTable*>(ws);
    b->sws = slot_ws(*cfg);
    b->slots.resize(cfg->max_slots);
    b->used = (int64_t)need;
    hipError_t e = hipGetDevice(&b->device);
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->staging[i]), sizeof(BatchTable), hipHostMallocDefault);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&b->copy_done[i], hipEventDisableTiming);
    for (int i = 0; i < kRing && e == hipSuccess; ++i) e = hipEventCreate(&b->step_ev[i]);
    if (e == hipSuccess) e = hipEventCreate(&b->ref);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        hsgd_batch_destroy(b);
        return hip_status(e, fn);
    }
    BatchLaunch& L = b->launch;
    L.dtype = cfg->dtype;
    L.max_class = maxd_class_host(cfg->max_D);
    L.max_n = cfg->max_N;
    L.max_d = cfg->max_D;
    // persistent grids: whole multiples of the CU count (so of the 8 XCDs)
    L.grid_small = 8 * cus;
    const int classes[4] = {8, 16, 32, 64};
    for (int c = 0; c < 4; ++c) {
        const int occ = classes[c] <= L.max_class ? batch_grad_occupancy(cfg->dtype, classes[c]) : 1;
        L.grid_grad[c] = (occ > 0 ? occ : 1) * cus;
    }
    *out = b;
    return HSGD_OK;
}

hsgd_status hsgd_batch_destroy(hsgd_batch* b) {
    clear_error();
    if (!b) return HSGD_OK;
    for (int i = 0; i < kRing; ++i)
        if (b->step_ev[i]) hipEventSynchronize(b->step_ev[i]);
    for (int i = 0; i < 2; ++i) {
        if (b->copy_done[i]) hipEventSynchronize(b->copy_done[i]);
        if (b->copy_done[i]) hipEventDestroy(b->copy_done[i]);
        if (b->staging[i]) hipHostFree(b->staging[i]);
    }
    for (int i = 0; i < kRing; ++i)
        if (b->step_ev[i]) hipEventDestroy(b->step_ev[i]);
    if (b->ref) hipEventDestroy(b->ref);
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->capture) hipStreamDestroy(b->capture);
    delete b;
    return HSGD_OK;
}

hsgd_status hsgd_batch_admit(hsgd_batch* b, const hsgd_request* r, int64_t* ticket) {
    clear_error();
    const char* fn = "hsgd_batch_admit";
    if (!b || !r || !ticket) return fail(HSGD_E_ARG, "%s: NULL pointer", fn);
    const hsgd_batch_config& c = b->cfg;
    if (r->stream_id < 0) return fail(HSGD_E_ARG, "%s: stream_id < 0", fn);
    if (r->L < 1 || r->L > kMaxBatchLevels) return fail(HSGD_E_ARG, "%s: L=%d outside [1, %d]", fn, r->L, kMaxBatchLevels);
    hsgd_status st;
    int total = 0;
    for (int l = 0; l < r->L; ++l) {
        st = check_mpi(&r->levels[l], fn);
        if (st) return st;
        st = check_views(&r->views[l], &r->levels[l], true, fn);
        if (st) return st;
        if (!(r->views[l].flags & HSGD_VIEWS_SHIFT_ONLY))
            return fail(HSGD_E_ARG, "%s: level %d warps are not shift-only (batched path)", fn, l);
        if (r->levels[l].dtype != c.dtype) return fail(HSGD_E_DTYPE, "%s: MPI dtype differs from the batch's", fn);
        if (r->iters[l] < 0 || (l > 0 && r->iters[l] < 1))
            return fail(HSGD_E_ARG, "%s: iters[%d]=%d (levels above 0 need >= 1)", fn, l, r->iters[l]);
        total += r->iters[l];
        if (l > 0) {
            const hsgd_mpi& p = r->levels[l - 1];
            const hsgd_mpi& f = r->levels[l];
            if (f.D != p.D || f.H != 2 * p.H || f.W != 2 * p.W)
                return fail(HSGD_E_SHAPE, "%s: level %d is not 2x level %d", fn, l, l - 1);
            if (r->views[l].N != r->views[0].N) return fail(HSGD_E_SHAPE, "%s: view count differs by level", fn);
            if (f.rgba == p.rgba || r->views[l].images == r->views[l - 1].images)
                return fail(HSGD_E_ARG, "%s: levels %d and %d alias", fn, l - 1, l);
        }
    }
    if (total < 1) return fail(HSGD_E_ARG, "%s: no iterations", fn);
    const hsgd_mpi& top = r->levels[r->L - 1];
    if (top.D > c.max_D || top.H > c.max_H || top.W > c.max_W || r->views[0].N > c.max_N)
        return fail(HSGD_E_SHAPE, "%s: frame %dx%dx%d with %d views exceeds the batch's limits", fn, top.W, top.H,
                    top.D, r->views[0].N);
    if (r->sel.k < 1 || r->sel.k > top.D || r->sel.k > c.max_k)
        return fail(HSGD_E_ARG, "%s: k=%d outside [1, min(D, max_k)]", fn, r->sel.k);
    if (std::isnan(r->sel.tau)) return fail(HSGD_E_ARG, "%s: tau is NaN", fn);
    if (r->sel.rule != HSGD_SELECT_TOPK && r->sel.rule != HSGD_SELECT_MVS)
        return fail(HSGD_E_ARG, "%s: unknown selection rule %d", fn, r->sel.rule);
    if (!std::isfinite(r->lr_rgb) || !std::isfinite(r->lr_alpha) || !std::isfinite(r->lambda_s))
        return fail(HSGD_E_ARG, "%s: learning rates and lambda_s must be finite", fn);

    auto it = b->streams.find(r->stream_id);
    if (it != b->streams.end() && it->second.in_flight)
        return fail(HSGD_E_CAPACITY, "%s: stream %d has a frame in flight", fn, r->stream_id);
    int free_slot = -1;
    for (int i = 0; i < c.max_slots; ++i)
        if (!b->slots[i].busy) {
            free_slot = i;
            break;
        }
    if (free_slot < 0) return fail(HSGD_E_CAPACITY, "%s: all %d slots busy", fn, c.max_slots);
    const int64_t bytes = resident_bytes(*r);
    if (it == b->streams.end()) {
        if (b->used + bytes > c.hbm_budget)
            return fail(HSGD_E_BUDGET, "%s: stream %d needs %lld bytes, %lld of %lld in use", fn, r->stream_id,
                        (long long)bytes, (long long)b->used, (long long)c.hbm_budget);
        Stream s;
        s.bytes = bytes;
        it = b->streams.emplace(r->stream_id, s).first;
        b->used += bytes;
    } else if (bytes != it->second.bytes) {
        return fail(HSGD_E_SHAPE, "%s: stream %d changed its buffers' sizes", fn, r->stream_id);
    }
    it->second.in_flight = true;
    Slot& s = b->slots[free_slot];
    s.busy = true;
    s.req = *r;
    s.step = 0;
    s.total = total;
    s.ticket = (int64_t)b->tickets.size();
    b->tickets.push_back(Ticket{});
    *ticket = s.ticket;
    return HSGD_OK;
}

hsgd_status hsgd_batch_step(hsgd_batch* b, hipStream_t stream, int32_t* n_active, int64_t* finished,
                            int32_t max_finished, int32_t* n_finished) {
    clear_error();
    const char* fn = "hsgd_batch_step";
    if (!b) return fail(HSGD_E_ARG, "%s: batch is NULL", fn);
    if (n_active) *n_active = 0;
    if (n_finished) *n_finished = 0;
    std::vector<int> order;
    for (int i = 0; i < b->cfg.max_slots; ++i)
        if (b->slots[i].busy) order.push_back(i);
    if (order.empty()) return HSGD_OK;

    const int cur = (int)(b->steps & 1);
    hipError_t e = hipSuccess;
    if (b->copy_used[cur]) e = hipEventSynchronize(b->copy_done[cur]);   // the step before last
    if (e != hipSuccess) return hip_status(e, fn);
    // the ring entry about to be reused: keep its completion time
    const int64_t old = b->steps - kRing;
    if (old >= 0) b->harvest(old);
    // Every step rewrites the one device table and continues the requests of the step
    // before it: on a stream other than that step's, wait for that step to finish first.
    if (b->steps > 0 && stream != b->last_stream) {
        e = hipStreamWaitEvent(stream, b->step_ev[(int)((b->steps - 1) % kRing)], 0);
        if (e != hipSuccess) return hip_status(e, fn);
    }
    fill_table(b, b->staging[cur], order);
    e = hipMemcpyAsync(b->dev_table, b->staging[cur], sizeof(BatchTable), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(b->copy_done[cur], stream);
    if (e != hipSuccess) return hip_status(e, fn);
    b->copy_used[cur] = true;
    if (!b->exec) {
        // captured once on the private stream (the caller's may be the legacy default
        // stream, which cannot capture); launched on the caller's stream every step
        hipGraph_t g = nullptr;
        e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_status(e, fn);
        const int le = launch_batch_step(b->dev_table, b->launch, b->capture);
        e = hipStreamEndCapture(b->capture, &g);
        if (le != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return hip_status((hipError_t)le, fn);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (g) hipGraphDestroy(g);
        if (e != hipSuccess) return hip_status(e, fn);
    }
    e = hipGraphLaunch(b->exec, stream);
    const int ri = (int)(b->steps % kRing);
    if (e == hipSuccess) e = hipEventRecord(b->step_ev[ri], stream);
    if (e != hipSuccess) return hip_status(e, fn);
    b->step_harvested[ri] = false;
    b->last_stream = stream;

    int nf = 0;
    for (int si : order) {
        Slot& s = b->slots[si];
        if (++s.step == s.total) {
            b->tickets[s.ticket].done_step = b->steps;
            b->streams[s.req.stream_id].in_flight = false;
            s.busy = false;
            if (finished && nf < max_finished) finished[nf] = s.ticket;
            ++nf;
        }
    }
    ++b->steps;
    if (n_active) *n_active = (int32_t)order.size();
    if (n_finished) *n_finished = nf < max_finished ? nf : max_finished;
    return HSGD_OK;
}

hsgd_status hsgd_batch_reference(hsgd_batch* b, hipStream_t stream) {
    clear_error();
    if (!b) return fail(HSGD_E_ARG, "hsgd_batch_reference: batch is NULL");
    hipError_t e = hipEventRecord(b->ref, stream);
    if (e == hipSuccess) e = hipEventSynchronize(b->ref);
    if (e != hipSuccess) return hip_status(e, "hsgd_batch_reference");
    b->have_ref = true;
    return HSGD_OK;
}

hsgd_status hsgd_batch_poll(hsgd_batch* b, int64_t ticket, int32_t* done, double* done_ms) {
    clear_error();
    const char* fn = "hsgd_batch_poll";
    if (!b || !done) return fail(HSGD_E_ARG, "%s: NULL pointer", fn);
    if (ticket < 0 || ticket >= (int64_t)b->tickets.size()) return fail(HSGD_E_ARG, "%s: unknown ticket", fn);
    *done = 0;
    if (done_ms) *done_ms = -1.0;
    const int64_t s = b->tickets[ticket].done_step;
    if (s < 0) return HSGD_OK;
    if (s + kRing <= b->steps - 1) {           // its ring entry was reused: harvested then
        *done = 1;
        return HSGD_OK;
    }
    const int i = (int)(s % kRing);
    if (!b->step_harvested[i]) {
        const hipError_t q = hipEventQuery(b->step_ev[i]);
        if (q == hipErrorNotReady) return HSGD_OK;
        if (q != hipSuccess) return hip_status(q, fn);
    }
    *done = 1;
    if (done_ms) *done_ms = b->harvest(s);
    return HSGD_OK;
}

hsgd_status hsgd_batch_release_stream(hsgd_batch* b, int32_t stream_id) {
    clear_error();
    if (!b) return fail(HSGD_E_ARG, "hsgd_batch_release_stream: batch is NULL");
    auto it = b->streams.find(stream_id);
    if (it == b->streams.end()) return HSGD_OK;
    if (it->second.in_flight)
        return fail(HSGD_E_CAPACITY, "hsgd_batch_release_stream: stream %d has a frame in flight", stream_id);
    b->used -= it->second.bytes;
    b->streams.erase(it);
    return HSGD_OK;
}

int64_t hsgd_batch_budget_used(const hsgd_batch* b) { return b ? b->used : 0; }

}  // extern "C"
