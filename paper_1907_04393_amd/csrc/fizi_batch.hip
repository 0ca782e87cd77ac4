// C ABI of the batched form: many camera streams of uneven resolution, one
// pipeline pass over all of them per frame step (include/fizi.h).
#include <algorithm>
#include <initializer_list>
#include <cstring>
#include <new>
#include <vector>

#include "fizi_host.h"

using namespace fizi;

struct fizi_batch {
    int n = 0;
    std::vector<Model> m;
    std::vector<Slot> slot;
    std::vector<uint64_t> frames;      // frames stepped per stream
    std::vector<uint32_t> epoch;       // dispatches per stream slot (band flag values)
    Tuning tune{};
    int max_wd = 0, max_ops = 0;
    uint8_t *d = nullptr;
    int device = 0, n_cu = 0;
    TableRing ring;
    StageClock clk;
    int mode = FIZI_BATCH_DIRECT;
    hipStream_t cap = nullptr;                 // capture stream for graphs
    hipGraphExec_t graph[kTabSlots] = {};
    uint8_t *persist = nullptr;                // fused-kernel barrier state
    hipEvent_t order_ev = nullptr;
    hipStream_t last_stream = nullptr;
    bool have_last = false;
    // pipelined modes: a second raw-mask buffer per stream (steps alternate
    // between the two, so that a step's classify never writes the bits its
    // predecessor's morphology is reading), the side stream of the back
    // halves and the stream of the table uploads, and per step parity the
    // events that order them
    std::vector<uint64_t *> raw2;
    int parity = 0;
    // graph form: the step whose back half is still to be enqueued
    int pend_slot = -1, pend_jobs = 0;
    // direct form: the parity of the step whose back half is enqueued on the
    // side stream but not yet joined to a caller's stream
    int pend_join = -1;
    hipStream_t side = nullptr, up = nullptr;
    hipEvent_t fork_ev = nullptr;
    hipEvent_t up_ev[2] = {}, cls_ev[2] = {}, join_ev[2] = {};
    hipGraphExec_t pgraph[kTabSlots][kTabSlots + 1] = {};   // by (slot, pending slot + 1)
};

namespace {

struct BatchLayout {
    size_t tables, persist;
    std::vector<size_t> model, slot, raw2;
    size_t total;
};

bool is_pipelined(int mode) { return mode == FIZI_BATCH_PIPELINED || mode == FIZI_BATCH_PIPELINED_GRAPH; }
bool is_persistent(int mode) { return mode == FIZI_BATCH_PERSISTENT || mode == FIZI_BATCH_PERSISTENT_GRAPH; }

// How much faster than the current shape an autotuner candidate must be.
constexpr double kTuneMargin = 0.01;

int check_streams(int32_t n, const fizi_geom *geoms, const fizi_params *params)
{
    if (n < 1 || n > kMaxJobs)
        return fail(FIZI_EINVAL, "n_streams must be in [1, 256]");
    if (!geoms || !params)
        return fail(FIZI_EINVAL, "null geometry or parameter array");
    for (int i = 0; i < n; ++i)
        FIZI_TRY(validate(&geoms[i], &params[i]));
    return FIZI_OK;
}

BatchLayout batch_layout(int32_t n, const fizi_geom *geoms, const fizi_params *params)
{
    BatchLayout L;
    size_t off = 0;
    L.tables = off;
    off += TableRing::device_bytes();
    L.persist = off;
    off += align256(persist_state_bytes());
    L.model.resize(n);
    L.slot.resize(n);
    L.raw2.resize(n);
    for (int i = 0; i < n; ++i) {
        L.model[i] = off;
        off += align256(model_bytes(geoms[i], params[i]));
        L.slot[i] = off;
        off += align256(slot_bytes(geoms[i]));
        L.raw2[i] = off;
        off += align256((size_t)geoms[i].height * (geoms[i].width / 64) * 8);
    }
    L.total = align256(off);
    return L;
}

int order_after_previous(fizi_batch *b, hipStream_t s)
{
    if (b->have_last && b->last_stream != s)
        FIZI_HIP(hipStreamWaitEvent(s, b->order_ev, 0));
    return FIZI_OK;
}

int mark_last(fizi_batch *b, hipStream_t s)
{
    FIZI_HIP(hipEventRecord(b->order_ev, s));
    b->last_stream = s;
    b->have_last = true;
    return FIZI_OK;
}

// Enqueues the table upload and the pipeline of one step on s (direct or
// persistent mode) with launch shapes that do not depend on the active set.
int enqueue_step(fizi_batch *b, int slot, int njobs, bool fixed, hipStream_t s, StageClock *clk)
{
    const Table &T = *b->ring.h[slot];
    FIZI_HIP(hipMemcpyAsync(b->ring.d[slot], &T, table_bytes(fixed ? b->n : njobs),
                            hipMemcpyHostToDevice, s));
    if (b->mode == FIZI_BATCH_PERSISTENT) {
        FIZI_HIP(launch_persistent(b->ring.d[slot], b->max_wd, b->max_ops, b->n_cu, b->tune, b->persist, s,
                                   clk ? clk->next(FIZI_STAGE_CLASSIFY) : StageEvents{}));
        return FIZI_OK;
    }
    return run_pipeline(b->ring.d[slot], T, njobs, b->n, b->max_wd, b->max_ops, b->tune, b->n_cu, fixed, s,
                        clk);
}

// Pipelined step, graph form: the table upload, gain and classify of `slot`
// on s and beside them, on the side stream, the morphology and components of
// the pending step `pend` (none when negative); s then waits for the side
// stream. The two halves touch disjoint memory: the front reads frames and
// models and writes this step's raw bits and gain sums; the back reads the
// other raw buffer and writes I_FIZI, the component scratch and the pointers.
int enqueue_pipelined(fizi_batch *b, int slot, int njobs, int pend, int pend_jobs, bool fixed, hipStream_t s,
                      hipStream_t side, StageClock *clk)
{
    const Table &T = *b->ring.h[slot];
    if (pend >= 0) {
        FIZI_HIP(hipEventRecord(b->fork_ev, s));
        FIZI_HIP(hipStreamWaitEvent(side, b->fork_ev, 0));
        FIZI_TRY(run_back(b->ring.d[pend], *b->ring.h[pend], pend_jobs, b->n, b->max_wd, b->max_ops, b->tune,
                          b->n_cu, fixed, side, clk, true));
        FIZI_HIP(hipEventRecord(b->join_ev[0], side));
    }
    FIZI_HIP(hipMemcpyAsync(b->ring.d[slot], &T, table_bytes(fixed ? b->n : njobs), hipMemcpyHostToDevice, s));
    FIZI_TRY(run_front(b->ring.d[slot], T, njobs, b->tune, b->n_cu, fixed, s, clk));
    if (pend >= 0)
        FIZI_HIP(hipStreamWaitEvent(s, b->join_ev[0], 0));
    return FIZI_OK;
}

int side_streams(fizi_batch *b)
{
    if (!b->side)
        FIZI_HIP(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
    if (!b->up)
        FIZI_HIP(hipStreamCreateWithFlags(&b->up, hipStreamNonBlocking));
    return FIZI_OK;
}

// Pipelined step, direct form. The table goes up on its own stream (it
// depends on nothing the device does), gain and classify follow on s, and
// the back half is enqueued at once on the side stream behind classify:
// it starts when classify ends, whether or not the next step has been
// called, and runs beside the next step's gain and classify. s joins the
// PREVIOUS step's back half after this classify (done by then, unless the
// back half is the longer one), so the outputs of a step are ordered on s
// after the next step, and the next classify never writes the raw buffer
// that back half reads.
int enqueue_pipelined_direct(fizi_batch *b, int slot, int njobs, hipStream_t s, StageClock *clk)
{
    const Table &T = *b->ring.h[slot];
    const int par = b->parity;
    FIZI_TRY(side_streams(b));
    FIZI_HIP(hipMemcpyAsync(b->ring.d[slot], &T, table_bytes(njobs), hipMemcpyHostToDevice, b->up));
    FIZI_HIP(hipEventRecord(b->up_ev[par], b->up));
    FIZI_HIP(hipStreamWaitEvent(s, b->up_ev[par], 0));
    FIZI_TRY(run_front(b->ring.d[slot], T, njobs, b->tune, b->n_cu, false, s, clk));
    FIZI_HIP(hipEventRecord(b->cls_ev[par], s));
    FIZI_HIP(hipStreamWaitEvent(b->side, b->cls_ev[par], 0));
    FIZI_TRY(run_back(b->ring.d[slot], T, njobs, b->n, b->max_wd, b->max_ops, b->tune, b->n_cu, false, b->side,
                      clk, true));
    FIZI_HIP(hipEventRecord(b->join_ev[par], b->side));
    FIZI_TRY(b->ring.finish(slot, b->side));
    if (b->pend_join >= 0)
        FIZI_HIP(hipStreamWaitEvent(s, b->join_ev[b->pend_join], 0));
    b->pend_join = par;
    return FIZI_OK;
}

// Graph of a pipelined step (slot, pending slot or -1), captured once: the
// capture forks onto the side stream and joins back.
int pgraph_for(fizi_batch *b, int slot, int pend)
{
    hipGraphExec_t &ge = b->pgraph[slot][pend + 1];
    if (ge)
        return FIZI_OK;
    if (!b->cap)
        FIZI_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    FIZI_TRY(side_streams(b));
    FIZI_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
    const int rc = enqueue_pipelined(b, slot, b->n, pend, b->n, true, b->cap, b->side, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc != FIZI_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return rc;
    }
    FIZI_HIP(e);
    const hipError_t e2 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    FIZI_HIP(e2);
    return FIZI_OK;
}

// Makes every step's outputs complete on s: enqueues the graph form's
// pending back half there, or joins the direct form's side stream.
int flush_pending(fizi_batch *b, hipStream_t s)
{
    if (b->pend_slot < 0 && b->pend_join < 0)
        return FIZI_OK;
    FIZI_TRY(order_after_previous(b, s));
    if (b->pend_slot >= 0) {
        const int p = b->pend_slot;
        FIZI_TRY(run_back(b->ring.d[p], *b->ring.h[p], b->pend_jobs, b->n, b->max_wd, b->max_ops, b->tune,
                          b->n_cu, false, s, &b->clk));
        b->pend_slot = -1;
        FIZI_TRY(b->ring.finish(p, s));
    }
    if (b->pend_join >= 0) {
        FIZI_HIP(hipStreamWaitEvent(s, b->join_ev[b->pend_join], 0));
        b->pend_join = -1;
    }
    return mark_last(b, s);
}

// Flushes on the stream of the last call and waits for all of the batch's work.
int drain(fizi_batch *b)
{
    if (b->pend_slot >= 0 || b->pend_join >= 0)
        FIZI_TRY(flush_pending(b, b->last_stream));
    if (b->have_last)
        FIZI_HIP(hipEventSynchronize(b->order_ev));
    return FIZI_OK;
}

// Graph of one table slot: upload + pipeline, captured once.
int graph_for(fizi_batch *b, int slot)
{
    if (b->graph[slot])
        return FIZI_OK;
    if (!b->cap)
        FIZI_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    FIZI_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
    const int rc = enqueue_step(b, slot, b->n, true, b->cap, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc != FIZI_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return rc;
    }
    FIZI_HIP(e);
    const hipError_t e2 = hipGraphInstantiate(&b->graph[slot], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    FIZI_HIP(e2);
    return FIZI_OK;
}

void drop_graphs(fizi_batch *b)
{
    for (int i = 0; i < kTabSlots; ++i) {
        if (b->graph[i]) {
            (void)hipGraphExecDestroy(b->graph[i]);
            b->graph[i] = nullptr;
        }
        for (int p = 0; p <= kTabSlots; ++p)
            if (b->pgraph[i][p]) {
                (void)hipGraphExecDestroy(b->pgraph[i][p]);
                b->pgraph[i][p] = nullptr;
            }
    }
}

}  // namespace

extern "C" {

size_t fizi_batch_state_bytes(int32_t n_streams, const fizi_geom *geoms, const fizi_params *params)
{
    if (check_streams(n_streams, geoms, params) != FIZI_OK)
        return 0;
    return batch_layout(n_streams, geoms, params).total;
}

int fizi_batch_create(int32_t n_streams, const fizi_geom *geoms, const fizi_params *params, void *d_state,
                      size_t state_bytes, fizi_batch **out)
{
    FIZI_TRY(check_streams(n_streams, geoms, params));
    if (!d_state || !out)
        return fail(FIZI_EINVAL, "null d_state or out");
    if (reinterpret_cast<uintptr_t>(d_state) % 256 != 0)
        return fail(FIZI_EINVAL, "d_state must be 256-byte aligned");
    const BatchLayout L = batch_layout(n_streams, geoms, params);
    if (state_bytes < L.total)
        return fail(FIZI_ENOMEM, "state block smaller than fizi_batch_state_bytes()");
    fizi_batch *b = new (std::nothrow) fizi_batch();
    if (!b)
        return fail(FIZI_ENOMEM, "host allocation failed");
    b->n = n_streams;
    b->d = static_cast<uint8_t *>(d_state);
    b->m.resize(n_streams);
    b->slot.resize(n_streams);
    b->frames.assign(n_streams, 0);
    b->epoch.assign(n_streams, 0);
    b->raw2.resize(n_streams);
    int max_w = 0;
    for (int i = 0; i < n_streams; ++i) {
        model_at(b->m[i], geoms[i], params[i], b->d + L.model[i]);
        b->slot[i] = slot_at(geoms[i], b->d + L.slot[i]);
        b->raw2[i] = reinterpret_cast<uint64_t *>(b->d + L.raw2[i]);
        max_w = std::max(max_w, geoms[i].width);
        b->max_ops = std::max(b->max_ops, morph_ops(params[i]));
    }
    b->max_wd = max_w / 64;
    b->tune = tuning_for(max_w, b->max_ops, true);
    b->persist = b->d + L.persist;
    int rc = device_cu_count(&b->device, &b->n_cu);
    if (rc == FIZI_OK)
        rc = b->ring.init(b->d + L.tables);
    if (rc == FIZI_OK) {
        hipError_t e = hipEventCreateWithFlags(&b->order_ev, kDeviceOrderEvent);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&b->fork_ev, kDeviceOrderEvent);
        for (int k = 0; k < 2 && e == hipSuccess; ++k) {
            e = hipEventCreateWithFlags(&b->up_ev[k], hipEventDisableTiming);
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&b->cls_ev[k], kDeviceOrderEvent);
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&b->join_ev[k], kDeviceOrderEvent);
        }
        if (e == hipSuccess)
            e = (hipError_t)launch_fill_u32(reinterpret_cast<uint32_t *>(b->persist), 0u,
                                             persist_state_bytes() / 4, nullptr);
        // band flags hold no epoch yet (epochs start at 1)
        for (int i = 0; i < n_streams && e == hipSuccess; ++i)
            e = (hipError_t)launch_fill_u32(b->slot[i].bflag, 0u, b->slot[i].nflags, nullptr);
        if (e == hipSuccess)
            e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess)
            rc = fail(FIZI_EHIP, std::string("fizi_batch_create: ") + hipGetErrorString(e));
    }
    if (rc != FIZI_OK) {
        const std::string msg = fizi_last_error();
        fizi_batch_destroy(b);
        return fail(rc, msg);
    }
    *out = b;
    return FIZI_OK;
}

int fizi_batch_learn(fizi_batch *b, int32_t stream_id, const uint8_t *d_frames, int32_t n_frames, int32_t reset,
                     void *stream)
{
    if (!b || !d_frames)
        return fail(FIZI_EINVAL, "null batch or frames");
    if (reinterpret_cast<uintptr_t>(d_frames) % 4 != 0)
        return fail(FIZI_EINVAL, "frames must be 4-byte aligned");
    if (stream_id < 0 || stream_id >= b->n)
        return fail(FIZI_EINVAL, "stream_id out of range");
    if (n_frames < 1)
        return fail(FIZI_EINVAL, "n_frames must be >= 1");
    Model &m = b->m[stream_id];
    if (!reset && !m.learned)
        return fail(FIZI_ESTATE, "learning without reset needs a learned model");
    hipStream_t s = static_cast<hipStream_t>(stream);
    FIZI_TRY(flush_pending(b, s));
    FIZI_TRY(order_after_previous(b, s));
    FIZI_TRY(learn_model(m, b->ring, b->tune, b->n_cu, d_frames, n_frames, reset, s, &b->clk));
    return mark_last(b, s);
}

int fizi_batch_relearn(fizi_batch *b, int32_t stream_id, const uint8_t *d_frames, int32_t n_frames,
                       const uint64_t *d_fizi_bits, void *stream)
{
    if (!b || !d_frames || !d_fizi_bits)
        return fail(FIZI_EINVAL, "null batch, frames or masks");
    if (reinterpret_cast<uintptr_t>(d_frames) % 4 != 0 || reinterpret_cast<uintptr_t>(d_fizi_bits) % 8 != 0)
        return fail(FIZI_EINVAL, "frames must be 4-byte and masks 8-byte aligned");
    if (stream_id < 0 || stream_id >= b->n)
        return fail(FIZI_EINVAL, "stream_id out of range");
    if (n_frames < 1)
        return fail(FIZI_EINVAL, "n_frames must be >= 1");
    Model &m = b->m[stream_id];
    if (!m.learned)
        return fail(FIZI_ESTATE, "relearning needs a learned model");
    hipStream_t s = static_cast<hipStream_t>(stream);
    FIZI_TRY(flush_pending(b, s));
    FIZI_TRY(order_after_previous(b, s));
    FIZI_TRY(learn_model(m, b->ring, b->tune, b->n_cu, d_frames, n_frames, 0, s, &b->clk, d_fizi_bits));
    return mark_last(b, s);
}

int fizi_batch_set_tracking(fizi_batch *b, int32_t stream_id, int32_t enable)
{
    if (!b)
        return fail(FIZI_EINVAL, "null batch");
    if (stream_id < 0 || stream_id >= b->n)
        return fail(FIZI_EINVAL, "stream_id out of range");
    FIZI_TRY(drain(b));
    Model &m = b->m[stream_id];
    FIZI_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(m.track), 0u, sizeof(TrackState) / 4, nullptr));
    FIZI_HIP(hipStreamSynchronize(nullptr));
    m.tracking = enable != 0;
    return FIZI_OK;
}

int fizi_batch_set_mode(fizi_batch *b, int32_t mode)
{
    if (!b)
        return fail(FIZI_EINVAL, "null batch");
    if (mode < FIZI_BATCH_DIRECT || mode > FIZI_BATCH_PIPELINED_GRAPH)
        return fail(FIZI_EINVAL, "unknown batch mode");
    FIZI_TRY(drain(b));
    if (is_persistent(mode) != is_persistent(b->mode))
        drop_graphs(b);
    b->mode = mode;
    return FIZI_OK;
}

int fizi_batch_step(fizi_batch *b, const uint8_t *const *h_frames, uint64_t *const *h_fizi_bits,
                    fizi_pointer *d_pointers, void *stream)
{
    if (!b || !h_frames || !d_pointers)
        return fail(FIZI_EINVAL, "null batch, frame array or pointer array");
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < b->n; ++i) {
        if (h_frames[i] && !b->m[i].learned)
            return fail(FIZI_ESTATE, "a stream in the step has no learned background");
        if (reinterpret_cast<uintptr_t>(h_frames[i]) % 4 != 0)
            return fail(FIZI_EINVAL, "frames must be 4-byte aligned");
    }
    FIZI_TRY(order_after_previous(b, s));
    int slot;
    FIZI_TRY(b->ring.take(&slot));
    Table &T = *b->ring.h[slot];
    const bool pipelined = is_pipelined(b->mode);
    // a step too small to fill the device (a few active streams, as in
    // serving) takes the contexts' short morphology bands when the four
    // kernels run it; the persistent step keeps the tuned bands
    size_t short_waves = 0;
    for (int i = 0; i < b->n; ++i)
        if (h_frames[i])
            short_waves += (size_t)((b->m[i].g.height + kShortBand - 1) / kShortBand);
    const bool short_chain =
        b->tune.short_bands && !is_persistent(b->mode) && short_waves <= (size_t)b->n_cu * 4;
    int k = 0;
    for (int i = 0; i < b->n; ++i) {
        if (!h_frames[i])
            continue;
        Job &J = T.jobs[k++];
        if (short_chain)
            fill_job(b->m[i], kShortBand, J, false);
        else
            fill_job(b->m[i], b->tune.morph_rows, J);
        set_scratch(J, b->slot[i]);
        if (pipelined && b->parity)
            J.raw = b->raw2[i];
        J.frame = h_frames[i];
        if (h_fizi_bits && h_fizi_bits[i])
            J.fizi = h_fizi_bits[i];
        J.out = d_pointers + i;
        J.frame_index = b->frames[i]++;
        if (++b->epoch[i] == 0)
            b->epoch[i] = 1;
        J.epoch = b->epoch[i];
    }
    set_prefixes(T, k, b->tune);
    if (pipelined) {
        if (k == 0) {
            FIZI_TRY(b->ring.finish(slot, s));
            return mark_last(b, s);
        }
        if (b->mode == FIZI_BATCH_PIPELINED) {
            FIZI_TRY(enqueue_pipelined_direct(b, slot, k, s, &b->clk));
            b->parity ^= 1;
            return mark_last(b, s);
        }
        const int pend = b->pend_slot;
        FIZI_TRY(pgraph_for(b, slot, pend));
        FIZI_HIP(hipGraphLaunch(b->pgraph[slot][pend + 1], s));
        b->parity ^= 1;
        // the pending step's table was read until the join: its slot is
        // reusable after this call
        if (pend >= 0)
            FIZI_TRY(b->ring.finish(pend, s));
        b->pend_slot = slot;
        b->pend_jobs = k;
        FIZI_TRY(b->ring.finish(slot, s));
        return mark_last(b, s);
    }
    const bool graphed = b->mode == FIZI_BATCH_GRAPH || b->mode == FIZI_BATCH_PERSISTENT_GRAPH;
    if (k > 0) {
        if (graphed) {
            const int saved = b->mode;
            b->mode = saved == FIZI_BATCH_GRAPH ? FIZI_BATCH_DIRECT : FIZI_BATCH_PERSISTENT;
            const int rc = graph_for(b, slot);
            b->mode = saved;
            FIZI_TRY(rc);
            FIZI_HIP(hipGraphLaunch(b->graph[slot], s));
        } else {
            FIZI_TRY(enqueue_step(b, slot, k, false, s, &b->clk));
        }
    }
    FIZI_TRY(b->ring.finish(slot, s));
    return mark_last(b, s);
}

int fizi_batch_flush(fizi_batch *b, void *stream)
{
    if (!b)
        return fail(FIZI_EINVAL, "null batch");
    return flush_pending(b, static_cast<hipStream_t>(stream));
}

int fizi_batch_get_tuning(fizi_batch *b, fizi_tuning *out)
{
    if (!b || !out)
        return fail(FIZI_EINVAL, "null argument");
    out->cls_iters = b->tune.cls_iters;
    out->morph_rows = b->tune.morph_rows;
    out->grid_per_cu = b->tune.grid_per_cu;
    out->mode = b->mode;
    out->short_bands = b->tune.short_bands;
    return FIZI_OK;
}

int fizi_batch_set_tuning(fizi_batch *b, const fizi_tuning *t)
{
    if (!b || !t)
        return fail(FIZI_EINVAL, "null argument");
    if (t->cls_iters != 1 && t->cls_iters != 2 && t->cls_iters != 4 && t->cls_iters != 8)
        return fail(FIZI_EINVAL, "cls_iters must be 1, 2, 4 or 8");
    if (t->morph_rows != 8 && t->morph_rows != 16 && t->morph_rows != 32 && t->morph_rows != 64)
        return fail(FIZI_EINVAL, "morph_rows must be 8, 16, 32 or 64");
    if (t->grid_per_cu < 1 || t->grid_per_cu > 64)
        return fail(FIZI_EINVAL, "grid_per_cu must be in [1, 64]");
    if (t->short_bands != 0 && t->short_bands != 1)
        return fail(FIZI_EINVAL, "short_bands must be 0 or 1");
    if (t->mode < FIZI_BATCH_DIRECT || t->mode > FIZI_BATCH_PIPELINED_GRAPH)
        return fail(FIZI_EINVAL, "unknown batch mode");
    FIZI_TRY(drain(b));
    drop_graphs(b);
    b->tune.cls_iters = t->cls_iters;
    b->tune.morph_rows = t->morph_rows;
    b->tune.grid_per_cu = t->grid_per_cu;
    b->tune.short_bands = t->short_bands;
    b->mode = t->mode;
    return FIZI_OK;
}

int fizi_batch_autotune(fizi_batch *b, const uint8_t *const *h_frames, fizi_pointer *d_pointers, int32_t steps,
                        void *stream, fizi_tuning *best, double *best_ms)
{
    if (!b || !h_frames || !d_pointers || !best || !best_ms)
        return fail(FIZI_EINVAL, "null argument");
    if (steps < 1)
        return fail(FIZI_EINVAL, "steps must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FIZI_HIP(hipEventCreate(&e0));
    FIZI_HIP(hipEventCreate(&e1));
    // ms per step of a candidate (the better of two timed runs: candidates
    // differ by about as much as one run varies), or +inf when it is not
    // valid here
    auto measure = [&](const fizi_tuning &t, double *ms) -> int {
        *ms = 1e30;
        if (fizi_batch_set_tuning(b, &t) != FIZI_OK)
            return FIZI_OK;
        for (int i = 0; i < 2; ++i)
            FIZI_TRY(fizi_batch_step(b, h_frames, nullptr, d_pointers, stream));
        for (int rep = 0; rep < 2; ++rep) {
            FIZI_HIP(hipEventRecord(e0, s));
            for (int i = 0; i < steps; ++i)
                FIZI_TRY(fizi_batch_step(b, h_frames, nullptr, d_pointers, stream));
            FIZI_TRY(fizi_batch_flush(b, stream));
            FIZI_HIP(hipEventRecord(e1, s));
            FIZI_HIP(hipEventSynchronize(e1));
            float el = 0.f;
            FIZI_HIP(hipEventElapsedTime(&el, e0, e1));
            uint32_t flags = 0;
            FIZI_TRY(fizi_batch_status(b, &flags));
            if (flags != 0)
                return FIZI_OK;
            *ms = std::min(*ms, (double)el / steps);
        }
        return FIZI_OK;
    };
    fizi_tuning cur;
    FIZI_TRY(fizi_batch_get_tuning(b, &cur));
    if (cur.cls_iters == 1)
        cur.cls_iters = 4;
    const fizi_tuning start = cur;
    double cur_ms;
    int rc = measure(cur, &cur_ms);
    auto sweep = [&](int32_t fizi_tuning::*field, std::initializer_list<int> values) -> int {
        fizi_tuning base = cur;
        for (int v : values) {
            fizi_tuning t = base;
            t.*field = v;
            if (v == base.*field)
                continue;
            double ms;
            FIZI_TRY(measure(t, &ms));
            // a candidate has to be clearly faster: shapes within timing
            // noise of each other would otherwise move the pick at random
            if (ms < cur_ms * (1.0 - kTuneMargin)) {
                cur_ms = ms;
                cur = t;
            }
        }
        return FIZI_OK;
    };
    if (rc == FIZI_OK)
        rc = sweep(&fizi_tuning::mode, {FIZI_BATCH_GRAPH, FIZI_BATCH_PERSISTENT_GRAPH, FIZI_BATCH_PIPELINED,
                                        FIZI_BATCH_PIPELINED_GRAPH});
    if (rc == FIZI_OK)
        rc = sweep(&fizi_tuning::cls_iters, {2, 4, 8});
    if (rc == FIZI_OK)
        rc = sweep(&fizi_tuning::grid_per_cu, {8, 16, 32, 64});
    if (rc == FIZI_OK)
        rc = sweep(&fizi_tuning::morph_rows, {8, 16, 32, 64});
    // the sweep's pick against the starting shape once more, the two timed
    // in turn three times: the pick stands only if it is still clearly
    // faster (one lucky timing in the sweep does not move the shape)
    if (rc == FIZI_OK && std::memcmp(&cur, &start, sizeof(cur)) != 0) {
        double a = 1e30, c = 1e30;
        for (int rep = 0; rep < 3 && rc == FIZI_OK; ++rep) {
            double ms = 1e30;
            rc = measure(start, &ms);
            a = std::min(a, ms);
            if (rc == FIZI_OK)
                rc = measure(cur, &ms);
            c = std::min(c, ms);
        }
        if (rc == FIZI_OK && !(c < a * (1.0 - kTuneMargin)) && a < 1e29) {
            cur = start;
            cur_ms = a;
        } else if (rc == FIZI_OK) {
            cur_ms = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    FIZI_TRY(rc);
    if (cur_ms >= 1e29)
        return fail(FIZI_EHIP, "no launch shape completed without error");
    FIZI_TRY(fizi_batch_set_tuning(b, &cur));
    *best = cur;
    *best_ms = cur_ms;
    return FIZI_OK;
}

int fizi_batch_status(fizi_batch *b, uint32_t *h_flags)
{
    if (!b || !h_flags)
        return fail(FIZI_EINVAL, "null argument");
    FIZI_TRY(drain(b));
    uint32_t *err = &reinterpret_cast<PersistState *>(b->persist)->error;
    FIZI_HIP(hipMemcpy(h_flags, err, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (*h_flags) {
        FIZI_HIP(launch_fill_u32(err, 0u, 1, nullptr));
        FIZI_HIP(hipStreamSynchronize(nullptr));
    }
    return FIZI_OK;
}

int fizi_batch_stage_timing(fizi_batch *b, int32_t enable)
{
    if (!b)
        return fail(FIZI_EINVAL, "null batch");
    return b->clk.enable(enable != 0);
}

int fizi_batch_stage_times(fizi_batch *b, double *h_ms, int64_t *h_launches)
{
    if (!b || !h_ms || !h_launches)
        return fail(FIZI_EINVAL, "null argument");
    return b->clk.read(h_ms, h_launches);
}

int fizi_batch_state_layout(fizi_batch *b, int32_t stream_id, fizi_layout *out)
{
    if (!b || !out || stream_id < 0 || stream_id >= b->n)
        return fail(FIZI_EINVAL, "bad batch, stream or output");
    const Model &m = b->m[stream_id];
    out->bgmin = (uint64_t)(m.bgmin - b->d);
    out->bgmax = (uint64_t)(m.bgmax - b->d);
    out->yref = (uint64_t)(reinterpret_cast<uint8_t *>(m.yref) - b->d);
    out->yref_rows = (uint64_t)m.yref_rows;
    out->total = 0;
    return FIZI_OK;
}

int fizi_batch_destroy(fizi_batch *b)
{
    if (!b)
        return FIZI_OK;
    // a pending half-step is dropped (its buffers may be gone by now)
    if (b->have_last)
        (void)hipEventSynchronize(b->order_ev);
    drop_graphs(b);
    if (b->cap)
        (void)hipStreamDestroy(b->cap);
    if (b->side)
        (void)hipStreamDestroy(b->side);
    if (b->up)
        (void)hipStreamDestroy(b->up);
    b->ring.destroy();
    b->clk.destroy();
    for (hipEvent_t e : {b->order_ev, b->fork_ev, b->up_ev[0], b->up_ev[1], b->cls_ev[0], b->cls_ev[1],
                         b->join_ev[0], b->join_ev[1]})
        if (e)
            (void)hipEventDestroy(e);
    delete b;
    return FIZI_OK;
}

}  // extern "C"
