// C ABI of the single-stream context: learn_background, process_frames,
// get_pointer (include/fizi.h).
#include <algorithm>
#include <cstring>
#include <new>

#include "fizi_host.h"

using namespace fizi;

namespace {

constexpr int kRing = 65536;   // pointers kept for get_pointer
constexpr int kRecs = 64;

// State block: model | job tables | chunk pointers | chunk scratch slots |
// a second raw-mask buffer per slot (consecutive chunks of a call alternate
// between the two, so that a chunk's classify never writes the bits the
// previous chunk's morphology is reading).
struct CtxLayout {
    size_t model, tables, ptrs, slots, slot_stride, raw2, raw2_stride, total;
};

CtxLayout ctx_layout(const fizi_geom &g, const fizi_params &p, int chunk)
{
    CtxLayout L{};
    size_t off = 0;
    L.model = off;
    off += align256(model_bytes(g, p));
    L.tables = off;
    off += TableRing::device_bytes();
    L.ptrs = off;
    off += align256((size_t)chunk * sizeof(fizi_pointer));
    L.slot_stride = align256(slot_bytes(g));
    L.slots = off;
    off += (size_t)chunk * L.slot_stride;
    L.raw2_stride = align256((size_t)g.height * (g.width / 64) * 8);
    L.raw2 = off;
    off += (size_t)chunk * L.raw2_stride;
    L.total = align256(off);
    return L;
}

}  // namespace

// Everything the kernels read of a one-job table: the header's entries for
// one job and the job, its per-call fields cleared (the gain launch brings
// them). Zero-filled first, so that padding compares equal.
struct OneJobKey {
    int32_t njobs, flow_nseg;
    int32_t gain_pre[2], cls_pre[2], mor_pre[2], flow_pre[3], flow_seg[2];
    Job job;
};

static OneJobKey one_job_key(const Table &T)
{
    OneJobKey k;
    std::memset(&k, 0, sizeof(k));
    k.njobs = T.h.njobs;
    k.flow_nseg = T.h.flow_nseg;
    for (int i = 0; i < 2; ++i) {
        k.gain_pre[i] = T.h.gain_pre[i];
        k.cls_pre[i] = T.h.cls_pre[i];
        k.mor_pre[i] = T.h.mor_pre[i];
        k.flow_seg[i] = T.h.flow_seg[i];
    }
    for (int i = 0; i < 3; ++i)
        k.flow_pre[i] = T.h.flow_pre[i];
    std::memcpy(&k.job, &T.jobs[0], sizeof(Job));
    k.job.frame = nullptr;
    k.job.fizi = k.job.hand = nullptr;
    k.job.out = k.job.hout = nullptr;
    k.job.frame_index = 0;
    return k;
}

struct fizi_ctx {
    Model m;
    int chunk = 0;
    Tuning tune{};
    uint8_t *d = nullptr;
    CtxLayout L{};
    int device = 0;
    int n_cu = 0;
    TableRing ring;
    // what the kernels read of each table slot on the device, as its last
    // one-frame call left it (job 0's per-call fields cleared), valid while
    // shadow_gen[slot] == gen; any other use of the ring (learning, calls of
    // several frames) makes it stale
    OneJobKey shadow[kTabSlots];
    uint64_t shadow_gen[kTabSlots] = {};
    uint64_t gen = 1;
    StageClock clk;
    // the last kRing pointers, indexed by frame: pinned, coherent host memory
    // that the component kernels store each final pointer into (d_ring is
    // its device-side address), so that no copy follows them
    fizi_pointer *h_ring = nullptr;
    fizi_pointer *d_ring = nullptr;
    // frames [f0, f1) are in the host pointer ring once `ev` (recorded after
    // the kernels that store them, default fences: the host reads what they
    // wrote) is done
    struct Rec {
        uint64_t f0, f1;
        hipEvent_t ev;
        bool valid;
    } recs[kRecs] = {};
    int next_rec = 0;
    hipEvent_t order_ev = nullptr;
    hipStream_t last_stream = nullptr;
    bool have_last = false;
    uint64_t next_frame = 0;
    // calls of several chunks: the back half of a chunk (morphology,
    // components, pointer copies) on a side stream beside the next chunk's
    // front, the job tables going up on their own stream
    hipStream_t side = nullptr, up = nullptr;
    hipEvent_t up_ev[2] = {}, cls_ev[2] = {}, join_ev[2] = {};
    // pipelined calls (fizi_set_pipelined): a call leaves its last chunk's
    // back half on the side stream; the next call joins it after its first
    // classify (or fizi_flush does), and chunks keep alternating raw buffers
    // across calls
    bool pipe_calls = false;
    int parity = 0;      // raw buffer of the next chunk
    int pend_join = -1;  // parity of the back half not yet joined, or -1
};

namespace {

// Calls on different streams run one after the other.
int order_after_previous(fizi_ctx *c, hipStream_t s)
{
    if (c->have_last && c->last_stream != s)
        FIZI_HIP(hipStreamWaitEvent(s, c->order_ev, 0));
    return FIZI_OK;
}

int mark_last(fizi_ctx *c, hipStream_t s)
{
    FIZI_HIP(hipEventRecord(c->order_ev, s));
    c->last_stream = s;
    c->have_last = true;
    return FIZI_OK;
}

// Orders s after the back half a pipelined call left pending.
int join_pending(fizi_ctx *c, hipStream_t s)
{
    if (c->pend_join >= 0) {
        FIZI_HIP(hipStreamWaitEvent(s, c->join_ev[c->pend_join], 0));
        c->pend_join = -1;
    }
    return FIZI_OK;
}

// Joins a pending back half on the stream of the last call and waits for
// all of the context's work.
int drain(fizi_ctx *c)
{
    if (c->pend_join >= 0) {
        FIZI_TRY(join_pending(c, c->last_stream));
        FIZI_TRY(mark_last(c, c->last_stream));
    }
    if (c->have_last)
        FIZI_HIP(hipEventSynchronize(c->order_ev));
    return FIZI_OK;
}

}  // namespace

extern "C" {

int fizi_default_params(fizi_params *out)
{
    if (!out)
        return fail(FIZI_EINVAL, "null output");
    out->alpha1_cdeg = 33000;
    out->alpha2_cdeg = 7500;
    out->gray_S = 20;
    out->bg_delta = 10;
    out->open_iters = 1;
    out->close_iters = 1;
    out->min_area = 1;
    out->click_fill_permille = 700;
    out->gain_row_stride = 8;
    out->gain_lo_q16 = 32768;
    out->gain_hi_q16 = 131072;
    out->brightness_mode = 0;
    out->click_debounce = 0;
    out->track_radius = 64;
    out->lum_hi = 0;
    return FIZI_OK;
}

int fizi_validate(const fizi_geom *geom, const fizi_params *params) { return validate(geom, params); }

size_t fizi_state_bytes(const fizi_geom *geom, const fizi_params *params, int32_t chunk_frames)
{
    if (validate(geom, params) != FIZI_OK || chunk_frames < 1 || chunk_frames > kMaxJobs)
        return 0;
    return ctx_layout(*geom, *params, chunk_frames).total;
}

int fizi_state_layout(const fizi_geom *geom, const fizi_params *params, int32_t chunk_frames,
                      fizi_layout *out)
{
    FIZI_TRY(validate(geom, params));
    if (chunk_frames < 1 || chunk_frames > kMaxJobs || !out)
        return fail(FIZI_EINVAL, "chunk_frames must be in [1, 256] and out non-null");
    const CtxLayout L = ctx_layout(*geom, *params, chunk_frames);
    Model m;
    model_at(m, *geom, *params, nullptr);
    out->bgmin = L.model + (uint64_t)(uintptr_t)m.bgmin;
    out->bgmax = L.model + (uint64_t)(uintptr_t)m.bgmax;
    out->yref = L.model + (uint64_t)(uintptr_t)m.yref;
    out->yref_rows = (uint64_t)m.yref_rows;
    out->total = L.total;
    return FIZI_OK;
}

int fizi_create(const fizi_geom *geom, const fizi_params *params, int32_t chunk_frames,
                void *d_state, size_t state_bytes, void *stream, fizi_ctx **out)
{
    FIZI_TRY(validate(geom, params));
    if (!out || !d_state)
        return fail(FIZI_EINVAL, "null d_state or out");
    if (chunk_frames < 1 || chunk_frames > kMaxJobs)
        return fail(FIZI_EINVAL, "chunk_frames must be in [1, 256]");
    if (reinterpret_cast<uintptr_t>(d_state) % 256 != 0)
        return fail(FIZI_EINVAL, "d_state must be 256-byte aligned");
    const CtxLayout L = ctx_layout(*geom, *params, chunk_frames);
    if (state_bytes < L.total)
        return fail(FIZI_ENOMEM, "state block smaller than fizi_state_bytes()");
    (void)stream;
    fizi_ctx *c = new (std::nothrow) fizi_ctx();
    if (!c)
        return fail(FIZI_ENOMEM, "host allocation failed");
    c->chunk = chunk_frames;
    c->d = static_cast<uint8_t *>(d_state);
    c->L = L;
    model_at(c->m, *geom, *params, c->d + L.model);
    c->tune = tuning_for(geom->width, morph_ops(*params), false);
    int rc = device_cu_count(&c->device, &c->n_cu);
    if (rc == FIZI_OK)
        rc = c->ring.init(c->d + L.tables);
    if (rc == FIZI_OK) {
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&c->h_ring), sizeof(fizi_pointer) * kRing,
                                     hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess)
            e = hipHostGetDevicePointer(reinterpret_cast<void **>(&c->d_ring), c->h_ring, 0);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&c->order_ev, kDeviceOrderEvent);
        for (int i = 0; i < kRecs && e == hipSuccess; ++i)
            e = hipEventCreateWithFlags(&c->recs[i].ev, hipEventDisableTiming);
        for (int k = 0; k < 2 && e == hipSuccess; ++k) {
            e = hipEventCreateWithFlags(&c->up_ev[k], hipEventDisableTiming);
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&c->cls_ev[k], kDeviceOrderEvent);
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&c->join_ev[k], kDeviceOrderEvent);
        }
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&c->up, hipStreamNonBlocking);
        if (e != hipSuccess)
            rc = fail(FIZI_EHIP, std::string("fizi_create: ") + hipGetErrorString(e));
    }
    if (rc != FIZI_OK) {
        const std::string msg = fizi_last_error();
        fizi_destroy(c);
        return fail(rc, msg);
    }
    *out = c;
    return FIZI_OK;
}

int learn_background(fizi_ctx *c, const uint8_t *d_frames, int32_t n_frames, int32_t reset, void *stream)
{
    if (!c || !d_frames)
        return fail(FIZI_EINVAL, "null context or frames");
    if (reinterpret_cast<uintptr_t>(d_frames) % 4 != 0)
        return fail(FIZI_EINVAL, "frames must be 4-byte aligned");
    if (n_frames < 1)
        return fail(FIZI_EINVAL, "n_frames must be >= 1");
    if (!reset && !c->m.learned)
        return fail(FIZI_ESTATE, "learning without reset needs a learned model");
    hipStream_t s = static_cast<hipStream_t>(stream);
    FIZI_TRY(order_after_previous(c, s));
    FIZI_TRY(join_pending(c, s));
    ++c->gen;
    FIZI_TRY(learn_model(c->m, c->ring, c->tune, c->n_cu, d_frames, n_frames, reset, s, &c->clk));
    return mark_last(c, s);
}

int relearn_background(fizi_ctx *c, const uint8_t *d_frames, int32_t n_frames, const uint64_t *d_fizi_bits,
                       void *stream)
{
    if (!c || !d_frames || !d_fizi_bits)
        return fail(FIZI_EINVAL, "null context, frames or masks");
    if (reinterpret_cast<uintptr_t>(d_frames) % 4 != 0 || reinterpret_cast<uintptr_t>(d_fizi_bits) % 8 != 0)
        return fail(FIZI_EINVAL, "frames must be 4-byte and masks 8-byte aligned");
    if (n_frames < 1)
        return fail(FIZI_EINVAL, "n_frames must be >= 1");
    if (!c->m.learned)
        return fail(FIZI_ESTATE, "relearn_background before learn_background");
    hipStream_t s = static_cast<hipStream_t>(stream);
    FIZI_TRY(order_after_previous(c, s));
    // the masks may come from a call whose back half is still pending
    FIZI_TRY(join_pending(c, s));
    ++c->gen;
    FIZI_TRY(learn_model(c->m, c->ring, c->tune, c->n_cu, d_frames, n_frames, 0, s, &c->clk, d_fizi_bits));
    return mark_last(c, s);
}

int process_frames(fizi_ctx *c, const uint8_t *d_frames, int32_t n_frames, uint64_t *d_fizi_bits,
                   uint64_t *d_hand_bits, fizi_pointer *d_pointers, void *stream)
{
    if (!c || !d_frames)
        return fail(FIZI_EINVAL, "null context or frames");
    if (reinterpret_cast<uintptr_t>(d_frames) % 4 != 0)
        return fail(FIZI_EINVAL, "frames must be 4-byte aligned");
    if (n_frames < 1)
        return fail(FIZI_EINVAL, "n_frames must be >= 1");
    if (!c->m.learned)
        return fail(FIZI_ESTATE, "process_frames before learn_background");
    hipStream_t s = static_cast<hipStream_t>(stream);
    FIZI_TRY(order_after_previous(c, s));
    const size_t W = c->m.g.width, H = c->m.g.height, px = W * H, words = H * (W / 64);
    fizi_pointer *internal = reinterpret_cast<fizi_pointer *>(c->d + c->L.ptrs);
    // several chunks: each chunk's back half runs beside the next chunk's
    // front (on the side stream; s joins it before the call ends, or, with
    // pipelined calls, after the next call's first classify)
    const bool pipelined = c->pipe_calls || n_frames > c->chunk;
    int par = c->pipe_calls ? c->parity : 0;
    int prev_join = c->pipe_calls ? c->pend_join : -1;
    for (int f0 = 0; f0 < n_frames; f0 += c->chunk) {
        const int k = std::min(c->chunk, n_frames - f0);
        int slot;
        FIZI_TRY(c->ring.take(&slot));
        Table &T = *c->ring.h[slot];
        const uint64_t fbase = c->next_frame + (uint64_t)f0;
        // a launch whose morphology, in short bands of one wave each, needs
        // at most one wave per SIMD is bound by the length of one wave's
        // chain of rows rather than by the total work: it takes that shape
        // (13 row steps per wave against 17 for 8-row bands). Larger launches
        // keep the tuned shape, which repeats fewer halo rows.
        const bool short_chain =
            c->tune.short_bands && (size_t)k * ((H + kShortBand - 1) / kShortBand) <= (size_t)c->n_cu * 4;
        for (int i = 0; i < k; ++i) {
            Job &J = T.jobs[i];
            if (short_chain)
                fill_job(c->m, kShortBand, J, false);
            else
                fill_job(c->m, c->tune.morph_rows, J);
            set_scratch(J, slot_at(c->m.g, c->d + c->L.slots + (size_t)i * c->L.slot_stride));
            if (pipelined && par)
                J.raw = reinterpret_cast<uint64_t *>(c->d + c->L.raw2 + (size_t)i * c->L.raw2_stride);
            const size_t f = (size_t)(f0 + i);
            J.frame = d_frames + f * px * 3;
            if (d_fizi_bits)
                J.fizi = d_fizi_bits + f * words;
            J.hand = d_hand_bits ? d_hand_bits + f * words : nullptr;
            J.out = d_pointers ? d_pointers + f : internal + i;
            J.hout = c->d_ring + (size_t)((fbase + (uint64_t)i) % kRing);
            J.frame_index = fbase + (uint64_t)i;
        }
        set_prefixes(T, k, c->tune);
        // the stream the chunk's back half goes to
        hipStream_t bs = s;
        if (pipelined) {
            c->shadow_gen[slot] = 0;
            FIZI_HIP(hipMemcpyAsync(c->ring.d[slot], &T, table_bytes(k), hipMemcpyHostToDevice, c->up));
            FIZI_HIP(hipEventRecord(c->up_ev[par], c->up));
            FIZI_HIP(hipStreamWaitEvent(s, c->up_ev[par], 0));
            FIZI_TRY(run_front(c->ring.d[slot], T, k, c->tune, c->n_cu, false, s, &c->clk));
            FIZI_HIP(hipEventRecord(c->cls_ev[par], s));
            FIZI_HIP(hipStreamWaitEvent(c->side, c->cls_ev[par], 0));
            bs = c->side;
            FIZI_TRY(run_back(c->ring.d[slot], T, k, k, (int)(W / 64), morph_ops(c->m.p), c->tune, c->n_cu,
                              false, bs, &c->clk, true));
        } else if (k == 1) {
            // a one-frame call: when the slot on the device already holds
            // this table apart from job 0's per-call fields (the previous
            // one-frame call in this slot left it so, its accumulators
            // zeroed), those fields go with the gain launch instead of an
            // upload
            const Job &J = T.jobs[0];
            const CallPatch P{J.frame, J.fizi, J.hand, J.out, J.hout, J.frame_index, 1};
            const OneJobKey key = one_job_key(T);
            const bool reuse =
                c->shadow_gen[slot] == c->gen && std::memcmp(&c->shadow[slot], &key, sizeof(key)) == 0;
            // stale until every kernel of this call is enqueued (a launch
            // that fails leaves the slot to a full upload next time)
            c->shadow_gen[slot] = 0;
            if (!reuse)
                FIZI_HIP(hipMemcpyAsync(c->ring.d[slot], &T, table_bytes(1), hipMemcpyHostToDevice, s));
            FIZI_TRY(run_pipeline(c->ring.d[slot], T, k, k, (int)(W / 64), morph_ops(c->m.p), c->tune, c->n_cu,
                                  false, s, &c->clk, &P));
            c->shadow[slot] = key;
            c->shadow_gen[slot] = c->gen;
        } else {
            c->shadow_gen[slot] = 0;
            FIZI_HIP(hipMemcpyAsync(c->ring.d[slot], &T, table_bytes(k), hipMemcpyHostToDevice, s));
            FIZI_TRY(run_pipeline(c->ring.d[slot], T, k, k, (int)(W / 64), morph_ops(c->m.p), c->tune, c->n_cu,
                                  false, s, &c->clk));
        }
        FIZI_TRY(c->ring.finish(slot, bs));
        if (pipelined) {
            FIZI_HIP(hipEventRecord(c->join_ev[par], c->side));
            // the chunk before this one is joined after this classify: the
            // next classify reuses its raw buffers
            if (prev_join >= 0)
                FIZI_HIP(hipStreamWaitEvent(s, c->join_ev[prev_join], 0));
            prev_join = par;
            par ^= 1;
        }
        // the ring holds a chunk's pointers once its back half is done
        fizi_ctx::Rec &r = c->recs[c->next_rec];
        c->next_rec = (c->next_rec + 1) % kRecs;
        r.f0 = fbase;
        r.f1 = fbase + k;
        FIZI_HIP(hipEventRecord(r.ev, bs));
        r.valid = true;
    }
    if (pipelined) {
        if (c->pipe_calls) {
            c->pend_join = prev_join;
            c->parity = par;
        } else {
            FIZI_HIP(hipStreamWaitEvent(s, c->join_ev[prev_join], 0));
        }
    }
    c->next_frame += (uint64_t)n_frames;
    return mark_last(c, s);
}

int get_pointer(fizi_ctx *c, int64_t frame_index, fizi_pointer *h_out)
{
    if (!c || !h_out)
        return fail(FIZI_EINVAL, "null context or output");
    if (frame_index < 0 || (uint64_t)frame_index >= c->next_frame)
        return fail(FIZI_ERANGE, "frame not submitted yet");
    if ((uint64_t)frame_index + kRing < c->next_frame)
        return fail(FIZI_ERANGE, "frame no longer kept (older than the last 65536)");
    // calls run in submission order, so the first recorded chunk that ends
    // after the frame finishes no earlier than the frame's own back half
    int best = -1;
    for (int i = 0; i < kRecs; ++i) {
        const fizi_ctx::Rec &r = c->recs[i];
        if (r.valid && r.f1 > (uint64_t)frame_index && (best < 0 || r.f0 < c->recs[best].f0))
            best = i;
    }
    if (best < 0)
        return fail(FIZI_ERANGE, "frame record missing");
    FIZI_HIP(hipEventSynchronize(c->recs[best].ev));
    *h_out = c->h_ring[(size_t)frame_index % kRing];
    return FIZI_OK;
}

int fizi_stage_timing(fizi_ctx *c, int32_t enable)
{
    if (!c)
        return fail(FIZI_EINVAL, "null context");
    return c->clk.enable(enable != 0);
}

int fizi_stage_times(fizi_ctx *c, double *h_ms, int64_t *h_launches)
{
    if (!c || !h_ms || !h_launches)
        return fail(FIZI_EINVAL, "null argument");
    return c->clk.read(h_ms, h_launches);
}

int fizi_set_tracking(fizi_ctx *c, int32_t enable)
{
    if (!c)
        return fail(FIZI_EINVAL, "null context");
    FIZI_TRY(drain(c));
    FIZI_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(c->m.track), 0u, sizeof(TrackState) / 4, nullptr));
    FIZI_HIP(hipStreamSynchronize(nullptr));
    c->m.tracking = enable != 0;
    return FIZI_OK;
}

int fizi_set_pipelined(fizi_ctx *c, int32_t enable)
{
    if (!c)
        return fail(FIZI_EINVAL, "null context");
    FIZI_TRY(drain(c));
    c->pipe_calls = enable != 0;
    c->parity = 0;
    return FIZI_OK;
}

int fizi_set_short_bands(fizi_ctx *c, int32_t enable)
{
    if (!c)
        return fail(FIZI_EINVAL, "null context");
    c->tune.short_bands = enable != 0;
    return FIZI_OK;
}

int fizi_flush(fizi_ctx *c, void *stream)
{
    if (!c)
        return fail(FIZI_EINVAL, "null context");
    hipStream_t s = static_cast<hipStream_t>(stream);
    FIZI_TRY(order_after_previous(c, s));
    FIZI_TRY(join_pending(c, s));
    return mark_last(c, s);
}

int fizi_destroy(fizi_ctx *c)
{
    if (!c)
        return FIZI_OK;
    if (c->have_last)
        (void)hipEventSynchronize(c->order_ev);
    // a pending back half, without touching the stream of the last call
    if (c->pend_join >= 0)
        (void)hipEventSynchronize(c->join_ev[c->pend_join]);
    c->ring.destroy();
    c->clk.destroy();
    if (c->h_ring)
        (void)hipHostFree(c->h_ring);
    for (hipEvent_t e : {c->order_ev, c->up_ev[0], c->up_ev[1], c->cls_ev[0], c->cls_ev[1], c->join_ev[0],
                         c->join_ev[1]})
        if (e)
            (void)hipEventDestroy(e);
    for (const fizi_ctx::Rec &r : c->recs)
        if (r.ev)
            (void)hipEventDestroy(r.ev);
    for (hipStream_t st : {c->side, c->up})
        if (st)
            (void)hipStreamDestroy(st);
    delete c;
    return FIZI_OK;
}

}  // extern "C"
