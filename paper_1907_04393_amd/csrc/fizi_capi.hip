// C ABI of the FIZI/Mouse pipeline: parameter checks, the state-block
// layout, contexts, job tables and the per-call launch sequence.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fizi_internal.h"

using namespace fizi;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define FIZI_HIP(expr)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(FIZI_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

constexpr int kMaxW = 8192;
constexpr int kMaxH = 8192;
constexpr int kTabSlots = 8;
constexpr int kRing = 65536;          // pointers kept for get_pointer
constexpr int kRecs = 64;
constexpr size_t kLdsBudget = 65536;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Direction (scaled by 6000) of the hexcone colour of hue a centi-degrees.
void hue_dir(int a, int d[3])
{
    const int k = a / 6000, f = a - 6000 * k;
    switch (k) {
    case 0: d[0] = 6000; d[1] = f; d[2] = 0; break;
    case 1: d[0] = 6000 - f; d[1] = 6000; d[2] = 0; break;
    case 2: d[0] = 0; d[1] = 6000; d[2] = f; break;
    case 3: d[0] = 0; d[1] = 6000 - f; d[2] = 6000; break;
    case 4: d[0] = f; d[1] = 0; d[2] = 6000; break;
    default: d[0] = 6000; d[1] = 0; d[2] = 6000 - f; break;
    }
}

// det[(1,1,1), d, p] = R (dB - dG) + G (dR - dB) + B (dG - dR); the three
// coefficients sum to zero, so it is kr (R - B) + kg (G - B).
void hue_coef(int a, int32_t *kr, int32_t *kg)
{
    int d[3];
    hue_dir(a, d);
    *kr = d[2] - d[1];
    *kg = d[0] - d[2];
}

HueTest make_hue(int a1, int a2)
{
    HueTest h{};
    hue_coef(a1, &h.k1r, &h.k1g);
    hue_coef(a2, &h.k2r, &h.k2g);
    int d[3];
    hue_dir(a1, d);
    h.dr = d[0];
    h.dg = d[1];
    h.db = d[2];
    h.dsum = d[0] + d[1] + d[2];
    const int L = ((a2 - a1) % 36000 + 36000) % 36000;
    h.mode = L == 0 ? 0 : (L < 18000 ? 1 : (L == 18000 ? 2 : 3));
    return h;
}

int validate(const fizi_geom *g, const fizi_params *p)
{
    if (!g || !p)
        return fail(FIZI_EINVAL, "null geometry or parameters");
    if (g->width < 64 || g->width % 64 != 0 || g->width > kMaxW)
        return fail(FIZI_EINVAL, "width must be a multiple of 64 in [64, 8192]");
    if (g->height < 1 || g->height > kMaxH)
        return fail(FIZI_EINVAL, "height must be in [1, 8192]");
    if (p->alpha1_cdeg < 0 || p->alpha1_cdeg >= 36000 || p->alpha2_cdeg < 0 || p->alpha2_cdeg >= 36000)
        return fail(FIZI_EINVAL, "alpha1_cdeg / alpha2_cdeg must be in [0, 36000)");
    if (p->gray_S < 0 || p->gray_S > 255)
        return fail(FIZI_EINVAL, "gray_S must be in [0, 255]");
    if (p->bg_delta < 0 || p->bg_delta > 255)
        return fail(FIZI_EINVAL, "bg_delta must be in [0, 255]");
    if (p->open_iters < 0 || p->open_iters > kMaxMorphIters || p->close_iters < 0 ||
        p->close_iters > kMaxMorphIters)
        return fail(FIZI_EINVAL, "open_iters / close_iters must be in [0, 3]");
    if (p->min_area < 0)
        return fail(FIZI_EINVAL, "min_area must be >= 0");
    if (p->click_fill_permille < 0 || p->click_fill_permille > 1000)
        return fail(FIZI_EINVAL, "click_fill_permille must be in [0, 1000]");
    if (p->gain_row_stride < 1 || p->gain_row_stride > 64)
        return fail(FIZI_EINVAL, "gain_row_stride must be in [1, 64]");
    if (p->gain_lo_q16 < 1 || p->gain_hi_q16 < p->gain_lo_q16 || p->gain_hi_q16 > (1 << 20))
        return fail(FIZI_EINVAL, "need 1 <= gain_lo_q16 <= gain_hi_q16 <= 2^20");
    return FIZI_OK;
}

struct Layout {
    size_t bgmin, bgmax, yref, yref_rows;
    size_t tables;        // kTabSlots device tables
    size_t ptrs;          // chunk internal pointers
    size_t slots, slot_stride;
    size_t raw, fz, parent, area, runs;   // offsets inside a slot
    size_t run_cap;
    size_t total;
};

Layout layout_of(const fizi_geom *g, const fizi_params *p, int chunk)
{
    Layout L{};
    const size_t W = g->width, H = g->height, px = W * H;
    const size_t words = H * (W / 64);
    size_t off = 0;
    L.bgmin = off; off = align256(off + px * 3);
    L.bgmax = off; off = align256(off + px * 3);
    L.yref_rows = (H + p->gain_row_stride - 1) / p->gain_row_stride;
    L.yref = off; off = align256(off + L.yref_rows * W * 2);
    L.tables = off; off = align256(off + kTabSlots * align256(sizeof(Table)));
    L.ptrs = off; off = align256(off + (size_t)chunk * sizeof(fizi_pointer));
    L.run_cap = px / 2;
    size_t so = 0;
    L.raw = so; so = align256(so + words * 8);
    L.fz = so; so = align256(so + words * 8);
    L.parent = so; so = align256(so + px * 4);
    L.area = so; so = align256(so + px * 4);
    L.runs = so; so = align256(so + L.run_cap * 8);
    L.slot_stride = so;
    L.slots = off; off += (size_t)chunk * so;
    L.total = align256(off);
    return L;
}

Tuning default_tuning(const fizi_geom *g, const fizi_params *p)
{
    Tuning t;
    t.cls_iters = 4;
    t.grid_per_cu = 8;
    const int nops = 2 * (p->open_iters + p->close_iters);
    const int wd = g->width / 64;
    int R = 32;
    while (R > 8 && 2ull * (R + 2 * nops) * wd * 8 > kLdsBudget)
        R /= 2;
    t.morph_rows = R;
    return t;
}

}  // namespace

struct fizi_ctx {
    fizi_geom g;
    fizi_params p;
    int chunk;
    Tuning tune;
    HueTest hue;
    uint8_t *d;
    size_t bytes;
    Layout L;
    bool learned;
    int device;
    int n_cu;
    Table *h_tab[kTabSlots];
    hipEvent_t tab_ev[kTabSlots];
    bool tab_used[kTabSlots];
    int next_tab;
    fizi_pointer *h_ring;
    struct Rec {
        uint64_t f0, f1;
        int slot;
        bool valid;
    } recs[kRecs];
    int next_rec;
    hipEvent_t order_ev;
    hipStream_t last_stream;
    bool have_last;
    uint64_t next_frame;
    // stage timing (measurement hook)
    bool timing;
    std::vector<hipEvent_t> tev[FIZI_NSTAGES];   // pairs: 2*i start, 2*i+1 end
    int tused[FIZI_NSTAGES];
    double tms[FIZI_NSTAGES];
    int64_t tcount[FIZI_NSTAGES];
};

namespace {

Table *dev_table(fizi_ctx *c, int slot)
{
    return reinterpret_cast<Table *>(c->d + c->L.tables + slot * align256(sizeof(Table)));
}

void fill_job_common(const fizi_ctx *c, Job &J)
{
    std::memset(&J, 0, sizeof(J));
    J.bgmin = c->d + c->L.bgmin;
    J.bgmax = c->d + c->L.bgmax;
    J.yref = reinterpret_cast<const uint16_t *>(c->d + c->L.yref);
    J.W = c->g.width;
    J.H = c->g.height;
    J.Wd = c->g.width / 64;
    J.rs = c->p.gain_row_stride;
    J.run_cap = (uint32_t)c->L.run_cap;
    J.delta = c->p.bg_delta;
    J.S1 = std::max(c->p.gray_S, 1);
    J.open_it = c->p.open_iters;
    J.close_it = c->p.close_iters;
    J.min_area = c->p.min_area;
    J.fill_pm = c->p.click_fill_permille;
    J.glo = c->p.gain_lo_q16;
    J.ghi = c->p.gain_hi_q16;
    J.hue = c->hue;
}

// Takes table slot `slot` for a new call: waits until its previous call has
// finished with it.
int take_slot(fizi_ctx *c, int *slot)
{
    const int s = c->next_tab;
    c->next_tab = (c->next_tab + 1) % kTabSlots;
    if (c->tab_used[s])
        FIZI_HIP(hipEventSynchronize(c->tab_ev[s]));
    *slot = s;
    return FIZI_OK;
}

int order_after_previous(fizi_ctx *c, hipStream_t s)
{
    if (c->have_last && c->last_stream != s)
        FIZI_HIP(hipStreamWaitEvent(s, c->order_ev, 0));
    return FIZI_OK;
}

int finish_call(fizi_ctx *c, int slot, hipStream_t s)
{
    FIZI_HIP(hipEventRecord(c->tab_ev[slot], s));
    c->tab_used[slot] = true;
    FIZI_HIP(hipEventRecord(c->order_ev, s));
    c->last_stream = s;
    c->have_last = true;
    return FIZI_OK;
}

size_t table_bytes(int njobs) { return sizeof(TableHeader) + (size_t)njobs * sizeof(Job); }

constexpr int kTimedLaunches = 16384;

// Records the start event of a timed stage launch; returns the pair index or -1.
int stage_begin(fizi_ctx *c, int stage, hipStream_t s)
{
    if (!c->timing || c->tused[stage] >= kTimedLaunches)
        return -1;
    const int i = c->tused[stage]++;
    if (hipEventRecord(c->tev[stage][2 * i], s) != hipSuccess)
        return -1;
    return i;
}

void stage_end(fizi_ctx *c, int stage, int i, hipStream_t s)
{
    if (i >= 0)
        (void)hipEventRecord(c->tev[stage][2 * i + 1], s);
}

// Launch of one stage, bracketed by its timing events when enabled.
#define FIZI_STAGE(c, stage, s, launch)                   \
    do {                                                  \
        const int ti_ = stage_begin((c), (stage), (s));   \
        FIZI_HIP(launch);                                 \
        stage_end((c), (stage), ti_, (s));                \
    } while (0)

}  // namespace

extern "C" {

const char *fizi_last_error(void) { return g_err.c_str(); }

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
    return FIZI_OK;
}

int fizi_validate(const fizi_geom *geom, const fizi_params *params) { return validate(geom, params); }

size_t fizi_state_bytes(const fizi_geom *geom, const fizi_params *params, int32_t chunk_frames)
{
    if (validate(geom, params) != FIZI_OK || chunk_frames < 1 || chunk_frames > kMaxJobs)
        return 0;
    return layout_of(geom, params, chunk_frames).total;
}

int fizi_state_layout(const fizi_geom *geom, const fizi_params *params, int32_t chunk_frames,
                      fizi_layout *out)
{
    int rc = validate(geom, params);
    if (rc != FIZI_OK)
        return rc;
    if (chunk_frames < 1 || chunk_frames > kMaxJobs || !out)
        return fail(FIZI_EINVAL, "chunk_frames must be in [1, 256] and out non-null");
    Layout L = layout_of(geom, params, chunk_frames);
    out->bgmin = L.bgmin;
    out->bgmax = L.bgmax;
    out->yref = L.yref;
    out->yref_rows = L.yref_rows;
    out->total = L.total;
    return FIZI_OK;
}

int fizi_create(const fizi_geom *geom, const fizi_params *params, int32_t chunk_frames,
                void *d_state, size_t state_bytes, void *stream, fizi_ctx **out)
{
    int rc = validate(geom, params);
    if (rc != FIZI_OK)
        return rc;
    if (!out || !d_state)
        return fail(FIZI_EINVAL, "null d_state or out");
    if (chunk_frames < 1 || chunk_frames > kMaxJobs)
        return fail(FIZI_EINVAL, "chunk_frames must be in [1, 256]");
    if (reinterpret_cast<uintptr_t>(d_state) % 256 != 0)
        return fail(FIZI_EINVAL, "d_state must be 256-byte aligned");
    Layout L = layout_of(geom, params, chunk_frames);
    if (state_bytes < L.total)
        return fail(FIZI_ENOMEM, "state block smaller than fizi_state_bytes()");
    (void)stream;
    fizi_ctx *c = new (std::nothrow) fizi_ctx();
    if (!c)
        return fail(FIZI_ENOMEM, "host allocation failed");
    c->g = *geom;
    c->p = *params;
    c->chunk = chunk_frames;
    c->tune = default_tuning(geom, params);
    c->hue = make_hue(params->alpha1_cdeg, params->alpha2_cdeg);
    c->d = static_cast<uint8_t *>(d_state);
    c->bytes = state_bytes;
    c->L = L;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device);
    for (int i = 0; i < kTabSlots && e == hipSuccess; ++i) {
        e = hipHostMalloc(reinterpret_cast<void **>(&c->h_tab[i]), sizeof(Table), hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&c->tab_ev[i], hipEventDisableTiming);
    }
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&c->h_ring), sizeof(fizi_pointer) * kRing,
                          hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        std::string msg = std::string("fizi_create: ") + hipGetErrorString(e);
        fizi_destroy(c);
        return fail(FIZI_EHIP, msg);
    }
    *out = c;
    return FIZI_OK;
}

int learn_background(fizi_ctx *c, const uint8_t *d_frames, int32_t n_frames, int32_t reset, void *stream)
{
    if (!c || !d_frames)
        return fail(FIZI_EINVAL, "null context or frames");
    if (n_frames < 1)
        return fail(FIZI_EINVAL, "n_frames must be >= 1");
    if (!reset && !c->learned)
        return fail(FIZI_ESTATE, "learning without reset needs a learned model");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = order_after_previous(c, s);
    if (rc)
        return rc;
    const size_t px = (size_t)c->g.width * c->g.height;
    uint8_t *bgmin = c->d + c->L.bgmin, *bgmax = c->d + c->L.bgmax;
    if (reset)
        FIZI_HIP(launch_make_yref(d_frames, reinterpret_cast<uint16_t *>(c->d + c->L.yref),
                                  c->g.width, c->g.height, c->p.gain_row_stride, s));
    const int gtiles = (int)c->L.yref_rows;
    for (int f0 = 0; f0 < n_frames; f0 += kMaxJobs) {
        const int m = std::min(kMaxJobs, n_frames - f0);
        int slot;
        if ((rc = take_slot(c, &slot)))
            return rc;
        Table *h = c->h_tab[slot];
        h->h.njobs = m;
        for (int i = 0; i <= m; ++i) {
            h->h.gain_pre[i] = i * gtiles;
            h->h.cls_pre[i] = 0;
            h->h.mor_pre[i] = 0;
        }
        for (int i = 0; i < m; ++i) {
            Job &J = h->jobs[i];
            fill_job_common(c, J);
            J.frame = d_frames + (size_t)(f0 + i) * px * 3;
        }
        Table *dt = dev_table(c, slot);
        FIZI_HIP(hipMemcpyAsync(dt, h, table_bytes(m), hipMemcpyHostToDevice, s));
        FIZI_STAGE(c, FIZI_STAGE_LEARN, s, launch_gain(dt, m * gtiles, c->n_cu, c->tune, s));
        FIZI_STAGE(c, FIZI_STAGE_LEARN, s,
                   launch_minmax(dt, m, bgmin, bgmax, (int)px, (reset && f0 == 0) ? 1 : 0, c->n_cu, s));
        if ((rc = finish_call(c, slot, s)))
            return rc;
    }
    c->learned = true;
    return FIZI_OK;
}

int process_frames(fizi_ctx *c, const uint8_t *d_frames, int32_t n_frames, uint64_t *d_fizi_bits,
                   uint64_t *d_hand_bits, fizi_pointer *d_pointers, void *stream)
{
    if (!c || !d_frames)
        return fail(FIZI_EINVAL, "null context or frames");
    if (n_frames < 1)
        return fail(FIZI_EINVAL, "n_frames must be >= 1");
    if (!c->learned)
        return fail(FIZI_ESTATE, "process_frames before learn_background");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = order_after_previous(c, s);
    if (rc)
        return rc;
    const size_t W = c->g.width, H = c->g.height, px = W * H, words = H * (W / 64);
    const int gtiles = (int)c->L.yref_rows;
    const int ctiles = (int)((px + cls_tile_px(c->tune) - 1) / cls_tile_px(c->tune));
    const int mtiles = (int)((H + c->tune.morph_rows - 1) / c->tune.morph_rows);
    const int nops = 2 * (c->p.open_iters + c->p.close_iters);
    fizi_pointer *internal = reinterpret_cast<fizi_pointer *>(c->d + c->L.ptrs);
    for (int f0 = 0; f0 < n_frames; f0 += c->chunk) {
        const int m = std::min(c->chunk, n_frames - f0);
        int slot;
        if ((rc = take_slot(c, &slot)))
            return rc;
        Table *h = c->h_tab[slot];
        h->h.njobs = m;
        for (int i = 0; i <= m; ++i) {
            h->h.gain_pre[i] = i * gtiles;
            h->h.cls_pre[i] = i * ctiles;
            h->h.mor_pre[i] = i * mtiles;
        }
        const uint64_t fbase = c->next_frame + (uint64_t)f0;
        for (int i = 0; i < m; ++i) {
            Job &J = h->jobs[i];
            fill_job_common(c, J);
            uint8_t *slotp = c->d + c->L.slots + (size_t)i * c->L.slot_stride;
            const size_t f = (size_t)(f0 + i);
            J.frame = d_frames + f * px * 3;
            J.raw = reinterpret_cast<uint64_t *>(slotp + c->L.raw);
            J.fizi = d_fizi_bits ? d_fizi_bits + f * words : reinterpret_cast<uint64_t *>(slotp + c->L.fz);
            J.hand = d_hand_bits ? d_hand_bits + f * words : nullptr;
            J.parent = reinterpret_cast<uint32_t *>(slotp + c->L.parent);
            J.area = reinterpret_cast<uint32_t *>(slotp + c->L.area);
            J.runs = reinterpret_cast<uint2 *>(slotp + c->L.runs);
            J.out = d_pointers ? d_pointers + f : internal + i;
            J.frame_index = fbase + (uint64_t)i;
        }
        Table *dt = dev_table(c, slot);
        FIZI_HIP(hipMemcpyAsync(dt, h, table_bytes(m), hipMemcpyHostToDevice, s));
        FIZI_STAGE(c, FIZI_STAGE_GAIN, s, launch_gain(dt, m * gtiles, c->n_cu, c->tune, s));
        FIZI_STAGE(c, FIZI_STAGE_CLASSIFY, s, launch_classify(dt, m * ctiles, c->n_cu, c->tune, s));
        FIZI_STAGE(c, FIZI_STAGE_MORPH, s,
                   launch_morph(dt, m * mtiles, (int)(W / 64), nops, c->n_cu, c->tune, s));
        FIZI_STAGE(c, FIZI_STAGE_RESOLVE, s, launch_resolve(dt, m, s));
        // pointers into the host ring for get_pointer
        const fizi_pointer *src = d_pointers ? d_pointers + f0 : internal;
        int done = 0;
        while (done < m) {
            const size_t pos = (size_t)((fbase + done) % kRing);
            const int n = (int)std::min<size_t>(m - done, kRing - pos);
            FIZI_HIP(hipMemcpyAsync(c->h_ring + pos, src + done, n * sizeof(fizi_pointer),
                                    hipMemcpyDeviceToHost, s));
            done += n;
        }
        if ((rc = finish_call(c, slot, s)))
            return rc;
        fizi_ctx::Rec &r = c->recs[c->next_rec];
        c->next_rec = (c->next_rec + 1) % kRecs;
        r.f0 = fbase;
        r.f1 = fbase + m;
        r.slot = slot;
        r.valid = true;
    }
    c->next_frame += (uint64_t)n_frames;
    return FIZI_OK;
}

int get_pointer(fizi_ctx *c, int64_t frame_index, fizi_pointer *h_out)
{
    if (!c || !h_out)
        return fail(FIZI_EINVAL, "null context or output");
    if (frame_index < 0 || (uint64_t)frame_index >= c->next_frame)
        return fail(FIZI_ERANGE, "frame not submitted yet");
    if ((uint64_t)frame_index + kRing < c->next_frame)
        return fail(FIZI_ERANGE, "frame no longer kept (older than the last 65536)");
    // chunks run in submission order, so the first recorded chunk that ends
    // after the frame finishes no earlier than the frame's own chunk
    int best = -1;
    for (int i = 0; i < kRecs; ++i) {
        const fizi_ctx::Rec &r = c->recs[i];
        if (r.valid && r.f1 > (uint64_t)frame_index && (best < 0 || r.f0 < c->recs[best].f0))
            best = i;
    }
    if (best < 0)
        return fail(FIZI_ERANGE, "frame record missing");
    FIZI_HIP(hipEventSynchronize(c->tab_ev[c->recs[best].slot]));
    *h_out = c->h_ring[(size_t)frame_index % kRing];
    return FIZI_OK;
}

int fizi_stage_timing(fizi_ctx *c, int32_t enable)
{
    if (!c)
        return fail(FIZI_EINVAL, "null context");
    if (enable && !c->timing) {
        for (int st = 0; st < FIZI_NSTAGES; ++st) {
            if (c->tev[st].empty()) {
                c->tev[st].resize(2 * kTimedLaunches, nullptr);
                for (auto &e : c->tev[st])
                    FIZI_HIP(hipEventCreate(&e));
            }
            c->tused[st] = 0;
            c->tms[st] = 0.0;
            c->tcount[st] = 0;
        }
    }
    c->timing = enable != 0;
    return FIZI_OK;
}

int fizi_stage_times(fizi_ctx *c, double *h_ms, int64_t *h_launches)
{
    if (!c || !h_ms || !h_launches)
        return fail(FIZI_EINVAL, "null argument");
    for (int st = 0; st < FIZI_NSTAGES; ++st) {
        for (int i = 0; i < c->tused[st]; ++i) {
            FIZI_HIP(hipEventSynchronize(c->tev[st][2 * i + 1]));
            float ms = 0.f;
            FIZI_HIP(hipEventElapsedTime(&ms, c->tev[st][2 * i], c->tev[st][2 * i + 1]));
            c->tms[st] += ms;
            c->tcount[st] += 1;
        }
        c->tused[st] = 0;
        h_ms[st] = c->tms[st];
        h_launches[st] = c->tcount[st];
        c->tms[st] = 0.0;
        c->tcount[st] = 0;
    }
    return FIZI_OK;
}

int fizi_destroy(fizi_ctx *c)
{
    if (!c)
        return FIZI_OK;
    if (c->have_last)
        (void)hipEventSynchronize(c->order_ev);
    for (int st = 0; st < FIZI_NSTAGES; ++st)
        for (auto &e : c->tev[st])
            if (e)
                (void)hipEventDestroy(e);
    for (int i = 0; i < kTabSlots; ++i) {
        if (c->h_tab[i])
            (void)hipHostFree(c->h_tab[i]);
        if (c->tab_ev[i])
            (void)hipEventDestroy(c->tab_ev[i]);
    }
    if (c->h_ring)
        (void)hipHostFree(c->h_ring);
    if (c->order_ev)
        (void)hipEventDestroy(c->order_ev);
    delete c;
    return FIZI_OK;
}

}  // extern "C"
