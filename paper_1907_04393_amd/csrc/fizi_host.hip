// Shared host-side building blocks (see fizi_host.h).
#include <algorithm>
#include <climits>
#include <cstring>

#include "fizi_host.h"

namespace fizi {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

}  // namespace fizi

extern "C" const char *fizi_last_error(void) { return fizi::g_err.c_str(); }

namespace fizi {

namespace {

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

}  // namespace

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
    if (p->brightness_mode != 0 && p->brightness_mode != 1)
        return fail(FIZI_EINVAL, "brightness_mode must be 0 or 1");
    if (p->click_debounce < 0 || p->click_debounce > 255)
        return fail(FIZI_EINVAL, "click_debounce must be in 0..255");
    if (p->track_radius < 0 || p->track_radius > 16384)
        return fail(FIZI_EINVAL, "track_radius must be in 0..16384");
    if (p->lum_hi != 0 && (p->lum_hi < 128 || p->lum_hi > 254))
        return fail(FIZI_EINVAL, "lum_hi must be 0 (off) or in 128..254");
    if (p->lum_hi != 0 && p->brightness_mode != 0)
        return fail(FIZI_EINVAL, "the over-exposure filter (lum_hi) works on corrected pixels: brightness_mode 0");
    return FIZI_OK;
}

int morph_ops(const fizi_params &p) { return 2 * (p.open_iters + p.close_iters); }

Tuning tuning_for(int max_width, int max_ops, bool batch)
{
    (void)max_width;
    (void)max_ops;
    Tuning t;
    t.cls_iters = 4;
    if (batch) {
        // the autotuner's pick on the 64-stream 640x480..3840x2160 workload
        // in the pipelined launch mode: 8 pixel groups per classify lane,
        // 16-row bands and a grid of 64 blocks per CU for the streaming
        // kernels (eight rounds of resident blocks even out the tail, and
        // leave slots free often enough for the back half that runs beside
        // them)
        t.cls_iters = 8;
        t.grid_per_cu = 64;
        t.morph_rows = 16;
    } else {
        // one stream (measured at 1920x1080): 8-row bands give a one-frame
        // call twice the morphology waves (p50 latency 0.10 ms against 0.13
        // with 16 rows) at the same chunked throughput
        t.grid_per_cu = 32;
        t.morph_rows = 8;
    }
    return t;
}

size_t model_bytes(const fizi_geom &g, const fizi_params &p)
{
    const size_t px = (size_t)g.width * g.height;
    const size_t rows = (g.height + p.gain_row_stride - 1) / p.gain_row_stride;
    return 2 * align256(px * 3) + align256(rows * g.width * 2) + align256(sizeof(TrackState));
}

void model_at(Model &m, const fizi_geom &g, const fizi_params &p, uint8_t *base)
{
    const size_t px = (size_t)g.width * g.height;
    m.g = g;
    m.p = p;
    m.hue = make_hue(p.alpha1_cdeg, p.alpha2_cdeg);
    m.yref_rows = (g.height + p.gain_row_stride - 1) / p.gain_row_stride;
    m.bgmin = base;
    m.bgmax = base + align256(px * 3);
    m.yref = reinterpret_cast<uint16_t *>(base + 2 * align256(px * 3));
    m.track = reinterpret_cast<TrackState *>(base + 2 * align256(px * 3) +
                                             align256((size_t)m.yref_rows * g.width * 2));
    m.learned = false;
    m.tracking = false;
}

size_t slot_bytes(const fizi_geom &g)
{
    const size_t px = (size_t)g.width * g.height, words = (size_t)g.height * (g.width / 64);
    return 2 * align256(words * 8) + 2 * align256(px * 4) + align256((px / 2) * 8) + align256((px / 8) * 8) +
           align256(flag_words(g) * 4);
}

Slot slot_at(const fizi_geom &g, uint8_t *base)
{
    const size_t px = (size_t)g.width * g.height, words = (size_t)g.height * (g.width / 64);
    Slot s;
    size_t o = 0;
    s.raw = reinterpret_cast<uint64_t *>(base + o);
    o += align256(words * 8);
    s.fz = reinterpret_cast<uint64_t *>(base + o);
    o += align256(words * 8);
    s.parent = reinterpret_cast<uint32_t *>(base + o);
    o += align256(px * 4);
    s.area = reinterpret_cast<uint32_t *>(base + o);
    o += align256(px * 4);
    s.runs = reinterpret_cast<uint2 *>(base + o);
    s.run_cap = (uint32_t)(px / 2);      // the most runs a mask can have
    o += align256((px / 2) * 8);
    // joins across band and segment borders; beyond this many, runs are
    // flagged for the component stage instead
    s.links = reinterpret_cast<uint2 *>(base + o);
    s.link_cap = (uint32_t)(px / 8);
    o += align256((px / 8) * 8);
    s.bflag = reinterpret_cast<uint32_t *>(base + o);
    s.nflags = flag_words(g);
    return s;
}

void fill_job(const Model &m, int band, Job &J, bool pack)
{
    std::memset(&J, 0, sizeof(J));
    J.bgmin = m.bgmin;
    J.bgmax = m.bgmax;
    J.yref = m.yref;
    J.W = m.g.width;
    J.H = m.g.height;
    J.Wd = m.g.width / 64;
    J.rs = m.p.gain_row_stride;
    J.band = band;
    // narrow frames under the default opening and closing share a wave
    // between bands: 4 bands of at most 16 words, or 2 of at most 32
    const bool packable = pack && m.p.open_iters == 1 && m.p.close_iters == 1;
    J.mgroup = !packable ? 64 : (J.Wd <= 16 ? 16 : (J.Wd <= 32 ? 32 : 64));
    J.delta = m.p.bg_delta;
    J.S1 = std::max(m.p.gray_S, 1);
    J.open_it = m.p.open_iters;
    J.close_it = m.p.close_iters;
    J.min_area = m.p.min_area;
    J.fill_pm = m.p.click_fill_permille;
    J.glo = m.p.gain_lo_q16;
    J.ghi = m.p.gain_hi_q16;
    J.scaled = m.p.brightness_mode;
    J.S_q16 = std::max((uint32_t)m.p.gray_S << 16, 1u);
    J.debounce = m.p.click_debounce;
    J.track_r2 = (uint32_t)m.p.track_radius * (uint32_t)m.p.track_radius;
    J.S0 = m.p.gray_S;
    J.lum2 = 2 * m.p.lum_hi;
    J.hue = m.hue;
    J.track = m.tracking ? m.track : nullptr;
}

void set_scratch(Job &J, const Slot &s)
{
    J.raw = s.raw;
    J.fizi = s.fz;
    J.parent = s.parent;
    J.area = s.area;
    J.runs = s.runs;
    J.run_cap = s.run_cap;
    J.links = s.links;
    J.link_cap = s.link_cap;
    J.bflag = s.bflag;
}

void set_prefixes(Table &T, int njobs, const Tuning &t)
{
    T.h.njobs = njobs;
    T.h.gain_pre[0] = T.h.cls_pre[0] = T.h.mor_pre[0] = 0;
    const int ctile = cls_tile_px(t);
    for (int i = 0; i < njobs; ++i) {
        const Job &J = T.jobs[i];
        const long px = (long)J.W * J.H;
        const int rows = (J.H + J.rs - 1) / J.rs;
        T.h.gain_pre[i + 1] = T.h.gain_pre[i] + (rows + kGainRows - 1) / kGainRows;
        T.h.cls_pre[i + 1] = T.h.cls_pre[i] + (int)((px + ctile - 1) / ctile);
        const int bands = (J.H + J.band - 1) / J.band, per = 64 / J.mgroup;
        T.h.mor_pre[i + 1] = T.h.mor_pre[i] + (bands + per - 1) / per;
    }
    // the persistent step's queue: jobs by size, largest first; every gain
    // tile ahead of the bands, so that a band rarely waits for its frame's
    // gain
    int order[kMaxJobs];
    for (int i = 0; i < njobs; ++i)
        order[i] = i;
    std::stable_sort(order, order + njobs, [&](int a, int b) {
        return (long)T.jobs[a].W * T.jobs[a].H > (long)T.jobs[b].W * T.jobs[b].H;
    });
    int k = 0, item = 0;
    auto push = [&](int j, int type) {
        const int n = type == 0 ? T.h.gain_pre[j + 1] - T.h.gain_pre[j]
                                : (T.jobs[j].H + 4 * T.jobs[j].band - 1) / (4 * T.jobs[j].band);
        T.h.flow_pre[k] = item;
        T.h.flow_seg[k] = (j << 1) | type;
        item += n;
        ++k;
    };
    for (int i = 0; i < njobs; ++i)
        push(order[i], 0);
    for (int i = 0; i < njobs; ++i)
        push(order[i], 1);
    T.h.flow_nseg = k;
    T.h.flow_pre[k] = item;
}

int TableRing::init(uint8_t *d_base)
{
    for (int i = 0; i < kTabSlots; ++i) {
        d[i] = reinterpret_cast<Table *>(d_base + i * align256(sizeof(Table)));
        FIZI_HIP(hipHostMalloc(reinterpret_cast<void **>(&h[i]), sizeof(Table), hipHostMallocDefault));
        std::memset(h[i], 0, sizeof(Table));
        // the host only waits for the slot's kernels to be done with it
        FIZI_HIP(hipEventCreateWithFlags(&ev[i], kDeviceOrderEvent));
    }
    return FIZI_OK;
}

void TableRing::destroy()
{
    for (int i = 0; i < kTabSlots; ++i) {
        if (used[i] && ev[i])
            (void)hipEventSynchronize(ev[i]);
        if (h[i])
            (void)hipHostFree(h[i]);
        if (ev[i])
            (void)hipEventDestroy(ev[i]);
        h[i] = nullptr;
        ev[i] = nullptr;
    }
}

int TableRing::take(int *slot)
{
    const int s = next;
    next = (next + 1) % kTabSlots;
    if (used[s])
        FIZI_HIP(hipEventSynchronize(ev[s]));
    *slot = s;
    return FIZI_OK;
}

int TableRing::finish(int slot, hipStream_t s)
{
    FIZI_HIP(hipEventRecord(ev[slot], s));
    used[slot] = true;
    return FIZI_OK;
}

int StageClock::enable(bool want)
{
    if (want && !on) {
        for (int st = 0; st < FIZI_NSTAGES; ++st) {
            if (ev[st].empty()) {
                ev[st].resize(2 * kTimedLaunches, nullptr);
                for (auto &e : ev[st])
                    FIZI_HIP(hipEventCreate(&e));
            }
            used[st] = 0;
        }
    }
    on = want;
    return FIZI_OK;
}

StageEvents StageClock::next(int stage)
{
    StageEvents e;
    if (!on || used[stage] >= kTimedLaunches)
        return e;
    const int i = used[stage]++;
    e.start = ev[stage][2 * i];
    e.stop = ev[stage][2 * i + 1];
    return e;
}

int StageClock::read(double *ms, int64_t *n)
{
    for (int st = 0; st < FIZI_NSTAGES; ++st) {
        double tot = 0.0;
        for (int i = 0; i < used[st]; ++i) {
            FIZI_HIP(hipEventSynchronize(ev[st][2 * i + 1]));
            float t = 0.f;
            FIZI_HIP(hipEventElapsedTime(&t, ev[st][2 * i], ev[st][2 * i + 1]));
            tot += t;
        }
        ms[st] = tot;
        n[st] = used[st];
        used[st] = 0;
    }
    return FIZI_OK;
}

void StageClock::destroy()
{
    for (int st = 0; st < FIZI_NSTAGES; ++st) {
        for (auto &e : ev[st])
            if (e)
                (void)hipEventDestroy(e);
        ev[st].clear();
    }
}

int device_cu_count(int *device, int *n_cu)
{
    FIZI_HIP(hipGetDevice(device));
    FIZI_HIP(hipDeviceGetAttribute(n_cu, hipDeviceAttributeMultiprocessorCount, *device));
    return FIZI_OK;
}

int learn_model(Model &m, TableRing &ring, const Tuning &t, int n_cu, const uint8_t *frames, int n,
                int reset, hipStream_t s, StageClock *clk, const uint64_t *masks)
{
    const size_t px = (size_t)m.g.width * m.g.height;
    if (reset)
        FIZI_HIP(launch_make_yref(frames, m.yref, m.g.width, m.g.height, m.p.gain_row_stride, s));
    for (int f0 = 0; f0 < n; f0 += kMaxJobs) {
        const int k = std::min(kMaxJobs, n - f0);
        int slot;
        FIZI_TRY(ring.take(&slot));
        Table &T = *ring.h[slot];
        for (int i = 0; i < k; ++i) {
            fill_job(m, t.morph_rows, T.jobs[i]);
            T.jobs[i].frame = frames + (size_t)(f0 + i) * px * 3;
            if (masks)
                T.jobs[i].fizi = const_cast<uint64_t *>(masks) + (size_t)(f0 + i) * (px / 64);
        }
        set_prefixes(T, k, t);
        FIZI_HIP(hipMemcpyAsync(ring.d[slot], &T, table_bytes(k), hipMemcpyHostToDevice, s));
        FIZI_HIP(launch_gain(ring.d[slot], T.h.gain_pre[k], n_cu, t, s));
        FIZI_HIP(launch_minmax(ring.d[slot], k, m.bgmin, m.bgmax, (int)px, (reset && f0 == 0) ? 1 : 0,
                               masks != nullptr, n_cu, s, clk ? clk->next(FIZI_STAGE_LEARN) : StageEvents{}));
        FIZI_TRY(ring.finish(slot, s));
    }
    m.learned = true;
    return FIZI_OK;
}

int run_front(const Table *d_tab, const Table &h, int njobs, const Tuning &t, int n_cu, bool fixed_grid,
              hipStream_t s, StageClock *clk, const CallPatch *patch)
{
    auto ev = [&](int st) { return clk ? clk->next(st) : StageEvents{}; };
    const int big = INT_MAX / 2;
    FIZI_HIP(launch_gain(d_tab, fixed_grid ? big : h.h.gain_pre[njobs], n_cu, t, s, ev(FIZI_STAGE_GAIN), patch));
    FIZI_HIP(launch_classify(d_tab, fixed_grid ? big : h.h.cls_pre[njobs], n_cu, t, s,
                             ev(FIZI_STAGE_CLASSIFY)));
    return FIZI_OK;
}

int run_back(const Table *d_tab, const Table &h, int njobs, int max_jobs, int max_wd, int max_ops,
             const Tuning &t, int n_cu, bool fixed_grid, hipStream_t s, StageClock *clk, bool beside,
             bool clear_acc)
{
    auto ev = [&](int st) { return clk ? clk->next(st) : StageEvents{}; };
    const int big = INT_MAX / 2;
    FIZI_HIP(launch_morph(d_tab, fixed_grid ? big : h.h.mor_pre[njobs], max_wd, max_ops, n_cu, t, s,
                          ev(FIZI_STAGE_MORPH)));
    // tracked consecutive frames of one stream are resolved in order
    const bool serial = njobs > 1 && h.jobs[0].track != nullptr && h.jobs[1].track == h.jobs[0].track;
    FIZI_HIP(launch_resolve(d_tab, fixed_grid ? max_jobs : njobs, s, ev(FIZI_STAGE_RESOLVE), serial, beside,
                            clear_acc));
    return FIZI_OK;
}

int run_pipeline(const Table *d_tab, const Table &h, int njobs, int max_jobs, int max_wd, int max_ops,
                 const Tuning &t, int n_cu, bool fixed_grid, hipStream_t s, StageClock *clk, const CallPatch *patch)
{
    FIZI_TRY(run_front(d_tab, h, njobs, t, n_cu, fixed_grid, s, clk, patch));
    return run_back(d_tab, h, njobs, max_jobs, max_wd, max_ops, t, n_cu, fixed_grid, s, clk, false,
                    patch != nullptr);
}

}  // namespace fizi
