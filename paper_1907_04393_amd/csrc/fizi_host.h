// Host-side building blocks shared by the single-stream context
// (fizi_capi.hip) and the multi-stream batch (fizi_batch.hip): parameter
// checks, the background model and scratch layouts, job tables, the launch
// sequence of one pipeline pass, and the stage clock.
#pragma once

#include <string>
#include <vector>

#include "fizi_internal.h"

namespace fizi {

int fail(int code, const std::string &msg);

#define FIZI_HIP(expr)                                                                          \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return ::fizi::fail(FIZI_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

#define FIZI_TRY(expr)          \
    do {                        \
        int rc_ = (expr);       \
        if (rc_ != FIZI_OK)     \
            return rc_;         \
    } while (0)

constexpr int kMaxW = 8192;
constexpr int kMaxH = 8192;
constexpr int kTabSlots = 8;
constexpr int kTimedLaunches = 16384;

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int validate(const fizi_geom *g, const fizi_params *p);
HueTest make_hue(int a1, int a2);
// Launch shapes for frames up to max_width wide and max_ops morphology steps,
// for a multi-stream batch or a single-stream context.
Tuning tuning_for(int max_width, int max_ops, bool batch);
int morph_ops(const fizi_params &p);

// Background model of one stream (Section 3.1 (i)) and its reference
// luminance rows (Section 3.2), inside a device block.
struct Model {
    fizi_geom g{};
    fizi_params p{};
    HueTest hue{};
    uint8_t *bgmin = nullptr;
    uint8_t *bgmax = nullptr;
    uint16_t *yref = nullptr;
    int yref_rows = 0;
    TrackState *track = nullptr;       // device memory, after the reference luminance
    bool learned = false;
    bool tracking = false;
};
size_t model_bytes(const fizi_geom &g, const fizi_params &p);
void model_at(Model &m, const fizi_geom &g, const fizi_params &p, uint8_t *base);

// Scratch of one frame in flight.
struct Slot {
    uint64_t *raw = nullptr;
    uint64_t *fz = nullptr;
    uint32_t *parent = nullptr;
    uint32_t *area = nullptr;
    uint2 *runs = nullptr;
    uint2 *links = nullptr;
    uint32_t *bflag = nullptr;           // persistent step: per band epoch
    uint32_t run_cap = 0, link_cap = 0;
    size_t nflags = 0;
};
// Band flags of the persistent step: one per 32 rows (its smallest band).
inline size_t flag_words(const fizi_geom &g) { return (size_t)(g.height + 31) / 32; }
size_t slot_bytes(const fizi_geom &g);
Slot slot_at(const fizi_geom &g, uint8_t *base);

// Job for one frame of a stream: model and thresholds; the caller sets the
// frame, scratch, outputs and frame index.
// band: the morphology band height in rows; pack: narrow frames may share a
// wave between bands (2 or 4 per wave)
void fill_job(const Model &m, int band, Job &J, bool pack = true);

// Morphology band height of launches too small to fill the device.
constexpr int kShortBand = 4;
void set_scratch(Job &J, const Slot &s);
// Tile prefix arrays of a table whose first njobs jobs are filled.
void set_prefixes(Table &T, int njobs, const Tuning &t);
inline size_t table_bytes(int njobs) { return sizeof(TableHeader) + (size_t)njobs * sizeof(Job); }

// Job tables: pinned staging copies, device copies, one event per slot.
struct TableRing {
    Table *h[kTabSlots] = {};
    Table *d[kTabSlots] = {};
    hipEvent_t ev[kTabSlots] = {};
    bool used[kTabSlots] = {};
    int next = 0;
    static size_t device_bytes() { return kTabSlots * align256(sizeof(Table)); }
    int init(uint8_t *d_base);
    void destroy();
    int take(int *slot);                 // waits until the slot's last call is done
    int finish(int slot, hipStream_t s); // records the slot's event on s
};

// Per-stage launch timing from the kernels' own dispatch events.
// Flags of the events that only order device work after other device work
// on the same GPU (a kernel's outputs read by a kernel on another stream, a
// buffer reused once the kernels reading it are done), or that the host
// waits on for completion alone, reading nothing the device wrote to host
// memory: no system-scope fence, which would write back the caches for the
// host at every record. The kernels' own dispatch fences make their writes
// visible to the device. An event that orders kernels after a host-to-device
// copy, or host reads after a device-to-host copy, keeps the default flags.
constexpr unsigned kDeviceOrderEvent = hipEventDisableTiming | hipEventDisableSystemFence;

struct StageClock {
    bool on = false;
    std::vector<hipEvent_t> ev[FIZI_NSTAGES];
    int used[FIZI_NSTAGES] = {};
    int enable(bool on);
    StageEvents next(int stage);
    int read(double *ms, int64_t *n);
    void destroy();
};

int device_cu_count(int *device, int *n_cu);

// Background learning of one stream from n frames (reset: reference from
// frames[0], model starts empty).
// Learning (and, with masks, partial re-learning: n I_FIZI bit masks whose
// set bits keep a frame's pixels out of the model).
int learn_model(Model &m, TableRing &ring, const Tuning &t, int n_cu, const uint8_t *frames, int n,
                int reset, hipStream_t s, StageClock *clk, const uint64_t *masks = nullptr);

// Enqueues gain, classify, morphology and components for the jobs of the
// table in device memory. With fixed_grid the launch shapes do not depend on
// the number of jobs (for graph capture); max_jobs bounds the resolve grid.
// patch: a one-frame launch whose slot was not uploaded again (job 0's
// per-call fields go with the gain launch, and the component stage zeroes
// the job's accumulators after use, for the next such launch).
int run_pipeline(const Table *d_tab, const Table &h, int njobs, int max_jobs, int max_wd, int max_ops,
                 const Tuning &t, int n_cu, bool fixed_grid, hipStream_t s, StageClock *clk,
                 const CallPatch *patch = nullptr);
// Its two halves: gain and classify (the front, which reads the frames and
// writes the raw bits), then morphology and components (the back, which
// reads the raw bits and writes I_FIZI and the pointers). beside: the back
// half runs beside another step's front (smaller component workgroups).
int run_front(const Table *d_tab, const Table &h, int njobs, const Tuning &t, int n_cu, bool fixed_grid,
              hipStream_t s, StageClock *clk, const CallPatch *patch = nullptr);
int run_back(const Table *d_tab, const Table &h, int njobs, int max_jobs, int max_wd, int max_ops,
             const Tuning &t, int n_cu, bool fixed_grid, hipStream_t s, StageClock *clk, bool beside = false,
             bool clear_acc = false);

}  // namespace fizi
