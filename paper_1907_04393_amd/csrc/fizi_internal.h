// Internal layout shared by the HIP kernels and the C-ABI host code.
//
// Work is described by a job table in device memory: one Job per frame to
// process (a frame of a context's stream, or a learning frame), with the
// pointers to its inputs, outputs and scratch, its geometry and thresholds,
// and a few accumulators the kernels update atomically. The host fills the
// table in pinned memory and copies it to the device ahead of the kernels,
// which also zeroes the accumulators for that call. Every kernel walks a flat
// list of tiles (grid-stride) and finds a tile's job by binary search in a
// prefix array, so one launch covers frames of any mix of resolutions and a
// launch's shape does not depend on the work it is given. The persistent
// step instead takes work items from an ordered queue (see TableHeader).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fizi.h"

namespace fizi {

constexpr int kMaxJobs = 256;          // jobs per table
constexpr uint16_t kYrefClipped = 0xFFFFu;
constexpr int kMaxMorphIters = 3;      // open_iters, close_iters <= 3
constexpr int kGainSlots = 16;         // gain sums are spread over 16 accumulators
constexpr int kGainRows = 4;           // sampled rows per gain tile

// Skin-hue test on one RGB triple, without division (Section 3.1 (iii)).
// For a hue a, let d_a be an RGB colour of hue a. The determinant
// D(a, p) = det[(1,1,1), d_a, p] = kr (R - B) + kg (G - B) is positive exactly
// when the hue of p lies in the open half-turn (a, a + 180) and zero when it
// is a or a + 180, because the hexcone hue is a monotone, odd-symmetric
// re-parametrisation of the angle around the gray axis. The closed interval
// [a1, a2] of length L is then
//   L = 0:        D1 == 0 and p points along d_a1 (3 d.p - sum(d) sum(p) > 0)
//   0 < L < 180:  D1 >= 0 and D2 <= 0
//   L = 180:      D1 >= 0
//   L > 180:      D1 >= 0 or D2 <= 0
// always together with chroma > 0.
struct HueTest {
    int32_t k1r, k1g;          // D(a1, p) coefficients
    int32_t k2r, k2g;          // D(a2, p) coefficients
    int32_t dr, dg, db, dsum;  // d_a1 (scaled by 6000) for the one-point case
    int32_t mode;              // 0: L = 0, 1: 0 < L < 180, 2: L = 180, 3: L > 180
    int32_t pad;
};

// Temporal tracking state of one stream (device memory): the previous
// frame's centroid pixel, valid when that frame had a hand, and the click
// debouncer (bit 0: the reported click; bits 8..15: consecutive frames whose
// own click differs from it).
struct TrackState {
    int32_t valid, x, y;
    uint32_t click;
};

struct Job {
    const uint8_t *frame;      // H*W*3
    const uint8_t *bgmin;      // H*W*3
    const uint8_t *bgmax;      // H*W*3
    const uint16_t *yref;      // ceil(H/rs) * W
    uint64_t *raw;             // H*Wd words: AND of the three masks
    uint64_t *fizi;            // H*Wd words: after opening and closing
    uint64_t *hand;            // H*Wd words or null
    uint32_t *parent;          // W*H: union-find parent, valid at run starts
    uint32_t *bflag;           // per row band of the persistent step: epoch when classified
    uint32_t *area;            // W*H: component area, valid at roots
    uint2 *runs;               // run_cap runs (first pixel, last pixel | link flag)
    uint2 *links;              // link_cap pairs of run starts to join
    fizi_pointer *out;         // one pointer
    fizi_pointer *hout;        // its slot in a host ring (pinned, device-mapped), or null
    TrackState *track;         // the stream's tracking state, or null (largest component)
    uint64_t frame_index;
    int32_t W, H, Wd, rs;
    uint32_t run_cap, link_cap;
    uint32_t epoch;            // this dispatch's number for its scratch slot (never 0)
    int32_t band;              // morphology band height (rows)
    int32_t mgroup;            // morphology lanes per row: 64, or 16 / 32 to pack 4 / 2 bands per wave
    int32_t delta, S1, open_it, close_it, min_area, fill_pm, glo, ghi;
    int32_t scaled;            // thresholds scaled by the gain instead of corrected pixels
    uint32_t S_q16;            // max(S * 2^16, 1): the gray tolerance against (max - min) * inv
    int32_t debounce;          // tracked streams: frames a change of the click needs
    uint32_t track_r2;         // tracked streams: squared radius of the nearest-component pick
    int32_t S0;                // gray tolerance S as given
    int32_t lum2;              // over-exposure filter: 2 lum_hi, 0 when off
    HueTest hue;
    // accumulators (zero when the table is uploaded)
    // gain sums over usable sampled pixels, sampled row r adding to slot
    // r % kGainSlots (fewer same-address atomics)
    unsigned long long num[kGainSlots], den[kGainSlots];
    uint32_t nruns, flags, nlinks, nflag;
    uint32_t gain_done, morph_done;   // persistent step: finished gain tiles, morphology bands
    uint32_t ginv;                    // persistent step: 0x80000000 | inverse gain, once known
    uint32_t pick;                    // deferred tracking: root of the largest component (or none)
};

// The persistent step's queue: segments of work items, in order
//   gain(o0), ..., gain(o[n-1]), bands(o0), ..., bands(o[n-1])
// over the jobs o sorted by size, largest first. A gain item is one gain
// tile; a band item is 4 * band rows: classify them, then run the
// morphology of the band above (and, for the last band, of this one) and,
// when a frame's last band is done, its components. An item only ever waits
// for items earlier in the queue.
struct TableHeader {
    int32_t njobs;
    int32_t flow_nseg;                    // 2 * njobs
    int32_t gain_pre[kMaxJobs + 1];   // gain tiles (kGainRows sampled rows)
    int32_t cls_pre[kMaxJobs + 1];    // classify tiles
    int32_t mor_pre[kMaxJobs + 1];    // morphology items (64 / mgroup bands each)
    int32_t flow_pre[2 * kMaxJobs + 1];   // first item of each queue segment
    int32_t flow_seg[2 * kMaxJobs];       // (job << 1) | (0: gain, 1: bands)
};

struct Table {
    TableHeader h;
    Job jobs[kMaxJobs];
};

static_assert(sizeof(TableHeader) % 8 == 0, "job array alignment");

// Launch shapes (tunable per resolution class).
struct Tuning {
    int cls_iters;      // classify tile = 1024 * cls_iters pixels (1, 2, 4, 8)
    int morph_rows;     // morphology band height (8, 16, 32, 64)
    int grid_per_cu;    // resident blocks per CU for the streaming kernels
    int short_bands = 1;   // launches too small to fill the device take short morphology bands
};

inline int cls_tile_px(const Tuning &t) { return 1024 * t.cls_iters; }

// Counters of the persistent step (device memory, zero between launches).
struct PersistState {
    unsigned int next;       // next queue item of the current launch
    unsigned int finished;   // blocks done with the current launch
    unsigned int error;      // a bounded wait gave up (sticky until read)
    unsigned int pad[61];
};
inline size_t persist_state_bytes() { return sizeof(PersistState); }

// Optional start/stop events taken from a kernel's own dispatch (measurement).
struct StageEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};

// Launches go through hipExtLaunchKernelGGL so that, when the caller asks for
// it, the start/stop events are taken from the kernel's own dispatch. `ev`
// is evaluated more than once: pass a variable.
#define FIZI_LAUNCH(kern, grid, block, lds, s, ev, ...)                                              \
    do {                                                                                           \
        if ((ev).start || (ev).stop)                                                               \
            hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, (ev).start, (ev).stop, 0, \
                                  __VA_ARGS__);                                                    \
        else                                                                                       \
            hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, __VA_ARGS__);                \
    } while (0)

// The per-call fields of job 0 of a one-frame launch, passed to the gain
// kernel by value when the table slot on the device already holds the rest
// of the job (valid != 0): the gain reads its frame from here, and its
// first workgroup writes these fields into the job for the kernels after it.
struct CallPatch {
    const uint8_t *frame;
    uint64_t *fizi, *hand;
    fizi_pointer *out, *hout;
    uint64_t frame_index;
    int32_t valid;
};

// Kernel launchers (fizi_kernels.hip). Each returns the hipError_t of its launch.
hipError_t launch_make_yref(const uint8_t *frame0, uint16_t *yref, int W, int H, int rs,
                            hipStream_t s);
hipError_t launch_gain(const Table *d_tab, int total_tiles, int n_cu, const Tuning &t,
                       hipStream_t s, StageEvents ev = {}, const CallPatch *patch = nullptr);
hipError_t launch_minmax(const Table *d_tab, int njobs, uint8_t *bgmin, uint8_t *bgmax,
                         int npx, int reset, bool masked, int n_cu, hipStream_t s, StageEvents ev = {});
hipError_t launch_classify(const Table *d_tab, int total_tiles, int n_cu, const Tuning &t,
                           hipStream_t s, StageEvents ev = {});
hipError_t launch_morph(const Table *d_tab, int total_tiles, int max_wd, int max_ops, int n_cu,
                        const Tuning &t, hipStream_t s, StageEvents ev = {});
// serial: one workgroup takes the jobs in table order (consecutive frames of
// one tracked stream); small: 256-thread workgroups, for a launch that runs
// beside a streaming kernel; clear_acc: each job's accumulators are zeroed
// once read (its table slot is then reused without an upload).
hipError_t launch_resolve(const Table *d_tab, int njobs, hipStream_t s, StageEvents ev = {}, bool serial = false,
                          bool small = false, bool clear_acc = false);
hipError_t launch_persistent(const Table *d_tab, int max_wd, int max_ops, int n_cu, const Tuning &t,
                             uint8_t *persist, hipStream_t s, StageEvents ev = {});
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);

}  // namespace fizi
