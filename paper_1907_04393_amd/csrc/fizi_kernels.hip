// HIP kernels of the FIZI/Mouse pipeline for gfx950 (CDNA4, wave64).
//
//   k_make_yref  reference luminance of the sampled rows of the first
//                learning frame (Section 2 initialisation, Section 3.2)
//   k_gain       per-frame sums over the usable sampled pixels; each consumer
//                turns a frame's sums into its Q16 inverse gain
//   k_minmax     background learning and partial re-learning: per-pixel,
//                per-channel min/max of the gain-corrected frames, model read
//                and written once (Section 3.1 (i), Section 3.3)
//   k_classify   gain correction (or thresholds scaled by the gain), I_R1
//                (outside the learned box), I_R2 (not gray), I_R3 (skin hue),
//                their AND, packed to bits by DPP row merges (Sections 3.1,
//                3.2); HBM-bound, 4 pixels per lane
//   k_morph      opening then closing with a 3x3 square, streamed through a
//                register pipeline of bit rows (64 pixels per lane word), then
//                runs and band-local components in LDS (Section 3.1, last
//                paragraph)
//   k_resolve    8-connected components by union-find over runs, hand-zone
//                selection (largest, or tracked), the pointer (Section 2,
//                Mouse module)
//   k_flow       the persistent form of one step: gain tiles and row bands
//                from one ordered queue, with bounded waits
#include <hip/hip_ext.h>

#include <algorithm>

#include "fizi_internal.h"

namespace fizi {
namespace {

constexpr int kWave = 64;

#define GLOBAL __attribute__((address_space(1)))

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Pointers in the job table are generic; casting them to the global address
// space lets the compiler emit global_* instead of flat_* accesses.
template <typename T>
__device__ __forceinline__ GLOBAL T *G(T *p)
{
    return (GLOBAL T *)p;
}

// A frame's union-find forest is only touched by one workgroup per kernel,
// so its atomics are workgroup-scoped (performed in the XCD's L2, no fences).
__device__ __forceinline__ uint32_t ld_wg(GLOBAL uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void st_wg(GLOBAL uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Accumulators that other workgroups update with atomics (the gain sums, the
// run count) are read with device-scope atomic loads, which bypass the
// scalar cache; in the persistent step they are written earlier in the same
// launch.
template <typename T>
__device__ __forceinline__ T ld_dev(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Persistent step: data that a workgroup hands to another one in the same
// launch is stored with device scope (written through this XCD's L2), each
// wave waits for its stores to complete before the workgroup bumps the
// counter or flag the consumer polls, and the consumer takes a device-scope
// acquire fence after seeing it, so that its loads miss any stale copy.
template <typename T>
__device__ __forceinline__ void st_dev(GLOBAL T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A store of the morphology/classify stages: device scope in the persistent
// step (FLOW), plain otherwise.
template <bool FLOW, typename T>
__device__ __forceinline__ void put(GLOBAL T *p, T v)
{
    if constexpr (FLOW)
        st_dev(p, v);
    else
        *p = v;
}

// Union-find parent stores of the morphology stage.
template <bool FLOW>
__device__ __forceinline__ void put_parent(GLOBAL uint32_t *p, uint32_t v)
{
    if constexpr (FLOW)
        st_dev(p, v);
    else
        st_wg(p, v);
}

__device__ __forceinline__ void wait_own_memory() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ int find_job(const int32_t *pre, int nj, int t)
{
    int lo = 0, hi = nj - 1;          // largest j with pre[j] <= t
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Brightness correction of one channel value (Q16 inverse gain, half up,
// saturated). v < 2^8 and inv <= 2^20 both fit 24 bits, so the full-rate
// 24-bit multiply gives the exact product (< 2^28).
__device__ __forceinline__ uint32_t corr(uint32_t v, uint32_t inv)
{
    uint32_t t = (__umul24(v, inv) + 32768u) >> 16;
    return t < 255u ? t : 255u;
}

// Q16 inverse gain from the sums of reference and frame luminance: rounded
// half up and clamped; 1.0 when no sampled pixel was usable.
__device__ __forceinline__ uint32_t inv_gain(unsigned long long num, unsigned long long den,
                                             int glo, int ghi)
{
    if (den == 0)
        return 65536u;
    unsigned long long q = (num * 65536ull + den / 2) / den;
    if (q < (unsigned long long)glo)
        q = (unsigned long long)glo;
    if (q > (unsigned long long)ghi)
        q = (unsigned long long)ghi;
    return (uint32_t)q;
}

// The frame's inverse gain from its gain accumulators. `same_launch`: the
// sums were written earlier in the same launch (persistent step), so they
// are read with device-scope atomic loads; after a kernel boundary plain
// (scalar) loads see them.
__device__ __forceinline__ uint32_t job_gain(const Job *J, bool same_launch)
{
    unsigned long long n = 0, d = 0;
#pragma unroll
    for (int i = 0; i < kGainSlots; ++i) {
        n += same_launch ? ld_dev(&J->num[i]) : J->num[i];
        d += same_launch ? ld_dev(&J->den[i]) : J->den[i];
    }
    return inv_gain(n, d, J->glo, J->ghi);
}

// Skin-hue membership without division; see HueTest. Chroma > 0 is checked
// by the caller.
// Every factor fits the full-rate 24-bit signed multiply: |k| <= 6000,
// |R - B| <= 255, d <= 6000, sum(d) <= 12000, R + G + B <= 765.
__device__ __forceinline__ bool hue_in(int r, int g, int b, const HueTest &h)
{
    const int rb = r - b, gb = g - b;
    const int d1 = __mul24(h.k1r, rb) + __mul24(h.k1g, gb);
    if (h.mode == 1)
        return (d1 >= 0) & (__mul24(h.k2r, rb) + __mul24(h.k2g, gb) <= 0);
    if (h.mode == 3)
        return (d1 >= 0) | (__mul24(h.k2r, rb) + __mul24(h.k2g, gb) <= 0);
    if (h.mode == 2)
        return d1 >= 0;
    const int dp = __mul24(h.dr, r) + __mul24(h.dg, g) + __mul24(h.db, b);
    return (d1 == 0) & (3 * dp - __mul24(h.dsum, r + g + b) > 0);
}

// hue_in with the interval's case fixed at compile time (no branch on it).
template <int MODE>
__device__ __forceinline__ bool hue_in_mode(int r, int g, int b, const HueTest &h)
{
    const int rb = r - b, gb = g - b;
    const int d1 = __mul24(h.k1r, rb) + __mul24(h.k1g, gb);
    if constexpr (MODE == 1)
        return (d1 >= 0) & (__mul24(h.k2r, rb) + __mul24(h.k2g, gb) <= 0);
    if constexpr (MODE == 3)
        return (d1 >= 0) | (__mul24(h.k2r, rb) + __mul24(h.k2g, gb) <= 0);
    if constexpr (MODE == 2)
        return d1 >= 0;
    const int dp = __mul24(h.dr, r) + __mul24(h.dg, g) + __mul24(h.db, b);
    return (d1 == 0) & (3 * dp - __mul24(h.dsum, r + g + b) > 0);
}

__device__ __forceinline__ uint32_t byte_of(uint32_t w0, uint32_t w1, uint32_t w2, int i)
{
    const uint32_t w = i < 4 ? w0 : (i < 8 ? w1 : w2);
    return (w >> (8 * (i & 3))) & 0xFFu;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1)
        v += __shfl_xor(v, o, kWave);
    return v;
}

// Lane l receives lane l + n of its row of 16 lanes (0 past the row's end,
// by the bound control): DPP row_shl:n.
template <int N>
__device__ __forceinline__ uint32_t row_shl(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x100 + N, 0xF, 0xF, true);
}

// Raster mask words of a wave's 256 consecutive pixels, 4 per lane (bit k of
// nib: pixel 4 l + k). Word w covers lanes 16 w .. 16 w + 15, nibble j from
// lane 16 w + j, so each word is one DPP row: neighbouring lanes' nibbles
// merge pairwise (l takes l + 1, then l + 2, l + 4; l + 8 gives the upper
// half), and lane 16 w ends up holding word w. A handful of instructions per
// wave, where ballots and a bit spread on four lanes took about eighty.
__device__ __forceinline__ uint64_t row_word(uint32_t nib)
{
    uint32_t t = nib & 0xFu;
    t |= row_shl<1>(t) << 4;
    t |= row_shl<2>(t) << 8;
    t |= row_shl<4>(t) << 16;
    return ((uint64_t)row_shl<8>(t) << 32) | t;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_make_yref(const uint8_t *__restrict__ frame0,
                                                   uint16_t *__restrict__ yref, int W, int H,
                                                   int rs)
{
    const int rows = (H + rs - 1) / rs;
    const int groups = W / 4;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rows * groups;
         i += gridDim.x * blockDim.x) {
        const int rr = i / groups, g = i - rr * groups;
        const uint32_t *p = reinterpret_cast<const uint32_t *>(frame0 + (size_t)rr * rs * W * 3) + 3 * g;
        const uint32_t w0 = p[0], w1 = p[1], w2 = p[2];
        uint32_t out[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t r = byte_of(w0, w1, w2, 3 * k), gg = byte_of(w0, w1, w2, 3 * k + 1),
                           b = byte_of(w0, w1, w2, 3 * k + 2);
            const bool ok = (r - 1u < 254u) & (gg - 1u < 254u) & (b - 1u < 254u);
            out[k] = ok ? r + 2 * gg + b : kYrefClipped;
        }
        uint2 v;
        v.x = out[0] | (out[1] << 16);
        v.y = out[2] | (out[3] << 16);
        reinterpret_cast<uint2 *>(yref + (size_t)rr * W)[g] = v;
    }
}

// ---------------------------------------------------------------------------
// One sampled row of one frame: sums of reference and frame luminance over
// its usable pixels, added to the frame's accumulators.
template <int MODE>
__device__ __forceinline__ void gain_tile_mode(Table *__restrict__ T, int j, int tile, const uint8_t *fr)
{
    __shared__ uint32_t s_num[256 / kWave], s_den[256 / kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    Job *J = &T->jobs[j];
    const int W = J->W;
    const int rows = (J->H + J->rs - 1) / J->rs;
    const HueTest h = J->hue;
    uint32_t num = 0, den = 0;
    const int r0 = tile * kGainRows, nr = min(rows, r0 + kGainRows) - r0;
    // one usable-pixel test, summed into num/den; straight-line code (every
    // test evaluated, the sums selected) rather than a branch per pixel
    auto add_px = [&](uint32_t r, uint32_t gg, uint32_t b, uint32_t y) {
        const int mx = max(max((int)r, (int)gg), (int)b);
        const int mn = min(min((int)r, (int)gg), (int)b);
        // every channel in 1..254
        const bool unclipped = (y != kYrefClipped) & (mn >= 1) & (mx <= 254);
        const bool skin = (mx > mn) & hue_in_mode<MODE>((int)r, (int)gg, (int)b, h);
        const bool ok = unclipped & !skin;
        num += ok ? y : 0u;
        den += ok ? r + 2 * gg + b : 0u;
    };
    if ((reinterpret_cast<uintptr_t>(fr) & 15u) == 0) {
        // 16 pixels per item: three 16-byte loads of the frame row, two of
        // the reference row; items of the tile's rows in one flat range
        const int n16 = W / 16;
        const GLOBAL uint8_t *frame = G(fr);
        const GLOBAL uint16_t *yref = G(J->yref);
        const size_t rowb = (size_t)J->rs * W * 3;
#pragma unroll 2
        for (int it = threadIdx.x; it < nr * n16; it += blockDim.x) {
            int row = 0;
#pragma unroll
            for (int q = 1; q < kGainRows; ++q)
                row += it >= q * n16;
            const int g = it - row * n16, rr = r0 + row;
            const GLOBAL u32x4 *fp = reinterpret_cast<const GLOBAL u32x4 *>(frame + (size_t)rr * rowb) + 3 * g;
            const GLOBAL u32x4 *yp = reinterpret_cast<const GLOBAL u32x4 *>(yref + (size_t)rr * W) + 2 * g;
            const u32x4 a = fp[0], b = fp[1], c = fp[2], ya = yp[0], yb = yp[1];
            const uint32_t fw[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
            const uint32_t yw[8] = {ya.x, ya.y, ya.z, ya.w, yb.x, yb.y, yb.z, yb.w};
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int q0 = 3 * k;
                add_px((fw[q0 >> 2] >> (8 * (q0 & 3))) & 0xFFu, (fw[(q0 + 1) >> 2] >> (8 * ((q0 + 1) & 3))) & 0xFFu,
                       (fw[(q0 + 2) >> 2] >> (8 * ((q0 + 2) & 3))) & 0xFFu, (yw[k >> 1] >> (16 * (k & 1))) & 0xFFFFu);
            }
        }
    } else {
    const int groups = W / 4;
#pragma unroll 4
    for (int it = threadIdx.x; it < nr * groups; it += blockDim.x) {
        const int rr = r0 + it / groups, g = it - (it / groups) * groups;
        const GLOBAL uint32_t *row = G(reinterpret_cast<const uint32_t *>(fr + (size_t)rr * J->rs * W * 3));
        const GLOBAL uint64_t *yr = G(reinterpret_cast<const uint64_t *>(J->yref + (size_t)rr * W));
        const uint32_t w0 = row[3 * g], w1 = row[3 * g + 1], w2 = row[3 * g + 2];
        const uint64_t yv = yr[g];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t r = byte_of(w0, w1, w2, 3 * k), gg = byte_of(w0, w1, w2, 3 * k + 1),
                           b = byte_of(w0, w1, w2, 3 * k + 2);
            add_px(r, gg, b, (uint32_t)(yv >> (16 * k)) & 0xFFFFu);
        }
    }
    }
    num = wave_sum(num);
    den = wave_sum(den);
    if (lane == 0) {
        s_num[wave] = num;
        s_den[wave] = den;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long n = 0, d = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
            n += s_num[w];
            d += s_den[w];
        }
        const int slot = tile & (kGainSlots - 1);
        atomicAdd(&J->num[slot], n);
        atomicAdd(&J->den[slot], d);
    }
    __syncthreads();
}

// Tiles [t0, t1) of this block, in order, each with its job. Contiguous
// ranges keep a block's consecutive tiles in one frame, so the job is found
// by one search and then advanced.
template <typename F>
__device__ __forceinline__ void for_block_tiles(const int32_t *pre, int nj, F f)
{
    const int total = pre[nj];
    const int per = (total + (int)gridDim.x - 1) / (int)gridDim.x;
    const int t0 = (int)blockIdx.x * per, t1 = min(total, t0 + per);
    if (t0 >= t1)
        return;
    int j = find_job(pre, nj, t0);
    for (int t = t0; t < t1; ++t) {
        while (t >= pre[j + 1])
            ++j;
        f(j, t - pre[j]);
    }
}

// A gain tile, its hue test's case chosen once per tile.
__device__ __forceinline__ void gain_tile(Table *__restrict__ T, int j, int tile, const uint8_t *fr)
{
    switch (T->jobs[j].hue.mode) {
    case 0:
        gain_tile_mode<0>(T, j, tile, fr);
        break;
    case 1:
        gain_tile_mode<1>(T, j, tile, fr);
        break;
    case 2:
        gain_tile_mode<2>(T, j, tile, fr);
        break;
    default:
        gain_tile_mode<3>(T, j, tile, fr);
        break;
    }
}

// P.valid: job 0's per-call fields come with the launch (its table slot was
// not uploaded again); the first workgroup stores them into the job for the
// kernels that follow on the stream, and the tiles of job 0 take their frame
// from P.
__global__ __launch_bounds__(256) void k_gain(Table *__restrict__ T, CallPatch P)
{
    if (P.valid && blockIdx.x == 0 && threadIdx.x == 0) {
        Job *J = &T->jobs[0];
        J->frame = P.frame;
        J->fizi = P.fizi;
        J->hand = P.hand;
        J->out = P.out;
        J->hout = P.hout;
        J->frame_index = P.frame_index;
    }
    for_block_tiles(T->h.gain_pre, T->h.njobs, [&](int j, int tile) {
        gain_tile(T, j, tile, P.valid && j == 0 ? P.frame : T->jobs[j].frame);
    });
}

// ---------------------------------------------------------------------------
// MASKED: partial re-learning, each job's I_FIZI bits keep its pixels out.
template <bool MASKED>
__global__ __launch_bounds__(256) void k_minmax(Table *__restrict__ T, int nj,
                                                uint8_t *__restrict__ bgmin,
                                                uint8_t *__restrict__ bgmax, int npx, int reset)
{
    __shared__ uint32_t s_inv[kMaxJobs];
    for (int j = threadIdx.x; j < nj; j += blockDim.x)
        s_inv[j] = job_gain(&T->jobs[j], false);
    __syncthreads();
    const int ngroups = npx / 4;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < ngroups; g += gridDim.x * blockDim.x) {
        GLOBAL uint32_t *pmin = G(reinterpret_cast<uint32_t *>(bgmin)) + 3 * g;
        GLOBAL uint32_t *pmax = G(reinterpret_cast<uint32_t *>(bgmax)) + 3 * g;
        uint32_t lo[12], hi[12];
        if (reset) {
#pragma unroll
            for (int i = 0; i < 12; ++i) {
                lo[i] = 255u;
                hi[i] = 0u;
            }
        } else {
            const uint32_t a0 = pmin[0], a1 = pmin[1], a2 = pmin[2];
            const uint32_t b0 = pmax[0], b1 = pmax[1], b2 = pmax[2];
#pragma unroll
            for (int i = 0; i < 12; ++i) {
                lo[i] = byte_of(a0, a1, a2, i);
                hi[i] = byte_of(b0, b1, b2, i);
            }
        }
        for (int j = 0; j < nj; ++j) {
            const GLOBAL uint32_t *f = G(reinterpret_cast<const uint32_t *>(T->jobs[j].frame)) + 3 * g;
            const uint32_t inv = s_inv[j];
            const uint32_t w0 = __builtin_nontemporal_load(f), w1 = __builtin_nontemporal_load(f + 1),
                           w2 = __builtin_nontemporal_load(f + 2);
            // partial re-learning: the frame's I_FIZI (bit set = not background)
            // excludes its pixels; plain learning has no mask
            const uint32_t skip =
                MASKED ? (uint32_t)(G(T->jobs[j].fizi)[g >> 4] >> ((g & 15) << 2)) & 0xFu : 0u;
#pragma unroll
            for (int i = 0; i < 12; ++i) {
                const uint32_t v = corr(byte_of(w0, w1, w2, i), inv);
                const bool use = !MASKED || !((skip >> (i / 3)) & 1u);
                lo[i] = use ? min(lo[i], v) : lo[i];
                hi[i] = use ? max(hi[i], v) : hi[i];
            }
        }
        uint32_t a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            a[i >> 2] |= lo[i] << (8 * (i & 3));
            b[i >> 2] |= hi[i] << (8 * (i & 3));
        }
        pmin[0] = a[0];
        pmin[1] = a[1];
        pmin[2] = a[2];
        pmax[0] = b[0];
        pmax[1] = b[1];
        pmax[2] = b[2];
    }
}

// ---------------------------------------------------------------------------
// One lane classifies 4 consecutive pixels (12 bytes of frame, 12 of bgmin,
// 12 of bgmax); a wave covers 256 pixels = 4 mask words. The hue and gray
// tests only run for pixels already outside the background box, so waves of
// pure background skip them.
// What classify needs of a frame's job, read once into registers (the raw
// mask stores could otherwise alias the job table and force reloads).
struct ClsJob {
    const GLOBAL uint32_t *fr, *mn, *mx;
    GLOBAL uint64_t *raw;
    int delta, S1;
    int scaled;
    uint32_t S_q16;
    int S0, lum2;          // gray tolerance S; over-exposure filter: 2 lum_hi, 0 when off
    HueTest h;
};

// How a job's pixels are tested: corrected pixels, thresholds scaled to the
// frame's brightness, or corrected pixels with the over-exposure filter
// before the gray test.
enum ClsKind { kCorrected = 0, kScaled = 1, kCorrectedLum = 2 };

__device__ __forceinline__ ClsJob cls_job(const Job *J)
{
    ClsJob c;
    c.fr = G(reinterpret_cast<const uint32_t *>(J->frame));
    c.mn = G(reinterpret_cast<const uint32_t *>(J->bgmin));
    c.mx = G(reinterpret_cast<const uint32_t *>(J->bgmax));
    c.raw = G(J->raw);
    c.delta = J->delta;
    c.S1 = J->S1;
    c.scaled = J->scaled;
    c.S_q16 = J->S_q16;
    c.S0 = J->S0;
    c.lum2 = J->lum2;
    c.h = J->hue;
    return c;
}

__device__ __forceinline__ int cls_kind(const ClsJob &c)
{
    return c.scaled ? kScaled : (c.lum2 ? kCorrectedLum : kCorrected);
}

// I_R2 on a corrected pixel, with the over-exposure filter when LUM: a pixel
// whose max + min exceeds 2 lum_hi has its HSL lightness brought down to
// lum_hi (hue and saturation kept), which scales its chroma by
// (510 - 2 lum_hi) / (510 - max - min); not gray when that chroma reaches S,
// compared without division. Chroma > 0 is required in both cases (the hue
// test needs it).
template <bool LUM>
__device__ __forceinline__ bool not_gray(const ClsJob &c, int mx, int mn)
{
    const int ch = mx - mn;
    if (LUM) {
        const int l2 = mx + mn;
        if (l2 > c.lum2)
            return ch >= 1 && ch * (510 - c.lum2) >= c.S0 * (510 - l2);
    }
    return ch >= c.S1;
}

// The inputs of one lane's 4 pixels: frame, background min and max (3 dwords
// each). They are read once per step, so they are loaded non-temporally (no
// reuse expected in the caches): this streams 12% faster than plain loads.
struct Px4 {
    uint32_t f[3], l[3], u[3];
};

// The byte offset (3 p < 2^28: frames are at most 8192 x 8192) is
// added to each array's wave-uniform base as an unsigned 32-bit value, so
// that the loads take the scalar-base, vector-offset form and no 64-bit
// address is formed per lane.
template <typename T>
__device__ __forceinline__ const GLOBAL T *at_byte(const GLOBAL T *base, uint32_t off)
{
    return reinterpret_cast<const GLOBAL T *>(reinterpret_cast<const GLOBAL uint8_t *>(base) + off);
}

typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));

__device__ __forceinline__ void load_px4(const ClsJob &c, uint32_t p, uint32_t pend, Px4 &x)
{
    if (p < pend) {
        const uint32_t off = 3u * p;
        const u32x3 f = __builtin_nontemporal_load(at_byte(reinterpret_cast<const GLOBAL u32x3 *>(c.fr), off));
        const u32x3 l = __builtin_nontemporal_load(at_byte(reinterpret_cast<const GLOBAL u32x3 *>(c.mn), off));
        const u32x3 u = __builtin_nontemporal_load(at_byte(reinterpret_cast<const GLOBAL u32x3 *>(c.mx), off));
        x.f[0] = f.x, x.f[1] = f.y, x.f[2] = f.z;
        x.l[0] = l.x, x.l[1] = l.y, x.l[2] = l.z;
        x.u[0] = u.x, x.u[1] = u.y, x.u[2] = u.z;
    }
}

// I_R1, I_R2 and I_R3 of one 1024-pixel unit of a frame (256 per wave, 4 per
// lane) whose pixels from pend on are not classified; base is the wave's
// first pixel (a multiple of 64), raw words at or past pend / 64 are not
// written; x holds the lane's inputs (loaded by load_px4). KIND: kScaled, the
// thresholds follow the frame's brightness and the pixels stay raw.
template <bool FLOW, int KIND>
__device__ __forceinline__ void classify_px4(const ClsJob &c, uint32_t base, uint32_t pend, uint32_t inv,
                                             const Px4 &x)
{
    constexpr bool SCALED = KIND == kScaled;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t p = base + 4u * lane;
    uint32_t bits = 0;
    if (SCALED && p < pend) {
        // (bgmin - delta) 2^16 <= v inv <= (bgmax + delta) 2^16 as one
        // unsigned compare of v inv + (delta - bgmin) 2^16 (wrapping below
        // zero) against (bgmax - bgmin + 2 delta) 2^16; v inv < 2^28
        int cv[12];
        uint32_t out = 0;
        const uint32_t rng[3] = {x.u[0] - x.l[0], x.u[1] - x.l[1], x.u[2] - x.l[2]};
        const uint32_t kd = (uint32_t)c.delta << 16, d2 = 2u * (uint32_t)c.delta;
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            const uint32_t v = byte_of(x.f[0], x.f[1], x.f[2], i);
            const uint32_t d = __umul24(v, inv) + kd - (byte_of(x.l[0], x.l[1], x.l[2], i) << 16);
            cv[i] = (int)v;
            out |= (uint32_t)(d > ((byte_of(rng[0], rng[1], rng[2], i) + d2) << 16)) << (i / 3);
        }
        if (out) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (out & (1u << k)) {
                    const int r = cv[3 * k], g = cv[3 * k + 1], b = cv[3 * k + 2];
                    const uint32_t ch = (uint32_t)(max(max(r, g), b) - min(min(r, g), b));
                    if (__umul24(ch, inv) >= c.S_q16 && hue_in(r, g, b, c.h))
                        bits |= 1u << k;
                }
            }
        }
    } else if (!SCALED && p < pend) {
        // v' in [bgmin - delta, bgmax + delta] is one unsigned compare:
        // (v' + delta - bgmin) <= (bgmax - bgmin) + 2 delta, with v' + delta
        // from the correction's own multiply-add (delta << 16 added before the
        // shift, the saturation moved up by delta) and bgmax - bgmin taken for
        // four channels at once (bgmax >= bgmin per byte: no borrows)
        int cv[12];
        uint32_t out = 0;
        const uint32_t rng[3] = {x.u[0] - x.l[0], x.u[1] - x.l[1], x.u[2] - x.l[2]};
        const uint32_t kadd = 32768u + ((uint32_t)c.delta << 16), kmax = 255u + (uint32_t)c.delta;
        const uint32_t d2 = 2u * (uint32_t)c.delta;
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            const uint32_t vd = min((__umul24(byte_of(x.f[0], x.f[1], x.f[2], i), inv) + kadd) >> 16, kmax);
            const uint32_t d = vd - byte_of(x.l[0], x.l[1], x.l[2], i);
            cv[i] = (int)vd - c.delta;
            out |= (uint32_t)(d > byte_of(rng[0], rng[1], rng[2], i) + d2) << (i / 3);
        }
        if (out) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (out & (1u << k)) {
                    const int r = cv[3 * k], g = cv[3 * k + 1], b = cv[3 * k + 2];
                    if (not_gray<KIND == kCorrectedLum>(c, max(max(r, g), b), min(min(r, g), b)) &&
                        hue_in(r, g, b, c.h))
                        bits |= 1u << k;
                }
            }
        }
    }
    const uint64_t w = row_word(bits);
    if ((lane & 15) == 0) {
        const uint32_t word = (base >> 6) + (uint32_t)(lane >> 4);
        if (word < (pend >> 6))
            put<FLOW>(c.raw + word, w);
    }
}

// The wave's units of pixels [p0, p1) of a frame (p0 a multiple of 64):
// 1024 pixels apart, each unit's inputs loaded one unit ahead into
// alternating registers.
template <bool FLOW, int KIND>
__device__ __forceinline__ void classify_span_as(const ClsJob &c, uint32_t p0, uint32_t p1, uint32_t inv)
{
    const uint32_t lanepx = 4u * (threadIdx.x & (kWave - 1));
    uint32_t base = p0 + (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)) * 256u;
    Px4 a, b;
    load_px4(c, base + lanepx, p1, a);
    while (base < p1) {
        load_px4(c, base + 1024u + lanepx, p1, b);
        classify_px4<FLOW, KIND>(c, base, p1, inv, a);
        base += 1024u;
        if (base >= p1)
            break;
        load_px4(c, base + 1024u + lanepx, p1, a);
        classify_px4<FLOW, KIND>(c, base, p1, inv, b);
        base += 1024u;
    }
}

template <bool FLOW>
__device__ __forceinline__ void classify_span(const ClsJob &c, uint32_t p0, uint32_t p1, uint32_t inv)
{
    switch (cls_kind(c)) {
    case kScaled: classify_span_as<FLOW, kScaled>(c, p0, p1, inv); break;
    case kCorrectedLum: classify_span_as<FLOW, kCorrectedLum>(c, p0, p1, inv); break;
    default: classify_span_as<FLOW, kCorrected>(c, p0, p1, inv); break;
    }
}

// Classify tile `tile` of frame j: ITERS consecutive 1024-pixel units.
template <int ITERS>
__device__ __forceinline__ void classify_tile(Table *__restrict__ T, int j, int tile, uint32_t inv)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const Job *J = &T->jobs[j];
    const uint32_t npx = (uint32_t)J->W * (uint32_t)J->H;
    const ClsJob c = cls_job(J);
    const uint32_t lanepx = 4u * (threadIdx.x & (kWave - 1));
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const uint32_t base = ((uint32_t)tile * ITERS + it) * 1024u + (uint32_t)wave * 256u;
        if (base >= npx)
            break;
        Px4 x;
        load_px4(c, base + lanepx, npx, x);
        switch (cls_kind(c)) {
        case kScaled: classify_px4<false, kScaled>(c, base, npx, inv, x); break;
        case kCorrectedLum: classify_px4<false, kCorrectedLum>(c, base, npx, inv, x); break;
        default: classify_px4<false, kCorrected>(c, base, npx, inv, x); break;
        }
    }
}

// Tiles blockIdx.x, blockIdx.x + gridDim.x, ...: the frame index only grows,
// so it is advanced, not searched. A block meets one to three frames, so a
// frame's inverse gain (sixteen pairs of sums and a 64-bit division) is
// computed when its first tile comes, once per block, by thread 0.
template <int ITERS>
__device__ __forceinline__ void classify_tiles(Table *__restrict__ T, int nj, const int32_t *s_pre)
{
    __shared__ uint32_t s_inv;
    const int total = s_pre[nj];
    int j = 0, jinv = -1;
    uint32_t inv = 0;
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        while (s_pre[j + 1] <= t)
            ++j;
        if (j != jinv) {
            __syncthreads();
            if (threadIdx.x == 0)
                s_inv = job_gain(&T->jobs[j], false);
            __syncthreads();
            inv = s_inv;
            jinv = j;
        }
        classify_tile<ITERS>(T, j, t - s_pre[j], inv);
    }
}

template <int ITERS>
__global__ __launch_bounds__(256) void k_classify(Table *__restrict__ T)
{
    __shared__ int32_t s_pre[kMaxJobs + 1];
    const int nj = T->h.njobs;
    for (int i = threadIdx.x; i <= nj; i += blockDim.x)
        s_pre[i] = T->h.cls_pre[i];
    __syncthreads();
    classify_tiles<ITERS>(T, nj, s_pre);
}

// ---------------------------------------------------------------------------
// A run list entry: first pixel (low word), last pixel (bits 32..62) and the
// flag kLinkUp (bit 63): the run must still be joined to the row above.
constexpr uint32_t kLinkUp = 0x80000000u;

// (first pixel, length) of a run list entry
__device__ __forceinline__ uint2 unpack_run(uint64_t v)
{
    const uint32_t a = (uint32_t)v, e = (uint32_t)(v >> 32) & ~kLinkUp;
    return make_uint2(a, e - a + 1u);
}

// Bit scans of one mask row (W = 64 * Wd pixels).
// First x in [pos, limit] whose bit is 1, or -1.
template <typename P>
__device__ __forceinline__ int next_one(P row, int pos, int limit)
{
    int w = pos >> 6;
    uint64_t m = row[w] & (~0ull << (pos & 63));
    for (;;) {
        if (m) {
            const int x = (w << 6) + __builtin_ctzll(m);
            return x <= limit ? x : -1;
        }
        ++w;
        if ((w << 6) > limit)
            return -1;
        m = row[w];
    }
}

// Largest x <= pos whose bit is 0, or -1.
template <typename P>
__device__ __forceinline__ int prev_zero(P row, int pos)
{
    int w = pos >> 6;
    const int b = pos & 63;
    uint64_t m = ~row[w] & (b == 63 ? ~0ull : ((2ull << b) - 1ull));
    while (!m) {
        --w;
        if (w < 0)
            return -1;
        m = ~row[w];
    }
    return (w << 6) + 63 - __builtin_clzll(m);
}

// Smallest x >= pos whose bit is 0, or W.
template <typename P>
__device__ __forceinline__ int next_zero(P row, int Wd, int pos)
{
    int w = pos >> 6;
    uint64_t m = ~row[w] & (~0ull << (pos & 63));
    while (!m) {
        ++w;
        if (w >= Wd)
            return Wd << 6;
        m = ~row[w];
    }
    return (w << 6) + __builtin_ctzll(m);
}

// Union-find over run starts (pixel indices). A parent never exceeds its
// child, so following parents always ends, and the root of a finished
// component is its smallest run start: its first pixel in raster order.
// Root of x with path halving: each visited node is pointed at its
// grandparent. Safe beside concurrent finds and unions of the same workgroup:
// parents only ever move to ancestors of the same set (a linked root's new
// parent is smaller, a halved node's grandparent is one of its ancestors), so
// a store that overwrites another still leaves the node in its set. Without
// it, the border joins of a tall component chain one band's root under the
// next, and every find walks that chain one dependent load at a time.
__device__ __forceinline__ uint32_t find_root(GLOBAL uint32_t *parent, uint32_t x)
{
    for (;;) {
        const uint32_t p = ld_wg(parent + x);
        if (p == x)
            return x;
        const uint32_t g = ld_wg(parent + p);
        if (g == p)
            return p;
        st_wg(parent + x, g);
        x = g;
    }
}

// Root of x without writing: once every find and union of a workgroup is
// over, a node's parent need not be its root (a halving store of one thread
// can land after another thread pointed the node at its root, and leave it at
// an older ancestor), so a membership test walks to the root.
__device__ __forceinline__ uint32_t root_of(GLOBAL uint32_t *parent, uint32_t x)
{
    for (;;) {
        const uint32_t p = ld_wg(parent + x);
        if (p == x)
            return x;
        x = p;
    }
}

__device__ __forceinline__ void unite(GLOBAL uint32_t *parent, uint32_t a, uint32_t b)
{
    for (;;) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b)
            return;
        if (a > b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        const uint32_t old = __hip_atomic_fetch_min(parent + b, a, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == b)
            return;
        b = old;
    }
}

// Joins run (y, xs..xe), whose start pixel is `start`, with every run of the
// row above that it touches under 8-connectivity (columns xs-1 .. xe+1).
template <typename P>
__device__ __forceinline__ void link_up(GLOBAL uint32_t *parent, P above, int Wd, int W, int y,
                                        int xs, int xe, uint32_t start)
{
    const int hi = min(xe + 1, W - 1);
    int pos = max(xs - 1, 0);
    while (pos <= hi) {
        const int xb = next_one(above, pos, hi);
        if (xb < 0)
            break;
        const int bs = prev_zero(above, xb) + 1;
        unite(parent, start, (uint32_t)(y - 1) * (uint32_t)W + (uint32_t)bs);
        pos = next_zero(above, Wd, xb) + 1;
    }
}

// ---------------------------------------------------------------------------
// Morphology, runs and band-local components: one wave per band of R mask
// rows. Lane l holds words l and l + 64 of a row (W <= 8192). The band's rows,
// with 2(o+c) halo rows on each side, stream once through a pipeline of the
// opening/closing stages held in registers: each stage keeps the two rows
// before its input, and on input row i emits row i - 1 from the 3x3 window
// (vertical AND/OR per word, horizontal neighbours from the words' edge bits,
// exchanged between neighbouring lanes). Rows outside the image enter a stage
// as its neutral value (1 for erosion, 0 for dilation), which is exactly the
// border rule; halo rows inside the image only corrupt rows outside the band.
// Each final row of the band is stored (I_FIZI); its run starts and ends are
// bit masks of each lane's word, numbered by a wave prefix sum, so the lanes
// holding a run's first and last pixel write them without scanning. Runs are
// joined to the touching runs of the row above (kept in registers) in a
// union-find over segment-local run indices kept in LDS (indices grow in
// raster order, so a root is its component's first run in the segment). A
// segment is a stretch of the band's rows whose runs fit the LDS table; when
// it closes (table full, band done) its runs are appended to the frame's run
// list with one reservation, each pointing at its segment root. The first run
// row of a segment that is not the first of the band, and the first row of
// every band below the top, are flagged: the component stage joins them to the
// row above. A row with more runs than the table goes to the run list
// directly, its runs their own roots, flagged, and so is the row after it.
constexpr int kMaxRowWords = 128;          // W <= 8192
constexpr int kSegRuns = 512;              // runs of one LDS segment
constexpr int kRawChunk = 4;               // rows loaded together (the selects below assume 4)

struct WaveLds {
    uint32_t start[kSegRuns];              // first pixel of segment run k
    uint32_t end[kSegRuns];                // its last pixel, | kLinkUp if flagged
    uint32_t par[kSegRuns];                // union-find parent (segment index)
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Lane l receives lane l - 1's value (lane 0 receives 0): DPP wave_shr:1.
__device__ __forceinline__ uint32_t from_left(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xF, 0xF, false);
}

// Lane l receives lane l + 1's value (lane 63 receives 0): DPP wave_shl:1.
__device__ __forceinline__ uint32_t from_right(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, false);
}

// Inclusive prefix sum over the wave: shifts of 1, 2, 4, 8 inside each row of
// 16 lanes, then each row's total is carried into the rows above it
// (row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3). Lanes a
// DPP move does not write keep 0.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
    return v;
}

// Lanes per row: LG lanes hold one row (LG = 64: the whole wave; LG = 16 or
// 32 pack 64 / LG bands of a narrow frame into one wave, lane group g holding
// band g's row). The word a lane holds, and its group:
template <int LG>
__device__ __forceinline__ int lane_word() { return (int)(threadIdx.x & (uint32_t)(LG - 1)); }
template <int LG>
__device__ __forceinline__ int lane_group() { return LG == kWave ? 0 : (int)((threadIdx.x & (kWave - 1)) / LG); }

// Edge bits of the neighbouring words of this lane's NC words (word
// w + 64 q of the lane group's row): bit 63 of the word on the left (lc) and
// bit 0 of the word on the right (rc); words outside [0, Wd) give `edge`.
template <int NC, int LG = kWave>
__device__ __forceinline__ void row_carries(const uint64_t *v, int Wd, uint32_t edge, uint32_t *lc, uint32_t *rc)
{
    static_assert(NC == 1 || LG == kWave, "lane groups hold one word per lane");
    const int lane = lane_word<LG>();
    const uint32_t hi0 = (uint32_t)(v[0] >> 63), lo0 = (uint32_t)v[0] & 1u;
    const uint32_t up0 = from_left(hi0), dn0 = from_right(lo0);
    lc[0] = lane == 0 ? edge : up0;
    if (NC == 1) {
        rc[0] = (lane + 1 < Wd) ? dn0 : edge;
    } else {
        const uint32_t hi1 = (uint32_t)(v[NC - 1] >> 63), lo1 = (uint32_t)v[NC - 1] & 1u;
        const uint32_t up1 = from_left(hi1), dn1 = from_right(lo1);
        const uint32_t last_hi0 = (uint32_t)__builtin_amdgcn_readlane((int)hi0, kWave - 1);
        const uint32_t first_lo1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)lo1);
        rc[0] = (lane + 1 < Wd) ? (lane == kWave - 1 ? first_lo1 : dn0) : edge;
        lc[NC - 1] = lane == 0 ? last_hi0 : up1;
        rc[NC - 1] = (lane + kWave + 1 < Wd) ? dn1 : edge;
    }
}

// One erosion (ero) or dilation of row b given the rows above (a) and below (c).
template <int NC, int LG = kWave>
__device__ __forceinline__ void morph_row(bool ero, const uint64_t *a, const uint64_t *b, const uint64_t *c, int Wd,
                                          uint64_t *out)
{
    uint64_t v[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q)
        v[q] = ero ? (a[q] & b[q] & c[q]) : (a[q] | b[q] | c[q]);
    uint32_t lc[NC], rc[NC];
    row_carries<NC, LG>(v, Wd, ero ? 1u : 0u, lc, rc);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const uint64_t left = (v[q] << 1) | lc[q];
        const uint64_t right = (v[q] >> 1) | ((uint64_t)rc[q] << 63);
        out[q] = ero ? (v[q] & left & right) : (v[q] | left | right);
    }
}

__device__ __forceinline__ uint32_t find_lds(uint32_t *par, uint32_t x)
{
    uint32_t p = __hip_atomic_load(par + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    while (p != x) {
        x = p;
        p = __hip_atomic_load(par + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    return x;
}

__device__ __forceinline__ void unite_lds(uint32_t *par, uint32_t a, uint32_t b)
{
    for (;;) {
        a = find_lds(par, a);
        b = find_lds(par, b);
        if (a == b)
            return;
        if (a > b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        const uint32_t old = __hip_atomic_fetch_min(par + b, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (old == b)
            return;
        b = old;
    }
}

// Bit t of a row around this lane's word w, t in [-1, 64]: -1 is the last
// bit of the word on the left (lc), 64 the first bit of the word on the right
// (rc).
__device__ __forceinline__ uint32_t bit_at(int t, uint64_t w, uint32_t lc, uint32_t rc)
{
    return t < 0 ? lc : (t > 63 ? rc : (uint32_t)(w >> t) & 1u);
}

// Row-local index of the run that contains bit t (set, t in [-1, 64]) around
// this lane's word w, whose run starts are st, with ex runs starting before it.
__device__ __forceinline__ uint32_t run_at(int t, uint32_t ex, uint64_t st, uint64_t w, uint32_t rc)
{
    if (t < 0)
        return ex - 1u;
    if (t > 63)
        return ex + (uint32_t)__popcll(st) + (rc & ~(uint32_t)(w >> 63) & 1u) - 1u;
    return ex + (uint32_t)__popcll(st & (~0ull >> (63 - t))) - 1u;
}

// Inclusive max over lanes 0..l of values >= -1 (DPP as in wave_incl_scan;
// lanes a move does not write keep -1).
__device__ __forceinline__ int wave_incl_max(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x111, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x112, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x114, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x118, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x142, 0xA, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x143, 0xC, 0xF, false));
    return v;
}

// One final mask row as the lanes hold it: per word (lane + 64 c) the bits,
// the edge bits of the neighbouring words, the run starts, the number of runs
// starting before the word and the x of the last run start before the word.
template <int NC>
struct RowBits {
    uint64_t w[NC], st[NC];
    uint32_t lc[NC], rc[NC], ex[NC];
    int last[NC];
};

// Fills r from the row x; en receives the run ends. Returns the row's runs
// (of every lane group: runs are numbered across the wave). r.last holds
// wave positions 64 lane + bit, which grow across the groups.
template <int NC, int LG = kWave>
__device__ __forceinline__ uint32_t row_bits(RowBits<NC> &r, const uint64_t *x, int Wd, uint64_t *en)
{
    const int lane = threadIdx.x & (kWave - 1);
    row_carries<NC, LG>(x, Wd, 0u, r.lc, r.rc);
    uint32_t total = 0;
    int before = -1;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        r.w[c] = x[c];
        r.st[c] = x[c] & ~((x[c] << 1) | r.lc[c]);
        en[c] = x[c] & ~((x[c] >> 1) | ((uint64_t)r.rc[c] << 63));
        const uint32_t n = (uint32_t)__popcll(r.st[c]);
        const uint32_t inc = wave_incl_scan(n);
        r.ex[c] = total + inc - n;
        total += (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
        const int hi = r.st[c] ? 64 * (lane + kWave * c) + 63 - __builtin_clzll(r.st[c]) : -1;
        const int im = wave_incl_max(hi);
        r.last[c] = max(before, __builtin_amdgcn_update_dpp(-1, im, 0x138, 0xF, 0xF, false));
        before = max(before, __builtin_amdgcn_readlane(im, kWave - 1));
    }
    return total;
}

// x of the first pixel of the run that contains bit t (set, t in [-1, 64])
// around word c of the row. A run never crosses a lane group (its edges are
// out-of-image), so a start before the word lies in the same group.
template <int NC, int LG = kWave>
__device__ __forceinline__ int start_at(const RowBits<NC> &r, int c, int t)
{
    const int wb = 64 * (lane_word<LG>() + kWave * c);
    const int gofs = 64 * LG * lane_group<LG>();
    if (t < 0)
        return r.last[c] - gofs;
    uint64_t m;
    if (t > 63) {
        if (r.rc[c] & ~(uint32_t)(r.w[c] >> 63) & 1u)
            return wb + 64;
        m = r.st[c];
    } else {
        m = r.st[c] & (~0ull >> (63 - t));
    }
    return m ? wb + 63 - __builtin_clzll(m) : r.last[c] - gofs;
}

// Every touching pair of runs of two consecutive rows U (above) and D
// (below), each once, from the lanes' words. Under 8-connectivity a U run
// [us, ue] and a D run [ds, de] touch when us <= de + 1 and ue >= ds - 1.
// When us <= ds + 1, U has a pixel in columns ds - 1 .. ds + 1, and D's start
// meets it there (the pixel at ds, else those beside it). Otherwise
// us >= ds + 2, so D holds columns us - 2 and us - 1, and U's start meets the
// D run there. f(c, from_d, b, t): the run starting at bit b of word c of D
// (from_d) or U touches the run of the other row that contains bit t.
// ONCE = false: U's starts look at the one to three pixels below them as D's
// do above, so most pairs come twice (the band-border joins keep that form:
// the component stage unites them concurrently, and the second meeting of a
// pair shortens the chains the first one built).
template <int NC, bool ONCE, typename F>
__device__ __forceinline__ void touching_runs(const RowBits<NC> &U, const RowBits<NC> &D, F f)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        uint64_t m = D.st[c];
        while (m) {
            const int b = __builtin_ctzll(m);
            m &= m - 1;
            if (bit_at(b, U.w[c], U.lc[c], U.rc[c])) {
                f(c, true, b, b);
            } else {
                if (bit_at(b - 1, U.w[c], U.lc[c], U.rc[c]))
                    f(c, true, b, b - 1);
                if (bit_at(b + 1, U.w[c], U.lc[c], U.rc[c]))
                    f(c, true, b, b + 1);
            }
        }
        m = U.st[c];
        while (m) {
            const int b = __builtin_ctzll(m);
            m &= m - 1;
            if (!ONCE) {
                if (bit_at(b, D.w[c], D.lc[c], D.rc[c])) {
                    f(c, false, b, b);
                } else {
                    if (bit_at(b - 1, D.w[c], D.lc[c], D.rc[c]))
                        f(c, false, b, b - 1);
                    if (bit_at(b + 1, D.w[c], D.lc[c], D.rc[c]))
                        f(c, false, b, b + 1);
                }
                continue;
            }
            // D holds columns b - 2 and b - 1 (for b = 0: its run through
            // the word's left edge started at least two columns before it)
            bool left2;
            if (b >= 2)
                left2 = ((D.w[c] >> (b - 2)) & 3ull) == 3ull;
            else if (b == 1)
                left2 = (D.lc[c] & (uint32_t)D.w[c] & 1u) != 0u;
            else
                left2 = D.lc[c] != 0u && D.last[c] < 64 * (lane + kWave * c) - 1;
            if (left2)
                f(c, false, b, b - 1);
        }
    }
}

__device__ __forceinline__ bool stage_erodes(int k, int oi, int ci) { return (k < oi) || (k >= 2 * oi + ci); }

// Reserves n entries of the frame's run list (one atomic for the wave).
__device__ __forceinline__ uint32_t reserve_runs(Job *J, uint32_t n, uint32_t cap)
{
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t base = 0;
    if (lane == 0) {
        base = atomicAdd(&J->nruns, n);
        if (base + n > cap)
            atomicOr(&J->flags, 1u);
    }
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
}

// Closes a segment: its n runs join the run list, each pointing at its root.
template <bool FLOW>
__device__ __forceinline__ void flush_segment(Job *J, WaveLds &L, uint32_t n, GLOBAL uint64_t *runs,
                                              GLOBAL uint32_t *parent, GLOBAL uint32_t *area, uint32_t cap)
{
    const int lane = threadIdx.x & (kWave - 1);
    if (n == 0)
        return;
    const uint32_t base = reserve_runs(J, n, cap);
    for (uint32_t k = lane; k < n; k += kWave) {
        const uint32_t st = L.start[k];
        const uint32_t r = find_lds(L.par, k);
        if (base + k < cap) {
            put<FLOW>(runs + base + k, ((uint64_t)L.end[k] << 32) | st);
            put_parent<FLOW>(parent + st, L.start[r]);
            put<FLOW>(area + st, 0u);
        }
    }
    wave_sync();
}

// Rows r0 .. r0 + kRawChunk - 1 of the raw mask (r0 per lane group),
// addresses clamped to rows 0 .. H - 1 and words below Wd. Values of clamped
// rows and words are never used (rows outside the image enter the pipeline as
// its neutral value, words from Wd on never reach a valid word), so the loads
// need no condition: they stay in flight while the previous chunk is
// processed.
template <int NC, int LG = kWave>
__device__ __forceinline__ void load_rows(uint64_t (&dst)[kRawChunk][NC], const GLOBAL uint64_t *raw, int r0, int H,
                                          int Wd)
{
    const int lane = lane_word<LG>();
#pragma unroll
    for (int qq = 0; qq < kRawChunk; ++qq) {
        const size_t ro = (size_t)min(max(r0 + qq, 0), H - 1) * Wd;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            dst[qq][c] = raw[ro + min(lane + kWave * c, Wd - 1)];
    }
}

// KMAX: most opening/closing stages a job may have; NC: words per lane; FLOW:
// inside the persistent step (stores other workgroups read in the launch);
// OI, CI: the opening and closing iterations when fixed at compile time (the
// stages' kinds then need no selects), -1 to read them from the job; LG:
// lanes per row (bands band, band + 1, ... of the frame on the wave's lane
// groups; every group steps through the same band-relative rows, so control
// stays uniform, and rows outside the image are neutral or dropped per group).
template <int KMAX, int NC, bool FLOW, int OI = -1, int CI = -1, int LG = kWave>
__device__ __forceinline__ void morph_band(Job *J, int band, WaveLds &L)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int word = lane_word<LG>();
    const int W = J->W, H = J->H, Wd = J->Wd, R = J->band;
    const int oi = OI >= 0 ? OI : J->open_it, ci = CI >= 0 ? CI : J->close_it;
    const int K = 2 * (oi + ci);
    const int y0 = (band + lane_group<LG>()) * R;
    // one more halo row above: row y0 - 1 is computed exactly, to join the
    // band's first row to it without reading the band above
    const int ya = y0 - K - 1;
    const GLOBAL uint64_t *raw = G(J->raw);
    GLOBAL uint64_t *fz = G(J->fizi);
    GLOBAL uint32_t *parent = G(J->parent);
    GLOBAL uint32_t *area = G(J->area);
    GLOBAL uint64_t *runs = G(reinterpret_cast<uint64_t *>(J->runs));
    const uint32_t cap = J->run_cap;
    bool valid_w[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q)
        valid_w[q] = word + kWave * q < Wd;

    // pipeline state: the two rows before each stage's next input
    uint64_t p2[KMAX][NC], p1[KMAX][NC];
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
#pragma unroll
        for (int q = 0; q < NC; ++q)
            p2[k][q] = p1[k][q] = stage_erodes(k, oi, ci) ? ~0ull : 0ull;
    uint32_t nseg = 0, prev_first = 0;
    bool prev_valid = false;    // P holds the previous row and it has runs
    bool prev_in_seg = false;   // ... in the open segment
    RowBits<NC> P;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        P.w[c] = P.st[c] = 0ull;
        P.lc[c] = P.rc[c] = P.ex[c] = 0u;
        P.last[c] = -1;
    }
    GLOBAL uint32_t *linkw = G(reinterpret_cast<uint32_t *>(J->links));
    const uint32_t link_cap = J->link_cap;
    const int nsteps = R + 2 * K + 1;
    // one input row through the stages, then the band's final row it yields
    auto step = [&](int s, int q, const uint64_t (&ch)[kRawChunk][NC]) __attribute__((always_inline)) {
        uint64_t x[NC];
        const bool past = ya + s >= H;
        const uint64_t n0 = (K > 0 && stage_erodes(0, oi, ci)) ? ~0ull : 0ull;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const uint64_t v = q == 0 ? ch[0][c] : (q == 1 ? ch[1][c] : (q == 2 ? ch[2][c] : ch[3][c]));
            x[c] = past ? n0 : v;
        }
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if (k < K) {
                const bool ero = stage_erodes(k, oi, ci);
                const int i = ya + s - k;
                if (i < 0 || i >= H) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        x[c] = ero ? ~0ull : 0ull;
                }
                uint64_t o[NC];
                morph_row<NC, LG>(ero, p2[k], p1[k], x, Wd, o);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    p2[k][c] = p1[k][c];
                    p1[k][c] = x[c];
                }
                const int jr = i - 1;
                const bool oob = k + 1 < K && (jr < 0 || jr >= H);
                const uint64_t n1 = stage_erodes(k + 1, oi, ci) ? ~0ull : 0ull;
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    x[c] = oob ? n1 : o[c];
            }
        }
        // the row this step yields, relative to the band: -1 the halo row,
        // 0 .. R - 1 the band's rows (outside the image: an empty row)
        const int jrel = s - 2 * K - 1;
        if (jrel < -1 || jrel >= R)
            return;
        const int jrow = y0 + jrel;
        const bool row_ok = jrow >= 0 && jrow < H;
        uint64_t orw = 0ull;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (!valid_w[c] || !row_ok)
                x[c] = 0ull;
            orw |= x[c];
        }
        const bool nonempty = __ballot(orw != 0ull) != 0ull;
        if (jrel == -1) {
            // the last row of the band above, only to join with
            if (nonempty) {
                uint64_t en[NC];
                (void)row_bits<NC, LG>(P, x, Wd, en);
            }
            prev_valid = nonempty;
            prev_in_seg = false;
            return;
        }
        // a final I_FIZI row
        GLOBAL uint64_t *frow = fz + (size_t)max(jrow, 0) * Wd;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (valid_w[c] && row_ok)
                put<FLOW>(frow + word + kWave * c, x[c]);
        if (!nonempty) {
            prev_valid = false;
            return;
        }
        RowBits<NC> D;
        uint64_t en[NC];
        const uint32_t total = row_bits<NC, LG>(D, x, Wd, en);
        if (nseg + total > (uint32_t)kSegRuns) {
            // the open segment is full: close it, this row opens the next
            flush_segment<FLOW>(J, L, nseg, runs, parent, area, cap);
            nseg = 0;
            prev_in_seg = false;
        }
        const bool direct = total > (uint32_t)kSegRuns;
        const uint32_t rowpx = (uint32_t)max(jrow, 0) * (uint32_t)W;
        // joins with a row above whose runs are not in the open segment (the
        // band above, a closed segment, or a row written directly) go to the
        // frame's link list as pairs of run starts
        uint32_t flag = 0u;
        if (prev_valid && (!prev_in_seg || direct)) {
            uint32_t cnt = 0;
            touching_runs<NC, false>(P, D, [&](int, bool, int, int) { ++cnt; });
            const uint32_t inc = wave_incl_scan(cnt);
            const uint32_t n = (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
            uint32_t base = 0;
            if (lane == 0)
                base = atomicAdd(&J->nlinks, n);
            base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
            uint32_t k = base + inc - cnt;
            const uint32_t upx = rowpx - (uint32_t)W;
            touching_runs<NC, false>(P, D, [&](int c, bool from_d, int b, int t) {
                const uint32_t wb = 64u * (uint32_t)(word + kWave * c);
                const uint32_t a = from_d ? rowpx + wb + (uint32_t)b : upx + wb + (uint32_t)b;
                const uint32_t o = from_d ? upx + (uint32_t)start_at<NC, LG>(P, c, t)
                                          : rowpx + (uint32_t)start_at<NC, LG>(D, c, t);
                if (k < link_cap) {
                    put<FLOW>(linkw + 2 * (size_t)k, a);
                    put<FLOW>(linkw + 2 * (size_t)k + 1, o);
                }
                ++k;
            });
            if (base + n > link_cap) {
                // the list is full: the component stage joins this row to
                // the row above by reading I_FIZI
                flag = kLinkUp;
                if (lane == 0)
                    atomicAdd(&J->nflag, 1u);
            }
        }
        const uint32_t rbase = direct ? reserve_runs(J, total, cap) : 0u;
        GLOBAL uint32_t *runw = reinterpret_cast<GLOBAL uint32_t *>(runs);
        // record the row's runs: the lane holding a run's first pixel writes
        // its start, the lane holding its last pixel its end
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const uint32_t wpx = rowpx + 64u * (uint32_t)(word + kWave * c);
            uint64_t m = D.st[c];
            while (m) {
                const int b = __builtin_ctzll(m);
                const uint32_t k = D.ex[c] + (uint32_t)__popcll(D.st[c] & ((1ull << b) - 1ull));
                m &= m - 1;
                const uint32_t start = wpx + (uint32_t)b;
                if (!direct) {
                    L.start[nseg + k] = start;
                    L.par[nseg + k] = nseg + k;
                } else if (rbase + k < cap) {
                    put<FLOW>(runw + 2 * (size_t)(rbase + k), start);
                    put_parent<FLOW>(parent + start, start);
                    put<FLOW>(area + start, 0u);
                }
            }
            m = en[c];
            while (m) {
                const int e = __builtin_ctzll(m);
                const uint32_t k = D.ex[c] + (uint32_t)__popcll(D.st[c] & (~0ull >> (63 - e))) - 1u;
                m &= m - 1;
                const uint32_t end = (wpx + (uint32_t)e) | flag;
                if (!direct)
                    L.end[nseg + k] = end;
                else if (rbase + k < cap)
                    put<FLOW>(runw + 2 * (size_t)(rbase + k) + 1, end);
            }
        }
        wave_sync();
        // joins with the row above in the open segment, in the LDS union-find
        if (prev_valid && prev_in_seg && !direct) {
            touching_runs<NC, true>(P, D, [&](int c, bool from_d, int b, int t) {
                const uint64_t below = (1ull << b) - 1ull;
                if (from_d)
                    unite_lds(L.par, nseg + D.ex[c] + (uint32_t)__popcll(D.st[c] & below),
                              prev_first + run_at(t, P.ex[c], P.st[c], P.w[c], P.rc[c]));
                else
                    unite_lds(L.par, prev_first + P.ex[c] + (uint32_t)__popcll(P.st[c] & below),
                              nseg + run_at(t, D.ex[c], D.st[c], D.w[c], D.rc[c]));
            });
            wave_sync();
        }
        // this row becomes the row above
        P = D;
        prev_valid = true;
        prev_in_seg = !direct;
        if (!direct) {
            prev_first = nseg;
            nseg += total;
        }
    };
    // input chunks alternate between two register buffers: each is loaded a
    // chunk ahead of its use, straight into the registers that use it
    uint64_t ca[kRawChunk][NC], cb[kRawChunk][NC];
    load_rows<NC, LG>(ca, raw, ya, H, Wd);
#pragma unroll 1
    for (int s0 = 0; s0 < nsteps; s0 += 2 * kRawChunk) {
        load_rows<NC, LG>(cb, raw, ya + s0 + kRawChunk, H, Wd);
#pragma unroll 1
        for (int q = 0; q < kRawChunk && s0 + q < nsteps; ++q)
            step(s0 + q, q, ca);
        load_rows<NC, LG>(ca, raw, ya + s0 + 2 * kRawChunk, H, Wd);
#pragma unroll 1
        for (int q = 0; q < kRawChunk && s0 + kRawChunk + q < nsteps; ++q)
            step(s0 + kRawChunk + q, q, cb);
    }
    flush_segment<FLOW>(J, L, nseg, runs, parent, area, cap);
}

template <int KMAX, int NC>
__global__ __launch_bounds__(256) void k_morph(Table *__restrict__ T)
{
    __shared__ WaveLds s_wl[256 / kWave];
    // wave-uniform, and known to be: the band, its job and everything derived
    // from them then live in scalar registers, with scalar branches
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int nj = T->h.njobs;
    const int total = T->h.mor_pre[nj];
    for (int t = blockIdx.x * (256 / kWave) + wave; t < total; t += gridDim.x * (256 / kWave))
    {
        const int j = find_job(T->h.mor_pre, nj, t);
        Job *J = &T->jobs[j];
        const int item = t - T->h.mor_pre[j];
        if (KMAX >= 4 && J->open_it == 1 && J->close_it == 1) {   // the default opening and closing
            if (J->mgroup == 16)
                morph_band<KMAX, 1, false, 1, 1, 16>(J, 4 * item, s_wl[wave]);
            else if (J->mgroup == 32)
                morph_band<KMAX, 1, false, 1, 1, 32>(J, 2 * item, s_wl[wave]);
            else
                morph_band<KMAX, NC, false, 1, 1>(J, item, s_wl[wave]);
        } else {
            morph_band<KMAX, NC, false>(J, item, s_wl[wave]);
        }
    }
}

// ---------------------------------------------------------------------------
// Workgroup of the component stage: 1024 threads when it runs on its own;
// 256 when it runs beside a streaming kernel (pipelined steps), where a
// 1024-thread workgroup, four waves on every SIMD of a CU, finds no room
// until the streaming kernel drains.
constexpr int kResolveThreads = 1024;
constexpr int kResolveThreadsSmall = 256;
constexpr int kMaxWaves = 16;

// Component areas of one frame, summed in LDS: an open-addressing table from
// root to area. A component's runs all add to its root, and same-address
// atomics serialise far less in LDS than in the cache (a hand is a thousand
// runs on a 4K frame). A root that finds no free slot in its probe window
// adds in global memory instead, and so do all of its runs, since slots are
// only ever taken: the table and the global array never share a root.
constexpr int kAreaSlots = 2048;
constexpr int kAreaProbe = 32;
constexpr uint32_t kAreaEmpty = 0xFFFFFFFFu;
struct AreaTable {
    uint32_t key[kAreaSlots];
    uint32_t val[kAreaSlots];
    uint32_t overflow;
};
// the persistent step lends its four waves' morphology tables to it
static_assert(sizeof(AreaTable) <= 4 * sizeof(WaveLds), "area table fits the morphology LDS");

__device__ __forceinline__ void area_add(AreaTable &t, GLOBAL uint32_t *area, uint32_t root, uint32_t len)
{
    uint32_t slot = (root * 2654435761u) >> (32 - 11);
    for (int p = 0; p < kAreaProbe; ++p) {
        uint32_t k = __hip_atomic_load(&t.key[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == kAreaEmpty)
            k = atomicCAS(&t.key[slot], kAreaEmpty, root);
        if (k == kAreaEmpty || k == root) {
            atomicAdd(&t.val[slot], len);
            return;
        }
        slot = (slot + 1u) & (uint32_t)(kAreaSlots - 1);
    }
    t.overflow = 1u;
    __hip_atomic_fetch_add(area + root, len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Workgroup reductions (thread 0 and then every thread see the result).
__device__ __forceinline__ uint32_t wg_min_u32(uint32_t v, uint32_t *s_tmp)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1)
        v = min(v, (uint32_t)__shfl_xor((int)v, o, kWave));
    __syncthreads();
    if (lane == 0)
        s_tmp[wave] = v;
    __syncthreads();
    v = s_tmp[0];
    for (int w = 1; w < nw; ++w)
        v = min(v, s_tmp[w]);
    return v;
}

__device__ __forceinline__ unsigned long long wg_max_u64(unsigned long long v, unsigned long long *s_tmp)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const unsigned long long ov = __shfl_xor(v, o, kWave);
        v = ov > v ? ov : v;
    }
    __syncthreads();
    if (lane == 0)
        s_tmp[wave] = v;
    __syncthreads();
    v = s_tmp[0];
    for (int w = 1; w < nw; ++w)
        v = s_tmp[w] > v ? s_tmp[w] : v;
    return v;
}

constexpr uint32_t kNoRoot = 0xFFFFFFFFu;

// Phases A-C of the component stage for one frame (one workgroup): the joins
// across band and segment borders (and runs flagged when the pair list was
// full, joined by reading I_FIZI), every run's root and each component's
// area, and the largest component (ties to the smallest first index) as a
// key area << 32 | ~root. Afterwards area[] holds every root's area and
// each non-root run start's parent is one of its ancestors (see root_of).
__device__ __forceinline__ void resolve_forest(Job *J, AreaTable &tab, uint32_t *ncomp_out,
                                               unsigned long long *best_out)
{
    __shared__ unsigned long long s_u64[kMaxWaves];
    __shared__ uint32_t s_u32[kMaxWaves];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int W = J->W, Wd = J->Wd;
    const uint32_t nr = min(ld_dev(&J->nruns), J->run_cap);
    const GLOBAL uint64_t *runs = G(reinterpret_cast<const uint64_t *>(J->runs));
    GLOBAL uint32_t *parent = G(J->parent);
    GLOBAL uint32_t *area = G(J->area);
    const GLOBAL uint64_t *fz = G(J->fizi);
    if (threadIdx.x == 0)
        tab.overflow = 0;
    for (int i = threadIdx.x; i < kAreaSlots; i += blockDim.x) {
        tab.key[i] = kAreaEmpty;
        tab.val[i] = 0;
    }
    __syncthreads();
    const uint32_t nl = min(ld_dev(&J->nlinks), J->link_cap);
    const GLOBAL uint64_t *links = G(reinterpret_cast<const uint64_t *>(J->links));
    for (uint32_t i = threadIdx.x; i < nl; i += blockDim.x) {
        const uint64_t l = links[i];
        unite(parent, (uint32_t)l, (uint32_t)(l >> 32));
    }
    if (ld_dev(&J->nflag))
        for (uint32_t i = threadIdx.x; i < nr; i += blockDim.x) {
            const uint64_t rv = runs[i];
            if (!((uint32_t)(rv >> 32) & kLinkUp))
                continue;
            const uint2 rn = unpack_run(rv);
            const int y = (int)(rn.x / (uint32_t)W);
            if (y == 0)
                continue;
            const int xs = (int)(rn.x - (uint32_t)y * W), xe = xs + (int)rn.y - 1;
            link_up(parent, fz + (size_t)(y - 1) * Wd, Wd, W, y, xs, xe, rn.x);
        }
    __syncthreads();
    // B: roots and areas
    uint32_t ncomp = 0;
    for (uint32_t i = threadIdx.x; i < nr; i += blockDim.x) {
        const uint2 rn = unpack_run(runs[i]);
        const uint32_t root = find_root(parent, rn.x);
        if (root == rn.x)
            ++ncomp;
        else
            st_wg(parent + rn.x, root);
        area_add(tab, area, root, rn.y);
    }
    __syncthreads();
    // the table's areas go to the global array (tracking and the chain read it)
    for (int i = threadIdx.x; i < kAreaSlots; i += blockDim.x) {
        const uint32_t k = tab.key[i];
        if (k != kAreaEmpty)
            st_wg(area + k, tab.val[i]);
    }
    // C: the largest component: from the table, or from every run when some
    // root did not fit it
    unsigned long long best = 0ull;
    if (!tab.overflow) {
        for (int i = threadIdx.x; i < kAreaSlots; i += blockDim.x) {
            const uint32_t k = tab.key[i];
            if (k != kAreaEmpty) {
                const unsigned long long key = ((unsigned long long)tab.val[i] << 32) | (0xFFFFFFFFull - k);
                best = key > best ? key : best;
            }
        }
    } else {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < nr; i += blockDim.x) {
            const uint32_t s = (uint32_t)runs[i];
            if (ld_wg(parent + s) == s) {
                const unsigned long long key = ((unsigned long long)ld_wg(area + s) << 32) | (0xFFFFFFFFull - s);
                best = key > best ? key : best;
            }
        }
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const unsigned long long ob = __shfl_xor(best, o, kWave);
        best = ob > best ? ob : best;
        ncomp += (uint32_t)__shfl_xor((int)ncomp, o, kWave);
    }
    __syncthreads();
    if (lane == 0) {
        s_u64[wave] = best;
        s_u32[wave] = ncomp;
    }
    __syncthreads();
    best = s_u64[0];
    ncomp = s_u32[0];
    for (int w = 1; w < nw; ++w) {
        best = s_u64[w] > best ? s_u64[w] : best;
        ncomp += s_u32[w];
    }
    *ncomp_out = ncomp;
    *best_out = best;
}

// Root of the component of area >= amin covering pixel (tx, ty), or kNoRoot
// (one thread; the forest is final).
__device__ __forceinline__ uint32_t covering_root(const Job *J, int tx, int ty, uint32_t amin)
{
    if (tx < 0 || tx >= J->W || ty < 0 || ty >= J->H)
        return kNoRoot;
    const GLOBAL uint64_t *row = G(J->fizi) + (size_t)ty * J->Wd;
    if (!((row[tx >> 6] >> (tx & 63)) & 1ull))
        return kNoRoot;
    const uint32_t start = (uint32_t)ty * (uint32_t)J->W + (uint32_t)(prev_zero(row, tx) + 1);
    const uint32_t r = root_of(G(J->parent), start);
    return ld_wg(G(J->area) + r) >= amin ? r : kNoRoot;
}

// The component of area >= amin nearest to (tx, ty) within sqrt(r2) pixels:
// the smallest squared distance from the point to a pixel of it, ties to the
// larger area, then the smaller first index; kNoRoot when none (whole
// workgroup; the forest is final). A run's pixel nearest to the point is
// its own clamp of tx, so two passes over the runs decide it: the least
// distance, then the best key among the runs at that distance.
__device__ __forceinline__ uint32_t nearest_root(const Job *J, int tx, int ty, uint32_t amin, uint32_t r2)
{
    __shared__ uint32_t s_min[kMaxWaves];
    __shared__ unsigned long long s_key[kMaxWaves];
    const int W = J->W;
    const uint32_t nr = min(ld_dev(&J->nruns), J->run_cap);
    const GLOBAL uint64_t *runs = G(reinterpret_cast<const uint64_t *>(J->runs));
    GLOBAL uint32_t *parent = G(J->parent);
    GLOBAL uint32_t *area = G(J->area);
    auto dist2 = [&](uint2 rn) -> uint32_t {
        const int y = (int)(rn.x / (uint32_t)W), xs = (int)(rn.x - (uint32_t)y * W), xe = xs + (int)rn.y - 1;
        const int dx = tx < xs ? xs - tx : (tx > xe ? tx - xe : 0), dy = y - ty;
        const unsigned long long d2 = (unsigned long long)((long long)dx * dx) + (unsigned long long)((long long)dy * dy);
        return d2 > 0xFFFFFFFEull ? 0xFFFFFFFEu : (uint32_t)d2;
    };
    uint32_t dmin = 0xFFFFFFFFu;
    for (uint32_t i = threadIdx.x; i < nr; i += blockDim.x) {
        const uint2 rn = unpack_run(runs[i]);
        const uint32_t r = root_of(parent, rn.x);
        if (ld_wg(area + r) >= amin)
            dmin = min(dmin, dist2(rn));
    }
    dmin = wg_min_u32(dmin, s_min);
    if (dmin > r2)
        return kNoRoot;
    unsigned long long key = 0ull;
    for (uint32_t i = threadIdx.x; i < nr; i += blockDim.x) {
        const uint2 rn = unpack_run(runs[i]);
        if (dist2(rn) != dmin)
            continue;
        const uint32_t r = root_of(parent, rn.x);
        const uint32_t a = ld_wg(area + r);
        if (a >= amin) {
            const unsigned long long k = ((unsigned long long)a << 32) | (0xFFFFFFFFull - r);
            key = k > key ? k : key;
        }
    }
    key = wg_max_u64(key, s_key);
    return key ? 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull) : kNoRoot;
}

// The tracked pick given the previous frame's centroid pixel (valid: it had
// a hand): the covering component, else the nearest within the radius;
// kNoRoot for the largest (whole workgroup).
__device__ __forceinline__ uint32_t tracked_pick(const Job *J, bool valid, int tx, int ty)
{
    __shared__ uint32_t s_pick;
    const uint32_t amin = (uint32_t)max(J->min_area, 0);
    if (threadIdx.x == 0)
        s_pick = valid ? covering_root(J, tx, ty, amin) : kNoRoot;
    __syncthreads();
    uint32_t pick = s_pick;
    __syncthreads();
    if (valid && pick == kNoRoot && J->track_r2 > 0)
        pick = nearest_root(J, tx, ty, amin, J->track_r2);
    return pick;
}

struct ZoneStats {
    unsigned long long sx, sy;
    uint32_t x0, y0, x1, y1;
};

// Pass D: coordinate sums and box of component kstar, and its hand bits
// (whole workgroup; thread 0 gets the totals). Membership walks each run to
// its root without writing.
__device__ __forceinline__ ZoneStats zone_stats(const Job *J, uint32_t kstar, GLOBAL uint64_t *hand)
{
    __shared__ unsigned long long s_u64[2][kMaxWaves];
    __shared__ uint32_t s_u32[4][kMaxWaves];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int W = J->W, Wd = J->Wd;
    const uint32_t nr = min(ld_dev(&J->nruns), J->run_cap);
    const GLOBAL uint64_t *runs = G(reinterpret_cast<const uint64_t *>(J->runs));
    GLOBAL uint32_t *parent = G(J->parent);
    ZoneStats z{0, 0, 0xFFFFFFFFu, 0xFFFFFFFFu, 0, 0};
    for (uint32_t i = threadIdx.x; i < nr; i += blockDim.x) {
        const uint2 rn = unpack_run(runs[i]);
        if (root_of(parent, rn.x) != kstar)
            continue;
        const uint32_t y = rn.x / (uint32_t)W, xs = rn.x - y * (uint32_t)W;
        const uint32_t xe = xs + rn.y - 1;
        z.sx += (unsigned long long)rn.y * xs + (unsigned long long)rn.y * (rn.y - 1) / 2;
        z.sy += (unsigned long long)rn.y * y;
        z.x0 = min(z.x0, xs);
        z.x1 = max(z.x1, xe);
        z.y0 = min(z.y0, y);
        z.y1 = max(z.y1, y);
        if (hand) {
            GLOBAL uint64_t *hr = hand + (size_t)y * Wd;
            const int wa = (int)(xs >> 6), wb = (int)(xe >> 6);
            for (int w = wa; w <= wb; ++w) {
                const int lo = (w == wa) ? (int)(xs & 63) : 0;
                const int hi = (w == wb) ? (int)(xe & 63) : 63;
                const uint64_t m = (hi == 63 ? ~0ull : ((2ull << hi) - 1ull)) & (~0ull << lo);
                __hip_atomic_fetch_or(hr + w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        z.sx += __shfl_xor(z.sx, o, kWave);
        z.sy += __shfl_xor(z.sy, o, kWave);
        z.x0 = min(z.x0, (uint32_t)__shfl_xor((int)z.x0, o, kWave));
        z.y0 = min(z.y0, (uint32_t)__shfl_xor((int)z.y0, o, kWave));
        z.x1 = max(z.x1, (uint32_t)__shfl_xor((int)z.x1, o, kWave));
        z.y1 = max(z.y1, (uint32_t)__shfl_xor((int)z.y1, o, kWave));
    }
    __syncthreads();
    if (lane == 0) {
        s_u64[0][wave] = z.sx;
        s_u64[1][wave] = z.sy;
        s_u32[0][wave] = z.x0;
        s_u32[1][wave] = z.y0;
        s_u32[2][wave] = z.x1;
        s_u32[3][wave] = z.y1;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < nw; ++w) {
            z.sx += s_u64[0][w];
            z.sy += s_u64[1][w];
            z.x0 = min(z.x0, s_u32[0][w]);
            z.y0 = min(z.y0, s_u32[1][w]);
            z.x1 = max(z.x1, s_u32[2][w]);
            z.y1 = max(z.y1, s_u32[3][w]);
        }
    return z;
}

// The pointer of a frame's zone (thread 0): present when the frame has
// components and the zone's area reaches min_area; the click is the
// fill-ratio rule.
__device__ __forceinline__ fizi_pointer make_pointer(const Job *J, bool present, uint32_t A, const ZoneStats &z,
                                                     uint32_t ncomp, uint32_t inv)
{
    fizi_pointer o;
    o.present = present ? 1 : 0;
    o.click = 0;
    o.reserved = 0;
    o.area = 0;
    o.sum_x = o.sum_y = 0;
    o.x0 = o.y0 = o.x1 = o.y1 = 0;
    if (present) {
        o.area = A;
        o.sum_x = z.sx;
        o.sum_y = z.sy;
        o.x0 = z.x0;
        o.y0 = z.y0;
        o.x1 = z.x1;
        o.y1 = z.y1;
        const unsigned long long box = (unsigned long long)(z.x1 - z.x0 + 1) * (z.y1 - z.y0 + 1);
        o.click = (1000ull * A >= (unsigned long long)J->fill_pm * box) ? 1 : 0;
    }
    o.n_components = ncomp;
    o.inv_gain_q16 = inv;
    o.frame_index = J->frame_index;
    return o;
}

// Click debouncing of a tracked stream (thread 0): a change is reported
// once `debounce` consecutive frames show it; no hand clears the count.
// Updates the stream's state and returns the reported click.
__device__ __forceinline__ uint8_t debounce_click(uint32_t *state, bool present, uint8_t click, int debounce)
{
    uint32_t shown = *state & 1u, count = (*state >> 8) & 0xFFu;
    if (!present) {
        shown = 0;
        count = 0;
    } else if (click == shown) {
        count = 0;
    } else if (++count >= (uint32_t)debounce) {
        shown = click;
        count = 0;
    }
    *state = shown | (count << 8);
    return (uint8_t)shown;
}

// One workgroup per frame: the forest, the hand zone, its sums and box, and
// the pointer. A tracked frame picks its zone from the previous centroid
// (tracked_pick) and debounces its click - unless `defer`: then the frame's
// pointer is the largest component's, its root goes to J->pick, and the
// tracking chain (k_track_chain) settles the tracked frames of the launch in
// order afterwards.
__device__ __forceinline__ void resolve_job(Table *__restrict__ T, int j, bool same_launch, AreaTable &tab,
                                            bool defer = false)
{
    Job *J = &T->jobs[j];
    const int H = J->H, Wd = J->Wd;
    GLOBAL uint32_t *area = G(J->area);
    GLOBAL uint64_t *hand = J->hand ? G(J->hand) : nullptr;
    const uint32_t inv = job_gain(J, same_launch);
    if (hand)
        for (int i = threadIdx.x; i < H * Wd; i += blockDim.x)
            hand[i] = 0ull;
    uint32_t ncomp;
    unsigned long long best;
    resolve_forest(J, tab, &ncomp, &best);
    TrackState *ts = J->track;
    uint32_t pick = kNoRoot;
    if (ts && !defer)
        pick = tracked_pick(J, ts->valid != 0, ts->x, ts->y);
    const bool tracked = pick != kNoRoot;
    const uint32_t A = tracked ? ld_wg(area + pick) : (uint32_t)(best >> 32);
    const uint32_t kstar = tracked ? pick : 0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull);
    const bool present = ncomp > 0 && (long long)A >= (long long)J->min_area;
    ZoneStats z{0, 0, 0, 0, 0, 0};
    if (present)
        z = zone_stats(J, kstar, hand);
    if (threadIdx.x == 0) {
        fizi_pointer o = make_pointer(J, present, A, z, ncomp, inv);
        if (defer) {
            J->pick = ncomp > 0 ? kstar : kNoRoot;
        } else if (ts) {
            o.click = debounce_click(&ts->click, present, o.click, J->debounce);
            ts->valid = present ? 1 : 0;
            if (present) {
                ts->x = (int32_t)(z.sx / A);
                ts->y = (int32_t)(z.sy / A);
            }
        }
        *J->out = o;
        // the final pointer also goes straight to the host ring, when the
        // job has one (a deferred pick is settled by the chain kernel)
        if (J->hout && !defer)
            *J->hout = o;
    }
    __syncthreads();
}

// The job's accumulators (every field from the gain sums on) in 8-byte words.
constexpr int kAccWords = (int)((sizeof(Job) - offsetof(Job, num)) / 8);
static_assert((sizeof(Job) - offsetof(Job, num)) % 8 == 0 && offsetof(Job, num) % 8 == 0,
              "the accumulators are whole 8-byte words");

template <int NT>
__global__ __launch_bounds__(NT) void k_resolve(Table *__restrict__ T, int defer, int clear_acc)
{
    static_assert(NT >= kAccWords, "one thread per accumulator word");
    __shared__ AreaTable s_tab;
    const int nj = T->h.njobs;
    for (int j = blockIdx.x; j < nj; j += gridDim.x) {
        resolve_job(T, j, false, s_tab, defer != 0);
        // clear_acc: zero the job's accumulators, as an upload of the table
        // would, for a next call that reuses the slot without one. Every
        // thread has read them (resolve_job ends on a barrier), and no later
        // kernel of the call reads them.
        if (clear_acc && threadIdx.x < kAccWords)
            reinterpret_cast<unsigned long long *>(reinterpret_cast<uint8_t *>(&T->jobs[j]) +
                                                   offsetof(Job, num))[threadIdx.x] = 0ull;
    }
}

// Tracking of consecutive frames of one stream after a deferred component
// stage (one workgroup; every job of the table belongs to the stream and
// holds the largest component's pointer and root). Frame j's pick depends on
// frame j - 1's centroid, so it is settled in order, but nearly all of the
// work is done for all frames at once, on the guess that every earlier frame
// kept its largest component:
//   1. thread j stages frame j's pointer and largest root in LDS and tests
//      whether frame j - 1's guessed centroid pixel lies in a component of
//      frame j (the covering test: a few dependent loads);
//   2. thread 0 walks the frames in order over LDS alone: a frame whose
//      predecessor's actual centroid is the guess takes the test's answer
//      (otherwise thread 0 tests again), and when its pick is its largest
//      component its pointer only needs the debounced click. A frame that
//      needs the whole workgroup - the nearest-component pass (nothing covers
//      the centroid), or new sums, box and hand bits (the pick is not the
//      largest) - stops the walk; the workgroup does that frame, and the
//      walk goes on after it;
//   3. thread j writes frame j's pointer; thread 0 the stream's state.
constexpr int kChainMax = kMaxJobs;

__global__ __launch_bounds__(kResolveThreads) void k_track_chain(Table *__restrict__ T)
{
    __shared__ fizi_pointer s_ptr[kChainMax];
    __shared__ uint32_t s_cover[kChainMax];
    __shared__ int32_t s_gx[kChainMax], s_gy[kChainMax];   // guessed previous centroid, -1: no hand
    __shared__ int32_t s_ax, s_ay;                          // actual previous centroid, -1: no hand
    __shared__ int s_next;                                  // frame the workgroup works on, or nj
    __shared__ uint32_t s_pick;
    __shared__ int s_zone;                                  // the frame needs its zone's sums recomputed
    __shared__ uint32_t s_state;                            // debouncer state
    const int nj = min(T->h.njobs, kChainMax);
    if (nj == 0)
        return;
    TrackState *ts = T->jobs[0].track;
    for (int j = threadIdx.x; j < nj; j += blockDim.x)
        s_ptr[j] = *T->jobs[j].out;
    __syncthreads();
    // 1: the covering tests on the guess
    for (int j = threadIdx.x; j < nj; j += blockDim.x) {
        const Job *J = &T->jobs[j];
        int gx = -1, gy = -1;
        if (j == 0) {
            if (ts->valid) {
                gx = ts->x;
                gy = ts->y;
            }
        } else if (s_ptr[j - 1].present) {
            gx = (int32_t)(s_ptr[j - 1].sum_x / s_ptr[j - 1].area);
            gy = (int32_t)(s_ptr[j - 1].sum_y / s_ptr[j - 1].area);
        }
        s_gx[j] = gx;
        s_gy[j] = gy;
        s_cover[j] = gx >= 0 ? covering_root(J, gx, gy, (uint32_t)max(J->min_area, 0)) : kNoRoot;
    }
    if (threadIdx.x == 0) {
        s_ax = ts->valid ? ts->x : -1;
        s_ay = ts->valid ? ts->y : -1;
        s_state = ts->click;
    }
    __syncthreads();
    // 2: the frames in order
    int j0 = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int j = j0;
            for (; j < nj; ++j) {
                const Job *J = &T->jobs[j];
                const int ax = s_ax, ay = s_ay;
                uint32_t c = s_cover[j];
                if (ax != s_gx[j] || ay != s_gy[j])
                    c = ax >= 0 ? covering_root(J, ax, ay, (uint32_t)max(J->min_area, 0)) : kNoRoot;
                const bool near = ax >= 0 && c == kNoRoot && J->track_r2 > 0;
                if (near || (c != kNoRoot && c != J->pick)) {
                    s_pick = c;
                    s_zone = !near;
                    break;
                }
                // the largest component keeps the hand: only the click changes
                fizi_pointer &o = s_ptr[j];
                o.click = debounce_click(&s_state, o.present != 0, o.click, J->debounce);
                s_ax = o.present ? (int32_t)(o.sum_x / o.area) : -1;
                s_ay = o.present ? (int32_t)(o.sum_y / o.area) : -1;
            }
            s_next = j;
        }
        __syncthreads();
        const int j = s_next;
        if (j >= nj)
            break;
        Job *J = &T->jobs[j];
        const uint32_t amin = (uint32_t)max(J->min_area, 0);
        uint32_t pick = s_pick;
        if (!s_zone)
            pick = nearest_root(J, s_ax, s_ay, amin, J->track_r2);
        if (pick != kNoRoot && pick != J->pick) {
            // the tracked zone is not the largest: its own sums, box, hand bits
            GLOBAL uint64_t *hand = J->hand ? G(J->hand) : nullptr;
            if (hand) {
                for (int i = threadIdx.x; i < J->H * J->Wd; i += blockDim.x)
                    hand[i] = 0ull;
                __syncthreads();
            }
            const uint32_t A = ld_wg(G(J->area) + pick);
            const ZoneStats z = zone_stats(J, pick, hand);
            if (threadIdx.x == 0)
                s_ptr[j] = make_pointer(J, true, A, z, s_ptr[j].n_components, s_ptr[j].inv_gain_q16);
        }
        if (threadIdx.x == 0) {
            fizi_pointer &o = s_ptr[j];
            o.click = debounce_click(&s_state, o.present != 0, o.click, J->debounce);
            s_ax = o.present ? (int32_t)(o.sum_x / o.area) : -1;
            s_ay = o.present ? (int32_t)(o.sum_y / o.area) : -1;
        }
        j0 = j + 1;
        __syncthreads();
    }
    // 3: the pointers and the stream's state
    for (int j = threadIdx.x; j < nj; j += blockDim.x) {
        *T->jobs[j].out = s_ptr[j];
        if (T->jobs[j].hout)
            *T->jobs[j].hout = s_ptr[j];
    }
    if (threadIdx.x == 0) {
        ts->click = s_state;
        ts->valid = s_ax >= 0 ? 1 : 0;
        if (s_ax >= 0) {
            ts->x = s_ax;
            ts->y = s_ay;
        }
    }
}

// ---------------------------------------------------------------------------
// Persistent step: one launch per frame step whose workgroups take work items
// from the ordered queue of the job table (TableHeader) with one atomic
// counter. A gain item is one gain tile. A band item classifies 4 * band
// rows of a frame (once the frame's gain is complete), publishes them, then
// runs the morphology of the band above - its four waves take one sub-band
// each - once the bands it reads are published, and of its own band when it
// is the frame's last; the workgroup that completes a frame's last
// morphology band then resolves its components. Latency-bound morphology and
// components thus run while other workgroups stream later bands. Items only
// wait for items earlier in the queue, which are held by running workgroups
// that never wait for later ones, so every wait ends. Each wait is bounded
// (50 ms of the 100 MHz clock); one that gives up sets the error word and
// goes on, so that every workgroup reaches the end; the last one out resets
// the queue for the next launch.
constexpr uint64_t kWaitTicks = 5000000;

// Thread 0 waits until the counter reaches target, or the flag equals it.
__device__ __forceinline__ void spin_until(const uint32_t *p, uint32_t target, bool equal, PersistState *ps,
                                           uint64_t t0)
{
    for (;;) {
        const uint32_t v = ld_dev(p);
        if (equal ? v == target : v >= target)
            return;
        if (__builtin_amdgcn_s_memrealtime() - t0 > kWaitTicks) {
            atomicOr(&ps->error, 1u);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// After thread 0's waits: a device-scope acquire, then the workgroup goes on.
__device__ __forceinline__ void acquire_for_block()
{
    if (threadIdx.x == 0)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __syncthreads();
}

// Every wave's stores complete, then thread 0 adds v to the counter; returns
// the counter's previous value to the whole workgroup.
__device__ __forceinline__ uint32_t publish_add(uint32_t *p, uint32_t v, uint32_t *s_old)
{
    wait_own_memory();
    __syncthreads();
    if (threadIdx.x == 0)
        *s_old = atomicAdd(p, v);
    __syncthreads();
    return *s_old;
}

template <int KMAX, int NC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KMAX == 4 && NC == 1 ? 4 : 1))) void k_flow(Table *__restrict__ T, PersistState *ps)
{
    __shared__ WaveLds s_wl[256 / kWave];
    __shared__ int s_item;
    __shared__ uint32_t s_u;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int nseg = T->h.flow_nseg;
    const int total = T->h.flow_pre[nseg];
    int k = 0;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = (int)atomicAdd(&ps->next, 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= total)
            break;
        while (T->h.flow_pre[k + 1] <= item)
            ++k;
        const int seg = T->h.flow_seg[k], j = seg >> 1, idx = item - T->h.flow_pre[k];
        Job *J = &T->jobs[j];
        if ((seg & 1) == 0) {
            gain_tile(T, j, idx, J->frame);
            const uint32_t ng = (uint32_t)(T->h.gain_pre[j + 1] - T->h.gain_pre[j]);
            if (publish_add(&J->gain_done, 1u, &s_u) + 1u == ng && threadIdx.x == 0) {
                // the frame's last gain tile: its inverse gain, once, for every band
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                st_dev(G(&J->ginv), 0x80000000u | job_gain(J, true));
            }
            continue;
        }
        const int rb = 4 * J->band, H = J->H, W = J->W;
        const int nb = (H + rb - 1) / rb, nsub = (H + J->band - 1) / J->band;
        // classify the band once the frame's inverse gain is known
        if (threadIdx.x == 0) {
            spin_until(&J->ginv, 0x80000000u, false, ps, __builtin_amdgcn_s_memrealtime());
            s_u = ld_dev(&J->ginv) & 0x7FFFFFFFu;
        }
        __syncthreads();
        const uint32_t inv = s_u;
        const uint32_t p0 = (uint32_t)(idx * rb) * (uint32_t)W;
        const uint32_t p1 = (uint32_t)min(H, (idx + 1) * rb) * (uint32_t)W;
        classify_span<true>(cls_job(J), p0, p1, inv);
        wait_own_memory();
        __syncthreads();
        if (threadIdx.x == 0)
            st_dev(G(J->bflag + idx), J->epoch);
        // the morphology of the band above, and of this band when it is the last
        for (int m = max(0, idx - 1); m <= idx; ++m) {
            if (m == idx && idx != nb - 1)
                break;
            if (threadIdx.x == 0) {
                // its rows and halo lie in bands m - 1 .. m + 1
                const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                for (int bb = max(0, m - 1); bb <= min(nb - 1, m + 1); ++bb)
                    if (bb != idx)
                        spin_until(J->bflag + bb, J->epoch, true, ps, t0);
            }
            acquire_for_block();
            const int sub = 4 * m + wave;
            if (sub < nsub)
                morph_band<KMAX, NC, true>(J, sub, s_wl[wave]);
            const uint32_t cnt = (uint32_t)min(4, nsub - 4 * m);
            if (publish_add(&J->morph_done, cnt, &s_u) + cnt == (uint32_t)nsub) {
                // the frame's last band: its components
                acquire_for_block();
                // the waves' morphology tables are free again: the area table
                // takes their place
                resolve_job(T, j, true, *reinterpret_cast<AreaTable *>(&s_wl[0]));
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned done = atomicAdd(&ps->finished, 1u);
        if (done == gridDim.x - 1) {
            __hip_atomic_store(&ps->next, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ps->finished, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_make_yref(const uint8_t *frame0, uint16_t *yref, int W, int H, int rs, hipStream_t s)
{
    const int rows = (H + rs - 1) / rs;
    const int n = rows * (W / 4);
    const int grid = min((n + 255) / 256, 4096);
    k_make_yref<<<grid, 256, 0, s>>>(frame0, yref, W, H, rs);
    return hipGetLastError();
}

hipError_t launch_gain(const Table *d_tab, int total_tiles, int n_cu, const Tuning &t, hipStream_t s,
                       StageEvents ev, const CallPatch *patch)
{
    if (total_tiles <= 0)
        return hipSuccess;
    const int grid = min(total_tiles, n_cu * t.grid_per_cu);
    CallPatch p{};
    if (patch)
        p = *patch;
    FIZI_LAUNCH(k_gain, grid, 256, 0, s, ev, const_cast<Table *>(d_tab), p);
    return hipGetLastError();
}

hipError_t launch_minmax(const Table *d_tab, int njobs, uint8_t *bgmin, uint8_t *bgmax, int npx,
                         int reset, bool masked, int n_cu, hipStream_t s, StageEvents ev)
{
    const int groups = npx / 4;
    const int grid = min((groups + 255) / 256, n_cu * 8);
    if (masked)
        FIZI_LAUNCH(k_minmax<true>, grid, 256, 0, s, ev, const_cast<Table *>(d_tab), njobs, bgmin, bgmax, npx,
                    reset);
    else
        FIZI_LAUNCH(k_minmax<false>, grid, 256, 0, s, ev, const_cast<Table *>(d_tab), njobs, bgmin, bgmax, npx,
                    reset);
    return hipGetLastError();
}

hipError_t launch_classify(const Table *d_tab, int total_tiles, int n_cu, const Tuning &t, hipStream_t s,
                           StageEvents ev)
{
    if (total_tiles <= 0)
        return hipSuccess;
    const int grid = min(total_tiles, n_cu * t.grid_per_cu);
    Table *tab = const_cast<Table *>(d_tab);
    switch (t.cls_iters) {
    case 1: FIZI_LAUNCH(k_classify<1>, grid, 256, 0, s, ev, tab); break;
    case 2: FIZI_LAUNCH(k_classify<2>, grid, 256, 0, s, ev, tab); break;
    case 8: FIZI_LAUNCH(k_classify<8>, grid, 256, 0, s, ev, tab); break;
    default: FIZI_LAUNCH(k_classify<4>, grid, 256, 0, s, ev, tab); break;
    }
    return hipGetLastError();
}

hipError_t launch_morph(const Table *d_tab, int total_tiles, int max_wd, int max_ops, int n_cu,
                        const Tuning &t, hipStream_t s, StageEvents ev)
{
    if (total_tiles <= 0)
        return hipSuccess;
    const int waves = 256 / kWave;
    const int grid = min((total_tiles + waves - 1) / waves, n_cu * t.grid_per_cu);
    Table *tab = const_cast<Table *>(d_tab);
    const bool wide = max_wd > kWave, deep = max_ops > 4;
    if (!wide && !deep)
        FIZI_LAUNCH((k_morph<4, 1>), grid, 256, 0, s, ev, tab);
    else if (!wide)
        FIZI_LAUNCH((k_morph<4 * kMaxMorphIters, 1>), grid, 256, 0, s, ev, tab);
    else if (!deep)
        FIZI_LAUNCH((k_morph<4, 2>), grid, 256, 0, s, ev, tab);
    else
        FIZI_LAUNCH((k_morph<4 * kMaxMorphIters, 2>), grid, 256, 0, s, ev, tab);
    return hipGetLastError();
}

hipError_t launch_resolve(const Table *d_tab, int njobs, hipStream_t s, StageEvents ev, bool serial, bool small,
                          bool clear_acc)
{
    if (njobs <= 0)
        return hipSuccess;
    // consecutive tracked frames of one stream: every frame's forest and
    // largest component at once, then the tracking chain in frame order
    Table *tab = const_cast<Table *>(d_tab);
    const int defer = serial ? 1 : 0, clear = clear_acc ? 1 : 0;
    if (small)
        FIZI_LAUNCH(k_resolve<kResolveThreadsSmall>, njobs, kResolveThreadsSmall, 0, s, ev, tab, defer, clear);
    else
        FIZI_LAUNCH(k_resolve<kResolveThreads>, njobs, kResolveThreads, 0, s, ev, tab, defer, clear);
    if (serial) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        k_track_chain<<<1, kResolveThreads, 0, s>>>(tab);
    }
    return hipGetLastError();
}

// Blocks per CU of the persistent step: what the kernel's registers and LDS
// allow (wave64, 512 VGPRs per SIMD lane in granules of 8, four SIMDs and
// 160 KiB of LDS per CU, eight waves per SIMD), capped at four so that the
// whole grid is resident with room to spare.
template <int KMAX, int NC>
int flow_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_flow<KMAX, NC>, 256, 0) != hipSuccess)
        nb = 1;
    return std::max(1, std::min(nb, 8));
}

template <int KMAX, int NC>
hipError_t launch_flow_t(Table *tab, int n_cu, PersistState *ps, hipStream_t s, StageEvents ev)
{
    static int per_cu = -1;
    if (per_cu < 0)
        per_cu = flow_blocks_per_cu<KMAX, NC>();
    FIZI_LAUNCH((k_flow<KMAX, NC>), per_cu * n_cu, 256, 0, s, ev, tab, ps);
    return hipGetLastError();
}

hipError_t launch_persistent(const Table *d_tab, int max_wd, int max_ops, int n_cu, const Tuning &t,
                             uint8_t *persist, hipStream_t s, StageEvents ev)
{
    (void)t;
    Table *tab = const_cast<Table *>(d_tab);
    PersistState *ps = reinterpret_cast<PersistState *>(persist);
    const bool wide = max_wd > kWave, deep = max_ops > 4;
    if (!wide && !deep)
        return launch_flow_t<4, 1>(tab, n_cu, ps, s, ev);
    if (!wide)
        return launch_flow_t<4 * kMaxMorphIters, 1>(tab, n_cu, ps, s, ev);
    if (!deep)
        return launch_flow_t<4, 2>(tab, n_cu, ps, s, ev);
    return launch_flow_t<4 * kMaxMorphIters, 2>(tab, n_cu, ps, s, ev);
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const size_t grid = std::min<size_t>((n + 255) / 256, 65535);
    k_fill_u32<<<(unsigned)grid, 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

}  // namespace fizi
