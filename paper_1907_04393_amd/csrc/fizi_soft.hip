// Soft (sigmoid-relaxed) skin mask for calibration, with its hand-written
// adjoint: m = sigmoid((theta - d) / T), d the Mahalanobis distance of the
// pixel's BT.601 chroma (Cb, Cr) from (mu_b, mu_r) under the covariance
// [[s_bb, s_br], [s_br, s_rr]]. Per-pixel arithmetic in FP32; gradient and
// loss sums in FP64, reduced in a fixed order (bitwise reproducible).
#include <atomic>
#include <cmath>
#include <mutex>

#include "fizi_host.h"

namespace fizi {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kSoftBlocksMax = 2048;
constexpr int kSoftOut = 8;        // 6 gradients, loss, unused
constexpr int kSoftU = 4;          // pixel groups per thread and iteration of the adjoint

// The inverse covariance P = S^-1 factors as P = L L^T, L lower triangular
// (S is positive definite), so that q = delta^T P delta = |w|^2 with w = L^T
// delta. Each component of w is an affine function of the pixel's R, G, B
// (the chroma transform folded in on the host), so a pixel costs two affine
// forms and one sum of squares. The gradient sums are taken in the w basis
// and brought back to u = P delta = L w once per workgroup, in FP64.
struct SoftParams {
    float w1[4], w2[4];            // w_i = c0 + cR R + cG G + cB B, coefficients (c0, cR, cG, cB)
    float z0, z1;                  // z log2(e) = z0 - z1 d: theta / T and 1 / T, times log2(e)
};

struct SoftChol {
    double l11, l21, l22;          // L = [[l11, 0], [l21, l22]]
};

// z is kept in base-2 units (z log2 e), so that the exponential and the
// logarithm are single hardware instructions with no scaling; rs = 1 / d;
// e = exp(-|z|); rc = 1 / (1 + e).
struct SoftPx {
    float m, z, rs, e, rc, w1, w2;
};

// Three transcendentals per pixel, each one hardware instruction (about one
// ulp, far inside the relative 1e-4 the calibration form needs): one
// reciprocal square root gives d and 1 / d, one exponential gives the
// sigmoid (and the BCE's softplus), one reciprocal. q = |w|^2 is 0 only
// where the pixel's chroma is the mean (w = 0, so every gradient term is 0
// whatever rs); 2^-100 is added to it, which changes no q above 2^-74 after
// rounding and holds rs = 2^50 and d = 2^-50 finite at the mean (the
// reading d = 0, up to a z change far below FP32 resolution).
__device__ __forceinline__ SoftPx soft_px(float r, float g, float b, const SoftParams &s)
{
    SoftPx o;
    o.w1 = fmaf(s.w1[3], b, fmaf(s.w1[2], g, fmaf(s.w1[1], r, s.w1[0])));
    o.w2 = fmaf(s.w2[3], b, fmaf(s.w2[2], g, fmaf(s.w2[1], r, s.w2[0])));
    const float q = fmaf(o.w1, o.w1, fmaf(o.w2, o.w2, 0x1p-100f));
    o.rs = __builtin_amdgcn_rsqf(q);
    o.z = fmaf(-s.z1, q * o.rs, s.z0);
    o.e = __builtin_amdgcn_exp2f(-fabsf(o.z));
    o.rc = __builtin_amdgcn_rcpf(1.0f + o.e);
    o.m = o.z >= 0.0f ? o.rc : o.e * o.rc;
    return o;
}

__device__ __forceinline__ uint32_t byte_at(uint32_t w0, uint32_t w1, uint32_t w2, int i)
{
    const uint32_t w = i < 4 ? w0 : (i < 8 ? w1 : w2);
    return (w >> (8 * (i & 3))) & 0xFFu;
}

__global__ __launch_bounds__(256) void k_soft_fwd(const uint8_t *__restrict__ frames, long long npx, SoftParams s,
                                                  float *__restrict__ mask)
{
    const long long groups = npx / 4;
    const uint32_t *f = reinterpret_cast<const uint32_t *>(frames);
    for (long long gi = blockIdx.x * (long long)blockDim.x + threadIdx.x; gi < groups;
         gi += (long long)gridDim.x * blockDim.x) {
        const uint32_t w0 = f[3 * gi], w1 = f[3 * gi + 1], w2 = f[3 * gi + 2];
        float4 out;
        out.x = soft_px(byte_at(w0, w1, w2, 0), byte_at(w0, w1, w2, 1), byte_at(w0, w1, w2, 2), s).m;
        out.y = soft_px(byte_at(w0, w1, w2, 3), byte_at(w0, w1, w2, 4), byte_at(w0, w1, w2, 5), s).m;
        out.z = soft_px(byte_at(w0, w1, w2, 6), byte_at(w0, w1, w2, 7), byte_at(w0, w1, w2, 8), s).m;
        out.w = soft_px(byte_at(w0, w1, w2, 9), byte_at(w0, w1, w2, 10), byte_at(w0, w1, w2, 11), s).m;
        reinterpret_cast<float4 *>(mask)[gi] = out;
    }
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)(npx - 4 * groups)) {
        const long long i = 4 * groups + threadIdx.x;
        mask[i] = soft_px(frames[3 * i], frames[3 * i + 1], frames[3 * i + 2], s).m;
    }
}

// Adds one pixel's contributions (FP32) to acc, gz being dL/dz up to a
// constant factor c. With u = S^-1 delta: dL/dmu = (gz / (T d)) u, dL/dS =
// (gz / (2 T d)) u u^T (the off-diagonal entry counted twice) and dL/dtheta
// = gz / T. The sums carry gq = gz / d = gz rs times w and w w^T (u = L w),
// and gz; the basis change and the constant factors (c / T, c / T, c / 2T,
// c / T, c / 2T, c / T) are applied to the sums.
__device__ __forceinline__ void soft_acc(const SoftPx &o, float gz, float *acc)
{
    const float gq = gz * o.rs;
    const float a = gq * o.w1, b = gq * o.w2;
    acc[0] += a;
    acc[1] += b;
    acc[2] = fmaf(a, o.w1, acc[2]);
    acc[3] = fmaf(a, o.w2, acc[3]);
    acc[4] = fmaf(b, o.w2, acc[4]);
    acc[5] += gz;
}

// dL/dz of one pixel from the upstream dL/dm (c = 1): dm m (1 - m), with
// m (1 - m) = e / (1 + e)^2 for either sign of z.
__device__ __forceinline__ float gz_upstream(const SoftPx &o, float dm) { return dm * (o.e * o.rc * o.rc); }

// Fused BCE: dL/dz = (m - y) / N (c = 1 / N, applied to the sums), and the
// pixel's BCE term in base-2 units, max(z, 0) - z y + log2(1 + e), is added
// to acc[6] (times ln 2 / N at the end).
__device__ __forceinline__ float gz_bce(const SoftPx &o, uint32_t y8, float *acc)
{
    const float y = fminf((float)y8, 1.0f);
    acc[6] += fmaf(-o.z, y, fmaxf(o.z, 0.0f)) + __builtin_amdgcn_logf(1.0f + o.e);
    return o.m - y;
}

// One group of 4 pixels (3 frame dwords) with its upstream gradients (dm) or
// ground-truth bytes (y4), added to acc in FP32.
template <bool BCE>
__device__ __forceinline__ void soft_group(uint32_t w0, uint32_t w1, uint32_t w2, const float *dm, uint32_t y4,
                                           const SoftParams &s, float *acc)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const SoftPx o = soft_px(byte_at(w0, w1, w2, 3 * k), byte_at(w0, w1, w2, 3 * k + 1),
                                 byte_at(w0, w1, w2, 3 * k + 2), s);
        const float gz = BCE ? gz_bce(o, (y4 >> (8 * k)) & 0xFFu, acc) : gz_upstream(o, dm[k]);
        soft_acc(o, gz, acc);
    }
}

// Output k of a workgroup's sums t (taken in the w basis) in the u basis:
// sum gq u = L sum gq w, sum gq u u^T = L (sum gq w w^T) L^T, the symmetric
// sums stored as (bb, br, rr); gz and the loss pass through.
__device__ __forceinline__ double to_u_basis(const double *t, int k, const SoftChol &L)
{
    switch (k) {
    case 0: return L.l11 * t[0];
    case 1: return fma(L.l21, t[0], L.l22 * t[1]);
    case 2: return L.l11 * L.l11 * t[2];
    case 3: return L.l11 * fma(L.l21, t[2], L.l22 * t[3]);
    case 4: return fma(L.l21 * L.l21, t[2], fma(2.0 * L.l21 * L.l22, t[3], L.l22 * L.l22 * t[4]));
    default: return t[k];
    }
}

// VEC: dL/dm is 16-byte and the ground truth 4-byte aligned, so a group's
// four values come in one load.
template <bool BCE, bool VEC>
__global__ __launch_bounds__(256) void k_soft_bwd(const uint8_t *__restrict__ frames, const float *__restrict__ dLdm,
                                                  const uint8_t *__restrict__ gt, long long npx, SoftParams s,
                                                  SoftChol L, double *__restrict__ partial)
{
    __shared__ double s_red[256 / 64][kSoftOut];
    __shared__ double s_tot[kSoftOut];
    double acc[kSoftOut] = {0, 0, 0, 0, 0, 0, 0, 0};
    const long long groups = npx / 4;
    const uint32_t *f = reinterpret_cast<const uint32_t *>(frames);
    const long long stride = (long long)gridDim.x * blockDim.x;
    // groups gi, gi + stride, ... (kSoftU of them) together: their loads in
    // flight at once, their pixels summed in FP32 before the FP64
    // accumulators
    for (long long g0 = blockIdx.x * (long long)blockDim.x + threadIdx.x; g0 < groups; g0 += kSoftU * stride) {
        uint32_t w[kSoftU][3];
        float dm[kSoftU][4] = {};
        uint32_t y4[kSoftU] = {};
        bool have[kSoftU];
#pragma unroll
        for (int u = 0; u < kSoftU; ++u) {
            const long long gi = g0 + u * stride;
            have[u] = gi < groups;
            if (!have[u])
                continue;
            w[u][0] = f[3 * gi];
            w[u][1] = f[3 * gi + 1];
            w[u][2] = f[3 * gi + 2];
            if (BCE) {
                if (VEC) {
                    y4[u] = reinterpret_cast<const uint32_t *>(gt)[gi];
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        y4[u] |= (uint32_t)gt[4 * gi + k] << (8 * k);
                }
            } else if (VEC) {
                const f32x4 v = reinterpret_cast<const f32x4 *>(dLdm)[gi];
                dm[u][0] = v.x;
                dm[u][1] = v.y;
                dm[u][2] = v.z;
                dm[u][3] = v.w;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    dm[u][k] = dLdm[4 * gi + k];
            }
        }
        float a8[kSoftOut] = {0, 0, 0, 0, 0, 0, 0, 0};   // up to 4 kSoftU pixels in FP32
#pragma unroll
        for (int u = 0; u < kSoftU; ++u)
            if (have[u])
                soft_group<BCE>(w[u][0], w[u][1], w[u][2], dm[u], y4[u], s, a8);
#pragma unroll
        for (int k = 0; k < kSoftOut - 1; ++k)
            acc[k] += (double)a8[k];
    }
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)(npx - 4 * groups)) {
        const long long i = 4 * groups + threadIdx.x;
        float a1[kSoftOut] = {0, 0, 0, 0, 0, 0, 0, 0};
        const SoftPx o = soft_px(frames[3 * i], frames[3 * i + 1], frames[3 * i + 2], s);
        const float gz = BCE ? gz_bce(o, gt[i], a1) : gz_upstream(o, dLdm[i]);
        soft_acc(o, gz, a1);
        for (int k = 0; k < kSoftOut - 1; ++k)
            acc[k] += (double)a1[k];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x / 64;
#pragma unroll
    for (int k = 0; k < kSoftOut; ++k) {
        double v = acc[k];
        for (int o = 32; o > 0; o >>= 1)
            v += __shfl_xor(v, o, 64);
        if (lane == 0)
            s_red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kSoftOut) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x / 64); ++w)
            v += s_red[w][threadIdx.x];
        s_tot[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x < kSoftOut)
        partial[blockIdx.x * kSoftOut + threadIdx.x] = to_u_basis(s_tot, threadIdx.x, L);
}

struct SoftScale {
    double k[kSoftOut];
};

// Fixed-order sum of the block partials: out[k] = sum_b partial[b][k] *
// scale[k], one workgroup per output k (each a fixed tree, so the result
// does not depend on timing).
__global__ __launch_bounds__(256) void k_soft_final(const double *__restrict__ partial, int nblocks, SoftScale scale,
                                                    double *__restrict__ out)
{
    __shared__ double s[256];
    const int k = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        v += partial[b * kSoftOut + k];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[k] = s[0] * scale.k[k];
}

// BT.601 chroma: Cb = 128 + cb . (R, G, B), Cr = 128 + cr . (R, G, B).
constexpr double kCb[3] = {-0.168736, -0.331264, 0.5};
constexpr double kCr[3] = {0.5, -0.418688, -0.081312};

int soft_params(const float p6[6], float T, SoftParams *s, SoftChol *L)
{
    if (!p6)
        return fail(FIZI_EINVAL, "null parameters");
    const double sbb = p6[2], sbr = p6[3], srr = p6[4];
    const double det = sbb * srr - sbr * sbr;
    if (!(det > 0.0) || !(sbb > 0.0))
        return fail(FIZI_EINVAL, "covariance must be positive definite");
    if (!(T > 0.0f) || !std::isfinite(T))
        return fail(FIZI_EINVAL, "temperature must be positive");
    // S^-1 = [[srr, -sbr], [-sbr, sbb]] / det = L L^T
    SoftChol c;
    c.l11 = std::sqrt(srr / det);
    c.l21 = -sbr / std::sqrt(srr * det);
    c.l22 = 1.0 / std::sqrt(srr);
    // w = L^T delta: w1 = l11 db + l21 dr, w2 = l22 dr, with db = 128 - mu_b
    // + cb . v and dr = 128 - mu_r + cr . v
    const double kb = 128.0 - (double)p6[0], kr = 128.0 - (double)p6[1];
    s->w1[0] = (float)(c.l11 * kb + c.l21 * kr);
    s->w2[0] = (float)(c.l22 * kr);
    for (int ch = 0; ch < 3; ++ch) {
        s->w1[ch + 1] = (float)(c.l11 * kCb[ch] + c.l21 * kCr[ch]);
        s->w2[ch + 1] = (float)(c.l22 * kCr[ch]);
    }
    const double log2e = 1.4426950408889634, inv_t = 1.0 / (double)T;
    s->z0 = (float)((double)p6[5] * inv_t * log2e);
    s->z1 = (float)(inv_t * log2e);
    if (L)
        *L = c;
    return FIZI_OK;
}

// Workgroups of a soft-mask launch: as many as are resident at once on the
// device (the kernel's own occupancy: the adjoints hold 70-80 VGPRs, so 6 or
// 7 of their workgroups fit a CU where the forward pass fits 8), at most one
// per 256 pixel groups and kSoftBlocksMax. Every workgroup of the
// grid-stride loops carries the same share of the pixels, so a grid larger
// than what is resident would leave a second, partial round behind the
// first. The occupancy is queried once per kernel.
template <typename K>
int soft_grid(K kernel, std::atomic<int> &per_cu, long long npx)
{
    int dev = 0, n_cu = 0;
    if (device_cu_count(&dev, &n_cu) != FIZI_OK)
        n_cu = 256;
    int nb = per_cu.load(std::memory_order_relaxed);
    if (nb < 1) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess || nb < 1)
            nb = 8;
        per_cu.store(nb, std::memory_order_relaxed);
    }
    const long long groups = (npx / 4 + 255) / 256;
    return (int)std::max<long long>(1, std::min<long long>(std::min(kSoftBlocksMax, n_cu * nb), groups));
}

std::atomic<int> g_fwd_per_cu{0};
std::atomic<int> g_bwd_per_cu[2][2];

template <bool BCE, bool VEC>
int bwd_grid(long long npx)
{
    return soft_grid(k_soft_bwd<BCE, VEC>, g_bwd_per_cu[BCE][VEC], npx);
}

int bwd_grid(bool bce, bool vec, long long npx)
{
    if (bce)
        return vec ? bwd_grid<true, true>(npx) : bwd_grid<true, false>(npx);
    return vec ? bwd_grid<false, true>(npx) : bwd_grid<false, false>(npx);
}

// Measurement hook of the soft-mask calls: dispatch events of each kernel
// (stages FIZI_SOFT_STAGE_*), like the contexts' stage clock.
StageClock g_soft_clk;
std::mutex g_soft_clk_mu;

StageEvents soft_ev(int stage)
{
    std::lock_guard<std::mutex> lock(g_soft_clk_mu);
    return g_soft_clk.next(stage);
}

int soft_backward(const uint8_t *frames, const float *dLdm, const uint8_t *gt, long long npx, const float p6[6],
                  float T, void *ws, size_t ws_bytes, double *out, int nout, void *stream)
{
    if (!frames || !out || !ws || (!dLdm && !gt))
        return fail(FIZI_EINVAL, "null argument");
    if (npx < 1)
        return fail(FIZI_EINVAL, "npx must be >= 1");
    if (reinterpret_cast<uintptr_t>(frames) % 4 != 0 || (dLdm && reinterpret_cast<uintptr_t>(dLdm) % 4 != 0))
        return fail(FIZI_EINVAL, "frames and dL/dm must be 4-byte aligned");
    if (ws_bytes < (size_t)kSoftBlocksMax * kSoftOut * sizeof(double))
        return fail(FIZI_ENOMEM, "workspace smaller than fizi_soft_workspace_bytes()");
    SoftParams s;
    SoftChol L;
    FIZI_TRY(soft_params(p6, T, &s, &L));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool vec = gt ? reinterpret_cast<uintptr_t>(gt) % 4 == 0 : reinterpret_cast<uintptr_t>(dLdm) % 16 == 0;
    const int grid = bwd_grid(gt != nullptr, vec, npx);
    double *partial = static_cast<double *>(ws);
    const StageEvents ev = soft_ev(FIZI_SOFT_STAGE_BACKWARD);
    if (gt) {
        if (vec)
            FIZI_LAUNCH((k_soft_bwd<true, true>), grid, 256, 0, st, ev, frames, dLdm, gt, npx, s, L, partial);
        else
            FIZI_LAUNCH((k_soft_bwd<true, false>), grid, 256, 0, st, ev, frames, dLdm, gt, npx, s, L, partial);
    } else {
        if (vec)
            FIZI_LAUNCH((k_soft_bwd<false, true>), grid, 256, 0, st, ev, frames, dLdm, gt, npx, s, L, partial);
        else
            FIZI_LAUNCH((k_soft_bwd<false, false>), grid, 256, 0, st, ev, frames, dLdm, gt, npx, s, L, partial);
    }
    FIZI_HIP(hipGetLastError());
    // dL/dmu_b, dL/dmu_r, dL/ds_bb, dL/ds_br, dL/ds_rr, dL/dtheta, loss: the
    // constant factors the kernel leaves out (c = 1 / N for the BCE, 1 for
    // an upstream dL/dm; the loss sum is in base-2 units)
    const double c = gt ? 1.0 / (double)npx : 1.0, ct = c / (double)T;
    const SoftScale scale{{ct, ct, 0.5 * ct, ct, 0.5 * ct, ct, c * 0.69314718055994531, 0.0}};
    const StageEvents ev_final = soft_ev(FIZI_SOFT_STAGE_FINAL);
    FIZI_LAUNCH(k_soft_final, nout, 256, 0, st, ev_final, partial, grid, scale, out);
    FIZI_HIP(hipGetLastError());
    return FIZI_OK;
}

}  // namespace
}  // namespace fizi

// Partial sums of the allocation-free BCE entry point: one row of 8 doubles
// per block of the backward kernel, for as many blocks as a launch ever
// uses (128 KiB). Every GPU the library runs on holds its own copy until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress gives on each device.
static __device__ __align__(256) double scratch[2048 * 8];

namespace fizi {
namespace {

static_assert(sizeof(scratch) == (size_t)kSoftBlocksMax * kSoftOut * sizeof(double),
              "one row of partial sums per block of the largest launch");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up once per device.
int scratch_of_current_device(double **out)
{
    int dev = 0;
    FIZI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(FIZI_EINVAL, "device ordinal beyond the library's table of 64 devices");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        FIZI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p)
            return fail(FIZI_EHIP, "hipGetSymbolAddress gave no address for the scratch array");
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return FIZI_OK;
}

}  // namespace
}  // namespace fizi

using namespace fizi;

extern "C" {

int fizi_soft_forward(const uint8_t *d_frames, int64_t npx, const float params6[6], float T, float *d_mask,
                      void *stream)
{
    if (!d_frames || !d_mask)
        return fail(FIZI_EINVAL, "null frames or mask");
    if (npx < 1)
        return fail(FIZI_EINVAL, "npx must be >= 1");
    if (reinterpret_cast<uintptr_t>(d_frames) % 4 != 0 || reinterpret_cast<uintptr_t>(d_mask) % 16 != 0)
        return fail(FIZI_EINVAL, "frames must be 4-byte and the mask 16-byte aligned");
    SoftParams s;
    FIZI_TRY(soft_params(params6, T, &s, nullptr));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const StageEvents ev = soft_ev(FIZI_SOFT_STAGE_FORWARD);
    FIZI_LAUNCH(k_soft_fwd, soft_grid(k_soft_fwd, g_fwd_per_cu, npx), 256, 0, st, ev, d_frames, npx, s, d_mask);
    FIZI_HIP(hipGetLastError());
    return FIZI_OK;
}

int fizi_soft_timing(int32_t enable)
{
    std::lock_guard<std::mutex> lock(g_soft_clk_mu);
    return g_soft_clk.enable(enable != 0);
}

int fizi_soft_times(double *h_ms, int64_t *h_launches)
{
    if (!h_ms || !h_launches)
        return fail(FIZI_EINVAL, "null argument");
    std::lock_guard<std::mutex> lock(g_soft_clk_mu);
    double ms[FIZI_NSTAGES];
    int64_t n[FIZI_NSTAGES];
    FIZI_TRY(g_soft_clk.read(ms, n));
    for (int k = 0; k < FIZI_SOFT_NSTAGES; ++k) {
        h_ms[k] = ms[k];
        h_launches[k] = n[k];
    }
    return FIZI_OK;
}

size_t fizi_soft_workspace_bytes(int64_t npx)
{
    (void)npx;
    return (size_t)kSoftBlocksMax * kSoftOut * sizeof(double);
}

int fizi_soft_backward(const uint8_t *d_frames, const float *d_dLdm, int64_t npx, const float params6[6], float T,
                       void *d_workspace, size_t workspace_bytes, double *d_grad6, void *stream)
{
    if (!d_dLdm)
        return fail(FIZI_EINVAL, "null dL/dm");
    return soft_backward(d_frames, d_dLdm, nullptr, npx, params6, T, d_workspace, workspace_bytes, d_grad6, 6,
                         stream);
}

int fizi_soft_bce(const uint8_t *d_frames, const uint8_t *d_gt, int64_t npx, const float params6[6], float T,
                  void *d_workspace, size_t workspace_bytes, double *d_out7, void *stream)
{
    if (!d_gt)
        return fail(FIZI_EINVAL, "null ground truth");
    return soft_backward(d_frames, nullptr, d_gt, npx, params6, T, d_workspace, workspace_bytes, d_out7, 7,
                         stream);
}

int fizi_soft_bce_static(const uint8_t *d_frames, const uint8_t *d_gt, int64_t npx, const float params6[6],
                         float T, double *d_out7, void *stream)
{
    if (!d_gt)
        return fail(FIZI_EINVAL, "null ground truth");
    if (npx >= 1 && (size_t)bwd_grid(true, reinterpret_cast<uintptr_t>(d_gt) % 4 == 0, npx) * kSoftOut *
                            sizeof(double) > sizeof(scratch))
        return fail(FIZI_ENOMEM, "the launch needs more partial sums than the 128 KiB static array holds");
    double *ws = nullptr;
    FIZI_TRY(scratch_of_current_device(&ws));
    // every block writes its whole row of partial sums before the final sum
    // reads it: nothing in the array has to start at zero
    return soft_backward(d_frames, nullptr, d_gt, npx, params6, T, ws, sizeof(scratch), d_out7, 7, stream);
}

}  // extern "C"
