/*
 * CPU oracle of the FIZI hand-mask pipeline and the Mouse pointer of
 * Magoules & Zou, "GPU Accelerated Contactless Human Machine Interface for
 * Driving Car" (arXiv 1907.04393): Section 2 (two-phase run: learn the
 * background, then per frame correct brightness, isolate the skin zones and
 * turn the hand zone into a pointer) and Section 3.1-3.2 (the three threshold
 * images, their AND, erosion/dilation, luminosity management).
 *
 * TEST INFRASTRUCTURE ONLY. This is a plain, slow, scalar restatement of the
 * definitions, written to be checked by eye against the paper. It shares no
 * code, header, table or constant generator with the GPU library; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * Where the paper is silent, garbled or self-contradictory, the readings taken
 * here are the ones listed in the design notes of the repository:
 *   R1  background learning = per-pixel, per-channel min/max over the
 *       gain-corrected user-free frames (Section 3.1 (i), the only formula the
 *       paper gives for the background model);
 *   R2  brightness correction = one global gain per frame, normalised to the
 *       first learning frame over sampled rows (Section 2 "brightness is also
 *       corrected", Section 3.2 "modify the dependent values consequently");
 *   R3  I_R1 keeps pixels OUTSIDE the learned [min - delta, max + delta] box in
 *       at least one channel (the prose of Section 3.1 (i) wins over its
 *       inverted formula);
 *   R4  I_R2 keeps pixels whose max_RGB - min_RGB >= S (the prose of
 *       Section 3.1 (ii) wins over the formula that lost its comparison);
 *   R5  I_R3 keeps pixels with chroma > 0 whose exact hexcone hue lies in the
 *       closed interval [alpha1, alpha2], wrapping through 360 when
 *       alpha1 > alpha2 (the "% 2 pi" of Section 3.1 (iii));
 *   R6  morphology = opening then closing with a 3x3 square, erosion treating
 *       out-of-image pixels as 1 and dilation treating them as 0;
 *   R7  the hand zone = the 8-connected component of largest area, ties going
 *       to the smallest first raster index (Section 2, Mouse module);
 *   R8  the pointer = area, coordinate sums, bounding box and a fill-ratio
 *       click (Section 2 "its movement, its state (click or not)");
 *   R9  partial re-learning (Section 3.3) widens the model with running
 *       frames at the pixels their I_FIZI marks as background;
 *   R10 temporal tracking (Section 2, the Mouse module "tracks" the hand):
 *       when the previous frame had a hand, with c its centroid pixel (floor
 *       of the coordinate sums over the area), the hand is the component of
 *       area >= min_area nearest to c - the smallest squared distance from c
 *       to one of its pixels, 0 for the component that covers c - provided
 *       that distance is at most track_radius pixels (ties: the larger area,
 *       then the smallest first raster index); otherwise R7 applies. With
 *       track_radius 0 only the component covering c keeps the hand;
 *   R12 adaptive thresholds (Section 3.2, "adaptive threshold or modify the
 *       dependent values consequently"): with brightness_mode 1 the pixels
 *       stay raw and the thresholds of I_R1 and I_R2 are brought to the
 *       frame's brightness instead (multiplied by the gain 2^16 / inv);
 *       the hue is the raw pixel's;
 *   R14 over-exposure filter (Section 3.2: an over-exposed hand looks white
 *       and is removed as gray, so the Luminosity component is modified in
 *       the most obvious cases): with lum_hi > 0, a corrected pixel whose HSL
 *       lightness exceeds lum_hi / 255 has it lowered to lum_hi / 255, hue
 *       and HSL saturation kept, before the gray test of I_R2; the box test
 *       I_R1 and the hue test I_R3 see the corrected pixel (the hue does not
 *       change with the lightness).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t alpha1_cdeg;          /* hue interval start, centi-degrees */
    int32_t alpha2_cdeg;          /* hue interval end, centi-degrees */
    int32_t gray_S;               /* gray tolerance S */
    int32_t bg_delta;             /* margin around the learned box */
    int32_t open_iters;           /* erosions then dilations */
    int32_t close_iters;          /* dilations then erosions */
    int32_t min_area;             /* smallest hand area reported present */
    int32_t click_fill_permille;  /* fill ratio that counts as a click */
    int32_t gain_row_stride;      /* rows sampled for the gain */
    int32_t gain_lo_q16;          /* clamp of the inverse gain, Q16 */
    int32_t gain_hi_q16;
    int32_t brightness_mode;      /* 0: correct the pixels, 1: scale the thresholds */
    int32_t click_debounce;       /* tracked streams: frames a click change needs
                                     (applied by the tracker of the Python oracle) */
    int32_t track_radius;         /* tracked streams: farthest distance (pixels)
                                     from the previous centroid pixel at which a
                                     component still keeps the hand */
    int32_t lum_hi;               /* over-exposure filter: 0 off, else the HSL
                                     lightness (x 255) over-exposed pixels are
                                     brought down to, 128..254 */
} orc_params;

typedef struct {
    uint32_t present, click, area, n_components, inv_gain_q16;
    uint32_t x0, y0, x1, y1;
    uint64_t sum_x, sum_y, frame_index;
} orc_pointer;

#define ORC_SENTINEL 0xFFFFu

static int imax(int a, int b) { return a > b ? a : b; }
static int imin(int a, int b) { return a < b ? a : b; }

/* ---- Section 3.1 (iii): hue on the hexcone --------------------------------
 * Hue in degrees as an exact fraction hnum / hden (hden = chroma > 0).
 * Returns 0 when the chroma is zero (hue undefined). */
int orc_hue_fraction(int r, int g, int b, int64_t *hnum, int64_t *hden)
{
    int mx = imax(r, imax(g, b));
    int mn = imin(r, imin(g, b));
    int c = mx - mn;
    int64_t num;
    if (c == 0)
        return 0;
    if (mx == r) {
        num = 60 * (int64_t)(g - b);          /* in (-60c, 60c] */
        if (num < 0)
            num += 360 * (int64_t)c;          /* wrap into [0, 360) */
    } else if (mx == g) {
        num = 120 * (int64_t)c + 60 * (int64_t)(b - r);
    } else {
        num = 240 * (int64_t)c + 60 * (int64_t)(r - g);
    }
    *hnum = num;
    *hden = c;
    return 1;
}

/* I_R3 membership: hue in [a1, a2] (centi-degrees), wrapping when a1 > a2. */
int orc_hue_in(int r, int g, int b, int a1, int a2)
{
    int64_t hn, hd;
    if (!orc_hue_fraction(r, g, b, &hn, &hd))
        return 0;
    int ge1 = 100 * hn >= (int64_t)a1 * hd;   /* h >= a1 / 100 */
    int le2 = 100 * hn <= (int64_t)a2 * hd;   /* h <= a2 / 100 */
    if (a1 <= a2)
        return ge1 && le2;
    return ge1 || le2;
}

/* ---- Section 2 / 3.2: brightness ------------------------------------------ */
int orc_yref_rows(int H, int rs) { return (H + rs - 1) / rs; }

/* Reference luminance of the first learning frame on the sampled rows, with a
 * sentinel where a channel is clipped (0 or 255). */
void orc_make_yref(const uint8_t *f0, int W, int H, int rs, uint16_t *yref)
{
    for (int y = 0; y < H; y += rs) {
        for (int x = 0; x < W; x++) {
            const uint8_t *p = f0 + ((size_t)y * W + x) * 3;
            uint16_t v;
            if (p[0] == 0 || p[0] == 255 || p[1] == 0 || p[1] == 255 || p[2] == 0 || p[2] == 255)
                v = ORC_SENTINEL;
            else
                v = (uint16_t)(p[0] + 2 * p[1] + p[2]);
            yref[(size_t)(y / rs) * W + x] = v;
        }
    }
}

/* Inverse gain of a frame, Q16: sum of the reference luminance over the sum of
 * the frame's luminance, over usable sampled pixels, rounded half up and
 * clamped. A pixel is usable when its reference is valid, none of its raw
 * channels is clipped, and its raw colour is not skin-hued. */
uint32_t orc_gain(const uint8_t *F, const uint16_t *yref, int W, int H, const orc_params *p)
{
    uint64_t num = 0, den = 0;
    int rs = p->gain_row_stride;
    for (int y = 0; y < H; y += rs) {
        for (int x = 0; x < W; x++) {
            uint16_t yr = yref[(size_t)(y / rs) * W + x];
            const uint8_t *q = F + ((size_t)y * W + x) * 3;
            int r = q[0], g = q[1], b = q[2];
            if (yr == ORC_SENTINEL)
                continue;
            if (r == 0 || r == 255 || g == 0 || g == 255 || b == 0 || b == 255)
                continue;
            if (orc_hue_in(r, g, b, p->alpha1_cdeg, p->alpha2_cdeg))
                continue;
            num += yr;
            den += (uint64_t)(r + 2 * g + b);
        }
    }
    if (den == 0)
        return 65536u;
    uint64_t inv = (num * 65536u + den / 2) / den;
    if (inv < (uint64_t)p->gain_lo_q16)
        inv = (uint64_t)p->gain_lo_q16;
    if (inv > (uint64_t)p->gain_hi_q16)
        inv = (uint64_t)p->gain_hi_q16;
    return (uint32_t)inv;
}

/* Corrected channel value: v * inv / 2^16, rounded half up, saturated at 255. */
int orc_correct_value(int v, uint32_t inv)
{
    uint64_t t = ((uint64_t)v * inv + 32768u) >> 16;
    return t > 255 ? 255 : (int)t;
}

void orc_correct(const uint8_t *F, uint32_t inv, size_t nbytes, uint8_t *out)
{
    for (size_t i = 0; i < nbytes; i++)
        out[i] = (uint8_t)orc_correct_value(F[i], inv);
}

/* ---- Section 2 initialisation + Section 3.1 (i): background learning ------
 * With reset, the reference luminance comes from frames[0] and the model
 * starts empty; otherwise learning continues from the given model. Every
 * frame is gain-corrected before it widens the per-channel [min, max]. */
int orc_learn(const uint8_t *frames, int n, int W, int H, const orc_params *p, int reset,
              uint8_t *bgmin, uint8_t *bgmax, uint16_t *yref, uint32_t *inv_out)
{
    size_t npx = (size_t)W * H;
    uint8_t *tmp;
    if (n < 0 || (reset && n < 1))
        return -1;
    if (reset) {
        orc_make_yref(frames, W, H, p->gain_row_stride, yref);
        memset(bgmin, 255, npx * 3);
        memset(bgmax, 0, npx * 3);
    }
    tmp = (uint8_t *)malloc(npx * 3);
    if (!tmp)
        return -2;
    for (int k = 0; k < n; k++) {
        const uint8_t *F = frames + (size_t)k * npx * 3;
        uint32_t inv = orc_gain(F, yref, W, H, p);
        if (inv_out)
            inv_out[k] = inv;
        orc_correct(F, inv, npx * 3, tmp);
        for (size_t i = 0; i < npx * 3; i++) {
            if (tmp[i] < bgmin[i])
                bgmin[i] = tmp[i];
            if (tmp[i] > bgmax[i])
                bgmax[i] = tmp[i];
        }
    }
    free(tmp);
    return 0;
}

/* ---- Section 3.3: partial re-learning --------------------------------------
 * "Dealing with the evolution of the luminosity implies sometimes to
 * re-initiate partly the machine learning" (Section 3.3). Reading R9: frames
 * seen while running widen the learned model exactly as learning frames do
 * (gain-corrected against the same reference luminance, per-channel min and
 * max), but only at the pixels the frame's I_FIZI marks as background
 * (fizi[k][i] == 0): the hand zone never enters the model. The reference
 * luminance is unchanged. fizi: n frames of W*H bytes, 0 or 1. */
int orc_relearn(const uint8_t *frames, const uint8_t *fizi, int n, int W, int H, const orc_params *p,
                uint8_t *bgmin, uint8_t *bgmax, const uint16_t *yref, uint32_t *inv_out)
{
    size_t npx = (size_t)W * H;
    uint8_t *tmp;
    if (n < 0)
        return -1;
    tmp = (uint8_t *)malloc(npx * 3);
    if (!tmp)
        return -2;
    for (int k = 0; k < n; k++) {
        const uint8_t *F = frames + (size_t)k * npx * 3;
        const uint8_t *M = fizi + (size_t)k * npx;
        uint32_t inv = orc_gain(F, yref, W, H, p);
        if (inv_out)
            inv_out[k] = inv;
        orc_correct(F, inv, npx * 3, tmp);
        for (size_t i = 0; i < npx; i++) {
            if (M[i])
                continue;
            for (int c = 0; c < 3; c++) {
                if (tmp[i * 3 + c] < bgmin[i * 3 + c])
                    bgmin[i * 3 + c] = tmp[i * 3 + c];
                if (tmp[i * 3 + c] > bgmax[i * 3 + c])
                    bgmax[i * 3 + c] = tmp[i * 3 + c];
            }
        }
    }
    free(tmp);
    return 0;
}

/* ---- Section 3.2: the over-exposure filter on the Luminosity (reading R14) --
 * HSL of an RGB pixel (channels over 255): lightness L = (max + min) / 2,
 * chroma C = max - min, saturation s = C / (1 - |2L - 1|). Over-exposed means
 * L > lum_hi / 255 (lum_hi >= 128, so L > 1/2 and 1 - |2L - 1| = 2 - 2L).
 * Bringing L down to L' = lum_hi / 255 with the hue and s kept gives the
 * chroma C' = s (2 - 2L'), all in units of 1/255:
 *   C' = C (510 - 2 lum_hi) / (510 - (max + min)),
 * and 0 for pure white (max + min = 510, C = 0). Returned as the exact
 * fraction *num / *den (den > 0). */
void orc_filtered_chroma(int r, int g, int b, int lum_hi, int64_t *num, int64_t *den)
{
    int mx = imax(r, imax(g, b)), mn = imin(r, imin(g, b));
    int c = mx - mn, l2 = mx + mn;
    if (lum_hi <= 0 || l2 <= 2 * lum_hi) {      /* not over-exposed: unchanged */
        *num = c;
        *den = 1;
    } else if (l2 == 510) {                      /* white: no hue to keep */
        *num = 0;
        *den = 1;
    } else {
        *num = (int64_t)c * (510 - 2 * lum_hi);
        *den = 510 - l2;
    }
}

/* ---- Section 3.1: the three threshold images and their AND ---------------- */
void orc_masks(const uint8_t *Fc, const uint8_t *bgmin, const uint8_t *bgmax, size_t npx,
               const orc_params *p, uint8_t *r1, uint8_t *r2, uint8_t *r3, uint8_t *raw)
{
    for (size_t i = 0; i < npx; i++) {
        const uint8_t *v = Fc + i * 3;
        int out = 0;
        for (int c = 0; c < 3; c++) {
            int lo = (int)bgmin[i * 3 + c] - p->bg_delta;
            int hi = (int)bgmax[i * 3 + c] + p->bg_delta;
            if ((int)v[c] < lo || (int)v[c] > hi)
                out = 1;
        }
        /* I_R2 on the pixel after the over-exposure filter (R14): its chroma
         * C' = num / den against S */
        int64_t num, den;
        orc_filtered_chroma(v[0], v[1], v[2], p->lum_hi, &num, &den);
        int notgray = num >= (int64_t)p->gray_S * den;
        int skin = orc_hue_in(v[0], v[1], v[2], p->alpha1_cdeg, p->alpha2_cdeg);
        if (r1) r1[i] = (uint8_t)out;
        if (r2) r2[i] = (uint8_t)notgray;
        if (r3) r3[i] = (uint8_t)skin;
        if (raw) raw[i] = (uint8_t)(out && notgray && skin);
    }
}

/* ---- Section 3.2, the other option: adaptive thresholds (reading R12) -----
 * The frame F stays raw. With the frame's gain g = 2^16 / inv (the factor
 * that maps the reference brightness to this frame's), channel v is inside
 * the learned box when (bgmin - delta) g <= v <= (bgmax + delta) g, and the
 * pixel is gray when max - min < S g. Both are compared exactly, as
 * v inv against bound 2^16. I_R3 is the hue of the raw pixel. */
void orc_masks_scaled(const uint8_t *F, const uint8_t *bgmin, const uint8_t *bgmax, size_t npx,
                      uint32_t inv, const orc_params *p, uint8_t *r1, uint8_t *r2, uint8_t *r3,
                      uint8_t *raw)
{
    const int64_t one = 65536;
    for (size_t i = 0; i < npx; i++) {
        const uint8_t *v = F + i * 3;
        int out = 0;
        for (int c = 0; c < 3; c++) {
            int64_t scaled = (int64_t)v[c] * inv;
            int64_t lo = ((int64_t)bgmin[i * 3 + c] - p->bg_delta) * one;
            int64_t hi = ((int64_t)bgmax[i * 3 + c] + p->bg_delta) * one;
            if (scaled < lo || scaled > hi)
                out = 1;
        }
        int mx = imax(v[0], imax(v[1], v[2]));
        int mn = imin(v[0], imin(v[1], v[2]));
        int notgray = (int64_t)(mx - mn) * inv >= (int64_t)p->gray_S * one;
        int skin = orc_hue_in(v[0], v[1], v[2], p->alpha1_cdeg, p->alpha2_cdeg);
        if (r1) r1[i] = (uint8_t)out;
        if (r2) r2[i] = (uint8_t)notgray;
        if (r3) r3[i] = (uint8_t)skin;
        if (raw) raw[i] = (uint8_t)(out && notgray && skin);
    }
}

/* ---- Section 3.1: erosion and dilation, 3x3 square ------------------------ */
void orc_erode(const uint8_t *in, uint8_t *out, int W, int H)
{
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int v = 1;
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int yy = y + dy, xx = x + dx;
                    if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                        continue;                 /* outside counts as 1 */
                    if (!in[(size_t)yy * W + xx])
                        v = 0;
                }
            out[(size_t)y * W + x] = (uint8_t)v;
        }
}

void orc_dilate(const uint8_t *in, uint8_t *out, int W, int H)
{
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int v = 0;
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int yy = y + dy, xx = x + dx;
                    if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                        continue;                 /* outside counts as 0 */
                    if (in[(size_t)yy * W + xx])
                        v = 1;
                }
            out[(size_t)y * W + x] = (uint8_t)v;
        }
}

/* Opening (erosions then dilations) followed by closing (dilations then
 * erosions). */
int orc_morph(const uint8_t *raw, int W, int H, int open_iters, int close_iters, uint8_t *out)
{
    size_t npx = (size_t)W * H;
    uint8_t *a = (uint8_t *)malloc(npx), *b = (uint8_t *)malloc(npx);
    if (!a || !b) {
        free(a);
        free(b);
        return -2;
    }
    memcpy(a, raw, npx);
    for (int i = 0; i < open_iters; i++) { orc_erode(a, b, W, H); memcpy(a, b, npx); }
    for (int i = 0; i < open_iters; i++) { orc_dilate(a, b, W, H); memcpy(a, b, npx); }
    for (int i = 0; i < close_iters; i++) { orc_dilate(a, b, W, H); memcpy(a, b, npx); }
    for (int i = 0; i < close_iters; i++) { orc_erode(a, b, W, H); memcpy(a, b, npx); }
    memcpy(out, a, npx);
    free(a);
    free(b);
    return 0;
}

/* ---- Section 2, Mouse module: components, hand zone, pointer -------------- */

/* 8-connected labelling by breadth-first search in raster order of the seeds.
 * labels[i] = 0 for background, 1..K for components numbered by their first
 * raster pixel. Returns K, or -2 on allocation failure. */
int orc_label(const uint8_t *m, int W, int H, int32_t *labels)
{
    size_t npx = (size_t)W * H;
    int32_t *queue = (int32_t *)malloc(npx * sizeof(int32_t) + 4);
    int k = 0;
    if (!queue)
        return -2;
    memset(labels, 0, npx * sizeof(int32_t));
    for (size_t s = 0; s < npx; s++) {
        if (!m[s] || labels[s])
            continue;
        k++;
        size_t head = 0, tail = 0;
        queue[tail++] = (int32_t)s;
        labels[s] = k;
        while (head < tail) {
            int32_t i = queue[head++];
            int y = i / W, x = i % W;
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int yy = y + dy, xx = x + dx;
                    if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                        continue;
                    size_t j = (size_t)yy * W + xx;
                    if (m[j] && !labels[j]) {
                        labels[j] = k;
                        queue[tail++] = (int32_t)j;
                    }
                }
        }
    }
    free(queue);
    return k;
}

/* Pointer of a binary FIZI image: the largest component (ties: smallest first
 * raster index) gives area, coordinate sums and bounding box; the click is a
 * filled-box test. hand (nullable) receives the selected component. */
/* The pointer of one I_FIZI mask. The hand zone is the component of largest
 * area (ties: smallest first raster index) - unless (track_x, track_y) is a
 * point (track_x >= 0, the previous frame's centroid pixel) with a component
 * of area >= min_area within track_radius of it: then the nearest such
 * component, by the squared distance from the point to its nearest pixel
 * (ties: larger area, then smaller first index) - reading R10, temporal
 * tracking. The point may lie outside the image. */
int orc_pointer_track(const uint8_t *fizi, int W, int H, const orc_params *p, uint32_t inv,
                      uint64_t frame_index, int32_t track_x, int32_t track_y, orc_pointer *out, uint8_t *hand);

int orc_pointer_of(const uint8_t *fizi, int W, int H, const orc_params *p, uint32_t inv,
                   uint64_t frame_index, orc_pointer *out, uint8_t *hand)
{
    return orc_pointer_track(fizi, W, H, p, inv, frame_index, -1, -1, out, hand);
}

int orc_pointer_track(const uint8_t *fizi, int W, int H, const orc_params *p, uint32_t inv,
                      uint64_t frame_index, int32_t track_x, int32_t track_y, orc_pointer *out, uint8_t *hand)
{
    size_t npx = (size_t)W * H;
    int32_t *labels = (int32_t *)malloc(npx * sizeof(int32_t) + 4);
    if (!labels)
        return -2;
    int K = orc_label(fizi, W, H, labels);
    if (K < 0) {
        free(labels);
        return K;
    }
    uint64_t *area = (uint64_t *)calloc((size_t)K + 1, sizeof(uint64_t));
    uint64_t *first = (uint64_t *)calloc((size_t)K + 1, sizeof(uint64_t));
    for (size_t i = npx; i-- > 0;) {
        int32_t l = labels[i];
        if (l) {
            area[l]++;
            first[l] = i;                         /* ends at the smallest index */
        }
    }
    int best = 0;
    for (int l = 1; l <= K; l++) {
        if (best == 0 || area[l] > area[best] || (area[l] == area[best] && first[l] < first[best]))
            best = l;
    }
    if (track_x >= 0 && K > 0) {
        /* squared distance from the point to the nearest pixel of each
         * component, by brute force over the pixels */
        uint64_t *dmin = (uint64_t *)malloc(((size_t)K + 1) * sizeof(uint64_t));
        if (!dmin) {
            free(area);
            free(first);
            free(labels);
            return -2;
        }
        for (int l = 0; l <= K; l++)
            dmin[l] = UINT64_MAX;
        for (size_t i = 0; i < npx; i++) {
            int32_t l = labels[i];
            if (!l)
                continue;
            int64_t dx = (int64_t)(i % W) - track_x, dy = (int64_t)(i / W) - track_y;
            uint64_t d2 = (uint64_t)(dx * dx + dy * dy);
            if (d2 < dmin[l])
                dmin[l] = d2;
        }
        uint64_t amin = (uint64_t)(p->min_area > 0 ? p->min_area : 0);
        uint64_t r2 = (uint64_t)p->track_radius * (uint64_t)p->track_radius;
        int near = 0;
        for (int l = 1; l <= K; l++) {
            if (area[l] < amin || dmin[l] > r2)
                continue;
            if (near == 0 || dmin[l] < dmin[near] ||
                (dmin[l] == dmin[near] && (area[l] > area[near] ||
                                           (area[l] == area[near] && first[l] < first[near]))))
                near = l;
        }
        if (near)
            best = near;
        free(dmin);
    }
    memset(out, 0, sizeof(*out));
    out->n_components = (uint32_t)K;
    out->inv_gain_q16 = inv;
    out->frame_index = frame_index;
    if (hand)
        memset(hand, 0, npx);
    if (best && area[best] >= (uint64_t)(p->min_area > 0 ? p->min_area : 0)) {
        uint32_t x0 = (uint32_t)W, y0 = (uint32_t)H, x1 = 0, y1 = 0;
        uint64_t sx = 0, sy = 0;
        for (size_t i = 0; i < npx; i++) {
            if (labels[i] != best)
                continue;
            uint32_t x = (uint32_t)(i % W), y = (uint32_t)(i / W);
            sx += x;
            sy += y;
            if (x < x0) x0 = x;
            if (x > x1) x1 = x;
            if (y < y0) y0 = y;
            if (y > y1) y1 = y;
            if (hand)
                hand[i] = 1;
        }
        out->present = 1;
        out->area = (uint32_t)area[best];
        out->sum_x = sx;
        out->sum_y = sy;
        out->x0 = x0;
        out->y0 = y0;
        out->x1 = x1;
        out->y1 = y1;
        uint64_t box = (uint64_t)(x1 - x0 + 1) * (uint64_t)(y1 - y0 + 1);
        out->click = (1000u * area[best] >= (uint64_t)p->click_fill_permille * box) ? 1u : 0u;
    }
    free(area);
    free(first);
    free(labels);
    return 0;
}

/* One running-phase frame end to end: gain, correction, the three masks and
 * their AND, morphology, then the pointer. raw / fizi / hand are byte masks
 * (nullable except fizi). */
int orc_process_track(const uint8_t *F, const uint8_t *bgmin, const uint8_t *bgmax,
                      const uint16_t *yref, int W, int H, const orc_params *p, uint64_t frame_index,
                      int32_t track_x, int32_t track_y, orc_pointer *out, uint8_t *raw_out, uint8_t *fizi,
                      uint8_t *hand);

int orc_process(const uint8_t *F, const uint8_t *bgmin, const uint8_t *bgmax,
                const uint16_t *yref, int W, int H, const orc_params *p, uint64_t frame_index,
                orc_pointer *out, uint8_t *raw_out, uint8_t *fizi, uint8_t *hand)
{
    return orc_process_track(F, bgmin, bgmax, yref, W, H, p, frame_index, -1, -1, out, raw_out, fizi, hand);
}

int orc_process_track(const uint8_t *F, const uint8_t *bgmin, const uint8_t *bgmax,
                      const uint16_t *yref, int W, int H, const orc_params *p, uint64_t frame_index,
                      int32_t track_x, int32_t track_y, orc_pointer *out, uint8_t *raw_out, uint8_t *fizi,
                      uint8_t *hand)
{
    size_t npx = (size_t)W * H;
    uint8_t *fc = (uint8_t *)malloc(npx * 3);
    uint8_t *raw = (uint8_t *)malloc(npx);
    int rc;
    if (!fc || !raw) {
        free(fc);
        free(raw);
        return -2;
    }
    uint32_t inv = orc_gain(F, yref, W, H, p);
    if (p->brightness_mode == 1) {
        orc_masks_scaled(F, bgmin, bgmax, npx, inv, p, NULL, NULL, NULL, raw);
    } else {
        orc_correct(F, inv, npx * 3, fc);
        orc_masks(fc, bgmin, bgmax, npx, p, NULL, NULL, NULL, raw);
    }
    if (raw_out)
        memcpy(raw_out, raw, npx);
    rc = orc_morph(raw, W, H, p->open_iters, p->close_iters, fizi);
    if (rc == 0)
        rc = orc_pointer_track(fizi, W, H, p, inv, frame_index, track_x, track_y, out, hand);
    free(fc);
    free(raw);
    return rc;
}
