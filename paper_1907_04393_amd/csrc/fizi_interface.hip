// The pointer's consumers, on the host: the Interface module's zone hit test
// (Section 2) and the driving application's virtual wheel (Section 4).
// Pointers are a few dozen bytes per frame, so this runs where the
// application reads them.
#include <cmath>

#include "fizi_host.h"

using namespace fizi;

namespace {

// The pointer's position: its centroid pixel (floor of the sums over the
// area); false without a hand.
bool position(const fizi_pointer &p, int64_t *x, int64_t *y)
{
    if (!p.present || p.area == 0)
        return false;
    *x = (int64_t)(p.sum_x / p.area);
    *y = (int64_t)(p.sum_y / p.area);
    return true;
}

double round_half_away(double v) { return v >= 0.0 ? std::floor(v + 0.5) : -std::floor(-v + 0.5); }

}  // namespace

extern "C" {

int fizi_zone_hit(const fizi_pointer *h_pointers, int32_t n, const fizi_zone *h_zones, int32_t n_zones,
                  int32_t *h_zone)
{
    if (n < 0 || n_zones < 0)
        return fail(FIZI_EINVAL, "negative count");
    if ((n > 0 && (!h_pointers || !h_zone)) || (n_zones > 0 && !h_zones))
        return fail(FIZI_EINVAL, "null array");
    for (int32_t i = 0; i < n; ++i) {
        int64_t x, y;
        int32_t hit = -1;
        if (position(h_pointers[i], &x, &y))
            for (int32_t z = 0; z < n_zones; ++z) {
                const fizi_zone &r = h_zones[z];
                if (x >= r.x0 && x <= r.x1 && y >= r.y0 && y <= r.y1) {
                    hit = z;
                    break;
                }
            }
        h_zone[i] = hit;
    }
    return FIZI_OK;
}

int fizi_drive_of(const fizi_pointer *h_pointers, int32_t n, const fizi_wheel *wheel, fizi_drive *h_out)
{
    if (n < 0)
        return fail(FIZI_EINVAL, "negative count");
    if (!wheel || (n > 0 && (!h_pointers || !h_out)))
        return fail(FIZI_EINVAL, "null argument");
    if (wheel->r_min < 0 || wheel->r_max < wheel->r_min || wheel->dead_cdeg < 0 ||
        wheel->full_cdeg <= wheel->dead_cdeg || wheel->full_cdeg > 18000)
        return fail(FIZI_EINVAL, "wheel needs 0 <= r_min <= r_max and 0 <= dead < full <= 18000");
    const double pi = 3.141592653589793;
    for (int32_t i = 0; i < n; ++i) {
        fizi_drive d{0, 0, 0, 0};
        int64_t x, y;
        if (position(h_pointers[i], &x, &y)) {
            const int64_t dx = x - wheel->cx, dy = y - wheel->cy;
            const int64_t d2 = dx * dx + dy * dy;
            const int64_t r0 = wheel->r_min, r1 = wheel->r_max;
            if (d2 >= r0 * r0 && d2 <= r1 * r1) {
                // image rows grow downwards: 12 o'clock is (0, -1)
                const double ang = std::atan2((double)dx, (double)-dy) * (180.0 / pi);
                int32_t cdeg = (int32_t)round_half_away(ang * 100.0);
                if (cdeg == -18000)
                    cdeg = 18000;
                const int32_t mag = cdeg < 0 ? -cdeg : cdeg;
                int32_t steer = 0;
                if (mag > wheel->dead_cdeg) {
                    const int64_t s = ((int64_t)(mag - wheel->dead_cdeg) * 1000) / (wheel->full_cdeg - wheel->dead_cdeg);
                    steer = (int32_t)(s < 1000 ? s : 1000);
                    if (cdeg < 0)
                        steer = -steer;
                }
                d.on_wheel = 1;
                d.angle_cdeg = cdeg;
                d.steer_permille = steer;
                d.accelerate = h_pointers[i].click ? 1 : 0;
            }
        }
        h_out[i] = d;
    }
    return FIZI_OK;
}

}  // extern "C"
