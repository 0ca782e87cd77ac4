"""CPU oracle of the pointer's consumers: the Interface module's zone hit test
(Section 2: "it determines the interface zone activated by the pointer") and
the driving application's virtual wheel (Section 4: the hand moves around an
imaginary wheel; the game controls left, right and speed).

TEST INFRASTRUCTURE ONLY: plain Python restating the readings below; only the
tests load it. Readings (R11): a pointer's position is its centroid pixel
(floor of the coordinate sums over the area); a zone is an inclusive pixel
rectangle and the activated zone is the first one (in list order) that holds
the position. On the wheel centred at (cx, cy), a pointer whose position lies
at a distance in [r_min, r_max] is on the wheel; its angle is measured from
12 o'clock, clockwise positive, in (-180, 180] degrees and reported in
hundredths of a degree (rounded half away from zero); steering is 0 within
the dead zone and grows linearly to +-1000 permille at full_cdeg (negative
is left); a closed palm (the pointer's click) accelerates."""
import math


def position(p):
    if not p["present"] or p["area"] == 0:
        return None
    return (p["sum_x"] // p["area"], p["sum_y"] // p["area"])


def zone_hit(p, zones):
    pos = position(p)
    if pos is None:
        return -1
    x, y = pos
    for i, (x0, y0, x1, y1) in enumerate(zones):
        if x0 <= x <= x1 and y0 <= y <= y1:
            return i
    return -1


def _round_half_away(v):
    return int(math.floor(v + 0.5)) if v >= 0 else -int(math.floor(-v + 0.5))


def drive_of(p, wheel):
    """wheel = (cx, cy, r_min, r_max, dead_cdeg, full_cdeg) -> dict."""
    cx, cy, r_min, r_max, dead, full = wheel
    off = dict(on_wheel=0, angle_cdeg=0, steer_permille=0, accelerate=0)
    pos = position(p)
    if pos is None:
        return off
    dx, dy = pos[0] - cx, pos[1] - cy
    d2 = dx * dx + dy * dy
    if d2 < r_min * r_min or d2 > r_max * r_max:
        return off
    # image y grows downwards: 12 o'clock is (0, -1), clockwise is +x first
    ang = math.degrees(math.atan2(dx, -dy))
    cdeg = _round_half_away(ang * 100.0)
    if cdeg == -18000:
        cdeg = 18000
    mag = abs(cdeg)
    if mag <= dead:
        steer = 0
    else:
        steer = min(1000, ((mag - dead) * 1000) // max(1, full - dead))
        steer = steer if cdeg > 0 else -steer
    return dict(on_wheel=1, angle_cdeg=cdeg, steer_permille=steer, accelerate=int(p["click"]))
