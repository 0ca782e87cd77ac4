"""The library's pointer consumers (fizi_zone_hit, fizi_drive_of; host code,
no GPU) against the interface oracle, on seeded random pointers, zones and
wheels, with the edge cases: no hand, zone borders, the wheel's rims, the
angles at 12 and 6 o'clock, and invalid arguments."""
import numpy as np
import pytest

from oracle import interface
from paper_1907_04393_amd import fizi


def records(rows):
    a = np.zeros(len(rows), dtype=fizi.POINTER_DTYPE)
    for i, r in enumerate(rows):
        for k, v in r.items():
            a[i][k] = v
    return a


def random_pointers(rng, n, W=640, H=480):
    rows = []
    for _ in range(n):
        area = int(rng.integers(1, 5000))
        x, y = int(rng.integers(0, W)), int(rng.integers(0, H))
        rows.append(dict(present=int(rng.random() < 0.9), click=int(rng.random() < 0.3), area=area,
                         sum_x=x * area + int(rng.integers(0, area)), sum_y=y * area + int(rng.integers(0, area))))
    return records(rows)


def as_oracle(rec):
    return {k: int(rec[k]) for k in ("present", "click", "area", "sum_x", "sum_y")}


@pytest.mark.parametrize("seed", range(4))
def test_zone_hit_matches_the_oracle(seed):
    rng = np.random.default_rng(seed)
    p = random_pointers(rng, 2000)
    zones = []
    for _ in range(int(rng.integers(1, 12))):
        x0, y0 = int(rng.integers(0, 600)), int(rng.integers(0, 440))
        zones.append((x0, y0, x0 + int(rng.integers(0, 200)), y0 + int(rng.integers(0, 200))))
    got = fizi.zone_hit(p, zones)
    want = [interface.zone_hit(as_oracle(r), zones) for r in p]
    assert got.tolist() == want


def test_zone_hit_borders_and_no_zones():
    zones = [(0, 0, 9, 9), (5, 5, 19, 19)]
    p = records([dict(present=1, area=1, sum_x=x, sum_y=y) for x, y in
                 [(0, 0), (9, 9), (10, 10), (19, 19), (20, 19)]] + [dict(present=0, area=1, sum_x=1, sum_y=1)])
    assert fizi.zone_hit(p, zones).tolist() == [0, 0, 1, 1, -1, -1]
    assert fizi.zone_hit(p, np.zeros((0, 4), np.int32)).tolist() == [-1] * len(p)
    assert fizi.zone_hit(records([]), zones).tolist() == []


@pytest.mark.parametrize("seed", range(4))
def test_drive_matches_the_oracle(seed):
    rng = np.random.default_rng(100 + seed)
    p = random_pointers(rng, 3000)
    dead = int(rng.integers(0, 3000))
    wheel = (int(rng.integers(200, 440)), int(rng.integers(150, 330)), int(rng.integers(0, 60)),
             int(rng.integers(60, 300)), dead, int(rng.integers(dead + 1, 18001)))
    got = fizi.drive_of(p, wheel)
    want = [[interface.drive_of(as_oracle(r), wheel)[k] for k in fizi.DRIVE_FIELDS] for r in p]
    assert got.tolist() == want
    assert got[:, 0].sum() > 0     # some pointers land on the wheel


def test_drive_every_pixel_around_a_wheel():
    """Every position of a 161 x 161 square around the wheel, so the rims, the
    axes and all rounding cases of the angle are covered."""
    wheel = (80, 80, 30, 70, 1500, 9000)
    rows = [dict(present=1, click=(x + y) & 1, area=1, sum_x=x, sum_y=y) for y in range(161) for x in range(161)]
    p = records(rows)
    got = fizi.drive_of(p, wheel)
    want = [[interface.drive_of(r, wheel)[k] for k in fizi.DRIVE_FIELDS] for r in rows]
    assert got.tolist() == want
    at = {(r["sum_x"], r["sum_y"]): g for r, g in zip(rows, got.tolist())}
    assert at[(80, 10)] == [1, 0, 0, 0]            # 12 o'clock on the outer rim (no click)
    assert at[(80, 150)][1] == 18000               # 6 o'clock is +180, never -180
    assert at[(80, 11)] == [1, 0, 0, 1]            # odd x + y clicks
    assert at[(80, 9)][0] == 0 and at[(80, 51)][0] == 0   # just outside both rims


@pytest.mark.parametrize("wheel", [(0, 0, -1, 5, 0, 100), (0, 0, 6, 5, 0, 100), (0, 0, 0, 5, 100, 100),
                                   (0, 0, 0, 5, -1, 100), (0, 0, 0, 5, 0, 18001)])
def test_drive_rejects_bad_wheels(wheel):
    with pytest.raises(fizi.FiziError):
        fizi.drive_of(records([dict(present=1, area=1)]), wheel)


def test_pointer_layout_is_checked():
    with pytest.raises(TypeError):
        fizi.zone_hit(np.zeros(4, np.int64), [(0, 0, 1, 1)])
