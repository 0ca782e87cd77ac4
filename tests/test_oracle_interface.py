"""Pins of the interface oracle (zone hit test, virtual wheel) on closed
forms: positions on the axes and diagonals of the wheel, zone borders."""
import pytest

from oracle import interface


def ptr(x, y, area=1, click=0, present=1):
    return dict(present=present, click=click, area=area, sum_x=x * area, sum_y=y * area)


def test_position_is_the_floor_of_the_mean():
    assert interface.position(dict(present=1, area=3, sum_x=10, sum_y=8)) == (3, 2)
    assert interface.position(ptr(0, 0, present=0)) is None


ZONES = [(0, 0, 9, 9), (5, 5, 19, 19), (30, 0, 39, 9)]


@pytest.mark.parametrize("xy,z", [((0, 0), 0), ((9, 9), 0), ((10, 10), 1), ((5, 5), 0), ((19, 19), 1),
                                  ((20, 19), -1), ((35, 5), 2), ((29, 5), -1)])
def test_zone_hit(xy, z):
    assert interface.zone_hit(ptr(*xy), ZONES) == z


def test_zone_hit_without_hand():
    assert interface.zone_hit(ptr(1, 1, present=0), ZONES) == -1


WHEEL = (100, 100, 40, 60, 1000, 9000)   # centre, radii, 10 deg dead zone, full at 90 deg


@pytest.mark.parametrize("dxy,cdeg", [((0, -50), 0), ((50, 0), 9000), ((0, 50), 18000), ((-50, 0), -9000),
                                      ((35, -35), 4500), ((-35, -35), -4500), ((35, 35), 13500),
                                      ((-35, 35), -13500)])
def test_wheel_angles_closed_form(dxy, cdeg):
    d = interface.drive_of(ptr(100 + dxy[0], 100 + dxy[1]), WHEEL)
    assert d["on_wheel"] == 1 and d["angle_cdeg"] == cdeg


def test_wheel_steering():
    assert interface.drive_of(ptr(100, 50), WHEEL)["steer_permille"] == 0
    # 45 deg: (4500 - 1000) / (9000 - 1000) = 437.5 permille -> 437
    assert interface.drive_of(ptr(135, 65), WHEEL)["steer_permille"] == 437
    assert interface.drive_of(ptr(65, 65), WHEEL)["steer_permille"] == -437
    assert interface.drive_of(ptr(150, 100), WHEEL)["steer_permille"] == 1000
    assert interface.drive_of(ptr(100, 150), WHEEL)["steer_permille"] == 1000     # clamped


def test_off_the_wheel_and_accelerate():
    assert interface.drive_of(ptr(100, 100), WHEEL)["on_wheel"] == 0           # the centre
    assert interface.drive_of(ptr(100, 39), WHEEL)["on_wheel"] == 0            # beyond r_max (61)
    assert interface.drive_of(ptr(100, 40), WHEEL)["on_wheel"] == 1            # exactly r_max
    assert interface.drive_of(ptr(100, 60), WHEEL)["on_wheel"] == 1            # exactly r_min
    assert interface.drive_of(ptr(100, 61), WHEEL)["on_wheel"] == 0
    assert interface.drive_of(ptr(100, 50, click=1), WHEEL)["accelerate"] == 1
    assert interface.drive_of(ptr(100, 50, present=0), WHEEL) == dict(on_wheel=0, angle_cdeg=0,
                                                                        steer_permille=0, accelerate=0)
