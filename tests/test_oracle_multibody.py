"""Pins of the oracle's rigid-body table (several bodies with their own
motion in one r field, the extrusion test of Sec. 4.5): a piston (body 1,
moving, owning the points behind its ownership box's face) drives a shock
onto a static wall (body 0) in 1D.

- Until the shock nears the wall, the gas is the single-body piston run's,
  bitwise, left of the wall's r profile (r to 1e-10: the piston's far tail
  beyond its box moves with body 0).
- The incident shock carries the Rankine-Hugoniot piston state; the shock
  reflected off the static wall brings the gas to rest with the state of a
  piston moving at -v_p into the incident plateau (the same jump relations
  in the plateau's frame). A wall that took the piston's velocity would
  leave the gas moving.
- r keeps the piston's r = 0.5 contour at x_p + v_p t and the wall's where
  it was.
"""
import math

import numpy as np
import pytest

import exact_solutions as ex
import oracle
from paper_2111_11806_amd import inputs

pytestmark = pytest.mark.filterwarnings("ignore")

N = 800
XP, XW, VP = 0.2, 0.8, 1.0


def two_body(n=N):
    return inputs.piston_wall_1d(n, v_p=VP, x_p=XP, x_w=XW, t_end=0.4)


def test_two_bodies_match_the_single_piston_until_the_wall():
    single = oracle.Oracle(inputs.piston_1d(N, v_p=VP, x_p=XP, t_end=0.25))
    dts = single.run()
    both = oracle.Oracle(two_body())
    both.run(dts=dts)
    a, b = both.get_state_prim()[:, 0, 0], single.get_state_prim()[:, 0, 0]
    x = (np.arange(N) + 0.5) / N
    left = x < XW - 0.05  # the shock is at 0.68; the wall's r profile starts at ~0.776
    assert np.abs(b[1][left]).max() > 0.5  # the shock is under way
    assert np.array_equal(a[:3, left], b[:3, left])
    # r differs only in the piston's far tail (r ~ 1e-12 after smearing),
    # which leaves the piston's box and is then carried by body 0 (at rest)
    assert np.abs(a[3][left] - b[3][left]).max() <= 1e-10
    # gas next to the wall still at rest, the wall's r untouched
    near = (x > XW - 0.04) & (x < XW)
    assert np.all(a[1][near] == 0.0) and np.all(a[2][near] == 1.0)


def test_shock_reflected_off_the_static_wall():
    S, rho_s, p_s = ex.piston_state(VP)
    # the incident plateau meets the wall at rest: a piston at -VP into it
    Sr, rho_r, p_r = ex.piston_state(VP, rho0=rho_s, p0=p_s)
    t_hit = (XW - XP) / S
    t = 0.4
    xr = XW - (Sr - VP) * (t - t_hit)  # the reflected shock moves left
    xp = XP + VP * t
    assert xp + 0.05 < xr < XW - 0.05
    o = oracle.Oracle(two_body())
    o.run(t_end=t)
    W = o.get_state_prim()[:, 0, 0]
    x = (np.arange(N) + 0.5) / N
    rest = (x > xr + 0.02) & (x < XW - 0.02)
    assert np.all(np.abs(W[1][rest]) < 0.02)                # at rest against the static wall
    assert np.all(np.abs(W[2][rest] - p_r) < 0.02 * p_r)
    assert np.all(np.abs(W[0][rest] - rho_r) < 0.02 * rho_r)
    plate = (x > xp + 0.02) & (x < xr - 0.02)
    assert np.all(np.abs(W[1][plate] - VP) < 0.02)          # moving with the piston
    assert np.all(np.abs(W[2][plate] - p_s) < 0.02 * p_s)
    # r = 0.5 contours: the piston's moved with it, the wall's stayed
    r = W[3]
    i = np.argmax(r < 0.5)
    assert abs(0.5 * (x[i - 1] + x[i]) - xp) < 2.0 / N
    j = N - 1 - np.argmax(r[::-1] < 0.5)
    assert abs(0.5 * (x[j] + x[j + 1]) - XW) < 1.0 / N


def test_a_body_outside_its_box_moves_with_body_0():
    """The same two-body run with the piston's box moved out of the domain:
    the piston then moves with body 0 (static) and drives nothing."""
    p = two_body()
    p.bodies = (dict(p.bodies[0], box_lo=(2.0, -math.inf, -math.inf), box_hi=(3.0, math.inf, math.inf)),)
    o = oracle.Oracle(p)
    o.run(t_end=0.1)
    W = o.get_state_prim()[:, 0, 0]
    assert np.abs(W[1]).max() == 0.0 and np.all(W[2] == 1.0)
