"""Pins of the oracle's ELVIRA normal (Sec. 3.3; Pilliod and Puckett's
method) and of the cut-cell fractions it is built on.

What fixes the answers independently of the oracle's code:
* the area of a rectangle below a straight line has a closed form (a
  triangle, a trapezoid or the complement of a triangle); the oracle clips
  the cell polygon instead;
* ELVIRA reproduces straight interfaces exactly: when a line crosses the
  3x3 block so that every column (or row) sum is an exact height, one
  candidate is the line itself and its fraction error is zero;
* the circle's cell fractions have an exact integral, and ELVIRA's normals
  converge to the radial direction (angle error O(h), the line's position
  O(h^2)) while central differences of a sharp field do not converge;
* the method commutes with the symmetries of the square block.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
from geometry_util import area_below_line, sharp_ramp
from paper_2111_11806_amd import inputs

pytestmark = pytest.mark.filterwarnings("ignore")


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def elvira(f, hx=1.0, hy=1.0):
    """f[a+1, b+1] = r(i+a, j+b); returns the unit normal or None."""
    L = oracle.lib()
    f9 = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(9))
    n = np.zeros(2)
    ok = L.orc_elvira_normal(_dp(f9), hx, hy, _dp(n))
    return n if ok else None


def cut_fraction(n, hx, hy, beta):
    L = oracle.lib()
    nv = np.ascontiguousarray(np.asarray(n, dtype=np.float64))
    return L.orc_cut_fraction(_dp(nv), hx, hy, beta)


def line_block(m, c, below, hx=1.0, hy=1.0):
    """3x3 fractions of the body {y <= m x + c} (below) or its complement,
    coordinates relative to the centre cell's centre."""
    f = np.zeros((3, 3))
    for a in range(-1, 2):
        for b in range(-1, 2):
            x0, x1 = (a - 0.5) * hx, (a + 0.5) * hx
            y0, y1 = (b - 0.5) * hy, (b + 0.5) * hy
            fr = area_below_line(x0, x1, y0, y1, m, c) / (hx * hy)
            f[a + 1, b + 1] = fr if below else 1.0 - fr
    return f


def test_cut_fraction_matches_closed_form():
    rng = np.random.default_rng(11)
    for _ in range(400):
        hx, hy = rng.uniform(0.5, 2.0, 2)
        th = rng.uniform(0, 2 * math.pi)
        n = np.array([math.cos(th), math.sin(th)])
        beta = rng.uniform(-1.0, 1.0) * 0.5 * (abs(n[0]) * hx + abs(n[1]) * hy) * 1.1
        got = cut_fraction(n, hx, hy, beta)
        # n.p <= beta  <=>  y <= (beta - n_x x)/n_y for n_y > 0, else the complement
        if abs(n[1]) > 1e-6:
            m, c = -n[0] / n[1], beta / n[1]
            a = area_below_line(-hx / 2, hx / 2, -hy / 2, hy / 2, m, c) / (hx * hy)
            want = a if n[1] > 0 else 1.0 - a
            assert abs(got - want) < 1e-12, (n, beta, got, want)
    # special cases: a line through the centre halves the cell; an axis line
    # gives a linear fraction
    for th in np.linspace(0, 2 * math.pi, 13):
        assert abs(cut_fraction([math.cos(th), math.sin(th)], 1.3, 0.7, 0.0) - 0.5) < 1e-14
    for beta in np.linspace(-0.6, 0.6, 7):
        want = min(1.0, max(0.0, beta / 1.2 + 0.5))
        assert abs(cut_fraction([1.0, 0.0], 1.2, 0.9, beta) - want) < 1e-14


@pytest.mark.parametrize("hy", [1.0, 0.6])
def test_elvira_reproduces_straight_lines(hy):
    """Random lines through the centre cell that stay within the block's
    rows over its width: the column candidates are exact, so the chosen
    normal is the line's own. Youngs' normal is not (first order)."""
    rng = np.random.default_rng(5)
    worst_e, worst_y = 0.0, 0.0
    for _ in range(300):
        m = rng.uniform(-1.0, 1.0) * 0.5 * hy
        c = rng.uniform(-0.5, 0.5) * hy
        assert abs(c) + 1.5 * abs(m) <= 1.5 * hy
        below = bool(rng.integers(2))
        f = line_block(m, c, below, 1.0, hy)
        if not (0.0 < f[1, 1] < 1.0):
            continue
        n = elvira(f, 1.0, hy)
        t = np.array([-m, 1.0]) / math.hypot(m, 1.0)
        if not below:
            t = -t
        worst_e = max(worst_e, np.abs(n - t).max())
        gy = np.array([(f[2, 1] - f[0, 1]) / 2.0, (f[1, 2] - f[1, 0]) / (2.0 * hy)])
        ny = -gy / np.linalg.norm(gy)
        worst_y = max(worst_y, np.abs(ny - t).max())
        # the transposed block is the same line as a graph over y
        nt = elvira(f.T, hy, 1.0)
        assert np.abs(nt - t[::-1]).max() < 1e-9
    assert worst_e < 1e-9, worst_e
    assert worst_y > 1e-3, worst_y


def test_elvira_block_symmetries():
    rng = np.random.default_rng(9)
    for _ in range(100):
        m = rng.uniform(-0.5, 0.5)
        c = rng.uniform(-0.4, 0.4)
        # a smooth, not straight, interface: perturb a line block
        f = np.clip(line_block(m, c, True) + rng.uniform(-0.05, 0.05, (3, 3)), 0.0, 1.0)
        f[1, 1] = min(max(f[1, 1], 0.05), 0.95)
        n = elvira(f)
        if n is None:
            continue
        assert abs(np.linalg.norm(n) - 1.0) < 1e-14
        nx_ = elvira(f[::-1, :])          # mirror x
        assert np.abs(nx_ - [-n[0], n[1]]).max() < 1e-12
        ny_ = elvira(f[:, ::-1])          # mirror y
        assert np.abs(ny_ - [n[0], -n[1]]).max() < 1e-12
        nt = elvira(f.T)                  # swap axes
        assert np.abs(nt - n[::-1]).max() < 1e-12


def test_elvira_undefined_cases():
    assert elvira(np.ones((3, 3))) is None
    assert elvira(np.zeros((3, 3))) is None
    f = np.full((3, 3), 0.3)
    assert elvira(f) is None             # no side for either family


def _disk_area(x0, x1, y0, y1, R):
    """Exact area of the rectangle inside the disk x^2 + y^2 <= R^2."""
    def G(x):  # antiderivative of sqrt(R^2 - x^2)
        x = max(-R, min(R, x))
        return 0.5 * (x * math.sqrt(max(R * R - x * x, 0.0)) + R * R * math.asin(x / R))
    lo, hi = max(x0, -R), min(x1, R)
    if hi <= lo:
        return 0.0
    pts = {lo, hi}
    for yy in (y0, y1):
        if abs(yy) < R:
            xb = math.sqrt(R * R - yy * yy)
            for v in (-xb, xb):
                if lo < v < hi:
                    pts.add(v)
    pts = sorted(pts)
    area = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        xm = 0.5 * (a + b)
        s = math.sqrt(max(R * R - xm * xm, 0.0))
        top_c = y1 <= s          # top clamp is the constant y1
        bot_c = y0 >= -s         # bottom clamp is the constant y0
        if (y1 <= -s) or (y0 >= s):
            continue
        top = (y1 * (b - a)) if top_c else (G(b) - G(a))
        bot = (y0 * (b - a)) if bot_c else -(G(b) - G(a))
        area += top - bot
    return area


def _circle_errors(R_cells, seed):
    """Mean angle error of the ELVIRA and Youngs normals against the radial
    direction over the cut cells of a disk of radius R_cells cells."""
    rng = np.random.default_rng(seed)
    cx, cy = rng.uniform(-0.5, 0.5, 2)
    n = int(2 * R_cells) + 8
    off = n // 2
    f = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            x0, y0 = i - off - 0.5 - cx, j - off - 0.5 - cy
            f[i, j] = _disk_area(x0, x0 + 1.0, y0, y0 + 1.0, R_cells)
    e_el, e_yo = [], []
    for i in range(1, n - 1):
        for j in range(1, n - 1):
            if not (1e-9 < f[i, j] < 1.0 - 1e-9):   # cut cells (the area carries rounding)
                continue
            t = np.array([i - off - cx, j - off - cy])
            t /= np.linalg.norm(t)
            ne = elvira(f[i - 1:i + 2, j - 1:j + 2])
            e_el.append(math.acos(min(1.0, float(ne @ t))))
            g = np.array([f[i + 1, j] - f[i - 1, j], f[i, j + 1] - f[i, j - 1]])
            ny = -g / np.linalg.norm(g)
            e_yo.append(math.acos(min(1.0, float(ny @ t))))
    return float(np.mean(e_el)), float(np.mean(e_yo))


def test_disk_fractions_exact():
    # the whole disk, and a quarter
    R = 3.7
    tot = sum(_disk_area(i - 0.5, i + 0.5, j - 0.5, j + 0.5, R) for i in range(-5, 6) for j in range(-5, 6))
    assert abs(tot - math.pi * R * R) < 1e-11
    assert abs(_disk_area(0.0, 5.0, 0.0, 5.0, R) - math.pi * R * R / 4) < 1e-12


def test_elvira_converges_on_a_circle():
    """Normals of a circle with exact cell fractions: ELVIRA's angle error
    halves with the cell size (first order in the angle, so second order in
    the position of the reconstructed line across a cell), while the
    central-difference (Youngs) normal of a sharp fraction field does not
    converge; ELVIRA is the more accurate at every resolution."""
    errs = [_circle_errors(R, 3) for R in (8.0, 16.0, 32.0)]
    el = [e[0] for e in errs]
    yo = [e[1] for e in errs]
    for a, b in zip(el, yo):
        assert a < b
    assert el[0] / el[2] > 3.0, el       # two halvings, first order ~4x
    assert yo[0] / yo[2] < 1.5, yo


def test_wedge_seeding_uses_the_exact_ramp_normal():
    """Whole seeding step on a sharp (exact-fraction) 25-degree ramp in a
    uniform stream: the seeded velocity of every partially covered rigid
    cell is the stream mirrored about the ramp's exact normal."""
    prob = sharp_ramp(inputs.wedge(60, 40, normal="elvira"), 25.0)
    nx, ny = prob.n[0], prob.n[1]
    th = math.radians(25.0)
    W = prob.W0
    orc = oracle.Oracle(prob)
    orc.seed()
    Wo = orc.get_state_prim()
    t = np.array([-math.sin(th), math.cos(th)])
    u_ref = np.array([1.0, 0.0]) - 2.0 * t[0] * t
    r = W[4, 0]
    part = (r > 0.5) & (r < 1.0)
    jj, ii = np.nonzero(part)
    inner = (ii > 1) & (ii < nx - 2) & (jj > 1) & (jj < ny - 2)
    assert inner.sum() > 20
    u = Wo[1, 0][part][inner]
    v = Wo[2, 0][part][inner]
    assert np.abs(u - u_ref[0]).max() < 1e-10
    assert np.abs(v - u_ref[1]).max() < 1e-10
