"""Closed-form solutions used to pin the oracle (independent of it).

* Exact Riemann solver for the 1D Euler equations with stiffened-gas
  equations of state p = (gamma - 1) rho e - gamma p_inf on each side (ideal
  gas: p_inf = 0), by Newton iteration on the pressure function of the
  classical exact solver, sampled at x/t.
* The Sod tube with a rigid wall: the initial Riemann problem, the reflection
  of the shock at the wall (a Riemann problem against the mirror state) and
  the interaction of the reflected shock with the contact (a third Riemann
  problem), composed into the piecewise exact solution.
* The moving piston: Rankine-Hugoniot state of the shock ahead of a piston.
"""
from __future__ import annotations

import math

import numpy as np


class Side:
    def __init__(self, rho, u, p, gamma=1.4, pinf=0.0):
        self.rho, self.u, self.p, self.g, self.pinf = float(rho), float(u), float(p), float(gamma), float(pinf)

    @property
    def c(self):
        return math.sqrt(self.g * (self.p + self.pinf) / self.rho)


def _f(pst, s):
    """Pressure function of one side and its derivative."""
    g, P, Pi = s.g, s.p + s.pinf, pst + s.pinf
    if pst > s.p:  # shock
        A = 2.0 / ((g + 1.0) * s.rho)
        B = (g - 1.0) / (g + 1.0) * P
        q = math.sqrt(A / (Pi + B))
        return (pst - s.p) * q, q * (1.0 - 0.5 * (pst - s.p) / (Pi + B))
    c = s.c
    e = (g - 1.0) / (2.0 * g)
    f = 2.0 * c / (g - 1.0) * ((Pi / P) ** e - 1.0)
    df = 1.0 / (s.rho * c) * (Pi / P) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star(L: Side, R: Side):
    """Star pressure and velocity of the Riemann problem (L, R)."""
    p = max(0.5 * (L.p + R.p), 1e-12 - min(L.pinf, R.pinf))
    lo = -min(L.pinf, R.pinf) + 1e-14 * max(1.0, abs(L.p) + abs(R.p))
    for _ in range(200):
        fL, dL = _f(p, L)
        fR, dR = _f(p, R)
        F = fL + fR + R.u - L.u
        pn = p - F / (dL + dR)
        if pn <= lo:
            pn = 0.5 * (p + lo)
        if abs(pn - p) <= 1e-15 * max(1.0, abs(p)):
            p = pn
            break
        p = pn
    fL, _ = _f(p, L)
    fR, _ = _f(p, R)
    u = 0.5 * (L.u + R.u) + 0.5 * (fR - fL)
    return p, u


def star_density(s: Side, pst, left: bool):
    g = s.g
    P, Pi = s.p + s.pinf, pst + s.pinf
    if pst > s.p:
        r = Pi / P
        k = (g - 1.0) / (g + 1.0)
        return s.rho * (r + k) / (k * r + 1.0)
    return s.rho * (Pi / P) ** (1.0 / g)


def shock_speed(s: Side, pst, left: bool):
    g = s.g
    P, Pi = s.p + s.pinf, pst + s.pinf
    m = math.sqrt((g + 1.0) / (2.0 * g) * Pi / P + (g - 1.0) / (2.0 * g))
    return s.u - s.c * m if left else s.u + s.c * m


def sample(L: Side, R: Side, xi):
    """Exact solution (rho, u, p) at x/t = xi (array)."""
    pst, ust = star(L, R)
    xi = np.asarray(xi, float)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for k, s in enumerate(xi.flat):
        if s <= ust:
            side, sgn = L, -1.0
        else:
            side, sgn = R, 1.0
        g = side.g
        if pst > side.p:  # shock
            S = shock_speed(side, pst, sgn < 0)
            if (sgn < 0 and s <= S) or (sgn > 0 and s >= S):
                val = (side.rho, side.u, side.p)
            else:
                val = (star_density(side, pst, sgn < 0), ust, pst)
        else:  # rarefaction
            c = side.c
            cst = c * ((pst + side.pinf) / (side.p + side.pinf)) ** ((g - 1.0) / (2.0 * g))
            head = side.u + sgn * c
            tail = ust + sgn * cst
            if (sgn < 0 and s <= head) or (sgn > 0 and s >= head):
                val = (side.rho, side.u, side.p)
            elif (sgn < 0 and s >= tail) or (sgn > 0 and s <= tail):
                val = (star_density(side, pst, sgn < 0), ust, pst)
            else:
                uu = 2.0 / (g + 1.0) * (-sgn * c + (g - 1.0) / 2.0 * side.u + s)
                cc = 2.0 / (g + 1.0) * (c - sgn * (g - 1.0) / 2.0 * (side.u - s))
                cc = abs(cc)
                rr = side.rho * (cc / c) ** (2.0 / (g - 1.0))
                pp = (side.p + side.pinf) * (cc / c) ** (2.0 * g / (g - 1.0)) - side.pinf
                val = (rr, uu, pp)
        rho.flat[k], u.flat[k], p.flat[k] = val
    return rho, u, p


def sod_wall_exact(x, t, x0=0.5, xw=0.85, gamma=1.4):
    """Exact solution of the Sod tube (1,0,1 | 0.125,0,0.1) at x0 with a rigid
    wall at xw, for times before the re-reflected shock returns to the wall.
    Returns (rho, u, p) on x (cells beyond the wall are NaN) and a dict of the
    wave data."""
    L = Side(1.0, 0.0, 1.0, gamma)
    R = Side(0.125, 0.0, 0.1, gamma)
    p1, u1 = star(L, R)
    rho1L = star_density(L, p1, True)
    rho1R = star_density(R, p1, False)
    S1 = shock_speed(R, p1, False)
    t1 = (xw - x0) / S1
    info = {"p_star": p1, "u_star": u1, "rho_starL": rho1L, "rho_starR": rho1R, "shock": S1,
            "fan_head": -L.c, "t_wall": t1}
    x = np.asarray(x, float)
    out = [np.full_like(x, np.nan) for _ in range(3)]
    if t <= t1:
        r_, u_, p_ = sample(L, R, (x - x0) / t)
        for a, b in zip(out, (r_, u_, p_)):
            a[:] = b
        m = x > xw
        for a in out:
            a[m] = np.nan
        return out, info
    # reflection at the wall: post-shock state against its mirror
    B = Side(rho1R, u1, p1, gamma)
    Bm = Side(rho1R, -u1, p1, gamma)
    p2, u2 = star(B, Bm)
    rho2 = star_density(B, p2, True)
    S2 = shock_speed(B, p2, True)
    t2 = (xw - x0 - S2 * t1) / (u1 - S2)
    xc2 = x0 + u1 * t2
    info.update({"p_refl": p2, "rho_refl": rho2, "refl_shock": S2, "t_meet": t2, "x_meet": xc2})
    # state left of contact and the reflected region
    A = Side(rho1L, u1, p1, gamma)
    C = Side(rho2, 0.0, p2, gamma)
    if t <= t2:
        # fan | A | contact | B | reflected shock | C | wall
        xs = xw + S2 * (t - t1)
        xcon = x0 + u1 * t
        r_, u_, p_ = sample(L, R, (x - x0) / t)
        for a, b in zip(out, (r_, u_, p_)):
            a[:] = b
        m = (x > xs) & (x <= xw)
        out[0][m], out[1][m], out[2][m] = rho2, 0.0, p2
        m = x > xw
        for a in out:
            a[m] = np.nan
        return out, info
    p3, u3 = star(A, C)
    rho3L = star_density(A, p3, True)
    rho3R = star_density(C, p3, False)
    S3 = shock_speed(A, p3, True) if p3 > A.p else None
    S4 = shock_speed(C, p3, False) if p3 > C.p else None
    info.update({"p_int": p3, "u_int": u3, "rho_intL": rho3L, "rho_intR": rho3R, "trans_shock": S3,
                 "rerefl_shock": S4})
    t3 = t2 + (xw - xc2) / S4
    info["t_rerefl_wall"] = t3
    assert t < t3, "exact solution only composed before the re-reflected shock reaches the wall"
    r_, u_, p_ = sample(L, R, (x - x0) / t)
    for a, b in zip(out, (r_, u_, p_)):
        a[:] = b
    xT = xc2 + S3 * (t - t2)
    xC = xc2 + u3 * (t - t2)
    x4 = xc2 + S4 * (t - t2)
    for lo, hi, st in ((xT, xC, (rho3L, u3, p3)), (xC, x4, (rho3R, u3, p3)), (x4, xw, (rho2, 0.0, p2))):
        m = (x > lo) & (x <= hi)
        out[0][m], out[1][m], out[2][m] = st
    m = x > xw
    for a in out:
        a[m] = np.nan
    info.update({"x_trans": xT, "x_contact": xC, "x_rerefl": x4})
    return out, info


def piston_state(v_p, rho0=1.0, p0=1.0, gamma=1.4):
    """Rankine-Hugoniot state ahead of a piston moving at v_p into gas at rest:
    returns (shock speed, rho, p)."""
    g = gamma
    c0 = math.sqrt(g * p0 / rho0)
    # shock speed from u2 = v_p: S^2 - (g+1)/2 v S - c0^2 = 0
    a = (g + 1.0) / 4.0 * v_p
    S = a + math.sqrt(a * a + c0 * c0)
    rho = rho0 * S / (S - v_p)
    p = p0 + rho0 * S * v_p
    return S, rho, p
