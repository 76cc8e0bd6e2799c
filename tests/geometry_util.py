"""Geometry for the tests (independent of both the oracle and the HIP path):
exact cut-cell fractions of simple shapes, and boxes holding a moving,
turning ellipse or ellipsoid."""
import math

import numpy as np

from paper_2111_11806_amd import inputs


def area_below_line(x0, x1, y0, y1, m, c):
    """Exact area of {x0<=x<=x1, y0<=y<=y1, y <= m x + c}: the integral of
    clamp(m x + c, y0, y1) - y0, split where the line leaves the strip."""
    pts = [x0, x1]
    if m != 0.0:
        for yy in (y0, y1):
            xb = (yy - c) / m
            if x0 < xb < x1:
                pts.append(xb)
    pts.sort()
    area = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        ya, yb = m * a + c, m * b + c
        mid = m * 0.5 * (a + b) + c
        if mid >= y1:
            area += (b - a) * (y1 - y0)
        elif mid > y0:
            area += 0.5 * (ya + yb) * (b - a) - y0 * (b - a)
    return area


def sharp_ramp(prob, angle_deg, x_wedge=0.5, stream=(1.0, 0.0)):
    """Turn a 2D single-gas problem into a uniform stream (rho = p = 1) over
    the body {y <= tan(angle) (x - x_wedge)} given by its exact cell
    fractions (whole cells exactly 0 or 1), transmissive boundaries."""
    nx, ny = prob.n[0], prob.n[1]
    dx, dy = prob.dx[0], prob.dx[1]
    m = math.tan(math.radians(angle_deg))
    W = np.zeros_like(prob.W0)
    W[0] = 1.0
    W[1] = stream[0]
    W[2] = stream[1]
    W[3] = 1.0
    for j in range(ny):
        for i in range(nx):
            x0, x1 = prob.origin[0] + i * dx, prob.origin[0] + (i + 1) * dx
            y0, y1 = prob.origin[1] + j * dy, prob.origin[1] + (j + 1) * dy
            fr = area_below_line(x0, x1, y0, y1, m, -m * x_wedge) / (dx * dy)
            W[4, 0, j, i] = 0.0 if fr < 1e-12 else (1.0 if fr > 1.0 - 1e-12 else fr)
    prob.sdf = None
    prob.W0 = W
    prob.bc = ["transmissive"] * 6
    prob.bc_states = {}
    return prob


def ellipsoid_problem(dim, n, W, motion=((0, 0, 0), (0, 0, 0)), centre=(0.5, 0.5, 0.5), bc="periodic"):
    """A gas box (n cells per side, periodic or transmissive) holding a
    rotated ellipse (2D) or ellipsoid (3D) with rigid motion (v, omega) about
    its centre; W: primitive state of the shape the problem needs."""
    dx = 1.0 / n
    shape = (n, n, n) if dim == 3 else (1, n, n)
    z = (np.arange(shape[0]) + 0.5) * dx
    y = (np.arange(shape[1]) + 0.5) * dx
    x = (np.arange(shape[2]) + 0.5) * dx
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    # a rotated ellipsoid (ellipse in 2D): semi-axes 0.15, 0.09, 0.07, its
    # r below 1e-14 on the domain boundary
    c = np.asarray(centre)
    R = np.array([[0.8, -0.6, 0.0], [0.6, 0.8, 0.0], [0.0, 0.0, 1.0]])
    P = np.stack([X - c[0], Y - c[1], (Z - c[2]) if dim == 3 else 0.0 * X], axis=-1) @ R
    ax = np.array([0.15, 0.09, 0.07 if dim == 3 else 1e9])
    sdf = (np.sqrt(((P / ax) ** 2).sum(axis=-1)) - 1.0) * 0.15
    prob = inputs.Problem(name="rot", dim=dim, n=(n, n, n if dim == 3 else 1), dx=(dx, dx, dx if dim == 3 else 1.0),
                          origin=(0.0, 0.0, 0.0), materials=[inputs.ideal(1.4)], solid=False,
                          bc=[bc] * 6, W0=W, sdf=sdf, width=1.0, v_r=motion[0], omega=motion[1],
                          center=tuple(c), recon="bvd_thinc", riemann="hllc", cfl=0.4, seed="original",
                          t_end=1.0)
    return prob, (X, Y, Z), dx
