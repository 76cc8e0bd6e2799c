"""Seeded synthetic inputs (initial states, signed distances, materials).

This module is shared by the GPU path, the CPU oracle and the tests. It holds
no arithmetic of the method itself: only grids, initial primitive fields,
signed-distance functions of the rigid bodies and material constants. The
conversion of a signed distance to the rigid volume fraction, every closure,
flux and update is implemented separately on each side.

Primitive field order (one plane per field, shape [nfields, nz, ny, nx]):
``phi_l`` (N-1), ``rho_l`` (N), ``u`` (dim), ``p``, [``Vbar`` (9), ``eps_p``],
``r``; the bracketed fields exist only for the elastoplastic system.

Workloads (sizes and states as the method's own test problems prescribe):

* ``sod_wall``        1D Sod tube with a static rigid wall at x = 0.85.
* ``shock_cylinder``  2D Mach 2.8 shock over a static rigid cylinder.
* ``air_water``       2D two-phase air/water (stiffened gases) with a rigid
                      ellipse moving at 100 m/s through a water column.
* ``copper_indenter`` 3D copper (Romenskii, perfect plasticity) in air with a
                      flat-ended rigid cylinder pressed in at 200 m/s.
* ``batch``           64 seeded 2D shock/rigid-ellipse instances.
* ``wedge``           2D planar shock reflecting from a static rigid wedge
                      (Mach 1.7 / 25 degrees, or Mach 10 / 30 degrees),
                      ELVIRA normals.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Problem:
    name: str
    dim: int
    n: tuple                      # (nx, ny, nz); unused dims are 1
    dx: tuple                     # cell sizes (3)
    origin: tuple                 # lower corner (3)
    materials: List[dict]
    solid: bool
    bc: List[str]                 # xlo, xhi, ylo, yhi, zlo, zhi
    W0: np.ndarray                # [nfields, nz, ny, nx]
    bc_states: Dict[int, np.ndarray] = dataclasses.field(default_factory=dict)
    sdf: Optional[np.ndarray] = None   # [nz, ny, nx], negative inside the body
    width: float = 1.0
    v_r: tuple = (0.0, 0.0, 0.0)
    omega: tuple = (0.0, 0.0, 0.0)
    center: tuple = (0.0, 0.0, 0.0)
    # further rigid bodies with their own motion, each a dict with v, omega,
    # center and its ownership box box_lo, box_hi (3-tuples); v_r, omega and
    # center above are body 0's, which moves every point no box claims
    bodies: tuple = ()
    # primitive state of the gas that fills a gap opening between a solid and
    # a rigid body; when set, the void-opening face modifier is on
    gap_gas: Optional[np.ndarray] = None
    recon: str = "bvd_thinc"
    riemann: str = "hllc"
    seed: str = "original"
    probe: str = "stepout"
    normal: str = "youngs"        # rigid-body normal: "youngs" or "elvira" (2D)
    plastic: bool = True
    thinc_beta: float = 1.6
    lm_mach: float = 0.1
    cfl: float = 0.4
    t_end: float = 0.0

    def body_table(self):
        """(v, omega, center, box_lo, box_hi), each (1 + len(bodies)) x 3,
        body 0 first (its box row unused)."""
        rows = [dict(v=self.v_r, omega=self.omega, center=self.center, box_lo=(0.0,) * 3, box_hi=(0.0,) * 3)]
        rows += list(self.bodies)
        return tuple(np.array([r[k] for r in rows], dtype=np.float64)
                     for k in ("v", "omega", "center", "box_lo", "box_hi"))

    @property
    def nmat(self):
        return len(self.materials)

    @property
    def nfields(self):
        return 2 * self.nmat + self.dim + 1 + (10 if self.solid else 0)

    @property
    def ncells(self):
        return int(np.prod(self.n))

    def field_names(self):
        N, D = self.nmat, self.dim
        names = [f"phi{l}" for l in range(N - 1)] + [f"rho{l}" for l in range(N)]
        names += ["u", "v", "w"][:D] + ["p"]
        if self.solid:
            names += [f"V{a}{b}" for a in range(3) for b in range(3)] + ["eps_p"]
        return names + ["r"]

    def cons_names(self):
        N, D = self.nmat, self.dim
        names = [f"arho{l}" for l in range(N)] + ["mx", "my", "mz"][:D] + ["E"]
        names += [f"phi{l}" for l in range(N - 1)]
        if self.solid:
            names += [f"V{a}{b}" for a in range(3) for b in range(3)] + ["aeps"]
        return names + ["r"]


def ideal(gamma):
    return {"kind": "ideal", "gamma": float(gamma)}


def stiffened(gamma, pinf):
    return {"kind": "stiffened", "gamma": float(gamma), "pinf": float(pinf)}


def romenskii(rho0, K0, G0, alpha, beta, Gamma0, sigY=0.0):
    return {"kind": "romenskii", "rho0": float(rho0), "K0": float(K0), "G0": float(G0),
            "alpha": float(alpha), "beta": float(beta), "Gamma0": float(Gamma0), "sigY": float(sigY)}


# Romenskii parameters of the method's Table 1 (SI units).
TABLE1 = {
    "aluminium": dict(rho0=2703.0, K0=76.3e9, G0=26.36e9, alpha=0.627, beta=2.288, Gamma0=1.484),
    "copper": dict(rho0=8960.0, K0=130.1e9, G0=43.33e9, alpha=1.0, beta=3.0, Gamma0=2.0),
    "steel": dict(rho0=8030.0, K0=156.2e9, G0=77.2e9, alpha=0.569, beta=2.437, Gamma0=1.563),
}


def _centres(n, dx, origin):
    return [origin[a] + (np.arange(n[a]) + 0.5) * dx[a] for a in range(3)]


def _mesh(prob_n, dx, origin):
    xs = _centres(prob_n, dx, origin)
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return X, Y, Z


def normal_shock_state(M, gamma, rho1, p1):
    """Post-shock (rho, u, p) of a shock of Mach M running into gas at rest."""
    g = gamma
    c1 = math.sqrt(g * p1 / rho1)
    p2 = p1 * (1.0 + 2.0 * g / (g + 1.0) * (M * M - 1.0))
    rho2 = rho1 * (g + 1.0) * M * M / ((g - 1.0) * M * M + 2.0)
    S = M * c1
    u2 = S * (1.0 - rho1 / rho2)
    return rho2, u2, p2


def ellipse_sdf(X, Y, cx, cy, a, b, angle=0.0):
    """Approximate signed distance to an ellipse: (q - 1)/|grad q| with
    q = sqrt((x'/a)^2 + (y'/b)^2) in the body frame; exact on the contour."""
    ca, sa = math.cos(angle), math.sin(angle)
    xr = (X - cx) * ca + (Y - cy) * sa
    yr = -(X - cx) * sa + (Y - cy) * ca
    q = np.sqrt((xr / a) ** 2 + (yr / b) ** 2)
    qs = np.maximum(q, 1e-12)
    gx = xr / (a * a * qs)
    gy = yr / (b * b * qs)
    gn = np.sqrt(gx * gx + gy * gy)
    d = np.where(q > 1e-9, (q - 1.0) / np.maximum(gn, 1e-300), -min(a, b))
    return d


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def sod_wall(n=400, recon="muscl"):
    """1D Sod tube on [0,1] with a static rigid wall r = 1 for x > 0.85."""
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    W = np.zeros((4, 1, 1, n))
    left = x < 0.5
    W[0, 0, 0] = np.where(left, 1.0, 0.125)
    W[1, 0, 0] = 0.0
    W[2, 0, 0] = np.where(left, 1.0, 0.1)
    sdf = (0.85 - x).reshape(1, 1, n)
    return Problem(name="sod_wall", dim=1, n=(n, 1, 1), dx=(dx, 1.0, 1.0), origin=(0.0, 0.0, 0.0),
                   materials=[ideal(1.4)], solid=False, bc=["transmissive"] * 6, W0=W, sdf=sdf,
                   width=1.0, recon=recon, riemann="hllc", cfl=0.8, t_end=0.3)


def shock_cylinder(nx=1024, ny=512, mach=2.8, riemann="hllc_lm", recon="bvd_thinc", x_shock=0.15):
    """2D Mach 2.8 planar shock (gamma 1.4, pre-shock rho = 1, p = 1) over a
    static rigid cylinder of radius 0.1 at (0.3, 0.25) on [0,1] x [0,0.5]."""
    dx = 1.0 / nx
    dy = 0.5 / ny
    X, Y, _ = _mesh((nx, ny, 1), (dx, dy, 1.0), (0.0, 0.0, 0.0))
    rho2, u2, p2 = normal_shock_state(mach, 1.4, 1.0, 1.0)
    post = X < x_shock
    W = np.zeros((5, 1, ny, nx))
    W[0] = np.where(post, rho2, 1.0)
    W[1] = np.where(post, u2, 0.0)
    W[2] = 0.0
    W[3] = np.where(post, p2, 1.0)
    sdf = np.sqrt((X - 0.3) ** 2 + (Y - 0.25) ** 2) - 0.1
    inflow = np.array([rho2, u2, 0.0, p2, 0.0])
    return Problem(name="shock_cylinder", dim=2, n=(nx, ny, 1), dx=(dx, dy, 1.0), origin=(0.0, 0.0, 0.0),
                   materials=[ideal(1.4)], solid=False,
                   bc=["dirichlet", "transmissive", "reflective", "reflective", "transmissive", "transmissive"],
                   bc_states={0: inflow}, W0=W, sdf=sdf, width=1.0, recon=recon, riemann=riemann,
                   cfl=0.4, t_end=0.3)


def wedge(nx=1200, ny=800, mach=1.7, angle_deg=25.0, x_wedge=0.5, x_shock=0.25, normal="elvira",
          recon="bvd_thinc", riemann="hllc"):
    """2D planar shock (gamma 1.4; quiescent rho = 1.4, p = 1) on [0,3] x
    [0,2] reflecting from a static rigid wedge: the region below the line
    through (x_wedge, 0) at angle_deg to the x axis. The default grid is the
    finest level of a 300 x 200 base grid with two refinements by 2, as a
    uniform grid. Mach 1.7 / 25 degrees runs to t = 1.2, Mach 10 / 30
    degrees to t = 0.2."""
    dx = 3.0 / nx
    dy = 2.0 / ny
    X, Y, _ = _mesh((nx, ny, 1), (dx, dy, 1.0), (0.0, 0.0, 0.0))
    rho2, u2, p2 = normal_shock_state(mach, 1.4, 1.4, 1.0)
    post = X < x_shock
    W = np.zeros((5, 1, ny, nx))
    W[0] = np.where(post, rho2, 1.4)
    W[1] = np.where(post, u2, 0.0)
    W[2] = 0.0
    W[3] = np.where(post, p2, 1.0)
    th = math.radians(angle_deg)
    sdf = math.cos(th) * Y - math.sin(th) * (X - x_wedge)   # distance to the ramp line
    inflow = np.array([rho2, u2, 0.0, p2, 0.0])
    return Problem(name="wedge", dim=2, n=(nx, ny, 1), dx=(dx, dy, 1.0), origin=(0.0, 0.0, 0.0),
                   materials=[ideal(1.4)], solid=False,
                   bc=["dirichlet", "transmissive", "reflective", "transmissive", "transmissive", "transmissive"],
                   bc_states={0: inflow}, W0=W, sdf=sdf, width=1.0, recon=recon, riemann=riemann,
                   normal=normal, cfl=0.4, t_end=1.2 if mach < 5 else 0.2)


def air_water(nx=2048, ny=1024, eps=1e-6):
    """2D air/water (both stiffened gases) with a rigid ellipse (semi-axes
    0.08 x 0.04 m at (0.25, 0.25) m) moving at 100 m/s towards a water column
    x in [0.45, 0.65] m; p = 1e5 Pa, at rest; SI units on [0,1] x [0,0.5] m."""
    dx = 1.0 / nx
    dy = 0.5 / ny
    X, Y, _ = _mesh((nx, ny, 1), (dx, dy, 1.0), (0.0, 0.0, 0.0))
    dcol = np.maximum(0.45 - X, X - 0.65)   # negative inside the column
    phi_w = eps + (1.0 - 2.0 * eps) * 0.5 * (1.0 - np.tanh(dcol / dx))
    phi_air = 1.0 - phi_w
    W = np.zeros((7, 1, ny, nx))
    W[0] = phi_air
    W[1] = 1.2
    W[2] = 1000.0
    W[3] = 0.0
    W[4] = 0.0
    W[5] = 1.0e5
    sdf = ellipse_sdf(X, Y, 0.25, 0.25, 0.08, 0.04)
    return Problem(name="air_water", dim=2, n=(nx, ny, 1), dx=(dx, dy, 1.0), origin=(0.0, 0.0, 0.0),
                   materials=[stiffened(1.4, 0.0), stiffened(4.4, 6.0e8)], solid=False,
                   bc=["transmissive"] * 6, W0=W, sdf=sdf, width=1.0, v_r=(100.0, 0.0, 0.0),
                   center=(0.25, 0.25, 0.0), recon="bvd_thinc", riemann="hllc", cfl=0.4, t_end=4.8e-3)


def copper_indenter(n=256, eps=1e-6, L=25.6e-3, gap=None):
    """3D copper block (z < L/2, Romenskii, rho0 8930, G0 46 GPa, perfect
    plasticity 0.12 GPa) under air, with a flat-ended rigid cylinder (axis z at
    the centre, radius 20/256 of the side) moving at -200 m/s along z. The flat
    end starts `gap` above the copper surface (default L/256 = 0.1 mm; a
    negative gap starts it that far inside the copper, in contact)."""
    h = L / n
    X, Y, Z = _mesh((n, n, n), (h, h, h), (0.0, 0.0, 0.0))
    cu = dict(TABLE1["copper"])
    cu.update(rho0=8930.0, G0=46.0e9)
    zc = 0.5 * L
    phi_cu = eps + (1.0 - 2.0 * eps) * 0.5 * (1.0 - np.tanh((Z - zc) / h))
    nf = 2 * 2 + 3 + 1 + 10
    W = np.zeros((nf, n, n, n))
    W[0] = phi_cu            # phi_Cu
    W[1] = cu["rho0"]        # rho_Cu
    W[2] = 1.2               # rho_air
    W[3:6] = 0.0             # u
    W[6] = 1.0e5             # p
    for a in range(3):
        W[7 + 4 * a] = 1.0   # Vbar = I
    W[16] = 0.0              # eps_p
    R = L * 20.0 / 256.0
    z_end = zc + (L / 256.0 if gap is None else gap)
    rad = np.sqrt((X - 0.5 * L) ** 2 + (Y - 0.5 * L) ** 2)
    sdf = np.maximum(rad - R, z_end - Z)
    mats = [romenskii(cu["rho0"], cu["K0"], cu["G0"], cu["alpha"], cu["beta"], cu["Gamma0"], 0.12e9),
            ideal(1.4)]
    return Problem(name="copper_indenter", dim=3, n=(n, n, n), dx=(h, h, h), origin=(0.0, 0.0, 0.0),
                   materials=mats, solid=True,
                   bc=["transmissive", "transmissive", "transmissive", "transmissive", "reflective",
                       "transmissive"],
                   W0=W, sdf=sdf, width=1.0, v_r=(0.0, 0.0, -200.0), center=(0.5 * L, 0.5 * L, z_end),
                   recon="bvd_thinc", riemann="hllc", cfl=0.3, t_end=2.5e-6)


def extrusion(nx=2048, ny=1728, eps=1e-6, x_block=100e-3, box_cells=12):
    """2D extrusion of an aluminium block by a piston through a rigid wedge
    (Sec. 4.5): x in [-21, 120] mm, y in [0, 120] mm, reflective walls at
    y = 0 and y = 120 mm, transmissive x faces. Aluminium of Table 1 with
    perfect plasticity at 0.2976 GPa fills the channel from the piston to
    x = x_block (air, gamma 1.4, beyond), at rest, p = 1e5 Pa. Two rigid
    bodies share the r field (union of signed distances): body 0 the static
    wedge, the region below the line from (0, 0) at 15 degrees to the x
    axis; body 1 the piston x < -20 mm, moving at 100 m/s along x, owning
    the points left of box_cells cells in front of its face (the box moves
    with it). The default grid is the finest level of the 256 x 216 base
    grid with three refinements by 2, as a uniform grid; t_end = 20 us,
    CFL 0.4."""
    x0, x1, y1 = -21e-3, 120e-3, 120e-3
    dx = (x1 - x0) / nx
    dy = y1 / ny
    X, Y, _ = _mesh((nx, ny, 1), (dx, dy, 1.0), (x0, 0.0, 0.0))
    al = TABLE1["aluminium"]
    phi_al = eps + (1.0 - 2.0 * eps) * 0.5 * (1.0 - np.tanh((X - x_block) / dx))
    W = np.zeros((17, 1, ny, nx))
    W[0] = phi_al            # phi_Al
    W[1] = al["rho0"]        # rho_Al
    W[2] = 1.2               # rho_air
    W[3:5] = 0.0             # u, v
    W[5] = 1.0e5             # p
    for a in range(3):
        W[6 + 4 * a] = 1.0   # Vbar = I
    W[15] = 0.0              # eps_p
    th = math.radians(15.0)
    x_piston = -20e-3
    sdf_wedge = math.cos(th) * Y - math.sin(th) * X
    sdf_piston = X - x_piston
    sdf = np.minimum(sdf_wedge, sdf_piston)
    inf = math.inf
    piston = dict(v=(100.0, 0.0, 0.0), omega=(0.0, 0.0, 0.0), center=(x_piston, 0.5 * y1, 0.0),
                  box_lo=(-inf, -inf, -inf), box_hi=(x_piston + box_cells * min(dx, dy), inf, inf))
    mats = [romenskii(al["rho0"], al["K0"], al["G0"], al["alpha"], al["beta"], al["Gamma0"], 0.2976e9),
            ideal(1.4)]
    return Problem(name="extrusion", dim=2, n=(nx, ny, 1), dx=(dx, dy, 1.0), origin=(x0, 0.0, 0.0),
                   materials=mats, solid=True,
                   bc=["transmissive", "transmissive", "reflective", "reflective", "transmissive", "transmissive"],
                   W0=W, sdf=sdf, width=1.0, v_r=(0.0, 0.0, 0.0), center=(0.0, 0.0, 0.0), bodies=(piston,),
                   recon="bvd_thinc", riemann="hllc", cfl=0.4, t_end=20e-6)


def batch(count=64, seed=2111, nmin=128, nmax=512, steps=200):
    """Seeded batch of 2D ideal-gas shock / rigid-ellipse instances.

    numpy default_rng(seed); per instance, in order: nx, ny ~ U{nmin..nmax};
    Mach ~ U[1.5, 3.0]; n_bodies ~ U{1..4}; per body: centre x ~ U[0.3, 0.85],
    y ~ U[0.15, 0.85] H, semi-axis a ~ U[0.03, 0.10], b ~ U[0.3 a, a], angle
    ~ U[0, pi). Domain [0,1] x [0, H = ny/nx], dx = 1/nx, quiescent (1,0,0,1),
    shock at x = 0.1, boundaries as the cylinder workload."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nx = int(rng.integers(nmin, nmax + 1))
        ny = int(rng.integers(nmin, nmax + 1))
        mach = float(rng.uniform(1.5, 3.0))
        nb = int(rng.integers(1, 5))
        H = ny / nx
        bodies = []
        for _ in range(nb):
            cx = float(rng.uniform(0.3, 0.85))
            cy = float(rng.uniform(0.15, 0.85)) * H
            a = float(rng.uniform(0.03, 0.10))
            b = float(rng.uniform(0.3 * a, a))
            ang = float(rng.uniform(0.0, math.pi))
            bodies.append((cx, cy, a, b, ang))
        dx = 1.0 / nx
        X, Y, _ = _mesh((nx, ny, 1), (dx, dx, 1.0), (0.0, 0.0, 0.0))
        rho2, u2, p2 = normal_shock_state(mach, 1.4, 1.0, 1.0)
        post = X < 0.1
        W = np.zeros((5, 1, ny, nx))
        W[0] = np.where(post, rho2, 1.0)
        W[1] = np.where(post, u2, 0.0)
        W[3] = np.where(post, p2, 1.0)
        sdf = np.min(np.stack([ellipse_sdf(X, Y, *bd) for bd in bodies]), axis=0)
        p = Problem(name=f"batch{k}", dim=2, n=(nx, ny, 1), dx=(dx, dx, 1.0), origin=(0.0, 0.0, 0.0),
                    materials=[ideal(1.4)], solid=False,
                    bc=["dirichlet", "transmissive", "reflective", "reflective", "transmissive", "transmissive"],
                    bc_states={0: np.array([rho2, u2, 0.0, p2, 0.0])}, W0=W, sdf=sdf, width=1.0,
                    recon="bvd_thinc", riemann="hllc_lm", cfl=0.4, t_end=1e9)
        out.append(p)
    return out


# ---------------------------------------------------------------------------
# Verification problems
# ---------------------------------------------------------------------------

def riemann_1d(left, right, materials, n=400, x0=0.5, length=1.0, t_end=0.2, cfl=0.5,
               recon="muscl", riemann="hllc", nfields=None):
    """1D shock tube with primitive left/right states (full W vectors without r)."""
    dx = length / n
    x = (np.arange(n) + 0.5) * dx
    left = np.asarray(left, float)
    right = np.asarray(right, float)
    nf = len(left) + 1
    W = np.zeros((nf, 1, 1, n))
    for q in range(nf - 1):
        W[q, 0, 0] = np.where(x < x0, left[q], right[q])
    return Problem(name="riemann", dim=1, n=(n, 1, 1), dx=(dx, 1.0, 1.0), origin=(0.0, 0.0, 0.0),
                   materials=materials, solid=False, bc=["transmissive"] * 6, W0=W, recon=recon,
                   riemann=riemann, cfl=cfl, t_end=t_end, seed="none")


def piston_1d(n=400, v_p=1.0, x_p=0.2, t_end=0.3, recon="muscl"):
    """Rigid piston (body x < x_p) moving at v_p into gas at rest (1, 0, 1)."""
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    W = np.zeros((4, 1, 1, n))
    W[0] = 1.0
    W[2] = 1.0
    sdf = (x - x_p).reshape(1, 1, n)
    return Problem(name="piston", dim=1, n=(n, 1, 1), dx=(dx, 1.0, 1.0), origin=(0.0, 0.0, 0.0),
                   materials=[ideal(1.4)], solid=False, bc=["transmissive"] * 6, W0=W, sdf=sdf, width=1.0,
                   v_r=(v_p, 0.0, 0.0), center=(x_p, 0.0, 0.0), recon=recon, riemann="hllc", cfl=0.5,
                   t_end=t_end)


def piston_channel(nx=64, ny=8, tilt=1e-12, v_p=1.0, x_p=0.2):
    """A flat rigid piston (body x < x_p + tilt y) moving at v_p into gas at
    rest (1, 0, 1) along a channel with reflective walls (a 1D flow); the
    tiny tilt turns the body normal toward the lower wall at rounding
    level."""
    dx = 1.0 / nx
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(x, y)
    W = np.zeros((5, 1, ny, nx))
    W[0] = 1.0
    W[3] = 1.0
    sdf = (X - x_p - tilt * Y).reshape(1, ny, nx)
    return Problem(name="piston_channel", dim=2, n=(nx, ny, 1), dx=(dx, dx, dx), origin=(0.0, 0.0, 0.0),
                   materials=[ideal(1.4)], solid=False,
                   bc=["transmissive", "transmissive", "reflective", "reflective", "transmissive", "transmissive"],
                   W0=W, sdf=sdf, width=1.0, v_r=(v_p, 0.0, 0.0), center=(x_p, 0.0, 0.0), recon="muscl",
                   riemann="hllc", cfl=0.5)


def piston_wall_1d(n=800, v_p=1.0, x_p=0.2, x_w=0.8, t_end=0.4, box_cells=20, recon="muscl"):
    """Gas at rest (1, 0, 1) between two rigid bodies with their own motion:
    a piston x < x_p moving at v_p (body 1, owning the points behind its box
    face box_cells cells ahead of it) and a static wall x > x_w (body 0)."""
    p = piston_1d(n, v_p=v_p, x_p=x_p, t_end=t_end, recon=recon)
    x = (np.arange(n) + 0.5) / n
    p.name = "piston_wall"
    p.sdf = np.minimum(x - x_p, x_w - x).reshape(1, 1, n)
    p.v_r, p.center = (0.0, 0.0, 0.0), (x_w, 0.0, 0.0)
    p.bodies = (dict(v=(v_p, 0.0, 0.0), omega=(0.0, 0.0, 0.0), center=(x_p, 0.0, 0.0),
                     box_lo=(-math.inf,) * 3, box_hi=(x_p + box_cells / n, math.inf, math.inf)),)
    return p


def quiescent_body(nx=64, ny=48, recon="bvd_thinc", riemann="hllc", seed="original"):
    """Gas at rest around a static rigid ellipse, reflective walls."""
    dx = 1.0 / nx
    X, Y, _ = _mesh((nx, ny, 1), (dx, dx, 1.0), (0.0, 0.0, 0.0))
    W = np.zeros((5, 1, ny, nx))
    W[0] = 1.4
    W[3] = 1.0
    sdf = ellipse_sdf(X, Y, 0.45, 0.5 * ny * dx, 0.2, 0.12, 0.3)
    return Problem(name="quiescent", dim=2, n=(nx, ny, 1), dx=(dx, dx, 1.0), origin=(0.0, 0.0, 0.0),
                   materials=[ideal(1.4)], solid=False, bc=["reflective"] * 6, W0=W, sdf=sdf, width=1.0,
                   recon=recon, riemann=riemann, seed=seed, cfl=0.4, t_end=1.0)


def periodic_box(dim=2, n=32, nmat=1, seed=7, recon="bvd_thinc", riemann="hllc"):
    """Smooth random periodic state without rigid bodies (r = 0)."""
    rng = np.random.default_rng(seed)
    shape = (n if dim > 2 else 1, n if dim > 1 else 1, n)
    dx = 1.0 / n
    X, Y, Z = _mesh((n, shape[1], shape[0]), (dx, dx, dx), (0.0, 0.0, 0.0))
    def smooth():
        a = rng.uniform(-1, 1, 3)
        return a[0] * np.sin(2 * np.pi * X + a[1]) + a[2] * np.cos(2 * np.pi * (Y + Z) + a[0])
    if nmat == 1:
        mats = [ideal(1.4)]
    else:
        mats = [stiffened(1.4, 0.0), stiffened(4.4, 6.0)]
    nf = 2 * nmat + dim + 1
    W = np.zeros((nf,) + shape)
    q = 0
    if nmat == 2:
        W[q] = 0.5 + 0.3 * np.tanh(3 * smooth()); q += 1
        W[q] = 1.0 + 0.2 * smooth(); q += 1
        W[q] = 3.0 + 0.5 * smooth(); q += 1
    else:
        W[q] = 1.0 + 0.3 * np.tanh(smooth()); q += 1
    for a in range(dim):
        W[q] = 0.3 * smooth(); q += 1
    W[q] = 1.0 + 0.2 * np.tanh(smooth()); q += 1
    W[q] = 0.0
    return Problem(name="periodic", dim=dim, n=(n, shape[1], shape[0]), dx=(dx, dx, dx), origin=(0.0, 0.0, 0.0),
                   materials=mats, solid=False, bc=["periodic"] * 6, W0=W, recon=recon, riemann=riemann,
                   seed="none", cfl=0.4, t_end=1.0)


def copper_piston_1d(n=400, v_p=30.0, length=10e-3, x_p=1e-3, eps=1e-6, t_end=1.2e-6, sigY=0.12e9):
    """1D copper (Romenskii, rho0 8930, G0 46 GPa, perfect plasticity) driven
    by a rigid piston (body x < x_p) moving at v_p; air as the second phase
    with a negligible volume fraction."""
    h = length / n
    x = (np.arange(n) + 0.5) * h
    cu = dict(TABLE1["copper"])
    cu.update(rho0=8930.0, G0=46.0e9)
    nf = 2 * 2 + 1 + 1 + 10
    W = np.zeros((nf, 1, 1, n))
    W[0] = 1.0 - eps     # phi_Cu
    W[1] = cu["rho0"]
    W[2] = 1.2
    W[3] = 0.0
    W[4] = 1.0e5
    for a in range(3):
        W[5 + 4 * a] = 1.0
    W[14] = 0.0
    sdf = (x - x_p).reshape(1, 1, n)
    mats = [romenskii(cu["rho0"], cu["K0"], cu["G0"], cu["alpha"], cu["beta"], cu["Gamma0"], sigY), ideal(1.4)]
    return Problem(name="copper_piston", dim=1, n=(n, 1, 1), dx=(h, 1.0, 1.0), origin=(0.0, 0.0, 0.0),
                   materials=mats, solid=True, bc=["transmissive"] * 6, W0=W, sdf=sdf, width=1.0,
                   v_r=(v_p, 0.0, 0.0), center=(x_p, 0.0, 0.0), recon="muscl", riemann="hllc", cfl=0.4,
                   t_end=t_end)


def copper_slab_wall(n=600, v=-20.0, length=12e-3, x_w=1e-3, slab=6e-3, eps=1e-6, t_end=4.0e-6,
                     face_mod=True, plastic=False, dim=1, axis=0, ntrans=4, wall_v=0.0):
    """Elastic copper slab (Romenskii, rho0 8930, G0 46 GPa; plasticity off by
    default) of thickness `slab` across axis `axis`, touching a static rigid
    wall (body at coordinate < x_w along that axis) and moving into it at
    v < 0; air around it. n cells along the axis, ntrans along the other
    axes of a 2D or 3D grid (periodic there). With the void-opening face
    modifier the slab leaves the wall when the reflected release wave reaches
    it (after 2 slab / c_L, c_L the longitudinal wave speed), at -v; without
    it the wall holds the slab in tension. wall_v: the wall's velocity along
    the axis (negative: it moves away from the slab)."""
    h = length / n
    shape = [1, 1, 1]  # nx, ny, nz
    for e in range(dim):
        shape[e] = n if e == axis else ntrans
    x = (np.arange(n) + 0.5) * h
    cu = dict(TABLE1["copper"])
    cu.update(rho0=8930.0, G0=46.0e9)
    nf = 2 * 2 + dim + 1 + 10
    prof = 0.5 * (np.tanh((x - x_w) / h) - np.tanh((x - x_w - slab) / h))
    bshape = [1, 1, 1]  # z, y, x order of the arrays
    bshape[2 - axis] = n
    ind = np.broadcast_to(prof.reshape(bshape), (shape[2], shape[1], shape[0]))
    W = np.zeros((nf, shape[2], shape[1], shape[0]))
    W[0] = eps + (1.0 - 2.0 * eps) * ind   # phi_Cu
    W[1] = cu["rho0"]
    W[2] = 1.2
    W[3 + axis] = v * ind
    W[3 + dim] = 1.0e5
    for a in range(3):
        W[4 + dim + 4 * a] = 1.0
    gap = np.zeros(nf)
    gap[0], gap[1], gap[2], gap[3 + dim] = eps, cu["rho0"], 1.2, 1.0e5
    for a in range(3):
        gap[4 + dim + 4 * a] = 1.0
    sdf = np.broadcast_to((x - x_w).reshape(bshape), ind.shape).copy()
    mats = [romenskii(cu["rho0"], cu["K0"], cu["G0"], cu["alpha"], cu["beta"], cu["Gamma0"], 0.12e9), ideal(1.4)]
    bc = ["periodic"] * 6
    bc[2 * axis] = bc[2 * axis + 1] = "transmissive"
    center = [0.0, 0.0, 0.0]
    center[axis] = x_w
    vr = [0.0, 0.0, 0.0]
    vr[axis] = wall_v
    return Problem(name="copper_slab_wall", dim=dim, n=tuple(shape), dx=(h, h, h) if dim > 1 else (h, 1.0, 1.0),
                   origin=(0.0, 0.0, 0.0), materials=mats, solid=True, bc=bc, W0=W, sdf=sdf, width=1.0,
                   v_r=tuple(vr), center=tuple(center), gap_gas=gap if face_mod else None,
                   recon="muscl", riemann="hllc", plastic=plastic, cfl=0.4, t_end=t_end)


def longitudinal_wave_speed(m):
    """sqrt((K0 + 4/3 G0) / rho0) of a Romenskii material at its reference
    state: the elastic wave speed of uniaxial strain."""
    return float(np.sqrt((m["K0"] + 4.0 / 3.0 * m["G0"]) / m["rho0"]))
