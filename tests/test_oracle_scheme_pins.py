"""Pins of three oracle parts that the exact-solution pins do not reach (no GPU).

* ``Oracle::bvd_select`` (Sec. 3.1, the BVD choice between the MUSCL and
  THINC candidates): hand-computed total-boundary-variation cases, and the
  end-to-end property the selection exists for -- a contact discontinuity
  advected once around a periodic box stays sharper, and closer to the exact
  translated profile, than with MUSCL alone.
* ``Oracle::hllc`` in its low-Mach form (Sec. 4.3, HLLC-LM): the numerical
  pressure dissipation of a symmetric compression face scales with the Mach
  number for HLLC and with its square below the Mach limit for HLLC-LM.
* ``Oracle::riemann_seed`` (Sec. 3.2, the Riemann variant of the seeding
  state): the star state against linear acoustics (impedance rho c) in the
  limit of a small wall-normal speed, against the exact Riemann solution at
  moderate speeds, and the stretch tensor against the kinematics of a
  uniaxial compression.
* ``Oracle::rigid_force`` torque and the r update under a rotating rigid
  motion (Sec. 2.3 v_r = v + omega x (x - c), Sec. 3.1 r terms): exact
  summation-by-parts identities for uniform and linear pressure, sum r dV
  conserved and the centroid carried at v while the body turns.
"""
import math

import numpy as np
import pytest

import exact_solutions as ex
import oracle
from geometry_util import ellipsoid_problem
from paper_2111_11806_amd import inputs

BETA = 1.6  # THINC steepness of every problem below (the inputs' default)


def _orc2d(riemann="hllc", recon="bvd_thinc"):
    p = inputs.shock_cylinder(16, 8, riemann=riemann, recon=recon)
    assert p.thinc_beta == BETA
    return oracle.Oracle(p)


# ---------------------------------------------------------------------------
# BVD selection (Oracle::candidates + Oracle::bvd_select)
# ---------------------------------------------------------------------------

def _select_on_profile(o, q, i):
    """Faces BVD selects for cell i of the 1D profile q (needs i-2 .. i+2)."""
    cand = [o.candidates(q[j - 1], q[j], q[j + 1]) for j in (i - 1, i, i + 1)]
    return o.bvd_select(*cand)


def test_bvd_selects_thinc_on_a_smeared_step():
    """q = 0, 0, 1/2, 1, 1: the middle cell is strictly monotone, its
    neighbours are not (both their candidates are the cell value). MUSCL
    faces 1/4, 3/4 give TBV = 1/2; the THINC profile centred in the cell
    (C = 1/2) has faces (1 -/+ tanh(beta/2))/2, TBV = 1 - tanh(beta/2) < 1/2:
    BVD must take THINC."""
    o = _orc2d()
    q = [0.0, 0.0, 0.0, 0.5, 1.0, 1.0, 1.0]
    ql, qr = _select_on_profile(o, q, 3)
    th = math.tanh(0.5 * BETA)
    assert 1.0 - th < 0.5
    assert ql == pytest.approx(0.5 * (1.0 - th), abs=1e-15)
    assert qr == pytest.approx(0.5 * (1.0 + th), abs=1e-15)
    # mirror image: decreasing step, faces swap roles
    ql2, qr2 = _select_on_profile(o, q[::-1], 3)
    assert ql2 == pytest.approx(qr, abs=1e-15) and qr2 == pytest.approx(ql, abs=1e-15)


def test_bvd_keeps_muscl_on_a_linear_ramp():
    """On a linear profile the MUSCL faces are exact and continuous across
    every face (TBV = 0): no candidate can be strictly smaller, so BVD must
    keep MUSCL (faces q_i -/+ 1/2 slope)."""
    o = _orc2d()
    for slope in (1.0, -0.37):
        q = [2.0 + slope * k for k in range(7)]
        ql, qr = _select_on_profile(o, q, 3)
        assert ql == pytest.approx(q[3] - 0.5 * slope, abs=1e-14)
        assert qr == pytest.approx(q[3] + 0.5 * slope, abs=1e-14)


def test_bvd_hand_built_candidates():
    """Candidate quadruples (MUSCL left, MUSCL right, THINC left, THINC right)
    chosen so that each possible slip changes the answer: the TBV compares the
    left neighbour's RIGHT face with the cell's left face and the cell's right
    face with the right neighbour's LEFT face, scheme by scheme; THINC only
    when strictly smaller (a tie keeps MUSCL). All values are exact in
    binary."""
    o = _orc2d()
    big = 100.0  # faces that must not enter the comparison
    c0 = [1.0, 2.0, 1.25, 1.75]
    # TBV_M = |1 - 1| + |2 - 2.5| = 0.5, TBV_T = |1.25 - 1.25| + |1.75 - 1.75| = 0 -> THINC
    cm = [big, 1.0, -big, 1.25]
    cp = [2.5, -big, 1.75, big]
    assert list(o.bvd_select(cm, c0, cp)) == [1.25, 1.75]
    # TBV_M = 0, TBV_T = 0 + |1.75 - 2.5| -> MUSCL
    cp = [2.0, -big, 2.5, big]
    assert list(o.bvd_select(cm, c0, cp)) == [1.0, 2.0]
    # tie: TBV_M = |0 - 1| + |1 - 1| = 1 = TBV_T = |0 - 0.5| + |0.5 - 1| -> MUSCL
    assert list(o.bvd_select([big, 0.0, big, 0.0], [1.0, 1.0, 0.5, 0.5], [1.0, big, 1.0, big])) == [1.0, 1.0]
    # a hair below the tie on the THINC side -> THINC
    assert list(o.bvd_select([big, 0.0, big, 0.0], [1.0, 1.0, 0.5, 0.5],
                             [1.0, big, 0.9990234375, big])) == [0.5, 0.5]
    # MUSCL-only reconstruction never selects the THINC faces
    om = _orc2d(recon="muscl")
    assert list(om.bvd_select(cm, c0, [2.5, -big, 1.75, big])) == [1.0, 2.0]


def _advect_square_wave(recon, n=100):
    """Density square wave (1 outside, 2 inside [0.3, 0.6)) carried by
    u = 1, p = 1 once around the periodic unit interval."""
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    rho0 = np.where((x >= 0.3) & (x < 0.6), 2.0, 1.0)
    W = np.zeros((4, 1, 1, n))
    W[0, 0, 0] = rho0
    W[1] = 1.0
    W[2] = 1.0
    prob = inputs.Problem(name="advect", dim=1, n=(n, 1, 1), dx=(dx, 1.0, 1.0), origin=(0.0, 0.0, 0.0),
                          materials=[inputs.ideal(1.4)], solid=False, bc=["periodic"] * 6, W0=W,
                          recon=recon, riemann="hllc", cfl=0.4, t_end=1.0, seed="none")
    o = oracle.Oracle(prob)
    o.run(t_end=1.0, cfl=0.4)
    Wp = o.get_state_prim()
    return rho0, Wp[0, 0, 0], Wp[1, 0, 0], Wp[2, 0, 0]


def _jump_widths(rho):
    """Cells strictly between 5% and 95% of the jump, around each of the two
    discontinuities (x = 0.3 and x = 0.6 on 100 cells)."""
    s = (rho - 1.0) / 1.0
    mid = (s > 0.05) & (s < 0.95)
    return int(mid[15:45].sum()), int(mid[45:75].sum())


def test_bvd_thinc_keeps_an_advected_contact_sharp():
    """The purpose of the selection (Sec. 3.1): after one period the BVD-THINC
    profile is closer to the exact (initial) profile in L1 than MUSCL's and
    each jump spans at most 3 cells, where MUSCL smears it over several more.
    Velocity and pressure stay uniform in both (contact preservation)."""
    exact, rb, ub, pb = _advect_square_wave("bvd_thinc")
    _, rm, um, pm = _advect_square_wave("muscl")
    eb = np.abs(rb - exact).mean()
    em = np.abs(rm - exact).mean()
    wb, wm = _jump_widths(rb), _jump_widths(rm)
    print("L1 bvd %.4f muscl %.4f, widths bvd %s muscl %s" % (eb, em, wb, wm))
    assert eb < 0.5 * em
    assert max(wb) <= 3 and min(wm) >= 2 * max(wb)
    for u, p in ((ub, pb), (um, pm)):
        assert np.abs(u - 1.0).max() < 1e-12 and np.abs(p - 1.0).max() < 1e-12
    # mass is conserved exactly (periodic)
    assert abs(rb.sum() - exact.sum()) < 1e-12 * exact.sum()


# ---------------------------------------------------------------------------
# HLLC-LM low-Mach ramp (Oracle::hllc with riemann = HLLC-LM)
# ---------------------------------------------------------------------------

def _pressure_dissipation(o, eps, v_t=0.0):
    """Symmetric compression face u_L = -u_R = eps c (rho = p = 1): the
    normal-momentum flux minus the central average of the physical fluxes,
    i.e. the scheme's numerical pressure."""
    c = math.sqrt(1.4)
    WL = np.array([1.0, eps * c, v_t, 1.0, 0.0])
    WR = np.array([1.0, -eps * c, v_t, 1.0, 0.0])
    F, us, _ = o.face_flux(WL, WR, 0)
    avg = 0.5 * (o.phys_flux(WL, 0) + o.phys_flux(WR, 0))
    assert abs(us) < 1e-15 and abs(F[0]) < 1e-15  # symmetric: no mass flux, wall at rest
    return F[1] - avg[1]


def test_hllc_lm_pressure_dissipation_scales_with_mach_squared():
    """Below the Mach limit the low-Mach correction (Sec. 4.3) must reduce the
    acoustic dissipation from O(Ma) to O(Ma^2): for eps in [1e-4, 1e-2] the
    log-log slope of the numerical pressure is 1 with HLLC and 2 with
    HLLC-LM; above the limit both fluxes coincide. The Mach number is that of
    the face-normal velocity: a tangential stream does not switch the
    correction off."""
    oh, ol = _orc2d("hllc"), _orc2d("hllc_lm")
    eps = np.array([1e-4, 1e-3, 1e-2])
    dh = np.array([_pressure_dissipation(oh, e) for e in eps])
    dl = np.array([_pressure_dissipation(ol, e) for e in eps])
    assert np.all(dh > 0) and np.all(dl > 0)
    sh = np.diff(np.log(dh)) / np.diff(np.log(eps))
    sl = np.diff(np.log(dl)) / np.diff(np.log(eps))
    print("slopes hllc", sh, "hllc_lm", sl)
    assert np.all(np.abs(sh - 1.0) < 0.01)
    assert np.all(np.abs(sl - 2.0) < 0.01)
    # HLLC: the acoustic dissipation rho c^2 eps (1 + eps) of the symmetric face
    assert dh[0] == pytest.approx(1.4 * 1e-4 * (1 + 1e-4), rel=1e-9)
    # tangential stream at Mach 0.5: same dissipation
    for e in eps:
        assert _pressure_dissipation(ol, e, v_t=0.5 * math.sqrt(1.4)) == pytest.approx(
            _pressure_dissipation(ol, e), rel=1e-12)
    # at and above the limit the correction is off
    for e in (0.1, 0.3):
        assert _pressure_dissipation(ol, e) == pytest.approx(_pressure_dissipation(oh, e), rel=1e-12)


# ---------------------------------------------------------------------------
# Riemann seeding state (Oracle::riemann_seed)
# ---------------------------------------------------------------------------

def _seed_case(o, w, n, v=(0.0, 0.0, 0.0), tangential=0.3):
    """Fluid state moving toward the wall (normal speed -w along the outward
    normal n) with a tangential component; returns (W, seeded state)."""
    t = np.array([-n[1], n[0], 0.0])
    u = -w * n + tangential * t
    W = np.array([1.0, u[0], u[1], 1.0, 0.3])
    Wm = o.mirror_state(W, n, np.asarray(v, float))
    return W, o.riemann_seed_state(Wm, W, n)


def test_riemann_seed_star_state_linear_acoustics_limit():
    """A wall that stops a fluid arriving at normal speed w raises the
    pressure by rho c w and the density by rho w / c to first order (linear
    acoustics): (p* - p)/(rho c w) -> 1 and (rho*/rho - 1)/(w/c) -> 1 with
    an error O(w/c), for compression and expansion alike."""
    o = _orc2d()
    c = math.sqrt(1.4)
    rng = np.random.default_rng(21)
    for wc in (1e-2, 1e-3, 1e-4, 1e-5, -1e-3, -1e-5):
        th = rng.uniform(0, 2 * math.pi)
        n = np.array([math.cos(th), math.sin(th), 0.0])
        W, Ws = _seed_case(o, wc * c, n)
        rp = (Ws[3] - 1.0) / (1.0 * c * wc * c)
        rr = (Ws[0] / 1.0 - 1.0) / wc
        assert abs(rp - 1.0) <= 3.0 * abs(wc), (wc, rp)
        assert abs(rr - 1.0) <= 3.0 * abs(wc), (wc, rr)
        assert Ws[4] == W[4]  # r is not a seeded quantity


def test_riemann_seed_star_state_against_exact_riemann_solution():
    """At moderate wall-normal speeds the seeded p* and rho* follow the exact
    solution of the symmetric Riemann problem (fluid against its mirror
    image) to within the O(w/c) error of the HLLC wave-speed estimates:
    relative error of p* - p and rho* - rho at most 2 w/c."""
    o = _orc2d()
    c = math.sqrt(1.4)
    n = np.array([0.6, 0.8, 0.0])
    for wc in (0.02, 0.05, 0.1, 0.2):
        w = wc * c
        _, Ws = _seed_case(o, w, n)
        # along n the mirror state is on the left (moving at +w), the fluid
        # on the right (moving at -w)
        L, R = ex.Side(1.0, w, 1.0), ex.Side(1.0, -w, 1.0)
        pst, ust = ex.star(L, R)
        assert abs(ust) < 1e-12
        rst = ex.star_density(R, pst, left=False)
        ep = abs((Ws[3] - 1.0) - (pst - 1.0)) / (pst - 1.0)
        er = abs((Ws[0] - 1.0) - (rst - 1.0)) / (rst - 1.0)
        print("w/c %.2f: p* seed %.6f exact %.6f; rho* seed %.6f exact %.6f" % (wc, Ws[3], pst, Ws[0], rst))
        assert ep <= 2.0 * wc and er <= 2.0 * wc


def test_riemann_seed_stretch_follows_uniaxial_compression():
    """Elastoplastic seeding: the stretch of the star state is the fluid-side
    stretch carried through the isochoric part of a uniaxial compression
    along n whose density ratio is the seeded one. From the stretch evolution
    (Sec. 2.1.1, the rate of Vbar is (L - tr(L)/3) Vbar), a velocity gradient
    L = a n n^T over a time gives Vbar* = exp(a (n n^T - I/3)) Vbar and
    rho*/rho = exp(-a); det Vbar is unchanged."""
    cu = inputs.romenskii(**inputs.TABLE1["copper"], sigY=0.12e9)
    W = np.zeros((17, 1, 1, 4))
    W[0] = 1.0 - 1e-6
    W[1] = cu["rho0"]
    W[2] = 1.2
    W[5] = 1e5
    for a in range(3):
        W[6 + 4 * a] = 1.0
    prob = inputs.Problem(name="unit", dim=2, n=(4, 1, 1), dx=(1.0, 1.0, 1.0), origin=(0, 0, 0),
                          materials=[cu, inputs.ideal(1.4)], solid=True, bc=["transmissive"] * 6, W0=W,
                          seed="riemann")
    o = oracle.Oracle(prob)
    rng = np.random.default_rng(3)
    for _ in range(10):
        th = rng.uniform(0, 2 * math.pi)
        n3 = np.array([math.cos(th), math.sin(th), 0.0])
        Wi = W[:, 0, 0, 0].copy()
        Wi[3:5] = -30.0 * n3[:2] + rng.normal(size=2)
        V = np.eye(3) + 1e-3 * rng.normal(size=(3, 3))
        V /= np.cbrt(np.linalg.det(V))
        Wi[6:15] = V.ravel()
        Wm = o.mirror_state(Wi, n3, np.zeros(3))
        Ws = o.riemann_seed_state(Wm, Wi, n3)
        chi = Ws[1] / Wi[1]  # density ratio of the solid phase
        assert chi > 1.0
        a = -math.log(chi)
        Nn = np.outer(n3, n3)
        w_, Q = np.linalg.eigh(a * (Nn - np.eye(3) / 3.0))
        E = Q @ np.diag(np.exp(w_)) @ Q.T
        Vs = Ws[6:15].reshape(3, 3)
        assert np.allclose(Vs, E @ V, rtol=0, atol=1e-13)
        assert np.linalg.det(Vs) == pytest.approx(np.linalg.det(V), rel=1e-13)
        assert Ws[2] / Wi[2] == pytest.approx(chi, rel=1e-13)  # every phase compresses alike


# ---------------------------------------------------------------------------
# Rigid motion with rotation (Sec. 2.3: v_r = v + omega x (x - c)) and the
# torque of the force reading (Oracle::rigid_force, Oracle::rhs r terms)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_torque_of_uniform_and_linear_pressure(dim):
    """The force reading F = sum -sigma . grad_h r dV with its torque
    T = sum (x - c) x (-sigma . grad_h r) dV about any centre c: for a
    uniform pressure both vanish; for p = a + b . x, summation by parts
    (central differences, r vanishing near the boundary) gives exactly
    F = -b sum r dV and T = -(sum r (x - c) dV) x b (the load of a
    hydrostatic gradient acts at the body's r-weighted centroid)."""
    n = 48 if dim == 2 else 28
    shape = (1, n, n) if dim == 2 else (n, n, n)
    W = np.zeros((3 + dim, *shape))
    W[0] = 1.0
    prob, (X, Y, Z), dx = ellipsoid_problem(dim, n, W, bc="transmissive")
    dV = dx ** dim
    c = np.array([0.31, 0.62, 0.4 if dim == 3 else 0.0])
    for b in (np.zeros(3), np.array([0.7, -0.3, 0.45 if dim == 3 else 0.0])):
        W[1 + dim] = 2.0 + b[0] * X + b[1] * Y + (b[2] * Z if dim == 3 else 0.0)
        prob.W0 = W
        o = oracle.Oracle(prob)
        F, T = o.rigid_force(c)
        r = o.get_state_prim()[-1]
        M0 = r.sum() * dV
        M1 = np.array([(r * (X - c[0])).sum(), (r * (Y - c[1])).sum(),
                       (r * (Z - c[2])).sum() if dim == 3 else 0.0]) * dV
        scale = 2.0 * M0 / dx
        assert np.allclose(F, -b * M0, rtol=0, atol=1e-10 * scale), (F, -b * M0)
        assert np.allclose(T, -np.cross(M1, b), rtol=0, atol=1e-10 * scale), (T, -np.cross(M1, b))
        if not b.any():
            assert np.abs(F).max() < 1e-10 * scale and np.abs(T).max() < 1e-10 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_rotating_translating_body_conserves_r(dim):
    """A rigid motion v + omega x (x - c) has zero divergence, and its
    component along a sweep does not vary along that sweep: the face
    velocities of a row are equal, the non-conservative r term vanishes and
    the upwind r fluxes telescope, so sum r dV is conserved to rounding in a
    periodic box while the body turns and moves (Sec. 3.1 r update). The
    rotation is checked too: after the steps the body's r-weighted centroid
    has moved by v t."""
    n = 48 if dim == 2 else 24
    shape = (1, n, n) if dim == 2 else (n, n, n)
    W = np.zeros((3 + dim, *shape))
    W[0] = 1.0
    W[1 + dim] = 1.0
    omega = (0.0, 0.0, 3.0) if dim == 2 else (0.8, -1.1, 2.0)
    v = (0.3, -0.2, 0.0) if dim == 2 else (0.3, -0.2, 0.15)
    prob, (X, Y, Z), dx = ellipsoid_problem(dim, n, W, motion=(v, omega))
    o = oracle.Oracle(prob)
    r0 = o.conserved_totals()[0][-1]
    dt = 0.25 * dx / (1.0 + 0.5)
    nsteps = 40 if dim == 2 else 16
    for _ in range(nsteps):
        o.step(dt)
    r1 = o.conserved_totals()[0][-1]
    assert r1 == pytest.approx(r0, rel=1e-13), (r0, r1)
    r = o.get_state_prim()[-1]
    cen = np.array([(r * X).sum(), (r * Y).sum(), (r * Z).sum() if dim == 3 else 0.0]) / r.sum()
    expect = np.array(prob.center) + np.array(v) * dt * nsteps
    if dim == 2:
        expect[2] = 0.0
    assert np.allclose(cen, expect, atol=0.05 * dx), (cen, expect)
