"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Both sides start from the same seeded inputs and take the same dt sequence
(the oracle's CFL steps). Bars, per conserved field (parity_util.BARS):
relative L1 <= 1e-10 and relative Linf <= 1e-8 for FP64, 1e-4 and 5e-3 for
FP32, components of a vector or tensor judged against at least 1% of their
family's mean norm (parity_util.FLOOR); FP64 reductions (force, torque,
totals, dt) to 1e-10 relative or better.
"""
import numpy as np
import pytest

import oracle
from paper_2111_11806_amd import inputs
from parity_util import announce, check_fields, rel_l1

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def rbdi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2111_11806_amd import rbdi as r
    r.load()
    return r


def _pair(rbdi, prob, nsteps, precision="fp64", t_end=None):
    announce(f"{prob.name} n={prob.n} steps={nsteps} {precision} recon={prob.recon} seed={prob.seed}")
    orc = oracle.Oracle(prob)
    dts = orc.run(nsteps=nsteps, t_end=t_end)
    gpu = rbdi.Solver(prob, precision)
    gpu.run(dts)
    st = gpu.status()
    assert st["nonphysical"] == 0
    return orc, gpu, dts


def _check(orc, gpu, precision="fp64", label=None):
    """Per-field relative L1 and Linf of the conserved state against the
    oracle's (bars of parity_util.BARS)."""
    p = orc.prob
    return check_fields(gpu.get_state_cons(), orc.get_state_cons(), p.cons_names(), precision,
                        label or f"{p.name} {precision}")


# ---------------------------------------------------------------------------
# 1D
# ---------------------------------------------------------------------------

def test_sod_wall_full_run_fp64(rbdi):
    """Sod tube with a static rigid wall (400 cells, MUSCL + HLLC, CFL 0.8) to
    t = 0.3: conserved fields, primitives and the wall force match."""
    prob = inputs.sod_wall(400)
    orc, gpu, dts = _pair(rbdi, prob, nsteps=10**6)
    assert abs(sum(dts) - 0.3) < 1e-12
    _check(orc, gpu)
    check_fields(gpu.get_state_prim(), orc.get_state_prim(), prob.field_names(), "fp64", "sod_wall primitives")
    Fg, _ = gpu.rigid_force([0, 0, 0])
    Fo, _ = orc.rigid_force([0, 0, 0])
    assert Fg[0] == pytest.approx(Fo[0], rel=1e-10)
    st = gpu.status()
    assert st["steps"] == len(dts) and st["seeded"] > 0


@pytest.mark.parametrize("recon", ["muscl", "bvd_thinc"])
@pytest.mark.parametrize("seed", ["original", "riemann"])
def test_piston_moving_body(rbdi, recon, seed):
    prob = inputs.piston_1d(300, recon=recon)
    prob.seed = seed
    orc, gpu, _ = _pair(rbdi, prob, nsteps=120)
    _check(orc, gpu)


def test_piston_in_a_channel(rbdi):
    """A flat piston in a reflective channel, its face tilted at rounding
    level toward the lower wall: the first row's probes start within half a
    cell of the outermost centres (pinned on the oracle to keep the flow 1D);
    the device path seeds them the same way."""
    prob = inputs.piston_channel()
    orc, gpu, _ = _pair(rbdi, prob, nsteps=30)
    _check(orc, gpu)


@pytest.mark.parametrize("n", [3, 5, 57, 58, 59, 117, 401])
def test_ragged_1d_sizes(rbdi, n):
    """Sizes below, at and around the 58-cell wavefront tile, periodic and
    reflective ends."""
    prob = inputs.riemann_1d([1.0, 0.3, 1.0], [0.125, -0.2, 0.1], [inputs.ideal(1.4)], n=n, t_end=0.05,
                             recon="bvd_thinc")
    prob.bc = ["reflective"] * 6
    orc, gpu, _ = _pair(rbdi, prob, nsteps=15)
    _check(orc, gpu)


@pytest.mark.parametrize("nx,ny", [(3, 3), (58, 58), (59, 117), (117, 59), (130, 5)])
def test_ragged_2d_sizes(rbdi, nx, ny):
    """2D grids below, at and around the 58-cell x segment and the 58-row y
    segment (tiles of 16 columns with ragged last tiles), with the cylinder,
    Dirichlet inflow and reflective walls, 20 steps."""
    prob = inputs.shock_cylinder(nx, ny)
    orc, gpu, _ = _pair(rbdi, prob, nsteps=20)
    _check(orc, gpu)


@pytest.mark.parametrize("n", [(59, 5, 17), (3, 61, 4), (17, 9, 60)])
def test_ragged_3d_sizes(rbdi, n):
    """Non-cubic 3D grids with ragged tiles along every direction: a
    pressure pulse over a static sphere, reflective and transmissive faces."""
    nx, ny, nz = n
    dx = 1.0 / max(n)
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    z = (np.arange(nz) + 0.5) * dx
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    W = np.zeros((6, nz, ny, nx))
    hot = X + 0.5 * Y + 0.25 * Z < 0.3
    W[0] = np.where(hot, 2.0, 1.0)
    W[1] = np.where(hot, 0.6, 0.0)
    W[2] = np.where(hot, -0.2, 0.0)
    W[3] = np.where(hot, 0.1, 0.0)
    W[4] = np.where(hot, 2.5, 1.0)
    c = (0.5 * nx * dx, 0.5 * ny * dx, 0.5 * nz * dx)
    sdf = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) - 0.3 * min(n) * dx
    prob = inputs.Problem(name="ragged3d", dim=3, n=(nx, ny, nz), dx=(dx, dx, dx), origin=(0.0, 0.0, 0.0),
                          materials=[inputs.ideal(1.4)], solid=False,
                          bc=["transmissive", "transmissive", "reflective", "transmissive", "reflective",
                              "reflective"],
                          W0=W, sdf=sdf, width=1.0, recon="bvd_thinc", riemann="hllc", cfl=0.4, t_end=1.0)
    orc, gpu, _ = _pair(rbdi, prob, nsteps=12)
    _check(orc, gpu)


def test_two_phase_1d_water_air(rbdi):
    eps = 1e-6
    mats = [inputs.stiffened(1.4, 0.0), inputs.stiffened(4.4, 6e8)]
    prob = inputs.riemann_1d([eps, 50.0, 1000.0, 0.0, 1e9], [1 - eps, 50.0, 1000.0, 0.0, 1e5], mats, n=300,
                             t_end=1e-4, recon="bvd_thinc")
    orc, gpu, _ = _pair(rbdi, prob, nsteps=60)
    _check(orc, gpu)


# ---------------------------------------------------------------------------
# 2D
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("riemann", ["hllc", "hllc_lm"])
def test_shock_cylinder_reduced_grid(rbdi, riemann):
    """Mach 2.8 shock over the cylinder on 160 x 80 (several tiles and ragged
    tails in x and y), 80 steps."""
    prob = inputs.shock_cylinder(160, 80, riemann=riemann)
    orc, gpu, _ = _pair(rbdi, prob, nsteps=80)
    _check(orc, gpu)
    Fg, Tg = gpu.rigid_force([0.3, 0.25, 0.0])
    Fo, To = orc.rigid_force([0.3, 0.25, 0.0])
    assert np.allclose(Fg, Fo, rtol=1e-10, atol=1e-12 * np.abs(Fo).max())
    assert np.allclose(Tg, To, rtol=1e-9, atol=1e-12 * max(np.abs(Fo).max(), 1e-300))
    ta, tf = gpu.conserved_totals()
    oa, of = orc.conserved_totals()
    assert np.allclose(ta, oa, rtol=1e-10, atol=1e-14)
    assert np.allclose(tf, of, rtol=1e-10, atol=1e-14)


def test_shock_cylinder_riemann_seeding_and_fixed_probe(rbdi):
    prob = inputs.shock_cylinder(128, 64)
    prob.seed = "riemann"
    prob.probe = "fixed"
    orc, gpu, _ = _pair(rbdi, prob, nsteps=50)
    _check(orc, gpu)


def test_shock_cylinder_fp32(rbdi):
    prob = inputs.shock_cylinder(160, 80)
    orc, gpu, _ = _pair(rbdi, prob, nsteps=80, precision="fp32")
    rl = _check(orc, gpu, "fp32")
    print("fp32 rel L1 per field", rl)


@pytest.mark.parametrize("normal", ["elvira", "youngs"])
def test_wedge_mach17(rbdi, normal):
    """Mach 1.7 shock onto the 25-degree wedge on 150 x 100 (several tiles,
    ragged tails; the body meets the reflective bottom boundary), 120 steps:
    the shock reaches the ramp and reflects from it."""
    prob = inputs.wedge(150, 100, normal=normal)
    orc, gpu, _ = _pair(rbdi, prob, nsteps=120)
    _check(orc, gpu)
    Fg, _ = gpu.rigid_force([0.5, 0.0, 0.0])
    Fo, _ = orc.rigid_force([0.5, 0.0, 0.0])
    assert np.allclose(Fg, Fo, rtol=1e-10, atol=1e-12 * np.abs(Fo).max())


def test_wedge_elvira_rectangular_cells(rbdi):
    """ELVIRA with dx != dy (150 x 80 on 3 x 2: cells 0.02 x 0.025), where
    the column and row sums carry different cell sizes."""
    prob = inputs.wedge(150, 80)
    assert prob.dx[0] != prob.dx[1]
    orc, gpu, _ = _pair(rbdi, prob, nsteps=100)
    _check(orc, gpu)


def test_wedge_mach10_elvira(rbdi):
    """Mach 10 shock onto the 30-degree wedge (double Mach reflection case),
    150 x 100, 80 steps, Riemann seeding."""
    prob = inputs.wedge(150, 100, mach=10.0, angle_deg=30.0)
    prob.seed = "riemann"
    orc, gpu, _ = _pair(rbdi, prob, nsteps=80)
    _check(orc, gpu)


def test_wedge_elvira_fp32(rbdi):
    prob = inputs.wedge(150, 100)
    orc, gpu, _ = _pair(rbdi, prob, nsteps=120, precision="fp32")
    _check(orc, gpu, "fp32")


def test_sharp_ramp_elvira_seeding(rbdi):
    """Exact cut-cell fractions of a 25-degree ramp in a uniform stream (the
    case ELVIRA reconstructs exactly): the states after one step (the first
    seeding and its three stages) and after ten steps match."""
    from geometry_util import sharp_ramp
    prob = sharp_ramp(inputs.wedge(90, 60, normal="elvira"), 25.0)
    orc, gpu, dts = _pair(rbdi, prob, nsteps=10)
    _check(orc, gpu)
    g1 = rbdi.Solver(prob, "fp64")
    g1.run(dts[:1])
    o1 = oracle.Oracle(prob)
    o1.run(dts=dts[:1])
    _check(o1, g1)


def _uniform_stream_with_body(prob, sdf, bc, stream=(1.2, 0.4)):
    W = np.zeros_like(prob.W0)
    W[0] = 1.0
    W[1] = stream[0]
    W[2] = stream[1]
    W[3] = 1.0
    prob.W0 = W
    prob.sdf = sdf
    prob.bc = bc
    return prob


def test_elvira_body_across_periodic_boundaries(rbdi):
    """A rotated ellipse cut by both periodic boundaries in a uniform stream:
    ELVIRA's 3x3 blocks wrap around the domain edges and corners."""
    prob = inputs.wedge(96, 64, normal="elvira")
    nx, ny = prob.n[0], prob.n[1]
    dx, dy = prob.dx[0], prob.dx[1]
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y)
    Lx, Ly = nx * dx, ny * dy
    best = None
    for sx in (-Lx, 0.0, Lx):          # periodic images of the body
        for sy in (-Ly, 0.0, Ly):
            d = inputs.ellipse_sdf(X + sx, Y + sy, 0.05, 0.1, 0.3, 0.18, angle=0.6)
            best = d if best is None else np.minimum(best, d)
    prob = _uniform_stream_with_body(prob, best[None], ["periodic"] * 4 + ["transmissive"] * 2)
    prob.bc_states = {}
    orc, gpu, _ = _pair(rbdi, prob, nsteps=40)
    _check(orc, gpu)
    assert gpu.status()["seeded"] > 0


def test_elvira_body_on_dirichlet_inflow(rbdi):
    """A cylinder cut by the Dirichlet inflow face (its ghost r is the
    boundary state's) and by the reflective bottom (corner blocks)."""
    prob = inputs.wedge(90, 60, normal="elvira")
    nx, ny = prob.n[0], prob.n[1]
    x = (np.arange(nx) + 0.5) * prob.dx[0]
    y = (np.arange(ny) + 0.5) * prob.dx[1]
    X, Y = np.meshgrid(x, y)
    sdf = np.sqrt((X - 0.05) ** 2 + (Y - 0.1) ** 2) - 0.35
    prob = _uniform_stream_with_body(prob, sdf[None], ["dirichlet", "transmissive", "reflective",
                                                        "transmissive", "transmissive", "transmissive"])
    prob.bc_states = {0: np.array([1.0, 1.2, 0.4, 1.0, 0.0])}
    orc, gpu, _ = _pair(rbdi, prob, nsteps=40)
    _check(orc, gpu)


def test_cfl_dt_matches(rbdi):
    prob = inputs.shock_cylinder(200, 100)
    orc = oracle.Oracle(prob)
    gpu = rbdi.Solver(prob, "fp64")
    for _ in range(3):
        dto = orc.compute_dt(0.4)
        dtg = gpu.compute_dt(0.4)
        assert dtg == pytest.approx(dto, rel=1e-13)
        orc.step(dto)
        gpu.step(dto)


def test_advance_device_dt_equals_host_loop(rbdi):
    """rbdi_advance (dt on the device, no host sync) equals compute_dt + step."""
    prob = inputs.shock_cylinder(128, 64)
    a = rbdi.Solver(prob, "fp64")
    b = rbdi.Solver(prob, "fp64")
    a.advance(0.4, 20, 0.0)
    for _ in range(20):
        b.step(b.compute_dt(0.4))
    assert np.array_equal(a.get_state_cons(), b.get_state_cons())
    assert a.status()["t"] == b.status()["t"]


def test_advance_clips_at_t_end(rbdi):
    prob = inputs.sod_wall(400)
    a = rbdi.Solver(prob, "fp64")
    a.advance(0.8, 2000, 0.3)
    st = a.status()
    assert st["t"] == pytest.approx(0.3, abs=1e-14)
    orc = oracle.Oracle(prob)
    dts = orc.run()
    assert st["steps"] == len(dts)
    check_fields(a.get_state_cons(), orc.get_state_cons(), prob.cons_names(), "fp64", "sod_wall advance")


def test_air_water_moving_ellipse(rbdi):
    """Two stiffened gases, THINC on r and phi, moving rigid ellipse (reduced
    grid 192 x 96, 40 steps)."""
    prob = inputs.air_water(192, 96)
    orc, gpu, _ = _pair(rbdi, prob, nsteps=40)
    _check(orc, gpu)


def test_air_water_moving_ellipse_elvira(rbdi):
    """The moving ellipse with ELVIRA normals: the band (normals, probes) is
    rebuilt every step from the advected r."""
    prob = inputs.air_water(192, 96)
    prob.normal = "elvira"
    orc, gpu, _ = _pair(rbdi, prob, nsteps=40)
    _check(orc, gpu)


def test_diagnostics_leave_the_state_alone(rbdi):
    """Kernel replays, timing and operator evaluation write only scratch
    buffers: the state and the following steps are bitwise those of a
    solver that never ran them."""
    prob = inputs.shock_cylinder(160, 80)
    a = rbdi.Solver(prob, "fp64")
    b = rbdi.Solver(prob, "fp64")
    a.advance(prob.cfl, 10)
    b.advance(prob.cfl, 10)
    a.set_kernel_timing(True)
    a.advance(prob.cfl, 3)
    a.kernel_times()
    a.set_kernel_timing(False)
    b.advance(prob.cfl, 3)
    u0 = a.get_state_cons()
    a.kernel_replay(0, 5)
    a.kernel_replay(1, 5)
    a.eval_rhs()
    assert np.array_equal(a.get_state_cons(), u0)
    a.advance(prob.cfl, 5)
    b.advance(prob.cfl, 5)
    assert np.array_equal(a.get_state_cons(), b.get_state_cons())
    assert a.status()["t"] == b.status()["t"]


@pytest.mark.parametrize("make,precision", [(lambda: inputs.shock_cylinder(300, 150), "fp64"),
                                            (lambda: inputs.sod_wall(400), "fp64"),
                                            (lambda: inputs.air_water(192, 96), "fp32")])
def test_autotune_keeps_state_and_results(rbdi, make, precision):
    """rbdi_autotune times real steps per x-sweep block size and puts the
    state back: afterwards the state, time and step count are those before
    the call, and further steps are bitwise those of an untuned solver; every
    block size gives the same results."""
    prob = make()
    a = rbdi.Solver(prob, precision)
    b = rbdi.Solver(prob, precision)
    a.advance(prob.cfl, 6)
    b.advance(prob.cfl, 6)
    u0, st0 = a.get_state_cons(), a.status()
    best, us = a.autotune(prob.cfl, 4)
    assert best in ((1,) if prob.dim == 1 else (1, 2, 4)) and us > 0.0
    st1 = a.status()
    assert np.array_equal(a.get_state_cons(), u0)
    assert st1["t"] == st0["t"] and st1["steps"] == st0["steps"] and st1["seeded"] == st0["seeded"]
    a.advance(prob.cfl, 5)
    b.advance(prob.cfl, 5)
    assert np.array_equal(a.get_state_cons(), b.get_state_cons())
    assert a.status()["t"] == b.status()["t"]
    if prob.dim > 1:
        for w in (1, 2, 4):
            c = rbdi.Solver(prob, precision)
            c.set_x_waves(w)
            c.advance(prob.cfl, 11)
            assert np.array_equal(c.get_state_cons(), b.get_state_cons()), w


def test_air_water_fp32(rbdi):
    """FP32 path on the two stiffened gases (p_inf of water 6e8 Pa against
    p = 1e5 Pa): the stored energy E~ = rho E - B(phi) keeps the pressure
    inversion free of cancellation. Conserved fields and primitives (p
    included) per field."""
    prob = inputs.air_water(256, 128)
    orc, gpu, _ = _pair(rbdi, prob, nsteps=40, precision="fp32")
    _check(orc, gpu, "fp32")
    check_fields(gpu.get_state_prim(), orc.get_state_prim(), prob.field_names(), "fp32", "air_water primitives")


@pytest.mark.parametrize("defect", ["tension_beyond_pinf", "fraction_above_one"])
def test_nonphysical_flag(rbdi, defect):
    """The admissibility flag of rbdi_status: a water cell pulled below
    p = -p_inf (its mixture sound speed squared turns negative), or a volume
    fraction above one, is reported after the step (first bad cell near that
    cell), while the same problem without the defect stays admissible."""
    prob = inputs.air_water(64, 32)
    names = prob.field_names()
    W = prob.W0.copy()
    j, i = 16, 40  # inside the water column
    assert W[names.index("phi0"), 0, j, i] < 0.5
    ref = rbdi.Solver(prob, "fp64")
    dt = 0.5 * ref.compute_dt(prob.cfl)
    ref.step(dt)
    assert ref.status()["nonphysical"] == 0
    if defect == "tension_beyond_pinf":
        W[names.index("p"), 0, j, i] = -6.5e8   # water p_inf is 6e8 Pa
    else:
        W[names.index("phi0"), 0, j, i] = 1.3
    prob.W0 = W
    s = rbdi.Solver(prob, "fp64")
    s.step(dt)
    st = s.status(raise_on_error=False)
    assert st["nonphysical"] == 1
    bad = st["first_bad"]
    # the flagged cell is the defect or a cell its update reached within the
    # step (three stages of a three-cell stencil)
    jb, ib = divmod(bad, prob.n[0])
    assert abs(jb - j) <= 9 and abs(ib - i) <= 9, (jb, ib)


def test_quiescent_body_bitwise_steady(rbdi):
    prob = inputs.quiescent_body(64, 40)
    gpu = rbdi.Solver(prob, "fp64")
    U0 = gpu.get_state_cons()
    for _ in range(20):
        gpu.step(0.004)
    assert np.array_equal(U0, gpu.get_state_cons())


def test_conservation_periodic_2d_two_phase(rbdi):
    prob = inputs.periodic_box(dim=2, n=48, nmat=2)
    gpu = rbdi.Solver(prob, "fp64")
    t0, _ = gpu.conserved_totals()
    for _ in range(200):
        gpu.step(0.2 * gpu.compute_dt(1.0))
    t1, _ = gpu.conserved_totals()
    nc = 2 + 2 + 1
    scale = np.abs(gpu.get_state_cons()[:nc]).sum(axis=(1, 2, 3)) / 48 ** 2
    assert np.all(np.abs(t1[:nc] - t0[:nc]) <= 1e-12 * scale)


@pytest.mark.parametrize("dim", [2, 3])
def test_rotating_translating_body_vs_oracle(rbdi, dim):
    """A rigid ellipse (2D) / ellipsoid (3D) turning and moving through gas
    with a pressure pulse: v_r = v + omega x (x - c) (Sec. 2.3) enters the r
    flux at the faces, the mirror state of every seeded cell, the band built
    every step and the CFL rate; force and torque about the moving centre
    (FP64 to 1e-10)."""
    from geometry_util import ellipsoid_problem
    n = 80 if dim == 2 else 26
    shape = (1, n, n) if dim == 2 else (n, n, n)
    W = np.zeros((3 + dim, *shape))
    dx = 1.0 / n
    g = (np.arange(n) + 0.5) * dx
    if dim == 2:
        Y, X = np.meshgrid(g, g, indexing="ij")
        d2 = (X - 0.2) ** 2 + (Y - 0.3) ** 2
    else:
        Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
        d2 = (X - 0.2) ** 2 + (Y - 0.3) ** 2 + (Z - 0.7) ** 2
    W[0] = 1.0 + 0.3 * np.exp(-d2 / 0.01).reshape(shape)
    W[1 + dim] = 1.0 + 0.8 * np.exp(-d2 / 0.01).reshape(shape)
    omega = (0.0, 0.0, 3.0) if dim == 2 else (0.8, -1.1, 2.0)
    v = (0.3, -0.2, 0.0) if dim == 2 else (0.3, -0.2, 0.15)
    prob, _, _ = ellipsoid_problem(dim, n, W, motion=(v, omega))
    prob.name = f"rotating{dim}d"
    nsteps = 60 if dim == 2 else 14
    orc, gpu, _ = _pair(rbdi, prob, nsteps=nsteps)
    _check(orc, gpu)
    assert gpu.status()["seeded"] > 0
    ctr = np.asarray(prob.center) + np.asarray(v) * orc.t
    Fg, Tg = gpu.rigid_force(ctr)
    Fo, To = orc.rigid_force(ctr)
    announce(f"  force {Fg} torque {Tg} (oracle {Fo} {To})")
    assert np.abs(To).max() > 0.0
    assert np.linalg.norm(Fg - Fo) <= 1e-10 * np.linalg.norm(Fo)
    assert np.linalg.norm(Tg - To) <= 1e-10 * np.linalg.norm(To)


# ---------------------------------------------------------------------------
# 3D
# ---------------------------------------------------------------------------

def test_periodic_3d_single_gas(rbdi):
    prob = inputs.periodic_box(dim=3, n=20, nmat=1)
    orc, gpu, _ = _pair(rbdi, prob, nsteps=10)
    _check(orc, gpu)


def test_3d_sphere_in_shock(rbdi):
    """A planar pressure pulse over a static rigid sphere on 24^3."""
    n = 24
    prob = inputs.periodic_box(dim=3, n=n, nmat=1)
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    W = np.zeros((6, n, n, n))
    W[0] = np.where(X < 0.2, 2.0, 1.0)
    W[1] = np.where(X < 0.2, 0.8, 0.0)
    W[4] = np.where(X < 0.2, 2.5, 1.0)
    prob.W0 = W
    prob.bc = ["transmissive"] * 6
    prob.sdf = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2) - 0.2
    prob.seed = "original"
    orc, gpu, _ = _pair(rbdi, prob, nsteps=12)
    _check(orc, gpu)


# ---------------------------------------------------------------------------
# Elastoplastic system
# ---------------------------------------------------------------------------

def test_copper_piston_1d_elastoplastic(rbdi):
    """Copper driven by a rigid piston: Romenskii closure, Hencky strain,
    solid HLLC, stretch-tensor non-conservative terms, plastic return."""
    prob = inputs.copper_piston_1d(200)
    orc, gpu, _ = _pair(rbdi, prob, nsteps=150)
    _check(orc, gpu)


def test_copper_2d_oblique_piston(rbdi):
    """2D copper/air with an oblique moving rigid wedge (shear and plastic flow
    in the plane), 96 x 64, 40 steps."""
    n = (96, 64)
    prob1 = inputs.copper_piston_1d(8)
    h = 10e-3 / n[0]
    X, Y = np.meshgrid((np.arange(n[0]) + 0.5) * h, (np.arange(n[1]) + 0.5) * h)
    W = np.zeros((17, 1, n[1], n[0]))
    phi = 1e-6 + (1 - 2e-6) * 0.5 * (1 - np.tanh((Y - 4.5e-3) / h))
    W[0] = phi
    W[1] = 8930.0
    W[2] = 1.2
    W[5] = 1.0e5
    for a in range(3):
        W[6 + 4 * a] = 1.0
    sdf = ((X - 2e-3) * np.cos(0.3) + (Y - 3e-3) * np.sin(0.3)).reshape(1, n[1], n[0])
    prob = inputs.Problem(name="copper2d", dim=2, n=(n[0], n[1], 1), dx=(h, h, 1.0), origin=(0, 0, 0),
                          materials=prob1.materials, solid=True,
                          bc=["transmissive", "transmissive", "reflective", "transmissive", "transmissive",
                              "transmissive"],
                          W0=W, sdf=sdf, width=1.0, v_r=(40.0, 10.0, 0.0), center=(2e-3, 3e-3, 0.0),
                          recon="bvd_thinc", riemann="hllc", cfl=0.3)
    orc, gpu, _ = _pair(rbdi, prob, nsteps=40)
    _check(orc, gpu)


def test_copper_indenter_3d_reduced(rbdi):
    """The 3D copper indenter workload on 24^3 (8 steps)."""
    prob = inputs.copper_indenter(24)
    orc, gpu, _ = _pair(rbdi, prob, nsteps=8)
    _check(orc, gpu)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_run_to_run_bitwise(rbdi, precision):
    """Determinism: the same problem advanced twice (device CFL steps, fixed-
    order reductions, no atomics on results) gives identical bits."""
    for prob, n in ((inputs.shock_cylinder(160, 80), 60), (inputs.copper_indenter(20), 6)):
        out = []
        for _ in range(2):
            s = rbdi.Solver(prob, precision)
            s.advance(prob.cfl, n, prob.t_end)
            F, T = s.rigid_force(prob.center)
            out.append((s.get_state_cons(), F, T, s.status()["t"]))
        assert np.array_equal(out[0][0], out[1][0])
        assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])
        assert out[0][3] == out[1][3]
