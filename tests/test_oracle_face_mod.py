"""Pins of the oracle's void-opening face modifier (Sec. 3.2, end) on an
elastic copper slab that strikes a static rigid wall.

Elastic-wave estimate (uniaxial strain, c_L = sqrt((K0 + 4/3 G0) / rho0)):
the impact sends a compression wave into the slab, which reflects at its
free face as a release wave; the wall pushes on the slab with the constant
traction rho0 c_L |v| for 2 L / c_L, during which the slab's mean velocity
rises linearly from v to -v, and then the slab is stress free and leaves at
-v. With the modifier the oracle must show exactly that (rebound at -v after
2 L / c_L); without it the wall, a mirror condition, holds the slab in
tension and pulls it back. The contact pressure is the elastic estimate's
mean stress K0 / (K0 + 4/3 G0) rho0 c_L |v|.
"""
import numpy as np
import pytest

import oracle
from paper_2111_11806_amd import inputs

V, SLAB, N = -20.0, 6e-3, 400


def _run(face_mod, t_stop, v=V, n=N, record_every=5):
    prob = inputs.copper_slab_wall(n=n, v=v, slab=SLAB, face_mod=face_mod)
    o = oracle.Oracle(prob)
    ts, um, pw = [], [], []
    k = 0
    while o.t < t_stop:
        o.step(o.compute_dt(prob.cfl))
        k += 1
        if k % record_every == 0 or o.t >= t_stop:
            U = o.get_state_cons()[:, 0, 0, :]
            W = o.get_state_prim()[:, 0, 0, :]
            m = W[-1] < 0.5
            ts.append(o.t)
            um.append((U[0] * W[3])[m].sum() / U[0][m].sum())
            pw.append(W[4][m][1])
    return prob, np.array(ts), np.array(um), np.array(pw), o


def _tc(prob):
    return 2.0 * SLAB / inputs.longitudinal_wave_speed(prob.materials[0])


@pytest.fixture(scope="module")
def with_mod():
    prob = inputs.copper_slab_wall(n=N, slab=SLAB)
    return _run(True, 1.5 * _tc(prob))


def test_rebound_velocity_and_contact_time(with_mod):
    prob, ts, um, _, o = with_mod
    tc = _tc(prob)
    # leaves at -v once the release wave is back at the wall ...
    assert um[-1] == pytest.approx(-V, rel=0.025)
    # ... and no later than about 2 L / c_L: the mean velocity crosses zero
    # at half the contact time and reaches 98% of -v at the contact time
    t0 = np.interp(0.0, um, ts)
    assert t0 == pytest.approx(0.5 * tc, rel=0.03)
    t98 = ts[np.argmax(um >= -0.98 * V)]
    assert t98 == pytest.approx(tc, rel=0.03)
    # after that the slab is free: its mean velocity no longer changes
    late = um[ts > 1.15 * tc]
    assert np.ptp(late) < 1e-3 * abs(V)


def test_contact_pressure_elastic_estimate(with_mod):
    prob, ts, um, pw, _ = with_mod
    tc = _tc(prob)
    m = prob.materials[0]
    cl = inputs.longitudinal_wave_speed(m)
    p_est = m["K0"] / (m["K0"] + 4.0 / 3.0 * m["G0"]) * m["rho0"] * cl * abs(V)
    during = pw[(ts > 0.1 * tc) & (ts < 0.9 * tc)]
    assert np.median(during) == pytest.approx(p_est, rel=0.05)


def test_wall_holds_the_slab_without_the_modifier():
    prob = inputs.copper_slab_wall(n=N, slab=SLAB, face_mod=False)
    tc = _tc(prob)
    _, ts, um, pw, _ = _run(False, 1.5 * tc, record_every=20)
    # the same rise to -v over the contact time ...
    assert np.interp(tc, ts, um) == pytest.approx(-V, rel=0.03)
    # ... then the mirror wall pulls the slab back (no separation)
    assert um[-1] < 0.1 * abs(V)
    assert pw[-1] < -0.5 * abs(pw[len(pw) // 4])


def test_slab_at_rest_on_the_wall_stays_at_rest():
    """Compressive (ambient) contact: the modifier's wall state is an exact
    mirror, so a slab at rest against the wall does not move."""
    prob = inputs.copper_slab_wall(n=200, v=0.0, slab=SLAB)
    o = oracle.Oracle(prob)
    W0 = o.get_state_prim()
    for _ in range(100):
        o.step(o.compute_dt(prob.cfl))
    W = o.get_state_prim()
    m = W[-1, 0, 0] < 0.5
    assert np.abs(W[3, 0, 0][m]).max() < 1e-9
    assert np.abs(W[4, 0, 0][m] - W0[4, 0, 0][m]).max() < 1e-6 * 1e5


def test_face_mod_arguments():
    prob = inputs.copper_slab_wall(n=50, slab=1e-3)
    o = oracle.Oracle(prob)
    with pytest.raises(ValueError):
        o.set_face_mod(2, prob.gap_gas)
    o.set_face_mod(0)
    fluid = inputs.sod_wall(50)
    of = oracle.Oracle(fluid)
    with pytest.raises(ValueError):
        of.set_face_mod(1, np.zeros(fluid.nfields))


def test_wall_through_a_cell_centre():
    """A wall through a cell centre leaves that cell at r = 0.5 exactly: a
    material cell, so the modifier acts on the face to its rigid neighbour
    (the strict product (0.5 - r_L)(0.5 - r_R) < 0 would never hold there and
    the wall would hold the slab)."""
    n, length, slab = 150, 3e-3, 1.5e-3
    h = length / n
    prob = inputs.copper_slab_wall(n=n, v=V, slab=slab, length=length, x_w=12.5 * h)
    o = oracle.Oracle(prob)
    r = o.get_state_prim()[-1, 0, 0]
    assert np.any(r == 0.5)
    tc = 2.0 * slab / inputs.longitudinal_wave_speed(prob.materials[0])
    o.run(t_end=1.5 * tc)
    U = o.get_state_cons()[:, 0, 0, :]
    W = o.get_state_prim()[:, 0, 0, :]
    m = W[-1] < 0.5
    assert (U[0] * W[3])[m].sum() / U[0][m].sum() == pytest.approx(-V, rel=0.03)


@pytest.mark.parametrize("dim,axis", [(2, 1), (3, 2)])
def test_slab_across_y_or_z_reproduces_the_1d_run(dim, axis):
    """The modifier in the y (2D) and z (3D) sweeps: a slab uniform across
    the other (periodic) axes is the 1D problem turned; every column must
    reproduce the pinned 1D run through the impact and the opening (conserved
    fields to 1e-10 of each field's largest value: the seeding's probes
    interpolate across identical columns, which rounds), with the normal
    momentum and the normal / tangential stretches exchanged."""
    n, length, slab = 150, 3e-3, 1.5e-3
    kw = dict(n=n, v=V, slab=slab, length=length, x_w=10 * length / n)
    p1 = inputs.copper_slab_wall(**kw)
    pd = inputs.copper_slab_wall(dim=dim, axis=axis, ntrans=3, **kw)
    o1, od = oracle.Oracle(p1), oracle.Oracle(pd)
    tc = 2.0 * slab / inputs.longitudinal_wave_speed(p1.materials[0])
    dts = o1.run(t_end=1.3 * tc)
    od.run(dts=dts)
    U1 = o1.get_state_cons()[:, 0, 0, :]
    Ud = od.get_state_cons()
    f1, fd = p1.cons_names(), pd.cons_names()
    mom = "m" + "xyz"[axis]
    pairs = [("arho0", "arho0"), ("arho1", "arho1"), ("mx", mom), ("E", "E"), ("phi0", "phi0"),
             ("V00", f"V{axis}{axis}"), ("V11", "V00"), ("V22", "V22" if axis == 1 else "V11"),
             ("aeps", "aeps"), ("r", "r")]
    for a, b in pairs:
        ref = U1[f1.index(a)]
        col = np.moveaxis(Ud[fd.index(b)], 2 - axis, -1).reshape(-1, n)
        scale = max(np.abs(ref).max(), 1e-300)
        assert np.abs(col - ref).max() <= 1e-10 * scale, (a, b, np.abs(col - ref).max() / scale)
    # the other momentum components stay zero
    for c in "xyz"[:dim]:
        if c != "xyz"[axis]:
            assert np.abs(Ud[fd.index("m" + c)]).max() == 0.0
    # and the slab has left the wall
    W1 = o1.get_state_prim()[:, 0, 0, :]
    m = W1[-1] < 0.5
    assert (U1[0] * W1[p1.field_names().index("u")])[m].sum() / U1[0][m].sum() > 0.9 * abs(V)


def test_wall_pulling_away_leaves_a_resting_slab_at_rest():
    """A moving wall (the rigid velocity enters the mirror state): the wall
    starts to move away from a slab at rest at 20 m/s. With the modifier the
    contact opens at once and the slab stays at rest (a free face); without
    it the mirror condition drags the slab after the wall, and the release
    wave reflected at the slab's free end doubles the pull (mean velocity
    near twice the wall's after 2 L / c_L)."""
    w = -20.0
    res = {}
    for fm in (True, False):
        prob = inputs.copper_slab_wall(n=N, v=0.0, slab=SLAB, wall_v=w, face_mod=fm)
        tc = _tc(prob)
        o = oracle.Oracle(prob)
        o.run(t_end=tc)
        U = o.get_state_cons()[:, 0, 0, :]
        W = o.get_state_prim()[:, 0, 0, :]
        m = W[-1] < 0.5
        res[fm] = (U[0] * W[3])[m].sum() / U[0][m].sum()
    assert abs(res[True]) < 0.01 * abs(w)
    assert res[False] < 1.5 * w
