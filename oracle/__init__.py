"""CPU FP64 oracle of the diffuse-interface rigid-body step (arXiv 2111.11806).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` import this package. The product path
(``paper_2111_11806_amd``) never imports it and shares no code with it; the
two meet only through the seeded input generators of
``paper_2111_11806_amd.inputs``, which hold no arithmetic of the method.

The numerics live in ``rbdi_oracle.cpp`` (plain C++17, FP64, no fast-math,
``-ffp-contract=off``). This module compiles it on demand with g++ and wraps
it with ctypes.

What pins each part of the oracle (tests marked ``not gpu``):

* EOS and closure (Sec. 2.1.2-2.2): ``p_ref = rho^2 de_ref/drho`` by
  complex-step differentiation, ``c^2`` against a finite-difference isentrope,
  stiffened-gas identities, pure-cell limits, water sound speed.
* THINC candidates (Sec. 3.1): cell average recomputed by quadrature, face
  values bounded, MUSCL slope against the van Leer formula on hand cases.
* BVD selection (Sec. 3.1): hand-computed total-boundary-variation cases
  (a smeared step takes THINC, a linear ramp keeps MUSCL, a tie keeps MUSCL,
  each neighbour face enters with its own scheme), and a contact advected
  once around a periodic box: sharper and closer to the exact profile than
  with MUSCL.
* HLLC (Sec. 3.1): consistency F(U,U) = F(U), contact preservation,
  equality of the central (LM) form with phi=1 and the Toro form; HLLC-LM
  (Sec. 4.3): the numerical pressure of a symmetric compression face scales
  as Ma with HLLC and as Ma^2 with HLLC-LM below the Mach limit.
* Reduced system end to end: exact Riemann solutions (Sod; stiffened-gas
  water/air), the exact Sod-and-wall solution with the reflected shock and its
  interaction with the contact, the Rankine-Hugoniot moving piston,
  quiescent preservation around a static body (bitwise), Abgrall interface,
  conservation to 1e-12 with periodic boundaries.
* Seeding (Sec. 3.2): a flat piston in a channel stays one-dimensional with
  its normal tilted toward a wall at rounding level (probe points near a
  domain face); Householder reflection identities, equality with an
  explicit rotate-reflect-rotate-back, the Riemann variant's S* = v_r.n; its
  p* and rho* against linear acoustics for small wall-normal speeds and the
  exact Riemann solution at moderate ones, its stretch against the
  kinematics of a uniaxial compression.
* ELVIRA normal (Sec. 3.3): cut fractions against the closed-form area
  below a line, exact reproduction of straight interfaces (and the seeded
  mirror state of a sharp ramp), convergence on a circle with exact cell
  areas, block symmetries.
* Force (O.6 reading): summation-by-parts identity, uniform and linear
  pressure fields.
* Elastoplastic closure: Hencky strain of diagonal and rotated stretches,
  elastic wave speed and plastic return invariants; a copper piston's
  elastic precursor at the Hugoniot elastic limit and its plastic wave at the
  bulk sound speed with the momentum-jump stress.
* Void-opening face modifier (Sec. 3.2, end): an elastic copper slab striking
  a rigid wall against the elastic-wave estimate (contact pressure, contact
  time 2 L / c_L, rebound at the impact speed); without the modifier the
  wall holds the slab; a slab at rest on the wall stays at rest, also when
  the wall starts to move away from it; the same
  slab across y (2D) or z (3D) reproduces the 1D run column by column. The gap
  gas that fills the opening (the reading taken for the deferred void model)
  is pinned only through the rebound.

Parity unpinned: the readings that no external solution distinguishes (the
exact HLLC-LM constants beyond the Ma^2 scaling, the phi star state, the
solid HLLC variant's star-region flux, the gap gas's velocity) are pinned
only by internal identities or by what they lead to.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rbdi_oracle.cpp")
_LIB = os.path.join(_HERE, "liborbdi.so")
_lock = threading.Lock()
_libs = {}

EOS = {"ideal": 0, "stiffened": 1, "romenskii": 2}
BC = {"transmissive": 0, "reflective": 1, "dirichlet": 2, "periodic": 3}
RECON = {"muscl": 0, "bvd_thinc": 1}
RIEMANN = {"hllc": 0, "hllc_lm": 1}
SEED = {"original": 0, "riemann": 1, "none": 2}
PROBE = {"stepout": 0, "fixed": 1}
NORMAL = {"youngs": 0, "elvira": 1}


# Build variants: the reference build, and one with FMA contraction allowed
# (-ffp-contract=fast with FMA instructions), used only to measure how far
# rounding-order changes alone move the oracle's results (the jitter floor).
_VARIANTS = {
    None: ("liborbdi.so", ["-ffp-contract=off", "-fno-fast-math"]),
    "contract": ("liborbdi_contract.so", ["-ffp-contract=fast", "-mfma", "-fno-fast-math"]),
}


def build(force: bool = False, variant=None) -> str:
    """Compile the oracle with g++ (plain -O2, OpenMP, no FMA contraction
    unless a variant asks for it)."""
    name, flags = _VARIANTS[variant]
    out = os.path.join(_HERE, name)
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = ["g++", "-std=c++17", "-O2", "-fopenmp"] + flags + ["-shared", "-fPIC", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


class _Desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dx", ctypes.c_double * 3), ("origin", ctypes.c_double * 3),
                ("nmat", ctypes.c_int), ("solid", ctypes.c_int), ("bc", ctypes.c_int * 6),
                ("recon", ctypes.c_int), ("riemann", ctypes.c_int), ("seed", ctypes.c_int),
                ("probe", ctypes.c_int), ("plastic", ctypes.c_int),
                ("thinc_beta", ctypes.c_double), ("lm_mach", ctypes.c_double), ("normal", ctypes.c_int)]


def lib(variant=None):
    with _lock:
        if variant not in _libs:
            L = ctypes.CDLL(build(variant=variant))
            vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
            L.orc_create.restype = vp
            L.orc_create.argtypes = [ctypes.POINTER(_Desc)]
            L.orc_destroy.argtypes = [vp]
            L.orc_nfields.argtypes = [vp]
            L.orc_set_material.argtypes = [vp, ip, ip, dp]
            L.orc_set_bc_state.argtypes = [vp, ip, dp]
            for nm in ("orc_set_state_prim", "orc_get_state_prim", "orc_get_state_cons", "orc_set_state_cons"):
                getattr(L, nm).argtypes = [vp, dp]
            L.orc_set_rigid_sdf.argtypes = [vp, dp, ctypes.c_double, dp, dp, dp]
            L.orc_set_rigid_motion.argtypes = [vp, dp, dp, dp]
            L.orc_set_rigid_bodies.argtypes = [vp, ip, dp, dp, dp, dp, dp]
            L.orc_set_face_mod.argtypes = [vp, ip, dp]
            L.orc_compute_dt.restype = ctypes.c_double
            L.orc_compute_dt.argtypes = [vp, ctypes.c_double]
            L.orc_step.argtypes = [vp, ctypes.c_double]
            L.orc_seed.argtypes = [vp]
            L.orc_rhs.argtypes = [vp, dp, ip]
            L.orc_time.restype = ctypes.c_double
            L.orc_time.argtypes = [vp]
            L.orc_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_long)]
            L.orc_rigid_force.argtypes = [vp, dp, dp, dp]
            L.orc_conserved_totals.argtypes = [vp, dp]
            L.orc_candidates.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
            L.orc_bvd_select.argtypes = [vp, dp, dp, dp, dp]
            L.orc_set_threads.argtypes = [ip]
            L.orc_get_threads.restype = ip
            L.orc_prim_to_cons.argtypes = [vp, dp, dp]
            L.orc_cons_to_prim.argtypes = [vp, dp, dp]
            L.orc_thermo.argtypes = [vp, dp, dp]
            L.orc_face_flux.argtypes = [vp, dp, dp, ip, dp]
            L.orc_phys_flux.argtypes = [vp, dp, ip, dp]
            L.orc_mirror_state.argtypes = [vp, dp, dp, dp, dp]
            L.orc_riemann_seed_state.argtypes = [vp, dp, dp, dp, dp]
            L.orc_solid_sources.argtypes = [vp, dp]
            L.orc_hencky.argtypes = [dp, dp]
            L.orc_phase_ref.argtypes = [ip, dp, ctypes.c_double, ctypes.c_double, dp]
            L.orc_elvira_normal.restype = ip
            L.orc_elvira_normal.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
            L.orc_cut_fraction.restype = ctypes.c_double
            L.orc_cut_fraction.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
            _libs[variant] = L
    return _libs[variant]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def set_threads(n):
    """OpenMP threads of the oracle's loops (for timing the CPU baseline)."""
    lib().orc_set_threads(int(n))


def get_threads():
    return int(lib().orc_get_threads())


def material_params(m) -> np.ndarray:
    kind = m["kind"]
    if kind == "ideal":
        return _arr([m["gamma"]])
    if kind == "stiffened":
        return _arr([m["gamma"], m["pinf"]])
    return _arr([m["rho0"], m["K0"], m["G0"], m["alpha"], m["beta"], m["Gamma0"], m.get("sigY", 0.0)])


class Oracle:
    """One oracle instance of a :class:`paper_2111_11806_amd.inputs.Problem`."""

    def __init__(self, prob, variant=None):
        L = lib(variant)
        self._L = L
        d = _Desc()
        d.dim = prob.dim
        d.nx, d.ny, d.nz = prob.n
        for a in range(3):
            d.dx[a] = prob.dx[a]
            d.origin[a] = prob.origin[a]
        d.nmat = len(prob.materials)
        d.solid = int(prob.solid)
        for q in range(6):
            d.bc[q] = BC[prob.bc[q]]
        d.recon = RECON[prob.recon]
        d.riemann = RIEMANN[prob.riemann]
        d.seed = SEED[prob.seed]
        d.probe = PROBE[prob.probe]
        d.plastic = int(prob.plastic)
        d.thinc_beta = prob.thinc_beta
        d.lm_mach = prob.lm_mach
        d.normal = NORMAL[prob.normal]
        self._h = L.orc_create(ctypes.byref(d))
        if not self._h:
            raise RuntimeError("orc_create failed")
        self.prob = prob
        self.nf = L.orc_nfields(self._h)
        assert self.nf == prob.nfields, (self.nf, prob.nfields)
        for l, m in enumerate(prob.materials):
            L.orc_set_material(self._h, l, EOS[m["kind"]], _dp(material_params(m)))
        for face, W in prob.bc_states.items():
            L.orc_set_bc_state(self._h, face, _dp(_arr(W, self.nf)))
        self.set_state_prim(prob.W0)
        if prob.sdf is not None:
            self.set_rigid_sdf(prob.sdf, prob.width, prob.v_r, prob.omega, prob.center)
        if prob.bodies:
            self.set_rigid_bodies(*prob.body_table())
        if prob.gap_gas is not None:
            self.set_face_mod(1, prob.gap_gas)

    def set_face_mod(self, mode, gap_gas=None):
        """Void-opening face modifier at solid-rigid faces: mode 0 off, 1 on;
        gap_gas: primitive state of the gas that fills an opening gap."""
        W = None if gap_gas is None else _dp(_arr(gap_gas, self.nf))
        if self._L.orc_set_face_mod(self._h, int(mode), W) != 0:
            raise ValueError("orc_set_face_mod: mode must be 0 or 1")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.orc_destroy(h)
            self._h = None

    @property
    def shape(self):
        nx, ny, nz = self.prob.n
        return (self.nf, nz, ny, nx)

    def set_state_prim(self, W):
        self._L.orc_set_state_prim(self._h, _dp(_arr(W, int(np.prod(self.shape)))))

    def set_state_cons(self, U):
        self._L.orc_set_state_cons(self._h, _dp(_arr(U, int(np.prod(self.shape)))))

    def get_state_prim(self):
        out = np.empty(self.shape)
        self._L.orc_get_state_prim(self._h, _dp(out))
        return out

    def get_state_cons(self):
        out = np.empty(self.shape)
        self._L.orc_get_state_cons(self._h, _dp(out))
        return out

    def set_rigid_sdf(self, sdf, width, v, omega, center):
        sdf = _arr(sdf, int(np.prod(self.shape[1:])))
        self._L.orc_set_rigid_sdf(self._h, _dp(sdf), float(width), _dp(_arr(v, 3)), _dp(_arr(omega, 3)),
                                _dp(_arr(center, 3)))

    def set_rigid_motion(self, v, omega, center):
        self._L.orc_set_rigid_motion(self._h, _dp(_arr(v, 3)), _dp(_arr(omega, 3)), _dp(_arr(center, 3)))

    def set_rigid_bodies(self, v, omega, center, box_lo, box_hi):
        """Motions of several bodies (rows: body 0 = every point no other
        body owns, bodies 1.. with ownership boxes [box_lo, box_hi))."""
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
        nb = v.shape[0]
        a = [np.ascontiguousarray(x, dtype=np.float64).reshape(nb, 3) for x in (v, omega, center, box_lo, box_hi)]
        rc = self._L.orc_set_rigid_bodies(self._h, nb, *[_dp(x) for x in a])
        if rc != 0:
            raise ValueError("orc_set_rigid_bodies: nbody must be 1..4")

    def compute_dt(self, cfl):
        return self._L.orc_compute_dt(self._h, float(cfl))

    def step(self, dt):
        self._L.orc_step(self._h, float(dt))

    def seed(self):
        self._L.orc_seed(self._h)

    def rhs(self, dirmask=7):
        """D(U) of the current state (no seeding; rigid mask from r)."""
        out = np.empty(self.shape)
        self._L.orc_rhs(self._h, _dp(out), int(dirmask))
        return out

    @property
    def t(self):
        return self._L.orc_time(self._h)

    def stats(self):
        out = (ctypes.c_long * 3)()
        self._L.orc_stats(self._h, out)
        return {"seeded": out[0], "probe_fail": out[1], "fallback": out[2]}

    def rigid_force(self, center):
        F = np.zeros(3)
        T = np.zeros(3)
        self._L.orc_rigid_force(self._h, _dp(_arr(center, 3)), _dp(F), _dp(T))
        return F, T

    def conserved_totals(self):
        out = np.zeros(2 * self.nf)
        self._L.orc_conserved_totals(self._h, _dp(out))
        return out[: self.nf], out[self.nf:]

    def run(self, t_end=None, cfl=None, nsteps=None, dts=None, progress=None):
        """Advance with the CFL step (clipped to t_end) and return the dt list.
        progress: optional callable(steps done, t), called about every 30 s."""
        out = []
        last = [time.perf_counter()]

        def tick():
            if progress is not None and time.perf_counter() - last[0] > 30.0:
                last[0] = time.perf_counter()
                progress(len(out), self.t)
        if dts is not None:
            for dt in dts:
                self.step(dt)
                out.append(dt)
                tick()
            return out
        cfl = self.prob.cfl if cfl is None else cfl
        t_end = self.prob.t_end if t_end is None else t_end
        k = 0
        while (nsteps is None or k < nsteps) and self.t < t_end * (1 - 1e-14):
            dt = min(self.compute_dt(cfl), t_end - self.t)
            self.step(dt)
            out.append(dt)
            k += 1
            tick()
        return out

    # ---- unit-level access used by the pins ----
    def candidates(self, qm, q0, qp):
        out = np.zeros(4)
        self._L.orc_candidates(self._h, qm, q0, qp, _dp(out))
        return out

    def bvd_select(self, cm, c0, cp):
        """Faces (left, right) BVD selects for a cell from the candidate
        quadruples of its left neighbour, itself and its right neighbour."""
        out = np.zeros(2)
        self._L.orc_bvd_select(self._h, _dp(_arr(cm, 4)), _dp(_arr(c0, 4)), _dp(_arr(cp, 4)), _dp(out))
        return out

    def prim_to_cons(self, W):
        U = np.zeros(self.nf)
        self._L.orc_prim_to_cons(self._h, _dp(_arr(W, self.nf)), _dp(U))
        return U

    def cons_to_prim(self, U):
        W = np.zeros(self.nf)
        self._L.orc_cons_to_prim(self._h, _dp(_arr(U, self.nf)), _dp(W))
        return W

    def thermo(self, W):
        out = np.zeros(24)
        self._L.orc_thermo(self._h, _dp(_arr(W, self.nf)), _dp(out))
        return {"rho": out[0], "p": out[1], "c2": out[2], "G": out[3], "sigY": out[4], "J2": out[5],
                "sigma": out[6:15].reshape(3, 3), "H": out[15:24].reshape(3, 3)}

    def face_flux(self, WL, WR, d):
        out = np.zeros(self.nf + 3)
        self._L.orc_face_flux(self._h, _dp(_arr(WL, self.nf)), _dp(_arr(WR, self.nf)), int(d), _dp(out))
        nt = self.nf - 1
        return out[:nt], out[nt], out[nt + 1: nt + 4]

    def phys_flux(self, W, d):
        F = np.zeros(self.nf)
        self._L.orc_phys_flux(self._h, _dp(_arr(W, self.nf)), int(d), _dp(F))
        return F[: self.nf - 1]

    def mirror_state(self, W, nrm, v):
        out = np.zeros(self.nf)
        self._L.orc_mirror_state(self._h, _dp(_arr(W, self.nf)), _dp(_arr(nrm, 3)), _dp(_arr(v, 3)), _dp(out))
        return out

    def riemann_seed_state(self, Wm, Wi, nrm):
        out = np.zeros(self.nf)
        self._L.orc_riemann_seed_state(self._h, _dp(_arr(Wm, self.nf)), _dp(_arr(Wi, self.nf)),
                                     _dp(_arr(nrm, 3)), _dp(out))
        return out

    def solid_sources(self, U):
        U = _arr(U, self.nf).copy()
        self._L.orc_solid_sources(self._h, _dp(U))
        return U


def hencky(V):
    V = _arr(V, 9)
    H = np.zeros(9)
    lib().orc_hencky(_dp(V), _dp(H))
    return H.reshape(3, 3)


def phase_ref(material, rho, J2=0.0):
    out = np.zeros(5)
    lib().orc_phase_ref(EOS[material["kind"]], _dp(material_params(material)), float(rho), float(J2), _dp(out))
    return {"rhoe_ref": out[0], "p_ref": out[1], "Gamma": out[2], "dpref_drho": out[3], "G": out[4]}
