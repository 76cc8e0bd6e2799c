"""Thin ctypes binding of librbdi (include/rbdi.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library. The names follow the C entry points. Loading fails loudly if
the library has not been built (``paper_2111_11806_amd.build.build()``);
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

EOS = {"ideal": 0, "stiffened": 1, "romenskii": 2}
BC = {"transmissive": 0, "reflective": 1, "dirichlet": 2, "periodic": 3}
RECON = {"muscl": 0, "bvd_thinc": 1}
RIEMANN = {"hllc": 0, "hllc_lm": 1}
SEED = {"original": 0, "riemann": 1, "none": 2}
PROBE = {"stepout": 0, "fixed": 1}
NORMAL = {"youngs": 0, "elvira": 1}
PRECISION = {"fp64": 0, "fp32": 1}

RBDI_OK = 0
RBDI_ERR_NONPHYSICAL = -4


class RbdiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rbdi error {code}: {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("dx", ctypes.c_double * 3),
                ("origin", ctypes.c_double * 3), ("nmat", ctypes.c_int), ("solid", ctypes.c_int),
                ("bc", ctypes.c_int * 6), ("recon", ctypes.c_int), ("riemann", ctypes.c_int),
                ("seed", ctypes.c_int), ("probe", ctypes.c_int), ("plastic", ctypes.c_int),
                ("thinc_beta", ctypes.c_double), ("lm_mach", ctypes.c_double), ("precision", ctypes.c_int),
                ("normal", ctypes.c_int)]


class Eos(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("gamma", ctypes.c_double), ("pinf", ctypes.c_double),
                ("rho0", ctypes.c_double), ("K0", ctypes.c_double), ("G0", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("Gamma0", ctypes.c_double),
                ("sigma_y", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("x_waves", ctypes.c_int), ("x_blocks", ctypes.c_int), ("x_xcd", ctypes.c_int),
                ("tile_cols", ctypes.c_int), ("t_blocks", ctypes.c_int), ("t_xcd", ctypes.c_int),
                ("x_us", ctypes.c_double), ("t_us", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_longlong), ("t", ctypes.c_double), ("last_dt", ctypes.c_double),
                ("band_cells", ctypes.c_longlong), ("seeded", ctypes.c_longlong),
                ("probe_fail", ctypes.c_longlong), ("nonphysical", ctypes.c_int), ("first_bad", ctypes.c_longlong),
                ("surr_net", ctypes.c_longlong), ("surr_exact", ctypes.c_longlong)]


_lib = None

EXPORTS = ["rbdi_create", "rbdi_destroy", "rbdi_nfields", "rbdi_set_stream", "rbdi_set_material",
           "rbdi_set_bc_state", "rbdi_set_state_prim", "rbdi_get_state_prim", "rbdi_get_state_cons",
           "rbdi_set_state_cons", "rbdi_set_rigid_sdf", "rbdi_set_rigid_motion", "rbdi_set_rigid_bodies", "rbdi_set_face_modifier",
           "rbdi_compute_dt",
           "rbdi_step", "rbdi_advance", "rbdi_status", "rbdi_rigid_force", "rbdi_conserved_totals",
           "rbdi_last_error", "rbdi_set_kernel_timing", "rbdi_kernel_times", "rbdi_unit_eval", "rbdi_eval_rhs",
           "rbdi_set_x_waves", "rbdi_autotune",
           "rbdi_kernel_replay",
           "rbdi_batch_create", "rbdi_batch_destroy", "rbdi_batch_set_stream", "rbdi_batch_set_tuning",
           "rbdi_batch_get_tuning", "rbdi_batch_autotune", "rbdi_batch_step", "rbdi_batch_advance",
           "rbdi_mlp_create", "rbdi_mlp_destroy", "rbdi_mlp_set_params", "rbdi_mlp_get_params", "rbdi_mlp_data",
           "rbdi_mlp_forward", "rbdi_mlp_grad", "rbdi_mlp_grad_noalloc", "rbdi_mlp_train", "rbdi_set_surrogate"]
NUM_KCLASS = 7
KCLASS = ["sweep_x", "sweep_y", "sweep_z", "seed", "band", "cfl_dt", "sources_mlp"]
N_MLP_PARAMS = 9158
MLP_GRAD_NOALLOC_MAX = 16384  # RBDI_MLP_GRAD_NOALLOC_MAX


def lib_path():
    return _build.LIB


def load():
    """Load librbdi.so (built in-tree). Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"librbdi is not built ({path}); run paper_2111_11806_amd.build.build()")
    L = ctypes.CDLL(path)
    vp, ip, dp, cp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_char_p
    L.rbdi_create.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(vp)]
    L.rbdi_destroy.argtypes = [vp]
    L.rbdi_nfields.argtypes = [vp]
    L.rbdi_set_stream.argtypes = [vp, vp]
    L.rbdi_set_material.argtypes = [vp, ip, ctypes.POINTER(Eos)]
    L.rbdi_set_bc_state.argtypes = [vp, ip, dp]
    for nm in ("rbdi_set_state_prim", "rbdi_get_state_prim", "rbdi_get_state_cons", "rbdi_set_state_cons"):
        getattr(L, nm).argtypes = [vp, vp, ip]
    L.rbdi_set_rigid_sdf.argtypes = [vp, vp, ip, ctypes.c_double, dp, dp, dp]
    L.rbdi_set_rigid_motion.argtypes = [vp, dp, dp, dp]
    L.rbdi_set_rigid_bodies.argtypes = [vp, ip, dp, dp, dp, dp, dp]
    L.rbdi_set_face_modifier.argtypes = [vp, ip, dp]
    L.rbdi_compute_dt.argtypes = [vp, ctypes.c_double, dp]
    L.rbdi_step.argtypes = [vp, ctypes.c_double]
    L.rbdi_advance.argtypes = [vp, ctypes.c_double, ip, ctypes.c_double]
    L.rbdi_status.argtypes = [vp, ctypes.POINTER(Stats)]
    L.rbdi_rigid_force.argtypes = [vp, dp, dp, dp]
    L.rbdi_conserved_totals.argtypes = [vp, dp]
    L.rbdi_last_error.restype = cp
    L.rbdi_set_kernel_timing.argtypes = [vp, ip]
    L.rbdi_kernel_times.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong)]
    L.rbdi_unit_eval.argtypes = [vp, ip, ip, dp, dp, dp, ip]
    L.rbdi_eval_rhs.argtypes = [vp, ip, dp]
    L.rbdi_kernel_replay.argtypes = [vp, ip, ip, dp]
    L.rbdi_set_x_waves.argtypes = [vp, ip]
    L.rbdi_autotune.argtypes = [vp, ctypes.c_double, ip, ctypes.POINTER(ctypes.c_int), dp]
    L.rbdi_batch_create.argtypes = [ip, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    L.rbdi_batch_destroy.argtypes = [vp]
    L.rbdi_batch_set_stream.argtypes = [vp, vp]
    L.rbdi_batch_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.rbdi_batch_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.rbdi_batch_autotune.argtypes = [vp, ip, ctypes.POINTER(Tuning)]
    L.rbdi_batch_step.argtypes = [vp, ctypes.c_double, dp]
    L.rbdi_batch_advance.argtypes = [vp, ctypes.c_double, ip, ctypes.c_double]
    fp = ctypes.POINTER(ctypes.c_float)
    L.rbdi_mlp_create.argtypes = [ctypes.POINTER(vp)]
    L.rbdi_mlp_destroy.argtypes = [vp]
    L.rbdi_mlp_set_params.argtypes = [vp, fp, ctypes.c_double]
    L.rbdi_mlp_get_params.argtypes = [vp, fp, dp]
    L.rbdi_mlp_data.argtypes = [dp, ip, ctypes.c_double, fp, fp]
    L.rbdi_mlp_forward.argtypes = [vp, fp, ip, fp]
    L.rbdi_mlp_grad.argtypes = [vp, fp, fp, ip, fp, fp]
    L.rbdi_mlp_grad_noalloc.argtypes = [vp, vp, vp, ip, vp, vp, vp]
    L.rbdi_mlp_train.argtypes = [vp, fp, fp, ip, ip, ip, ctypes.c_float, fp]
    L.rbdi_set_surrogate.argtypes = [vp, vp]
    _lib = L
    return L


def _check(rc):
    if rc != RBDI_OK:
        raise RbdiError(rc, load().rbdi_last_error().decode())
    return rc


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def make_eos(m) -> Eos:
    e = Eos()
    e.kind = EOS[m["kind"]]
    if m["kind"] in ("ideal", "stiffened"):
        e.gamma = m["gamma"]
        e.pinf = m.get("pinf", 0.0)
    else:
        e.rho0, e.K0, e.G0 = m["rho0"], m["K0"], m["G0"]
        e.alpha, e.beta, e.Gamma0 = m["alpha"], m["beta"], m["Gamma0"]
        e.sigma_y = m.get("sigY", 0.0)
    return e


def make_desc(prob, precision="fp64") -> Desc:
    d = Desc()
    d.dim = prob.dim
    for a in range(3):
        d.n[a] = prob.n[a]
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
    d.precision = PRECISION[precision]
    d.normal = NORMAL[prob.normal]
    return d


class Solver:
    """One librbdi instance of a :class:`paper_2111_11806_amd.inputs.Problem`."""

    def __init__(self, prob, precision="fp64", stream=None):
        L = load()
        h = ctypes.c_void_p()
        _check(L.rbdi_create(ctypes.byref(make_desc(prob, precision)), ctypes.byref(h)))
        self._h = h
        self.prob = prob
        self.precision = precision
        self.nf = L.rbdi_nfields(h)
        if stream is not None:
            self.set_stream(stream)
        for l, m in enumerate(prob.materials):
            _check(L.rbdi_set_material(h, l, ctypes.byref(make_eos(m))))
        for face, W in prob.bc_states.items():
            _check(L.rbdi_set_bc_state(h, face, _dp(_arr(W, self.nf))))
        self.set_state_prim(prob.W0)
        if prob.sdf is not None:
            self.set_rigid_sdf(prob.sdf, prob.width, prob.v_r, prob.omega, prob.center)
        if prob.bodies:
            self.set_rigid_bodies(*prob.body_table())
        if prob.gap_gas is not None:
            self.set_face_modifier(1, prob.gap_gas)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            load().rbdi_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        nx, ny, nz = self.prob.n
        return (self.nf, nz, ny, nx)

    def set_stream(self, stream):
        """stream: a torch.cuda.Stream, a raw hipStream_t integer, or None."""
        raw = getattr(stream, "cuda_stream", stream)
        _check(load().rbdi_set_stream(self._h, ctypes.c_void_p(raw or 0)))

    def set_state_prim(self, W):
        if hasattr(W, "data_ptr"):
            _check(load().rbdi_set_state_prim(self._h, ctypes.c_void_p(W.data_ptr()), 1))
        else:
            a = _arr(W, int(np.prod(self.shape)))
            _check(load().rbdi_set_state_prim(self._h, a.ctypes.data_as(ctypes.c_void_p), 0))

    def set_state_cons(self, U):
        a = _arr(U, int(np.prod(self.shape)))
        _check(load().rbdi_set_state_cons(self._h, a.ctypes.data_as(ctypes.c_void_p), 0))

    def get_state_prim(self):
        out = np.empty(self.shape)
        _check(load().rbdi_get_state_prim(self._h, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def get_state_cons(self):
        out = np.empty(self.shape)
        _check(load().rbdi_get_state_cons(self._h, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def get_state_cons_device(self, ptr):
        """Conserved state into FP64 device memory at ptr (shape self.shape)."""
        _check(load().rbdi_get_state_cons(self._h, ctypes.c_void_p(int(ptr)), 1))

    def set_state_cons_device(self, ptr):
        """Conserved state from FP64 device memory at ptr (shape self.shape)."""
        _check(load().rbdi_set_state_cons(self._h, ctypes.c_void_p(int(ptr)), 1))

    def set_rigid_sdf(self, sdf, width, v, omega, center):
        a = _arr(sdf, int(np.prod(self.shape[1:])))
        _check(load().rbdi_set_rigid_sdf(self._h, a.ctypes.data_as(ctypes.c_void_p), 0, float(width),
                                         _dp(_arr(v, 3)), _dp(_arr(omega, 3)), _dp(_arr(center, 3))))

    def set_rigid_motion(self, v, omega, center):
        _check(load().rbdi_set_rigid_motion(self._h, _dp(_arr(v, 3)), _dp(_arr(omega, 3)), _dp(_arr(center, 3))))

    def set_rigid_bodies(self, v, omega, center, box_lo, box_hi):
        """Motions of several bodies: rows of v, omega, center (body 0 moves
        every point no other body owns) and of the ownership boxes
        [box_lo, box_hi) of bodies 1.. (row 0 ignored)."""
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
        nb = v.shape[0]
        a = [np.ascontiguousarray(x, dtype=np.float64).reshape(nb, 3) for x in (v, omega, center, box_lo, box_hi)]
        _check(load().rbdi_set_rigid_bodies(self._h, nb, *[_dp(x) for x in a]))

    def set_face_modifier(self, mode, gap_gas=None):
        """Void-opening face modifier at solid-rigid faces: mode 0 off, 1 on;
        gap_gas: primitive state of the gas that fills an opening gap."""
        W = None if gap_gas is None else _dp(_arr(gap_gas, self.nf))
        _check(load().rbdi_set_face_modifier(self._h, int(mode), W))

    def compute_dt(self, cfl):
        out = ctypes.c_double()
        _check(load().rbdi_compute_dt(self._h, float(cfl), ctypes.byref(out)))
        return out.value

    def step(self, dt):
        _check(load().rbdi_step(self._h, float(dt)))

    def advance(self, cfl, nsteps, t_end=0.0):
        _check(load().rbdi_advance(self._h, float(cfl), int(nsteps), float(t_end)))

    def status(self, raise_on_error=True):
        st = Stats()
        rc = load().rbdi_status(self._h, ctypes.byref(st))
        if rc != RBDI_OK and (raise_on_error or rc != RBDI_ERR_NONPHYSICAL):
            _check(rc)
        return {k: getattr(st, k) for k, _ in Stats._fields_}

    @property
    def t(self):
        return self.status(raise_on_error=False)["t"]

    def rigid_force(self, center):
        F = np.zeros(3)
        T = np.zeros(3)
        _check(load().rbdi_rigid_force(self._h, _dp(_arr(center, 3)), _dp(F), _dp(T)))
        return F, T

    def conserved_totals(self):
        out = np.zeros(2 * self.nf)
        _check(load().rbdi_conserved_totals(self._h, _dp(out)))
        return out[: self.nf], out[self.nf:]

    def set_kernel_timing(self, enable):
        _check(load().rbdi_set_kernel_timing(self._h, int(bool(enable))))

    def kernel_times(self):
        """{class: (total ms, launches)} of the launches recorded since the last call."""
        ms = np.zeros(NUM_KCLASS)
        n = (ctypes.c_longlong * NUM_KCLASS)()
        _check(load().rbdi_kernel_times(self._h, _dp(ms), n))
        return {KCLASS[c]: (float(ms[c]), int(n[c])) for c in range(NUM_KCLASS)}

    def kernel_replay(self, cls, reps=20):
        """Mean duration (us) of the x (0), y (1) or z (2) sweep of the middle
        RK stage, launched reps times back to back on the last step's buffers."""
        out = ctypes.c_double()
        _check(load().rbdi_kernel_replay(self._h, int(cls), int(reps), ctypes.byref(out)))
        return out.value

    def set_x_waves(self, waves):
        """Wavefronts per x-sweep block (1, 2, 4; 0 = the library's choice)."""
        _check(load().rbdi_set_x_waves(self._h, int(waves)))

    def autotune(self, cfl, nsteps=10):
        """Time nsteps steps per x-sweep block size from the current state
        (restored after each trial) and keep the fastest: (waves, us/step)."""
        best = ctypes.c_int()
        us = ctypes.c_double()
        _check(load().rbdi_autotune(self._h, ctypes.c_double(cfl), int(nsteps), ctypes.byref(best),
                                    ctypes.byref(us)))
        return best.value, us.value

    def eval_rhs(self, dirmask=7):
        """D(U) of the current state, [nf, nz, ny, nx], over the directions of
        dirmask (diagnostic)."""
        out = np.empty(self.shape)
        _check(load().rbdi_eval_rhs(self._h, int(dirmask), _dp(out)))
        return out

    def unit_flux(self, WL, WR, d):
        """HLLC flux of faces (n x nf primitive left/right states) along d:
        returns (F [n, nf-1], u* [n], Vbar* row [n, 3])."""
        WL = _arr(WL).reshape(-1, self.nf)
        WR = _arr(WR).reshape(-1, self.nf)
        n = WL.shape[0]
        out = np.zeros((n, self.nf + 3))
        _check(load().rbdi_unit_eval(self._h, 0, int(d), _dp(WL), _dp(WR), _dp(out), n))
        return out[:, : self.nf - 1], out[:, self.nf - 1], out[:, self.nf:]

    def unit_closure(self, U):
        """Closure of conserved states (n x nf): returns (W, c2, sigma [n,3,3])."""
        U = _arr(U).reshape(-1, self.nf)
        n = U.shape[0]
        out = np.zeros((n, self.nf + 10))
        _check(load().rbdi_unit_eval(self._h, 1, 0, _dp(U), _dp(U), _dp(out), n))
        return out[:, : self.nf], out[:, self.nf], out[:, self.nf + 1:].reshape(n, 3, 3)

    def unit_sources(self, U):
        U = _arr(U).reshape(-1, self.nf)
        out = np.zeros_like(U)
        _check(load().rbdi_unit_eval(self._h, 2, 0, _dp(U), _dp(U), _dp(out), U.shape[0]))
        return out

    def run(self, dts):
        for dt in dts:
            self.step(dt)

    def set_surrogate(self, mlp):
        """Close the elastoplastic sources with the network (None: exact)."""
        self._mlp = mlp
        _check(load().rbdi_set_surrogate(self._h, None if mlp is None else mlp._m))


def _tuning_dict(t):
    return {k: getattr(t, k) for k, _ in Tuning._fields_}


class Batch:
    """Many :class:`Solver` instances advanced together (rbdi_batch_*). The
    members stay readable through their own methods; stepping them on their
    own is refused while the batch exists."""

    def __init__(self, solvers, stream=None):
        L = load()
        self.members = list(solvers)
        arr = (ctypes.c_void_p * len(self.members))(*[m._h.value for m in self.members])
        b = ctypes.c_void_p()
        _check(L.rbdi_batch_create(len(self.members), arr, ctypes.byref(b)))
        self._b = b
        if stream is not None:
            self.set_stream(stream)

    def close(self):
        b = getattr(self, "_b", None)
        if b:
            load().rbdi_batch_destroy(b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        raw = getattr(stream, "cuda_stream", stream)
        _check(load().rbdi_batch_set_stream(self._b, ctypes.c_void_p(raw or 0)))

    def tuning(self):
        t = Tuning()
        _check(load().rbdi_batch_get_tuning(self._b, ctypes.byref(t)))
        return _tuning_dict(t)

    def set_tuning(self, **kw):
        t = Tuning()
        _check(load().rbdi_batch_get_tuning(self._b, ctypes.byref(t)))
        for k, v in kw.items():
            setattr(t, k, v)
        _check(load().rbdi_batch_set_tuning(self._b, ctypes.byref(t)))

    def autotune(self, reps=5):
        t = Tuning()
        _check(load().rbdi_batch_autotune(self._b, int(reps), ctypes.byref(t)))
        return _tuning_dict(t)

    def step(self, dts=None, cfl=0.0):
        """One step of every member: dts[i] > 0 fixed, <= 0 (or dts None) CFL."""
        if dts is None:
            _check(load().rbdi_batch_step(self._b, float(cfl), None))
        else:
            a = _arr(dts, len(self.members))
            _check(load().rbdi_batch_step(self._b, float(cfl), _dp(a)))

    def advance(self, cfl, nsteps, t_end=0.0):
        _check(load().rbdi_batch_advance(self._b, float(cfl), int(nsteps), float(t_end)))


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _f32(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def mlp_data(V, tau_max):
    """Features z and exact targets t (n x 6 each) of stretch tensors V (n x 9)."""
    V = _arr(V).reshape(-1, 9)
    n = V.shape[0]
    z = np.zeros((n, 6), np.float32)
    t = np.zeros((n, 6), np.float32)
    _check(load().rbdi_mlp_data(_dp(V), n, float(tau_max), _fp(z), _fp(t)))
    return z, t


class Mlp:
    """The surrogate network (rbdi_mlp_*)."""

    def __init__(self, params=None, tau_max=0.01):
        L = load()
        m = ctypes.c_void_p()
        _check(L.rbdi_mlp_create(ctypes.byref(m)))
        self._m = m
        if params is not None:
            self.set_params(params, tau_max)

    def close(self):
        m = getattr(self, "_m", None)
        if m:
            load().rbdi_mlp_destroy(m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, tau_max):
        _check(load().rbdi_mlp_set_params(self._m, _fp(_f32(params, N_MLP_PARAMS)), float(tau_max)))

    def params(self):
        p = np.zeros(N_MLP_PARAMS, np.float32)
        tm = ctypes.c_double()
        _check(load().rbdi_mlp_get_params(self._m, _fp(p), ctypes.byref(tm)))
        return p, tm.value

    def forward(self, z):
        z = _f32(z).reshape(-1, 6)
        y = np.zeros_like(z)
        _check(load().rbdi_mlp_forward(self._m, _fp(z), z.shape[0], _fp(y)))
        return y

    def grad(self, z, t):
        z = _f32(z).reshape(-1, 6)
        t = _f32(t).reshape(-1, 6)
        g = np.zeros(N_MLP_PARAMS, np.float32)
        loss = ctypes.c_float()
        _check(load().rbdi_mlp_grad(self._m, _fp(z), _fp(t), z.shape[0], _fp(g), ctypes.byref(loss)))
        return g, loss.value

    def grad_noalloc(self, z, t, grad, loss, stream=None):
        """rbdi_mlp_grad_noalloc on device tensors: z, t (n x 6 float32),
        grad (9158 float32) and loss (1 float32), all contiguous on the
        network's GPU; enqueued on stream (a torch stream, None = the null
        stream), no synchronisation."""
        for name, a, n in (("z", z, None), ("t", t, None), ("grad", grad, N_MLP_PARAMS), ("loss", loss, 1)):
            if not (a.is_cuda and a.dtype.is_floating_point and a.element_size() == 4 and a.is_contiguous()):
                raise ValueError(f"{name}: a contiguous float32 device tensor is required")
            if n is not None and a.numel() != n:
                raise ValueError(f"{name}: expected {n} values, got {a.numel()}")
        if z.numel() % 6 or z.numel() != t.numel():
            raise ValueError("z and t must both be n x 6")
        sp = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(load().rbdi_mlp_grad_noalloc(self._m, z.data_ptr(), t.data_ptr(), z.numel() // 6, grad.data_ptr(),
                                            loss.data_ptr(), sp))

    def train(self, z, t, batch=4096, iters=1000, lr=1e-3):
        z = _f32(z).reshape(-1, 6)
        t = _f32(t).reshape(-1, 6)
        losses = np.zeros(iters, np.float32)
        _check(load().rbdi_mlp_train(self._m, _fp(z), _fp(t), z.shape[0], int(batch), int(iters), float(lr),
                                     _fp(losses)))
        return losses
