"""ctypes binding of the AGIS CPU oracle -- TEST INFRASTRUCTURE ONLY.

The oracle (``agis_oracle.c``) is a plain double-precision CPU implementation
of the source, attitude and calibration updating blocks and the frame rotator
of the Gaia astrometric core solution, written from the paper.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may use it;
the GPU library never loads, calls or links it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
P = ctypes.POINTER
c_d, c_i64, c_i32, c_i8, c_f = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_int8, ctypes.c_float


class World(ctypes.Structure):
    _fields_ = [("n_knots", c_i64), ("knots", P(c_d)), ("gamma_c", c_d), ("t_ep", c_d), ("t_fr", c_d),
                ("lambda_reg", c_d), ("seg_len", c_i32), ("seg_overlap", c_i32), ("eph_radius_au", c_d),
                ("eph_L0", c_d), ("eph_Lrate", c_d), ("eps_obl", c_d), ("au_m", c_d), ("c_mps", c_d),
                ("year_s", c_d)]


class Obs(ctypes.Structure):
    _fields_ = [("n", c_i64), ("t", P(c_d)), ("eta_obs", P(c_d)), ("sigma", P(c_f)), ("src", P(c_i32)),
                ("fov", P(c_i8)), ("cell", P(c_i32))]


class State(ctypes.Structure):
    _fields_ = [("n_src", c_i64), ("n_att", c_i64), ("n_cells", c_i64), ("s", P(c_d)), ("a", P(c_d)),
                ("c", P(c_d))]


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "agis_oracle.c")
    hdr = os.path.join(_HERE, "agis_oracle.h")
    newest = max(os.path.getmtime(src), os.path.getmtime(hdr))
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c99", "-D_DEFAULT_SOURCE", "-O2", "-fno-fast-math",
                               "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_qmul.argtypes = [P(c_d), P(c_d), P(c_d)]
        L.orc_qconj.argtypes = [P(c_d), P(c_d)]
        L.orc_qinv.argtypes = [P(c_d), P(c_d)]
        L.orc_frame_rotate.argtypes = [P(c_d), P(c_d), P(c_d)]
        L.orc_vector_rotate.argtypes = [P(c_d), P(c_d), P(c_d)]
        L.orc_quat2mat.argtypes = [P(c_d), P(c_d)]
        L.orc_qrot.argtypes = [P(c_d), P(c_d)]
        L.orc_left_index.argtypes = [P(c_d), c_i64, c_d]
        L.orc_left_index.restype = c_i64
        L.orc_bspline.argtypes = [P(c_d), c_i64, c_d, P(c_d)]
        L.orc_chol_c1.argtypes = [P(c_d), ctypes.c_int]
        L.orc_chol_c1.restype = ctypes.c_int
        L.orc_chol_c2.argtypes = [P(c_d), ctypes.c_int, P(c_d)]
        L.orc_chol_c3.argtypes = [P(c_d), ctypes.c_int, P(c_d)]
        L.orc_band_c1.argtypes = [P(c_d), ctypes.c_int, ctypes.c_int]
        L.orc_band_c1.restype = ctypes.c_int
        L.orc_band_c2.argtypes = [P(c_d), ctypes.c_int, ctypes.c_int, P(c_d)]
        L.orc_band_c3.argtypes = [P(c_d), ctypes.c_int, ctypes.c_int, P(c_d)]
        L.orc_observe.argtypes = [P(World), P(Obs), P(State), c_i64, c_i64, P(c_d), P(c_d), P(c_d), P(c_i8),
                                  P(c_d), P(c_d), P(c_d), P(c_d), P(c_i64), P(c_d), P(c_d)]
        L.orc_ephemeris.argtypes = [P(World), c_d, P(c_d), P(c_d)]
        L.orc_normal_triad.argtypes = [c_d, c_d, P(c_d), P(c_d), P(c_d)]
        L.orc_source_update.argtypes = [P(World), P(Obs), P(State), P(c_d), P(c_d), P(c_i32), P(c_d)]
        L.orc_attitude_update.argtypes = [P(World), P(Obs), P(State), P(c_d)]
        L.orc_attitude_update.restype = c_i64
        L.orc_attitude_segment.argtypes = [P(World), P(Obs), P(State), c_i64, P(c_d), P(c_i64), P(c_i64)]
        L.orc_attitude_segment.restype = c_i64
        L.orc_num_segments.argtypes = [P(World)]
        L.orc_num_segments.restype = c_i64
        L.orc_calibration_update.argtypes = [P(World), P(Obs), P(State), P(c_d)]
        L.orc_iterate_sac.argtypes = [P(World), P(Obs), P(State), P(c_d)]
        L.orc_frame_fit.argtypes = [P(World), P(State), P(c_d), P(c_d), P(c_d)]
        L.orc_frame_apply.argtypes = [P(World), P(State), P(c_d)]
        _lib = L
    return _lib


def _p(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(P(ct))


def _vec(x, n=None):
    a = np.ascontiguousarray(x, dtype=np.float64)
    if n is not None:
        assert a.size == n
    return a


# --- small math helpers ----------------------------------------------------
def qmul(a, b):
    a, b = _vec(a, 4), _vec(b, 4)
    o = np.empty(4)
    lib().orc_qmul(_p(a, c_d), _p(b, c_d), _p(o, c_d))
    return o


def qconj(a):
    a = _vec(a, 4); o = np.empty(4)
    lib().orc_qconj(_p(a, c_d), _p(o, c_d))
    return o


def qinv(a):
    a = _vec(a, 4); o = np.empty(4)
    lib().orc_qinv(_p(a, c_d), _p(o, c_d))
    return o


def frame_rotate(q, v):
    q, v = _vec(q, 4), _vec(v, 3); o = np.empty(3)
    lib().orc_frame_rotate(_p(q, c_d), _p(v, c_d), _p(o, c_d))
    return o


def vector_rotate(q, v):
    q, v = _vec(q, 4), _vec(v, 3); o = np.empty(3)
    lib().orc_vector_rotate(_p(q, c_d), _p(v, c_d), _p(o, c_d))
    return o


def quat2mat(q):
    q = _vec(q, 4); o = np.empty(9)
    lib().orc_quat2mat(_p(q, c_d), _p(o, c_d))
    return o.reshape(3, 3)


def qrot(phi):
    phi = _vec(phi, 3); o = np.empty(4)
    lib().orc_qrot(_p(phi, c_d), _p(o, c_d))
    return o


def left_index(knots, t):
    k = _vec(knots)
    return int(lib().orc_left_index(_p(k, c_d), k.size, float(t)))


def bspline(knots, ell, t):
    k = _vec(knots); o = np.empty(4)
    lib().orc_bspline(_p(k, c_d), int(ell), float(t), _p(o, c_d))
    return o


def chol_solve(N, b):
    """Algorithms C1-C3 on a dense matrix: returns (U, x, defect)."""
    n = N.shape[0]
    U = np.ascontiguousarray(N, dtype=np.float64).copy()
    x = _vec(b).copy()
    d = lib().orc_chol_c1(_p(U, c_d), n)
    lib().orc_chol_c2(_p(U, c_d), n, _p(x, c_d))
    lib().orc_chol_c3(_p(U, c_d), n, _p(x, c_d))
    return U, x, d


def band_solve(UB, b, hb):
    n = UB.shape[0]
    U = np.ascontiguousarray(UB, dtype=np.float64).copy()
    x = _vec(b).copy()
    d = lib().orc_band_c1(_p(U, c_d), n, hb)
    lib().orc_band_c2(_p(U, c_d), n, hb, _p(x, c_d))
    lib().orc_band_c3(_p(U, c_d), n, hb, _p(x, c_d))
    return U, x, d


def normal_triad(alpha, delta):
    p, q, r = np.empty(3), np.empty(3), np.empty(3)
    lib().orc_normal_triad(float(alpha), float(delta), _p(p, c_d), _p(q, c_d), _p(r, c_d))
    return p, q, r


# --- problem wrapper --------------------------------------------------------
class Problem:
    """Holds the world constants, observations and a mutable state (s, a, c).

    ``consts`` keys: gamma_c, t_ep, t_fr, lambda_reg, seg_len, seg_overlap,
    eph_radius_au, eph_L0, eph_Lrate, eps_obl, au_m, c_mps, year_s.
    """

    def __init__(self, consts, knots, t, eta_obs, sigma, src, fov, cell, s, a, c):
        self.knots = _vec(knots)
        self.t = _vec(t)
        self.eta_obs = _vec(eta_obs)
        self.sigma = np.ascontiguousarray(sigma, dtype=np.float32)
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.fov = np.ascontiguousarray(fov, dtype=np.int8)
        self.cell = np.ascontiguousarray(cell, dtype=np.int32)
        self.s = np.ascontiguousarray(s, dtype=np.float64).copy()
        self.a = np.ascontiguousarray(a, dtype=np.float64).copy()
        self.c = np.ascontiguousarray(c, dtype=np.float64).copy()
        self.consts = dict(consts)
        self.world = World(n_knots=self.knots.size, knots=_p(self.knots, c_d), gamma_c=consts["gamma_c"],
                           t_ep=consts["t_ep"], t_fr=consts["t_fr"], lambda_reg=consts["lambda_reg"],
                           seg_len=int(consts["seg_len"]), seg_overlap=int(consts["seg_overlap"]),
                           eph_radius_au=consts["eph_radius_au"], eph_L0=consts["eph_L0"],
                           eph_Lrate=consts["eph_Lrate"], eps_obl=consts["eps_obl"], au_m=consts["au_m"],
                           c_mps=consts["c_mps"], year_s=consts["year_s"])
        self._refresh()

    def _refresh(self):
        self.obs = Obs(n=self.t.size, t=_p(self.t, c_d), eta_obs=_p(self.eta_obs, c_d), sigma=_p(self.sigma, c_f),
                       src=_p(self.src, c_i32), fov=_p(self.fov, c_i8), cell=_p(self.cell, c_i32))
        self.state = State(n_src=self.s.shape[0], n_att=self.a.shape[0], n_cells=self.c.size,
                           s=_p(self.s, c_d), a=_p(self.a, c_d), c=_p(self.c, c_d))

    def set_eta_obs(self, eta_obs):
        self.eta_obs = _vec(eta_obs).copy()
        self._refresh()

    def set_state(self, s=None, a=None, c=None):
        if s is not None:
            self.s = np.ascontiguousarray(s, dtype=np.float64).copy()
        if a is not None:
            self.a = np.ascontiguousarray(a, dtype=np.float64).copy()
        if c is not None:
            self.c = np.ascontiguousarray(c, dtype=np.float64).copy()
        self._refresh()

    def observe(self, i0=0, i1=None, partials=False):
        n = self.t.size
        i1 = n if i1 is None else i1
        out = dict(eta=np.zeros(n), phi=np.zeros(n), zeta=np.zeros(n), f=np.zeros(n, np.int8), R=np.zeros(n),
                   bspl=np.zeros((n, 4)), ell=np.zeros(n, np.int64), qraw=np.zeros((n, 4)), D=np.zeros(n))
        if partials:
            out["dsrc"] = np.zeros((n, 5))
            out["dq"] = np.zeros((n, 4))
        lib().orc_observe(ctypes.byref(self.world), ctypes.byref(self.obs), ctypes.byref(self.state), i0, i1,
                          _p(out["eta"], c_d), _p(out["phi"], c_d), _p(out["zeta"], c_d), _p(out["f"], c_i8),
                          _p(out["R"], c_d), _p(out.get("dsrc"), c_d), _p(out.get("dq"), c_d),
                          _p(out["bspl"], c_d), _p(out["ell"], c_i64), _p(out["qraw"], c_d), _p(out["D"], c_d))
        return out

    def ephemeris(self, t):
        b, v = np.empty(3), np.empty(3)
        lib().orc_ephemeris(ctypes.byref(self.world), float(t), _p(b, c_d), _p(v, c_d))
        return b, v

    def source_update(self):
        ns = self.s.shape[0]
        d, Q, de = np.zeros((ns, 5)), np.zeros(ns), np.zeros(ns, np.int32)
        self.var = np.zeros((ns, 5))
        lib().orc_source_update(ctypes.byref(self.world), ctypes.byref(self.obs), ctypes.byref(self.state),
                                _p(d, c_d), _p(Q, c_d), _p(de, c_i32), _p(self.var, c_d))
        return d, Q, de

    def attitude_update(self):
        d = np.zeros_like(self.a)
        de = lib().orc_attitude_update(ctypes.byref(self.world), ctypes.byref(self.obs), ctypes.byref(self.state),
                                       _p(d, c_d))
        return d, int(de)

    def attitude_segment(self, K):
        d = np.full_like(self.a, np.nan)
        lo, hi = c_i64(), c_i64()
        de = lib().orc_attitude_segment(ctypes.byref(self.world), ctypes.byref(self.obs), ctypes.byref(self.state),
                                        int(K), _p(d, c_d), ctypes.byref(lo), ctypes.byref(hi))
        return d, int(de), lo.value, hi.value

    def num_segments(self):
        return int(lib().orc_num_segments(ctypes.byref(self.world)))

    def calibration_update(self):
        d = np.zeros_like(self.c)
        lib().orc_calibration_update(ctypes.byref(self.world), ctypes.byref(self.obs), ctypes.byref(self.state),
                                     _p(d, c_d))
        return d

    def iterate_sac(self):
        self.var = np.zeros((self.s.shape[0], 5))
        lib().orc_iterate_sac(ctypes.byref(self.world), ctypes.byref(self.obs), ctypes.byref(self.state),
                              _p(self.var, c_d))

    def frame_fit(self, s_ref, weighted=True):
        """Frame rotator fit; weighted by the variances of the last S update
        (unit weights before any, or with weighted=False)."""
        s_ref = np.ascontiguousarray(s_ref, dtype=np.float64)
        eo = np.zeros(6)
        var = getattr(self, "var", None) if weighted else None
        lib().orc_frame_fit(ctypes.byref(self.world), ctypes.byref(self.state), _p(s_ref, c_d), _p(var, c_d),
                            _p(eo, c_d))
        return eo

    def frame_apply(self, eo):
        eo = _vec(eo, 6)
        lib().orc_frame_apply(ctypes.byref(self.world), ctypes.byref(self.state), _p(eo, c_d))

    def iterate(self, s_ref=None):
        """One S[AC] iteration, then (if s_ref is given) the frame rotator."""
        self.iterate_sac()
        if s_ref is not None:
            eo = self.frame_fit(s_ref)
            self.frame_apply(eo)
            return eo
        return None


def problem_from_world(world, eta_obs=None, state="start"):
    """Build a Problem from a synth.World; eta_obs defaults to zeros."""
    n = world.t.size
    eta = np.zeros(n) if eta_obs is None else eta_obs
    if state == "start":
        s, a, c = world.src_start, world.att_start, world.cal_start
    else:
        s, a, c = world.src_true, world.att_true, world.cal_true
    return Problem(world.consts, world.knots, world.t, eta, world.sigma, world.src, world.fov, world.cell, s, a, c)


def observed_field_angles(world):
    """eta_obs = eta(t | s_true, a_true) - c_true(cell) + noise (Sect. 3.5 at the truth)."""
    pr = problem_from_world(world, eta_obs=None, state="truth")
    out = pr.observe()
    return out["eta"] - world.cal_true[world.cell] + world.eps
