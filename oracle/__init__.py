"""ctypes binding of the AGIS CPU oracle -- TEST INFRASTRUCTURE ONLY.

The oracle (``agis_oracle.c``) is a plain double-precision CPU implementation
of the source, attitude and calibration updating blocks and the frame rotator
of the Gaia astrometric core solution, written from the paper.  The same
source built in x87 extended precision serves as the reference against which
the FP64 rounding floor of any implementation is measured.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may use it;
the GPU library never loads, calls or links it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
P = ctypes.POINTER
c_d, c_i64, c_i32, c_i8, c_f = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_int8, ctypes.c_float

# Two builds of the same source: "double" (the oracle) and "extended" (x87
# 80-bit long double, the reference that the FP64 rounding floor is measured
# against).  name -> (ctypes real, numpy dtype, library file, extra flags)
PRECISIONS = {
    "double": (ctypes.c_double, np.float64, "liboracle.so", []),
    "extended": (ctypes.c_longdouble, np.longdouble, "liboracle_x.so", ["-DORC_EXTENDED"]),
}


def _structs(c_r):
    class World(ctypes.Structure):
        _fields_ = [("n_knots", c_i64), ("knots", P(c_r)), ("gamma_c", c_r), ("t_ep", c_r), ("t_fr", c_r),
                    ("lambda_reg", c_r), ("seg_len", c_i32), ("seg_overlap", c_i32), ("eph_radius_au", c_r),
                    ("eph_L0", c_r), ("eph_Lrate", c_r), ("eps_obl", c_r), ("au_m", c_r), ("c_mps", c_r),
                    ("year_s", c_r), ("robust", c_i32), ("eps_bucket", c_i32), ("geo_ccds", c_i32),
                    ("geo_ac_cells", c_i32), ("defl", c_r), ("ppn", c_i32), ("geo_small_days", c_i32)]

    class Obs(ctypes.Structure):
        _fields_ = [("n", c_i64), ("t", P(c_r)), ("eta_obs", P(c_r)), ("sigma", P(c_f)), ("src", P(c_i32)),
                    ("fov", P(c_i8)), ("cell", P(c_i32)), ("sigma_eff", P(c_r)), ("ccd", P(c_i8)),
                    ("mu", P(c_f)), ("ac_cell", P(c_i32))]

    class State(ctypes.Structure):
        _fields_ = [("n_src", c_i64), ("n_att", c_i64), ("n_cells", c_i64), ("s", P(c_r)), ("a", P(c_r)),
                    ("c", P(c_r)), ("n_buckets", c_i64), ("eps_a2", P(c_r)), ("src_eps2", P(c_r)),
                    ("src_D", P(c_r)), ("geo", P(c_r)), ("g0", c_r)]

    return World, Obs, State


World, Obs, State = _structs(c_d)
_STRUCTS = {"double": (World, Obs, State), "extended": _structs(ctypes.c_longdouble)}


def _lib_path(precision):
    return os.path.join(_HERE, PRECISIONS[precision][2])


def build(force: bool = False) -> str:
    """Compile both builds of the oracle (FP64 and x87 extended)."""
    src = os.path.join(_HERE, "agis_oracle.c")
    hdr = os.path.join(_HERE, "agis_oracle.h")
    newest = max(os.path.getmtime(src), os.path.getmtime(hdr))
    for precision, (_, _, _, flags) in PRECISIONS.items():
        path = _lib_path(precision)
        if force or not os.path.exists(path) or os.path.getmtime(path) < newest:
            tmp = path + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-std=c99", "-D_DEFAULT_SOURCE", *flags, "-O2", "-fno-fast-math",
                                   "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
            os.replace(tmp, path)
    return _lib_path("double")


_libs = {}


def lib(precision="double"):
    if precision not in _libs:
        path = _lib_path(precision)
        if not os.path.exists(path):
            build()
        c_r = PRECISIONS[precision][0]
        World, Obs, State = _STRUCTS[precision]
        L = ctypes.CDLL(path)
        L.orc_qmul.argtypes = [P(c_r), P(c_r), P(c_r)]
        L.orc_qconj.argtypes = [P(c_r), P(c_r)]
        L.orc_qinv.argtypes = [P(c_r), P(c_r)]
        L.orc_frame_rotate.argtypes = [P(c_r), P(c_r), P(c_r)]
        L.orc_vector_rotate.argtypes = [P(c_r), P(c_r), P(c_r)]
        L.orc_quat2mat.argtypes = [P(c_r), P(c_r)]
        L.orc_qrot.argtypes = [P(c_r), P(c_r)]
        L.orc_left_index.argtypes = [P(c_r), c_i64, c_r]
        L.orc_left_index.restype = c_i64
        L.orc_bspline.argtypes = [P(c_r), c_i64, c_r, P(c_r)]
        L.orc_chol_c1.argtypes = [P(c_r), ctypes.c_int]
        L.orc_chol_c1.restype = ctypes.c_int
        L.orc_chol_c2.argtypes = [P(c_r), ctypes.c_int, P(c_r)]
        L.orc_chol_c3.argtypes = [P(c_r), ctypes.c_int, P(c_r)]
        L.orc_band_c1.argtypes = [P(c_r), ctypes.c_int, ctypes.c_int]
        L.orc_band_c1.restype = ctypes.c_int
        L.orc_band_c2.argtypes = [P(c_r), ctypes.c_int, ctypes.c_int, P(c_r)]
        L.orc_band_c3.argtypes = [P(c_r), ctypes.c_int, ctypes.c_int, P(c_r)]
        L.orc_observe.argtypes = [P(World), P(Obs), P(State), c_i64, c_i64, P(c_r), P(c_r), P(c_r), P(c_i8),
                                  P(c_r), P(c_r), P(c_r), P(c_r), P(c_i64), P(c_r), P(c_r)]
        L.orc_ephemeris.argtypes = [P(World), c_r, P(c_r), P(c_r)]
        L.orc_normal_triad.argtypes = [c_r, c_r, P(c_r), P(c_r), P(c_r)]
        L.orc_source_update.argtypes = [P(World), P(Obs), P(State), P(c_r), P(c_r), P(c_i32), P(c_r)]
        L.orc_attitude_update.argtypes = [P(World), P(Obs), P(State), P(c_r)]
        L.orc_attitude_update.restype = c_i64
        L.orc_attitude_segment.argtypes = [P(World), P(Obs), P(State), c_i64, P(c_r), P(c_i64), P(c_i64)]
        L.orc_attitude_segment.restype = c_i64
        L.orc_num_segments.argtypes = [P(World)]
        L.orc_num_segments.restype = c_i64
        L.orc_calibration_update.argtypes = [P(World), P(Obs), P(State), P(c_r)]
        L.orc_iterate_sac.argtypes = [P(World), P(Obs), P(State), P(c_r)]
        L.orc_global_update.argtypes = [P(World), P(Obs), P(State)]
        L.orc_global_update.restype = c_r
        L.orc_normal_rhs.argtypes = [P(World), P(Obs), P(State), P(c_r), P(c_r), P(c_r)]
        L.orc_normal_quadratic.argtypes = [P(World), P(Obs), P(State), P(c_r)]
        L.orc_normal_quadratic.restype = c_r
        L.orc_frozen_sigma.argtypes = [P(World), P(Obs), P(State), P(c_r)]
        L.orc_frame_fit.argtypes = [P(World), P(State), P(c_r), P(c_r), P(c_r)]
        L.orc_frame_apply.argtypes = [P(World), P(State), P(c_r)]
        L.orc_weight_function.argtypes = [c_r]
        L.orc_weight_function.restype = c_r
        L.orc_quantile.argtypes = [P(c_r), c_i64, c_r]
        L.orc_quantile.restype = c_r
        L.orc_excess_attitude_noise.argtypes = [P(World), P(Obs), P(State)]
        _libs[precision] = L
    return _libs[precision]


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


def weight_function(z):
    """Downweighting function w(z) of eq:dw."""
    return float(lib().orc_weight_function(float(z)))


def quantile(x, p):
    """p-quantile, linear interpolation at (n - 1) p (type 7)."""
    x = _vec(x)
    return float(lib().orc_quantile(_p(x, c_d), x.size, float(p)))


def normal_triad(alpha, delta):
    p, q, r = np.empty(3), np.empty(3), np.empty(3)
    lib().orc_normal_triad(float(alpha), float(delta), _p(p, c_d), _p(q, c_d), _p(r, c_d))
    return p, q, r


# --- problem wrapper --------------------------------------------------------
class Problem:
    """Holds the world constants, observations and a mutable state (s, a, c).

    ``consts`` keys: gamma_c, t_ep, t_fr, lambda_reg, seg_len, seg_overlap,
    eph_radius_au, eph_L0, eph_Lrate, eps_obl, au_m, c_mps, year_s, and for
    the robust mode robust (0/1), eps_bucket (knot intervals per bucket) and
    eps_a_init (initial excess attitude noise [rad]).
    ``precision``: "double" (the oracle) or "extended" (the same code in x87
    extended precision; arrays are then numpy longdouble).
    """

    def __init__(self, consts, knots, t, eta_obs, sigma, src, fov, cell, s, a, c, precision="double",
                 sigma_eff=None, ccd=None, mu=None, geo=None, ac_cell=None, g0=0.0):
        self.precision = precision
        self._cr, self._dt = PRECISIONS[precision][0], PRECISIONS[precision][1]
        self._World, self._Obs, self._State = _STRUCTS[precision]
        self._L = lib(precision)
        self.knots = self._arr(knots)
        self.t = self._arr(t)
        self.eta_obs = self._arr(eta_obs)
        self.sigma = np.ascontiguousarray(sigma, dtype=np.float32)
        # the frozen sigma_eff of the hybrid scheme, replacing sigma (or None)
        self.sigma_eff = None if sigma_eff is None else self._arr(sigma_eff).copy()
        # geometric calibration (consts geo_ccds > 0): CCD index and AC pixel
        # coordinate per record, coefficients [n_cells][geo_ccds][3]; with
        # ac_cell (the across-scan records' calibration cells) the AC term
        # too, its coefficients after the AL ones; with consts geo_small_days
        # the small-scale AL term, [K][geo_ccds][1966] coefficients last
        geo_ccds = int(consts.get("geo_ccds", 0) or 0)
        if geo_ccds > 0:
            self.ccd = np.ascontiguousarray(ccd, dtype=np.int8)
            self.mu = np.ascontiguousarray(mu, dtype=np.float32)
            self.ac_cell = None if ac_cell is None else np.ascontiguousarray(ac_cell, dtype=np.int32)
            self.geo = self._arr(np.reshape(geo, -1)).copy()
            n_ac = 0 if ac_cell is None else int(consts.get("geo_ac_cells", 0) or 0)
            sd = int(consts.get("geo_small_days", 0) or 0)
            n_k = (np.size(c) // 2 + sd - 1) // sd if sd > 0 else 0
            assert self.geo.size == (np.size(c) + n_ac) * geo_ccds * 3 + n_k * geo_ccds * 1966
        else:
            self.ccd = self.mu = self.geo = self.ac_cell = None
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.fov = np.ascontiguousarray(fov, dtype=np.int8)
        self.cell = np.ascontiguousarray(cell, dtype=np.int32)
        self.s = self._arr(s).copy()
        self.a = self._arr(a).copy()
        self.c = self._arr(c).copy()
        self.consts = dict(consts)
        cr = self._cr
        self.world = self._World(n_knots=self.knots.size, knots=_p(self.knots, cr), gamma_c=consts["gamma_c"],
                                 t_ep=consts["t_ep"], t_fr=consts["t_fr"], lambda_reg=consts["lambda_reg"],
                                 seg_len=int(consts["seg_len"]), seg_overlap=int(consts["seg_overlap"]),
                                 eph_radius_au=consts["eph_radius_au"], eph_L0=consts["eph_L0"],
                                 eph_Lrate=consts["eph_Lrate"], eps_obl=consts["eps_obl"], au_m=consts["au_m"],
                                 c_mps=consts["c_mps"], year_s=consts["year_s"],
                                 robust=int(consts.get("robust", 0)), eps_bucket=int(consts.get("eps_bucket", 8)),
                                 geo_ccds=geo_ccds, geo_ac_cells=int(consts.get("geo_ac_cells", 0) or 0),
                                 defl=float(consts.get("defl", 0.0) or 0.0), ppn=int(consts.get("ppn", 0) or 0),
                                 geo_small_days=int(consts.get("geo_small_days", 0) or 0) if geo_ccds > 0 else 0)
        n_iv = self.knots.size - 7
        if self.world.robust:
            # three components (along scan, across scan preceding and
            # following field of view), n_buckets each
            nb = (n_iv + self.world.eps_bucket - 1) // self.world.eps_bucket
            self.eps_a2 = self._arr(np.full(3 * nb, float(consts.get("eps_a_init", 0.0)) ** 2))
        else:
            self.eps_a2 = self._zeros(0)
        # robust 2: excess source noise eps_i^2 and its significance D per source
        self.src_eps2 = self._zeros(self.s.shape[0]) if self.world.robust == 2 else None
        self.src_D = self._zeros(self.s.shape[0]) if self.world.robust == 2 else None
        self._g0 = g0                       # the global parameter of eq:gammaPPN (gamma = 1 + g0)
        self._refresh()

    @property
    def g0(self):
        return float(self.state.g0)

    def _arr(self, x):
        return np.ascontiguousarray(x, dtype=self._dt)

    def _zeros(self, shape):
        return np.zeros(shape, dtype=self._dt)

    def _refresh(self):
        cr = self._cr
        if hasattr(self, "state"):
            self._g0 = self.state.g0            # kept across the struct's rebuild
        self.obs = self._Obs(n=self.t.size, t=_p(self.t, cr), eta_obs=_p(self.eta_obs, cr),
                             sigma=_p(self.sigma, c_f), src=_p(self.src, c_i32), fov=_p(self.fov, c_i8),
                             cell=_p(self.cell, c_i32), sigma_eff=_p(self.sigma_eff, cr),
                             ccd=_p(self.ccd, c_i8), mu=_p(self.mu, c_f), ac_cell=_p(self.ac_cell, c_i32))
        self.state = self._State(n_src=self.s.shape[0], n_att=self.a.shape[0], n_cells=self.c.size,
                                 s=_p(self.s, cr), a=_p(self.a, cr), c=_p(self.c, cr),
                                 n_buckets=self.eps_a2.size // 3, eps_a2=_p(self.eps_a2, cr),
                                 src_eps2=_p(self.src_eps2, cr), src_D=_p(self.src_D, cr), geo=_p(self.geo, cr),
                                 g0=self._g0)

    def set_eta_obs(self, eta_obs):
        self.eta_obs = self._arr(eta_obs).copy()
        self._refresh()

    def set_state(self, s=None, a=None, c=None, eps_a2=None, geo=None, g0=None):
        if g0 is not None:
            self.state.g0 = g0
        if geo is not None:
            assert np.size(geo) == self.geo.size
            self.geo = self._arr(np.reshape(geo, -1)).copy()
        if eps_a2 is not None:
            assert np.size(eps_a2) == self.eps_a2.size
            self.eps_a2 = self._arr(eps_a2).copy()
        if s is not None:
            self.s = self._arr(s).copy()
        if a is not None:
            self.a = self._arr(a).copy()
        if c is not None:
            self.c = self._arr(c).copy()
        self._refresh()

    def observe(self, i0=0, i1=None, partials=False):
        n = self.t.size
        i1 = n if i1 is None else i1
        z = self._zeros
        out = dict(eta=z(n), phi=z(n), zeta=z(n), f=np.zeros(n, np.int8), R=z(n),
                   bspl=z((n, 4)), ell=np.zeros(n, np.int64), qraw=z((n, 4)), D=z(n))
        if partials:
            out["dsrc"] = z((n, 5))
            out["dq"] = z((n, 4))
        cr = self._cr
        self._L.orc_observe(ctypes.byref(self.world), ctypes.byref(self.obs), ctypes.byref(self.state), i0, i1,
                            _p(out["eta"], cr), _p(out["phi"], cr), _p(out["zeta"], cr), _p(out["f"], c_i8),
                            _p(out["R"], cr), _p(out.get("dsrc"), cr), _p(out.get("dq"), cr),
                            _p(out["bspl"], cr), _p(out["ell"], c_i64), _p(out["qraw"], cr), _p(out["D"], cr))
        return out

    def ephemeris(self, t):
        b, v = self._zeros(3), self._zeros(3)
        self._L.orc_ephemeris(ctypes.byref(self.world), t, _p(b, self._cr), _p(v, self._cr))
        return b, v

    def source_update(self):
        ns = self.s.shape[0]
        d, Q, de = self._zeros((ns, 5)), self._zeros(ns), np.zeros(ns, np.int32)
        self.var = self._zeros((ns, 5))
        cr = self._cr
        self._L.orc_source_update(ctypes.byref(self.world), ctypes.byref(self.obs), ctypes.byref(self.state),
                                  _p(d, cr), _p(Q, cr), _p(de, c_i32), _p(self.var, cr))
        return d, Q, de

    def attitude_update(self):
        d = np.zeros_like(self.a)
        de = self._L.orc_attitude_update(ctypes.byref(self.world), ctypes.byref(self.obs),
                                         ctypes.byref(self.state), _p(d, self._cr))
        return d, int(de)

    def attitude_segment(self, K):
        d = np.full_like(self.a, np.nan)
        lo, hi = c_i64(), c_i64()
        de = self._L.orc_attitude_segment(ctypes.byref(self.world), ctypes.byref(self.obs),
                                          ctypes.byref(self.state), int(K), _p(d, self._cr), ctypes.byref(lo),
                                          ctypes.byref(hi))
        return d, int(de), lo.value, hi.value

    def num_segments(self):
        return int(self._L.orc_num_segments(ctypes.byref(self.world)))

    def excess_attitude_noise(self):
        """Re-estimate eps_a^2 per bucket from the residuals at the current state."""
        self._L.orc_excess_attitude_noise(ctypes.byref(self.world), ctypes.byref(self.obs),
                                          ctypes.byref(self.state))
        return self.eps_a2.copy()

    def calibration_update(self):
        """The calibration update (per cell, or with the geometric model the
        flat [n_cells][geo_ccds][3] coefficients), applied to the state."""
        d = np.zeros_like(self.c if self.geo is None else self.geo)
        self._L.orc_calibration_update(ctypes.byref(self.world), ctypes.byref(self.obs), ctypes.byref(self.state),
                                       _p(d, self._cr))
        return d

    def global_update(self):
        """The update of g0 from eq:normG (Sect. 5.4), applied; returns it."""
        return float(self._L.orc_global_update(ctypes.byref(self.world), ctypes.byref(self.obs),
                                               ctypes.byref(self.state)))

    def normal_rhs(self):
        """Right-hand sides of the S, A and C normal equations at the current
        state: (rs [n_src][5], ra [n_att][4], rc [n_cells])."""
        rs, ra, rc = self._zeros(self.s.shape), self._zeros(self.a.shape), self._zeros(self.c.shape)
        cr = self._cr
        self._L.orc_normal_rhs(ctypes.byref(self.world), ctypes.byref(self.obs), ctypes.byref(self.state),
                               _p(rs, cr), _p(ra, cr), _p(rc, cr))
        return rs, ra, rc

    def normal_quadratic(self, v):
        """v' N v for the normal matrix of the three blocks at the current
        state (v: sources, then attitude, then calibration unknowns)."""
        v = self._arr(v)
        assert v.size == 5 * self.s.shape[0] + 4 * self.a.shape[0] + self.c.size
        return self._L.orc_normal_quadratic(ctypes.byref(self.world), ctypes.byref(self.obs),
                                            ctypes.byref(self.state), _p(v, self._cr))

    def frozen_sigma(self):
        """sigma_eff = 1 / sqrt(W) (the Problem's real type, input order) of
        every observation at the current state, W the A/C weight."""
        out = self._zeros(self.t.size)
        self._L.orc_frozen_sigma(ctypes.byref(self.world), ctypes.byref(self.obs), ctypes.byref(self.state),
                                 _p(out, self._cr))
        return out

    def iterate_sac(self):
        self.var = self._zeros((self.s.shape[0], 5))
        self._L.orc_iterate_sac(ctypes.byref(self.world), ctypes.byref(self.obs), ctypes.byref(self.state),
                                _p(self.var, self._cr))

    def frame_fit(self, s_ref, weighted=True):
        """Frame rotator fit; weighted by the variances of the last S update
        (unit weights before any, or with weighted=False)."""
        s_ref = self._arr(s_ref)
        eo = self._zeros(6)
        var = getattr(self, "var", None) if weighted else None
        cr = self._cr
        self._L.orc_frame_fit(ctypes.byref(self.world), ctypes.byref(self.state), _p(s_ref, cr), _p(var, cr),
                              _p(eo, cr))
        return eo

    def frame_apply(self, eo):
        eo = self._arr(eo)
        assert eo.size == 6
        self._L.orc_frame_apply(ctypes.byref(self.world), ctypes.byref(self.state), _p(eo, self._cr))

    def iterate(self, s_ref=None):
        """One S[AC] iteration, then (if s_ref is given) the frame rotator."""
        self.iterate_sac()
        if s_ref is not None:
            eo = self.frame_fit(s_ref)
            self.frame_apply(eo)
            return eo
        return None


def problem_from_world(world, eta_obs=None, state="start", precision="double"):
    """Build a Problem from a synth.World; eta_obs defaults to zeros."""
    n = world.t.size
    eta = np.zeros(n) if eta_obs is None else eta_obs
    which = "start" if state == "start" else "true"
    s, a, c = getattr(world, f"src_{which}"), getattr(world, f"att_{which}"), getattr(world, f"cal_{which}")
    return Problem(world.consts, world.knots, world.t, eta, world.sigma, world.src, world.fov, world.cell, s, a, c,
                   precision=precision, ccd=getattr(world, "ccd", None), mu=getattr(world, "mu", None),
                   geo=world_geo(world, which), ac_cell=getattr(world, "ac_cell", None),
                   g0=getattr(world, f"g0_{which}", 0.0))


def basic_angle(geo, n_cells, n_ccd):
    """The basic-angle offset of each short interval (day), a monitored
    quantity (Sect. 3.4, eq:DeltaGamma): over the AF CCDs, the sum of f times
    the AL constant term of field of view f (f = +1 preceding, the day's even
    cell; -1 following, its odd cell) divided by the number of AF CCDs (62 in
    the paper, n_ccd here).  geo: the flat coefficients, AL groups first
    ([n_cells][n_ccd][3])."""
    c0 = np.asarray(geo, dtype=np.float64)[:3 * n_cells * n_ccd].reshape(n_cells // 2, 2, n_ccd, 3)[:, :, :, 0]
    f = np.array([1.0, -1.0])
    return np.einsum("f,jfn->j", f, c0) / n_ccd


def world_geo(world, which="true"):
    """The world's geometric coefficients (true or start): AL, then AC and
    small-scale where the world has them; None without the geometric model."""
    g = getattr(world, f"geo_{which}", None)
    if g is None:
        return None
    parts = [g] + [x for x in (getattr(world, f"geo_ac_{which}", None), getattr(world, f"geo_small_{which}", None))
                   if x is not None]
    return np.concatenate([np.reshape(x, -1) for x in parts])


def observed_field_angles(world, chunk=1 << 24):
    """eta_obs = eta(t | s_true, a_true) - c_true(cell) + noise (Sect. 3.5 at
    the truth); for an across-scan observation (cell < 0) zeta(t | s_true,
    a_true) + noise (eq:resAC; minus the true AC geometric term where the
    world has one).  Evaluated over chunks
    of at most `chunk` observations (memory: the model's outputs per
    observation)."""
    n = world.t.size
    out = np.empty(n)
    consts = dict(world.consts)
    consts["robust"] = 0                       # the model alone; no robust state
    geo_ccds = int(consts.get("geo_ccds", 0) or 0)
    for i0 in range(0, max(n, 1), chunk):
        i1 = min(n, i0 + chunk)
        sl = slice(i0, i1)
        pr = Problem(consts, world.knots, world.t[sl], np.zeros(i1 - i0), world.sigma[sl], world.src[sl],
                     world.fov[sl], world.cell[sl], world.src_true, world.att_true, world.cal_true,
                     ccd=None if geo_ccds == 0 else world.ccd[sl], mu=None if geo_ccds == 0 else world.mu[sl],
                     geo=None if geo_ccds == 0 else world_geo(world, "true"),
                     ac_cell=None if getattr(world, "ac_cell", None) is None else world.ac_cell[sl],
                     g0=getattr(world, "g0_true", 0.0))
        o = pr.observe()
        # the residual of eta_obs = 0 is the calibration minus the computed
        # field angle (eq:resAL; eq:resAC across scan), so eta_obs = eta -
        # calibration + noise makes it the noise at the truth
        out[sl] = -np.asarray(o["R"]) + world.eps[sl]
    return out
