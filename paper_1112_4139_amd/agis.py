"""ctypes binding of libagis (include/agis.h): argument marshalling only.

Every function below has the name of the C entry point it calls and only
converts arguments: NumPy arrays are passed as host pointers (AGIS_HOST),
torch tensors on the GPU as device pointers (AGIS_DEVICE).  All computation
happens in the library's HIP kernels; if the library is missing the import
fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libagis.so")

AGIS_OK = 0
AGIS_HOST, AGIS_DEVICE = 0, 1
AGIS_FP64, AGIS_MIXED = 0, 1
ERRORS = {-1: "E_INVALID_ARG", -2: "E_SHAPE", -3: "E_RANGE", -4: "E_DEVICE", -5: "E_OOM", -6: "E_NUMERIC",
          -7: "E_STATE"}

P = ctypes.POINTER
c_d, c_i64, c_i32, c_i8, c_f = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_int8, ctypes.c_float


class agis_config_t(ctypes.Structure):
    _fields_ = [("n_knots", c_i64), ("knots", P(c_d)), ("gamma_c", c_d), ("t_ep", c_d), ("t_fr", c_d),
                ("lambda_reg", c_d), ("seg_len", c_i32), ("seg_overlap", c_i32), ("eph_radius_au", c_d),
                ("eph_L0", c_d), ("eph_Lrate", c_d), ("eps_obl", c_d), ("au_m", c_d), ("c_mps", c_d),
                ("year_s", c_d), ("precision", c_i32), ("device", c_i32), ("stream", ctypes.c_void_p),
                ("robust", c_i32), ("eps_bucket", c_i32), ("eps_a_init", c_d), ("defl", c_d), ("ppn", c_i32)]


class agis_obs_soa_t(ctypes.Structure):
    _fields_ = [("n", c_i64), ("t", ctypes.c_void_p), ("eta_obs", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("src", ctypes.c_void_p), ("fov", ctypes.c_void_p), ("cell", ctypes.c_void_p)]


class agis_block_stats_t(ctypes.Structure):
    _fields_ = [("n_obs", c_i64), ("n_units", c_i64), ("defect", c_i64), ("rms_update", c_d * 5),
                ("max_update", c_d * 5), ("chi2", c_d), ("ms", c_d)]

    def as_dict(self):
        return dict(n_obs=self.n_obs, n_units=self.n_units, defect=self.defect, rms_update=list(self.rms_update),
                    max_update=list(self.max_update), chi2=self.chi2, ms=self.ms)


class agis_iter_stats_t(ctypes.Structure):
    _fields_ = [("s", agis_block_stats_t), ("a", agis_block_stats_t), ("c", agis_block_stats_t),
                ("eps_omega", c_d * 6), ("ms", c_d)]


class agis_cg_stats_t(ctypes.Structure):
    _fields_ = [("alpha", c_d), ("beta", c_d), ("rho", c_d), ("cycle_start", c_i32), ("breakdown", c_i32),
                ("ms", c_d)]


class agis_learned_stats_t(ctypes.Structure):
    _fields_ = [("iterations", c_i32), ("gated", c_i32), ("accepted", c_i32), ("q_plain", c_d), ("q_cand", c_d)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libagis.so not built at {LIB_PATH}; run __graft_entry__.build()")
_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_ctx_p = ctypes.c_void_p
_sig = {
    "agis_version": ([], ctypes.c_int),
    "agis_create": ([P(agis_config_t), P(_ctx_p)], ctypes.c_int),
    "agis_destroy": ([_ctx_p], None),
    "agis_last_error": ([_ctx_p], ctypes.c_char_p),
    "agis_load_observations": ([_ctx_p, P(agis_obs_soa_t), c_i64, c_i64, ctypes.c_int], ctypes.c_int),
    "agis_set_sources": ([_ctx_p, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_get_sources": ([_ctx_p, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_set_attitude": ([_ctx_p, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_get_attitude": ([_ctx_p, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_set_calibration": ([_ctx_p, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_get_calibration": ([_ctx_p, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_load_geometry": ([_ctx_p, c_i64, _vp, _vp, c_i32, _vp, c_i32, c_i32, ctypes.c_int], ctypes.c_int),
    "agis_basic_angle": ([_ctx_p, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_global_update": ([_ctx_p, P(c_d)], ctypes.c_int),
    "agis_set_global": ([_ctx_p, c_d], ctypes.c_int),
    "agis_get_global": ([_ctx_p, P(c_d)], ctypes.c_int),
    "agis_set_geo_calibration": ([_ctx_p, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_get_geo_calibration": ([_ctx_p, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_source_update": ([_ctx_p, P(agis_block_stats_t)], ctypes.c_int),
    "agis_attitude_update": ([_ctx_p, P(agis_block_stats_t)], ctypes.c_int),
    "agis_calibration_update": ([_ctx_p, P(agis_block_stats_t)], ctypes.c_int),
    "agis_attitude_calibration_update": ([_ctx_p, P(agis_block_stats_t), P(agis_block_stats_t)], ctypes.c_int),
    "agis_set_frame_reference": ([_ctx_p, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_frame_fit": ([_ctx_p, P(c_d)], ctypes.c_int),
    "agis_frame_apply": ([_ctx_p, P(c_d)], ctypes.c_int),
    "agis_iterate": ([_ctx_p, c_i32, P(agis_iter_stats_t)], ctypes.c_int),
    "agis_iterate_graph": ([_ctx_p, ctypes.c_int32], ctypes.c_int),
    "agis_autotune": ([_ctx_p, P(c_i32)], ctypes.c_int),
    "agis_get_tuning": ([_ctx_p, P(c_i32)], ctypes.c_int),
    "agis_residuals": ([_ctx_p, _vp, ctypes.c_int], ctypes.c_int),
    "agis_problem_size": ([_ctx_p, P(c_i64), P(c_i64), P(c_i64), P(c_i64), P(c_i64)], ctypes.c_int),
    "agis_kernel_times": ([_ctx_p, P(c_d)], ctypes.c_int),
    "agis_set_excess_noise": ([_ctx_p, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_get_excess_noise": ([_ctx_p, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_excess_noise_update": ([_ctx_p], ctypes.c_int),
    "agis_learned_reset": ([_ctx_p], ctypes.c_int),
    "agis_learned_record": ([_ctx_p], ctypes.c_int),
    "agis_learned_features": ([_ctx_p, c_i32, c_i64, _vp, _vp, ctypes.c_int], ctypes.c_int),
    "agis_mlp_init": ([_ctx_p, c_i32, ctypes.c_uint64], ctypes.c_int),
    "agis_mlp_load": ([_ctx_p, c_i32, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_mlp_get_weights": ([_ctx_p, c_i32, c_i64, _vp, ctypes.c_int], ctypes.c_int),
    "agis_mlp_forward": ([_ctx_p, c_i32, c_i64, _vp, _vp, ctypes.c_int], ctypes.c_int),
    "agis_mlp_gradient": ([_ctx_p, c_i32, c_i64, _vp, _vp, _vp, P(ctypes.c_float), ctypes.c_int], ctypes.c_int),
    "agis_mlp_train_step": ([_ctx_p, c_i32, c_i64, _vp, _vp, ctypes.c_int, ctypes.c_float, P(ctypes.c_float)],
                            ctypes.c_int),
    "agis_mlp_train": ([_ctx_p, c_i32, c_i64, _vp, _vp, ctypes.c_int, c_i32, c_i32, ctypes.c_float, ctypes.c_uint64,
                        _vp], ctypes.c_int),
    "agis_chi2": ([_ctx_p, P(c_d)], ctypes.c_int),
    "agis_chi2_noalloc": ([_ctx_p, _vp, ctypes.c_int], ctypes.c_int),
    "agis_learned_apply": ([_ctx_p], ctypes.c_int),
    "agis_asi_step": ([_ctx_p, ctypes.c_int32, c_d, P(c_d), P(c_d)], ctypes.c_int),
    "agis_cg_iterate": ([_ctx_p, c_i32, c_i32, P(agis_cg_stats_t)], ctypes.c_int),
    "agis_freeze_weights": ([_ctx_p, c_i32], ctypes.c_int),
    "agis_get_source_noise": ([_ctx_p, c_i64, _vp, _vp, ctypes.c_int], ctypes.c_int),
    "agis_learned_step": ([_ctx_p, P(c_d), P(c_d), P(c_i32)], ctypes.c_int),
    "agis_iterate_learned": ([_ctx_p, c_i32, c_i32, P(agis_learned_stats_t)], ctypes.c_int),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTS = tuple(_sig)


class AgisError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _check(rc, ctx):
    if rc != AGIS_OK:
        raise AgisError(rc, (_lib.agis_last_error(ctx) or b"").decode())


def _ptr(x, dtype):
    """(pointer, where, keepalive) for a NumPy array or a torch tensor."""
    try:
        import torch
        if isinstance(x, torch.Tensor):
            want = {np.float64: torch.float64, np.float32: torch.float32, np.int32: torch.int32,
                    np.int8: torch.int8}[dtype]
            if x.dtype != want or not x.is_contiguous():
                raise TypeError(f"tensor must be contiguous {want}")
            return ctypes.c_void_p(x.data_ptr()), (AGIS_DEVICE if x.is_cuda else AGIS_HOST), x
    except ImportError:
        pass
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data_as(ctypes.c_void_p), AGIS_HOST, a


def agis_version() -> int:
    return _lib.agis_version()


def agis_create(consts: dict, knots, precision=AGIS_FP64, device=0, stream=None):
    k = np.ascontiguousarray(knots, dtype=np.float64)
    cfg = agis_config_t(n_knots=k.size, knots=k.ctypes.data_as(P(c_d)), gamma_c=consts["gamma_c"],
                        t_ep=consts["t_ep"], t_fr=consts["t_fr"], lambda_reg=consts["lambda_reg"],
                        seg_len=int(consts["seg_len"]), seg_overlap=int(consts["seg_overlap"]),
                        eph_radius_au=consts["eph_radius_au"], eph_L0=consts["eph_L0"],
                        eph_Lrate=consts["eph_Lrate"], eps_obl=consts["eps_obl"], au_m=consts["au_m"],
                        c_mps=consts["c_mps"], year_s=consts["year_s"], precision=precision, device=device,
                        stream=stream, robust=int(consts.get("robust", 0)),
                        eps_bucket=int(consts.get("eps_bucket", 8)),
                        eps_a_init=float(consts.get("eps_a_init", 0.0)), defl=float(consts.get("defl", 0.0) or 0.0),
                        ppn=int(consts.get("ppn", 0) or 0))
    ctx = _ctx_p()
    rc = _lib.agis_create(ctypes.byref(cfg), ctypes.byref(ctx))
    _check(rc, None)
    return ctx


def agis_destroy(ctx):
    _lib.agis_destroy(ctx)


def agis_last_error(ctx) -> str:
    return (_lib.agis_last_error(ctx) or b"").decode()


def agis_load_observations(ctx, t, eta_obs, sigma, src, fov, cell, n_src, n_cells):
    cols = [_ptr(t, np.float64), _ptr(eta_obs, np.float64), _ptr(sigma, np.float32), _ptr(src, np.int32),
            _ptr(fov, np.int8), _ptr(cell, np.int32)]
    wheres = {w for _, w, _ in cols}
    if len(wheres) != 1:
        raise ValueError("observation columns must all be host arrays or all device tensors")
    n = len(cols[-1][2])
    obs = agis_obs_soa_t(n, *[p for p, _, _ in cols])
    _check(_lib.agis_load_observations(ctx, ctypes.byref(obs), int(n_src), int(n_cells), wheres.pop()), ctx)


def _set(fn, ctx, n, x):
    p, where, keep = _ptr(x, np.float64)
    _check(fn(ctx, int(n), p, where), ctx)


def _get(fn, ctx, n, width, out=None):
    if out is None:
        out = np.empty((n, width) if width > 1 else n, dtype=np.float64)
    p, where, keep = _ptr(out, np.float64)
    _check(fn(ctx, int(n), p, where), ctx)
    return out


def agis_set_sources(ctx, s5):
    _set(_lib.agis_set_sources, ctx, len(s5), s5)


def agis_get_sources(ctx, n, out=None):
    return _get(_lib.agis_get_sources, ctx, n, 5, out)


def agis_set_attitude(ctx, a4):
    _set(_lib.agis_set_attitude, ctx, len(a4), a4)


def agis_get_attitude(ctx, n, out=None):
    return _get(_lib.agis_get_attitude, ctx, n, 4, out)


def agis_set_calibration(ctx, c):
    _set(_lib.agis_set_calibration, ctx, len(c), c)


def agis_get_calibration(ctx, n, out=None):
    return _get(_lib.agis_get_calibration, ctx, n, 1, out)


def agis_load_geometry(ctx, ccd, mu, n_ccd, ac_cell=None, n_ac_cells=0, small_days=0):
    """Enable the geometric calibration: CCD index (int8) and across-scan
    pixel coordinate (float32) of every record, in input order; with
    ac_cell (int32, each across-scan record's AC cell) and n_ac_cells the
    across-scan term too; with small_days > 0 the small-scale AL term per
    CCD, long interval of that many days and pixel column."""
    pc, wc, kc = _ptr(ccd, np.int8)
    pm, wm, km = _ptr(mu, np.float32)
    pa, wa, ka = (None, wc, None) if ac_cell is None else _ptr(ac_cell, np.int32)
    if wc != wm or wa != wc:
        raise ValueError("ccd, mu and ac_cell must all be host arrays or all device tensors")
    _check(_lib.agis_load_geometry(ctx, int(len(ccd)), pc, pm, int(n_ccd), pa, int(n_ac_cells), int(small_days), wc),
           ctx)


def agis_basic_angle(ctx, n_days):
    """The basic-angle offset of each day from the AL constant terms
    (eq:DeltaGamma) [rad]."""
    out = np.empty(int(n_days), np.float64)
    _check(_lib.agis_basic_angle(ctx, int(n_days), out.ctypes.data_as(_vp), 0), ctx)
    return out


def agis_global_update(ctx):
    """The global block's solve and update of g0 at the current parameters;
    returns (update of g0, g1)."""
    out = (c_d * 2)()
    _check(_lib.agis_global_update(ctx, out), ctx)
    return out[0], out[1]


def agis_set_global(ctx, g0):
    _check(_lib.agis_set_global(ctx, float(g0)), ctx)


def agis_get_global(ctx):
    """(g0, the last update of g0, the last g1)."""
    out = (c_d * 3)()
    _check(_lib.agis_get_global(ctx, out), ctx)
    return out[0], out[1], out[2]


def agis_set_geo_calibration(ctx, c):
    _set(_lib.agis_set_geo_calibration, ctx, np.size(c), np.reshape(c, -1) if isinstance(c, np.ndarray) else c)


def agis_get_geo_calibration(ctx, n, out=None):
    return _get(_lib.agis_get_geo_calibration, ctx, n, 1, out)


def agis_source_update(ctx):
    st = agis_block_stats_t()
    _check(_lib.agis_source_update(ctx, ctypes.byref(st)), ctx)
    return st.as_dict()


def agis_attitude_update(ctx):
    st = agis_block_stats_t()
    _check(_lib.agis_attitude_update(ctx, ctypes.byref(st)), ctx)
    return st.as_dict()


def agis_calibration_update(ctx):
    st = agis_block_stats_t()
    _check(_lib.agis_calibration_update(ctx, ctypes.byref(st)), ctx)
    return st.as_dict()


def agis_attitude_calibration_update(ctx):
    sa, sc = agis_block_stats_t(), agis_block_stats_t()
    _check(_lib.agis_attitude_calibration_update(ctx, ctypes.byref(sa), ctypes.byref(sc)), ctx)
    return sa.as_dict(), sc.as_dict()


def agis_set_frame_reference(ctx, s_ref):
    if s_ref is None:
        n = ctypes.c_int64()
        _lib.agis_problem_size(ctx, None, ctypes.byref(n), None, None, None)
        _check(_lib.agis_set_frame_reference(ctx, n.value, None, AGIS_HOST), ctx)
        return
    _set(_lib.agis_set_frame_reference, ctx, len(s_ref), s_ref)


def agis_frame_fit(ctx):
    eo = (c_d * 6)()
    _check(_lib.agis_frame_fit(ctx, eo), ctx)
    return np.array(eo[:])


def agis_frame_apply(ctx, eps_omega):
    eo = (c_d * 6)(*[float(x) for x in eps_omega])
    _check(_lib.agis_frame_apply(ctx, eo), ctx)


def agis_iterate(ctx, n_iter, stats=True):
    if stats:
        arr = (agis_iter_stats_t * max(int(n_iter), 1))()
        _check(_lib.agis_iterate(ctx, int(n_iter), arr), ctx)
        return [dict(s=x.s.as_dict(), a=x.a.as_dict(), c=x.c.as_dict(), eps_omega=list(x.eps_omega), ms=x.ms)
                for x in arr[:n_iter]]
    _check(_lib.agis_iterate(ctx, int(n_iter), None), ctx)
    return None


def agis_iterate_graph(ctx, n_iter):
    _check(_lib.agis_iterate_graph(ctx, int(n_iter)), ctx)


def agis_autotune(ctx):
    g = c_i32()
    _check(_lib.agis_autotune(ctx, ctypes.byref(g)), ctx)
    return g.value


def agis_get_tuning(ctx):
    """The launch choices in effect: lanes per source, robust S path (0 HBM
    columns, 1 rows then LDS, 2 all in LDS, 3 rows in registers), paired
    quantile selection, fused excess-noise estimate, register cache of the
    column path's inner rounds (0 none, 1 / 2: 32 / 64 lanes per source)."""
    out = (c_i32 * 5)()
    _check(_lib.agis_get_tuning(ctx, out), ctx)
    return dict(lanes_per_source=out[0], robust_s_path=out[1], paired_selection=bool(out[2]),
                fused_excess_noise=bool(out[3]), irls_cache=out[4])


def agis_residuals(ctx, out=None):
    if out is None:
        n = ctypes.c_int64()
        _lib.agis_problem_size(ctx, ctypes.byref(n), None, None, None, None)
        out = np.empty(n.value, dtype=np.float64)
    p, where, keep = _ptr(out, np.float64)
    _check(_lib.agis_residuals(ctx, p, where), ctx)
    return out


def agis_set_excess_noise(ctx, eps_a2):
    _set(_lib.agis_set_excess_noise, ctx, len(eps_a2), eps_a2)


def agis_get_excess_noise(ctx, n, out=None):
    return _get(_lib.agis_get_excess_noise, ctx, n, 1, out)


def agis_excess_noise_update(ctx):
    _check(_lib.agis_excess_noise_update(ctx), ctx)


MLP_IN = (22, 18)
MLP_OUT = (4, 4)           # mixing coefficients of the four recorded updates
MLP_NT = (5, 4)            # target columns: update components
MLP_NW = tuple(64 * f + 64 + 64 * 64 + 64 + o * 64 + o for f, o in zip(MLP_IN, MLP_OUT))


def _fptr(x):
    return _ptr(x, np.float32)


def agis_learned_reset(ctx):
    _check(_lib.agis_learned_reset(ctx), ctx)


def agis_learned_record(ctx):
    _check(_lib.agis_learned_record(ctx), ctx)


def agis_learned_features(ctx, which):
    sz = agis_problem_size(ctx)
    n = sz["n_src"] if which == 0 else sz["n_att"]
    X = np.empty((n, MLP_IN[which]), np.float32)
    sc = np.empty(n, np.float32)
    _check(_lib.agis_learned_features(ctx, int(which), n, X.ctypes.data_as(ctypes.c_void_p),
                                      sc.ctypes.data_as(ctypes.c_void_p), AGIS_HOST), ctx)
    return X, sc


def agis_mlp_init(ctx, which, seed):
    _check(_lib.agis_mlp_init(ctx, int(which), int(seed)), ctx)


def agis_mlp_load(ctx, which, w):
    p, where, keep = _fptr(w)
    _check(_lib.agis_mlp_load(ctx, int(which), MLP_NW[which], p, where), ctx)


def agis_mlp_get_weights(ctx, which):
    w = np.empty(MLP_NW[which], np.float32)
    _check(_lib.agis_mlp_get_weights(ctx, int(which), w.size, w.ctypes.data_as(ctypes.c_void_p), AGIS_HOST), ctx)
    return w


def agis_mlp_forward(ctx, which, X):
    X = np.ascontiguousarray(X, np.float32)
    Y = np.empty((X.shape[0], MLP_OUT[which]), np.float32)
    _check(_lib.agis_mlp_forward(ctx, int(which), X.shape[0], X.ctypes.data_as(ctypes.c_void_p),
                                 Y.ctypes.data_as(ctypes.c_void_p), AGIS_HOST), ctx)
    return Y


def agis_mlp_gradient(ctx, which, X, T):
    X = np.ascontiguousarray(X, np.float32)
    T = np.ascontiguousarray(T, np.float32)
    g = np.empty(MLP_NW[which], np.float32)
    loss = ctypes.c_float()
    _check(_lib.agis_mlp_gradient(ctx, int(which), X.shape[0], X.ctypes.data_as(ctypes.c_void_p),
                                  T.ctypes.data_as(ctypes.c_void_p), g.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(loss), AGIS_HOST), ctx)
    return g, loss.value


def agis_mlp_train_step(ctx, which, X, T, lr):
    """One Adam step on the whole batch (X, T): NumPy arrays (host) or torch
    tensors on the device; returns the batch loss before the step."""
    px, wx, kx = _fptr(X)
    pt, wt, kt = _fptr(T)
    if wx != wt:
        raise ValueError("X and T must both be host arrays or both device tensors")
    loss = ctypes.c_float()
    _check(_lib.agis_mlp_train_step(ctx, int(which), int(X.shape[0]), px, pt, wx, float(lr), ctypes.byref(loss)), ctx)
    return loss.value


def agis_mlp_train(ctx, which, X, T, steps, batch, lr, seed=0):
    X = np.ascontiguousarray(X, np.float32)
    T = np.ascontiguousarray(T, np.float32)
    losses = np.empty(max(int(steps), 1), np.float32)
    _check(_lib.agis_mlp_train(ctx, int(which), X.shape[0], X.ctypes.data_as(ctypes.c_void_p),
                               T.ctypes.data_as(ctypes.c_void_p), AGIS_HOST, int(steps), int(batch), float(lr),
                               int(seed), losses.ctypes.data_as(ctypes.c_void_p)), ctx)
    return losses[:steps]


def agis_chi2(ctx):
    q = c_d()
    _check(_lib.agis_chi2(ctx, ctypes.byref(q)), ctx)
    return q.value


def agis_chi2_noalloc(ctx, out=None):
    """chi^2 through the allocation-free entry point: returned as a float
    (host), or written into out[0] when out is a float64 torch tensor on the
    device."""
    if out is None:
        q = c_d()
        _check(_lib.agis_chi2_noalloc(ctx, ctypes.byref(q), AGIS_HOST), ctx)
        return q.value
    p, where, keep = _ptr(out, np.float64)
    _check(_lib.agis_chi2_noalloc(ctx, p, where), ctx)
    return out


def agis_learned_apply(ctx):
    _check(_lib.agis_learned_apply(ctx), ctx)


def agis_asi_step(ctx, stride=1, lambda_max=0.99):
    lam, f = c_d(), c_d()
    _check(_lib.agis_asi_step(ctx, int(stride), float(lambda_max), ctypes.byref(lam), ctypes.byref(f)), ctx)
    return dict(lam=lam.value, factor=f.value)


def agis_cg_iterate(ctx, n_eval, restart=40, stats=True):
    """n_eval evaluations of the conjugate-gradient scheme; per evaluation a
    dict (alpha, beta, rho, cycle_start, breakdown, ms) when stats."""
    if stats:
        arr = (agis_cg_stats_t * max(int(n_eval), 1))()
        _check(_lib.agis_cg_iterate(ctx, int(n_eval), int(restart), arr), ctx)
        return [dict(alpha=x.alpha, beta=x.beta, rho=x.rho, cycle_start=x.cycle_start, breakdown=x.breakdown,
                     ms=x.ms) for x in arr[:n_eval]]
    _check(_lib.agis_cg_iterate(ctx, int(n_eval), int(restart), None), ctx)
    return None


def agis_get_source_noise(ctx, n):
    """(eps_i^2, D) per source of the last source update (robust mode 2)."""
    e, d = np.zeros(n), np.zeros(n)
    _check(_lib.agis_get_source_noise(ctx, int(n), e.ctypes.data, d.ctypes.data, AGIS_HOST), ctx)
    return e, d


def agis_freeze_weights(ctx, freeze=True):
    _check(_lib.agis_freeze_weights(ctx, 1 if freeze else 0), ctx)


def agis_learned_step(ctx):
    qp, qc, acc = c_d(), c_d(), c_i32()
    _check(_lib.agis_learned_step(ctx, ctypes.byref(qp), ctypes.byref(qc), ctypes.byref(acc)), ctx)
    return dict(q_plain=qp.value, q_candidate=qc.value, accepted=bool(acc.value))


def agis_iterate_learned(ctx, n_blocks, m):
    """n_blocks blocks of the learned-accelerated scheme (m iterations, a
    record and, from the fourth record on, the gated step); per block a dict
    (iterations, gated, accepted, q_plain, q_candidate)."""
    arr = (agis_learned_stats_t * max(int(n_blocks), 1))()
    _check(_lib.agis_iterate_learned(ctx, int(n_blocks), int(m), arr), ctx)
    return [dict(iterations=x.iterations, gated=bool(x.gated), accepted=bool(x.accepted), q_plain=x.q_plain,
                 q_candidate=x.q_cand) for x in arr[:n_blocks]]


def agis_problem_size(ctx):
    v = [ctypes.c_int64() for _ in range(5)]
    _check(_lib.agis_problem_size(ctx, *[ctypes.byref(x) for x in v]), ctx)
    return dict(zip(["n_obs", "n_src", "n_att", "n_cells", "n_segments"], [x.value for x in v]))


def agis_kernel_times(ctx):
    ms = (c_d * 6)()
    _check(_lib.agis_kernel_times(ctx, ms), ctx)
    return dict(zip(["source_update", "ac_pass", "band_solve", "calib_solve", "frame", "excess_noise"], ms[:]))


class Solver:
    """Owns one context; the problem is described by a synth.World-like
    object (consts, knots, observation columns, parameter arrays)."""

    def __init__(self, consts, knots, precision=AGIS_FP64, device=0, stream=None):
        self.ctx = agis_create(consts, knots, precision, device, stream)

    def close(self):
        if self.ctx is not None:
            agis_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
