"""Seeded synthetic inputs shared by the CPU oracle and the HIP solver.

This module is input generation only.  It draws the true source parameters,
finds when each star crosses a field of view under a simplified nominal
scanning law (``world.c``), lays out the per-CCD observation times, draws the
true attitude coefficients (nominal orientation sampled at the B-spline
support mid-times, perturbed by small random rotations), the true and start
calibration offsets, and the observation noise.

It holds none of the astrometric solution's arithmetic: it never evaluates
the observation model, residuals, partial derivatives, normal equations or
solvers.  The observed field angle of each observation (which needs the
observation model at the true parameters) is therefore *not* produced here;
consumers compute it with their own model implementation.

Conventions shared as data (both implementations read them from the dict):
  t        seconds from the reference epoch t_ep = 0 (TCB-like)
  angles   radians; proper motions in radians per Julian year (365.25 d)
  ephemeris  circular barycentric orbit of radius ``eph_radius_au`` AU in the
           ecliptic, longitude L(t) = eph_L0 + eph_Lrate * t, rotated to the
           equatorial frame by ``eps_obl`` about X
  sources  rows (alpha, delta, parallax, pm_alpha*, pm_delta)
  attitude rows (x, y, z, w) B-spline coefficients, order M = 4
  cells    cell = 2 * day + (fov == -1), day counted from the mission start;
           cell = -1 marks an across-scan (AC) observation, which has no
           calibration parameter
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")

MAS = np.pi / (180.0 * 3600.0 * 1000.0)
UAS = MAS / 1000.0
ARCSEC = MAS * 1000.0
DEG = np.pi / 180.0
DAY = 86400.0
YEAR = 365.25 * DAY
AU_M = 149597870700.0
C_MPS = 299792458.0
GM_SUN = 1.32712440018e20              # heliocentric gravitational constant [m^3 s^-2]


class _Law(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "L0", "Lrate", "xi", "nu0", "Pprec", "Omega0", "wspin", "gamma", "eps_obl", "zeta_max")]


def build(force: bool = False) -> str:
    """Compile world.c into libsynth.so (gcc, OpenMP)."""
    src = os.path.join(_HERE, "world.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        lib.syn_nominal_quat.argtypes = [P(_Law), ctypes.c_int64, P(ctypes.c_double), P(ctypes.c_double)]
        lib.syn_count_transits.argtypes = [P(_Law), ctypes.c_int64, P(ctypes.c_double), P(ctypes.c_double),
                                           ctypes.c_double, ctypes.c_double, P(ctypes.c_int64)]
        lib.syn_fill_transits.argtypes = [P(_Law), ctypes.c_int64, P(ctypes.c_double), P(ctypes.c_double),
                                          ctypes.c_double, ctypes.c_double, P(ctypes.c_int64),
                                          P(ctypes.c_double), P(ctypes.c_int8)]
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclass
class WorldSpec:
    """Recipe of one synthetic workload (sizes, distributions, seeds)."""
    n_src: int = 20000
    years: float = 1.0
    knot_dt: float = 1800.0           # attitude knot interval [s]
    ccd_per_transit: int = 1          # 1 (single line at eta0 = 0) or 9 (AF1..AF9)
    sigma_al: float = 100.0 * UAS     # AL standard uncertainty [rad]
    ac_obs: bool = False              # one across-scan observation per transit (first CCD line)
    sigma_ac: float = 0.0             # AC standard uncertainty [rad]; 0: sigma_al * 520 / 92
    noise: bool = True                # add N(0, sigma) observation noise
    outlier_frac: float = 0.0         # fraction of obs whose noise is N(0, 50 mas)
    att_true_pert: float = 10.0 * MAS
    start_offset: float = 50.0 * MAS
    cal_true_sd: float = 1.0 * MAS
    seg_len: int = 240                # attitude segment length [knot intervals]
    seg_overlap: int = 12             # L
    lambda_reg: float = 1e-2
    seed_truth: int = 0
    seed_noise: int = 1
    seed_start: int = 2
    seed_outlier: int = 3
    dec_band: tuple | None = None     # optional (dec_min, dec_max) [rad] to concentrate stars
    min_transits: int = 0             # keep only stars with at least this many transits
    robust: bool = False              # downweighting and excess attitude noise in the solvers
    eps_bucket: int = 8               # knot intervals per excess-attitude-noise bucket
    eps_a_init: float = 50.0 * MAS    # excess attitude noise assumed before the first attitude update
    # large-scale AL geometric calibration (Sect. 3.4): per calibration cell
    # (day and field of view) and CCD, three shifted-Legendre coefficients
    # in the across-scan pixel coordinate, in place of one offset per cell;
    # true coefficients N(0, geo_sd[r]), the constant terms summing to zero
    # over the fields of view and CCDs of each day
    geo_cal: bool = False
    geo_sd: tuple = (1.0 * MAS, 0.3 * MAS, 0.1 * MAS)
    # with geo_cal and ac_obs: the large-scale AC calibration too (three
    # coefficients per AC cell and CCD for the across-scan records, an AC
    # cell being a field of view and a 'long' interval of geo_ac_days days,
    # whose constant terms sum to zero over the cell's CCDs, eq:cc3); each
    # transit's AC record is then taken on one of its CCD lines, drawn
    # uniformly, at that line's time
    geo_ac: bool = False
    geo_ac_days: int = 30
    # with geo_cal: the small-scale AL calibration too, one value per CCD,
    # long interval of geo_small_days days and pixel column m = round(mu);
    # true values N(0, geo_small_sd) less their least-squares quadratic in
    # the column centre (eq:cc2) per CCD and interval, start values zero
    geo_small: bool = False
    geo_small_days: int = 30
    geo_small_sd: float = 0.2 * MAS
    # the Sun's gravitational light deflection in the model, with the PPN
    # parameter gamma = 1 + g0 (eq:gammaPPN) solved by the global block:
    # true g0 = 0 (general relativity), start value g0_start
    ppn: bool = False
    g0_start: float = 1e-3


@dataclass
class World:
    spec: WorldSpec
    consts: dict
    knots: np.ndarray
    src_true: np.ndarray
    att_true: np.ndarray
    cal_true: np.ndarray
    src_start: np.ndarray
    att_start: np.ndarray
    cal_start: np.ndarray
    t: np.ndarray
    src: np.ndarray
    fov: np.ndarray
    cell: np.ndarray
    sigma: np.ndarray
    eps: np.ndarray
    eta_nominal: np.ndarray           # the fiducial line eta0 of each observation [rad]
    extra: dict = field(default_factory=dict)
    # geometric calibration worlds: CCD index and across-scan pixel coordinate
    # of each record, and the coefficients [n_cells][n_ccd][3] (true, start)
    ccd: np.ndarray | None = None
    mu: np.ndarray | None = None
    geo_true: np.ndarray | None = None
    geo_start: np.ndarray | None = None
    # geo_ac worlds: each record's AC calibration cell (-1 for along-scan
    # records), and the AC coefficients [n_ac_cells][n_ccd][3]
    ac_cell: np.ndarray | None = None
    geo_ac_true: np.ndarray | None = None
    geo_ac_start: np.ndarray | None = None
    # geo_small worlds: the small-scale coefficients [K][n_ccd][1966]
    geo_small_true: np.ndarray | None = None
    geo_small_start: np.ndarray | None = None
    # the global parameter g0 (true and start values)
    g0_true: float = 0.0
    g0_start: float = 0.0

    @property
    def n_obs(self) -> int:
        return int(self.t.shape[0])

    @property
    def n_att(self) -> int:
        return int(self.att_true.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cal_true.shape[0])


def default_law() -> dict:
    return dict(L0=0.3, Lrate=2.0 * np.pi / YEAR, xi=45.0 * DEG, nu0=0.7, Pprec=63.0 * DAY,
                Omega0=0.2, wspin=60.0 * ARCSEC, gamma=106.5 * DEG, eps_obl=23.4392811 * DEG,
                zeta_max=0.35 * DEG)


def _law_struct(law: dict) -> _Law:
    return _Law(**{k: float(law[k]) for k in [f[0] for f in _Law._fields_]})


def knot_sequence(t_beg: float, t_end: float, dt: float) -> np.ndarray:
    """Regular knots of spacing dt with 4-fold knots at both ends (M = 4)."""
    K = int(round((t_end - t_beg) / dt))
    inner = t_beg + dt * np.arange(K + 1, dtype=np.float64)
    inner[-1] = t_end
    return np.concatenate([np.full(3, t_beg), inner, np.full(3, t_end)])


def nominal_quaternions(law: dict, t: np.ndarray) -> np.ndarray:
    lib = _load()
    t = np.ascontiguousarray(t, dtype=np.float64)
    q = np.empty((t.shape[0], 4), dtype=np.float64)
    L = _law_struct(law)
    lib.syn_nominal_quat(ctypes.byref(L), t.shape[0], _ptr(t, ctypes.c_double), _ptr(q, ctypes.c_double))
    return q


def find_transits(law: dict, ra: np.ndarray, dec: np.ndarray, t0: float, t1: float):
    """Transit times and fov codes grouped by star; returns (offsets, t, fov)."""
    lib = _load()
    ra = np.ascontiguousarray(ra, dtype=np.float64)
    dec = np.ascontiguousarray(dec, dtype=np.float64)
    n = ra.shape[0]
    counts = np.empty(n, dtype=np.int64)
    L = _law_struct(law)
    lib.syn_count_transits(ctypes.byref(L), n, _ptr(ra, ctypes.c_double), _ptr(dec, ctypes.c_double),
                           t0, t1, _ptr(counts, ctypes.c_int64))
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    tt = np.empty(off[-1], dtype=np.float64)
    ff = np.empty(off[-1], dtype=np.int8)
    lib.syn_fill_transits(ctypes.byref(L), n, _ptr(ra, ctypes.c_double), _ptr(dec, ctypes.c_double),
                          t0, t1, _ptr(off, ctypes.c_int64), _ptr(tt, ctypes.c_double), _ptr(ff, ctypes.c_int8))
    return off, tt, ff


def _qmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product of quaternion rows {x, y, z, w} (generic algebra)."""
    ax, ay, az, aw = a[:, 0], a[:, 1], a[:, 2], a[:, 3]
    bx, by, bz, bw = b[:, 0], b[:, 1], b[:, 2], b[:, 3]
    return np.stack([aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw,
                     aw * bw - ax * bx - ay * by - az * bz], axis=1)


def _small_rotation(phi: np.ndarray) -> np.ndarray:
    """Unit quaternions of rotation vectors phi (rows), axis-angle form."""
    ang = np.sqrt((phi * phi).sum(axis=1))
    out = np.zeros((phi.shape[0], 4))
    out[:, 3] = 1.0
    nz = ang > 0
    s = np.sin(0.5 * ang[nz]) / ang[nz]
    out[nz, :3] = phi[nz] * s[:, None]
    out[nz, 3] = np.cos(0.5 * ang[nz])
    return out


def _sign_continuous(q: np.ndarray) -> np.ndarray:
    q = q.copy()
    for i in range(1, q.shape[0]):
        if np.dot(q[i], q[i - 1]) < 0.0:
            q[i] = -q[i]
    return q


def _sign_continuous_fast(q: np.ndarray) -> np.ndarray:
    # flips are cumulative: q_i keeps its sign iff an even number of negative
    # neighbour products occur up to i
    d = (q[1:] * q[:-1]).sum(axis=1) < 0.0
    flips = np.concatenate([[0], np.cumsum(d)]) % 2
    return np.where(flips[:, None] == 1, -q, q)


def _unit_norm_ends(knots: np.ndarray, a: np.ndarray, n_end: int = 6, n_iter: int = 8) -> np.ndarray:
    """Rescale the first and last n_end coefficients so that the spline's
    norm stays close to one over the end intervals too.  The closed-form
    rescaling above assumes equally spaced knots; next to the 4-fold end
    knots the B-spline weights differ, and so would the norm.  The scales
    are fitted by Gauss-Newton to |q(t)|^2 = 1 on a dense sample of the
    end intervals (SciPy's B-spline basis), the other coefficients held."""
    from scipy.interpolate import BSpline
    N = a.shape[0]
    if N < 2 * n_end + 4:
        return a
    a = a.copy()
    for side in (0, 1):
        idx = np.arange(n_end) if side == 0 else np.arange(N - n_end, N)
        t0, t1 = (knots[3], knots[3 + n_end - 2]) if side == 0 else (knots[N - n_end + 2], knots[N])
        ts = np.linspace(t0, t1, 40 * n_end)
        ts[-1] = np.nextafter(ts[-1], -np.inf) if side == 0 else ts[-1]
        B = BSpline.design_matrix(ts, knots, 3).toarray()
        sc = np.ones(n_end)
        for _ in range(n_iter):
            a_s = a.copy()
            a_s[idx] *= sc[:, None]
            q = B @ a_s                                   # (samples, 4)
            res = 1.0 - (q * q).sum(axis=1)
            # d|q|^2 / d sc_m = 2 q . (B_m a_m)
            J = 2.0 * np.stack([(q * (B[:, m][:, None] * a[m])).sum(axis=1) for m in idx], axis=1)
            sc += np.linalg.lstsq(J, res, rcond=None)[0]
        a[idx] *= sc[:, None]
    return a


def make_world(spec: WorldSpec, law: dict | None = None, progress=None) -> World:
    """Generate one seeded synthetic workload (no observed field angles).
    progress(message), if given, is called at each stage."""
    say = progress if progress is not None else (lambda m: None)
    law = dict(default_law() if law is None else law)
    T = spec.years * YEAR
    t_beg, t_end = -0.5 * T, 0.5 * T
    knots = knot_sequence(t_beg, t_end, spec.knot_dt)
    N = knots.shape[0] - 4

    rng = np.random.default_rng(spec.seed_truth)
    # with a primary-source selection, draw extra candidates and keep the
    # first n_src that pass it
    n = spec.n_src if spec.min_transits <= 0 else int(spec.n_src * 1.5) + 64
    ra = rng.uniform(0.0, 2.0 * np.pi, n)
    if spec.dec_band is None:
        sd = rng.uniform(-1.0, 1.0, n)
    else:
        sd = rng.uniform(np.sin(spec.dec_band[0]), np.sin(spec.dec_band[1]), n)
    dec = np.arcsin(sd)
    plx = rng.exponential(1.0 * MAS, n)
    pma = rng.normal(0.0, 5.0 * MAS, n)
    pmd = rng.normal(0.0, 5.0 * MAS, n)
    src_true = np.stack([ra, dec, plx, pma, pmd], axis=1)

    # true attitude: nominal orientation at the Greville abscissa of each
    # B-spline (mean of its three interior knots), right-multiplied by a
    # random small rotation
    tgrev = (knots[1:N + 1] + knots[2:N + 2] + knots[3:N + 3]) / 3.0
    qn = _sign_continuous_fast(nominal_quaternions(law, tgrev))
    pert = _small_rotation(rng.normal(0.0, spec.att_true_pert, (N, 3)))
    att_true = _sign_continuous_fast(_qmul(qn, pert))
    # The coefficients of a spline sweeping a rotation are unit quaternions
    # spread by a 4-D angle beta between neighbours; the cubic spline through
    # them has norm close to 2/3 + (cos beta_- + cos beta_+)/6 at the knots.
    # Rescale so that the true spline stays close to unit norm (its scale is
    # unobservable; this keeps the attitude regularisation term near zero at
    # the truth).
    cosb = np.clip((att_true[1:] * att_true[:-1]).sum(axis=1), -1.0, 1.0)
    scale = np.ones(N)
    scale[1:-1] = 2.0 / 3.0 + (cosb[:-1] + cosb[1:]) / 6.0
    att_true = att_true / scale[:, None]
    att_true = _unit_norm_ends(knots, att_true)

    n_days = int(np.ceil(T / DAY - 1e-9))
    n_cells = 2 * n_days
    g = rng.normal(0.0, spec.cal_true_sd, n_days)
    cal_true = np.empty(n_cells)
    cal_true[0::2] = g
    cal_true[1::2] = -g

    # transits and per-CCD observation times
    say(f"transit search: {n} stars, {spec.years} yr")
    off, tt, ff = find_transits(law, ra, dec, t_beg, t_end)
    say(f"{tt.shape[0]} transits")
    ntr = np.diff(off)
    if spec.min_transits > 0:
        # primary-source selection: keep only well-observed stars (the
        # first n_src candidates with at least min_transits transits)
        ok = ntr >= spec.min_transits
        if ok.sum() < spec.n_src:
            raise RuntimeError("not enough candidate sources pass the transit selection")
        ok &= np.cumsum(ok) <= spec.n_src
        keep_tr = np.repeat(ok, ntr)
        tt, ff = tt[keep_tr], ff[keep_tr]
        ntr = ntr[ok]
        src_true = src_true[ok]
        ra, dec = ra[ok], dec[ok]
        n = int(ok.sum())
    if spec.ccd_per_transit == 1:
        eta0 = np.array([0.0])
    else:
        eta0 = (np.arange(1, 10) - 5) * 300.0 * ARCSEC
    nc = eta0.shape[0]
    # along scan, images move toward decreasing field angle: the image is on
    # the line eta0 at time t_c - eta0 / wspin; sort per transit by time
    order = np.argsort(-eta0, kind="stable")
    eta0 = eta0[order]
    t_obs = (tt[:, None] - eta0[None, :] / law["wspin"]).reshape(-1)
    fov = np.repeat(ff, nc)
    src_idx = np.repeat(np.repeat(np.arange(n, dtype=np.int32), ntr), nc)
    eta_nom = np.tile(eta0, tt.shape[0])
    keep = (t_obs >= t_beg) & (t_obs <= t_end)
    t_obs, fov, src_idx, eta_nom = t_obs[keep], fov[keep], src_idx[keep], eta_nom[keep]
    ccd = mu = mu_tr = ac_cell = None
    if spec.geo_cal:
        # CCD index in the order the image crosses the lines; one across-scan
        # pixel coordinate per transit, drawn uniformly over the 1966 pixel
        # columns (a stand-in for the star's position across the field)
        rng_g = np.random.default_rng([spec.seed_truth, 7])
        mu_tr = rng_g.uniform(13.5, 1979.5, tt.shape[0]).astype(np.float32)
        ccd = np.tile(np.arange(nc, dtype=np.int8), tt.shape[0])[keep]
        mu = np.repeat(mu_tr, nc)[keep]
    day = np.floor((t_obs - t_beg) / DAY).astype(np.int64)
    day = np.minimum(day, n_days - 1)
    cell = (2 * day + (fov == -1)).astype(np.int32)
    sigma = np.full(t_obs.shape[0], spec.sigma_al, dtype=np.float32)

    say(f"{t_obs.shape[0]} observations; noise and start values")
    rng_n = np.random.default_rng(spec.seed_noise)
    if spec.noise:
        eps = rng_n.standard_normal(t_obs.shape[0]) * sigma.astype(np.float64)
    else:
        eps = np.zeros(t_obs.shape[0])
    if spec.outlier_frac > 0.0:
        rng_o = np.random.default_rng(spec.seed_outlier)
        bad = rng_o.random(t_obs.shape[0]) < spec.outlier_frac
        eps[bad] = rng_o.normal(0.0, 50.0 * MAS, int(bad.sum()))
    if spec.ac_obs:
        # across-scan observations, appended after the along-scan ones: one
        # per transit at the time of its first CCD line, AC uncertainty in
        # the ratio of the paper's bright-star figures (520 / 92 uas), noise
        # from a stream of its own
        ccd_tr = np.zeros(tt.shape[0], np.int64)
        if spec.geo_cal and spec.geo_ac:
            ccd_tr = np.random.default_rng([spec.seed_truth, 9]).integers(0, nc, tt.shape[0])
        t_ac = tt - eta0[ccd_tr] / law["wspin"]
        src_tr = np.repeat(np.arange(n, dtype=np.int32), ntr)
        k_ac = (t_ac >= t_beg) & (t_ac <= t_end)
        t_ac, f_ac, s_ac = t_ac[k_ac], ff[k_ac], src_tr[k_ac]
        sig_ac = spec.sigma_ac if spec.sigma_ac > 0.0 else spec.sigma_al * 520.0 / 92.0
        sg_ac = np.full(t_ac.shape[0], sig_ac, dtype=np.float32)
        if spec.noise:
            e_ac = np.random.default_rng([spec.seed_noise, 1]).standard_normal(t_ac.shape[0]) * sg_ac.astype(
                np.float64)
        else:
            e_ac = np.zeros(t_ac.shape[0])
        t_obs = np.concatenate([t_obs, t_ac])
        fov = np.concatenate([fov, f_ac])
        src_idx = np.concatenate([src_idx, s_ac])
        eta_nom = np.concatenate([eta_nom, eta0[ccd_tr[k_ac]]])
        n_al = cell.shape[0]
        cell = np.concatenate([cell, np.full(t_ac.shape[0], -1, np.int32)])
        sigma = np.concatenate([sigma, sg_ac])
        eps = np.concatenate([eps, e_ac])
        if spec.geo_cal:
            ccd = np.concatenate([ccd, ccd_tr[k_ac].astype(np.int8)])
            mu = np.concatenate([mu, mu_tr[k_ac]])
        if spec.geo_cal and spec.geo_ac:
            # the AC record's calibration cell: its long interval and field
            # of view
            day_ac = np.minimum(np.floor((t_ac - t_beg) / DAY).astype(np.int64), n_days - 1)
            ac_cell = np.full(t_obs.shape[0], -1, np.int32)
            ac_cell[n_al:] = (2 * (day_ac // spec.geo_ac_days) + (f_ac == -1)).astype(np.int32)

    rng_s = np.random.default_rng(spec.seed_start)
    so = spec.start_offset
    src_start = src_true.copy()
    src_start[:, 0] += rng_s.normal(0.0, so, n) / np.cos(dec)
    src_start[:, 1] += rng_s.normal(0.0, so, n)
    src_start[:, 2] += rng_s.normal(0.0, so, n)
    src_start[:, 3] += rng_s.normal(0.0, so, n)
    src_start[:, 4] += rng_s.normal(0.0, so, n)
    att_start = _qmul(att_true, _small_rotation(rng_s.normal(0.0, so, (N, 3))))
    dcal = rng_s.normal(0.0, so, n_days)
    cal_start = cal_true.copy()
    cal_start[0::2] += dcal
    cal_start[1::2] -= dcal
    geo_true = geo_start = None
    if spec.geo_cal:
        # the geometric coefficients replace the per-cell offsets, which
        # stay zero; the constant terms sum to zero over each day's fields
        # of view and CCDs (eq:cc1)
        cal_true = np.zeros(n_cells)
        cal_start = np.zeros(n_cells)
        rng_g = np.random.default_rng([spec.seed_truth, 8])
        geo_true = rng_g.normal(0.0, 1.0, (n_cells, nc, 3)) * np.asarray(spec.geo_sd)[None, None, :]
        geo_start = geo_true + np.random.default_rng([spec.seed_start, 8]).normal(0.0, 0.5 * so, (n_cells, nc, 3))
        for g in (geo_true, geo_start):
            day_mean = g[:, :, 0].reshape(n_days, 2 * nc).mean(axis=1)
            g[:, :, 0] -= np.repeat(day_mean, 2)[:, None]
    geo_ac_true = geo_ac_start = None
    n_ac_cells = 0
    if spec.geo_cal and spec.geo_ac and spec.ac_obs:
        n_ac_cells = 2 * ((n_days + spec.geo_ac_days - 1) // spec.geo_ac_days)
        rng_g = np.random.default_rng([spec.seed_truth, 10])
        geo_ac_true = rng_g.normal(0.0, 1.0, (n_ac_cells, nc, 3)) * np.asarray(spec.geo_sd)[None, None, :]
        geo_ac_start = geo_ac_true + np.random.default_rng([spec.seed_start, 10]).normal(0.0, 0.5 * so,
                                                                                         (n_ac_cells, nc, 3))
        for g in (geo_ac_true, geo_ac_start):
            g[:, :, 0] -= g[:, :, 0].mean(axis=1)[:, None]          # eq:cc3 per cell
    geo_small_true = geo_small_start = None
    if spec.geo_cal and spec.geo_small:
        n_k = (n_days + spec.geo_small_days - 1) // spec.geo_small_days
        xm = (np.arange(14, 1980) - 13.5) / 1966.0
        Lm = np.stack([np.ones_like(xm), 2.0 * xm - 1.0, 6.0 * xm * xm - 6.0 * xm + 1.0], axis=1)
        v = np.random.default_rng([spec.seed_truth, 11]).normal(0.0, spec.geo_small_sd, (n_k, nc, 1966))
        coef = np.linalg.lstsq(Lm, v.reshape(-1, 1966).T, rcond=None)[0]
        geo_small_true = v - (Lm @ coef).T.reshape(n_k, nc, 1966)
        geo_small_start = np.zeros_like(geo_small_true)

    consts = dict(
        gamma_c=law["gamma"], t_ep=0.0, t_fr=0.0, lambda_reg=spec.lambda_reg,
        seg_len=spec.seg_len, seg_overlap=spec.seg_overlap,
        eph_radius_au=1.01, eph_L0=law["L0"], eph_Lrate=law["Lrate"], eps_obl=law["eps_obl"],
        au_m=AU_M, c_mps=C_MPS, year_s=YEAR, t_beg=t_beg, t_end=t_end, law=law,
        robust=int(spec.robust), eps_bucket=spec.eps_bucket, eps_a_init=spec.eps_a_init,
        geo_ccds=nc if spec.geo_cal else 0, geo_ac_cells=int(n_ac_cells),
        geo_small_days=spec.geo_small_days if spec.geo_cal and spec.geo_small else 0,
        defl=GM_SUN / (C_MPS ** 2 * AU_M) if spec.ppn else 0.0, ppn=int(spec.ppn))
    return World(spec=spec, consts=consts, knots=knots, src_true=src_true, att_true=att_true,
                 cal_true=cal_true, src_start=src_start, att_start=att_start, cal_start=cal_start,
                 t=np.ascontiguousarray(t_obs), src=np.ascontiguousarray(src_idx),
                 fov=np.ascontiguousarray(fov), cell=np.ascontiguousarray(cell),
                 sigma=np.ascontiguousarray(sigma), eps=np.ascontiguousarray(eps),
                 eta_nominal=np.ascontiguousarray(eta_nom),
                 ccd=None if ccd is None else np.ascontiguousarray(ccd),
                 mu=None if mu is None else np.ascontiguousarray(mu), geo_true=geo_true, geo_start=geo_start,
                 ac_cell=None if ac_cell is None else np.ascontiguousarray(ac_cell), geo_ac_true=geo_ac_true,
                 geo_ac_start=geo_ac_start, geo_small_true=geo_small_true, geo_small_start=geo_small_start,
                 g0_true=0.0, g0_start=float(spec.g0_start) if spec.ppn else 0.0)
