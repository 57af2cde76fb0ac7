"""Named synthetic workloads (recipes only: sizes, distributions, seeds).

``gaia``   Gaia-like nominal scanning law: spin 60"/s (6 h), precession 63 d,
           solar aspect 45 deg, basic angle 106.5 deg, across-scan half
           width 0.35 deg.
``mini``   the same law with the spin slowed ten-fold and the across-scan
           width widened ten-fold.  At a 1200 s knot interval it keeps the
           Gaia ratios that matter for the solution -- the spin angle per
           knot interval (0.5 deg), about 18 transits per star per year and
           about ten transits per knot interval for 20 000 stars -- at a
           size a plain CPU implementation iterates in well under a second.
"""
from __future__ import annotations

from . import ARCSEC, DEG, MAS, UAS, WorldSpec, default_law


def gaia_law() -> dict:
    return default_law()


def mini_law() -> dict:
    law = default_law()
    law["wspin"] = law["wspin"] / 10.0
    law["zeta_max"] = law["zeta_max"] * 10.0
    return law


# name -> (law factory, WorldSpec).  Attitude segments are 240 knot
# intervals with L = 12 on each side.  Primary sources (Sect. 6.2) must admit
# a five-parameter solution: the 1-year workloads keep stars with at least
# six transits (a star seen on fewer occasions has a singular or nearly
# singular 5x5 system).
WORKLOADS = {
    # 20 000 stars, 1 yr, one AL observation per transit (~343k obs),
    # 1200 s knots (~105k attitude unknowns), 732 cells; the tiny workload
    "tiny": (mini_law, WorldSpec(n_src=20000, years=1.0, knot_dt=1200.0, ccd_per_transit=1,
                                 seg_len=240, seg_overlap=12, lambda_reg=1e-2, min_transits=6)),
    # small parity cases (seconds on one CPU core)
    "small": (mini_law, WorldSpec(n_src=4000, years=1.0, knot_dt=1200.0, ccd_per_transit=1,
                                  seg_len=240, seg_overlap=12, lambda_reg=1e-2, min_transits=6)),
    "small9": (mini_law, WorldSpec(n_src=3000, years=0.5, knot_dt=1200.0, ccd_per_transit=9,
                                   seg_len=100, seg_overlap=12, lambda_reg=1e-2)),
    # the small-scale geometric calibration needs many records per pixel
    # column: 20 000 stars over 60 days (two 30-day long intervals), 9 AF
    # observations per transit (~15 records per column, CCD and interval)
    "geo9": (mini_law, WorldSpec(n_src=20000, years=60.0 / 365.25, knot_dt=1200.0, ccd_per_transit=9,
                                 seg_len=100, seg_overlap=12, lambda_reg=1e-2, geo_cal=True)),
    # 1M stars, 1 yr, 9 AF observations per transit (~160M obs), 30 s knots;
    # segments of 130 intervals: 8,092 band systems, four per wavefront, all
    # resident on the chip at once
    "gaia1": (gaia_law, WorldSpec(n_src=1_000_000, years=1.0, knot_dt=30.0, ccd_per_transit=9,
                                  seg_len=130, seg_overlap=12, lambda_reg=1e-2, min_transits=6)),
    # 2M stars, 5 yr, 9 AF observations per transit (~1.6G obs), 1% outliers,
    # robust solvers (downweighting, excess attitude noise in 8-interval buckets)
    "gaia5": (gaia_law, WorldSpec(n_src=2_000_000, years=5.0, knot_dt=30.0, ccd_per_transit=9,
                                  seg_len=240, seg_overlap=12, lambda_reg=1e-2, outlier_frac=0.01,
                                  robust=True)),
    # iteration-scheme comparisons beyond the tiny world: the miniature law,
    # 40 000 stars, 1 yr, 9 AF observations and one across-scan record per
    # transit (~7M records, about 20x tiny), 1200 s knots (~26k coefficients,
    # ~27 transits per interval)
    "mid9_ac": (mini_law, WorldSpec(n_src=40000, years=1.0, knot_dt=1200.0, ccd_per_transit=9,
                                    seg_len=240, seg_overlap=12, lambda_reg=1e-2, min_transits=6,
                                    ac_obs=True)),
    # robust parity cases: the tiny and small worlds with 1% outliers
    "tiny_robust": (mini_law, WorldSpec(n_src=20000, years=1.0, knot_dt=1200.0, ccd_per_transit=1,
                                        seg_len=240, seg_overlap=12, lambda_reg=1e-2, min_transits=6,
                                        outlier_frac=0.01, robust=True)),
    "small_robust": (mini_law, WorldSpec(n_src=4000, years=1.0, knot_dt=1200.0, ccd_per_transit=1,
                                         seg_len=240, seg_overlap=12, lambda_reg=1e-2, min_transits=6,
                                         outlier_frac=0.01, robust=True)),
}


def workload(name: str, **overrides):
    """(law, spec) for a named workload, with optional WorldSpec overrides."""
    import dataclasses
    law_f, spec = WORKLOADS[name]
    return law_f(), dataclasses.replace(spec, **overrides)


def make(name: str, progress=None, **overrides):
    from . import make_world
    law, spec = workload(name, **overrides)
    return make_world(spec, law, progress=progress)
