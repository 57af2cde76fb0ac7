"""Pins of the oracle's global block (Sect. 5.4, eq:normG) with the PPN
parameter gamma = 1 + g0 (eq:gammaPPN) and the Sun's gravitational light
deflection in the model (eq:astro), and of the pseudo-parameter g1 (a
global parallax shift, solved with g0, never applied).

World: the tiny world with the deflection on (the Sun at the barycentre of
the synthetic system, observer on its circular orbit of 1.01 AU), true g0 = 0.

* The deflection against its closed form: a source at elongation psi from
  the Sun appears displaced by (1 + gamma) GM / (c^2 r) cot(psi / 2), away
  from the Sun (4.03 mas at psi = 90 deg and r = 1.01 AU).
* One global update at the truth with g0 = 1e-3 returns g0 to zero.
* g1: all parallaxes shifted by 0.1 mas at the truth move g0 by less than
  1% of what a g0-only fit would take from them.
* With noise, at the start values, the update equals the weighted least
  squares of R on (dR/dg0, dR/dg1) by central differences of the model
  (the analytic partials are first order in v/c, so to 2e-4).
* Noise-free S[ACG] iterations from the truth with g0 = 1e-3 bring g0
  down monotonically, slowly: the S block takes up part of the deflection
  error into the parallaxes first (the correlation that the paper notes
  slows the simple iteration with g0).
"""
import numpy as np
import pytest

import oracle
import synth
import synth.configs as C

MAS, UAS = synth.MAS, synth.UAS


@pytest.fixture(scope="module")
def ppn_world(oracle_lib):
    w = C.make("tiny", ppn=True, noise=False)
    return w, oracle_lib.observed_field_angles(w)


def _consts(w, **over):
    c = dict(w.consts)
    c.update(over)
    return c


def _problem(w, eta, idx, consts, g0=0.0):
    return oracle.Problem(consts, w.knots, w.t[idx], eta[idx], w.sigma[idx], w.src[idx], w.fov[idx], w.cell[idx],
                          w.src_true, w.att_true, w.cal_true, g0=g0)


def test_deflection_closed_form(ppn_world):
    w, eta = ppn_world
    rng = np.random.default_rng(3)
    idx = np.sort(rng.choice(np.flatnonzero(w.cell >= 0), 400, replace=False))
    on = _problem(w, eta, idx, w.consts).observe()
    off = _problem(w, eta, idx, _consts(w, defl=0.0)).observe()
    dphi = np.asarray(on["phi"]) - np.asarray(off["phi"])
    dzeta = np.asarray(on["zeta"]) - np.asarray(off["zeta"])
    zeta = np.asarray(off["zeta"])
    disp = np.hypot(np.cos(zeta) * dphi, dzeta)
    # elongation of the source from the Sun, seen from the observer
    L = oracle.lib()
    pr = _problem(w, eta, idx, w.consts)
    ra, dec = w.src_true[w.src[idx], 0], w.src_true[w.src[idx], 1]
    rdir = np.stack([np.cos(dec) * np.cos(ra), np.cos(dec) * np.sin(ra), np.sin(dec)], axis=1)
    psi = np.empty(idx.size)
    toward = np.empty(idx.size)
    q = np.asarray(off["qraw"])
    for n, t in enumerate(w.t[idx]):
        b, v = np.zeros(3), np.zeros(3)
        L.orc_ephemeris(pr.world, float(t), b.ctypes.data_as(oracle.P(oracle.c_d)), v.ctypes.data_as(oracle.P(oracle.c_d)))
        sun = -b / np.linalg.norm(b)
        psi[n] = np.arccos(np.clip(sun @ rdir[n], -1.0, 1.0))
        # the displacement in the scanning frame against the Sun's direction there
        qn = q[n] / np.linalg.norm(q[n])
        s_srs = oracle.frame_rotate(qn, sun)
        p, z = float(off["phi"][n]), float(off["zeta"][n])
        e_phi = np.array([-np.sin(p), np.cos(p), 0.0])
        e_zeta = np.array([-np.sin(z) * np.cos(p), -np.sin(z) * np.sin(p), np.cos(z)])
        toward[n] = (np.cos(z) * dphi[n] * e_phi + dzeta[n] * e_zeta) @ s_srs
        r_au = np.linalg.norm(b)
        psi[n] = psi[n]
        disp[n] /= w.consts["defl"] / r_au
    ref = 2.0 / np.tan(psi / 2.0)                     # (1 + gamma) cot(psi / 2), gamma = 1
    print(f"elongations {np.degrees(psi.min()):.0f}..{np.degrees(psi.max()):.0f} deg; "
          f"max |displacement / closed form - 1| {np.abs(disp / ref - 1).max():.1e}; "
          f"at 90 deg and 1.01 AU: {2.0 * w.consts['defl'] / 1.01 / MAS:.3f} mas")
    np.testing.assert_allclose(disp, ref, rtol=2e-4)
    assert np.all(toward < 0.0)                       # away from the Sun


def test_global_update_recovers_g0(oracle_lib, ppn_world):
    w, eta = ppn_world
    pr = oracle_lib.problem_from_world(w, eta, state="truth")
    pr.set_state(g0=1e-3)
    d = pr.global_update()
    print(f"update {d:.6e}, g0 after {pr.g0:.2e}")
    assert abs(pr.g0) < 1e-8


def test_g1_takes_a_parallax_shift(oracle_lib, ppn_world):
    w, eta = ppn_world
    pr = oracle_lib.problem_from_world(w, eta, state="truth")
    s = w.src_true.copy()
    s[:, 2] += 0.1 * MAS
    pr.set_state(s=s)
    R = np.asarray(pr.observe()["R"])
    # a g0-only weighted fit of these residuals, with dR/dg0 by central differences
    h = 1e-4
    pr.set_state(g0=h)
    Rp = np.asarray(pr.observe()["R"])
    pr.set_state(g0=-h)
    Rm = np.asarray(pr.observe()["R"])
    pr.set_state(g0=0.0)
    g = (Rp - Rm) / (2 * h)
    W = 1.0 / w.sigma.astype(np.float64) ** 2
    d_only = -np.sum(W * g * R) / np.sum(W * g * g)
    d = pr.global_update()
    print(f"g0 update with g1 {d:.3e}, g0-only fit {d_only:.3e}")
    assert abs(d_only) > 1e-4 and abs(d) < 0.01 * abs(d_only)


def test_global_update_is_the_joint_lstsq(oracle_lib):
    w = C.make("tiny", ppn=True)
    eta = oracle_lib.observed_field_angles(w)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    R = np.asarray(pr.observe()["R"])
    h0, h1 = 1e-4, 1e-3 * MAS
    cols = []
    for step in ((h0, 0.0), (0.0, h1)):
        out = []
        for sgn in (1.0, -1.0):
            q = oracle_lib.problem_from_world(w, eta, state="start")
            s = w.src_start.copy()
            s[:, 2] += sgn * step[1]
            q.set_state(s=s, g0=w.g0_start + sgn * step[0])
            out.append(np.asarray(q.observe()["R"]))
        cols.append((out[0] - out[1]) / (2 * max(step)))
    J = np.stack(cols, axis=1)                        # dR/dg0, dR/dg1
    sw = 1.0 / w.sigma.astype(np.float64)
    ref = np.linalg.lstsq(J * sw[:, None], -R * sw, rcond=None)[0]
    d = pr.global_update()
    print(f"g0 update {d:.6e}, joint lstsq by differences {ref[0]:.6e} (g1 {ref[1] / UAS:.3f} uas)")
    assert abs(d - ref[0]) <= 2e-4 * abs(ref[0])


def test_iterations_bring_g0_down(oracle_lib, ppn_world):
    w, eta = ppn_world
    pr = oracle_lib.problem_from_world(w, eta, state="truth")
    pr.set_state(g0=1e-3)
    g = []
    for _ in range(30):
        pr.iterate(s_ref=w.src_true)
        g.append(pr.g0)
    print("g0 every 5 S[ACG] iterations:", ", ".join(f"{x:.2e}" for x in g[4::5]))
    assert all(0.0 < b < a for a, b in zip(g[1:], g[2:])) and g[-1] < 0.15e-3
