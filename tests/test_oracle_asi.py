"""Pins of the oracle's accelerated simple iteration (Sect. 4.7) against what
the mathematics fixes: on a linear stand-in whose iteration contracts every
parameter towards a known fixed point by a known ratio, the accelerated step
has a closed form (one geometric mode: the step lands on the fixed point; two
modes: the slow one is removed and the fast one moves by the factor the
parallaxes give); the ratio is clamped; a negative ratio takes no step."""
import numpy as np
import pytest

from oracle.asi import AcceleratedIteration


class LinearStandIn:
    """x <- x* + rho (x - x*) per parameter, rho per parameter class; the
    declination is held at its fixed point so that cos(delta) is constant
    and the right-ascension conversion is exact to rounding."""

    def __init__(self, rho_s, rho_a, rho_c, seed=0):
        rng = np.random.default_rng(seed)
        n, N, nc = 300, 40, 6
        self.s_star = np.column_stack([rng.uniform(0, 6, n), rng.uniform(-1.2, 1.2, n), rng.normal(size=(n, 3))])
        self.a_star, self.c_star = rng.normal(size=(N, 4)), rng.normal(size=nc)
        self.s = self.s_star + 1e-3 * rng.normal(size=(n, 5))
        self.s[:, 1] = self.s_star[:, 1]
        self.a = self.a_star + 1e-3 * rng.normal(size=(N, 4))
        self.c = self.c_star + 1e-3 * rng.normal(size=nc)
        self.rho_s, self.rho_a, self.rho_c = np.asarray(rho_s, float), rho_a, rho_c

    def iterate(self, s_ref):
        self.s = self.s_star + self.rho_s * (self.s - self.s_star)
        self.a = self.a_star + self.rho_a * (self.a - self.a_star)
        self.c = self.c_star + self.rho_c * (self.c - self.c_star)

    def set_state(self, s=None, a=None, c=None):
        self.s, self.a, self.c = s.copy(), a.copy(), c.copy()


def _err(p):
    return (np.abs(p.s - p.s_star).max(), np.abs(p.a - p.a_star).max(), np.abs(p.c - p.c_star).max())


def test_one_mode_lands_on_the_fixed_point():
    rho = 0.9
    p = LinearStandIn([rho, 1.0, rho, rho, rho], rho, rho)
    acc = AcceleratedIteration(p, None, stride=7)
    e0 = max(_err(p))
    out = acc.run(3, 4)                       # three records of four iterations, then the step
    assert len(out) == 1
    lam, f = out[0]
    rho_block = rho ** 4                      # the ratio of successive record updates
    assert abs(lam - rho_block) < 1e-12 and abs(f - rho_block / (1 - rho_block)) < 1e-10
    assert max(_err(p)) < 1e-12 * e0 * 1e3    # the fixed point to rounding
    assert acc.updates == []                  # a new history


def test_two_modes_closed_form():
    """Sources contract by 0.95 per iteration, attitude and calibration by
    0.5: lambda is the sources' ratio; the attitude and calibration move by
    the same factor times their own newest update."""
    r1, r2 = 0.95, 0.5
    p = LinearStandIn([r1, 1.0, r1, r1, r1], r2, r2)
    acc = AcceleratedIteration(p, None, stride=1)
    for _ in range(2):
        for _ in range(3):
            p.iterate(None)
        acc.record()
    a_before, ua = p.a.copy(), acc.updates[-1][1]
    lam, f = acc.step()
    assert abs(lam - r1 ** 3) < 1e-12
    assert _err(p)[0] < 1e-12
    # attitude: x + f u1 with u1 = (rho2^3 - 1) (x_prev - x*) = (1 - rho2^-3) (x - x*)
    np.testing.assert_allclose(p.a - p.a_star, (a_before - p.a_star) * (1 + f * (1 - r2 ** -3)), rtol=1e-9,
                               atol=1e-15)
    np.testing.assert_allclose(p.a, a_before + f * ua, rtol=0, atol=1e-15)


def test_ratio_is_clamped():
    rho = 0.998
    p = LinearStandIn([rho, 1.0, rho, rho, rho], rho, rho)
    acc = AcceleratedIteration(p, None, stride=1, lambda_max=0.99)
    lam, f = acc.run(2, 1, first_step=2)[0]
    assert lam == 0.99 and abs(f - 99.0) < 1e-9


def test_negative_ratio_takes_no_step():
    p = LinearStandIn([-0.5, 1.0, -0.5, -0.5, -0.5], 0.3, 0.3)
    acc = AcceleratedIteration(p, None, stride=1)
    s0 = None
    for _ in range(3):
        p.iterate(None)
        acc.record()
        s0 = p.s.copy()
    lam, f = acc.step()
    assert lam == 0.0 and f == 0.0
    assert np.array_equal(p.s, s0) and len(acc.updates) == 3     # history kept


def test_invalid_arguments():
    p = LinearStandIn([0.5] * 5, 0.5, 0.5)
    with pytest.raises(ValueError):
        AcceleratedIteration(p, None, stride=0)
    with pytest.raises(ValueError):
        AcceleratedIteration(p, None, lambda_max=1.0)
    acc = AcceleratedIteration(p, None)
    p.iterate(None)
    acc.record()
    with pytest.raises(ValueError):
        acc.step()
