"""Preconditioned conjugate gradients for AGIS (Sect. 4.7) on the oracle --
TEST INFRASTRUCTURE ONLY (tests, smoke check and benchmark baseline).

The paper names conjugate gradients as its baseline scheme and states that
it uses the same S, A and C block solves as the simple iteration in the role
of the preconditioner K, but leaves the algorithm to a companion paper.  The
scheme here is the textbook preconditioned CG (Polak-Ribiere form) for the
normal equations N x = b of the problem linearised at the current
parameters, with these definitions:

* unknowns: sources (d alpha*, d delta, d parallax, d mu_alpha*, d mu_delta),
  attitude coefficients, calibration parameters; a step v moves the state as
  the block updates do (alpha by v_alpha* / cos delta, the rest additively);
* r(x): the right-hand sides b - N x of the three blocks at state x
  (Problem.normal_rhs);
* z(x) = K^-1 r(x): the S, A and C block updates computed at one and the
  same state x (block Jacobi: A and C do not see the S update);
* p'N p: the quadratic form of the normal matrix at the current state
  (Problem.normal_quadratic), the one product with N the recurrences need;
* an iteration:
      alpha = r'z / p'N p,  x <- x + alpha p,  (r, z) <- (r(x), z(x))
      beta = max(0, r'(z - z_old) / r_old'z_old)      (Polak-Ribiere)
      p <- z + beta p
  r and z are evaluated at each new iterate rather than updated by
  recurrences, so the model's slight non-linearity and rounding do not
  accumulate in them;
* a cycle starts with the frame rotator, when a frame reference is given,
  and one evaluation at x (r, z, p = z); it runs `restart` iterations, then
  the next step starts a new cycle.  A non-positive or non-finite p'N p
  leaves x unchanged and starts a new cycle.

An iteration costs one pass of every block (as one simple iteration does)
plus one pass over the observations for p'N p.
"""
from __future__ import annotations

import numpy as np


def step_state(s, a, c, v, f, n_src, n_att):
    """State moved by f v (v in the unknowns' coordinates)."""
    vs = v[:5 * n_src].reshape(n_src, 5)
    s2 = s.copy()
    s2[:, 0] = s[:, 0] + f * vs[:, 0] / np.cos(s[:, 1])
    s2[:, 1:] = s[:, 1:] + f * vs[:, 1:]
    a2 = a + f * v[5 * n_src:5 * n_src + 4 * n_att].reshape(n_att, 4)
    c2 = c + f * v[5 * n_src + 4 * n_att:]
    return s2, a2, c2


def evaluate(pr):
    """(r, z) at the problem's current state, which is left unchanged."""
    s, a, c = pr.s.copy(), pr.a.copy(), pr.c.copy()
    rs, ra, rc = pr.normal_rhs()
    zs, _, _ = pr.source_update()
    pr.set_state(s=s)
    za, _ = pr.attitude_update()
    pr.set_state(a=a)
    zc = pr.calibration_update()
    pr.set_state(c=c)
    return np.concatenate([rs.ravel(), ra.ravel(), rc]), np.concatenate([zs.ravel(), za.ravel(), zc])


def freeze(pr):
    """The switch of the hybrid scheme: a Problem without robust weighting
    whose sigma is the robust problem's sigma_eff = 1 / sqrt(W) at its
    current state (the fixed weighted least-squares problem CG solves)."""
    from oracle import Problem
    consts = dict(pr.consts)
    consts["robust"] = 0
    out = Problem(consts, pr.knots, pr.t, pr.eta_obs, pr.sigma, pr.src, pr.fov, pr.cell, pr.s, pr.a, pr.c,
                  precision=pr.precision, sigma_eff=pr.frozen_sigma())
    if getattr(pr, "var", None) is not None:
        out.var = pr.var.copy()        # the frame rotator's weights from the last S update
    return out


class CG:
    """Iteration state of the scheme; step() and run() advance the Problem's
    state."""

    def __init__(self, pr, restart=40, s_ref=None):
        if getattr(pr, "geo", None) is not None:
            raise ValueError("conjugate gradients: the oracle's normal equations carry the cell offsets only")
        self.pr, self.restart, self.s_ref = pr, int(restart), s_ref
        self.k = 0                     # iterations done in the current cycle (0: a cycle starts next)
        self.r = self.z = self.p = None
        self.rho = 0.0
        self.alpha = self.beta = 0.0

    def step(self):
        """The start of a cycle or one CG iteration (one evaluation each)."""
        pr = self.pr
        ns, na = pr.s.shape[0], pr.a.shape[0]
        if self.k == 0:
            if self.s_ref is not None:
                pr.frame_apply(pr.frame_fit(self.s_ref))
            self.r, self.z = evaluate(pr)
            self.p = self.z.copy()
            self.rho = self.r @ self.z
            self.alpha = self.beta = 0.0
            self.k = 1
            return
        pnp = pr.normal_quadratic(self.p)
        if not (np.isfinite(pnp) and pnp > 0.0):
            self.k = 0
            self.alpha = self.beta = 0.0
            return
        alpha = self.rho / pnp
        pr.set_state(*step_state(pr.s, pr.a, pr.c, self.p, alpha, ns, na))
        r, z = evaluate(pr)
        rho = r @ z
        beta = (rho - r @ self.z) / self.rho if self.rho != 0.0 else 0.0
        beta = max(beta, 0.0)
        self.p = z + beta * self.p
        self.r, self.z, self.rho = r, z, rho
        self.alpha, self.beta = alpha, beta
        self.k = self.k + 1 if self.k < self.restart else 0

    def run(self, n):
        for _ in range(int(n)):
            self.step()
