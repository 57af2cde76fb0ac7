"""Accelerated simple iteration (Sect. 4.7) over the oracle -- TEST
INFRASTRUCTURE ONLY (the GPU library never loads it).

The simple iteration converges geometrically once its slowest mode
dominates: successive updates then shrink by a nearly constant ratio
lambda (the dominant eigenvalue of the iteration), and the updates still to
come add up to lambda / (1 - lambda) times the newest one.  The paper derives
lambda from the parallax updates of a subset of the sources (parallaxes do
not move with the frame orientation) without fixing the estimator; the
reading used here is the least-squares ratio

    lambda = sum u1 u2 / sum u2^2

of the newest (u1) to the previous (u2) parallax update over the sources 0,
stride, 2 stride, ..., clamped to [0, lambda_max].  Every parameter then
moves by f = lambda / (1 - lambda) times its newest update, and the history
of updates starts again.  An "update" is the change of the parameters over
one record period of m simple iterations (S[AC] and the frame rotator), the
right ascension measured as d alpha* = d alpha cos delta (Sect. 5.1.3,
footnote to eq:ubardiff) at the newer of the two states.

Everything here is plain NumPy on the oracle's state arrays.
"""
from __future__ import annotations

import numpy as np


class AcceleratedIteration:
    """Holds the update history of one oracle Problem."""

    def __init__(self, problem, s_ref, stride=16, lambda_max=0.99):
        if stride < 1 or not 0.0 <= lambda_max < 1.0:
            raise ValueError("stride >= 1 and 0 <= lambda_max < 1")
        self.pr = problem
        self.s_ref = s_ref
        self.stride = int(stride)
        self.lambda_max = float(lambda_max)
        self.reset()

    def _state(self):
        return self.pr.s.copy(), self.pr.a.copy(), self.pr.c.copy()

    def reset(self):
        """The current parameters become the anchor of a new history."""
        self.anchor = self._state()
        self.updates = []                    # newest last

    def record(self):
        """The change since the anchor becomes the newest update."""
        s, a, c = self._state()
        ds = s - self.anchor[0]
        ds[:, 0] = ds[:, 0] * np.cos(s[:, 1])
        self.updates.append((ds, a - self.anchor[1], c - self.anchor[2]))
        self.anchor = (s, a, c)

    def ratio(self):
        """lambda from the two newest parallax updates (clamped)."""
        u1 = self.updates[-1][0][::self.stride, 2]
        u2 = self.updates[-2][0][::self.stride, 2]
        den = np.sum(u2 * u2)
        lam = np.sum(u1 * u2) / den if den > 0 else 0.0
        if not np.isfinite(lam) or lam < 0:
            lam = 0.0
        return min(lam, self.lambda_max)

    def step(self):
        """The accelerated step: (lambda, f).  With f > 0 every parameter
        moves by f times its newest update and a new history starts; with
        lambda = 0 nothing changes and the history goes on."""
        if len(self.updates) < 2:
            raise ValueError("fewer than two recorded updates")
        lam = self.ratio()
        f = lam / (1.0 - lam)
        if f > 0:
            us, ua, uc = self.updates[-1]
            s = self.pr.s.copy()
            s[:, 0] = s[:, 0] + f * us[:, 0] / np.cos(s[:, 1])
            s[:, 1:] = s[:, 1:] + f * us[:, 1:]
            self.pr.set_state(s=s, a=self.pr.a + f * ua, c=self.pr.c + f * uc)
            self.reset()
        return lam, f

    def run(self, n_blocks, m, first_step=3):
        """n_blocks blocks of m simple iterations, each followed by a record
        and, once the history holds first_step records, the accelerated
        step.  Returns the (lambda, f) of every step tried."""
        out = []
        for _ in range(n_blocks):
            for _ in range(m):
                self.pr.iterate(self.s_ref)
            self.record()
            if len(self.updates) >= first_step:
                out.append(self.step())
        return out
