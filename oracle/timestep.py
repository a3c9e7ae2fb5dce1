"""Adaptive time steps (Sec. 2.3.3), FP64.

Test infrastructure only (see ``oracle/__init__``).

The paper bounds each time increment by the particles' largest velocity and acceleration and by
the expansion, without giving the rule. Readings:
* The interval [a0, a1] of a kick is the largest with a1 <= a0 (1 + eta_e), a1 <= a_final,
  vmax Delta(a0, a1) <= eta_v (the largest drift over the interval, in fine cells) and
  gmax K(a0, a1) Delta(a0, a1) <= eta_a (the drift that the largest velocity change would cause),
  with Delta, K the drift and kick factors, vmax the largest |p| and gmax the largest force per
  unit kick factor. When hi = min(a0 (1 + eta_e), a_final) satisfies both, a1 = hi; otherwise a1
  is found by 60 bisection steps on [a0, hi].
* Scheme: the DKD leapfrog with merged drifts; positions live at the geometric midpoints of the
  kick intervals, so the drift of step j ends at the middle of interval j + 1, which is therefore
  chosen before step j runs, from the maxima of step j - 1 (velocities after its kick, forces at
  its positions). The first two intervals use the largest speed of the initial state and no
  force.

Pins (tests/test_oracle_timestep.py): in Einstein-de Sitter the factors have closed forms,
Delta = 2 (a0^-1/2 - a1^-1/2) and K = 2 (a1^1/2 - a0^1/2), so the expansion-, velocity- and
acceleration-limited steps are known exactly; an adaptive run of the 1-D Zel'dovich plane wave
stays on the exact solution before shell crossing.
"""
from __future__ import annotations

import numpy as np

from .cosmology import Cosmology
from .pm import pm_accel


def next_a(cosmo: Cosmology, a0: float, vmax: float, gmax: float, eta_v: float, eta_a: float, eta_e: float,
           a_final: float) -> float:
    """End of the next kick interval starting at a0."""
    hi = min(a0 * (1.0 + eta_e), a_final)

    def ok(a1):
        d = cosmo.drift_factor(a0, a1)
        if vmax * d > eta_v:
            return False
        return gmax * cosmo.kick_factor(a0, a1) * d <= eta_a

    if ok(hi):
        return hi
    lo = a0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if ok(mid):
            lo = mid
        else:
            hi = mid
    if not lo > a0:
        raise RuntimeError("the adaptive time step collapsed to zero")
    return lo


def schedule_from_maxima(cosmo: Cosmology, a_init: float, a_final: float, vmax, gmax, eta_v: float,
                         eta_a: float, eta_e: float):
    """The interval ends a_0 .. a_m implied by a log of maxima (index 0: the initial state, j + 1:
    step j): a_1 and a_2 from the initial maxima, a_{i} from the maxima of step i - 3."""
    a = [a_init]
    for i in range(1, len(vmax) + 2):
        m = max(i - 2, 0)
        a.append(a_final if a[-1] >= a_final else
                 next_a(cosmo, a[-1], vmax[m], gmax[m], eta_v, eta_a, eta_e, a_final))
    return np.array(a)


class AdaptivePMRun:
    """The oracle's uncompressed PM run (oracle.pm) on the adaptive schedule, with its own maxima."""

    def __init__(self, x, p, nm: int, cosmo: Cosmology, a_init: float, a_final: float, eta_v: float,
                 eta_a: float, eta_e: float):
        self.x = np.mod(np.asarray(x, np.float64), nm)
        self.p = np.asarray(p, np.float64).copy()
        self.nm, self.cosmo, self.af = nm, cosmo, a_final
        self.eta = (eta_v, eta_a, eta_e)
        v0 = float(np.sqrt((self.p**2).sum(axis=1)).max())
        self.vmax, self.gmax = [v0], [0.0]
        a1 = self._next(a_init, v0, 0.0)
        self.a = [a_init, a1, a_final if a1 >= a_final else self._next(a1, v0, 0.0)]
        self.ah = [np.sqrt(self.a[0] * self.a[1])]
        self.x = np.mod(self.x + self.p * cosmo.drift_factor(a_init, self.ah[0]), nm)
        self.j = 0

    def _next(self, a0, v, g):
        return next_a(self.cosmo, a0, v, g, *self.eta, self.af)

    @property
    def done(self):
        return self.j > 0 and self.a[self.j] >= self.af

    def advance(self):
        j = self.j
        a = self.a
        ah = self.af if a[j + 1] >= self.af else np.sqrt(a[j + 1] * a[j + 2])
        self.ah.append(ah)
        acc = pm_accel(self.x, self.nm, self.cosmo.omega_m)
        self.p = self.p + acc * self.cosmo.kick_factor(a[j], a[j + 1])
        self.vmax.append(float(np.sqrt((self.p**2).sum(axis=1)).max()))
        self.gmax.append(float(np.sqrt((acc**2).sum(axis=1)).max()))
        self.x = np.mod(self.x + self.p * self.cosmo.drift_factor(self.ah[j], ah), self.nm)
        a.append(self.af if a[j + 2] >= self.af else self._next(a[j + 2], self.vmax[-1], self.gmax[-1]))
        self.j += 1

    def run(self, max_steps: int = 100000):
        while not self.done and self.j < max_steps:
            self.advance()
        return self.x, self.p
