"""Model potentials V(q) and their gradients, FP64 (test infrastructure only).

The potential substep needs V at the grid points (Eq. (21)) and the gradient
dV/dq for the Ehrenfest update of the momentum-grid centre (Eq. (47)).  Each
class takes broadcastable per-axis coordinate arrays ``qs`` (see Grid.mesh).

* Harmonic / general quadratic: Sec. III.A, Eq. (60) (the Duschinsky model uses a
  full symmetric K).
* Morse diatom + exponential repulsion: the form of the modified Secrest-Johnson
  surface, Sec. III.B, Eq. (61), generalised to
      V = De (1 - exp(-a (q1 - re)))^2 + A exp(-b (q2 - c q1)),
  which is Eq. (61) for De = D, a = beta, re = 0, A = 1, b = alpha, c = 1.
* Henon-Heiles: Sec. III.C.
"""
from __future__ import annotations

import numpy as np


class Free:
    kind = "free"

    def __init__(self, D):
        self.D = D

    def V(self, qs):
        return np.zeros(np.broadcast_shapes(*[q.shape for q in qs]))

    def grad(self, qs):
        shape = np.broadcast_shapes(*[q.shape for q in qs])
        return [np.zeros(shape) for _ in qs]


class Quadratic:
    """V = 1/2 (q - s)^T K (q - s), K real symmetric."""
    kind = "quadratic"

    def __init__(self, K, s):
        self.K = np.asarray(K, dtype=np.float64)
        self.s = np.asarray(s, dtype=np.float64)
        self.D = len(self.s)

    def V(self, qs):
        x = [q - self.s[l] for l, q in enumerate(qs)]
        v = 0.0
        for a in range(self.D):
            for b in range(self.D):
                v = v + 0.5 * self.K[a, b] * x[a] * x[b]
        return v + np.zeros(np.broadcast_shapes(*[q.shape for q in qs]))

    def grad(self, qs):
        shape = np.broadcast_shapes(*[q.shape for q in qs])
        x = [q - self.s[l] for l, q in enumerate(qs)]
        return [sum(self.K[a, b] * x[b] for b in range(self.D)) + np.zeros(shape)
                for a in range(self.D)]


class Harmonic(Quadratic):
    """V = 1/2 sum_l k_l (q_l - s_l)^2 (diagonal K)."""
    kind = "harmonic"

    def __init__(self, k, s=None):
        k = np.asarray(k, dtype=np.float64)
        super().__init__(np.diag(k), np.zeros_like(k) if s is None else s)
        self.k = k


class MorseRepulsion:
    """V(r, rho) = De (1 - exp(-a (r - re)))^2 + A exp(-b (rho - c r)); D = 1 keeps the
    Morse term alone."""
    kind = "morse_repulsion"

    def __init__(self, De, a, re, A, b, c):
        self.De, self.a, self.re, self.A, self.b, self.c = map(float, (De, a, re, A, b, c))

    def V(self, qs):
        r = qs[0]
        e = np.exp(-self.a * (r - self.re))
        v = self.De * (1 - e) ** 2
        if len(qs) > 1:                       # D = 1: the Morse oscillator alone
            v = v + self.A * np.exp(-self.b * (qs[1] - self.c * r))
        return v + np.zeros(np.broadcast_shapes(*[q.shape for q in qs]))

    def grad(self, qs):
        r = qs[0]
        shape = np.broadcast_shapes(*[q.shape for q in qs])
        e = np.exp(-self.a * (r - self.re))
        dr = 2 * self.De * self.a * e * (1 - e)
        if len(qs) == 1:
            return [dr + np.zeros(shape)]
        rep = self.A * np.exp(-self.b * (qs[1] - self.c * r))
        return [dr + self.b * self.c * rep + np.zeros(shape), -self.b * rep + np.zeros(shape)]


class HenonHeiles:
    """V = kappa/2 sum_l q_l^2 + lam sum_{l<D} (q_l^2 q_{l+1} - q_{l+1}^3 / 3)."""
    kind = "henon_heiles"

    def __init__(self, D, kappa, lam):
        self.D, self.kappa, self.lam = int(D), float(kappa), float(lam)

    def V(self, qs):
        v = sum(0.5 * self.kappa * q ** 2 for q in qs)
        for l in range(self.D - 1):
            v = v + self.lam * (qs[l] ** 2 * qs[l + 1] - qs[l + 1] ** 3 / 3.0)
        return v + np.zeros(np.broadcast_shapes(*[q.shape for q in qs]))

    def grad(self, qs):
        shape = np.broadcast_shapes(*[q.shape for q in qs])
        g = [self.kappa * q + np.zeros(shape) for q in qs]
        for l in range(self.D - 1):
            g[l] = g[l] + 2 * self.lam * qs[l] * qs[l + 1]
            g[l + 1] = g[l + 1] + self.lam * (qs[l] ** 2 - qs[l + 1] ** 2)
        return g


def from_spec(kind: str, params: dict, D: int):
    """Build a potential from the (kind, params) vocabulary of the workloads module."""
    if kind == "free":
        return Free(D)
    if kind == "harmonic":
        return Harmonic(params["k"], params.get("s"))
    if kind == "quadratic":
        return Quadratic(params["K"], params["s"])
    if kind == "morse_repulsion":
        return MorseRepulsion(params["De"], params["a"], params["re"], params["A"],
                              params["b"], params.get("c", 0.5))
    if kind == "henon_heiles":
        return HenonHeiles(D, params["kappa"], params["lam"])
    raise ValueError(kind)
