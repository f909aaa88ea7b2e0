"""Closed-form results that pin the oracle (test infrastructure only).

None of this is the method itself; these are textbook results used to check it.

* Gaussian wavepackets in Heller's parameterisation (the thawed Gaussian the paper
  cites as a future comparison in Sec. IV):
      psi(q) = N0 det(Q)^(-1/2) exp{(i/hbar)[x^T P Q^-1 x / 2 + p.x + S]},  x = q - q_t,
  with Q0 = 1, P0 = i hbar diag(1/sigma^2).  For T = p^T m^-1 p / 2 and a quadratic V
  both exact substeps map Gaussians to Gaussians:
      kinetic (time h):    Q += h m^-1 P,  q_t += h m^-1 p_t,  S += h p^T m^-1 p / 2
      potential (time h):  P -= h K Q,     p_t -= h grad V(q_t), S -= h V(q_t)
  so the *exact* split-operator product applied to a Gaussian has a closed form: the
  grid algorithm must reproduce it to the grid's spectral accuracy, and its grid
  centres must follow the Stoermer-Verlet map of (q_t, p_t) (Sec. II.H).
* The exact quadratic-Hamiltonian evolution (linear flow of (q, p), matrix exponential).
* The Morse ground state and its energy.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg
import scipy.special


@dataclass
class GaussianParams:
    Q: np.ndarray          # (D, D) complex
    P: np.ndarray          # (D, D) complex
    q: np.ndarray          # (D,) real
    p: np.ndarray          # (D,) real
    S: float
    N0: float
    sqrt_det: complex      # det(Q)^(1/2) on a continuous branch

    def copy(self):
        return GaussianParams(self.Q.copy(), self.P.copy(), self.q.copy(), self.p.copy(),
                              self.S, self.N0, self.sqrt_det)


def initial(q0, p0, sigma, hbar=1.0) -> GaussianParams:
    sigma = np.asarray(sigma, float)
    D = len(sigma)
    N0 = float(np.prod((np.pi * sigma ** 2) ** -0.25))
    return GaussianParams(np.eye(D, dtype=complex), 1j * hbar * np.diag(1.0 / sigma ** 2),
                          np.array(q0, float), np.array(p0, float), 0.0, N0, 1.0 + 0j)


def _update_sqrt_det(g: GaussianParams) -> None:
    r = np.sqrt(complex(np.linalg.det(g.Q)))
    g.sqrt_det = r if abs(r - g.sqrt_det) <= abs(r + g.sqrt_det) else -r


def kinetic(g: GaussianParams, h: float, minv) -> None:
    minv = np.diag(minv) if np.ndim(minv) == 1 else np.asarray(minv)
    g.Q = g.Q + h * minv @ g.P
    g.S = g.S + h * 0.5 * g.p @ minv @ g.p
    g.q = g.q + h * minv @ g.p
    _update_sqrt_det(g)


def potential(g: GaussianParams, h: float, K, s) -> None:
    K = np.asarray(K, float)
    x = g.q - np.asarray(s, float)
    g.P = g.P - h * K @ g.Q
    g.p = g.p - h * K @ x
    g.S = g.S - h * 0.5 * x @ K @ x


def split_operator(g: GaussianParams, dt: float, nsteps: int, gammas, K, s, minv,
                   split: str = "TVT") -> GaussianParams:
    """The exact TVT/VTV split-operator product (Eqs. (5)-(6)) acting on a Gaussian."""
    g = g.copy()
    for _ in range(int(nsteps)):
        for gk in gammas:
            h = gk * dt
            if split == "TVT":
                kinetic(g, h / 2, minv)
                potential(g, h, K, s)
                kinetic(g, h / 2, minv)
            else:
                potential(g, h / 2, K, s)
                kinetic(g, h, minv)
                potential(g, h / 2, K, s)
    return g


def exact_quadratic(g0: GaussianParams, t: float, K, s, minv) -> GaussianParams:
    """Exact evolution under H = p^T m^-1 p / 2 + (q-s)^T K (q-s) / 2 (linear flow)."""
    K = np.asarray(K, float)
    minv = np.diag(minv) if np.ndim(minv) == 1 else np.asarray(minv)
    D = K.shape[0]
    A = np.zeros((2 * D, 2 * D))
    A[:D, D:] = minv
    A[D:, :D] = -K
    # integrate the branch of det(Q)^(1/2) along the path in small increments
    n_sub = max(1, int(np.ceil(abs(t) / 0.01)))
    g = g0.copy()
    s = np.asarray(s, float)
    x0, p0 = g0.q - s, g0.p.copy()
    for i in range(1, n_sub + 1):
        Phi = scipy.linalg.expm(A * (t * i / n_sub))
        g.Q = Phi[:D, :D] @ g0.Q + Phi[:D, D:] @ g0.P
        g.P = Phi[D:, :D] @ g0.Q + Phi[D:, D:] @ g0.P
        _update_sqrt_det(g)
    Phi = scipy.linalg.expm(A * t)
    z = Phi @ np.concatenate([x0, p0])
    g.q = z[:D] + s
    g.p = z[D:]
    g.S = g0.S + 0.5 * (g.p @ (g.q - s) - p0 @ x0)      # int L dt for a quadratic H
    return g


def values(g: GaussianParams, qs, hbar=1.0) -> np.ndarray:
    """psi(q) sampled on broadcastable coordinate arrays."""
    D = len(qs)
    A = g.P @ np.linalg.inv(g.Q)
    x = [qs[l] - g.q[l] for l in range(D)]
    expo = 0.0
    for a in range(D):
        for b in range(D):
            expo = expo + 0.5 * A[a, b] * x[a] * x[b]
        expo = expo + g.p[a] * x[a]
    expo = expo + g.S
    shape = np.broadcast_shapes(*[q.shape for q in qs])
    return g.N0 / g.sqrt_det * np.exp(1j * expo / hbar) * np.ones(shape)


# ---------------------------------------------------------------------------
# Morse oscillator V = De (1 - exp(-a (r - re)))^2, reduced mass mu
# ---------------------------------------------------------------------------
def morse_lambda(De, a, mu, hbar=1.0):
    return np.sqrt(2 * mu * De) / (a * hbar)


def morse_ground_energy(De, a, mu, hbar=1.0):
    omega = a * np.sqrt(2 * De / mu)
    return hbar * omega / 2 - (hbar * omega) ** 2 / (16 * De)


def morse_ground_state(r, De, a, re, mu, hbar=1.0):
    """phi_0 = C z^(lam - 1/2) exp(-z/2), z = 2 lam exp(-a (r - re)),
    normalised with C^2 = a / Gamma(2 lam - 1)."""
    lam = morse_lambda(De, a, mu, hbar)
    z = 2 * lam * np.exp(-a * (r - re))
    logc = 0.5 * (np.log(a) - scipy.special.gammaln(2 * lam - 1))
    return np.exp(logc + (lam - 0.5) * np.log(z) - z / 2)
