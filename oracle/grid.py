"""Grids and the grid Fourier transforms of the dynamic Fourier method (FP64).

Test infrastructure only: the product path never imports this package.

Paper: Choi & Vanicek, "A time-reversible integrator for the time-dependent
Schroedinger equation on an adaptive grid" (arXiv:1909.06412).  Equation numbers
below count the paper's displayed equations in order of appearance.

* Sec. II.B, Eqs. (9)-(10): tensor-product grid x_l^I = x_ctr,l + (i_l - N_l/2) dx_l,
  with dq_l dp_l = 2 pi hbar / N_l.
* Sec. II.B, Eqs. (12)-(16): discretised Fourier transforms, the scaled
  wavefunctions psi^J = psi(q^J)/sqrt(C_p), psi~^K = psi~(p^K)/sqrt(C_q), and the
  phase t_KJ.
* Sec. II.C, Eqs. (17)-(20): matrix form f(q_ctr, p_ctr), f~ = f^-1 = f^dagger.

The transforms here follow the paper literally: f = N^(-1/2) exp(-2 pi i <K,J>)
exp(-i t_KJ / hbar), with t_KJ split into its J-only, K-only and constant parts,
and the DFT done by scipy's FFT (library primitive).  The brute-force matrices at
the bottom build the same objects element by element for tiny grids.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.fft

# Threads of the FFT library primitive (scipy.fft's `workers`); 1 unless a caller
# (a large test, the all-core CPU baseline) asks for more.  The arithmetic does not
# depend on it.
FFT_WORKERS = 1


def set_fft_workers(n: int) -> None:
    global FFT_WORKERS
    FFT_WORKERS = max(1, int(n))


class Grid:
    """A tensor-product grid of D axes (Sec. II.B, Eqs. (9)-(10)).

    N      -- points per axis (each even, as required by the (i - N/2) offset)
    dq     -- position spacings; the momentum spacings follow from dq dp = 2 pi hbar / N.
    """

    def __init__(self, N, dq, hbar: float = 1.0):
        self.N = tuple(int(n) for n in N)
        self.D = len(self.N)
        self.dq = np.asarray(dq, dtype=np.float64).reshape(self.D)
        self.hbar = float(hbar)
        self.dp = 2.0 * np.pi * self.hbar / (np.asarray(self.N, dtype=np.float64) * self.dq)
        for n in self.N:
            if n < 2 or n % 2:
                raise ValueError("each N_l must be even and >= 2")

    @property
    def size(self) -> int:
        return int(np.prod(self.N))

    # ---- grid points, Eq. (10) -----------------------------------------
    def axis_points(self, ctr, spacing):
        return [ctr[l] + (np.arange(n) - n / 2) * spacing[l] for l, n in enumerate(self.N)]

    def q_axes(self, q_ctr):
        return self.axis_points(np.asarray(q_ctr, float), self.dq)

    def p_axes(self, p_ctr):
        return self.axis_points(np.asarray(p_ctr, float), self.dp)

    def mesh(self, axes):
        """Broadcastable per-axis coordinate arrays of the full grid."""
        out = []
        for l, a in enumerate(axes):
            sh = [1] * self.D
            sh[l] = self.N[l]
            out.append(a.reshape(sh))
        return out

    def q_mesh(self, q_ctr):
        return self.mesh(self.q_axes(q_ctr))

    def p_mesh(self, p_ctr):
        return self.mesh(self.p_axes(p_ctr))

    # ---- prefactors of Eqs. (12)-(13) ----------------------------------
    def C_q(self) -> float:
        return float(np.prod(self.dq / np.sqrt(2 * np.pi * self.hbar)))

    def C_p(self) -> float:
        return float(np.prod(self.dp / np.sqrt(2 * np.pi * self.hbar)))

    # ---- t_KJ of Eq. (16), split into its parts --------------------------
    def _t_parts(self, q_ctr, p_ctr):
        """exp(-i t_KJ/hbar) = exp(-i c/hbar) * prod_l a_l(j_l) * prod_l b_l(k_l) with
        c = sum_l (p_ctr,l - dp_l N_l/2)(q_ctr,l - dq_l N_l/2),
        a_l(j) = exp(-i (p_ctr,l j dq_l - pi hbar j)/hbar),
        b_l(k) = exp(-i (q_ctr,l k dp_l - pi hbar k)/hbar)."""
        hb = self.hbar
        c = 0.0
        a, b = [], []
        for l, n in enumerate(self.N):
            c += (p_ctr[l] - self.dp[l] * n / 2) * (q_ctr[l] - self.dq[l] * n / 2)
            j = np.arange(n)
            a.append(np.exp(-1j * (p_ctr[l] * j * self.dq[l] - np.pi * hb * j) / hb))
            b.append(np.exp(-1j * (q_ctr[l] * j * self.dp[l] - np.pi * hb * j) / hb))
        return np.exp(-1j * c / hb), self.mesh(a), self.mesh(b)

    def f(self, psi, q_ctr, p_ctr):
        """psi~ = f(q_ctr, p_ctr) psi on scaled wavefunctions (Eqs. (14), (17), (19))."""
        const, a, b = self._t_parts(np.asarray(q_ctr, float), np.asarray(p_ctr, float))
        u = psi.astype(np.complex128, copy=True)
        for al in a:
            u = u * al
        x = scipy.fft.fftn(u, norm="ortho", workers=FFT_WORKERS)   # N^(-1/2) sum_J exp(-2 pi i <K,J>) u_J
        for bl in b:
            x = x * bl
        return const * x

    def f_tilde(self, psit, q_ctr, p_ctr):
        """psi = f~(q_ctr, p_ctr) psi~ = f(q_ctr, p_ctr)^dagger psi~ (Eqs. (15), (18), (20))."""
        const, a, b = self._t_parts(np.asarray(q_ctr, float), np.asarray(p_ctr, float))
        x = psit.astype(np.complex128, copy=True)
        for bl in b:
            x = x * np.conj(bl)
        u = scipy.fft.ifftn(x, norm="ortho", workers=FFT_WORKERS)  # N^(-1/2) sum_K exp(+2 pi i <J,K>) x_K
        for al in a:
            u = u * np.conj(al)
        return np.conj(const) * u

    # ---- scaling between physical and scaled wavefunctions (Sec. II.B, II.D)
    def to_scaled_q(self, psi_phys):
        return psi_phys / np.sqrt(self.C_p())

    def to_physical_q(self, psi_scaled):
        return psi_scaled * np.sqrt(self.C_p())

    def to_physical_p(self, psit_scaled):
        return psit_scaled * np.sqrt(self.C_q())

    # ---- inner product, Eq. (28) ----------------------------------------
    def inner_q(self, psi_phys, phi_phys) -> complex:
        return complex(np.prod(self.dq) * np.vdot(psi_phys, phi_phys))


# --------------------------------------------------------------------------
# Brute-force forms for tiny grids (test pins only; O(N^2) element loops).
# --------------------------------------------------------------------------
def multi_indices(N):
    return list(itertools.product(*[range(n) for n in N]))


def f_matrix_bruteforce(grid: Grid, q_ctr, p_ctr) -> np.ndarray:
    """[f]_KJ = N^(-1/2) exp(-2 pi i <K,J>) exp(-i t_KJ/hbar), every element from
    Eqs. (16) and (19) directly, with <K,J> = sum_l k_l j_l / N_l."""
    idx = multi_indices(grid.N)
    n = len(idx)
    hb = grid.hbar
    F = np.empty((n, n), dtype=np.complex128)
    for a, K in enumerate(idx):
        for b, J in enumerate(idx):
            kj = sum(K[l] * J[l] / grid.N[l] for l in range(grid.D))
            t = 0.0
            for l in range(grid.D):
                Nl, dq, dp = grid.N[l], grid.dq[l], grid.dp[l]
                t += ((p_ctr[l] - dp * Nl / 2) * (q_ctr[l] - dq * Nl / 2)
                      + p_ctr[l] * J[l] * dq + q_ctr[l] * K[l] * dp
                      - np.pi * hb * (J[l] + K[l]))
            F[a, b] = np.exp(-2j * np.pi * kj) * np.exp(-1j * t / hb) / np.sqrt(n)
    return F


def fourier_q_to_p_bruteforce(grid: Grid, psi_phys, q_ctr, p_ctr) -> np.ndarray:
    """psi~(p^K) = C_q sum_J psi(q^J) exp(-i p^K . q^J / hbar), Eq. (12), element by element."""
    idx = multi_indices(grid.N)
    qa, pa = grid.q_axes(q_ctr), grid.p_axes(p_ctr)
    flat = psi_phys.reshape(-1)
    out = np.empty(len(idx), dtype=np.complex128)
    for a, K in enumerate(idx):
        acc = 0j
        for b, J in enumerate(idx):
            pq = sum(pa[l][K[l]] * qa[l][J[l]] for l in range(grid.D))
            acc += flat[b] * np.exp(-1j * pq / grid.hbar)
        out[a] = grid.C_q() * acc
    return out.reshape(grid.N)
