"""The time-reversible adaptive-grid split-operator integrator, plain FP64 (test
infrastructure only: tests, the smoke check and the CPU baseline of the bench use it).

Paper: Choi & Vanicek, arXiv:1909.06412.  Equation numbers count the paper's
displayed equations in order of appearance.

State: the paper's scaled wavefunction psi^J = psi(q^J)/sqrt(C_p) (Sec. II.B) on a
q-grid centred at q_ctr, with the p-grid centred at p_ctr, and the time t.

* Potential substep (Sec. II.G.1, Eqs. (42)-(47)): psi <- U_V(h, q_0) psi (Eq. (21)),
  q_ctr fixed, p_ctr <- p_ctr - h <dV/dq>, the expectation taken in the state
  before the phase (it commutes with U_V, so before or after is the same).
* Kinetic substep (Sec. II.G.2, Eqs. (48)-(53), (55)):
  U_T,adpt(h) = f~(q_h, p_0) U~_T(h, p_0) f(q_0, p_0), q_h = q_0 + h m^-1 <p~>,
  <p~> taken from psi~ = f(q_0, p_0) psi (time-independent during the substep).
* Strang TVT / VTV stages (Eq. (5) and the remark after Eq. (6)), symmetric
  compositions (Eq. (6)).
* Observables: norm by Eq. (28); <q>, <p>, energy (Sec. III.A).
* Naive adaptive grid and the fixed grid (Sec. II.F, Eqs. (29)-(34)).

Readings where the paper leaves a choice (each also listed in the design notes):
  - <O> is normalised by the discrete norm reduced in the same pass.
  - The kinetic shift uses <p~> of the transformed state (Eq. (49)), not p_ctr.
  - The initial grid centres are the analytic expectation values (q0, p0).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .grid import Grid


@dataclass
class Wavepacket:
    grid: Grid
    psi: np.ndarray                  # scaled psi^J (Sec. II.B)
    q_ctr: np.ndarray
    p_ctr: np.ndarray
    t: float = 0.0
    log: list = field(default_factory=list)

    def copy(self) -> "Wavepacket":
        return Wavepacket(self.grid, self.psi.copy(), self.q_ctr.copy(), self.p_ctr.copy(),
                          self.t, [])

    def physical(self) -> np.ndarray:
        """psi(q^J): scale back with sqrt(C_p) (Sec. II.D)."""
        return self.grid.to_physical_q(self.psi)


def from_physical(grid: Grid, psi_phys, q_ctr, p_ctr, t: float = 0.0) -> Wavepacket:
    return Wavepacket(grid, grid.to_scaled_q(np.asarray(psi_phys, dtype=np.complex128)),
                      np.array(q_ctr, dtype=np.float64), np.array(p_ctr, dtype=np.float64), t)


def gaussian_values(qs, q0, p0, sigma, hbar=1.0):
    """prod_l (pi sigma_l^2)^(-1/4) exp[-(q_l-q0_l)^2/(2 sigma_l^2) + i p0_l (q_l-q0_l)/hbar]
    (the Gaussian of Sec. III.B, Eq. (62), one factor per axis)."""
    out = 1.0 + 0j
    for l, q in enumerate(qs):
        x = q - q0[l]
        out = out * ((np.pi * sigma[l] ** 2) ** -0.25
                     * np.exp(-x ** 2 / (2 * sigma[l] ** 2) + 1j * p0[l] * x / hbar))
    return out


def gaussian(grid: Grid, q0, p0, sigma, q_ctr=None, p_ctr=None) -> Wavepacket:
    q_ctr = np.array(q0 if q_ctr is None else q_ctr, dtype=np.float64)
    p_ctr = np.array(p0 if p_ctr is None else p_ctr, dtype=np.float64)
    vals = gaussian_values(grid.q_mesh(q_ctr), q0, p0, sigma, grid.hbar)
    vals = vals * np.ones(grid.N)
    return from_physical(grid, vals, q_ctr, p_ctr)


def _inv_mass_matrix(inv_mass, D):
    m = np.asarray(inv_mass, dtype=np.float64)
    return np.diag(m) if m.ndim == 1 else m.reshape(D, D)


def kinetic_T(ps, minv):
    """T(p) = 1/2 p^T m^-1 p, Eq. (3)."""
    D = len(ps)
    t = 0.0
    for a in range(D):
        for b in range(D):
            if minv[a, b] != 0.0:
                t = t + 0.5 * minv[a, b] * ps[a] * ps[b]
    return t


# ---------------------------------------------------------------------------
# Substeps
# ---------------------------------------------------------------------------
def V_substep(wp: Wavepacket, h: float, pot, *, move_grid: bool = True) -> None:
    """Sec. II.G.1: psi <- U_V(h, q_0) psi (Eq. (45)), q fixed (Eq. (46)),
    p <- p - h <dV/dq>_{psi_0} (Eq. (47))."""
    g = wp.grid
    qs = g.q_mesh(wp.q_ctr)
    w = np.abs(wp.psi) ** 2
    n = w.sum()
    if move_grid:
        grad = pot.grad(qs)
        force = np.array([np.sum(w * gl) / n for gl in grad])
    wp.psi = wp.psi * np.exp(-1j * h * pot.V(qs) / g.hbar)          # Eq. (21)
    if move_grid:
        wp.p_ctr = wp.p_ctr - h * force


def T_substep(wp: Wavepacket, h: float, inv_mass, *, move_grid: bool = True) -> None:
    """Sec. II.G.2, Eq. (55): psi <- f~(q_h, p_0) U~_T(h, p_0) f(q_0, p_0) psi with
    q_h = q_0 + h m^-1 <p~> (Eqs. (49), (52)); p unchanged (Eq. (53))."""
    g = wp.grid
    minv = _inv_mass_matrix(inv_mass, g.D)
    q0, p0 = wp.q_ctr, wp.p_ctr
    psit = g.f(wp.psi, q0, p0)                                       # to the p-grid at p_0
    ps = g.p_mesh(p0)
    if move_grid:
        w = np.abs(psit) ** 2
        n = w.sum()
        pmean = np.array([np.sum(w * pl) / n for pl in ps])          # <p~>, Eq. (49)
        q_new = q0 + h * (minv @ pmean)                              # Eq. (52)
    else:
        q_new = q0
    psit = psit * np.exp(-1j * h * kinetic_T(ps, minv) / g.hbar)    # Eq. (22)
    wp.psi = g.f_tilde(psit, q_new, p0)                              # back on the moved q-grid
    wp.q_ctr = np.array(q_new, dtype=np.float64)


# ---------------------------------------------------------------------------
# Stages, compositions, steps
# ---------------------------------------------------------------------------
def stage(wp: Wavepacket, h: float, pot, inv_mass, split: str = "TVT",
          move_grid: bool = True) -> None:
    """TVT: U_T(h/2) U_V(h) U_T(h/2) (Eq. (5)); VTV exchanges T and V."""
    if split == "TVT":
        T_substep(wp, h / 2, inv_mass, move_grid=move_grid)
        V_substep(wp, h, pot, move_grid=move_grid)
        T_substep(wp, h / 2, inv_mass, move_grid=move_grid)
    elif split == "VTV":
        V_substep(wp, h / 2, pot, move_grid=move_grid)
        T_substep(wp, h, inv_mass, move_grid=move_grid)
        V_substep(wp, h / 2, pot, move_grid=move_grid)
    else:
        raise ValueError(split)


def strang():
    return np.array([1.0])


def triple_jump(order: int) -> np.ndarray:
    """Symmetric triple-jump composition (Yoshida 1990, cited with Eq. (6)): from order
    2n to 2n+2 with (a, b, a), a = 1/(2 - 2^(1/(2n+1))), b = 1 - 2a."""
    if order < 2 or order % 2:
        raise ValueError("order must be even and >= 2")
    g = np.array([1.0])
    for n in range(1, order // 2):
        x = 2.0 ** (1.0 / (2 * n + 1))
        a = 1.0 / (2.0 - x)
        b = 1.0 - 2.0 * a
        g = np.concatenate([a * g, b * g, a * g])
    return g


def suzuki_fractal(order: int) -> np.ndarray:
    """Suzuki's fractal composition (Suzuki 1990, cited with Eq. (6)): from order 2n to
    2n+2 with (a, a, 1-4a, a, a), a = 1/(4 - 4^(1/(2n+1)))."""
    if order < 2 or order % 2:
        raise ValueError("order must be even and >= 2")
    g = np.array([1.0])
    for n in range(1, order // 2):
        x = 4.0 ** (1.0 / (2 * n + 1))
        a = 1.0 / (4.0 - x)
        g = np.concatenate([a * g, a * g, (1 - 4 * a) * g, a * g, a * g])
    return g


def composition(comp: str, order: int, gammas=None) -> np.ndarray:
    if comp == "strang" or order == 2 and comp != "user":
        return strang()
    if comp == "suzuki":
        return suzuki_fractal(order)
    if comp == "triple_jump":
        return triple_jump(order)
    if comp == "user":
        return np.asarray(gammas, dtype=np.float64)
    raise ValueError(comp)


def step(wp: Wavepacket, dt: float, gammas, pot, inv_mass, split="TVT",
         move_grid: bool = True) -> None:
    """U_comp(dt) = U_TVT(gamma_Nc dt) ... U_TVT(gamma_1 dt), Eq. (6)."""
    for gk in gammas:
        stage(wp, gk * dt, pot, inv_mass, split, move_grid)
    wp.t += dt


def propagate(wp: Wavepacket, dt: float, nsteps: int, gammas, pot, inv_mass,
              split="TVT", move_grid: bool = True, callback=None) -> Wavepacket:
    for i in range(int(nsteps)):
        step(wp, dt, gammas, pot, inv_mass, split, move_grid)
        if callback is not None:
            callback(i + 1, wp)
    return wp


# ---------------------------------------------------------------------------
# The naive adaptive grid and the fixed grid (Sec. II.F)
# ---------------------------------------------------------------------------
def naive_step(wp: Wavepacket, dt: float, gammas, pot, inv_mass, split="TVT") -> None:
    """Eqs. (29)-(34): propagate on the frozen grid, then re-centre on the new
    expectation values: psi(q_dt) = f~(q_dt, p_dt) f(q_0, p_dt) psi_dt(q_0)."""
    g = wp.grid
    q0, p0 = wp.q_ctr.copy(), wp.p_ctr.copy()
    step(wp, dt, gammas, pot, inv_mass, split, move_grid=False)
    w = np.abs(wp.psi) ** 2
    qs = g.q_mesh(q0)
    q_new = np.array([np.sum(w * ql) / w.sum() for ql in qs])
    psit = g.f(wp.psi, q0, p0)
    wt = np.abs(psit) ** 2
    ps = g.p_mesh(p0)
    p_new = np.array([np.sum(wt * pl) / wt.sum() for pl in ps])
    psit = g.f(wp.psi, q0, p_new)
    wp.psi = g.f_tilde(psit, q_new, p_new)
    wp.q_ctr, wp.p_ctr = q_new, p_new


# ---------------------------------------------------------------------------
# Observables and grid tools
# ---------------------------------------------------------------------------
def observables(wp: Wavepacket, pot, inv_mass) -> dict:
    g = wp.grid
    minv = _inv_mass_matrix(inv_mass, g.D)
    phys = wp.physical()
    norm = float(np.prod(g.dq) * np.sum(np.abs(phys) ** 2))            # Eq. (28)
    qs = g.q_mesh(wp.q_ctr)
    w = np.abs(wp.psi) ** 2
    w = w / w.sum()
    q_mean = np.array([np.sum(w * ql) for ql in qs])
    psit = g.f(wp.psi, wp.q_ctr, wp.p_ctr)
    wt = np.abs(psit) ** 2
    wt = wt / wt.sum()
    ps = g.p_mesh(wp.p_ctr)
    p_mean = np.array([np.sum(wt * pl) for pl in ps])
    e_kin = float(np.sum(wt * kinetic_T(ps, minv)))
    e_pot = float(np.sum(w * pot.V(qs)))
    return dict(norm=norm, q=q_mean, p=p_mean, q_ctr=wp.q_ctr.copy(), p_ctr=wp.p_ctr.copy(),
                Ekin=e_kin, Epot=e_pot, E=e_kin + e_pot, t=wp.t)


def regrid(wp: Wavepacket, new_q_ctr) -> Wavepacket:
    """Trigonometric interpolation of the state onto a q-grid centred at new_q_ctr,
    keeping p_ctr: f~(q_new, p_ctr) f(q_ctr, p_ctr) psi (Sec. II.C transforms; the
    interpolation used to compare grids in Appendix A)."""
    out = wp.copy()
    g = wp.grid
    out.psi = g.f_tilde(g.f(wp.psi, wp.q_ctr, wp.p_ctr), new_q_ctr, wp.p_ctr)
    out.q_ctr = np.array(new_q_ctr, dtype=np.float64)
    return out


def inner(wp_a: Wavepacket, wp_b: Wavepacket) -> complex:
    """<psi|phi> of Eq. (28) for two states on the same grid."""
    return wp_a.grid.inner_q(wp_a.physical(), wp_b.physical())


def autocorrelation(wp: Wavepacket, psi0_fn) -> complex:
    """<psi_0|psi_t> with psi_0 evaluated analytically on the current grid points
    (Sec. III.C)."""
    g = wp.grid
    ref = psi0_fn(g.q_mesh(wp.q_ctr)) * np.ones(g.N)
    return g.inner_q(ref, wp.physical())


def spectrum(times, acf, energies, t_damp: float = 30.0, hbar: float = 1.0):
    """sigma(E) ~ Re int_0^T <psi_0|psi_t> f(t) exp(i E t / hbar) dt with
    f(t) = exp[-(t/t_damp)^2] (Fig. 9 caption); trapezoidal rule."""
    times = np.asarray(times)
    acf = np.asarray(acf)
    f = np.exp(-(times / t_damp) ** 2)
    out = []
    for E in energies:
        y = acf * f * np.exp(1j * E * times / hbar)
        out.append(np.real(np.trapezoid(y, times)))
    return np.array(out)


def state_distance(wp_a: Wavepacket, wp_b: Wavepacket) -> float:
    """|| psi_a - psi_b || (Eq. (28) norm) for two states on the same grid."""
    d = wp_a.physical() - wp_b.physical()
    return float(np.sqrt(np.prod(wp_a.grid.dq) * np.sum(np.abs(d) ** 2)))
