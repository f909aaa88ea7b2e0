"""Pins of the FP64 CPU oracle against things other than itself: brute-force sums,
closed forms, invariants, and numbers printed in the paper (arXiv:1909.06412).

Each test names the part of the oracle it pins.  CPU only.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import closed_forms as cf

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "printed_numbers.txt")


def golden():
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, val, dec = line.split()[:3]
            out[name] = (float(val), int(dec))
    return out


def _rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# Transforms (Sec. II.B-C): brute force, unitarity, discretised continuous FT
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N,D", [((4,), 1), ((6,), 1), ((4, 2), 2), ((2, 4, 2), 3)])
def test_f_equals_bruteforce_matrix(N, D):
    rng = _rng(1)
    g = O.Grid(N, rng.uniform(0.2, 0.9, D), hbar=rng.uniform(0.5, 2.0))
    qc, pc = rng.uniform(-3, 3, D), rng.uniform(-3, 3, D)
    F = O.f_matrix_bruteforce(g, qc, pc)
    psi = W.random_state(N, seed=3)
    np.testing.assert_allclose(g.f(psi, qc, pc).reshape(-1), F @ psi.reshape(-1),
                               rtol=0, atol=1e-13)
    np.testing.assert_allclose(g.f_tilde(psi, qc, pc).reshape(-1),
                               F.conj().T @ psi.reshape(-1), rtol=0, atol=1e-13)
    # f~ = f^-1 = f^dagger (Eq. (20))
    np.testing.assert_allclose(F @ F.conj().T, np.eye(F.shape[0]), atol=1e-13)


@pytest.mark.parametrize("N", [(6,), (4, 4)])
def test_scaled_transform_matches_discretised_fourier_integral(N):
    """psi~^K = psi~(p^K)/sqrt(C_q) with psi~(p^K) from Eq. (12) summed term by term."""
    rng = _rng(2)
    D = len(N)
    g = O.Grid(N, rng.uniform(0.3, 0.8, D), hbar=1.3)
    qc, pc = rng.uniform(-2, 2, D), rng.uniform(-2, 2, D)
    phys = W.random_state(N, seed=5)
    brute = O.fourier_q_to_p_bruteforce(g, phys, qc, pc) / math.sqrt(g.C_q())
    np.testing.assert_allclose(g.f(g.to_scaled_q(phys), qc, pc), brute, atol=1e-12)


def test_spacings_satisfy_dq_dp():
    g = O.Grid((8, 6, 10), (0.3, 0.7, 0.11), hbar=0.9)
    np.testing.assert_allclose(g.dq * g.dp * np.array(g.N), 2 * np.pi * 0.9, rtol=1e-15)


# ---------------------------------------------------------------------------
# Whole machinery: exact discrete-Gaussian map for quadratic V (P1), centres vs
# Stoermer-Verlet (P3)
# ---------------------------------------------------------------------------
def _grid_vs_map(w, nsteps, gam):
    g = O.Grid(w["N"], w["dq"], w["hbar"])
    wp = O.gaussian(g, w["q0"], w["p0"], w["sigma"])
    kind, par = w["potential"]
    pot = O.potentials.from_spec(kind, par, w["D"])
    O.run(wp, w["dt"], nsteps, gam, pot, w["inv_mass"], w["split"])
    K = pot.K
    g0 = cf.initial(w["q0"], w["p0"], w["sigma"], w["hbar"])
    gm = cf.split_operator(g0, w["dt"], nsteps, gam, K, pot.s, w["inv_mass"], w["split"])
    ref = cf.values(gm, g.q_mesh(wp.q_ctr), w["hbar"])
    err = math.sqrt(np.prod(g.dq) * np.sum(np.abs(wp.physical() - ref) ** 2))
    return err, wp, gm


def test_P1_harmonic_1d_thousand_steps():
    w = W.harmonic_1d()
    err, wp, gm = _grid_vs_map(w, w["steps"], O.composition("strang", 2))
    assert err < 1e-12
    np.testing.assert_allclose(wp.q_ctr, gm.q, atol=1e-12)     # Verlet centres (Sec. II.H)
    np.testing.assert_allclose(wp.p_ctr, gm.p, atol=1e-12)


@pytest.mark.parametrize("split", ["TVT", "VTV"])
def test_P1_harmonic_3d_suzuki4(split):
    w = W.harmonic_3d(seed=1, n=48, dq=0.3, dt=0.05)
    w["split"] = split
    err, wp, gm = _grid_vs_map(w, 8, O.composition("suzuki", 4))
    assert err < 1e-11
    np.testing.assert_allclose(wp.q_ctr, gm.q, atol=1e-12)
    np.testing.assert_allclose(wp.p_ctr, gm.p, atol=1e-12)


def test_P1_full_K_and_full_inverse_mass():
    """Non-diagonal K (Duschinsky model, Table I) and non-diagonal m^-1."""
    w = W.duschinsky_3d(n=40, dq=0.35)
    w["inv_mass"] = np.array([[2.0, 0.1, 0.0], [0.1, 1.0, -0.05], [0.0, -0.05, 2.5]])
    w["dt"] = 0.02
    w["q0"], w["p0"] = [-0.5, 0.3, 0.2], [0.4, -0.2, 0.1]
    err, wp, gm = _grid_vs_map(w, 15, O.composition("triple_jump", 4))
    assert err < 1e-10
    np.testing.assert_allclose(wp.q_ctr, gm.q, atol=1e-12)


def test_P1_centres_leave_initial_grid():
    """The grid follows the packet well beyond the initial grid's span."""
    w = W.harmonic_1d()
    w["q0"], w["p0"], w["N"] = [0.0], [20.0], [128]
    w["potential"] = ("harmonic", {"k": [0.01], "s": [0.0]})
    err, wp, gm = _grid_vs_map(w, 150, O.composition("strang", 2))
    assert abs(wp.q_ctr[0]) > 20.0
    assert err < 1e-11


# ---------------------------------------------------------------------------
# Convergence order against the exact solution (P2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("comp,order,dts", [
    ("strang", 2, (0.2, 0.1)), ("suzuki", 4, (0.2, 0.1)), ("triple_jump", 4, (0.2, 0.1)),
    ("triple_jump", 6, (0.2, 0.1)), ("suzuki", 6, (0.2, 0.1)), ("triple_jump", 8, (0.2, 0.1)),
    ("triple_jump", 10, (0.2, 0.1))])
def test_P2_observed_order(comp, order, dts):
    gam = O.composition(comp, order)
    errs = []
    for dt in dts:
        g = O.Grid([64], [0.3])
        wp = O.gaussian(g, [0.5], [0.3], [1.0])
        pot = O.potentials.Harmonic([2.25])
        O.run(wp, dt, int(round(3.0 / dt)), gam, pot, [1.0])
        ge = cf.exact_quadratic(cf.initial([0.5], [0.3], [1.0]), 3.0, [[2.25]], [0.0], [1.0])
        ex = cf.values(ge, g.q_mesh(wp.q_ctr))
        errs.append(math.sqrt(0.3 * np.sum(np.abs(wp.physical() - ex) ** 2)))
    slope = math.log2(errs[0] / errs[1])
    assert abs(slope - order) < 0.35, (errs, slope)


def test_P2_exact_ho_solution_is_a_solution():
    """The closed-form exact evolution agrees with the Strang map as dt -> 0 and with
    the period: after 2 pi / omega the coherent state returns up to the phase -1."""
    g0 = cf.initial([1.0], [0.0], [1.0])
    ge = cf.exact_quadratic(g0, 2 * np.pi, [[1.0]], [0.0], [1.0])
    q = [np.linspace(-5, 5, 11)]
    np.testing.assert_allclose(cf.values(ge, q), -cf.values(g0, q), atol=1e-12)


# ---------------------------------------------------------------------------
# Invariants: norm (P4), reversibility (P5), merging (P7)
# ---------------------------------------------------------------------------
def _hh(n=8, D=3, lam=0.111803):
    w = W.henon_heiles_8d(n=n, D=D, dq=0.8, lam=lam)
    g = O.Grid(w["N"], w["dq"])
    return w, g, O.gaussian(g, w["q0"], w["p0"], w["sigma"]), \
        O.potentials.from_spec(*w["potential"], w["D"])


def test_P4_norm_conserved_anharmonic():
    w, g, wp, pot = _hh()
    n0 = O.observables(wp, pot, w["inv_mass"])["norm"]
    O.run(wp, 0.05, 60, O.composition("suzuki", 4), pot, w["inv_mass"])
    assert abs(O.observables(wp, pot, w["inv_mass"])["norm"] - n0) < 2e-12   # 900 substeps of rounding


def test_P5_time_reversible():
    w, g, wp, pot = _hh()
    start = wp.copy()
    gam = O.composition("triple_jump", 6)
    O.run(wp, 0.05, 20, gam, pot, w["inv_mass"])
    assert O.state_distance(wp, start) > 1e-2 or np.linalg.norm(wp.q_ctr - start.q_ctr) > 1e-2
    O.run(wp, -0.05, 20, gam, pot, w["inv_mass"])
    np.testing.assert_allclose(wp.q_ctr, start.q_ctr, atol=1e-12)
    np.testing.assert_allclose(wp.p_ctr, start.p_ctr, atol=1e-12)
    assert O.state_distance(wp, start) < 1e-12


def test_P5_morse_repulsion_reversible_vtv():
    w = W.morse_repulsion_2d(64, 64, steps=0, precision="c128")
    g = O.Grid(w["N"], w["dq"])
    wp = O.gaussian(g, w["q0"], w["p0"], w["sigma"])
    pot = O.potentials.from_spec(*w["potential"], 2)
    start = wp.copy()
    O.run(wp, 2.0, 40, O.composition("strang", 2), pot, w["inv_mass"], "VTV")
    O.run(wp, -2.0, 40, O.composition("strang", 2), pot, w["inv_mass"], "VTV")
    assert O.state_distance(wp, start) < 1e-11


def test_P7_kinetic_substeps_merge():
    w, g, wp, pot = _hh(D=2)
    a = wp.copy()
    b = wp.copy()
    O.V_substep(a, 0.3, pot)
    O.V_substep(b, 0.3, pot)
    O.T_substep(a, 0.13, w["inv_mass"])
    O.T_substep(a, 0.29, w["inv_mass"])
    O.T_substep(b, 0.42, w["inv_mass"])
    np.testing.assert_allclose(a.q_ctr, b.q_ctr, atol=1e-14)
    assert O.state_distance(a, b) < 1e-14
    O.V_substep(a, 0.2, pot)
    O.V_substep(a, 0.1, pot)
    O.V_substep(b, 0.3, pot)
    np.testing.assert_allclose(a.p_ctr, b.p_ctr, atol=1e-14)
    assert O.state_distance(a, b) < 1e-14


# ---------------------------------------------------------------------------
# Special cases (P8)
# ---------------------------------------------------------------------------
def test_P8_free_particle_exact_for_any_dt():
    g = O.Grid([96, 96], [0.35, 0.3])
    wp = O.gaussian(g, [0.3, -1.0], [1.5, -0.7], [1.0, 1.3])
    pot = O.potentials.Free(2)
    O.run(wp, 0.9, 2, O.composition("strang", 2), pot, [1.0, 0.5])
    ge = cf.exact_quadratic(cf.initial([0.3, -1.0], [1.5, -0.7], [1.0, 1.3]), 1.8,
                            np.zeros((2, 2)), [0, 0], [1.0, 0.5])
    ref = cf.values(ge, g.q_mesh(wp.q_ctr))
    assert math.sqrt(0.105 * np.sum(np.abs(wp.physical() - ref) ** 2)) < 1e-12
    # energy is exactly conserved for V = 0 (P12)
    e = O.observables(wp, pot, [1.0, 0.5])["E"]
    assert abs(e - (0.5 * 1.5 ** 2 + 0.25 * 0.7 ** 2 + 0.25 + 0.125 / 1.69)) < 1e-12


def test_P8_henon_heiles_lambda0_is_product_of_1d_runs():
    """With lambda = 0 the 3-D HH model is three uncoupled oscillators: the adaptive
    algorithm on a product state gives the product of three 1-D runs."""
    w, g, wp, pot = _hh(n=8, D=3, lam=0.0)
    gam = O.composition("suzuki", 4)
    O.run(wp, 0.1, 10, gam, pot, w["inv_mass"])
    prod = 1.0
    for l in range(3):
        g1 = O.Grid([8], [0.8])
        w1 = O.gaussian(g1, [2.0], [0.0], [1.0])
        O.run(w1, 0.1, 10, gam, O.potentials.Harmonic([1.0]), [1.0])
        assert abs(w1.q_ctr[0] - wp.q_ctr[l]) < 1e-13
        sh = [1, 1, 1]
        sh[l] = 8
        prod = prod * w1.physical().reshape(sh)
    np.testing.assert_allclose(wp.physical(), prod, atol=1e-13)


def test_P8_morse_ground_state_energy_and_stationarity():
    """Morse eigenstate: the energy observable gives E0 and propagation only rotates
    the phase by exp(-i E0 t); the grid centres stay at <r> (closed form via digamma)."""
    import scipy.special
    De, a, re, mu = 2.0, 1.0, 0.0, 4.0
    E0 = cf.morse_ground_energy(De, a, mu)
    lam = cf.morse_lambda(De, a, mu)
    r_mean = re + (math.log(2 * lam) - scipy.special.digamma(2 * lam - 1)) / a
    g = O.Grid([192], [0.08])
    phi = cf.morse_ground_state(g.q_axes([r_mean])[0], De, a, re, mu)
    wp = O.from_physical(g, phi, [r_mean], [0.0])
    pot = O.potentials.MorseRepulsion(De, a, re, 0.0, 1.0, 0.0)
    obs = O.observables(wp, pot, [1 / mu])
    assert abs(obs["norm"] - 1.0) < 1e-12
    assert abs(obs["q"][0] - r_mean) < 1e-12
    assert abs(obs["E"] - E0) < 1e-11
    O.run(wp, 0.01, 100, O.composition("suzuki", 4), pot, [1 / mu])
    ref = phi * np.exp(-1j * E0 * 1.0)
    assert abs(wp.q_ctr[0] - r_mean) < 1e-8
    assert np.max(np.abs(wp.physical() - ref)) < 1e-7


# ---------------------------------------------------------------------------
# Stability (P9)
# ---------------------------------------------------------------------------
def _verlet_matrix(gam, dt, k):
    """2x2 matrix of one composed step acting on the centres (q, p) of a unit-mass
    oscillator: the Stoermer-Verlet map of Sec. II.H composed as in Eq. (6)."""
    M = np.eye(2)
    for gk in gam:
        h = gk * dt
        half = np.array([[1.0, h / 2], [0.0, 1.0]])
        kick = np.array([[1.0, 0.0], [-h * k, 1.0]])
        M = half @ kick @ half @ M
    return M


@pytest.mark.parametrize("comp,order,dts", [("strang", 2, (1.3, 1.4)),
                                            ("triple_jump", 10, (0.3, 0.9))])
def test_P9_grid_centres_diverge_beyond_verlet_bound(comp, order, dts):
    """Eq. (57): for Strang the centres are stable iff dt < T_osc/pi = 2/omega (here
    omega = 1.5); for a composition iff the composed Verlet matrix has |trace| <= 2.
    The grid algorithm's centres diverge exactly when that linear map does."""
    gam = O.composition(comp, order)
    for dt in dts:
        tr = abs(np.trace(_verlet_matrix(gam, dt, 2.25)))
        g = O.Grid([32], [0.4375])
        wp = O.gaussian(g, [1.0], [0.5], [1.0])
        O.run(wp, dt, 60, gam, O.potentials.Harmonic([2.25]), [1.0])
        grew = (not np.isfinite(wp.q_ctr[0])) or abs(wp.q_ctr[0]) > 1e3
        assert grew == (tr > 2.0), (dt, tr, wp.q_ctr)
    if comp == "strang":
        assert abs(np.trace(_verlet_matrix(gam, 2 / 1.5 - 1e-9, 2.25))) < 2.0
        assert abs(np.trace(_verlet_matrix(gam, 2 / 1.5 + 1e-9, 2.25))) > 2.0


# ---------------------------------------------------------------------------
# Composition tables (P10)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("comp,order,stages", [
    ("suzuki", 4, 5), ("suzuki", 6, 25), ("suzuki", 8, 125), ("suzuki", 10, 625),
    ("triple_jump", 4, 3), ("triple_jump", 6, 9), ("triple_jump", 8, 27),
    ("triple_jump", 10, 81)])
def test_P10_composition_tables(comp, order, stages):
    g = O.composition(comp, order)
    assert len(g) == stages
    assert abs(g.sum() - 1.0) < 1e-13
    np.testing.assert_array_equal(g, g[::-1])                 # gamma_{N+1-k} = gamma_k
    assert abs(np.sum(g ** 3)) < 1e-13                         # order >= 4 condition
    if order >= 6:
        assert abs(np.sum(g ** 5)) < 1e-12


# ---------------------------------------------------------------------------
# Printed numbers (P11)
# ---------------------------------------------------------------------------
def test_P11_energy_duschinsky_model():
    G = golden()
    val, dec = G["E0_duschinsky_3d"]
    w = W.duschinsky_3d()                                     # K13 = +0.017 reading
    g = O.Grid(w["N"], w["dq"])
    wp = O.gaussian(g, w["q0"], w["p0"], w["sigma"])
    pot = O.potentials.from_spec(*w["potential"], 3)
    E = O.observables(wp, pot, w["inv_mass"])["E"]
    assert abs(E - val) < 0.5 * 10 ** -dec
    # the printed K13 = -0.017 would give 142.055: the sign reading is documented
    w2 = W.duschinsky_3d(k13=-0.017)
    pot2 = O.potentials.from_spec(*w2["potential"], 3)
    assert abs(O.observables(wp, pot2, w2["inv_mass"])["E"] - 142.055) < 5e-4


def test_P11_overlap_harmonic():
    val, dec = golden()["overlap_harmonic_3d"]
    w = W.duschinsky_3d()
    g = O.Grid(w["N"], w["dq"])
    psi0 = O.gaussian(g, [0, 0, 0], [0, 0, 0], [1, 1, 1], q_ctr=[0, 0, 0])
    phi0 = O.gaussian(g, [-1, 1, 1], [0, 0, 0], [1, 1, 1], q_ctr=[0, 0, 0])
    assert abs(abs(O.inner(psi0, phi0)) - val) < 0.5 * 10 ** -dec


def test_P11_overlap_secrest_johnson():
    val, dec = golden()["overlap_secrest_2d"]
    w = W.secrest_johnson_2d()
    g = O.Grid(w["N"], w["dq"])
    ctr = [0.0, 24.0]                      # ranges (-14, 14) and (0, 48)
    psi0 = O.gaussian(g, w["q0"], w["p0"], w["sigma"], q_ctr=ctr, p_ctr=[0, -3.56])
    phi0 = O.gaussian(g, w["q0"], [0.0, -3.0], w["sigma"], q_ctr=ctr, p_ctr=[0, -3.56])
    assert abs(abs(O.inner(psi0, phi0)) - val) < 0.5 * 10 ** -dec


# ---------------------------------------------------------------------------
# Energy (P12), regrid, naive grid (N1), autocorrelation
# ---------------------------------------------------------------------------
def test_P12_energy_error_order_two():
    errs = []
    for dt in (0.1, 0.05):
        g = O.Grid([64], [0.3])
        wp = O.gaussian(g, [0.5], [0.3], [1.0])
        pot = O.potentials.Harmonic([2.25])
        e0 = O.observables(wp, pot, [1.0])["E"]
        O.run(wp, dt, int(round(1.0 / dt)), O.composition("strang", 2), pot, [1.0])
        errs.append(abs(O.observables(wp, pot, [1.0])["E"] - e0))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_regrid_round_trip_and_interpolation():
    g = O.Grid([48, 56], [0.35, 0.3])
    wp = O.gaussian(g, [0.2, -0.4], [0.5, 1.0], [1.0, 0.8])
    moved = O.regrid(wp, [1.37, -2.11])
    ref = O.propagate.gaussian_values(g.q_mesh([1.37, -2.11]), [0.2, -0.4], [0.5, 1.0],
                                      [1.0, 0.8])
    assert np.max(np.abs(moved.physical() - ref)) < 1e-11
    back = O.regrid(moved, wp.q_ctr)
    assert O.state_distance(back, wp) < 1e-13


def test_N1_naive_grid_breaks_reversibility():
    """Fig. 5: the naive adaptive grid is not time-reversible, the proposed one is."""
    gam = O.composition("triple_jump", 4)
    pot = O.potentials.Harmonic([2.25, 1.0])
    g = O.Grid([32, 32], [0.45, 0.45])
    a = O.gaussian(g, [1.0, -0.5], [0.3, 0.8], [1.0, 1.0])
    b = a.copy()
    for _ in range(10):
        O.naive_step(a, 0.2, gam, pot, [1.0, 1.0])
    for _ in range(10):
        O.naive_step(a, -0.2, gam, pot, [1.0, 1.0])
    O.run(b, 0.2, 10, gam, pot, [1.0, 1.0])
    O.run(b, -0.2, 10, gam, pot, [1.0, 1.0])
    start = O.gaussian(g, [1.0, -0.5], [0.3, 0.8], [1.0, 1.0])
    assert O.state_distance(b, start) < 1e-12
    assert O.state_distance(a, start) > 1e-6


def test_autocorrelation_coherent_state():
    """For the 1-D coherent state |<psi0|psi_t>| = exp(-|alpha0 - alpha_t|^2/2) with
    alpha = (q + i p)/sqrt(2) (unit mass, frequency and hbar), up to the split error."""
    g = O.Grid([64], [0.25])
    wp = O.gaussian(g, [1.0], [0.0], [1.0])
    f0 = lambda qs: O.propagate.gaussian_values(qs, [1.0], [0.0], [1.0])
    assert abs(O.autocorrelation(wp, f0) - 1.0) < 1e-13
    O.run(wp, 0.01, 100, O.composition("suzuki", 4), O.potentials.Harmonic([1.0]), [1.0])
    a_t = (math.cos(1.0) - 1j * math.sin(1.0)) / math.sqrt(2)
    expect = math.exp(-abs(1 / math.sqrt(2) - a_t) ** 2 / 2)
    assert abs(abs(O.autocorrelation(wp, f0)) - expect) < 1e-9


# ---------------------------------------------------------------------------
# The pins catch plausible mistakes planted in the oracle (CPU only)
# ---------------------------------------------------------------------------
def _p1_error():
    """Wavefunction error against the closed-form map plus the centres' distance from
    the Stoermer-Verlet centres (a wrong grid shift still samples a correct function,
    so the centres are what expose it)."""
    w = W.harmonic_3d(seed=2, n=48, dq=0.3, dt=0.05)
    err, wp, gm = _grid_vs_map(w, 5, O.composition("strang", 2))
    return err + np.linalg.norm(wp.q_ctr - gm.q) + np.linalg.norm(wp.p_ctr - gm.p)


def test_planted_mistakes_fail_P1(monkeypatch):
    assert _p1_error() < 1e-11

    # 1. sign error in the kinetic grid shift (q_h = q_0 - h m^-1 <p>)
    def wrong_shift(wp, h, inv_mass, move_grid=True):
        g = wp.grid
        q0, p0 = wp.q_ctr, wp.p_ctr
        psit = g.f(wp.psi, q0, p0)
        ps = g.p_mesh(p0)
        w = np.abs(psit) ** 2
        pm = np.array([np.sum(w * pl) / w.sum() for pl in ps])
        q_new = q0 - h * np.asarray(inv_mass) * pm
        psit = psit * np.exp(-1j * h * sum(0.5 * m * pl ** 2 for m, pl in zip(inv_mass, ps)))
        wp.psi = g.f_tilde(psit, q_new, p0)
        wp.q_ctr = q_new
    monkeypatch.setattr(O.propagate, "T_substep", wrong_shift)
    assert _p1_error() > 1e-6
    monkeypatch.undo()

    # 2. dropped (-1)^j factor in t_KJ (the pi hbar j term)
    orig_parts = O.Grid._t_parts

    def parts_no_sign(self, q_ctr, p_ctr):
        c, a, b = orig_parts(self, q_ctr, p_ctr)
        a = [al * np.exp(-1j * np.pi * np.arange(al.size).reshape(al.shape)) for al in a]
        return c, a, b
    monkeypatch.setattr(O.Grid, "_t_parts", parts_no_sign)
    assert _p1_error() > 1e-6
    monkeypatch.undo()

    # 3. potential force with the wrong sign
    orig_V = O.propagate.V_substep

    def wrong_force(wp, h, pot, move_grid=True):
        p = wp.p_ctr.copy()
        orig_V(wp, h, pot, move_grid=move_grid)
        wp.p_ctr = 2 * p - wp.p_ctr
    monkeypatch.setattr(O.propagate, "V_substep", wrong_force)
    assert _p1_error() > 1e-6
    monkeypatch.undo()
    assert _p1_error() < 1e-11


# ---------------------------------------------------------------------------
# Finite-difference gradient of the objective (pin for the adjoint reference)
# ---------------------------------------------------------------------------
def test_fd_gradient_matches_closed_form_gaussian_map():
    """d J / d k for a 1-D harmonic packet: oracle finite differences of whole grid
    propagations vs finite differences of the closed-form Gaussian map sampled on the
    final grid."""
    R_d, wdt = 0.5, 0.3

    def J_grid(k):
        g = O.Grid([48], [0.3])
        wp = O.gaussian(g, [1.0], [0.2], [1.0])
        O.run(wp, 0.05, 40, O.composition("strang", 2), O.potentials.Harmonic([k]), [1.0])
        x = g.q_axes(wp.q_ctr)[0]
        W_ = 1.0 / (1.0 + np.exp(-(R_d - x) / wdt))
        return 0.3 * np.sum(W_ * np.abs(wp.physical()) ** 2)

    def J_map(k):
        gm = cf.split_operator(cf.initial([1.0], [0.2], [1.0]), 0.05, 40,
                               O.composition("strang", 2), [[k]], [0.0], [1.0])
        x = gm.q + (np.arange(48) - 24) * 0.3
        W_ = 1.0 / (1.0 + np.exp(-(R_d - x) / wdt))
        return 0.3 * np.sum(W_ * np.abs(cf.values(gm, [x])) ** 2)

    h = 1e-4
    d_grid = (J_grid(1.3 + h) - J_grid(1.3 - h)) / (2 * h)
    d_map = (J_map(1.3 + h) - J_map(1.3 - h)) / (2 * h)
    assert abs(d_grid) > 1e-2
    assert abs(d_grid - d_map) < 1e-8
