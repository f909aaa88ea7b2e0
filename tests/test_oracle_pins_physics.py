"""Pins of the oracle's potential gradients, Ehrenfest moments, naive and fixed grids
and the adjoint objective (arXiv:1909.06412), each against something other than the
oracle itself:

* every potential's gradient against central differences of its own V, and the
  Henon-Heiles V against the textbook saddle points of the two-mode model;
* the potential substep's momentum-grid move (Sec. II.G.1, Eq. (47)) against the
  momentum expectation value of the kicked state computed spectrally through the
  grid transform (Ehrenfest: exp(ihV) p exp(-ihV) = p - h dV/dq holds exactly for any
  h, so the spectral <p> moves by -h<dV/dq> to the grid's spectral accuracy);
* the kinetic substep's position-grid move (Eq. (52)) against <q> of the result;
* the naive adaptive grid (Sec. II.F, Eqs. (29)-(34)) and the fixed grid against the
  closed-form split-operator map of a Gaussian in a quadratic potential;
* the objective J (window, transmitted probability) and its finite-difference
  gradient against the same closed-form map integrated by quadrature.

A planted-mistake test at the end shows that each pin fails on a plausible error in
the part it pins.  CPU only.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.special

import oracle as O
import workloads as W
from oracle import closed_forms as cf
from oracle import gradient as OG

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---------------------------------------------------------------------------
# Gradients against central differences of V
# ---------------------------------------------------------------------------
def _potentials():
    rng = np.random.default_rng(11)
    K = rng.uniform(-0.3, 0.3, (3, 3))
    K = K + K.T + np.diag([2.0, 1.5, 3.0])
    return [
        ("henon_heiles_3d", O.potentials.HenonHeiles(3, 1.0, 0.111803), 3, 2.5),
        ("henon_heiles_8d_strong", O.potentials.HenonHeiles(8, 0.7, 0.6), 8, 2.0),
        ("morse_repulsion_2d", O.potentials.MorseRepulsion(0.17, 1.0, 1.4, 10.0, 2.0, 0.5),
         2, 1.5),
        ("secrest_johnson_2d", O.potentials.MorseRepulsion(20.0, 0.158, 0.0, 1.0, 0.3, 1.0),
         2, 3.0),
        ("morse_1d", O.potentials.MorseRepulsion(2.0, 1.3, 0.4, 5.0, 1.0, 0.5), 1, 1.0),
        ("quadratic_full_K", O.potentials.Quadratic(K, [0.3, -0.2, 0.5]), 3, 2.0),
        ("harmonic", O.potentials.Harmonic([1.0, 1.44, 2.25], [0.1, 0.2, -0.3]), 3, 2.0),
    ]


def _fd_error(pot, D, spread, seed=3, npts=40):
    """max over random points of |grad - central difference of V| / (1 + |grad|)."""
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-spread, spread, (npts, D)) + (1.4 if pot.kind == "morse_repulsion" else 0)
    worst = 0.0
    for x in pts:
        qs = [np.array(v) for v in x]
        g = np.array([float(gl) for gl in pot.grad(qs)])
        fd = np.empty(D)
        for l in range(D):
            hstep = 1e-5 * max(1.0, abs(x[l]))
            xp, xm = x.copy(), x.copy()
            xp[l] += hstep
            xm[l] -= hstep
            fd[l] = (float(pot.V([np.array(v) for v in xp]))
                     - float(pot.V([np.array(v) for v in xm]))) / (2 * hstep)
        worst = max(worst, float(np.max(np.abs(g - fd)) / (1.0 + np.max(np.abs(g)))))
    return worst


@pytest.mark.parametrize("name,pot,D,spread", _potentials(), ids=[p[0] for p in _potentials()])
def test_gradient_is_derivative_of_V(name, pot, D, spread):
    """The Ehrenfest force of Eq. (47) needs dV/dq: each potential's grad equals the
    central difference of its V (step 1e-5, truncation ~1e-10)."""
    assert _fd_error(pot, D, spread) < 1e-8


@pytest.mark.parametrize("lam", [0.111803, 0.5, 1.0])
def test_henon_heiles_two_mode_saddles(lam):
    """The two-mode Henon-Heiles surface (Sec. III.C with D = 2, kappa = 1) has its three
    saddle points at (0, 1/lam) and (+-sqrt(3)/(2 lam), -1/(2 lam)), all at the escape
    energy 1/(6 lam^2), and its minimum at the origin (Henon & Heiles 1964, lam = 1)."""
    pot = O.potentials.HenonHeiles(2, 1.0, lam)
    for x, y in [(0.0, 1 / lam), (math.sqrt(3) / (2 * lam), -1 / (2 * lam)),
                 (-math.sqrt(3) / (2 * lam), -1 / (2 * lam))]:
        qs = [np.array(x), np.array(y)]
        assert abs(float(pot.V(qs)) - 1 / (6 * lam ** 2)) < 1e-12 / lam ** 2
        assert max(abs(float(g)) for g in pot.grad(qs)) < 1e-12 / lam
    assert float(pot.V([np.array(0.0), np.array(0.0)])) == 0.0


def test_morse_repulsion_limits():
    """Eq. (61) form: the Morse part has its minimum 0 at r = re and tends to De as the
    diatom dissociates; the repulsion decays with the atom-diatom distance rho - c r and
    is A at rho = c r."""
    pot = O.potentials.MorseRepulsion(0.17, 1.0, 1.4, 10.0, 2.0, 0.5)
    far = np.array(1e3)
    assert abs(float(pot.V([np.array(1.4), far]))) < 1e-15
    assert abs(float(pot.V([np.array(60.0), np.array(1e4)])) - 0.17) < 1e-12
    assert abs(float(pot.V([np.array(1.4), np.array(0.7)])) - 10.0) < 1e-12


# ---------------------------------------------------------------------------
# Ehrenfest pins of the substeps' grid moves
# ---------------------------------------------------------------------------
def _p_mean_spectral(wp):
    """<p> of the state from |f(q_ctr, p_ctr) psi|^2 on the momentum grid (Eq. (49))."""
    g = wp.grid
    pt = g.f(wp.psi, wp.q_ctr, wp.p_ctr)
    wt = np.abs(pt) ** 2
    return np.array([np.sum(wt * pl) / wt.sum() for pl in g.p_mesh(wp.p_ctr)])


def _q_mean(wp):
    g = wp.grid
    w = np.abs(wp.psi) ** 2
    return np.array([np.sum(w * ql) / w.sum() for ql in g.q_mesh(wp.q_ctr)])


def _ehrenfest_cases():
    hh = W.henon_heiles_8d(n=24, D=3, dq=0.45, lam=0.111803)
    hh["q0"] = [2.0, -1.0, 0.5]           # unequal |q_l|: the lam (q_l^2 - q_l+1^2) terms count
    mr = W.morse_repulsion_2d(96, 192, steps=0, precision="c128")
    mr["q0"] = [1.4, 3.2]                 # on the repulsive wall: a strong force along rho
    return [
        ("henon_heiles_3d", hh, 0.2),
        ("morse_repulsion_wall", mr, 2.0),
    ]


@pytest.mark.parametrize("name,w,h", _ehrenfest_cases(), ids=[c[0] for c in _ehrenfest_cases()])
def test_ehrenfest_potential_substep_moves_p_grid(name, w, h):
    """After U_V(h) the spectral <p> has moved by -h <dV/dq> (exact for the operator,
    spectral on the grid), and so has p_ctr (Eq. (47)).  The phase uses V, the grid move
    uses grad V: this ties the two."""
    g = O.Grid(w["N"], w["dq"])
    wp = O.gaussian(g, w["q0"], w["p0"], w["sigma"])
    pot = O.potentials.from_spec(*w["potential"], w["D"])
    p_before = _p_mean_spectral(wp)
    pc_before = wp.p_ctr.copy()
    O.V_substep(wp, h, pot)
    dp_spec = _p_mean_spectral(wp) - p_before
    dp_grid = wp.p_ctr - pc_before
    assert np.max(np.abs(dp_spec)) > 1e-2                      # a real kick
    np.testing.assert_allclose(dp_grid, dp_spec, rtol=0, atol=1e-9 * (1 + np.max(np.abs(dp_spec))))


@pytest.mark.parametrize("minv", [[1.0, 0.5, 2.0], [[1.0, 0.2, 0.0], [0.2, 0.7, -0.1],
                                                   [0.0, -0.1, 1.5]]])
def test_ehrenfest_kinetic_substep_moves_q_grid(minv):
    """After U_T(h) the state's <q> has moved by h m^-1 <p> (free flight), and so has
    q_ctr (Eq. (52)); the state then sits centred on its own <q> again."""
    w = W.henon_heiles_8d(n=32, D=3, dq=0.4, lam=0.111803)
    g = O.Grid(w["N"], w["dq"])
    wp = O.gaussian(g, [0.3, -0.2, 0.6], [1.1, -0.7, 0.4], [1.0, 0.8, 1.2])
    pot = O.potentials.from_spec(*w["potential"], 3)
    O.V_substep(wp, 0.3, pot)                                   # a non-Gaussian state
    q_before = _q_mean(wp)
    qc_before = wp.q_ctr.copy()
    p = _p_mean_spectral(wp)
    h = 0.35
    O.T_substep(wp, h, minv)
    m = np.diag(minv) if np.ndim(minv) == 1 else np.asarray(minv)
    expect = h * m @ p
    np.testing.assert_allclose(_q_mean(wp) - q_before, expect, rtol=0, atol=1e-10)
    np.testing.assert_allclose(wp.q_ctr - qc_before, expect, rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# Naive adaptive grid and fixed grid against the closed-form Gaussian map
# ---------------------------------------------------------------------------
QUAD = dict(k=[1.44, 0.81], s=[0.4, -0.3])


def _quad_setup(N=(64, 72), dq=(0.32, 0.3)):
    g = O.Grid(list(N), list(dq))
    q0, p0, sig = [1.0, -0.8], [0.6, 1.1], [1.0, 0.85]
    wp = O.gaussian(g, q0, p0, sig)
    pot = O.potentials.Harmonic(QUAD["k"], QUAD["s"])
    return g, wp, pot, cf.initial(q0, p0, sig)


def test_naive_grid_matches_closed_form_map():
    """Eqs. (29)-(34): each naive step propagates on the frozen grid (for quadratic V the
    exact split-operator product, so the closed-form Gaussian map) and re-centres the
    grid on the new <q>, <p>, which for a Gaussian are its centre parameters.  The state
    on the moved grid is the closed-form Gaussian sampled there."""
    g, wp, pot, g0 = _quad_setup()
    gam = O.composition("suzuki", 4)
    dt, n = 0.15, 6
    for _ in range(n):
        O.naive_step(wp, dt, gam, pot, [1.0, 1.0])
    gm = cf.split_operator(g0, dt, n, gam, np.diag(QUAD["k"]), QUAD["s"], [1.0, 1.0])
    np.testing.assert_allclose(wp.q_ctr, gm.q, rtol=0, atol=1e-11)
    np.testing.assert_allclose(wp.p_ctr, gm.p, rtol=0, atol=1e-11)
    assert np.max(np.abs(wp.q_ctr - np.array([1.0, -0.8]))) > 0.3       # the grid moved
    ref = cf.values(gm, g.q_mesh(wp.q_ctr))
    assert np.max(np.abs(wp.physical() - ref)) < 1e-10


def test_fixed_grid_matches_closed_form_map():
    """Grid centres frozen (the paper's fixed-grid comparison, Sec. III.A): the centres
    never move and the state is the closed-form split-operator map on the initial grid."""
    g, wp, pot, g0 = _quad_setup(N=(96, 96), dq=(0.3, 0.3))
    qc, pc = wp.q_ctr.copy(), wp.p_ctr.copy()
    gam = O.composition("triple_jump", 4)
    O.run(wp, 0.1, 12, gam, pot, [1.0, 1.0], move_grid=False)
    np.testing.assert_array_equal(wp.q_ctr, qc)
    np.testing.assert_array_equal(wp.p_ctr, pc)
    gm = cf.split_operator(g0, 0.1, 12, gam, np.diag(QUAD["k"]), QUAD["s"], [1.0, 1.0])
    assert np.max(np.abs(gm.q - qc)) > 0.3
    ref = cf.values(gm, g.q_mesh(qc))
    assert np.max(np.abs(wp.physical() - ref)) < 1e-10


# ---------------------------------------------------------------------------
# Objective and its finite-difference gradient against the closed-form map
# ---------------------------------------------------------------------------
def _J_closed(gm, R_d, wdt, c, D, hbar=1.0):
    """J = int expit((R_d - R)/w) rho_R(R) dR with rho_R the Gaussian density of
    R = rho - c r (D = 2) or R = q (D = 1) for the closed-form Gaussian; |psi|^2 has
    covariance (hbar/2) Im(P Q^-1)^-1.  Integrated by adaptive quadrature."""
    A = gm.P @ np.linalg.inv(gm.Q)
    cov = 0.5 * hbar * np.linalg.inv(np.imag(A))
    v = np.array([1.0]) if D == 1 else np.array([-c, 1.0])
    mu = float(v @ gm.q)
    sd = math.sqrt(float(v @ cov @ v))
    dens = lambda R: math.exp(-0.5 * ((R - mu) / sd) ** 2) / (sd * math.sqrt(2 * math.pi))
    f = lambda R: scipy.special.expit((R_d - R) / wdt) * dens(R)
    val, _ = scipy.integrate.quad(f, mu - 12 * sd, mu + 12 * sd, points=[R_d],
                                  epsabs=1e-14, epsrel=1e-13, limit=200)
    return val


def _objective_workload(D):
    if D == 1:
        return dict(name="obj_1d", D=1, N=[128], dq=[0.15], inv_mass=[1.0], hbar=1.0,
                    potential=("harmonic", {"k": [1.3], "s": [0.0]}),
                    q0=[1.0], p0=[0.2], sigma=[1.0], dt=0.05, steps=40, split="TVT",
                    comp="strang", order=2), (0.5, 0.45)
    return dict(name="obj_2d", D=2, N=[96, 96], dq=[0.2, 0.2], inv_mass=[1.0, 0.6], hbar=1.0,
                potential=("harmonic", {"k": [1.3, 0.8], "s": [0.2, -0.1]}),
                q0=[0.6, 0.4], p0=[0.3, -0.5], sigma=[0.9, 1.1], dt=0.05, steps=30,
                split="VTV", comp="suzuki", order=4), (0.1, 0.6)


def _closed_form_J(w, k, nsteps, R_d, wdt, c=0.5):
    g0 = cf.initial(w["q0"], w["p0"], w["sigma"])
    gm = cf.split_operator(g0, w["dt"], nsteps, O.composition(w["comp"], w["order"]),
                           np.diag(k), w["potential"][1]["s"], w["inv_mass"], w["split"])
    return _J_closed(gm, R_d, wdt, c, w["D"])


@pytest.mark.parametrize("D", [1, 2])
def test_objective_and_fd_gradient_match_closed_form(D):
    """oracle.gradient.run_objective / transmitted / window / fd_gradient against the
    closed-form map: J to the grid's spectral accuracy, dJ/dk_l by central differences of
    the quadrature value.  The window is at least three grid spacings wide, so the grid
    sum of W |psi|^2 is a spectrally accurate quadrature (error ~ exp(-pi^2 w/dq))."""
    w, (R_d, wdt) = _objective_workload(D)
    n = w["steps"]
    k = list(w["potential"][1]["k"])
    J = OG.run_objective(w, w["potential"][1], n, R_d, wdt)
    Jc = _closed_form_J(w, k, n, R_d, wdt)
    assert 0.05 < J < 0.95
    assert abs(J - Jc) < 1e-11
    names = [("k", l) for l in range(D)]
    fd = OG.fd_gradient(w, names, n, R_d, wdt)
    ref = []
    for l in range(D):
        hstep = 1e-4 * max(abs(k[l]), 1.0)
        kp, km = list(k), list(k)
        kp[l] += hstep
        km[l] -= hstep
        ref.append((_closed_form_J(w, kp, n, R_d, wdt) - _closed_form_J(w, km, n, R_d, wdt))
                   / (2 * hstep))
    ref = np.array(ref)
    assert np.max(np.abs(ref)) > 1e-2
    np.testing.assert_allclose(fd, ref, rtol=0, atol=1e-7)


# ---------------------------------------------------------------------------
# Each pin above fails on a plausible mistake planted in the oracle
# ---------------------------------------------------------------------------
def _hh_gradient_lambda_sign(self, qs):
    shape = np.broadcast_shapes(*[q.shape for q in qs])
    g = [self.kappa * q + np.zeros(shape) for q in qs]
    for l in range(self.D - 1):
        g[l] = g[l] + 2 * self.lam * qs[l] * qs[l + 1]
        g[l + 1] = g[l + 1] - self.lam * (qs[l] ** 2 - qs[l + 1] ** 2)     # planted sign
    return g


def _morse_gradient_repulsion_sign(self, qs):
    r = qs[0]
    shape = np.broadcast_shapes(*[q.shape for q in qs])
    e = np.exp(-self.a * (r - self.re))
    dr = 2 * self.De * self.a * e * (1 - e)
    rep = self.A * np.exp(-self.b * (qs[1] - self.c * r))
    return [dr - self.b * self.c * rep + np.zeros(shape), -self.b * rep + np.zeros(shape)]


def _naive_unmoved_p_grid(wp, dt, gammas, pot, inv_mass, split="TVT"):
    g = wp.grid
    q0, p0 = wp.q_ctr.copy(), wp.p_ctr.copy()
    O.propagate.step(wp, dt, gammas, pot, inv_mass, split, move_grid=False)
    w = np.abs(wp.psi) ** 2
    q_new = np.array([np.sum(w * ql) / w.sum() for ql in g.q_mesh(q0)])
    psit = g.f(wp.psi, q0, p0)
    wt = np.abs(psit) ** 2
    p_new = np.array([np.sum(wt * pl) / wt.sum() for pl in g.p_mesh(p0)])
    wp.psi = g.f_tilde(psit, q_new, p_new)          # planted: p-grid not moved before f~
    wp.q_ctr, wp.p_ctr = q_new, p_new


def _window_wrong_R(qs, R_d, w, c=0.5):
    if len(qs) == 1:
        R = qs[0]
    else:
        r, rho = qs
        R = rho + c * r                              # planted sign
    return 1.0 / (1.0 + np.exp(-(R_d - R) / w))


def test_planted_mistakes_fail_the_pins(monkeypatch):
    pots = {p[0]: p for p in _potentials()}

    # 1. Henon-Heiles gradient: sign of the lam (q_l^2 - q_{l+1}^2) term
    _, pot, D, spread = pots["henon_heiles_3d"]
    monkeypatch.setattr(O.potentials.HenonHeiles, "grad", _hh_gradient_lambda_sign)
    assert _fd_error(pot, D, spread) > 1e-3
    with pytest.raises(AssertionError):
        test_ehrenfest_potential_substep_moves_p_grid(*_ehrenfest_cases()[0])
    monkeypatch.undo()

    # 2. Morse + repulsion gradient: sign of the repulsion's r term
    _, pot, D, spread = pots["morse_repulsion_2d"]
    monkeypatch.setattr(O.potentials.MorseRepulsion, "grad", _morse_gradient_repulsion_sign)
    assert _fd_error(pot, D, spread) > 1e-3
    with pytest.raises(AssertionError):
        test_ehrenfest_potential_substep_moves_p_grid(*_ehrenfest_cases()[1])
    monkeypatch.undo()

    # 3. naive grid: resampled without first moving the momentum grid
    monkeypatch.setattr(O.propagate, "naive_step", _naive_unmoved_p_grid)
    monkeypatch.setattr(O, "naive_step", _naive_unmoved_p_grid)
    with pytest.raises(AssertionError):
        test_naive_grid_matches_closed_form_map()
    monkeypatch.undo()

    # 4. fixed grid: the potential substep still moves p_ctr
    orig_V = O.propagate.V_substep

    def V_ignores_flag(wp, h, pot, move_grid=True):
        orig_V(wp, h, pot, move_grid=True)
    monkeypatch.setattr(O.propagate, "V_substep", V_ignores_flag)
    with pytest.raises(AssertionError):
        test_fixed_grid_matches_closed_form_map()
    monkeypatch.undo()

    # 5. objective: R = rho + c r in the window
    monkeypatch.setattr(OG, "window", _window_wrong_R)
    with pytest.raises(AssertionError):
        test_objective_and_fd_gradient_match_closed_form(2)
    monkeypatch.undo()

    # 6. objective: the dq volume element dropped
    def transmitted_no_volume(wp, R_d, w, c=0.5):
        g = wp.grid
        Wn = OG.window(g.q_mesh(wp.q_ctr), R_d, w, c)
        return float(np.sum(Wn * np.abs(wp.physical()) ** 2))
    monkeypatch.setattr(OG, "transmitted", transmitted_no_volume)
    with pytest.raises(AssertionError):
        test_objective_and_fd_gradient_match_closed_form(1)
    monkeypatch.undo()

    # 7. kinetic substep: q_ctr moved by h <p> without m^-1
    orig_T = O.propagate.T_substep

    def T_no_mass(wp, h, inv_mass, move_grid=True):
        D = wp.grid.D
        orig_T(wp, h, [1.0] * D, move_grid=move_grid)
    monkeypatch.setattr(O.propagate, "T_substep", T_no_mass)
    monkeypatch.setattr(O, "T_substep", T_no_mass)
    with pytest.raises(AssertionError):
        test_ehrenfest_kinetic_substep_moves_q_grid([1.0, 0.5, 2.0])
    monkeypatch.undo()

    # with everything restored the pins pass again
    assert _fd_error(pots["henon_heiles_3d"][1], 3, 2.5) < 1e-8
    test_naive_grid_matches_closed_form_map()
    test_objective_and_fd_gradient_match_closed_form(2)
