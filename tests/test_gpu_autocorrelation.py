"""<psi_0|psi_t> on the GPU (psi_0 re-evaluated analytically on the moved grid,
Sec. III.C) against the oracle, and the spectrum of the Henon-Heiles series."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _mg():
    import paper_1909_06412_amd as mg
    return mg


def test_coherent_state_autocorrelation_closed_form():
    """1-D coherent state: |<psi0|psi_t>| = exp(-|alpha0 - alpha_t|^2 / 2), alpha = (q + i p)/sqrt(2)."""
    mg = _mg()
    w = W.harmonic_1d()
    m = mg.from_workload(w)
    a0 = m.autocorrelation(w["q0"], w["p0"], w["sigma"])
    assert abs(a0 - 1.0) < 1e-13
    m.set_scheme("TVT", "suzuki", 4)
    m.step(0.01, 100)
    a = m.autocorrelation(w["q0"], w["p0"], w["sigma"])
    m.close()
    a_t = (math.cos(1.0) - 1j * math.sin(1.0)) / math.sqrt(2)
    expect = math.exp(-abs(1 / math.sqrt(2) - a_t) ** 2 / 2)
    assert abs(abs(a) - expect) < 1e-9


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_henon_heiles_autocorrelation_series_and_spectrum(precision):
    mg = _mg()
    w = W.henon_heiles_8d(n=16, D=3, dq=0.625)
    w["dt"] = 0.05
    g = O.Grid(w["N"], w["dq"], w["hbar"])
    wp = O.gaussian(g, w["q0"], w["p0"], w["sigma"])
    pot = O.potentials.from_spec(*w["potential"], w["D"])
    gam = O.composition(w["comp"], w["order"])
    f0 = lambda qs: O.propagate.gaussian_values(qs, w["q0"], w["p0"], w["sigma"])
    m = mg.from_workload(w, precision=precision)
    times, got, ref = [0.0], [m.autocorrelation(w["q0"], w["p0"], w["sigma"])], [O.autocorrelation(wp, f0)]
    for k in range(1, 41):
        m.step(w["dt"], 1)
        O.run(wp, w["dt"], 1, gam, pot, w["inv_mass"], w["split"])
        times.append(k * w["dt"])
        got.append(m.autocorrelation(w["q0"], w["p0"], w["sigma"]))
        ref.append(O.autocorrelation(wp, f0))
    m.close()
    got, ref = np.array(got), np.array(ref)
    err = np.max(np.abs(got - ref))
    tol = 1e-12 if precision == "c128" else 2e-6
    print(f"[acf] HH 16^3 {precision}: max |acf_gpu - acf_oracle| = {err:.3e}, |acf(2)| = {abs(got[-1]):.4f}",
          flush=True)
    assert err < tol
    assert abs(got[-1]) < 0.99                 # the packet has moved off psi_0
    E = np.linspace(0.0, 6.0, 61)
    sg = mg.spectrum(times, got, E, t_damp=30.0)
    sr = O.spectrum(times, ref, E, t_damp=30.0)
    assert np.max(np.abs(sg - sr)) < (1e-11 if precision == "c128" else 1e-5)
