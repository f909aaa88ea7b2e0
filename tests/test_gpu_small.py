"""The one-wave path (one-dimensional grids of at most 64 points: a whole mg_step call
in one launch of one wave, the state in FP64 registers between substeps) against the
FP64 oracle on the same seeded inputs, and against the library's general path (a
context with MG_OPT_PROFILE set keeps the general sweeps and finalize launches)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

SCHEMES = [("TVT", "strang", 2), ("VTV", "suzuki", 4), ("TVT", "triple_jump", 6)]
POTENTIALS = {
    "harmonic": ("harmonic", {"k": [1.44], "s": [0.3]}),
    "morse": ("morse_repulsion", {"De": 8.0, "a": 0.5, "re": 0.0, "A": 0.0, "b": 0.0, "c": 0.0}),
}


def _mg():
    import paper_1909_06412_amd as mg
    return mg


def _case(n, scheme, pot):
    split, comp, order = scheme
    w = W.scaled(W.harmonic_1d(), name=f"1d_{n}", N=[n], dq=[10.0 / n], potential=POTENTIALS[pot],
                 q0=[0.4], p0=[0.7], sigma=[1.0], dt=0.05, split=split, comp=comp, order=order)
    return w


def _oracle(w, nsteps):
    g = O.Grid(w["N"], w["dq"], w["hbar"])
    wp = O.gaussian(g, w["q0"], w["p0"], w["sigma"])
    pot = O.potentials.from_spec(*w["potential"], 1)
    O.run(wp, w["dt"], nsteps, O.composition(w["comp"], w["order"]), pot, w["inv_mass"], w["split"])
    return wp


@pytest.mark.parametrize("n", [8, 16, 30, 50, 64])
@pytest.mark.parametrize("scheme", SCHEMES, ids=["tvt-strang", "vtv-suzuki4", "tvt-tj6"])
@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_one_wave_path_matches_oracle_and_general_path(n, scheme, precision):
    mg = _mg()
    pot = "morse" if n in (16, 50) else "harmonic"
    w = _case(n, scheme, pot)
    nsteps = 20
    ref = _oracle(w, nsteps)
    m = mg.from_workload(w, precision=precision)
    m.step(w["dt"], nsteps)
    psi, q, p, t = m.get_state()
    m.close()
    g = mg.from_workload(w, precision=precision)
    g.set_option(mg.MG_OPT_PROFILE, 1)   # the general path
    g.step(w["dt"], nsteps)
    psi_g, q_g, p_g, _ = g.get_state()
    g.close()
    phys = ref.physical()
    e = float(np.linalg.norm(psi - phys) / np.linalg.norm(phys))
    em = float(np.max(np.abs(psi - phys)) / np.max(np.abs(phys)))
    eg = float(np.linalg.norm(psi - psi_g) / np.linalg.norm(psi_g))
    print(f"[small] n={n} {scheme} {pot} {precision}: vs oracle {e:.3e} (max {em:.3e}), "
          f"vs general path {eg:.3e}, dq {np.max(np.abs(q - ref.q_ctr)):.1e} dp {np.max(np.abs(p - ref.p_ctr)):.1e}",
          flush=True)
    # complex64: the state is rounded once on the way in and once on the way out
    tol = 1e-12 if precision == "c128" else 1e-6
    assert e < tol and em < tol
    assert np.max(np.abs(q - ref.q_ctr)) < tol and np.max(np.abs(p - ref.p_ctr)) < tol
    assert abs(t - nsteps * w["dt"]) < 1e-12
    # the general path rounds the complex64 state at every sweep; complex128 agrees closely
    assert eg < (1e-12 if precision == "c128" else 1e-5)
    if precision == "c128":
        assert np.max(np.abs(q - q_g)) < 1e-13 and np.max(np.abs(p - p_g)) < 1e-13
