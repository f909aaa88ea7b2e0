"""Full-size checks on the 8-D Henon-Heiles workload of Sec. III.C: 16^8 = 2^32 grid
points, propagated through the C ABI exactly as the benchmark does (the radix-16
sweep kernels, the same tiles and launches, complex64 and complex128).  The oracle
cannot hold 2^32 points, so two cases whose exact answer is a product of
one-dimensional states, evaluated at sampled grid points one by one:

* separable (lambda = 0): the Hamiltonian and the initial Gaussian are products over
  the axes.  The split-operator factors and the Fourier transforms then factorise,
  and the Ehrenfest moment of axis l (Sec. II.G) depends on axis l's marginal only,
  so the 8-D state is the product of eight 1-D oracle runs of 16 points and the grid
  centres are theirs, axis by axis;
* coupled (the benchmark's lambda): the moving-grid scheme is time reversible
  (Sec. II.G), so n steps forward and n steps back return the initial Gaussian (a
  product of 1-D factors) and the initial grid.

Samples: half uniform over the grid, half drawn per axis from the 1-D densities
|psi_l|^2 (where the state lives); the error is the relative l2 error over them.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
TOL64 = 1e-5
NSAMP = 1 << 16


def _mg():
    import paper_1909_06412_amd as mg
    return mg


def _axis_oracle(w, l, nsteps, dt):
    """1-D oracle run of axis l of a separable workload (V = kappa q^2 / 2)."""
    g = O.Grid([w["N"][l]], [w["dq"][l]], w["hbar"])
    wp = O.gaussian(g, [w["q0"][l]], [w["p0"][l]], [w["sigma"][l]])
    kappa = w["potential"][1]["kappa"]
    pot = O.potentials.from_spec("henon_heiles", {"kappa": kappa, "lam": 0.0}, 1)
    if nsteps:
        O.run(wp, dt, nsteps, O.composition(w["comp"], w["order"]), pot, [w["inv_mass"][l]], w["split"])
    return wp


def _samples(w, dens, seed):
    """NSAMP flat indices (row-major, axis 0 outermost) and their per-axis digits."""
    rng = np.random.default_rng(seed)
    D, n = w["D"], w["N"][0]
    h = NSAMP // 2
    dig = np.empty((NSAMP, D), dtype=np.int64)
    dig[:h] = rng.integers(0, n, size=(h, D))
    for l in range(D):
        p = dens[l] / dens[l].sum()
        dig[h:, l] = rng.choice(n, size=NSAMP - h, p=p)
    flat = np.zeros(NSAMP, dtype=np.int64)
    for l in range(D):
        flat = flat * n + dig[:, l]
    return flat, dig


def _gpu_samples(m, flat):
    import torch
    v = m.state_view()
    idx = torch.from_numpy(flat).to(v.device)
    s = v.index_select(0, idx).to(torch.complex128).cpu().numpy()
    return s / np.sqrt(np.prod(np.asarray(m.dq)))


def _product(factors, dig):
    out = np.ones(dig.shape[0], dtype=np.complex128)
    for l, f in enumerate(factors):
        out = out * f[dig[:, l]]
    return out


def _release(m):
    import torch
    m.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _run_full(w, precision):
    mg = _mg()
    return mg.from_workload(w, precision=precision)


@pytest.mark.parametrize("precision,split,comp,order", [
    ("c64", "TVT", "suzuki", 4), ("c128", "TVT", "suzuki", 4),
    ("c64", "VTV", "strang", 2), ("c64", "TVT", "triple_jump", 4)])
def test_separable_16e8_matches_product_of_axis_oracles(precision, split, comp, order):
    w = W.henon_heiles_8d(lam=0.0)
    w["split"], w["comp"], w["order"] = split, comp, order
    # distinct axes, so that a transposed axis or a wrong digit order shows
    w["q0"] = [2.0 - 0.15 * l for l in range(8)]
    w["p0"] = [0.2 * l - 0.7 for l in range(8)]
    w["sigma"] = [0.8 + 0.05 * l for l in range(8)]
    nsteps = 3
    axes = [_axis_oracle(w, l, nsteps, w["dt"]) for l in range(8)]
    fac = [a.physical() for a in axes]
    flat, dig = _samples(w, [np.abs(f) ** 2 for f in fac], seed=11)
    ref = _product(fac, dig)
    print(f"[full] separable 16^8 {precision} {split} {comp}{order}: {nsteps} steps", flush=True)
    m = _run_full(w, precision)
    try:
        m.step(w["dt"], nsteps)
        got = _gpu_samples(m, flat)
        q, p, _ = m.centres()
    finally:
        _release(m)
    e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    dq = max(abs(q[l] - axes[l].q_ctr[0]) for l in range(8))
    dp = max(abs(p[l] - axes[l].p_ctr[0]) for l in range(8))
    print(f"[full] separable 16^8 {precision} {split} {comp}{order}: sampled state {e:.3e} dq {dq:.3e} "
          f"dp {dp:.3e}", flush=True)
    tc = 1e-12 if precision == "c128" else 1e-6
    assert dq < tc and dp < tc
    assert e < (TOL128 if precision == "c128" else TOL64)


def test_coupled_16e8_round_trip_returns_initial_gaussian():
    w = W.henon_heiles_8d()
    nsteps = 2
    g1 = O.Grid([16], [w["dq"][0]], w["hbar"])
    fac = [O.gaussian(g1, [w["q0"][l]], [w["p0"][l]], [w["sigma"][l]]).physical() for l in range(8)]
    flat, dig = _samples(w, [np.abs(f) ** 2 for f in fac], seed=12)
    ref = _product(fac, dig)
    print(f"[full] coupled 16^8 c64: {nsteps} steps forward and back", flush=True)
    m = _run_full(w, "c64")
    try:
        m.step(w["dt"], nsteps)
        mid = _gpu_samples(m, flat)
        m.step(-w["dt"], nsteps)
        got = _gpu_samples(m, flat)
        q, p, _ = m.centres()
    finally:
        _release(m)
    e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    moved = float(np.linalg.norm(mid - ref) / np.linalg.norm(ref))
    dq = float(np.max(np.abs(np.asarray(q) - np.asarray(w["q0"]))))
    dp = float(np.max(np.abs(np.asarray(p) - np.asarray(w["p0"]))))
    print(f"[full] coupled 16^8 c64: after forward {moved:.3e}, after return {e:.3e} dq {dq:.3e} dp {dp:.3e}",
          flush=True)
    assert moved > 1e-3          # the forward steps did change the state
    assert dq < 1e-6 and dp < 1e-6
    assert e < TOL64


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_three_pass_plan_matches_four_sweep_plan(precision):
    """Engine 0 runs 16^8 kinetic substeps in three passes per direction (one axis
    split into two 4-point digits); engine 2 in the four radix-16 sweeps.  Same
    arithmetic up to rounding: the sampled states and the centres agree."""
    mg = _mg()
    w = W.henon_heiles_8d()
    w["q0"] = [2.0 - 0.15 * l for l in range(8)]
    w["p0"] = [0.2 * l - 0.7 for l in range(8)]
    nsteps = 2
    g1 = O.Grid([16], [w["dq"][0]], w["hbar"])
    fac = [O.gaussian(g1, [w["q0"][l]], [w["p0"][l]], [w["sigma"][l]]).physical() for l in range(8)]
    flat, _ = _samples(w, [np.abs(f) ** 2 for f in fac], seed=13)
    out = []
    for engine in (0, 2):
        print(f"[full] coupled 16^8 {precision} engine {engine}: {nsteps} steps", flush=True)
        m = _run_full(w, precision)
        try:
            m.set_option(mg.MG_OPT_ENGINE, engine)
            m.step(w["dt"], nsteps)
            out.append((_gpu_samples(m, flat), *m.centres()[:2]))
        finally:
            _release(m)
    (s0, q0, p0), (s2, q2, p2) = out
    e = float(np.linalg.norm(s0 - s2) / np.linalg.norm(s2))
    dq = float(np.max(np.abs(q0 - q2)))
    dp = float(np.max(np.abs(p0 - p2)))
    print(f"[full] three-pass vs four-sweep {precision}: sampled state {e:.3e} dq {dq:.3e} dp {dp:.3e}",
          flush=True)
    tol = (1e-7, 1e-6) if precision == "c64" else (1e-13, 1e-12)
    assert dq < tol[0] and dp < tol[0]
    assert e < tol[1]


def test_three_pass_plan_graph_replays_match_eager():
    """MG_OPT_GRAPH on the 16^8 complex64 grid (the three-pass plan's launches
    captured once and replayed): every replay equals an eager context fed the same
    calls bit for bit, with eager work (observables) between the replays."""
    import torch
    mg = _mg()
    w = W.henon_heiles_8d()
    g1 = O.Grid([16], [w["dq"][0]], w["hbar"])
    fac = [O.gaussian(g1, [w["q0"][l]], [w["p0"][l]], [w["sigma"][l]]).physical() for l in range(8)]
    flat, _ = _samples(w, [np.abs(f) ** 2 for f in fac], seed=14)
    print("[full] graph 16^8 c64: eager and captured contexts", flush=True)
    a = _run_full(w, "c64")
    b = _run_full(w, "c64")
    try:
        b.set_option(mg.MG_OPT_GRAPH, 1)
        for rep in range(3):
            a.step(w["dt"], 1)
            b.step(w["dt"], 1)          # rep 0 captures, reps 1-2 replay
            sa, sb = _gpu_samples(a, flat), _gpu_samples(b, flat)
            qa, pa, ta = a.centres()
            qb, pb, tb = b.centres()
            d = float(np.max(np.abs(sa - sb)))
            print(f"[full] graph 16^8 c64 replay {rep}: max |eager - replay| = {d:.3e}", flush=True)
            assert d == 0.0
            assert np.array_equal(qa, qb) and np.array_equal(pa, pb) and ta == tb
            if rep == 1:
                oa, ob = a.observables(), b.observables()   # eager work between replays
                assert oa["norm"] == ob["norm"]
            torch.cuda.synchronize()
    finally:
        _release(a)
        _release(b)
