"""GPU parity of each workload at its own size (through the C ABI) against the FP64
oracle, element by element (max |psi_gpu - psi_oracle| / max |psi_oracle|) and in
relative l2, with the grid centres:

* 3-D harmonic model (32^3, t_f = 5): orders 2-10 over the whole horizon, also
  against the exact harmonic solution (Sec. III.A, convergence study);
* atom-diatom model on the 256^2 grid: a few hundred steps in both precisions;
* 256 atom-diatom packets of uneven shapes in one batch (every packet propagated;
  a seeded sample of 16 compared one by one), two launch shapes;
* coupled 8-D Henon-Heiles (Sec. III.C) on the 16-point kernels: 16^6 against the
  full oracle, and the 16^8 headline grid through its potential substep;
* user-supplied composition coefficients and the renormalisation option.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import closed_forms as cf

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
TOL64 = 1e-5


def _mg():
    import paper_1909_06412_amd as mg
    return mg


def _errs(psi, ref):
    l2 = float(np.linalg.norm((psi - ref).ravel()) / np.linalg.norm(ref.ravel()))
    mx = float(np.max(np.abs(psi - ref)) / np.max(np.abs(ref)))
    return l2, mx


def _oracle(w, nsteps, gam=None):
    g = O.Grid(w["N"], w["dq"], w["hbar"])
    wp = O.gaussian(g, w["q0"], w["p0"], w["sigma"])
    pot = O.potentials.from_spec(*w["potential"], w["D"])
    gam = O.composition(w["comp"], w["order"]) if gam is None else gam
    O.run(wp, w["dt"], nsteps, gam, pot, w["inv_mass"], w["split"])
    return wp


def _check(tag, psi, q, p, wp, tol, tol_ctr):
    l2, mx = _errs(psi, wp.physical())
    dq = float(np.max(np.abs(q - wp.q_ctr)))
    dp = float(np.max(np.abs(p - wp.p_ctr)))
    print(f"[configs] {tag}: l2 {l2:.3e} max {mx:.3e} dq {dq:.2e} dp {dp:.2e}", flush=True)
    assert l2 < tol and mx < tol, (l2, mx)
    assert dq < tol_ctr and dp < tol_ctr, (dq, dp)
    return l2, mx


# ---------------------------------------------------------------------------
# 3-D harmonic model, 32^3, t_f = 5
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [2, 4, 6, 8, 10])
def test_harmonic_3d_orders_to_final_time(order):
    """Seed 0 at dt = 0.1 up to t_f = 5 (50 steps; 81 stages a step at order 10):
    complex128 within 1e-11 of the oracle over the whole horizon, and its error
    against the exact harmonic solution is the oracle's."""
    mg = _mg()
    w = W.harmonic_3d(seed=0, order=order, dt=0.1, t_final=5.0)
    n = w["steps"]
    wp = _oracle(w, n)
    m = mg.from_workload(w, precision="c128")
    m.step(w["dt"], n)
    psi, q, p, t = m.get_state()
    m.close()
    _check(f"32^3 order {order} c128 t={t:.2f}", psi, q, p, wp, 1e-11, 1e-11)
    pot = O.potentials.from_spec(*w["potential"], 3)
    ge = cf.exact_quadratic(cf.initial(w["q0"], w["p0"], w["sigma"]), 5.0, pot.K, pot.s, w["inv_mass"])
    ex = cf.values(ge, wp.grid.q_mesh(q))
    dv = math.sqrt(np.prod(wp.grid.dq))
    e_gpu = float(np.linalg.norm(psi - ex) * dv)
    e_orc = float(np.linalg.norm(wp.physical() - cf.values(ge, wp.grid.q_mesh(wp.q_ctr))) * dv)
    print(f"[configs] 32^3 order {order}: error vs exact solution gpu {e_gpu:.3e} oracle {e_orc:.3e}",
          flush=True)
    assert abs(e_gpu - e_orc) < 1e-10


@pytest.mark.parametrize("order", [2, 4, 10])
def test_harmonic_3d_c64_to_final_time(order):
    """complex64 over the whole horizon: 50 stages (order 2) to 4050 stages (order
    10).  Its error is FP32 rounding that a moving grid keeps from averaging out (the
    state barely changes in the grid's frame, so each stage rounds nearly the same
    numbers the same way): measured l2 1.2e-5 (max 3.3e-6) after 4050 stages, so runs
    beyond 1000 stages are held to 2e-5 in l2 and 1e-5 element-wise."""
    mg = _mg()
    w = W.harmonic_3d(seed=0, order=order, dt=0.1, t_final=5.0, precision="c64")
    n = w["steps"]
    wp = _oracle(w, n)
    m = mg.from_workload(w, precision="c64")
    m.step(w["dt"], n)
    psi, q, p, _ = m.get_state()
    m.close()
    stages = n * len(O.composition(w["comp"], w["order"]))
    l2, mx = _check(f"32^3 order {order} c64 ({stages} stages)", psi, q, p, wp,
                    TOL64 if stages <= 1000 else 2e-5, 1e-6)
    assert mx < TOL64


# ---------------------------------------------------------------------------
# Atom-diatom model at 256^2
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision,tol,tol_ctr", [("c128", 1e-11, 1e-11), ("c64", TOL64, 1e-6)])
def test_atom_diatom_256sq(precision, tol, tol_ctr):
    mg = _mg()
    w = W.morse_repulsion_2d(256, 256, steps=0, precision=precision)
    n = 300
    wp = _oracle(w, n)
    m = mg.from_workload(w, precision=precision)
    m.step(w["dt"], n)
    psi, q, p, _ = m.get_state()
    norm = m.observables()["norm"]
    m.close()
    _check(f"256^2 {precision} {n} steps (norm-1 {norm - 1:.2e})", psi, q, p, wp, tol, tol_ctr)


# ---------------------------------------------------------------------------
# 256 packets in one batch
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision,shape", [("c64", 0), ("c64", 5), ("c128", 5)])
def test_batch_256_packets_sampled(precision, shape):
    mg = _mg()
    ws = W.morse_batch(B=256, steps=0, precision=precision)
    b = mg.batch_from_workloads(ws, precision=precision)
    b.set_config(shape)
    n = 100
    b.step(ws[0]["dt"], n)
    rng = np.random.default_rng(5)
    pick = sorted(rng.choice(256, 16, replace=False).tolist())
    tol, tol_ctr = (TOL64, 1e-6) if precision == "c64" else (1e-11, 1e-11)
    try:
        for i in pick:
            wp = _oracle(ws[i], n)
            psi, q, p, _ = b.get_state(i)
            _check(f"batch[{i}] {ws[i]['N']} {precision} shape {shape}", psi, q, p, wp, tol, tol_ctr)
    finally:
        b.close()


# ---------------------------------------------------------------------------
# Coupled Henon-Heiles on the 16-point kernels
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision,tol,tol_ctr", [("c128", TOL128, 1e-12), ("c64", TOL64, 1e-6)])
def test_coupled_henon_heiles_16e6_two_steps(precision, tol, tol_ctr):
    """lambda = 0.111803 on 16^6 (16.8 M points), two Suzuki-4 steps against the full
    oracle (its FFTs on 16 threads)."""
    mg = _mg()
    O.grid.set_fft_workers(16)
    try:
        w = W.henon_heiles_8d(n=16, D=6, dq=0.625, precision=precision)
        w["q0"] = [2.0 - 0.1 * l for l in range(6)]
        w["p0"] = [0.05 * l for l in range(6)]
        n = 2
        wp = _oracle(w, n)
    finally:
        O.grid.set_fft_workers(1)
    m = mg.from_workload(w, precision=precision)
    m.step(w["dt"], n)
    psi, q, p, _ = m.get_state()
    m.close()
    _check(f"coupled HH 16^6 {precision}", psi, q, p, wp, tol, tol_ctr)


def _axis_run(N, dq, q0, p0, sigma, h):
    """1-D oracle: the kinetic substep U_T,adpt(h) on axis l's Gaussian (16 points)."""
    g = O.Grid([N], [dq])
    wp = O.gaussian(g, [q0], [p0], [sigma])
    O.T_substep(wp, h, [1.0])
    return wp


@pytest.mark.parametrize("precision,tol,tol_ctr", [("c128", TOL128, 1e-12), ("c64", TOL64, 1e-7)])
def test_coupled_henon_heiles_16e8_potential_substep(precision, tol, tol_ctr):
    """The headline 16^8 grid (lambda = 0.111803) through its potential substep.
    One Strang step T(h/2) V(h) T(h/2), then the free potential and a step of -h/2
    (= T(-h/2), the kinetic substeps merge exactly and leave the grid where it was)
    leaves V(h) T(h/2) psi0.  T(h/2) psi0 is the product of eight 1-D oracle kinetic
    substeps (the kinetic operator and psi0 factorise), and V(h) multiplies each point
    by exp(-i h V(q)) on that grid: the oracle's V at sampled grid points, and p_ctr
    moves by -h <dV/dq> (Eq. (47)), whose expectation under the product density is a
    sum over the three coordinates each dV/dq_m involves.  This exercises the coupled
    potential epilogue of the three-pass 16^8 plan (the outer-axis terms included)."""
    import torch
    mg = _mg()
    w = W.henon_heiles_8d(precision=precision)
    w["q0"] = [2.0 - 0.1 * l for l in range(8)]
    w["p0"] = [0.1 * l - 0.3 for l in range(8)]
    D, N, dq, h = 8, 16, w["dq"][0], 0.01
    axes = [_axis_run(N, dq, w["q0"][l], w["p0"][l], w["sigma"][l], h / 2) for l in range(D)]
    fac = [a.physical()[:] for a in axes]
    q_ctr = np.array([a.q_ctr[0] for a in axes])
    pot = O.potentials.from_spec(*w["potential"], D)
    # <dV/dq_m> under the product density: dV/dq_m depends on q_{m-1}, q_m, q_{m+1}
    dens = [np.abs(f) ** 2 / np.sum(np.abs(f) ** 2) for f in fac]
    qax = [q_ctr[l] + (np.arange(N) - N / 2) * dq for l in range(D)]
    force = np.zeros(D)
    for mm in range(D):
        ls = [l for l in (mm - 1, mm, mm + 1) if 0 <= l < D]
        qs, wgt = [], 1.0
        for l in range(D):
            sh = [1] * len(ls)
            if l in ls:
                k = ls.index(l)
                sh[k] = N
                qs.append(qax[l].reshape(sh))
                wgt = wgt * dens[l].reshape(sh)
            else:
                qs.append(np.zeros([1] * len(ls)))
        force[mm] = float(np.sum(wgt * pot.grad(qs)[mm]))
    p_ref = np.array(w["p0"]) - h * force
    # sampled points: half uniform, half from the 1-D densities
    rng = np.random.default_rng(23)
    ns = 1 << 16
    dig = np.empty((ns, D), dtype=np.int64)
    dig[: ns // 2] = rng.integers(0, N, size=(ns // 2, D))
    for l in range(D):
        dig[ns // 2:, l] = rng.choice(N, size=ns - ns // 2, p=dens[l])
    flat = np.zeros(ns, dtype=np.int64)
    for l in range(D):
        flat = flat * N + dig[:, l]
    qs = [qax[l][dig[:, l]] for l in range(D)]
    ref = np.ones(ns, dtype=np.complex128)
    for l in range(D):
        ref = ref * fac[l][dig[:, l]]
    ref = ref * np.exp(-1j * h * pot.V(qs))
    print(f"[configs] 16^8 potential substep {precision}: running", flush=True)
    m = mg.from_workload(w, precision=precision)
    try:
        m.set_scheme("TVT", "strang", 2)
        m.step(h, 1)
        m.set_potential("free", {})
        m.step(-h / 2, 1)
        v = m.state_view()
        got = v.index_select(0, torch.from_numpy(flat).to(v.device)).to(torch.complex128).cpu().numpy()
        got = got / np.sqrt(dq ** D)
        q, p, _ = m.centres()
    finally:
        m.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    l2, mx = _errs(got, ref)
    dqc, dpc = float(np.max(np.abs(q - q_ctr))), float(np.max(np.abs(p - p_ref)))
    print(f"[configs] 16^8 potential substep {precision}: sampled l2 {l2:.3e} max {mx:.3e} "
          f"dq {dqc:.2e} dp {dpc:.2e}", flush=True)
    assert np.max(np.abs(h * force)) > 1e-3
    assert l2 < tol and mx < tol
    assert dqc < tol_ctr and dpc < tol_ctr


# ---------------------------------------------------------------------------
# Options: user compositions, renormalisation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_user_gammas_equal_builtin_family(precision):
    """MG_COMP_USER with Suzuki's fourth-order coefficients (from the oracle's closed
    form) gives the built-in family's result bit for bit, single grid and batch."""
    mg = _mg()
    gam = O.composition("suzuki", 4)
    w = W.harmonic_3d(seed=4, order=4, dt=0.05, precision=precision)
    out = []
    for comp in ("suzuki", "user"):
        m = mg.from_workload(w, precision=precision)
        m.set_scheme("TVT", comp, 4, gammas=gam if comp == "user" else None)
        m.step(w["dt"], 6)
        out.append(m.get_state())
        m.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])
    ws = W.morse_batch(B=6, steps=0, precision=precision)
    res = []
    for comp in ("suzuki", "user"):
        b = mg.batch_from_workloads(ws, precision=precision)
        b.set_scheme("TVT", comp, 4, gammas=gam if comp == "user" else None)
        b.step(ws[0]["dt"], 4)
        res.append([b.get_state(i)[0] for i in range(len(ws))])
        b.close()
    for a, c in zip(*res):
        assert np.array_equal(a, c)


def test_user_gammas_rejected_when_not_a_composition():
    mg = _mg()
    w = W.harmonic_1d()
    m = mg.from_workload(w)
    try:
        for bad in ([0.5, 0.6], [0.3, 0.4, 0.2]):         # sum != 1, not a palindrome
            with pytest.raises(mg.MgError):
                m.set_scheme("TVT", "user", 4, gammas=bad)
    finally:
        m.close()


def test_renormalize_option():
    """MG_OPT_RENORMALIZE rescales to the FP64 norm after every potential substep: in
    complex128 (norm already exact) the result equals the plain run to rounding; in
    complex64 the norm stays at one to FP32 rounding and the state follows the
    oracle."""
    mg = _mg()
    w = W.morse_repulsion_2d(128, 96, steps=0, precision="c128")
    n = 60
    wp = _oracle(w, n)
    runs = {}
    for prec in ("c128", "c64"):
        for ren in (0, 1):
            m = mg.from_workload(w, precision=prec)
            m.set_option(mg.MG_OPT_RENORMALIZE, ren)
            m.step(w["dt"], n)
            psi, q, p, _ = m.get_state()
            runs[(prec, ren)] = (psi, q, p, m.observables()["norm"])
            m.close()
    a, b = runs[("c128", 0)], runs[("c128", 1)]
    assert _errs(b[0], a[0])[0] < 1e-13
    assert abs(b[3] - 1.0) < 1e-13
    for ren in (0, 1):
        psi, q, p, norm = runs[("c64", ren)]
        _check(f"renormalize={ren} c64 norm-1 {norm - 1:.2e}", psi, q, p, wp, TOL64, 1e-6)
    assert abs(runs[("c64", 1)][3] - 1.0) < 1e-6
