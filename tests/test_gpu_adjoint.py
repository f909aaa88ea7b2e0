"""GPU adjoint (gradient of the transmitted-probability objective with respect to
potential parameters) against central finite differences of whole FP64 oracle
propagations.  The oracle has no adjoint of its own; its finite-difference
gradient is pinned to the closed-form Gaussian map in the oracle pin tests.

Cases: the Morse + exponential-repulsion packet (parameters A and b of the
repulsion), TVT and VTV splittings, Strang and 4th-order Suzuki compositions,
checkpoint intervals from every step to the whole run, a 1-D harmonic oscillator
(gradient with respect to the force constant), the FP32 storage path, and the
per-packet batched adjoint over packets of uneven shapes."""
import numpy as np
import pytest

import oracle as O
import oracle.gradient as OG
import workloads as W

pytestmark = pytest.mark.gpu

# window of the objective: W = 1/(1 + exp(-(R_d - R)/w)) on R = rho - r/2
RD, WD = 2.55, 0.1
NSTEPS = 150
# Relative step of the oracle's central differences.  On these grids the central
# differences agree across steps 1e-4 .. 3e-6 to ~1e-11 (A) and ~3e-10 (b), which sets
# FD_ATOL; the adjoint itself is the exact derivative of the discrete map.
FD_REL = 3e-5
FD_ATOL = 2e-9
FD_RTOL = 1e-7
# Physical spans of the (r, rho) grid.  They keep the repulsive wall on the grid below
# ~1e2 Eh: where the wall reaches 1e4..1e8 Eh (the 9.6 x 16 spans of the scattering
# runs) the phase exp(-i h V) turns so fast with b that finite differences of any
# practical step leave the linear regime, while the adjoint stays exact.
SPAN = (3.2, 6.0)


def _mg():
    import paper_1909_06412_amd as mg
    return mg


def morse_case(n1=48, n2=64, split="TVT", comp="strang", order=2, precision="c128", rho0=3.2,
               p0=-19.2):
    """A packet started close to the repulsive wall, so that the window straddles it
    and the parameters of the repulsion move the transmitted probability."""
    w = W.morse_repulsion_2d(n1, n2, p0_rho=p0, steps=NSTEPS, precision=precision)
    w = W.scaled(w, dq=[SPAN[0] / n1, SPAN[1] / n2], q0=[w["q0"][0], rho0], dt=0.2,
                 split=split, comp=comp, order=order)
    return w


def harmonic_case(precision="c128"):
    w = W.harmonic_1d()
    return W.scaled(w, precision=precision)


def gpu_adjoint(w, ids, K, nsteps=NSTEPS, window=(RD, WD)):
    mg = _mg()
    m = mg.from_workload(w)
    J, g = m.adjoint(w["dt"], nsteps, K, window, ids)
    psi, q, p, t = m.get_state()
    m.close()
    return J, g, (psi, q, p, t)


def fd_harmonic(w, nsteps, rel=1e-4):
    kind, base = w["potential"]
    k0 = np.asarray(base["k"], float)
    out = []
    for l in range(len(k0)):
        h = rel * max(abs(k0[l]), 1.0)
        vals = []
        for sgn in (1, -1):
            k = k0.copy()
            k[l] += sgn * h
            par = dict(base)
            par["k"] = list(k)
            vals.append(OG.run_objective(w, par, nsteps, RD_H, WD_H))
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.array(out)


RD_H, WD_H = 0.5, 0.3


def _report(tag, J, g, Jref, gref):
    print(f"[adjoint] {tag}: J {J:.15f} ref {Jref:.15f}  grad {g} ref {gref}", flush=True)


@pytest.fixture(scope="module")
def morse_ref():
    w = morse_case()
    Jref = OG.run_objective(w, w["potential"][1], NSTEPS, RD, WD)
    gref = OG.fd_gradient(w, ["A", "b"], NSTEPS, RD, WD, rel=FD_REL)
    return w, Jref, gref


def test_morse_objective_is_nontrivial(morse_ref):
    w, Jref, gref = morse_ref
    assert 0.05 < Jref < 0.95
    assert np.all(np.abs(gref) > 1e-3)


@pytest.mark.parametrize("K", [1, 7, NSTEPS])
def test_morse_gradient_c128(morse_ref, K):
    w, Jref, gref = morse_ref
    J, g, _ = gpu_adjoint(w, [3, 4], K)
    _report(f"morse c128 K={K}", J, g, Jref, gref)
    assert abs(J - Jref) < 1e-11
    np.testing.assert_allclose(g, gref, rtol=FD_RTOL, atol=FD_ATOL)


def test_checkpoint_interval_does_not_change_the_gradient():
    w = morse_case()
    _, g1, _ = gpu_adjoint(w, [3, 4], 1)
    _, g2, _ = gpu_adjoint(w, [3, 4], 16)
    np.testing.assert_allclose(g1, g2, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("split,comp,order", [("VTV", "strang", 2), ("TVT", "suzuki", 4),
                                              ("VTV", "triple_jump", 4)])
def test_morse_gradient_schemes(split, comp, order):
    w = morse_case(split=split, comp=comp, order=order)
    n = 20
    Jref = OG.run_objective(w, w["potential"][1], n, RD, WD)
    gref = OG.fd_gradient(w, ["A", "b"], n, RD, WD, rel=FD_REL)
    J, g, _ = gpu_adjoint(w, [3, 4], 6, nsteps=n)
    _report(f"morse {split} {comp}{order}", J, g, Jref, gref)
    assert abs(J - Jref) < 1e-11
    np.testing.assert_allclose(g, gref, rtol=FD_RTOL, atol=FD_ATOL)


def test_ragged_shape_gradient():
    """Axis lengths with radix-3 and radix-5 factors (90 x 72)."""
    w = morse_case(n1=90, n2=72)
    n = 30
    Jref = OG.run_objective(w, w["potential"][1], n, RD, WD)
    gref = OG.fd_gradient(w, ["A", "b"], n, RD, WD, rel=FD_REL)
    J, g, _ = gpu_adjoint(w, [4, 3], 8, nsteps=n)
    _report("morse 90x72", J, g, Jref, gref[::-1])
    assert abs(J - Jref) < 1e-11
    np.testing.assert_allclose(g, gref[::-1], rtol=FD_RTOL, atol=FD_ATOL)


def test_adjoint_leaves_the_propagated_state():
    mg = _mg()
    w = morse_case()
    _, _, (psi, q, p, t) = gpu_adjoint(w, [3], 5, nsteps=20)
    m = mg.from_workload(w)
    m.step(w["dt"], 20)
    psi2, q2, p2, t2 = m.get_state()
    m.close()
    assert np.linalg.norm(psi - psi2) / np.linalg.norm(psi2) < 1e-11
    assert np.max(np.abs(q - q2)) < 1e-11 and np.max(np.abs(p - p2)) < 1e-10
    assert abs(t - t2) < 1e-12


def test_harmonic_1d_gradient():
    w = harmonic_case()
    n = 40
    Jref = OG.run_objective(w, w["potential"][1], n, RD_H, WD_H)
    gref = fd_harmonic(w, n)
    J, g, _ = gpu_adjoint(w, [0], 9, nsteps=n, window=(RD_H, WD_H))
    _report("harmonic 1d", J, g, Jref, gref)
    assert abs(gref[0]) > 1e-3
    assert abs(J - Jref) < 1e-11
    np.testing.assert_allclose(g, gref, rtol=FD_RTOL, atol=FD_ATOL)


def test_morse_gradient_c64(morse_ref):
    w, Jref, gref = morse_ref
    J, g, _ = gpu_adjoint(W.scaled(w, precision="c64"), [3, 4], 10)
    _report("morse c64", J, g, Jref, gref)
    # FP32 storage over 450 substeps: the objective itself moves by ~3e-5 relative
    assert abs(J - Jref) < 1e-4 * abs(Jref)
    np.testing.assert_allclose(g, gref, rtol=2e-4, atol=1e-7)


def test_batch_adjoint_matches_single_packets():
    mg = _mg()
    ws = [morse_case(n1, n2, p0=p0) for (n1, n2), p0 in
          zip([(48, 64), (72, 90), (96, 80)], [-19.2, -15.0, -25.0])]
    b = mg.batch_from_workloads(ws, precision="c128")
    J, g = b.adjoint(ws[0]["dt"], 25, 5, (RD, WD), [3, 4])
    b.close()
    for i, w in enumerate(ws):
        Ji, gi, _ = gpu_adjoint(w, [3, 4], 5, nsteps=25)
        print(f"[adjoint] batch packet {i}: J {J[i]:.15f} single {Ji:.15f}", flush=True)
        # the batch kernel runs unfused substeps; the single-packet forward fuses them
        assert abs(J[i] - Ji) < 1e-12
        np.testing.assert_allclose(g[i], gi, rtol=1e-9, atol=1e-13)


def test_unsupported_parameter_is_rejected():
    mg = _mg()
    w = morse_case()
    m = mg.from_workload(w)
    with pytest.raises(mg.MgError):
        m.adjoint(w["dt"], 2, 1, (RD, WD), [0])    # De: not offered
    with pytest.raises(mg.MgError):
        m.adjoint(w["dt"], 2, 0, (RD, WD), [3])    # K < 1
    m.close()


def test_batch_adjoint_multi_tile_packets():
    """Packets larger than one LDS tile of the batch kernel (complex64: 16384 points)
    sweep through global memory tile by tile inside the persistent adjoint; complex64
    and complex128 batches agree with each other and with single-packet adjoints."""
    mg = _mg()
    shapes = [(48, 64), (192, 96), (150, 162), (90, 72)]
    ws = [morse_case(n1, n2, p0=p0) for (n1, n2), p0 in zip(shapes, [-19.2, -15.0, -25.0, -21.0])]
    n, K = 30, 7
    res = {}
    for prec in ("c128", "c64"):
        b = mg.batch_from_workloads(ws, precision=prec)
        res[prec] = b.adjoint(ws[0]["dt"], n, K, (RD, WD), [3, 4])
        b.close()
    for i, w in enumerate(ws):
        Ji, gi, _ = gpu_adjoint(w, [3, 4], K, nsteps=n)
        J128, g128 = res["c128"][0][i], res["c128"][1][i]
        J64, g64 = res["c64"][0][i], res["c64"][1][i]
        print(f"[adjoint] batch {w['N']}: J {J128:.15f} single {Ji:.15f} c64 {J64:.9f}; "
              f"grad {g128} c64 {g64}", flush=True)
        assert abs(J128 - Ji) < 1e-12
        np.testing.assert_allclose(g128, gi, rtol=1e-9, atol=1e-13)
        assert abs(J64 - J128) < 1e-4 * abs(J128)
        np.testing.assert_allclose(g64, g128, rtol=2e-3, atol=1e-6)


def test_autograd_function():
    """torch.autograd through the adjoint: the gradient equals mg_adjoint's, J at a
    moved theta equals the oracle's objective there, and a batch's J (one entry
    per packet, shared theta) back-propagates the weighted sum of the packets'
    gradients."""
    import torch
    mg = _mg()
    w = morse_case()
    n, K = 40, 8
    m = mg.from_workload(w)
    theta = torch.tensor([9.5, 2.1], dtype=torch.float64, requires_grad=True)
    J = mg.transmitted_probability(m, theta, w["dt"], n, K, (RD, WD), [3, 4])
    J.backward()
    m.close()
    par = dict(w["potential"][1], A=9.5, b=2.1)
    Jref = OG.run_objective(w, par, n, RD, WD)
    wr = W.scaled(w, potential=("morse_repulsion", par))
    _, gr, _ = gpu_adjoint(wr, [3, 4], K, nsteps=n)
    print(f"[adjoint] autograd: J {J.item():.15f} oracle {Jref:.15f} grad {theta.grad.numpy()} adjoint {gr}",
          flush=True)
    assert abs(J.item() - Jref) < 1e-11
    np.testing.assert_allclose(theta.grad.numpy(), gr, rtol=1e-13, atol=0)
    ws = [morse_case(48, 64, p0=-19.2), morse_case(72, 90, p0=-16.0)]
    b = mg.batch_from_workloads(ws, precision="c128")
    th = torch.tensor([10.0, 2.0], dtype=torch.float64, requires_grad=True)
    Jb = mg.transmitted_probability(b, th, ws[0]["dt"], 20, 5, (RD, WD), [3, 4])
    (Jb * torch.tensor([1.0, -2.0], dtype=torch.float64)).sum().backward()
    b.close()
    b2 = mg.batch_from_workloads(ws, precision="c128")
    _, g2 = b2.adjoint(ws[0]["dt"], 20, 5, (RD, WD), [3, 4])
    b2.close()
    np.testing.assert_allclose(th.grad.numpy(), g2[0] - 2.0 * g2[1], rtol=1e-12, atol=1e-16)
