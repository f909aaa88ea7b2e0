"""mg_propagate_noalloc (the propagation of mg_step with its plan buffers in the
library's file-scope device scratch array, no device allocation) against the
context entry points on the same input: calls in a row, each on a smaller grid
(and the other precision and sweep kernels; the last one on the one-wave path of
one-dimensional grids), each equal to mg_create + mg_step bit for bit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _case(w, precision, nsteps):
    import torch
    import paper_1909_06412_amd as mg
    m = mg.from_workload(w, precision=precision)
    q0, p0, _ = m.centres()
    buf = m.state_view().clone()                   # the initial state, device copy
    print(f"[noalloc] {w['name']} {precision}: {int(np.prod(w['N']))} points, {nsteps} steps", flush=True)
    m.step(w["dt"], nsteps)
    ref = m.state_view().clone()
    qr, pr, _ = m.centres()
    m.close()
    q, p = mg.propagate_noalloc(buf.data_ptr(), w["N"], w["dq"], w["inv_mass"], w["hbar"], precision,
                                w["potential"], (w["split"], w["comp"], w["order"], None), q0, p0,
                                w["dt"], nsteps)
    torch.cuda.synchronize()
    same = bool(torch.equal(buf, ref))
    print(f"[noalloc] {w['name']} {precision}: bit-equal {same}, "
          f"max|diff| {float((buf - ref).abs().max()):.3e}", flush=True)
    assert same
    assert np.array_equal(q, qr) and np.array_equal(p, pr)
    assert np.max(np.abs(q - q0)) > 1e-3                 # the grid moved


def test_noalloc_matches_step_two_calls():
    # first call: coupled 16^6 Henon-Heiles (16-point kernels), complex64, Suzuki-4
    w1 = W.henon_heiles_8d(n=16, D=6, dq=0.625, precision="c64")
    w1["q0"] = [2.0 - 0.1 * l for l in range(6)]
    _case(w1, "c64", 3)
    # second call, smaller: atom-diatom 64 x 80 (Stockham sweeps), complex128, VTV
    w2 = W.morse_repulsion_2d(64, 80, steps=0, precision="c128")
    w2["split"] = "VTV"
    _case(w2, "c128", 25)
    # third call, smaller still: the 64-point oscillator (the one-wave path), complex64
    _case(W.harmonic_1d(), "c64", 100)


def test_noalloc_rejects_bad_arguments():
    import torch
    import paper_1909_06412_amd as mg
    w = W.harmonic_1d()
    buf = torch.zeros(64, dtype=torch.complex128, device="cuda")
    with pytest.raises(mg.MgError) as ei:
        mg.propagate_noalloc(buf.data_ptr() + 16, w["N"], w["dq"], w["inv_mass"], 1.0, "c128", w["potential"],
                             ("TVT", "strang", 2, None), [1.0], [0.0], 0.01, 1)
    assert ei.value.status == mg.MG_EINVAL and "aligned" in str(ei.value)
    with pytest.raises(mg.MgError) as ei:
        mg.propagate_noalloc(buf.data_ptr(), [63], w["dq"], w["inv_mass"], 1.0, "c128", w["potential"],
                             ("TVT", "strang", 2, None), [1.0], [0.0], 0.01, 1)
    assert ei.value.status == mg.MG_EINVAL
