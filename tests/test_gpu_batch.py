"""GPU parity of the batched persistent engine (one launch for every packet and
every step) against the FP64 oracle, packet by packet.  The packets have uneven
shapes: some fit one LDS tile and stay resident for the whole run, others sweep
through global memory; lengths include radix-3 and radix-5 factors."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

SHAPES = [(64, 64), (72, 90), (128, 96), (180, 192), (100, 80), (150, 162)]


def _mg():
    import paper_1909_06412_amd as mg
    return mg


def oracle_packet(w, nsteps):
    g = O.Grid(w["N"], w["dq"], w["hbar"])
    wp = O.gaussian(g, w["q0"], w["p0"], w["sigma"])
    pot = O.potentials.from_spec(*w["potential"], w["D"])
    O.run(wp, w["dt"], nsteps, O.composition(w["comp"], w["order"]), pot, w["inv_mass"], w["split"])
    return wp


def _batch_workloads(split="TVT", comp="strang", order=2, precision="c128"):
    ws = []
    rng = np.random.default_rng(11)
    for k, (n1, n2) in enumerate(SHAPES):
        w = W.morse_repulsion_2d(n1, n2, p0_rho=float(rng.uniform(-27.1, -13.55)), steps=0,
                                 precision=precision)
        w["split"], w["comp"], w["order"] = split, comp, order
        ws.append(w)
    return ws


def _check(ws, nsteps, precision, tol, tol_ctr):
    mg = _mg()
    b = mg.batch_from_workloads(ws, precision=precision)
    assert b.points == sum(int(np.prod(w["N"])) for w in ws)
    b.step(ws[0]["dt"], nsteps)
    worst = 0.0
    for i, w in enumerate(ws):
        wp = oracle_packet(w, nsteps)
        psi, q, p, t = b.get_state(i)
        ref = wp.physical()
        e = np.linalg.norm(psi - ref) / np.linalg.norm(ref)
        print(f"[batch parity] packet {i} {w['N']} {precision} err {e:.3e} "
              f"dq {np.max(np.abs(q - wp.q_ctr)):.2e}", flush=True)
        assert e < tol, (i, e)
        assert np.max(np.abs(q - wp.q_ctr)) < tol_ctr
        assert np.max(np.abs(p - wp.p_ctr)) < tol_ctr
        assert abs(t - nsteps * ws[0]["dt"]) < 1e-12
        worst = max(worst, e)
    b.close()
    return worst


@pytest.mark.parametrize("split,comp,order", [("TVT", "strang", 2), ("VTV", "strang", 2),
                                              ("TVT", "suzuki", 4)])
def test_batch_c128_matches_oracle(split, comp, order):
    ws = _batch_workloads(split, comp, order, "c128")
    _check(ws, 12 if order == 2 else 4, "c128", 1e-12, 1e-12)


def test_batch_c64_matches_oracle():
    ws = _batch_workloads(precision="c64")
    _check(ws, 20, "c64", 1e-5, 1e-6)


def test_batch_henon_heiles_3d_mixed_shapes():
    mg = _mg()
    ws = []
    for shape in [(16, 16, 16), (12, 10, 18), (24, 20, 30), (8, 8, 8)]:
        w = W.henon_heiles_8d(n=8, D=3, dq=0.6, lam=0.111803, precision="c128")
        w["N"] = list(shape)
        w["dq"] = [9.0 / n for n in shape]
        w["q0"] = [1.0, 0.5, -0.5]
        ws.append(w)
    _check(ws, 3, "c128", 1e-12, 1e-12)


def test_batch_matches_single_context_and_observables():
    mg = _mg()
    ws = _batch_workloads(precision="c128")[:3]
    b = mg.batch_from_workloads(ws)
    b.step(ws[0]["dt"], 7)
    obs = b.observables()
    for i, w in enumerate(ws):
        m = mg.from_workload(w)
        m.step(w["dt"], 7)
        ob1 = m.observables()
        for k in ("norm", "E"):
            assert abs(obs[i][k] - ob1[k]) < 1e-12 * max(1, abs(ob1[k]))
        np.testing.assert_allclose(obs[i]["q_ctr"], ob1["q_ctr"], atol=1e-12)
        m.close()
    b.close()


def test_launch_shapes_and_autotune():
    """Every launch shape of the batch step kernel (threads, LDS tile) propagates the
    same physics: each agrees with the oracle packet by packet; the autotuner times
    the shapes on the batch's own state and restores that state bit for bit."""
    mg = _mg()
    ws = _batch_workloads(precision="c64")
    nsteps = 20
    refs = [oracle_packet(w, nsteps).physical() for w in ws]
    b = mg.batch_from_workloads(ws, precision="c64")
    psi0 = [b.get_state(i) for i in range(len(ws))]
    chosen, ms = b.autotune(ws[0]["dt"], 5)
    print(f"[batch] autotune: shapes {[b.config(k) for k in range(b.N_CONFIGS)]} ms/step {ms} -> {chosen}",
          flush=True)
    assert 0 <= chosen < b.N_CONFIGS and np.all(ms > 0)
    for i in range(len(ws)):
        p, q, pc, t = b.get_state(i)
        assert np.array_equal(p, psi0[i][0]) and np.array_equal(q, psi0[i][1])
        assert np.array_equal(pc, psi0[i][2]) and t == psi0[i][3]
    b.close()
    for k in range(mg.MovingGridBatch.N_CONFIGS):
        b = mg.batch_from_workloads(ws, precision="c64")
        b.set_config(k)
        b.step(ws[0]["dt"], nsteps)
        worst = 0.0
        for i, ref in enumerate(refs):
            psi, *_ = b.get_state(i)
            worst = max(worst, np.linalg.norm(psi - ref) / np.linalg.norm(ref))
        print(f"[batch] shape {k} {b.config(k)}: worst packet error vs oracle {worst:.3e}", flush=True)
        assert worst < 2e-5
        b.close()


def test_launch_shapes_c128():
    """Every complex128 launch shape, in-place and ping-pong transforms alike,
    matches the oracle packet by packet at the double-precision bar."""
    mg = _mg()
    ws = _batch_workloads(precision="c128")
    nsteps = 10
    refs = [oracle_packet(w, nsteps).physical() for w in ws]
    for k in range(mg.MovingGridBatch.N_CONFIGS):
        b = mg.batch_from_workloads(ws, precision="c128")
        b.set_config(k)
        b.step(ws[0]["dt"], nsteps)
        worst = 0.0
        for i, ref in enumerate(refs):
            psi, *_ = b.get_state(i)
            worst = max(worst, np.linalg.norm(psi - ref) / np.linalg.norm(ref))
        print(f"[batch] c128 shape {k} {b.config(k)}: worst packet error vs oracle {worst:.3e}", flush=True)
        assert worst < 1e-12
        b.close()


@pytest.mark.parametrize("split,comp,order", [("VTV", "strang", 2), ("TVT", "suzuki", 4), ("VTV", "triple_jump", 4)])
def test_streaming_shape_schemes(split, comp, order):
    """The streaming launch shape (one launch per sweep over every packet's tiles,
    potential-only units as one pointwise launch) follows the oracle for both splits
    and higher-order compositions, complex128 at the double-precision bar."""
    mg = _mg()
    ws = _batch_workloads(split, comp, order, "c128")
    nsteps = 6
    b = mg.batch_from_workloads(ws, precision="c128")
    b.set_config(mg.MovingGridBatch.N_CONFIGS - 1)
    b.step(ws[0]["dt"], nsteps)
    worst = 0.0
    for i, w in enumerate(ws):
        wp = oracle_packet(w, nsteps)
        psi, q, p, t = b.get_state(i)
        ref = wp.physical()
        worst = max(worst, np.linalg.norm(psi - ref) / np.linalg.norm(ref))
        assert np.max(np.abs(q - wp.q_ctr)) < 1e-11 and np.max(np.abs(p - wp.p_ctr)) < 1e-11
        assert abs(t - nsteps * ws[0]["dt"]) < 1e-12
    print(f"[batch] streaming shape {split} {comp} {order}: worst packet error vs oracle {worst:.3e}", flush=True)
    assert worst < 1e-12
    b.close()
