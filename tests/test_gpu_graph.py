"""MG_OPT_GRAPH: the launches of a step call captured once as a hipGraph and
replayed.  Every replay is checked against an eager context fed the same calls,
with eager work (observables, state reads) and synchronisations between the
replays; a changed step count, time step or scheme must re-capture."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _mg():
    import paper_1909_06412_amd as mg
    return mg


def _pair(w, precision):
    mg = _mg()
    a = mg.from_workload(w, precision=precision)
    b = mg.from_workload(w, precision=precision)
    b.set_option(mg.MG_OPT_GRAPH, 1)
    return a, b


def _same(a, b, tag):
    pa, qa, pa_, ta = a.get_state()
    pb, qb, pb_, tb = b.get_state()
    d = float(np.max(np.abs(pa - pb)))
    print(f"[graph] {tag}: max |eager - replay| = {d:.3e}", flush=True)
    assert d == 0.0
    assert np.array_equal(qa, qb) and np.array_equal(pa_, pb_) and ta == tb


@pytest.mark.parametrize("case", ["harmonic_32^3", "henon_heiles_16^4", "harmonic_1d_64"])
@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_step_graph_replays_match_eager(case, precision):
    # harmonic_1d_64 fits one tile: its sweeps run the finalize in their one workgroup
    if case == "harmonic_32^3":
        w = W.harmonic_3d(seed=1, order=4, dt=0.05)
    elif case == "harmonic_1d_64":
        w = W.harmonic_1d()
    else:
        w = W.henon_heiles_8d(n=16, D=4, dq=0.625)
    a, b = _pair(w, precision)
    for rep in range(3):
        a.step(w["dt"], 4)
        b.step(w["dt"], 4)           # rep 0 captures, reps 1-2 replay
        _same(a, b, f"{case} {precision} replay {rep}")
        oa, ob = a.observables(), b.observables()   # eager work between replays
        assert oa["norm"] == ob["norm"]
    a.step(w["dt"], 2)
    b.step(w["dt"], 2)               # new step count: re-capture
    _same(a, b, f"{case} {precision} nsteps changed")
    for m in (a, b):
        m.set_scheme("VTV", "strang", 2)
    a.step(w["dt"], 3)
    b.step(w["dt"], 3)               # new scheme: re-capture
    b.step(w["dt"], 3)
    a.step(w["dt"], 3)
    _same(a, b, f"{case} {precision} scheme changed")
    a.close()
    b.close()


@pytest.mark.parametrize("shape", [0, 5])
def test_batch_graph_replays_match_eager(shape):
    """Persistent shape 0 (one captured launch) and the streaming shape 5 (a
    captured sequence of sweep and update launches)."""
    mg = _mg()
    ws = W.morse_batch(B=12, precision="c64")
    a = mg.batch_from_workloads(ws, precision="c64")
    b = mg.batch_from_workloads(ws, precision="c64")
    a.set_config(shape)
    b.set_config(shape)
    b.set_option(mg.MG_OPT_GRAPH, 1)
    dt = ws[0]["dt"]
    for rep, (h, n) in enumerate([(dt, 5), (dt, 5), (dt, 5), (0.5 * dt, 5), (0.5 * dt, 5), (dt, 3)]):
        a.step(h, n)
        b.step(h, n)
        oa, ob = a.observables(), b.observables()
        for i in range(len(ws)):
            pa, *_ = a.get_state(i)
            pb, *_ = b.get_state(i)
            assert np.array_equal(pa, pb), (rep, i)
            assert oa[i]["norm"] == ob[i]["norm"]
        print(f"[graph] batch shape {shape} call {rep} (dt {h}, {n} steps): replay == eager", flush=True)
    a.close()
    b.close()
