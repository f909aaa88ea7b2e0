"""The C-ABI library loads and exports every entry point that include/mgso.h
declares; argument validation that happens before any device work.  CPU only:
no compute call reaches a GPU here."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgso.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1909_06412_amd import _lib
    return _lib.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mg_create", "mg_set_gaussian", "mg_set_potential", "mg_set_scheme", "mg_step",
                 "mg_observables", "mg_adjoint", "mg_batch_step"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_1909_06412_amd import _lib
    assert sorted(_lib.exported_symbols()) == declared_functions()


@pytest.mark.parametrize("D,N", [(0, []), (9, [4] * 9), (1, [7]), (1, [5]), (2, [8, 14]),
                                 (1, [8192]), (1, [0])])
def test_create_rejects_bad_shapes_without_touching_the_device(lib, D, N):
    from paper_1909_06412_amd import _lib
    h = ctypes.c_void_p()
    Narr = np.asarray(N if N else [0], dtype=np.int32)
    dq = np.ones(max(D, 1))
    st = lib.mg_create(D, Narr.ctypes.data_as(_lib._ip), _lib.dptr(dq), _lib.dptr(dq), 1.0, 0,
                       None, ctypes.byref(h))
    assert st == _lib.MG_EINVAL
    assert not h.value


def test_create_rejects_bad_scalars(lib):
    from paper_1909_06412_amd import _lib
    h = ctypes.c_void_p()
    N = np.asarray([8], dtype=np.int32)
    for dq, hbar, prec in [(np.array([0.0]), 1.0, 0), (np.array([0.1]), 0.0, 0),
                           (np.array([0.1]), 1.0, 7), (np.array([np.nan]), 1.0, 0)]:
        st = lib.mg_create(1, N.ctypes.data_as(_lib._ip), _lib.dptr(dq), _lib.dptr(np.ones(1)),
                           hbar, prec, None, ctypes.byref(h))
        assert st == _lib.MG_EINVAL


@pytest.mark.parametrize("B,D", [(0, 2), (-1, 2), (1, 0), (1, 9)])
def test_batch_create_rejects_bad_counts_without_touching_the_device(lib, B, D):
    from paper_1909_06412_amd import _lib
    h = ctypes.c_void_p()
    N = np.full(max(B, 1) * max(D, 1), 64, dtype=np.int32)
    dq = np.ones(max(B, 1) * max(D, 1))
    st = lib.mg_batch_create(B, D, N.ctypes.data_as(_lib._ip), _lib.dptr(dq), _lib.dptr(dq), 1.0, 0,
                             None, ctypes.byref(h))
    assert st == _lib.MG_EINVAL
    assert not h.value


def test_null_context_calls_fail_cleanly(lib):
    from paper_1909_06412_amd import _lib
    assert lib.mg_step(None, 0.1, 1) == _lib.MG_EINVAL
    assert lib.mg_observables(None, None) == _lib.MG_EINVAL
    assert lib.mg_state_bytes(None) == 0
    assert isinstance(lib.mg_last_error(None), bytes)


def test_spectrum_host_function_matches_oracle():
    """mg_spectrum is host arithmetic (no device work): it must equal the oracle's
    trapezoidal transform of the same autocorrelation series."""
    import numpy as np
    import oracle as O
    import paper_1909_06412_amd as mg
    t = np.linspace(0.0, 40.0, 801)
    acf = np.exp(-1j * 1.3 * t) * np.exp(-0.01 * t) + 0.3 * np.exp(-1j * 2.7 * t)
    E = np.linspace(0.0, 4.0, 57)
    got = mg.spectrum(t, acf, E, t_damp=30.0)
    ref = O.spectrum(t, acf, E, t_damp=30.0)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    # peaks at the two frequencies of the synthetic series
    assert abs(E[np.argmax(got)] - 1.3) < 0.08


def test_binding_knows_every_batch_launch_shape():
    txt = open(HEADER).read()
    n = int(re.search(r"#define MG_BATCH_CONFIGS (\d+)", txt).group(1))
    import paper_1909_06412_amd as mg
    assert mg.MovingGridBatch.N_CONFIGS == n


def test_noalloc_entry_rejects_bad_arguments_before_device_work(lib):
    """mg_propagate_noalloc validates its arguments on the host: a missing buffer, an
    odd axis or a bad dt return MG_EINVAL with a message, before any HIP call."""
    from paper_1909_06412_amd import _lib
    N = np.asarray([8], dtype=np.int32)
    one = np.ones(1)
    q, p = np.zeros(1), np.zeros(1)
    st = lib.mg_propagate_noalloc(1, N.ctypes.data_as(_lib._ip), _lib.dptr(one), _lib.dptr(one), 1.0, 0, 0,
                                  None, 0, 0, 0, 2, None, 0, None, _lib.dptr(q), _lib.dptr(p), 0.1, 1, None)
    assert st == _lib.MG_EINVAL
    assert b"bad argument" in lib.mg_last_error(None)
    st = lib.mg_propagate_noalloc(1, N.ctypes.data_as(_lib._ip), _lib.dptr(one), _lib.dptr(one), 1.0, 0, 0,
                                  None, 0, 0, 0, 2, None, 0, ctypes.c_void_p(256), _lib.dptr(q), _lib.dptr(p),
                                  float("nan"), 1, None)
    assert st == _lib.MG_EINVAL
    hdr = open(HEADER).read()
    assert int(re.search(r"#define MG_NOALLOC_SCRATCH_BYTES \(1u << (\d+)\)", hdr).group(1)) == 20


def test_binding_refuses_a_library_built_from_other_sources(monkeypatch):
    """The library embeds the sha256 of its sources and flags; lib() compares it with
    the sources beside it, so a stale build cannot be tested or measured silently."""
    from paper_1909_06412_amd import _lib, build
    L = _lib.lib()
    assert L.mg_build_hash().decode() == build.source_hash()
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(build, "source_hash", lambda: "0" * 64)
    with pytest.raises(ImportError, match="other sources"):
        _lib.lib()
