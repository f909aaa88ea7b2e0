"""Moving-grid split-operator propagation on MI355X (gfx950).

Time-reversible adaptive-grid integrator of Choi & Vanicek (arXiv:1909.06412):
split-operator steps of the dynamic Fourier method on a tensor-product grid whose
centres follow the Ehrenfest moments <p> and <dV/dq> within each kinetic and
potential substep, composed symmetrically to orders 2-10.

All arithmetic runs in libmgso.so (hand-written HIP kernels); this package only
marshals arguments.  PyTorch, when present, provides device memory and the stream.
"""
from __future__ import annotations

import numpy as np

from . import _lib as L
from ._lib import (MgError, MG_C128, MG_C64, MG_POT_FREE, MG_POT_HARMONIC,  # noqa: F401
                   MG_POT_MORSE_REP, MG_POT_HENON_HEILES, MG_POT_QUADRATIC, MG_TVT, MG_VTV,
                   MG_COMP_STRANG, MG_COMP_SUZUKI, MG_COMP_TRIPLE_JUMP, MG_COMP_USER,
                   MG_OPT_ENGINE, MG_OPT_GRAPH, MG_OPT_PROFILE, MG_OPT_RENORMALIZE, MG_OPT_GRID, MG_EUNSTABLE,
                   MG_EINVAL, MG_ESTATE)

_POT = {"free": MG_POT_FREE, "harmonic": MG_POT_HARMONIC, "morse_repulsion": MG_POT_MORSE_REP,
        "henon_heiles": MG_POT_HENON_HEILES, "quadratic": MG_POT_QUADRATIC}
_COMP = {"strang": MG_COMP_STRANG, "suzuki": MG_COMP_SUZUKI, "triple_jump": MG_COMP_TRIPLE_JUMP,
         "user": MG_COMP_USER}
_SPLIT = {"TVT": MG_TVT, "VTV": MG_VTV}
_PREC = {"c128": MG_C128, "c64": MG_C64}


def potential_params(kind: str, params: dict, D: int) -> np.ndarray:
    """Flatten a (kind, params) spec into the mg_set_potential parameter list."""
    if kind == "free":
        return np.zeros(0)
    if kind == "harmonic":
        s = params.get("s", [0.0] * D)
        return np.concatenate([np.asarray(params["k"], float), np.asarray(s, float)])
    if kind == "quadratic":
        return np.concatenate([np.asarray(params["K"], float).reshape(-1),
                               np.asarray(params["s"], float)])
    if kind == "morse_repulsion":
        return np.array([params["De"], params["a"], params["re"], params["A"], params["b"],
                         params.get("c", 0.5)], float)
    if kind == "henon_heiles":
        return np.array([params["kappa"], params["lam"]], float)
    raise ValueError(kind)


def _torch_stream_and_alloc():
    try:
        import torch
    except ImportError:
        return None, None
    if not torch.cuda.is_available():
        return None, None
    return torch.cuda.current_stream().cuda_stream, torch


class MovingGrid:
    """One wavepacket on a moving grid (wraps an mg_ctx)."""

    def __init__(self, N, dq, inv_mass, hbar=1.0, precision="c128", use_torch=True):
        self.D = len(N)
        self.N = [int(n) for n in N]
        self.dq = [float(x) for x in np.asarray(dq, dtype=np.float64).reshape(-1)]
        self.precision = precision
        lib = L.lib()
        stream, torch = _torch_stream_and_alloc() if use_torch else (None, None)
        h = L.C.c_void_p()
        Narr = np.ascontiguousarray(np.asarray(self.N, dtype=np.int32))
        st = lib.mg_create(self.D, Narr.ctypes.data_as(L._ip), L.dptr(L.f64(dq, self.D)),
                           L.dptr(L.f64(inv_mass, self.D)), float(hbar), _PREC[precision],
                           stream, L.C.byref(h))
        if st != 0:
            raise L.MgError(st, "mg_create: " + (lib.mg_last_error(None) or b"").decode())
        self.h = h
        self._bufs = []
        if torch is not None:
            # the state lives in a torch allocation; the out-of-place workspace (only
            # observables and the naive grid mode use it, the step does not) is left
            # to the library, which allocates it on first use
            nb = lib.mg_state_bytes(h)
            psi = torch.empty(nb, dtype=torch.uint8, device="cuda")
            self._bufs = [psi]
            L.check(lib.mg_bind_buffers(h, psi.data_ptr(), None), h)

    def close(self):
        if getattr(self, "h", None):
            L.lib().mg_destroy(self.h)
            self.h = None
            self._bufs = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- state -----------------------------------------------------------
    def set_gaussian(self, q0, p0, sigma):
        D = self.D
        L.check(L.lib().mg_set_gaussian(self.h, L.dptr(L.f64(q0, D)), L.dptr(L.f64(p0, D)),
                                        L.dptr(L.f64(sigma, D))), self.h)

    def set_state(self, psi_phys, q_ctr, p_ctr, t=0.0):
        a = np.ascontiguousarray(np.asarray(psi_phys, dtype=np.complex128).reshape(self.N))
        v = a.view(np.float64).reshape(-1)
        L.check(L.lib().mg_set_state(self.h, L.dptr(v), L.dptr(L.f64(q_ctr, self.D)),
                                     L.dptr(L.f64(p_ctr, self.D)), float(t)), self.h)

    def get_state(self):
        psi = np.empty(self.N, dtype=np.complex128)
        q = np.empty(self.D)
        p = np.empty(self.D)
        t = np.empty(1)
        L.check(L.lib().mg_get_state(self.h, L.dptr(psi.view(np.float64).reshape(-1)), L.dptr(q),
                                     L.dptr(p), L.dptr(t)), self.h)
        return psi, q, p, float(t[0])

    def centres(self):
        """(q_ctr, p_ctr, t) without copying the state."""
        q = np.empty(self.D)
        p = np.empty(self.D)
        t = np.empty(1)
        L.check(L.lib().mg_get_state(self.h, None, L.dptr(q), L.dptr(p), L.dptr(t)), self.h)
        return q, p, float(t[0])

    def state_view(self):
        """The bound device state as a flat torch complex tensor of N_total elements
        (row-major, axis 0 outermost), holding psi(q) * sqrt(prod dq); None without
        torch buffers.  A view, not a copy: read it between steps only."""
        if not self._bufs:
            return None
        import torch
        n = int(np.prod(self.N))
        dt = torch.complex64 if self.precision == "c64" else torch.complex128
        return self._bufs[0].view(dt)[:n]

    # --- model -----------------------------------------------------------
    def set_potential(self, kind, params):
        pr = potential_params(kind, params, self.D)
        self.set_potential_flat(kind, pr)

    def set_potential_flat(self, kind, flat):
        """mg_set_potential with the flat parameter list (see potential_params)."""
        pr = L.f64(flat)
        L.check(L.lib().mg_set_potential(self.h, _POT[kind], L.dptr(pr) if pr.size else None,
                                         int(pr.size)), self.h)
        self.potential = (kind, pr.copy())

    def set_scheme(self, split="TVT", comp="strang", order=2, gammas=None):
        g = None if gammas is None else L.f64(gammas)
        L.check(L.lib().mg_set_scheme(self.h, _SPLIT[split], _COMP[comp], int(order),
                                      L.dptr(g), 0 if g is None else int(g.size)), self.h)

    def set_option(self, option, value):
        L.check(L.lib().mg_set_option(self.h, int(option), int(value)), self.h)

    # --- propagation -----------------------------------------------------
    def step(self, dt, nsteps=1):
        L.check(L.lib().mg_step(self.h, float(dt), int(nsteps)), self.h)

    def observables(self):
        D = self.D
        out = np.empty(4 + 4 * D)
        L.check(L.lib().mg_observables(self.h, L.dptr(out)), self.h)
        return dict(norm=out[0], q=out[1:1 + D].copy(), p=out[1 + D:1 + 2 * D].copy(),
                    q_ctr=out[1 + 2 * D:1 + 3 * D].copy(), p_ctr=out[1 + 3 * D:1 + 4 * D].copy(),
                    Ekin=out[1 + 4 * D], Epot=out[2 + 4 * D], E=out[1 + 4 * D] + out[2 + 4 * D],
                    t=out[3 + 4 * D])

    def regrid(self, new_q_ctr):
        L.check(L.lib().mg_regrid(self.h, L.dptr(L.f64(new_q_ctr, self.D))), self.h)

    def profile_read(self, reset=True):
        n = L.C.c_int64()
        ms = L.C.c_double()
        by = L.C.c_double()
        L.check(L.lib().mg_profile_read(self.h, L.C.byref(n), L.C.byref(ms), L.C.byref(by),
                                        int(reset)), self.h)
        return n.value, ms.value, by.value

    def autocorrelation(self, q0, p0, sigma):
        """<psi_0|psi_t> with psi_0 the Gaussian (q0, p0, sigma) on the current grid."""
        out = np.zeros(2)
        L.check(L.lib().mg_autocorrelation(self.h, L.dptr(L.f64(q0, self.D)), L.dptr(L.f64(p0, self.D)),
                                           L.dptr(L.f64(sigma, self.D)), L.dptr(out)), self.h)
        return complex(out[0], out[1])

    def profile_class(self):
        """(sweep, dir, epi, group_axes, mode) of the kernel class profile_read reports."""
        v = [L.C.c_int() for _ in range(5)]
        L.check(L.lib().mg_profile_class(self.h, *[L.C.byref(x) for x in v]), self.h)
        return tuple(x.value for x in v)

    def adjoint(self, dt, nsteps, K, window, param_ids):
        ids = np.ascontiguousarray(np.asarray(param_ids, dtype=np.int32))
        J = np.empty(1)
        g = np.empty(len(ids))
        L.check(L.lib().mg_adjoint(self.h, float(dt), int(nsteps), int(K), L.dptr(L.f64(window, 2)),
                                   ids.ctypes.data_as(L._ip), int(ids.size), L.dptr(J), L.dptr(g)),
                self.h)
        return float(J[0]), g


def from_workload(w: dict, precision=None, use_torch=True) -> MovingGrid:
    """Create, initialise and configure a MovingGrid from a workloads-module dict."""
    mg = MovingGrid(w["N"], w["dq"], w["inv_mass"], w["hbar"], precision or w["precision"],
                    use_torch=use_torch)
    kind, par = w["potential"]
    mg.set_potential(kind, par)
    mg.set_scheme(w["split"], w["comp"], w["order"])
    mg.set_gaussian(w["q0"], w["p0"], w["sigma"])
    return mg


def propagate_noalloc(psi_dev_ptr, N, dq, inv_mass, hbar, precision, potential, scheme, q_ctr, p_ctr,
                      dt, nsteps, stream=None):
    """mg_propagate_noalloc: nsteps of dt on the caller's device buffer (address
    psi_dev_ptr, holding psi(q^J) sqrt(prod dq) in `precision`) without any device
    allocation.  potential = (kind, params dict); scheme = (split, comp, order,
    gammas or None).  Returns the new (q_ctr, p_ctr)."""
    D = len(N)
    kind, par = potential
    pr = potential_params(kind, par, D)
    split, comp, order, gammas = scheme
    g = None if gammas is None else L.f64(gammas)
    Narr = np.ascontiguousarray(np.asarray(N, dtype=np.int32))
    q = L.f64(q_ctr, D).copy()
    p = L.f64(p_ctr, D).copy()
    if stream is None:
        stream, _ = _torch_stream_and_alloc()
    st = L.lib().mg_propagate_noalloc(D, Narr.ctypes.data_as(L._ip), L.dptr(L.f64(dq, D)),
                                      L.dptr(L.f64(inv_mass, D)), float(hbar), _PREC[precision], _POT[kind],
                                      L.dptr(pr) if pr.size else None, int(pr.size), _SPLIT[split],
                                      _COMP[comp], int(order), L.dptr(g), 0 if g is None else int(g.size),
                                      L.C.c_void_p(int(psi_dev_ptr)), L.dptr(q), L.dptr(p), float(dt),
                                      int(nsteps), stream)
    if st != 0:
        raise L.MgError(st, (L.lib().mg_last_error(None) or b"").decode())
    return q, p


class MovingGridBatch:
    """Many independent wavepackets with their own grids, propagated by one
    persistent kernel launch per mg_batch_step (wraps an mg_batch)."""

    def __init__(self, shapes, dqs, inv_mass, hbar=1.0, precision="c64"):
        shapes = [list(map(int, s)) for s in shapes]
        self.B = len(shapes)
        self.D = len(shapes[0])
        self.shapes = shapes
        self.precision = precision
        lib = L.lib()
        stream, _ = _torch_stream_and_alloc()
        Narr = np.ascontiguousarray(np.asarray(shapes, dtype=np.int32).reshape(-1))
        dq = L.f64(np.asarray(dqs, dtype=float).reshape(-1), self.B * self.D)
        h = L.C.c_void_p()
        st = lib.mg_batch_create(self.B, self.D, Narr.ctypes.data_as(L._ip), L.dptr(dq),
                                 L.dptr(L.f64(inv_mass, self.D)), float(hbar), _PREC[precision],
                                 stream, L.C.byref(h))
        if st != 0:
            raise L.MgError(st, "mg_batch_create: " + (lib.mg_last_error(None) or b"").decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            L.lib().mg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def points(self):
        return int(L.lib().mg_batch_points(self.h))

    def set_gaussian(self, q0, p0, sigma):
        n = self.B * self.D
        L.check(L.lib().mg_batch_set_gaussian(self.h, L.dptr(L.f64(q0, n)), L.dptr(L.f64(p0, n)),
                                              L.dptr(L.f64(sigma, n))), self.h)

    def set_potential(self, kind, params):
        pr = potential_params(kind, params, self.D)
        self.set_potential_flat(kind, pr)

    def set_potential_flat(self, kind, flat):
        """mg_batch_set_potential with the flat parameter list (see potential_params)."""
        pr = L.f64(flat)
        L.check(L.lib().mg_batch_set_potential(self.h, _POT[kind], L.dptr(pr) if pr.size else None,
                                               int(pr.size)), self.h)
        self.potential = (kind, pr.copy())

    def set_scheme(self, split="TVT", comp="strang", order=2, gammas=None):
        g = None if gammas is None else L.f64(gammas)
        L.check(L.lib().mg_batch_set_scheme(self.h, _SPLIT[split], _COMP[comp], int(order), L.dptr(g),
                                            0 if g is None else int(g.size)), self.h)

    def set_option(self, option, value):
        L.check(L.lib().mg_batch_set_option(self.h, int(option), int(value)), self.h)

    N_CONFIGS = 6  # MG_BATCH_CONFIGS

    def config(self, index):
        """(threads per workgroup, tile points) of launch shape `index`."""
        th, tl = L.C.c_int32(), L.C.c_int32()
        L.check(L.lib().mg_batch_config(self.h, int(index), L.C.byref(th), L.C.byref(tl)), self.h)
        return th.value, tl.value

    def set_config(self, index):
        L.check(L.lib().mg_batch_set_config(self.h, int(index)), self.h)

    def autotune(self, dt, probe_steps=20):
        """Time every launch shape on the current state (restored afterwards) and keep
        the fastest: returns (chosen index, ms per step of each shape)."""
        ms = np.zeros(self.N_CONFIGS)
        ch = L.C.c_int32()
        L.check(L.lib().mg_batch_autotune(self.h, float(dt), int(probe_steps), L.dptr(ms), L.C.byref(ch)),
                self.h)
        return ch.value, ms

    def step(self, dt, nsteps=1):
        L.check(L.lib().mg_batch_step(self.h, float(dt), int(nsteps)), self.h)

    def observables(self):
        D = self.D
        out = np.empty(self.B * (4 + 4 * D))
        L.check(L.lib().mg_batch_observables(self.h, L.dptr(out)), self.h)
        out = out.reshape(self.B, 4 + 4 * D)
        return [dict(norm=o[0], q=o[1:1 + D].copy(), p=o[1 + D:1 + 2 * D].copy(),
                     q_ctr=o[1 + 2 * D:1 + 3 * D].copy(), p_ctr=o[1 + 3 * D:1 + 4 * D].copy(),
                     Ekin=o[1 + 4 * D], Epot=o[2 + 4 * D], E=o[1 + 4 * D] + o[2 + 4 * D], t=o[3 + 4 * D])
                for o in out]

    def get_state(self, idx):
        N = self.shapes[idx]
        psi = np.empty(N, dtype=np.complex128)
        q = np.empty(self.D)
        p = np.empty(self.D)
        t = np.empty(1)
        L.check(L.lib().mg_batch_get_state(self.h, int(idx), L.dptr(psi.view(np.float64).reshape(-1)),
                                           L.dptr(q), L.dptr(p), L.dptr(t)), self.h)
        return psi, q, p, float(t[0])

    def set_state(self, idx, psi_phys, q_ctr, p_ctr, t=0.0):
        a = np.ascontiguousarray(np.asarray(psi_phys, dtype=np.complex128).reshape(self.shapes[idx]))
        L.check(L.lib().mg_batch_set_state(self.h, int(idx), L.dptr(a.view(np.float64).reshape(-1)),
                                           L.dptr(L.f64(q_ctr, self.D)), L.dptr(L.f64(p_ctr, self.D)),
                                           float(t)), self.h)

    def adjoint(self, dt, nsteps, K, window, param_ids):
        ids = np.ascontiguousarray(np.asarray(param_ids, dtype=np.int32))
        J = np.empty(self.B)
        g = np.empty(self.B * len(ids))
        L.check(L.lib().mg_batch_adjoint(self.h, float(dt), int(nsteps), int(K), L.dptr(L.f64(window, 2)),
                                         ids.ctypes.data_as(L._ip), int(ids.size), L.dptr(J), L.dptr(g)),
                self.h)
        return J, g.reshape(self.B, len(ids))


def batch_from_workloads(ws, precision=None) -> MovingGridBatch:
    """A batch from a list of workloads-module dicts sharing D, masses, potential and scheme."""
    w0 = ws[0]
    b = MovingGridBatch([w["N"] for w in ws], [w["dq"] for w in ws], w0["inv_mass"], w0["hbar"],
                        precision or w0["precision"])
    kind, par = w0["potential"]
    b.set_potential(kind, par)
    b.set_scheme(w0["split"], w0["comp"], w0["order"])
    b.set_gaussian([w["q0"] for w in ws], [w["p0"] for w in ws], [w["sigma"] for w in ws])
    return b


def spectrum(times, acf, energies, t_damp=30.0, hbar=1.0):
    """Re int <psi_0|psi_t> exp(-(t/t_damp)^2) exp(i E t / hbar) dt (mg_spectrum)."""
    t = L.f64(times)
    a = np.ascontiguousarray(np.asarray(acf, dtype=np.complex128).reshape(-1)).view(np.float64)
    e = L.f64(energies)
    out = np.zeros(e.size)
    st = L.lib().mg_spectrum(L.dptr(t), L.dptr(a), int(t.size), L.dptr(e), int(e.size), float(t_damp),
                             float(hbar), L.dptr(out))
    if st != 0:
        raise MgError(st, "mg_spectrum: bad arguments")
    return out


# ---------------------------------------------------------------------------
# Autograd: the adjoint of a whole propagation as a differentiable function.
# ---------------------------------------------------------------------------
def _autograd_function():
    import torch

    class TransmittedProbability(torch.autograd.Function):
        """J(theta): the window objective of mg_adjoint after `nsteps` steps of `dt`,
        with the potential parameters `param_ids` (indices into the flat
        mg_set_potential list) set to theta.  The forward pass runs the library's
        adjoint (forward propagation with checkpoints every K steps, then the
        reverse sweep) and keeps dJ/dtheta for the backward pass.  For a batch, J
        has one entry per packet and the packets share theta."""

        @staticmethod
        def forward(ctx, theta, prop, dt, nsteps, K, window, param_ids):
            kind, flat = prop.potential
            flat = flat.copy()
            th = theta.detach().to("cpu", torch.float64).numpy()
            for i, pid in enumerate(param_ids):
                flat[pid] = th[i]
            prop.set_potential_flat(kind, flat)
            J, g = prop.adjoint(dt, nsteps, K, window, list(param_ids))
            ctx.save_for_backward(torch.as_tensor(np.asarray(g), dtype=torch.float64))
            ctx.theta_dtype, ctx.theta_device = theta.dtype, theta.device
            return torch.as_tensor(np.asarray(J), dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            (g,) = ctx.saved_tensors
            gth = (gJ.to(torch.float64).reshape(-1, 1) * g.reshape(gJ.numel(), -1)).sum(0)
            return gth.to(ctx.theta_dtype).to(ctx.theta_device), None, None, None, None, None, None

    return TransmittedProbability


_TP = None


def transmitted_probability(prop, theta, dt, nsteps, K, window, param_ids):
    """Differentiable J(theta) (torch): see TransmittedProbability.  `prop` is a
    MovingGrid or MovingGridBatch holding the initial state; the propagation stays
    applied, so set the initial state again before the next evaluation."""
    global _TP
    if _TP is None:
        _TP = _autograd_function()
    return _TP.apply(theta, prop, float(dt), int(nsteps), int(K), tuple(window), tuple(int(i) for i in param_ids))
