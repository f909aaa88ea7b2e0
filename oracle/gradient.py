"""Objective and finite-difference gradients for the adjoint check (test
infrastructure only).  The oracle has no adjoint: its gradient of a final
observable with respect to potential parameters is a central finite difference of
whole FP64 propagations.

Objective (a "transmitted probability" past a dividing line on the final grid):
    J = sum_J W(q^J) |psi(q^J)|^2 prod_l dq_l,   W = 1 / (1 + exp(-(R_d - R)/w)),
with R = rho - c r for the atom-diatom coordinates q = (r, rho), or R = q for a
single coordinate.
"""
from __future__ import annotations

import numpy as np

from . import potentials, propagate


def window(qs, R_d, w, c=0.5):
    if len(qs) == 1:
        R = qs[0]
    else:
        r, rho = qs
        R = rho - c * r
    return 1.0 / (1.0 + np.exp(-(R_d - R) / w))


def transmitted(wp, R_d, w, c=0.5) -> float:
    g = wp.grid
    W = window(g.q_mesh(wp.q_ctr), R_d, w, c)
    return float(np.prod(g.dq) * np.sum(W * np.abs(wp.physical()) ** 2))


def run_objective(workload: dict, params: dict, nsteps: int, R_d: float, w: float) -> float:
    """Propagate the workload's initial Gaussian with the given potential parameters
    and return J at the end."""
    grid = propagate.Grid(workload["N"], workload["dq"], workload["hbar"])
    kind, _ = workload["potential"]
    pot = potentials.from_spec(kind, params, workload["D"])
    wp = propagate.gaussian(grid, workload["q0"], workload["p0"], workload["sigma"])
    gam = propagate.composition(workload["comp"], workload["order"])
    propagate.propagate(wp, workload["dt"], nsteps, gam, pot, workload["inv_mass"],
                        workload["split"])
    return transmitted(wp, R_d, w, params.get("c", 0.5))


def fd_gradient(workload: dict, names, nsteps: int, R_d: float, w: float, rel=1e-4):
    """Central differences of J with respect to the named potential parameters.  A name
    is a scalar parameter ("A") or an entry of an array parameter (("k", 0))."""
    _, base = workload["potential"]
    out = []
    for nm in names:
        key, idx = (nm, None) if isinstance(nm, str) else nm
        value = base[key] if idx is None else base[key][idx]
        hstep = rel * max(abs(value), 1.0)
        moved = []
        for sign in (1.0, -1.0):
            par = dict(base)
            if idx is None:
                par[key] = value + sign * hstep
            else:
                arr = list(base[key])
                arr[idx] = value + sign * hstep
                par[key] = arr
            moved.append(run_objective(workload, par, nsteps, R_d, w))
        out.append((moved[0] - moved[1]) / (2 * hstep))
    return np.array(out)
