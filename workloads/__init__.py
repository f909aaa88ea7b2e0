"""Seeded synthetic inputs for the moving-grid split-operator workloads.

This module only *describes* inputs: grid shapes and spacings, model parameters,
initial-Gaussian parameters drawn from seeded generators, and random test states.
It holds none of the propagation arithmetic.  The HIP path and the CPU oracle both
take their inputs from here and from nowhere else they share.

Every workload is a plain dict with the keys

    name, D, N (list[int]), dq (list[float]), inv_mass (list[float]), hbar,
    potential = (kind, params)   kind in {"free", "harmonic", "quadratic",
                                           "morse_repulsion", "henon_heiles"}
    q0, p0, sigma                 initial Gaussian (paper's form, Sec. III.B):
                                  prod_l (pi sigma_l^2)^(-1/4)
                                  exp[-(q_l-q0_l)^2/(2 sigma_l^2) + i p0_l (q_l-q0_l)/hbar]
    dt, steps, split ("TVT" | "VTV"), comp ("strang" | "suzuki" | "triple_jump"),
    order, precision ("c128" | "c64")

The initial grid centres are (q0, p0): the expectation values of the analytic state.

Potential parameter conventions (shared vocabulary, no arithmetic here):
    free              {}
    harmonic          {"k": [D], "s": [D]}          V = 1/2 sum_l k_l (q_l - s_l)^2
    quadratic         {"K": [D][D], "s": [D]}       V = 1/2 (q - s)^T K (q - s)
    morse_repulsion   {"De","a","re","A","b","c"}   (D = 2, q = (r, rho))
                      V = De (1 - exp(-a (r - re)))^2 + A exp(-b (rho - c r))
    henon_heiles      {"kappa","lam"}               Sec. III.C
"""
from __future__ import annotations

import copy
import math

import numpy as np

__all__ = [
    "harmonic_1d", "harmonic_3d", "harmonic_3d_seeds", "morse_repulsion_2d",
    "henon_heiles_8d", "morse_batch", "duschinsky_3d", "secrest_johnson_2d",
    "random_state", "scaled", "C5_LENGTHS",
]


# --------------------------------------------------------------------------
# Config 1: 1-D harmonic oscillator, 64 points spanning 16 about q0 = 1.
# --------------------------------------------------------------------------
def harmonic_1d() -> dict:
    return dict(
        name="harmonic_1d_64", D=1, N=[64], dq=[16.0 / 64], inv_mass=[1.0], hbar=1.0,
        potential=("harmonic", {"k": [1.0], "s": [0.0]}),
        q0=[1.0], p0=[0.0], sigma=[1.0],
        dt=0.01, steps=1000, split="TVT", comp="strang", order=2, precision="c128",
    )


# --------------------------------------------------------------------------
# Config 2: 3-D harmonic model, omega = (1, 1.2, 1.5), 32^3 moving grid,
# (q0, p0) ~ U[-2, 2]^3 from numpy's default_rng(seed).
# --------------------------------------------------------------------------
HARMONIC_3D_OMEGA = (1.0, 1.2, 1.5)
HARMONIC_3D_DTS = (0.1, 0.05, 0.02, 0.01, 0.005, 0.002, 0.001)
HARMONIC_3D_ORDERS = (2, 4, 6, 8, 10)


def harmonic_3d(seed: int = 0, n: int = 32, dq: float = 0.4375, order: int = 4,
                dt: float = 0.01, t_final: float = 5.0, precision: str = "c128") -> dict:
    rng = np.random.default_rng(seed)
    q0 = rng.uniform(-2.0, 2.0, 3)
    p0 = rng.uniform(-2.0, 2.0, 3)
    comp = "strang" if order == 2 else ("suzuki" if order == 4 else "triple_jump")
    return dict(
        name=f"harmonic_3d_{n}^3_seed{seed}", D=3, N=[n] * 3, dq=[dq] * 3,
        inv_mass=[1.0] * 3, hbar=1.0,
        potential=("harmonic", {"k": [w * w for w in HARMONIC_3D_OMEGA], "s": [0.0] * 3}),
        q0=q0.tolist(), p0=p0.tolist(), sigma=[1.0] * 3,
        dt=dt, steps=int(round(t_final / dt)), split="TVT", comp=comp, order=order,
        precision=precision,
    )


def harmonic_3d_seeds(seeds=(0, 1, 2, 3, 4), **kw) -> list:
    return [harmonic_3d(seed=s, **kw) for s in seeds]


# --------------------------------------------------------------------------
# Config 3: collinear atom-diatom model in Jacobi coordinates (r, rho), atomic
# units.  Morse diatom (De = 0.17, a = 1.0, re = 1.4) plus the repulsion
# A exp(-b R) on the nearest-atom distance R = rho - r/2 (A = 10, b = 2).
# Reduced masses 918 (diatom) and 1836 (atom-diatom): the 2:1 mass ratio.
# Initial state: harmonic ground state of the Morse well in r
# (sigma_r = (mu_r omega_M)^(-1/2), omega_M = a sqrt(2 De / mu_r)) times an
# incoming Gaussian in rho (sigma 0.4, rho0 = 7.5, p0 = -19.2: about 0.1 Eh of
# collision energy).  Spans 9.6 in r and 16 in rho.
# --------------------------------------------------------------------------
MORSE_REP = {"De": 0.17, "a": 1.0, "re": 1.4, "A": 10.0, "b": 2.0, "c": 0.5}
MORSE_MU = (918.0, 1836.0)
MORSE_SPAN = (9.6, 16.0)


def _morse_sigma_r() -> float:
    omega_m = MORSE_REP["a"] * math.sqrt(2.0 * MORSE_REP["De"] / MORSE_MU[0])
    return 1.0 / math.sqrt(MORSE_MU[0] * omega_m)


def morse_repulsion_2d(n1: int = 256, n2: int = 256, p0_rho: float = -19.2,
                       steps: int = 20000, precision: str = "c64") -> dict:
    return dict(
        name=f"morse_repulsion_{n1}x{n2}", D=2, N=[n1, n2],
        dq=[MORSE_SPAN[0] / n1, MORSE_SPAN[1] / n2],
        inv_mass=[1.0 / MORSE_MU[0], 1.0 / MORSE_MU[1]], hbar=1.0,
        potential=("morse_repulsion", dict(MORSE_REP)),
        q0=[MORSE_REP["re"], 7.5], p0=[0.0, p0_rho], sigma=[_morse_sigma_r(), 0.4],
        dt=0.05, steps=steps, split="TVT", comp="strang", order=2, precision=precision,
    )


# --------------------------------------------------------------------------
# Config 4: 8-D Henon-Heiles (Sec. III.C): kappa = 1, lambda = 0.111803, unit
# masses, Gaussian displaced by 2 in every coordinate, 16^8 grid with spacing
# 0.625 (span 10 per axis), 4th-order Suzuki composition.
# --------------------------------------------------------------------------
def henon_heiles_8d(n: int = 16, D: int = 8, dq: float = 0.625, lam: float = 0.111803,
                    steps: int = 5000, precision: str = "c64") -> dict:
    return dict(
        name=f"henon_heiles_{D}d_{n}^{D}", D=D, N=[n] * D, dq=[dq] * D,
        inv_mass=[1.0] * D, hbar=1.0,
        potential=("henon_heiles", {"kappa": 1.0, "lam": lam}),
        q0=[2.0] * D, p0=[0.0] * D, sigma=[1.0] * D,
        dt=0.01, steps=steps, split="TVT", comp="suzuki", order=4, precision=precision,
    )


# --------------------------------------------------------------------------
# Config 5: 256 independent Morse+repulsion packets.  Per-packet axis lengths
# are drawn from the 15 even 5-smooth lengths below with default_rng(0); the
# physical spans are those of config 3, so spacings vary per packet.  The
# incoming momenta are drawn next from the same generator, U[-27.1, -13.55]
# (0.05 to 0.2 Eh of collision energy).
# --------------------------------------------------------------------------
C5_LENGTHS = (64, 72, 80, 90, 96, 100, 108, 120, 128, 144, 150, 160, 162, 180, 192)
C5_WINDOW = {"R_d": 2.5, "w": 0.1}


def morse_batch(B: int = 256, seed: int = 0, steps: int = 10000, precision: str = "c64",
                lengths=C5_LENGTHS) -> list:
    rng = np.random.default_rng(seed)
    shapes = rng.choice(np.asarray(lengths), (B, 2))
    p0s = rng.uniform(-27.1, -13.55, B)
    out = []
    for b in range(B):
        w = morse_repulsion_2d(int(shapes[b, 0]), int(shapes[b, 1]), float(p0s[b]),
                               steps=steps, precision=precision)
        w["name"] = f"morse_batch[{b}]"
        out.append(w)
    return out


# --------------------------------------------------------------------------
# The paper's own model parameterisations (Sec. III.A, Table I; Sec. III.B).
# --------------------------------------------------------------------------
def duschinsky_3d(k13: float = 0.017, n: int = 32, dq: float = 0.4375) -> dict:
    """Table I.  The printed K13 is -0.017; the printed E0 = 140.389 is
    reproduced with +0.017, which is the default here (documented reading)."""
    omega = [2.0, 1.0, 2.5]
    K = [[1.997, -0.04, k13], [-0.04, 1.015, 0.04], [k13, 0.04, 2.48]]
    return dict(
        name="duschinsky_3d", D=3, N=[n] * 3, dq=[dq] * 3,
        inv_mass=omega, hbar=1.0,                        # T = sum omega_l p_l^2 / 2
        potential=("quadratic", {"K": K, "s": [-7.0, 7.0, 7.0]}),
        q0=[0.0] * 3, p0=[0.0] * 3, sigma=[1.0] * 3,     # ground state of H_g, hbar = 1
        dt=50.0 / 2 ** 9, steps=2 ** 9, split="TVT", comp="triple_jump", order=10,
        precision="c128",
    )


def secrest_johnson_2d(n1: int = 128, n2: int = 128, p0: float = -3.56) -> dict:
    """Sec. III.B: V = D (1 - exp(-beta q1))^2 + exp(-alpha (q2 - q1)),
    beta = 0.158, D = 20, alpha = 0.3, m = (1, 2/3); initial q1 range (-14, 14),
    q2 range (0, 48); sigma0^2 = 8, q0 = 24."""
    return dict(
        name="secrest_johnson_2d", D=2, N=[n1, n2], dq=[28.0 / n1, 48.0 / n2],
        inv_mass=[1.0, 1.5], hbar=1.0,
        potential=("morse_repulsion", {"De": 20.0, "a": 0.158, "re": 0.0, "A": 1.0,
                                       "b": 0.3, "c": 1.0}),
        q0=[0.0, 24.0], p0=[0.0, p0], sigma=[1.0, math.sqrt(8.0)],
        dt=0.1, steps=100, split="VTV", comp="triple_jump", order=10, precision="c128",
    )


# --------------------------------------------------------------------------
# Generic seeded test inputs.
# --------------------------------------------------------------------------
def random_state(shape, seed: int = 0) -> np.ndarray:
    """Smooth-enveloped random complex field (physical psi values), not normalised."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(tuple(shape)) + 1j * rng.standard_normal(tuple(shape))
    env = np.ones(tuple(shape))
    for ax, n in enumerate(shape):
        x = (np.arange(n) - n / 2) / max(n / 4, 1)
        sh = [1] * len(shape)
        sh[ax] = n
        env = env * np.exp(-0.5 * x ** 2).reshape(sh)
    return z * env


def scaled(w: dict, **over) -> dict:
    """Copy of a workload with some fields replaced."""
    out = copy.deepcopy(w)
    out.update(over)
    return out
