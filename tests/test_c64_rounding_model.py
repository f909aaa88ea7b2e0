"""A float32 model of the complex64 path's roots of unity (CPU only).

Norm preservation (Sec. II.G) is what keeps the moving grid's norm at one; in
complex64 every DFT can only keep it up to rounding.  This test models the 16-point
DFT of the register kernels (4 x 4 decomposition, twiddles W16^(n2 k1)) and the
256-point transform of the Stockham passes in float32 arithmetic with numpy
(explicit rounding after every operation, FMAs rounded once), on random unit inputs
and on smooth packets, and compares two ways of applying the twiddles:

* rounded: each constant (cos, sin) rounded to float32 on its own.  Every such root
  has c^2 + s^2 - 1 of a few 1e-8 with the same sign for the 16-point constants, so
  the DFT loses about 2.3e-8 of the norm per transform on average;
* compensated: each constant carried as hi + lo float32 pair and multiplied with
  FMAs (what the kernels do for complex64), which acts as the exact root to FP64
  accuracy: no systematic loss, only unbiased rounding noise.

It pins the mechanism and the size of the bias that the compensated constants
remove; the GPU tests measure the kernels themselves.
"""
import math

import numpy as np

F32 = np.float32


def _r(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def _d(x):
    return x.astype(np.float64)


def _dft4(v):
    a0 = (_r(_d(v[0][0]) + v[2][0]), _r(_d(v[0][1]) + v[2][1]))
    a1 = (_r(_d(v[0][0]) - v[2][0]), _r(_d(v[0][1]) - v[2][1]))
    b0 = (_r(_d(v[1][0]) + v[3][0]), _r(_d(v[1][1]) + v[3][1]))
    b1 = (_r(_d(v[1][0]) - v[3][0]), _r(_d(v[1][1]) - v[3][1]))
    rb = (b1[1], -b1[0])                                    # -i b1 (forward)
    add = lambda p, q: (_r(_d(p[0]) + q[0]), _r(_d(p[1]) + q[1]))
    sub = lambda p, q: (_r(_d(p[0]) - q[0]), _r(_d(p[1]) - q[1]))
    return [add(a0, b0), add(a1, rb), sub(a0, b0), sub(a1, rb)]


def _rotate(v, c, s, compensated):
    """v * (c + i s) in float32: one product rounded, then an FMA (rounded); or with
    hi + lo constants, the lo products folded in before the two FMAs."""
    x, y = _d(v[0]), _d(v[1])
    ch, sh = float(F32(c)), float(F32(s))
    if not compensated:
        return (_r(x * ch - _d(_r(y * sh))), _r(y * ch + _d(_r(x * sh))))
    cl, sl = float(F32(c - ch)), float(F32(s - sh))
    tr = _r(-y * sl + _d(_r(x * cl)))
    ti = _r(y * cl + _d(_r(x * sl)))
    return (_r(x * ch + _d(_r(-y * sh + _d(tr)))), _r(y * ch + _d(_r(x * sh + _d(ti)))))


def _dft16(x, compensated):
    y = [None] * 16
    for n2 in range(4):
        v = _dft4([x[n2], x[4 + n2], x[8 + n2], x[12 + n2]])
        for k1 in range(4):
            y[4 * n2 + k1] = v[k1]
    for n2 in range(1, 4):
        for k1 in range(1, 4):
            m = n2 * k1
            if m == 4:
                y[4 * n2 + k1] = (y[4 * n2 + k1][1], -y[4 * n2 + k1][0])
            else:
                ang = -math.pi * m / 8
                y[4 * n2 + k1] = _rotate(y[4 * n2 + k1], math.cos(ang), math.sin(ang), compensated)
    out = [None] * 16
    for k1 in range(4):
        v = _dft4([y[k1], y[4 + k1], y[8 + k1], y[12 + k1]])
        for k2 in range(4):
            out[k1 + 4 * k2] = v[k2]
    return out


def _split(z):
    return [(z[i].real.astype(np.float32), z[i].imag.astype(np.float32)) for i in range(z.shape[0])]


def _join(v):
    return np.array([_d(a) + 1j * _d(b) for a, b in v])


def _norm_change_16(z, compensated):
    x = _split(z)
    X = _join(_dft16(x, compensated))
    xin = _join(x)
    ratio = np.sum(np.abs(X) ** 2, axis=0) / 16 / np.sum(np.abs(xin) ** 2, axis=0) - 1
    err = np.max(np.abs(X - np.fft.fft(xin, axis=0))) / np.max(np.abs(X))
    return ratio, err


def test_sixteen_point_dft_norm_bias():
    rng = np.random.default_rng(0)
    M = 40000
    z = rng.standard_normal((16, M)) + 1j * rng.standard_normal((16, M))
    plain, e1 = _norm_change_16(z, False)
    comp, e2 = _norm_change_16(z, True)
    sem = np.std(comp) / math.sqrt(M)
    # rounded constants: 4/16 of the energy meets (c1, s1), 4/16 meets sqrt(1/2)
    c1, s1, r2 = F32(math.cos(math.pi / 8)), F32(math.sin(math.pi / 8)), F32(math.sqrt(0.5))
    predicted = 0.25 * (float(c1) ** 2 + float(s1) ** 2 - 1) + 0.25 * (2 * float(r2) ** 2 - 1)
    assert abs(np.mean(plain) - predicted) < 0.1 * abs(predicted)       # -2.3e-8
    assert abs(np.mean(comp)) < 4 * sem + 2e-10                          # no bias
    assert e1 < 3e-7 and e2 < 3e-7                                       # both are DFTs


def _fft256(z, compensated):
    """256 = 16 x 16: DFT16 over n1 (n = 16 n1 + n2), twiddles W256^(n2 k1) from a
    table (rounded per entry, or hi + lo), DFT16 over n2; X[k1 + 16 k2]."""
    M = z.shape[1]
    a = z.reshape(16, 16, M)
    y = np.empty((16, 16, M), dtype=np.complex128)
    for n2 in range(16):
        o = _join(_dft16(_split(a[:, n2, :]), True))
        y[:, n2, :] = o
    for k1 in range(1, 16):
        for n2 in range(1, 16):
            ang = -2 * math.pi * ((n2 * k1) % 256) / 256
            v = (y[k1, n2].real.astype(np.float32), y[k1, n2].imag.astype(np.float32))
            o = _rotate(v, math.cos(ang), math.sin(ang), compensated)
            y[k1, n2] = _d(o[0]) + 1j * _d(o[1])
    out = np.empty((16, 16, M), dtype=np.complex128)
    for k1 in range(16):
        out[k1] = _join(_dft16(_split(y[k1]), True))
    return out.transpose(1, 0, 2).reshape(256, M)


def test_table_twiddles_norm_bias_on_smooth_packets():
    """Smooth packets (Gaussians 4-8 points wide near the grid centre, the shape every
    workload has): rounded table entries leave a systematic loss of several 1e-9 per
    256-point transform, hi + lo entries none beyond the noise."""
    rng = np.random.default_rng(1)
    j = np.arange(256)
    cols = []
    for _ in range(48):
        ctr, sig, k = 128 + rng.uniform(-3, 3), rng.uniform(4, 8), rng.uniform(-0.3, 0.3)
        cols.append(np.exp(-(j - ctr) ** 2 / (2 * sig ** 2) + 1j * k * (j - ctr)))
    z = np.array(cols).T.astype(np.complex64).astype(np.complex128)
    n0 = np.sum(np.abs(z) ** 2, axis=0)
    plain = np.sum(np.abs(_fft256(z, False)) ** 2, axis=0) / 256 / n0 - 1
    comp = np.sum(np.abs(_fft256(z, True)) ** 2, axis=0) / 256 / n0 - 1
    assert np.mean(plain) < -3e-9
    assert abs(np.mean(comp)) < 3 * np.std(comp) / math.sqrt(len(comp)) + 1e-10
