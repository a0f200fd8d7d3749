"""The error band behind the breaking screen of the single-precision tile
pass 1, checked on the CPU against exact integer arithmetic.

The kernel stages the fixed-point shadow of every box point relative to a
reference point, a = float(s - s_ref), and forms per bond the strain in
units of the shadow scale, e' = (M/x) . (a_j - a_i), in single precision
with the table entries M/x rounded to float.  Its screen and its finer test
rely on

    |e' x - M . (s_j - s_i)| <= 2^-21 D + 2^-24 A,

D = sum_c |a_jc - a_ic|, A = the sum of the |a| >= 2^24 of both ends (the
quantisation of the shadow itself adds at most sqrt(3) on top).  Here the
kernel's operations are replayed in numpy float32 in the kernel's order
(difference, product, two fused multiply-adds) on random shadows up to the
2^30 range, with magnitudes chosen around the 2^24 boundary where the
staged values start to round, and the exact side is computed from the
integers.  The per-box slack the kernel uses, sqrt(3) + 2^-21 6 a_max +
2^-24 6 a_max, then bounds every bond of a box by D <= 6 a_max and
A <= 6 a_max.
"""

import numpy as np


def _stencil(reach=3, delta=3.015):
    o = np.array([(a, b, c) for a in range(-reach, reach + 1) for b in range(-reach, reach + 1)
                  for c in range(-reach, reach + 1) if 0 < a * a + b * b + c * c <= delta * delta], np.int64)
    return o


def _fma32(a, b, c):
    # a * b + c rounded once to float32: the float32 product is exact in
    # float64, and the float64 sum of it and a float32 lies within half a
    # float64 unit of the exact sum, far below half a float32 unit
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def _case(rng, n, mag_lo, mag_hi, dx=6e-4):
    off = _stencil()
    k = rng.integers(0, off.shape[0], n)
    o = off[k].astype(np.float64)
    x = np.sqrt((o * o).sum(axis=1)) * dx
    M = o * dx / x[:, None]
    mx = (M / x[:, None]).astype(np.float32)  # the table entries M/x as float
    # shadows relative to the reference: magnitudes log-uniform in [mag_lo, mag_hi)
    def mag(size):
        m = np.exp(rng.uniform(np.log(mag_lo), np.log(mag_hi), size))
        return (np.sign(rng.uniform(-1, 1, size)) * m).astype(np.int64)
    ref = rng.integers(-2 ** 28, 2 ** 28, (n, 3))
    di = mag((n, 3))
    # the neighbour: close to the row (a strained bond) or anywhere in range
    near = rng.uniform(size=n) < 0.5
    dj = np.where(near[:, None], di + rng.integers(-2 ** 12, 2 ** 12, (n, 3)), mag((n, 3)))
    si = np.clip(ref + di, -(2 ** 30) + 1, 2 ** 30 - 1)
    sj = np.clip(ref + dj, -(2 ** 30) + 1, 2 ** 30 - 1)
    ai = (si - ref).astype(np.float32)  # exact integers rounded once to float
    aj = (sj - ref).astype(np.float32)
    f = aj - ai  # float32 difference
    ev = mx[:, 1] * f[:, 1]
    ev = _fma32(mx[:, 0], f[:, 0], ev)
    ev = _fma32(mx[:, 2], f[:, 2], ev)
    exact = (M * (sj - si).astype(np.float64)).sum(axis=1)
    err = np.abs(ev.astype(np.float64) * x - exact)
    D = np.abs(aj.astype(np.float64) - ai.astype(np.float64)).sum(axis=1)
    big = lambda a: np.where(np.abs(a) >= 2.0 ** 24, np.abs(a), 0.0).sum(axis=1)
    A = big(ai.astype(np.float64)) + big(aj.astype(np.float64))
    bound = 2.0 ** -21 * D + 2.0 ** -24 * A
    return err, bound, D, A, np.maximum(np.abs(ai).max(axis=1), np.abs(aj).max(axis=1)).astype(np.float64)


def test_band_holds_below_and_above_2_24():
    rng = np.random.default_rng(2309)
    for lo, hi in ((1.0, 2.0 ** 20), (2.0 ** 22, 2.0 ** 26), (2.0 ** 26, 2.0 ** 30)):
        err, bound, D, A, am = _case(rng, 200_000, lo, hi)
        # a small absolute allowance for the float64 evaluation of the exact side
        assert np.all(err <= bound + 1e-9 * (1.0 + D)), (lo, hi, float(np.max(err - bound)))
        # the per-box slack of the kernel bounds every bond of the box
        slack = 6 * 2.0 ** -21 * am + np.where(am >= 2.0 ** 24, 6 * 2.0 ** -24 * am, 0.0)
        assert np.all(bound <= slack * (1 + 1e-12))


def test_band_is_not_loose_by_orders_of_magnitude():
    # where the staged values round (above 2^24) the error does reach a
    # sizeable part of the bound: the bound is not vacuous
    rng = np.random.default_rng(7)
    err, bound, D, A, am = _case(rng, 200_000, 2.0 ** 26, 2.0 ** 30)
    assert np.max(err / bound) > 0.05
