"""The mixed kernel's cutoff band, checked on the host: its fixed-point
displacement arithmetic, replayed in numpy operation for operation (wrapping
32-bit differences, an exact unit, FP64 products and sums with separate
roundings), never moves r^2 further from the FP64 r^2 of the unquantised
positions than the bound the band is built from, for pairs near rc, across
periodic faces, in boxes from 10 to 400."""
import numpy as np

TWO32 = 4294967296.0


def fixed(x, L):
    # rint(x 2^32 / L) mod 2^32, as the quantisation kernel computes it
    return (np.rint(x * (TWO32 / L)).astype(np.int64) & 0xFFFFFFFF).astype(np.uint32)


def r2_fixed(qi, qj, L):
    d = (qj - qi).view(np.int32).astype(np.float64) * (L / TWO32)   # wrapping difference
    return (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]


def r2_fp64(xi, xj, L):
    t = xj - xi
    t = np.where(t > 0.5 * L, t - L, np.where(t < -0.5 * L, t + L, t))
    return (t[:, 0] * t[:, 0] + t[:, 1] * t[:, 1]) + t[:, 2] * t[:, 2]


def bound(r, L):
    e = 1.0001 * L / TWO32
    return 2.0 * np.sqrt(3.0) * r * e + 3.0 * e * e


def test_fixed_point_r2_stays_within_the_band_bound():
    rng = np.random.Generator(np.random.PCG64(1806))
    worst = 0.0
    for L in (10.0, 50.797, 110.6, 167.577, 400.0):
        for rc in (2.5, 3.0):
            m = 200_000
            xi = rng.uniform(0.0, L, (m, 3))
            # a third of the atoms hug a face, so their partners cross it
            face = rng.integers(0, 3, m // 3)
            xi[np.arange(m // 3), face] = rng.uniform(L - 1e-3, L, m // 3) % L
            u = rng.normal(size=(m, 3))
            u /= np.linalg.norm(u, axis=1, keepdims=True)
            r = rc * np.concatenate([1.0 + rng.uniform(-2e-6, 2e-6, m // 2),
                                     rng.uniform(0.8, 1.001, m - m // 2)])
            xj = xi + r[:, None] * u
            xj = xj - L * np.floor(xj / L)
            xj[xj >= L] = 0.0
            a = r2_fixed(fixed(xi, L), fixed(xj, L), L)
            b = r2_fp64(xi, xj, L)
            rr = np.sqrt(b)
            assert np.all(rr <= 1.001 * rc + 1e-9)
            err = np.abs(a - b)
            lim = bound(rr, L) + 1e-12 * rc * rc
            assert np.all(err <= lim), (L, rc, float((err / lim).max()))
            worst = max(worst, float((err / lim).max()))
    # the bound is not loose by orders of magnitude (it would hide a lost term)
    assert worst > 0.05


def test_band_decides_like_fp64_outside_it():
    """Outside the band the fixed-point test and the FP64 test agree; every
    disagreement lies inside it."""
    rng = np.random.Generator(np.random.PCG64(57))
    L, rc = 50.797, 3.0
    m = 400_000
    xi = rng.uniform(0.0, L, (m, 3))
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = rc * (1.0 + rng.uniform(-1e-6, 1e-6, m))
    xj = xi + r[:, None] * u
    xj = xj - L * np.floor(xj / L)
    xj[xj >= L] = 0.0
    a = r2_fixed(fixed(xi, L), fixed(xj, L), L)
    b = r2_fp64(xi, xj, L)
    rc2 = rc * rc
    band = 2.0 * bound(1.001 * rc, L) + 1e-12 * rc2
    lo, hi = rc2 - band, rc2 + band
    decided = (a < lo) | (a >= hi)
    assert np.all((a[decided] < lo) == (b[decided] < rc2))
    assert np.any(~decided) and np.any((a < rc2) != (b < rc2))   # the band is needed
