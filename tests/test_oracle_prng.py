"""Pins of the oracle's counter-based generator and samplers.

Philox4x64-10 is checked against numpy.random.Philox (the same published
generator; numpy advances its 256-bit counter by one before each block).  The
Gaussian table is checked against a float64 evaluation with scipy-free numpy
and against the exact symmetry of the distribution.
"""
import numpy as np
import pytest


def numpy_block(ctr, key):
    """numpy's Philox output for counter `ctr` (numpy increments first)."""
    c = [int(x) for x in ctr]
    # predecessor of the 256-bit counter
    v = c[0] | (c[1] << 64) | (c[2] << 128) | (c[3] << 192)
    v = (v - 1) % (1 << 256)
    pre = [(v >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    bg = np.random.Philox(counter=np.array(pre, dtype=np.uint64),
                          key=np.array([int(key[0]), int(key[1])], dtype=np.uint64))
    return bg.random_raw(4)


def test_philox_vs_numpy(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(1)
    cases = [([0, 0, 0, 0], [0, 0]), ([1, 2, 3, 4], [5, 6]), ([2**64 - 1, 0, 7, 0], [2**63, 1])]
    for _ in range(20):
        cases.append((list(rng.integers(0, 2**64, size=4, dtype=np.uint64)),
                      list(rng.integers(0, 2**64, size=2, dtype=np.uint64))))
    for ctr, key in cases:
        assert np.array_equal(O.philox(ctr, key), numpy_block(ctr, key)), (ctr, key)


def test_stream_layout(oracle_mod):
    O = oracle_mod
    seed, dom, obj = 2003, 5, 1234567
    for w in [0, 1, 3, 4, 7, 65535, 1 << 20]:
        blk = numpy_block([w // 4, obj, dom, 0], [seed, 0])
        assert O.draw_word(seed, dom, obj, w) == int(blk[w % 4])


def test_cdt_table_float64_and_symmetry(oracle_mod):
    O = oracle_mod
    T = [int(x) for x in O.cdt_table()]
    assert len(T) == 38
    t = np.arange(-19, 20, dtype=np.float64)
    rho = np.exp(-t * t / (2 * 3.2 * 3.2))
    cdf = np.cumsum(rho) / rho.sum()
    for k in range(38):
        approx = cdf[k] * 2.0**64
        assert abs(T[k] - approx) <= max(2.0**13, approx * 1e-14), k
    # P(X <= t) + P(X <= -t-1) = 1 exactly, so floors add to 2^64 - 1
    for k in range(38):
        mirror = 37 - k  # t = k - 19  ->  -t - 1 = 18 - k  -> index 37 - k
        assert T[k] + T[mirror] == 2**64 - 1
    assert all(T[k] < T[k + 1] for k in range(37))


def test_cdt_inversion(oracle_mod):
    O = oracle_mod
    T = [int(x) for x in O.cdt_table()]
    assert O.cdt_sample(0) == -19
    for k in range(38):
        assert O.cdt_sample(T[k] - 1) == k - 19
        assert O.cdt_sample(T[k]) == k - 18
    assert O.cdt_sample(2**64 - 1) == 19


def test_sampler_statistics(oracle_mod):
    O = oracle_mod
    n = 1 << 18
    tern = O.sample_ternary(11, 4, 9, n)
    counts = np.bincount(tern + 1, minlength=3)
    chi2 = ((counts - n / 3) ** 2 / (n / 3)).sum()
    assert set(np.unique(tern)) <= {-1, 0, 1} and chi2 < 20
    g = O.sample_gaussian(11, 5, 9, n)
    assert abs(g.mean()) < 0.05 and abs(g.var() - 10.24) < 0.2 and np.abs(g).max() <= 19
    q = O.find_primes(17, [50])[0]
    u = O.sample_uniform(11, 2, 3, q, n)
    assert int(u.max()) < q and abs(u.astype(np.float64).mean() / q - 0.5) < 0.01


def test_samplers_follow_stream(oracle_mod):
    O = oracle_mod
    seed, dom, obj = 7, 4, 3
    tern = O.sample_ternary(seed, dom, obj, 16)
    for c in range(16):
        assert tern[c] == O.draw_word(seed, dom, obj, c) % 3 - 1
    q = O.find_primes(13, [40])[0]
    u = O.sample_uniform(seed, 2, obj, q, 8)
    for c in range(8):
        hi, lo = O.draw_word(seed, 2, obj, 2 * c), O.draw_word(seed, 2, obj, 2 * c + 1)
        assert int(u[c]) == ((hi << 64) | lo) % q


def _cdt_exact_mpmath():
    import mpmath
    with mpmath.workdps(120):
        sigma = mpmath.mpf(16) / 5  # 3.2 exactly
        rho = [mpmath.exp(-mpmath.mpf(t * t) / (2 * sigma * sigma)) for t in range(-19, 20)]
        total = mpmath.fsum(rho)
        out, acc, margin = [], mpmath.mpf(0), mpmath.mpf(1)
        for k in range(38):
            acc += rho[k]
            v = acc / total * mpmath.mpf(2) ** 64
            f = mpmath.floor(v)
            margin = min(margin, v - f, f + 1 - v)
            out.append(int(f))
        return out, margin


def _cdt_exact_decimal():
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 90
        two_sigma2 = 2 * (Decimal(16) / Decimal(5)) ** 2
        rho = [(-Decimal(t * t) / two_sigma2).exp() for t in range(-19, 20)]
        total = sum(rho, Decimal(0))
        out, acc = [], Decimal(0)
        for k in range(38):
            acc += rho[k]
            out.append(int((acc / total * Decimal(2) ** 64).to_integral_value(rounding="ROUND_FLOOR")))
        return out


def test_cdt_table_exact(oracle_mod):
    """The 38 stored thresholds T[t] = floor(2^64 P(X <= t)) of the
    sigma = 3.2 discrete Gaussian on [-19, 19] (the error distribution of
    key generation and encryption, CKKS Scheme Description), recomputed in the
    test at 120 digits with mpmath and at 90 digits with the standard
    library's decimal, and equal to the oracle's table in every bit.  Every
    value lies more than 2^-200 from an integer, so the floors are robust."""
    T = [int(x) for x in oracle_mod.cdt_table()]
    ref, margin = _cdt_exact_mpmath()
    assert T == ref
    assert T == _cdt_exact_decimal()
    import mpmath
    assert margin > mpmath.mpf(2) ** -200
