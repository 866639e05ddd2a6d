"""Pins of the oracle's FP64 encode/decode (Methods, Batch Encoding and
Decoding) and of the slot rotation convention.

Encode is checked against a direct solve of the canonical-embedding
Vandermonde system with numpy.linalg; decode against direct evaluation of the
polynomial at the slot roots with mpmath.
"""
import mpmath
import numpy as np
import pytest


def slot_roots(N):
    two_n = 2 * N
    e = [pow(5, j, two_n) for j in range(N // 2)]
    return e


@pytest.mark.parametrize("log_n", [3, 4, 5, 6])
def test_encode_vandermonde(oracle_mod, log_n):
    O = oracle_mod
    N = 1 << log_n
    rng = np.random.default_rng(log_n)
    z = rng.normal(size=N // 2) + 1j * rng.normal(size=N // 2)
    scale = 2.0**20
    e = slot_roots(N)
    exps = e + [2 * N - x for x in e]
    V = np.array([[np.exp(1j * np.pi * ex * k / N) for k in range(N)] for ex in exps])
    rhs = scale * np.concatenate([z, np.conj(z)])
    m = np.linalg.solve(V, rhs)
    assert np.max(np.abs(m.imag)) < 1e-6
    want = np.where(m.real >= 0, np.floor(m.real + 0.5), -np.floor(-m.real + 0.5)).astype(np.int64)
    assert np.array_equal(O.encode(z, log_n, scale), want)


@pytest.mark.parametrize("log_n", [3, 5])
def test_decode_direct_mpmath(oracle_mod, log_n):
    O = oracle_mod
    N = 1 << log_n
    rng = np.random.default_rng(7)
    m = rng.integers(-1000, 1000, size=N)
    scale = 64.0
    got = O.decode(m.astype(np.float64), log_n, scale)
    mpmath.mp.dps = 30
    for j, ex in enumerate(slot_roots(N)):
        root = mpmath.exp(1j * mpmath.pi * ex / N)
        val = mpmath.fsum(int(m[k]) * root**k for k in range(N)) / scale
        assert abs(complex(val) - got[j]) < 1e-9


def test_constant_vector_encodes_to_constant(oracle_mod):
    O = oracle_mod
    for log_n in (4, 10, 12):
        N = 1 << log_n
        m = O.encode(np.full(N // 2, 0.3), log_n, 2.0**30)
        assert m[0] == round(0.3 * 2**30) and not np.any(m[1:])


@pytest.mark.parametrize("log_n", [10, 12, 14, 16])
def test_encode_decode_roundtrip(oracle_mod, log_n):
    O = oracle_mod
    N = 1 << log_n
    rng = np.random.default_rng(log_n)
    z = rng.normal(0, 0.01, size=N // 2)
    scale = 2.0**40
    m = O.encode(z, log_n, scale)
    back = O.decode(m.astype(np.float64), log_n, scale)
    # rounding moves each coefficient by <= 1/2; the embedding spreads it over
    # N coefficients: |error| <= N / (2 scale)
    assert np.max(np.abs(back - z)) <= N / (2 * scale)
    assert np.max(np.abs(back.imag)) <= N / (2 * scale)


@pytest.mark.parametrize("log_n,k", [(4, 1), (5, 3), (6, -2), (10, 7), (12, 1 << 9)])
def test_rotation_convention(oracle_mod, log_n, k):
    """phi_g with g = 5^k moves slot j + k to slot j (left rotation)."""
    O = oracle_mod
    N = 1 << log_n
    rng = np.random.default_rng(3)
    z = rng.normal(size=N // 2)
    scale = 2.0**30
    m = O.encode(z, log_n, scale)
    g = O.galois_elt(log_n, k)
    assert g == pow(5, k % (N // 2), 2 * N)
    r = O.automorphism_coeff(m, g)
    back = O.decode(r.astype(np.float64), log_n, scale)
    assert np.allclose(back.real, np.roll(z, -k), atol=1e-6)


@pytest.mark.parametrize("log_n", [4, 6, 9])
def test_automorphism_ntt_matches_coefficient_form(oracle_mod, log_n):
    O = oracle_mod
    N = 1 << log_n
    ora = O.Oracle(log_n, (30, 30), (31,))
    rng = np.random.default_rng(log_n)
    a = rng.integers(-50, 50, size=N)
    A = ora.signed_to_ntt(a)
    for g in [5, 25, 2 * N - 1, O.galois_elt(log_n, 3)]:
        want = ora.signed_to_ntt(O.automorphism_coeff(a, g))
        assert np.array_equal(ora.automorphism_ntt(A, g), want)
