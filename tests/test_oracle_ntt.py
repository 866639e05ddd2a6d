"""Pins of the oracle's negacyclic NTT.

The transform's definition -- evaluation of a at psi^(2 brev(i) + 1) -- is
evaluated here with Python integers; the negacyclic property is checked
against a schoolbook product written with Python integers.
"""
import random

import numpy as np
import pytest


def brev(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


def py_ntt_def(a, q, psi):
    N = len(a)
    bits = N.bit_length() - 1
    out = []
    for i in range(N):
        e = 2 * brev(i, bits) + 1
        out.append(sum(int(a[j]) * pow(psi, e * j, q) for j in range(N)) % q)
    return out


def py_negacyclic(a, b, q):
    N = len(a)
    out = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            p = int(a[i]) * int(b[j])
            if k < N:
                out[k] += p
            else:
                out[k - N] -= p
    return [x % q for x in out]


def rand_poly(rng, N, q):
    return np.array([rng.randrange(q) for _ in range(N)], dtype=np.uint64)


@pytest.mark.parametrize("log_n,bits", [(4, 30), (5, 40), (6, 50), (4, 17)])
def test_ntt_matches_definition(oracle_mod, log_n, bits):
    O = oracle_mod
    rng = random.Random(log_n * 100 + bits)
    q = O.find_primes(log_n + 1, [bits])[0]
    psi = O.min_psi(q, log_n)
    a = rand_poly(rng, 1 << log_n, q)
    want = py_ntt_def(a, q, psi)
    assert [int(x) for x in O.ntt(a, q, psi)] == want
    assert [int(x) for x in O.ntt_direct(a, q, psi)] == want


@pytest.mark.parametrize("log_n", [4, 5, 6, 7, 8])
def test_ntt_negacyclic_product(oracle_mod, log_n):
    O = oracle_mod
    rng = random.Random(log_n)
    N = 1 << log_n
    for bits in (30, 50):
        q = O.find_primes(log_n + 1, [bits])[0]
        psi = O.min_psi(q, log_n)
        a, b = rand_poly(rng, N, q), rand_poly(rng, N, q)
        A, B = O.ntt(a, q, psi), O.ntt(b, q, psi)
        C = np.array([int(x) * int(y) % q for x, y in zip(A, B)], dtype=np.uint64)
        c = O.intt(C, q, psi)
        assert [int(x) for x in c] == py_negacyclic(a, b, q)
        assert [int(x) for x in O.negacyclic_mul(a, b, q)] == py_negacyclic(a, b, q)


def test_ntt_direct_vs_fast_256(oracle_mod):
    O = oracle_mod
    rng = random.Random(9)
    q = O.find_primes(9, [50])[0]
    psi = O.min_psi(q, 8)
    a = rand_poly(rng, 256, q)
    assert np.array_equal(O.ntt(a, q, psi), O.ntt_direct(a, q, psi))


@pytest.mark.parametrize("log_n", [10, 12, 14, 16])
def test_ntt_roundtrip_and_special_inputs(oracle_mod, log_n):
    O = oracle_mod
    N = 1 << log_n
    q = O.find_primes(log_n + 1, [50])[0]
    psi = O.min_psi(q, log_n)
    rng = np.random.default_rng(log_n)
    a = rng.integers(0, q, size=N, dtype=np.uint64)
    assert np.array_equal(O.intt(O.ntt(a, q, psi), q, psi), a)
    # NTT(1) = (1, ..., 1)
    one = np.zeros(N, dtype=np.uint64)
    one[0] = 1
    assert np.all(O.ntt(one, q, psi) == 1)
    # NTT(X)[i] = psi^(2 brev(i) + 1)
    x = np.zeros(N, dtype=np.uint64)
    x[1] = 1
    got = O.ntt(x, q, psi)
    bits = log_n
    for i in [0, 1, 2, 3, N // 2, N - 1]:
        assert int(got[i]) == pow(psi, 2 * brev(i, bits) + 1, q)
    # the sum over all N evaluation points (odd powers of psi) is N * a_0
    b = rng.integers(0, q, size=N, dtype=np.uint64)
    B = O.ntt(b, q, psi)
    assert sum(int(v) for v in B) % q == N * int(b[0]) % q
