"""Pins of the oracle's modular arithmetic, primes and NTT roots.

Each check compares against something other than the oracle: Python's big
integers, or sympy's primality test and primitive roots.
"""
import random

import pytest
import sympy

Q_SMALL = [17, 97, 7681, 12289]


def big_ints_edge(q, rng, n=200):
    vals = [0, 1, 2, q - 2, q - 1, q // 2, (q + 1) // 2]
    vals += [rng.randrange(q) for _ in range(n)]
    return [v for v in vals if 0 <= v < q]


def test_mulmod_exhaustive_small(oracle_mod):
    O = oracle_mod
    for q in (17, 97):
        for a in range(q):
            for b in range(q):
                assert O.mulmod(a, b, q) == a * b % q
                assert O.addmod(a, b, q) == (a + b) % q
                assert O.submod(a, b, q) == (a - b) % q


@pytest.mark.parametrize("bits", [13, 30, 40, 50, 62])
def test_mulmod_random_edges(oracle_mod, bits):
    O = oracle_mod
    rng = random.Random(bits)
    q = sympy.prevprime(1 << bits)
    vals = big_ints_edge(q, rng, 60)
    for a in vals:
        for b in vals[:20]:
            assert O.mulmod(a, b, q) == a * b % q
            assert O.addmod(a, b, q) == (a + b) % q
            assert O.submod(a, b, q) == (a - b) % q
    for _ in range(200):
        a, b = rng.randrange(1 << 64), rng.randrange(1 << 64)
        assert O.mulmod(a, b, q) == (a % q) * (b % q) % q


def test_powmod_invmod(oracle_mod):
    O = oracle_mod
    rng = random.Random(3)
    for q in Q_SMALL + [sympy.prevprime(1 << 50)]:
        for _ in range(50):
            a = rng.randrange(1, q)
            e = rng.randrange(1 << 62)
            assert O.powmod(a, e, q) == pow(a, e, q)
            assert O.invmod(a, q) * a % q == 1


def test_is_prime_matches_sympy(oracle_mod):
    O = oracle_mod
    rng = random.Random(5)
    # strong pseudoprimes to several small bases, Carmichael numbers, prime squares
    tricky = [561, 1105, 1729, 2047, 3215031751, 3825123056546413051, 318665857834031151167461 % (1 << 64),
              (1 << 61) - 1, (1 << 62) - 57, 4294967291 ** 2 % (1 << 64), 999999000001, 2, 3, 4, 1, 0]
    for n in tricky:
        assert O.is_prime(n) == sympy.isprime(n), n
    for _ in range(3000):
        n = rng.randrange(1 << 64) | 1
        assert O.is_prime(n) == sympy.isprime(n), n
    for n in range(2000):
        assert O.is_prime(n) == sympy.isprime(n), n


def _rule_primes_bruteforce(log_m, bits):
    """Prime rule restated as a scan with sympy: for each bit size in order,
    the largest prime k*M+1 of that bit length not already taken."""
    M = 1 << log_m
    out = []
    for b in bits:
        k = ((1 << b) - 1) // M
        while True:
            c = k * M + 1
            assert c >= 1 << (b - 1)
            if sympy.isprime(c) and c not in out:
                out.append(c)
                break
            k -= 1
    return out


@pytest.mark.parametrize("log_m,bits", [
    (13, [40, 30, 30, 40]),
    (15, [50] * 10),
    (17, [50] * 28),
    (17, [50] * 12),
])
def test_find_primes(oracle_mod, log_m, bits):
    O = oracle_mod
    got = O.find_primes(log_m, bits)
    assert got == _rule_primes_bruteforce(log_m, bits)
    for q, b in zip(got, bits):
        assert q.bit_length() == b and (q - 1) % (1 << log_m) == 0


def _rule_primes_sympy(log_m, b, count):
    """The first `count` primes q = k M + 1 < 2^b (M = 2^log_m), largest k
    first, found with sympy's primality test."""
    M = 1 << log_m
    out, k = [], ((1 << b) - 1) // M
    while len(out) < count:
        c = k * M + 1
        assert c >= 1 << (b - 1)
        if sympy.isprime(c):
            out.append(c)
        k -= 1
    return out


def test_find_primes_n4096_chain(oracle_mod):
    # The N=2^12 chain (M = 2^13): the first two 40-bit and the first two
    # 30-bit primes of the rule, found independently with sympy; mixed bit
    # sizes take the next unused prime of each size.
    O = oracle_mod
    p40, p30 = _rule_primes_sympy(13, 40, 2), _rule_primes_sympy(13, 30, 2)
    assert p40 == [1099511480321, 1099511390209] and p30 == [1073692673, 1073668097]
    assert O.find_primes(13, [40, 40]) == p40
    assert O.find_primes(13, [30, 30]) == p30
    assert O.find_primes(13, [40, 30, 30, 40]) == [p40[0], p30[0], p30[1], p40[1]]


@pytest.mark.parametrize("q,log_n", [(7681, 8), (12289, 9), (12289, 10), (97, 4), (17, 3)])
def test_min_psi_bruteforce(oracle_mod, q, log_n):
    O = oracle_mod
    N = 1 << log_n
    psi = O.min_psi(q, log_n)
    want = min(x for x in range(2, q) if pow(x, N, q) == q - 1)
    assert psi == want


@pytest.mark.parametrize("log_n,bits", [(12, 40), (14, 50), (16, 50)])
def test_min_psi_large(oracle_mod, log_n, bits):
    O = oracle_mod
    N = 1 << log_n
    q = O.find_primes(log_n + 1, [bits])[0]
    psi = O.min_psi(q, log_n)
    assert pow(psi, N, q) == q - 1
    # all primitive 2N-th roots from sympy's generator of Z_q^*
    g = sympy.primitive_root(q)
    w = pow(g, (q - 1) // (2 * N), q)
    w2 = w * w % q
    best, y = w, w
    for _ in range(N - 1):
        y = y * w2 % q
        best = min(best, y)
    assert psi == best
