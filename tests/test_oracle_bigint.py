"""Third vote on the oracle's key switching: Python big-integer arithmetic in
the coefficient domain at N = 16.

The oracle computes ModUp, ModDown, key switching, relinearization, hoisted
rotations and rotate-and-sum on residues in the NTT domain with 128-bit
`% q` products (Methods, Dynamic Hoisting: RNS decomposition into dnum
digits, ModUp, key inner product, ModDown; Methods, Lazy Relinearization).
This file recomputes the same operations a different way and demands the
same bits:

  * residues leave the NTT domain by evaluating the definition of the
    inverse transform (a_j = N^-1 sum_i A_i psi^-(2 brev(i) + 1) j) and are
    joined into integers by CRT;
  * the fast base conversion of digit d is taken as the exact integer
    v_d = sum_{i in D_d} [x_i (Q_d / q_i)^-1]_{q_i} (Q_d / q_i), before any
    reduction, then reduced by each modulus of the extended basis;
  * the key inner product is an integer negacyclic product in
    Z[X] / (X^N + 1), reduced modulo PQ;
  * ModDown is the exact division (U - w) / P with
    w = sum_k [U (P / p_k)^-1]_{p_k} (P / p_k), checked to leave no
    remainder, instead of a product by P^-1 modulo each q_i;
  * an automorphism X -> X^g acts on integer coefficients with signs;
  * results return to the NTT domain by evaluating the forward definition.

Parameter sets use alpha = 2 special primes with dnum = 2 and 3 digits, and
one chain whose last digit is partial (one limb).  Inputs are full-range
residues and keys are both the oracle's own key-switching keys and uniform
residues (a key's structure does not enter the arithmetic).
"""
import numpy as np
import pytest

LOG_N = 4
N = 1 << LOG_N
TWO_N = 2 * N

PARAMS = [
    dict(q_bits=(30, 30, 30, 30), p_bits=(31, 31)),              # alpha 2, dnum 2
    dict(q_bits=(40, 30, 30, 30, 30, 30), p_bits=(41, 41)),      # alpha 2, dnum 3
    dict(q_bits=(36, 30, 30, 30, 30), p_bits=(37, 37)),          # alpha 2, dnum 3, last digit one limb
]


# ---- transforms from their definitions -----------------------------------------

def brev(i, bits):
    return int(format(i, "0%db" % bits)[::-1], 2)


def ntt_def(a, q, psi):
    """A_i = a(psi^(2 brev(i) + 1)), the NTT-domain convention."""
    out = []
    for i in range(N):
        r = pow(psi, 2 * brev(i, LOG_N) + 1, q)
        acc, x = 0, 1
        for j in range(N):
            acc += int(a[j]) * x
            x = x * r % q
        out.append(acc % q)
    return out


def intt_def(A, q, psi):
    """a_j = N^-1 sum_i A_i psi^(-(2 brev(i) + 1) j)."""
    ninv = pow(N, -1, q)
    pinv = pow(psi, -1, q)
    out = []
    for j in range(N):
        acc = 0
        for i in range(N):
            acc += int(A[i]) * pow(pinv, (2 * brev(i, LOG_N) + 1) * j, q)
        out.append(acc * ninv % q)
    return out


def crt(residue_rows, mods):
    """Per coefficient, the integer in [0, prod mods) with these residues."""
    M = 1
    for m in mods:
        M *= m
    out = []
    for j in range(N):
        x = 0
        for r, m in zip(residue_rows, mods):
            Mi = M // m
            x += (int(r[j]) * pow(Mi % m, -1, m) % m) * Mi
        out.append(x % M)
    return out


def negacyclic(a, b, M):
    out = [0] * N
    for i in range(N):
        if a[i] == 0:
            continue
        for j in range(N):
            k = i + j
            if k < N:
                out[k] += a[i] * b[j]
            else:
                out[k - N] -= a[i] * b[j]
    return [v % M for v in out]


def automorphism(a, g):
    """X^j -> X^(j g): coefficient j moves to j g mod 2N, negated past N."""
    out = [0] * N
    for j in range(N):
        e = j * g % TWO_N
        if e < N:
            out[e] += a[j]
        else:
            out[e - N] -= a[j]
    return out


def galois(step):
    return pow(5, step % (N // 2), TWO_N)


# ---- the scheme's key-switching pieces in big integers --------------------------

class BigInt:
    def __init__(self, ora):
        self.q = list(ora.q)
        self.p = list(ora.p)
        self.mods = self.q + self.p
        self.psi = list(ora.psi)
        for m, s in zip(self.mods, self.psi):
            assert pow(s, N, m) == m - 1  # a primitive 2N-th root (N a power of two)
        self.alpha = len(self.p)
        self.digits = [list(range(a, min(a + self.alpha, len(self.q)))) for a in range(0, len(self.q), self.alpha)]
        self.Q = int(np.prod([int(x) for x in self.q], dtype=object))
        self.P = int(np.prod([int(x) for x in self.p], dtype=object))

    # domain changes
    def to_coeff(self, rows, limb0=0):
        return [intt_def(r, self.mods[limb0 + l], self.psi[limb0 + l]) for l, r in enumerate(rows)]

    def to_ntt(self, ints, limbs):
        """integer polynomial -> NTT-domain residues on the listed limbs"""
        return np.array([ntt_def([v % self.mods[l] for v in ints], self.mods[l], self.psi[l]) for l in limbs],
                        dtype=np.uint64)

    def poly_Q(self, rows):
        """NTT-domain [nq][N] -> integer polynomial modulo Q"""
        return crt(self.to_coeff(rows), self.q)

    def key_PQ(self, rows):
        """NTT-domain [nq + np][N] -> integer polynomial modulo PQ"""
        return crt(self.to_coeff(rows), self.mods)

    # ModUp: the exact integer of each digit's fast base conversion
    def raise_digits(self, x_rows):
        xh = self.to_coeff(x_rows)
        out = []
        for D in self.digits:
            Qd = int(np.prod([self.q[i] for i in D], dtype=object))
            v = [0] * N
            for i in D:
                qi = self.q[i]
                fac = Qd // qi
                inv = pow(fac % qi, -1, qi)
                for j in range(N):
                    v[j] += (xh[i][j] * inv % qi) * fac
            # v = x_d + u Q_d with 0 <= u < |D|: congruent to x on the digit's limbs
            for i in D:
                assert all(v[j] % self.q[i] == xh[i][j] for j in range(N))
                assert all(0 <= v[j] < len(D) * Qd for j in range(N))
            out.append(v)
        return out

    # ModDown: exact division by P
    def moddown(self, U):
        r = []
        for u in U:
            u %= self.Q * self.P
            w = 0
            for pk in self.p:
                fac = self.P // pk
                w += (u % pk) * pow(fac % pk, -1, pk) % pk * fac
            assert (u - w) % self.P == 0
            r.append((u - w) // self.P)
        return r

    def inner(self, digits, keys):
        """U_k = sum over keys and digits of phi_g(v_d) * key_{d,k} mod PQ;
        keys: list of (ksk [dnum][2][ne][N], g)."""
        PQ = self.P * self.Q
        U = [[0] * N, [0] * N]
        for ksk, gk in keys:
            for d, v in enumerate(digits):
                vg = automorphism(v, gk) if gk != 1 else v
                for k in range(2):
                    prod = negacyclic(vg, self.key_PQ(ksk[d][k]), PQ)
                    U[k] = [(a + b) % PQ for a, b in zip(U[k], prod)]
        return U

    def keyswitch(self, x_rows, ksk):
        U = self.inner(self.raise_digits(x_rows), [(ksk, 1)])
        return [self.moddown(U[0]), self.moddown(U[1])]

    def ct_ints(self, ct):
        return [self.poly_Q(ct[0]), self.poly_Q(ct[1])]

    def ct_rows(self, c0, c1):
        limbs = range(len(self.q))
        return np.stack([self.to_ntt(c0, limbs), self.to_ntt(c1, limbs)])


def rotate_sum_big(B, y0, y1, plan, rks):
    """Rotate-and-sum with a block plan: block b starting at level j0 adds
    rot_{t 2^j0}(y) for t = 1 .. 2^k_b - 1 from one raise of y.c1, all key
    products summed in PQ and one ModDown."""
    Q = B.Q
    key, j0 = 0, 0
    for kb in plan:
        digits = B.raise_digits(B.ct_rows(y0, y1)[1])
        keys, c0sum = [], [0] * N
        for t in range(1, 1 << kb):
            g = galois(t << j0)
            keys.append((rks[key], g))
            key += 1
            c0sum = [a + b for a, b in zip(c0sum, automorphism(y0, g))]
        U = B.inner(digits, keys)
        m0, m1 = B.moddown(U[0]), B.moddown(U[1])
        y0 = [(a + b + c) % Q for a, b, c in zip(y0, c0sum, m0)]
        y1 = [(a + b) % Q for a, b in zip(y1, m1)]
        j0 += kb
    return y0, y1


def setup(O, prm, seed=31):
    ora = O.Oracle(LOG_N, prm["q_bits"], prm["p_bits"])
    assert ora.alpha == 2 and ora.dnum == -(-ora.nq // 2)
    return ora, BigInt(ora), np.random.default_rng(seed)


def uniform_rows(rng, mods, shape_prefix=()):
    out = np.empty(shape_prefix + (len(mods), N), dtype=np.uint64)
    for l, m in enumerate(mods):
        out[..., l, :] = rng.integers(0, m, size=shape_prefix + (N,), dtype=np.uint64)
    return out


# ---- the votes ----------------------------------------------------------------------

@pytest.mark.parametrize("prm", PARAMS)
def test_modup_bits(oracle_mod, prm):
    O = oracle_mod
    ora, B, rng = setup(O, prm)
    for _ in range(2):
        x = uniform_rows(rng, ora.q)
        got = ora.modup(x)  # [dnum][ne][N]
        digits = B.raise_digits(x)
        for d, v in enumerate(digits):
            want = B.to_ntt(v, range(ora.ne))
            assert np.array_equal(got[d], want), d


@pytest.mark.parametrize("prm", PARAMS)
def test_moddown_bits(oracle_mod, prm):
    O = oracle_mod
    ora, B, rng = setup(O, prm, seed=32)
    for _ in range(2):
        u = uniform_rows(rng, ora.primes)
        got = ora.moddown(u)
        want = B.to_ntt(B.moddown(B.key_PQ(u)), range(ora.nq))
        assert np.array_equal(got, want)


@pytest.mark.parametrize("prm", PARAMS)
@pytest.mark.parametrize("keykind", ["oracle", "uniform"])
def test_keyswitch_and_relin_bits(oracle_mod, prm, keykind):
    O = oracle_mod
    ora, B, rng = setup(O, prm, seed=33)
    s = ora.secret(5)
    if keykind == "oracle":
        rlk = ora.relin_key(6, s)
    else:
        rlk = uniform_rows(rng, ora.primes, (ora.dnum, 2))
    x = uniform_rows(rng, ora.q)
    ks = ora.keyswitch(x, rlk)
    want = B.keyswitch(x, rlk)
    assert np.array_equal(ks, B.ct_rows(*want))
    ct3 = uniform_rows(rng, ora.q, (3,))
    got = ora.relin(ct3, rlk)
    k0, k1 = B.keyswitch(ct3[2], rlk)
    Q = B.Q
    d0, d1 = B.poly_Q(ct3[0]), B.poly_Q(ct3[1])
    want = B.ct_rows([(a + b) % Q for a, b in zip(d0, k0)], [(a + b) % Q for a, b in zip(d1, k1)])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("prm", PARAMS)
def test_rotate_hoisted_bits(oracle_mod, prm):
    O = oracle_mod
    ora, B, rng = setup(O, prm, seed=34)
    s = ora.secret(5)
    steps = [1, 2, 3, -1, 5]
    rks = [ora.rot_key(7, s, k) for k in steps[:3]] + [uniform_rows(rng, ora.primes, (ora.dnum, 2))
                                                        for _ in steps[3:]]
    ct = uniform_rows(rng, ora.q, (2,))
    got = ora.rotate_hoisted(ct, steps, rks)
    c0, _ = B.ct_ints(ct)
    digits = B.raise_digits(ct[1])  # one raise shared by every step
    Q = B.Q
    for t, (k, rk) in enumerate(zip(steps, rks)):
        g = galois(k)
        U = B.inner(digits, [(rk, g)])
        r0 = [(a + b) % Q for a, b in zip(automorphism(c0, g), B.moddown(U[0]))]
        assert np.array_equal(got[t], B.ct_rows(r0, B.moddown(U[1]))), k


@pytest.mark.parametrize("prm", PARAMS)
@pytest.mark.parametrize("plan", [(1, 1, 1), (2, 1), (1, 2), (3,)])
def test_rotate_sum_bits(oracle_mod, prm, plan):
    O = oracle_mod
    ora, B, rng = setup(O, prm, seed=35)
    s = ora.secret(5)
    steps = ora.rotsum_steps(list(plan))
    rks = [ora.rot_key(8, s, k) for k in steps]
    ct = uniform_rows(rng, ora.q, (2,))
    got = ora.rotate_sum(ct, list(plan), rks)
    y0, y1 = rotate_sum_big(B, *B.ct_ints(ct), plan, rks)
    assert np.array_equal(got, B.ct_rows(y0, y1))


def test_pairwise_pipeline_bits(oracle_mod):
    """Algorithm 1 (Server Executes) at N = 16: per pair the triples of the
    squared differences summed over the packed ciphertexts, one
    relinearization, rotate-and-sum; SumDis[i] = sum over j != i."""
    O = oracle_mod
    ora, B, rng = setup(O, PARAMS[1], seed=36)
    s = ora.secret(5)
    rlk = ora.relin_key(9, s)
    plan = [2, 1]
    rks = [ora.rot_key(9, s, k) for k in ora.rotsum_steps(plan)]
    n, ln = 3, 2
    cts = uniform_rows(rng, ora.q, (n, ln, 2))
    got = ora.pairwise(cts, rlk, plan, rks)
    Q = B.Q
    ints = [[B.ct_ints(cts[i, k]) for k in range(ln)] for i in range(n)]
    dist = []
    for i in range(n):
        for j in range(i + 1, n):
            t0, t1, t2 = [0] * N, [0] * N, [0] * N
            for k in range(ln):
                d0 = [(a - b) % Q for a, b in zip(ints[i][k][0], ints[j][k][0])]
                d1 = [(a - b) % Q for a, b in zip(ints[i][k][1], ints[j][k][1])]
                t0 = [(a + b) % Q for a, b in zip(t0, negacyclic(d0, d0, Q))]
                t1 = [(a + 2 * b) % Q for a, b in zip(t1, negacyclic(d0, d1, Q))]
                t2 = [(a + b) % Q for a, b in zip(t2, negacyclic(d1, d1, Q))]
            k0, k1 = B.keyswitch(B.to_ntt(t2, range(ora.nq)), rlk)
            y0, y1 = rotate_sum_big(B, [(a + b) % Q for a, b in zip(t0, k0)], [(a + b) % Q for a, b in zip(t1, k1)],
                                    plan, rks)
            dist.append(B.ct_rows(y0, y1))
    assert np.array_equal(got["dist"], np.stack(dist))
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    for i in range(n):
        acc0, acc1 = [0] * N, [0] * N
        for p, (a, b) in enumerate(pairs):
            if i in (a, b):
                e0, e1 = B.ct_ints(dist[p])
                acc0 = [(u + v) % Q for u, v in zip(acc0, e0)]
                acc1 = [(u + v) % Q for u, v in zip(acc1, e1)]
        assert np.array_equal(got["sumdis"][i], B.ct_rows(acc0, acc1)), i


def test_vote_catches_a_planted_mistake(oracle_mod):
    """The third vote is sharp: a ModDown with a rounding offset (one
    plausible variant of the conversion) or a digit raised by exact CRT
    instead of the fast conversion gives different bits."""
    O = oracle_mod
    ora, B, rng = setup(O, PARAMS[0], seed=37)
    u = uniform_rows(rng, ora.primes)
    U = B.key_PQ(u)
    exact = B.to_ntt(B.moddown(U), range(ora.nq))
    rounded = B.to_ntt([((v + B.P // 2) % (B.P * B.Q)) for v in U], range(ora.ne))
    # ModDown of U + P/2 is the rounded division: differs from the oracle's
    assert not np.array_equal(ora.moddown(rounded), exact)
    x = uniform_rows(rng, ora.q)
    xh = B.to_coeff(x)
    D = B.digits[0]
    exact_crt = crt([xh[i] for i in D], [B.q[i] for i in D])
    raised = ora.modup(x)[0]
    other = ora.nq  # the first P limb is outside every digit
    assert not np.array_equal(raised[other], ntt_def([v % B.mods[other] for v in exact_crt], B.mods[other],
                                                     B.psi[other]))
