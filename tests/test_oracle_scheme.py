"""Pins of the oracle's CKKS scheme operations on tiny parameter sets.

Exact identities are checked against Python big-integer arithmetic
(negacyclic schoolbook products, CRT); approximate ones against noise bounds
derived from the sampler supports.
"""
import numpy as np
import pytest

TERN_MAX, GAUSS_MAX = 1, 19


def centered(x, Q):
    x %= Q
    return x - Q if x > Q // 2 else x


def py_negacyclic_int(a, b):
    N = len(a)
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
    return out


def dec_ints(ora, res):
    """centred integers of a coefficient-domain residue array [nq][N]."""
    return ora.crt(res)


def diff_inf(ora, res_a, res_b):
    Q = 1
    for q in ora.q:
        Q *= q
    a, b = ora.crt(res_a), ora.crt(res_b)
    return max(abs(centered(x - y, Q)) for x, y in zip(a, b))


def make(O, log_n=5, q_bits=(30, 28, 28), p_bits=(30,), seed=5):
    ora = O.Oracle(log_n, q_bits, p_bits)
    s = ora.secret(seed)
    pk = ora.pk(seed, s)
    return ora, s, pk


PARAMS = [dict(log_n=5, q_bits=(30, 28, 28), p_bits=(30,)),
          dict(log_n=4, q_bits=(40, 40, 40, 40), p_bits=(41, 41)),
          dict(log_n=6, q_bits=(45, 40, 40, 40, 40), p_bits=(46, 46))]


@pytest.mark.parametrize("prm", PARAMS)
def test_pk_and_ksk_structure(oracle_mod, prm):
    O = oracle_mod
    ora, s, pk = make(O, **prm)
    N = ora.N
    # pk0 + pk1 s = e  (small) on every limb
    sh = ora.signed_to_ntt(s)
    e = ora.poly_intt(np.array([[(int(a) + int(b) * int(c)) % q for a, b, c in zip(pk[0][l], pk[1][l], sh[l])]
                                for l, q in enumerate(ora.q)], dtype=np.uint64))
    vals = ora.crt(e)
    assert max(abs(v) for v in vals) <= GAUSS_MAX
    # ksk_d0 + ksk_d1 s - G_d s' = e_d, with G_d = P on digit d's limbs, 0 elsewhere
    s2 = O.secret_square(s)
    k = ora.relin_key(9, s)
    P = 1
    for p in ora.p:
        P *= p
    she = ora.signed_to_ntt(s, ora.ne)
    s2e = ora.signed_to_ntt(s2, ora.ne)
    for d in range(ora.dnum):
        rows = []
        for l, m in enumerate(ora.primes):
            g = P % m if (l < ora.nq and l // ora.alpha == d) else 0
            rows.append([(int(k0) + int(k1) * int(x) - g * int(y)) % m
                         for k0, k1, x, y in zip(k[d][0][l], k[d][1][l], she[l], s2e[l])])
        r = np.array(rows, dtype=np.uint64)
        coeff = np.vstack([ora.poly_intt(r[l:l + 1], l) for l in range(ora.ne)])
        ints = O.crt_centered(coeff, ora.primes)
        assert max(abs(v) for v in ints) <= GAUSS_MAX


@pytest.mark.parametrize("prm", PARAMS)
def test_encrypt_decrypt(oracle_mod, prm):
    O = oracle_mod
    ora, s, pk = make(O, **prm)
    N = ora.N
    rng = np.random.default_rng(1)
    m = rng.integers(-(1 << 20), 1 << 20, size=(3, N))
    ct = ora.encrypt(42, 100, m, pk)
    bound = 2 * GAUSS_MAX * N + GAUSS_MAX
    for t in range(3):
        got = ora.crt(ora.decrypt(ct[t], s))
        assert max(abs(g - int(x)) for g, x in zip(got, m[t])) <= bound
    # zero randomness: exact
    z = np.zeros(N, dtype=np.int64)
    ct0 = ora.encrypt_with(m[0], z, z, z, pk)
    assert ora.crt(ora.decrypt(ct0, s)) == [int(x) for x in m[0]]
    # encrypt draws follow the stream: object 101 is the second plaintext
    r = O.sample_ternary(42, O.DOM_ENC_V, 101, N)
    e0 = O.sample_gaussian(42, O.DOM_ENC_E0, 101, N)
    e1 = O.sample_gaussian(42, O.DOM_ENC_E1, 101, N)
    assert np.array_equal(ora.encrypt_with(m[1], r, e0, e1, pk), ct[1])


@pytest.mark.parametrize("prm", PARAMS[:2])
def test_tensor_exact_identity(oracle_mod, prm):
    """Dec3(ct x ct') = Dec(ct) * Dec(ct') in Z_Q[X]/(X^N+1), exactly."""
    O = oracle_mod
    ora, s, pk = make(O, **prm)
    N = ora.N
    rng = np.random.default_rng(2)
    m = rng.integers(-(1 << 15), 1 << 15, size=(2, N))
    a, b = ora.encrypt(3, 0, m, pk)
    Q = 1
    for q in ora.q:
        Q *= q
    da, db = ora.crt(ora.decrypt(a, s)), ora.crt(ora.decrypt(b, s))
    want = [centered(x, Q) for x in py_negacyclic_int(da, db)]
    got = ora.crt(ora.decrypt(ora.mul(a, b), s))
    assert got == want
    # square = mul(a, a); sub is exact
    sq = ora.mul(a, a)
    got_sq = ora.crt(ora.decrypt(sq, s))
    assert got_sq == [centered(x, Q) for x in py_negacyclic_int(da, da)]
    d = ora.sub(a, b)
    assert ora.crt(ora.decrypt(d, s)) == [centered(x - y, Q) for x, y in zip(da, db)]
    # lazy accumulation of triples decrypts to the sum of the products
    acc = ora.add(ora.mul(a, b), sq)
    assert ora.crt(ora.decrypt(acc, s)) == [centered(x + y, Q) for x, y in zip(want, got_sq)]


def ks_bound(ora):
    P = 1
    for p in ora.p:
        P *= p
    qd = max(int(np.prod([float(q) for q in ora.q[d * ora.alpha:(d + 1) * ora.alpha]]))
             for d in range(ora.dnum))
    ratio = qd / P
    return 2 * ora.dnum * ora.alpha * ora.N * GAUSS_MAX * max(1.0, ratio) + (ora.np_ + 1) * (ora.N + 1)


@pytest.mark.parametrize("prm", PARAMS)
def test_modup_property(oracle_mod, prm):
    """Raised digit limbs hold x_d + u Q_d with 0 <= u < alpha (fast BConv)."""
    O = oracle_mod
    ora, s, pk = make(O, **prm)
    rng = np.random.default_rng(4)
    x = np.array([rng.integers(0, q, size=ora.N, dtype=np.uint64) for q in ora.q])
    X = ora.modup(x)
    xc = ora.poly_intt(x)
    for d in range(ora.dnum):
        lim = list(range(d * ora.alpha, min((d + 1) * ora.alpha, ora.nq)))
        Qd = 1
        for i in lim:
            Qd *= ora.q[i]
        xd = O.crt_centered(xc[lim], [ora.q[i] for i in lim])
        xd = [v % Qd for v in xd]
        for l, r in enumerate(ora.primes):
            Xl = ora.poly_intt(X[d][l:l + 1], l)[0]
            if l in lim:
                assert np.array_equal(X[d][l], x[l])
                continue
            for t in range(ora.N):
                u = (int(Xl[t]) - xd[t]) * pow(Qd % r, -1, r) % r
                assert u < len(lim)


@pytest.mark.parametrize("prm", PARAMS)
def test_moddown_property(oracle_mod, prm):
    """ModDown(u) = floor(U / P) - w mod Q with 0 <= w < K."""
    O = oracle_mod
    ora, s, pk = make(O, **prm)
    rng = np.random.default_rng(6)
    u = np.array([rng.integers(0, m, size=ora.N, dtype=np.uint64) for m in ora.primes])
    r = ora.moddown(u)
    uc = np.vstack([ora.poly_intt(u[l:l + 1], l) for l in range(ora.ne)])
    rc = ora.poly_intt(r)
    P, Q = 1, 1
    for p in ora.p:
        P *= p
    for q in ora.q:
        Q *= q
    U = [v % (P * Q) for v in O.crt_centered(uc, ora.primes)]
    R = [v % Q for v in O.crt_centered(rc, ora.q)]
    for t in range(ora.N):
        w = (U[t] // P - R[t]) % Q
        assert w < ora.np_


@pytest.mark.parametrize("prm", PARAMS)
def test_relin_and_keyswitch(oracle_mod, prm):
    O = oracle_mod
    ora, s, pk = make(O, **prm)
    N = ora.N
    rng = np.random.default_rng(8)
    m = rng.integers(-(1 << 12), 1 << 12, size=(2, N))
    a, b = ora.encrypt(3, 0, m, pk)
    t3 = ora.mul(a, b)
    rlk = ora.relin_key(9, s)
    ct = ora.relin(t3, rlk)
    assert diff_inf(ora, ora.decrypt(ct, s), ora.decrypt(t3, s)) <= ks_bound(ora)
    # zero-error key: only the ModDown rounding remains
    ne, dnum = ora.ne, ora.dnum
    a_all = np.array([[rng.integers(0, q, size=N, dtype=np.uint64) for q in ora.primes] for _ in range(dnum)])
    zero_e = np.zeros((dnum, N), dtype=np.int64)
    k0 = ora.ksk_with(s, O.secret_square(s), a_all, zero_e)
    ct0 = ora.relin(t3, k0)
    assert diff_inf(ora, ora.decrypt(ct0, s), ora.decrypt(t3, s)) <= (ora.np_ + 1) * (N + 1)


@pytest.mark.parametrize("prm", PARAMS)
def test_rotation_hoisted(oracle_mod, prm):
    O = oracle_mod
    ora, s, pk = make(O, **prm)
    N = ora.N
    rng = np.random.default_rng(10)
    z = rng.normal(size=N // 2)
    scale = 2.0**20
    m = O.encode(z, ora.log_n, scale)
    ct = ora.encrypt(5, 0, m[None], pk)[0]
    steps = [1, 2, 3, N // 4]
    rks = [ora.rot_key(9, s, k) for k in steps]
    outs = ora.rotate_hoisted(ct, steps, rks)
    for k, o in zip(steps, outs):
        dec = ora.crt(ora.decrypt(o, s))
        back = O.decode(np.array(dec, dtype=np.float64), ora.log_n, scale)
        assert np.allclose(back.real, np.roll(z, -k), atol=1e-2)
        # non-hoisted order (permute, then raise) agrees after decryption
        g = O.galois_elt(ora.log_n, k)
        pc = ora.automorphism_ntt(ct, g)
        ks = ora.keyswitch(pc[1], rks[steps.index(k)])
        alt = ora.add(np.stack([pc[0], np.zeros_like(pc[0])]), ks)
        assert diff_inf(ora, ora.decrypt(alt, s), ora.decrypt(o, s)) <= 2 * ks_bound(ora)
        # exact message part: phi_g(Dec(ct)) up to key-switch noise
        want = O.automorphism_coeff(np.array(ora.crt(ora.decrypt(ct, s)), dtype=np.int64), g)
        assert max(abs(x - int(y)) for x, y in zip(dec, want)) <= ks_bound(ora)
    # one step through the hoisted path equals the first entry bit for bit
    one = ora.rotate_hoisted(ct, steps[:1], rks[:1])
    assert np.array_equal(one[0], outs[0])


@pytest.mark.parametrize("plan", [None, "two", "full"])
@pytest.mark.parametrize("prm", PARAMS[:2])
def test_rotate_sum_trace(oracle_mod, prm, plan):
    """sum_t phi_{5^t}(X^k) = (N/2) X^k for k in {0, N/2}, 0 otherwise, so
    Dec(rotate_sum(ct)) = (N/2)(m_0 + m_{N/2} X^{N/2}) + key-switch noise."""
    O = oracle_mod
    ora, s, pk = make(O, **prm)
    N, L = ora.N, ora.log_n - 1
    plan = {None: [1] * L, "two": [2] + [1] * (L - 2), "full": [L]}[plan]
    rng = np.random.default_rng(11)
    m = rng.integers(-(1 << 16), 1 << 16, size=N)
    ct = ora.encrypt(5, 0, m[None], pk)[0]
    dec0 = ora.crt(ora.decrypt(ct, s))
    rks = [ora.rot_key(9, s, k) for k in ora.rotsum_steps(plan)]
    out = ora.rotate_sum(ct, plan, rks)
    dec = ora.crt(ora.decrypt(out, s))
    want = [0] * N
    want[0] = (N // 2) * dec0[0]
    want[N // 2] = (N // 2) * dec0[N // 2]
    bound = N * L * ks_bound(ora)
    assert max(abs(x - y) for x, y in zip(dec, want)) <= bound
    assert abs(dec[0] - want[0]) < abs(want[0]) * 1e-3 + bound


@pytest.mark.parametrize("prm", PARAMS[:2])
def test_masked_sum_exact(oracle_mod, prm):
    """Dec(sum_i ct_i * pt_i) = sum_i pt_i * Dec(ct_i) exactly (constant masks)."""
    O = oracle_mod
    ora, s, pk = make(O, **prm)
    N = ora.N
    n, ln = 3, 2
    rng = np.random.default_rng(12)
    m = rng.integers(-(1 << 20), 1 << 20, size=(n * ln, N))
    cts = ora.encrypt(5, 0, m, pk).reshape(n, ln, 2, ora.nq, N)
    w = [0, 1, 7]
    masks = np.stack([ora.signed_to_ntt(np.array([w[i]] + [0] * (N - 1))) for i in range(n)])
    agg = ora.masked_sum(cts, masks)
    Q = 1
    for q in ora.q:
        Q *= q
    for k in range(ln):
        decs = [ora.crt(ora.decrypt(cts[i, k], s)) for i in range(n)]
        want = [centered(sum(w[i] * decs[i][t] for i in range(n)), Q) for t in range(N)]
        assert ora.crt(ora.decrypt(agg[k], s)) == want


# ---- rescaling (levels of the CKKS Scheme Description) ------------------------

def _residues(ints, mods):
    return np.array([[v % q for v in ints] for q in mods], dtype=np.uint64)


@pytest.mark.parametrize("prm", PARAMS)
def test_rescale_exact_multiples_and_rounding(oracle_mod, prm):
    """Closed forms of rounding division: rescaling q_t x + d with |d| < q_t / 2
    gives x exactly, for every level and integer polynomials x filling most of
    Q_{t-1} (both signs)."""
    O = oracle_mod
    ora = O.Oracle(prm["log_n"], prm["q_bits"], prm["p_bits"])
    rng = np.random.default_rng(11)
    N = ora.N
    for nlimb in range(2, ora.nq + 1):
        mods = [int(q) for q in ora.q[:nlimb]]
        qt = mods[-1]
        Qlow = 1
        for q in mods[:-1]:
            Qlow *= q
        comps = []
        want = []
        for comp in range(2):
            x = [int(rng.integers(-(1 << 62), 1 << 62)) * int(rng.integers(0, 1 << 20)) % Qlow for _ in range(N)]
            x = [v - Qlow if v > Qlow // 2 else v for v in x]
            d = [int(rng.integers(-(qt // 2), qt // 2 + 1)) for _ in range(N)]
            d[0], d[1] = qt // 2, -(qt // 2)  # the extremes of the rounding interval
            c = [qt * a + b for a, b in zip(x, d)]
            comps.append(ora.poly_ntt(_residues(c, mods)))
            want.append(x)
        ct = np.stack(comps)
        got = ora.rescale(ct, nlimb)
        assert got.shape == (2, nlimb - 1, N)
        for comp in range(2):
            vals = O.crt_centered(ora.poly_intt(got[comp]), mods[:-1])
            assert vals == want[comp], (nlimb, comp)


def test_rescale_of_encryption_decrypts_to_quotient(oracle_mod):
    """Encrypt m q_t (scale Delta q_t) and rescale: the decryption at the lower
    level is m up to (fresh noise) / q_t plus the rounding term (1 + ||s||_1) / 2."""
    O = oracle_mod
    ora, s, pk = make(O, log_n=6, q_bits=(45, 40, 40, 40, 40), p_bits=(46, 46))
    N, t = ora.N, ora.nq - 1
    qt = int(ora.q[t])
    rng = np.random.default_rng(4)
    m = rng.integers(-(1 << 20), 1 << 20, size=N)
    mq = np.array([int(v) * qt for v in m], dtype=object)
    # the plaintext m q_t exceeds int64, so encrypt it through its residues
    pt = ora.poly_ntt(_residues([int(v) for v in mq], ora.q))
    zero = ora.encrypt(8, 0, np.zeros((1, N), dtype=np.int64), pk)[0]
    ct = zero.copy()
    for l, q in enumerate(ora.q):
        ct[0, l] = [(int(a) + int(b)) % int(q) for a, b in zip(zero[0, l], pt[l])]
    rs = ora.rescale(ct)
    sh = ora.signed_to_ntt(s, t)
    low = [int(q) for q in ora.q[:t]]
    dec = ora.poly_intt(np.array([[(int(a) + int(b) * int(c)) % q for a, b, c in zip(rs[0, l], rs[1, l], sh[l])]
                                  for l, q in enumerate(low)], dtype=np.uint64))
    vals = O.crt_centered(dec, low)
    bound = 1 + (1 + N) / 2  # noise / q_t < 1, rounding of both components
    assert max(abs(v - int(x)) for v, x in zip(vals, m)) <= bound
