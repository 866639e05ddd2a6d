"""GPU parity: every device call of the C ABI against the CPU oracle on the
same seeded inputs, bit for bit.

Inputs are the oracle's (its encryptions, or synthetic residues from
synth); the GPU never supplies an expected value.  Sizes span several NTT
tiles and the ragged tails of the workloads.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def L():
    from paper_2408_06197_amd import lancelot
    lancelot.lib()
    return lancelot


def up(torch, arr):
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.uint64).view(np.int64)).cuda()


def down(t):
    return t.cpu().numpy().view(np.uint64)


def make_pair(L, O, log_n, qb, pb, seed, steps=(), log_m=0):
    """GPU context (KGC role) and oracle with the same parameters and keys."""
    ctx = L.Context(log_n, qb, pb, log_m=log_m, device=0)
    ctx.keygen(seed)
    if steps:
        ctx.keygen_rotation(seed, list(steps))
    ora = O.Oracle(log_n, qb, pb, log_m=(log_m or None))
    assert ora.primes == ctx.moduli
    s = ora.secret(seed)
    keys = {"s": s, "pk": ora.pk(seed, s), "rlk": ora.relin_key(seed, s)}
    keys["rot"] = {k: ora.rot_key(seed, s, k) for k in steps}
    return ctx, ora, keys


TINY = (5, (30, 28, 28), (30,))
TINY_A2 = (6, (45, 40, 40, 40, 40), (46, 46))
CFG1 = (synth.CFG1.log_n, synth.CFG1.q_bits, synth.CFG1.p_bits)
K8 = (10, (50,) * 16, (50,) * 8)  # eight special primes: digits of 8 limbs (dnum 2), ModDown from 8 limbs


# ---- NTT ---------------------------------------------------------------------

@pytest.mark.parametrize("log_n", [3, 4, 5, 8, 11, 12, 13, 14, 15, 16, 17])
def test_ntt_bitexact(torch, L, oracle_mod, log_n):
    O = oracle_mod
    qb, pb = (50, 50, 40), (50, 45)
    ctx = L.Context(log_n, qb, pb, device=0)
    ora = O.Oracle(log_n, qb, pb)
    count = 3 if log_n <= 14 else 2
    x = synth.uniform_residues(1000 + log_n, ctx.moduli, (count, 1 << log_n))  # [count][ne][N]
    g = up(torch, x)
    ctx.ntt_fwd(g, nlimb=ctx.ne)
    got = down(g)
    for c in range(count):
        want = np.vstack([ora.poly_ntt(x[c][l:l + 1], l) for l in range(ctx.ne)])
        assert np.array_equal(got[c], want), (log_n, c)
    ctx.ntt_inv(g, nlimb=ctx.ne)
    assert np.array_equal(down(g), x)
    # only the special-prime limbs (limb0 = n_q)
    y = np.ascontiguousarray(x[:, ctx.nq:, :])
    gy = up(torch, y)
    ctx.ntt_fwd(gy, nlimb=ctx.np, limb0=ctx.nq)
    want = np.vstack([ora.poly_ntt(y[0][k:k + 1], ctx.nq + k) for k in range(ctx.np)])
    assert np.array_equal(down(gy)[0], want)


def test_ntt_mixed_degree_chain(torch, L, oracle_mod):
    """Primes = 1 mod 2^17 for every degree (the mixed-degree micro-workload's chain)."""
    O = oracle_mod
    for log_n in (12, 14, 16):
        ctx = L.Context(log_n, (50, 50, 50), (50,), log_m=17, device=0)
        ora = O.Oracle(log_n, (50, 50, 50), (50,), log_m=17)
        x = synth.uniform_residues(7 + log_n, ctx.moduli[:3], (2, 1 << log_n))
        g = up(torch, x)
        ctx.ntt_fwd(g, nlimb=3)
        for c in range(2):
            assert np.array_equal(down(g)[c], ora.poly_ntt(x[c]))


def test_ntt_micro_workload_sampled(torch, L, oracle_mod):
    """The mixed-degree micro-workload at full size, in the launch
    configuration bench.py times: sampled polys of every degree against the
    oracle, the inverse restoring every poly exactly, the same bits with the
    two passes run per sub-batch."""
    import bench
    O = oracle_mod
    ctxs = bench.d4_contexts(L)
    polys = bench.d4_polys(torch, ctxs, 4004)
    keep = [(x.clone(), None if y is None else y.clone()) for x, y in polys]
    bench.d4_ntt(ctxs, polys)
    for ctx, (x, y), (a, b), (ln, cnt, nq, k) in zip(ctxs, polys, keep, bench.D4):
        ora = O.Oracle(ln, (50,) * nq, (50,) * k, log_m=17)
        assert ora.primes == ctx.moduli
        g = x.shape[0]
        for grp in (0, g // 2, g - 1):
            src, got = down(a[grp]), down(x[grp])
            for l in (0, nq - 1):
                assert np.array_equal(got[l], ora.poly_ntt(src[l:l + 1], l)[0]), (ln, grp, l)
        if y is not None:
            src, got = down(b[0]), down(y[0])
            r = src.shape[0]
            assert np.array_equal(got[r - 1], ora.poly_ntt(src[r - 1:r], r - 1)[0]), (ln, "tail")
    fwd = [(x.clone(), None if y is None else y.clone()) for x, y in polys]
    bench.d4_ntt(ctxs, polys, inverse=True)
    for (x, y), (a, b) in zip(polys, keep):
        assert torch.equal(x, a) and (y is None or torch.equal(y, b))
    for c in ctxs:
        c.set_tuning("ntt_sub_kb", 32768)
    bench.d4_ntt(ctxs, polys)
    for (x, y), (a, b) in zip(polys, fwd):
        assert torch.equal(x, a) and (y is None or torch.equal(y, b))


def test_hoisted_keyswitch_micro_sampled(torch, L, oracle_mod):
    """dnum = 3 hoisted rotations of the micro-workload's c1's (2^12 and
    2^14 chains, all log2(N/2) steps) against the oracle on sampled c1's."""
    import bench
    O = oracle_mod
    for ln, cnt, nq, k in bench.D4[:2]:
        ctx = L.Context(ln, (50,) * nq, (50,) * k, log_m=17, device=0)
        ora = O.Oracle(ln, (50,) * nq, (50,) * k, log_m=17)
        assert ctx.dnum == 3
        steps = bench.d4_rotation_steps(ln)
        ctx.keygen(4104)
        ctx.keygen_rotation(4104, steps)
        s = ora.secret(4104)
        rks = [ora.rot_key(4104, s, t) for t in steps]
        ct = synth.uniform_residues(ln, ctx.q, (6, 2, ctx.N))
        out = down(ctx.rotate_hoisted(up(torch, ct), steps))
        for c in (0, 5):
            want = ora.rotate_hoisted(ct[c], steps, rks)
            assert np.array_equal(out[c], want), (ln, c)


# ---- keys, encryption, decryption ---------------------------------------------

@pytest.mark.parametrize("prm", [TINY, TINY_A2, CFG1])
def test_keys_bitexact(torch, L, oracle_mod, prm):
    steps = [1, 2, 3, -1]
    ctx, ora, keys = make_pair(L, oracle_mod, *prm, seed=2001, steps=steps)
    assert np.array_equal(ctx.secret(), keys["s"])
    assert np.array_equal(ctx.pk(), keys["pk"])
    assert np.array_equal(ctx.ksk(0), keys["rlk"])
    for k in steps:
        assert np.array_equal(ctx.ksk(1, k), keys["rot"][k]), k


@pytest.mark.parametrize("prm", [TINY, TINY_A2, CFG1])
def test_encrypt_decrypt_bitexact(torch, L, oracle_mod, prm):
    O = oracle_mod
    ctx, ora, keys = make_pair(L, O, *prm, seed=5)
    rng = np.random.default_rng(3)
    m = rng.integers(-(1 << 40), 1 << 40, size=(5, ctx.N), dtype=np.int64)
    want = ora.encrypt(77, 1000, m, keys["pk"])
    got = ctx.encrypt(torch.from_numpy(m).cuda(), seed=77, first_object=1000)
    assert np.array_equal(down(got), want)
    dec = down(ctx.decrypt(got))
    for t in range(5):
        assert np.array_equal(dec[t], ora.decrypt(want[t], keys["s"]))
    # triples
    t3 = ora.mul(want[0], want[1])
    d3 = down(ctx.decrypt(up(torch, t3[None]), ncomp=3))[0]
    assert np.array_equal(d3, ora.decrypt(t3, keys["s"]))


# ---- element-wise ---------------------------------------------------------------

@pytest.mark.parametrize("prm", [TINY, CFG1])
def test_elementwise_bitexact(torch, L, oracle_mod, prm):
    O = oracle_mod
    ctx, ora, keys = make_pair(L, O, *prm, seed=9)
    rng = np.random.default_rng(4)
    m = rng.integers(-(1 << 30), 1 << 30, size=(6, ctx.N), dtype=np.int64)
    cts = ora.encrypt(1, 0, m, keys["pk"])
    a, b = up(torch, cts[:3]), up(torch, cts[3:])
    sub, add = down(ctx.ct_sub(a, b)), down(ctx.ct_add(a, b))
    mul, sq = down(ctx.ct_mul(a, b)), down(ctx.ct_square(a))
    for t in range(3):
        assert np.array_equal(sub[t], ora.sub(cts[t], cts[3 + t]))
        assert np.array_equal(add[t], ora.add(cts[t], cts[3 + t]))
        assert np.array_equal(mul[t], ora.mul(cts[t], cts[3 + t]))
        assert np.array_equal(sq[t], ora.mul(cts[t], cts[t]))
    # three-component add (lazy accumulation of triples)
    acc = down(ctx.ct_add(ctx.ct_mul(a, b), ctx.ct_square(a), ncomp=3))
    assert np.array_equal(acc[1], ora.add(ora.mul(cts[1], cts[4]), ora.mul(cts[1], cts[1])))
    # plaintext multiply and masked aggregation
    pts = synth.uniform_residues(5, ctx.q, (3, ctx.N))
    mp = down(ctx.mul_plain(a, up(torch, pts)))
    for t in range(3):
        assert np.array_equal(mp[t], ora.mul_plain(cts[t], pts[t]))
    client_cts = cts.reshape(3, 2, 2, ctx.nq, ctx.N)
    masks = np.stack([ora.signed_to_ntt(np.array([w] + [0] * (ctx.N - 1))) for w in (0, 1, 5)])
    ms = down(ctx.masked_sum(up(torch, client_cts), up(torch, masks)))
    assert np.array_equal(ms, ora.masked_sum(client_cts, masks))


def test_elementwise_aliasing(torch, L, oracle_mod):
    """In-place element-wise calls equal their out-of-place results; outputs that overlap an input any
    other way (shifted, or of another layout) are rejected before anything runs."""
    O = oracle_mod
    ctx, ora, keys = make_pair(L, O, *TINY, seed=9)
    rng = np.random.default_rng(5)
    m = rng.integers(-(1 << 20), 1 << 20, size=(8, ctx.N), dtype=np.int64)
    cts = up(torch, ora.encrypt(1, 0, m, keys["pk"]))  # [8][2][nq][N]
    a, b = cts[:3].clone(), cts[3:6].clone()
    want_sub, want_add = ctx.ct_sub(a, b), ctx.ct_add(a, b)
    x = a.clone()
    ctx.ct_sub(x, b, out=x)
    assert torch.equal(x, want_sub)
    y = b.clone()
    ctx.ct_add(a, y, out=y)
    assert torch.equal(y, want_add)
    pts = up(torch, synth.uniform_residues(6, ctx.q, (3, ctx.N)))
    want_mp = ctx.mul_plain(a, pts)
    z = a.clone()
    ctx.mul_plain(z, pts, out=z)
    assert torch.equal(z, want_mp)
    S = 2 * ctx.nq * ctx.N  # words per ciphertext
    flat = cts.clone().view(-1)

    def view(off, count, ncomp=2):
        return flat[off: off + count * ncomp * ctx.nq * ctx.N].view(count, ncomp, ctx.nq, ctx.N)

    bad = [
        lambda: ctx.ct_sub(view(0, 3), view(3 * S, 3), out=view(S // 2, 3)),      # shifted over a
        lambda: ctx.ct_add(view(0, 3), view(3 * S, 3), out=view(3 * S + 8, 3)),  # shifted over b
        lambda: ctx.ct_square(view(0, 2), out=view(0, 2, 3)),                   # another layout
        lambda: ctx.ct_mul(view(0, 2), view(2 * S, 2), out=view(2 * S, 2, 3)),
        lambda: ctx.mul_plain(view(0, 2), view(2 * S, 1), out=view(2 * S, 2)),  # over pt
        lambda: ctx.masked_sum(view(0, 4).view(2, 2, 2, ctx.nq, ctx.N), view(4 * S, 1),
                               out=view(S, 2)),
        lambda: ctx.pair_triples(view(0, 4).view(2, 2, 2, ctx.nq, ctx.N), out=view(2 * S, 1, 3)),
    ]
    before = flat.clone()
    for i, f in enumerate(bad):
        with pytest.raises(L.LancelotError) as e:
            f()
        assert e.value.code == L.LC_EINVAL, i
    torch.cuda.synchronize()
    assert torch.equal(flat, before)  # nothing was launched


@pytest.mark.parametrize("shape", [0, 1, 2])
@pytest.mark.parametrize("log_n,n,ln", [(6, 11, 9), (9, 8, 8), (12, 17, 3)])
def test_masked_sum_shapes_bitexact(torch, L, oracle_mod, log_n, n, ln, shape):
    """Masked aggregation with full-range masks: client groups of 8 with a
    ragged last group, (k, comp) row blocks with a ragged last block, and a
    limb-coefficient range that ends inside a workgroup (N = 2^6)."""
    O = oracle_mod
    prm = (log_n, (50, 45, 40), (50,))
    ctx = L.Context(*prm, device=0)
    ora = O.Oracle(*prm)
    cts = synth.uniform_residues(300 + n, ctx.q, (n, ln, 2, ctx.N))
    masks = synth.uniform_residues(400 + n, ctx.q, (n, ctx.N))
    ctx.set_tuning("ms_shape", shape)
    got = down(ctx.masked_sum(up(torch, cts), up(torch, masks)))
    assert np.array_equal(got, ora.masked_sum(cts, masks))


@pytest.mark.parametrize("prm,n,ln", [(TINY_A2, 5, 3), (CFG1, 3, 11)], ids=["n64", "n4096"])
def test_mask_aggregate_bitexact(torch, L, oracle_mod, prm, n, ln):
    """ServerUpdate with encrypted masks: sum_i ct_i[k] (x) M_i relinearized,
    against the oracle's own tensor, add and relinearization; and at decrypt
    level the weighted sum of the clients' plaintexts, at scale 2^25 x 2^25
    (fresh-noise products are about 2^-11 of that)."""
    from paper_2408_06197_amd import robust
    O = oracle_mod
    ctx, ora, keys = make_pair(L, O, *prm, seed=31)
    rng = np.random.default_rng(12)
    x = rng.uniform(-1, 1, size=(n * ln, ctx.N))
    m = np.round(x * 2.0 ** 25).astype(np.int64)
    cts = ora.encrypt(6, 0, m, keys["pk"]).reshape(n, ln, 2, ctx.nq, ctx.N)
    w = robust.weights("multikrum", [0, n - 1], n)
    mk = ora.encrypt(7, 10_000, robust.mask_plaintexts(w, ctx.N, 2.0 ** 25), keys["pk"])
    got = down(ctx.mask_aggregate(up(torch, cts), up(torch, mk)))
    for k in (0, ln - 1):
        t = ora.mul(cts[0, k], mk[0])
        for i in range(1, n):
            t = ora.add(t, ora.mul(cts[i, k], mk[i]))
        assert np.array_equal(got[k], ora.relin(t, keys["rlk"])), k
    dec = down(ctx.decrypt(up(torch, got)))
    want = (x.reshape(n, ln, ctx.N) * w[:, None, None]).sum(0)
    for k in range(ln):
        vals = ctx.crt_to_double(dec[k][:, :16]) / 2.0 ** 50
        assert np.max(np.abs(vals - want[k, :16])) < 2.0 ** -6, k


# ---- key switching ---------------------------------------------------------------

@pytest.mark.parametrize("prm", [TINY, TINY_A2, CFG1])
def test_relin_bitexact(torch, L, oracle_mod, prm):
    O = oracle_mod
    ctx, ora, keys = make_pair(L, O, *prm, seed=11)
    rng = np.random.default_rng(6)
    m = rng.integers(-(1 << 20), 1 << 20, size=(6, ctx.N), dtype=np.int64)
    cts = ora.encrypt(2, 0, m, keys["pk"])
    t3 = np.stack([ora.mul(cts[i], cts[i + 3]) for i in range(3)])
    got = down(ctx.relin(up(torch, t3)))
    for i in range(3):
        assert np.array_equal(got[i], ora.relin(t3[i], keys["rlk"])), i


@pytest.mark.parametrize("prm,multi", [(TINY, 1), (TINY_A2, 1), (CFG1, 1), (CFG1, 0), (K8, 1), (K8, 0)],
                         ids=["n32", "n64_a2", "n4096", "n4096_per_key", "n1024_k8", "n1024_k8_per_key"])
def test_rotate_hoisted_bitexact(torch, L, oracle_mod, prm, multi):
    """Literal hoisted rotations against the oracle: from 2^10 on, through the
    inner product that stages each source tile once for all keys (multi 1)
    and through one gather per key (multi 0)."""
    O = oracle_mod
    steps = [1, 2, 5, -3]
    ctx, ora, keys = make_pair(L, O, *prm, seed=13, steps=steps)
    ctx.set_tuning("hoist_multi", multi)
    rng = np.random.default_rng(7)
    m = rng.integers(-(1 << 20), 1 << 20, size=(2, ctx.N), dtype=np.int64)
    cts = ora.encrypt(3, 0, m, keys["pk"])
    got = down(ctx.rotate_hoisted(up(torch, cts), steps))
    for c in range(2):
        want = ora.rotate_hoisted(cts[c], steps, [keys["rot"][k] for k in steps])
        assert np.array_equal(got[c], want), c


def test_rotate_hoisted_batches_and_key_groups(torch, L, oracle_mod):
    """The source-major form across its batch and key-group edges: 40
    ciphertexts (a workspace limit that holds 32 of them: batches of 32 and
    8; without it, one batch) and 11 steps (key groups of 8 and 3) give the
    per-key form's bits, and sampled outputs equal the oracle."""
    O = oracle_mod
    steps = [1, 2, 3, 4, 5, 7, 16, 64, -1, -9, 1000]
    ctx, ora, keys = make_pair(L, O, *CFG1, seed=31, steps=steps)
    cts = synth.uniform_residues(32, ctx.q, (40, 2, ctx.N))
    g = up(torch, cts)
    ctx.set_tuning("hoist_multi", 1)
    whole = down(ctx.rotate_hoisted(g, steps))
    per_ct = (ctx.nq + ctx.dnum * ctx.ne + 2 * 8 * ctx.ne + 2 * ctx.nq) * ctx.N * 8
    ctx.set_workspace_limit(32 * per_ct)
    multi = down(ctx.rotate_hoisted(g, steps))
    assert np.array_equal(multi, whole)
    ctx.set_tuning("hoist_multi", 0)
    per_key = down(ctx.rotate_hoisted(g, steps))
    assert np.array_equal(multi, per_key)
    rks = [keys["rot"][k] for k in steps]
    for c in (0, 31, 32, 39):
        want = ora.rotate_hoisted(cts[c], steps, rks)
        assert np.array_equal(multi[c], want), c


@pytest.mark.parametrize("plan", ["ones", "twos", "three"])
@pytest.mark.parametrize("prm", [TINY, TINY_A2, K8])
def test_rotate_sum_bitexact(torch, L, oracle_mod, prm, plan):
    O = oracle_mod
    levels = prm[0] - 1
    plan = {"ones": [1] * levels, "twos": [2] * (levels // 2) + [1] * (levels % 2),
            "three": [3] + [1] * (levels - 3)}[plan]
    ora0 = O.Oracle(*prm)
    steps = ora0.rotsum_steps(plan)
    ctx, ora, keys = make_pair(L, O, *prm, seed=17, steps=steps)
    rng = np.random.default_rng(8)
    m = rng.integers(-(1 << 20), 1 << 20, size=(3, ctx.N), dtype=np.int64)
    cts = ora.encrypt(4, 0, m, keys["pk"])
    g = up(torch, cts)
    ctx.rotate_sum(g, plan)
    got = down(g)
    for c in range(3):
        want = ora.rotate_sum(cts[c], plan, [keys["rot"][k] for k in steps])
        assert np.array_equal(got[c], want), c


@pytest.mark.parametrize("prm,plan", [(CFG1, (3, 3, 3, 2)), (CFG1, (2, 3, 3, 3)), (TINY_A2, (3, 2))],
                         ids=["n4096-3332", "n4096-2333", "n64-32"])
def test_rotate_sum_cycle_walk_bitexact(torch, L, oracle_mod, prm, plan):
    """Blocks of 3 and 7 rotations through the cycle-walking inner product
    (walks of the tile map up to 64 tiles long at N = 2^12; one tile at
    N = 64) and through the per-key gather, both equal to the oracle."""
    O = oracle_mod
    plan = list(plan)
    ora0 = O.Oracle(*prm)
    steps = ora0.rotsum_steps(plan)
    ctx, ora, keys = make_pair(L, O, *prm, seed=19, steps=steps)
    rng = np.random.default_rng(9)
    m = rng.integers(-(1 << 20), 1 << 20, size=(11, ctx.N), dtype=np.int64)  # 11: a ragged group of 8
    cts = ora.encrypt(5, 0, m, keys["pk"])
    want = [ora.rotate_sum(cts[c], plan, [keys["rot"][k] for k in steps]) for c in (0, 7, 10)]
    ctx.set_tuning("mac_cycle_min", 1)  # every block walks, even one-tile cycles
    # xcd: the workgroups of one key tile grouped on one XCD (two groups of
    # ciphertexts at 8 per workgroup, segment count padded)
    for cyc, cts_per_wg, fold, one, xcd in ((1, 8, 1, 1, 0), (1, 16, 1, 1, 0), (1, 8, 0, 1, 0), (1, 16, 0, 0, 0),
                                            (1, 8, 1, 0, 0), (0, 8, 1, 1, 0), (1, 8, 1, 1, 1), (1, 8, 0, 0, 1),
                                            (1, 8, 1, 0, 1)):
        ctx.set_tuning("mac_cycle", cyc)
        ctx.set_tuning("mac_cycle_cts", cts_per_wg)
        ctx.set_tuning("mac_short_cts", cts_per_wg)
        ctx.set_tuning("mac_cycle_c0", fold)
        ctx.set_tuning("mac_cycle_short", one)  # 1: cycles of <= 2 tiles take the no-walk kernel
        ctx.set_tuning("mac_xcd", xcd)
        g = up(torch, cts)
        ctx.rotate_sum(g, plan)
        got = down(g)
        for w, c in zip(want, (0, 7, 10)):
            assert np.array_equal(got[c], w), (cyc, cts_per_wg, fold, one, xcd, c)


def test_rotate_sum_cycle_walk_full_size(torch, L, oracle_mod):
    """N = 2^16, 24 + 4 limbs (dnum 6), the (3,3,3,3,3) plan that the bench
    autotunes to: cycles of the tile map up to 1024 tiles, several segments
    per cycle, and a last block (rotations by multiples of 2^12) whose tile
    map is the identity; two ciphertexts against the oracle."""
    O = oracle_mod
    prm = (16, (50,) * 24, (50,) * 4)
    plan = [3, 3, 3, 3, 3]
    ora0 = O.Oracle(*prm)
    steps = ora0.rotsum_steps(plan)
    ctx, ora, keys = make_pair(L, O, *prm, seed=23, steps=steps)
    cts = synth.uniform_residues(24, ctx.q, (2, 2, ctx.N))
    rks = [keys["rot"][k] for k in steps]
    want = [ora.rotate_sum(cts[c], plan, rks) for c in range(2)]
    # (shortest walked cycle, ciphertexts per workgroup, c0 folded, short cycles without a walk)
    for cmin, cts_per_wg, fold, one in ((1, 8, 1, 0), (1, 16, 0, 1), (16, 16, 1, 1), (16, 8, 0, 1)):
        ctx.set_tuning("mac_cycle_min", cmin)
        ctx.set_tuning("mac_cycle_cts", cts_per_wg)
        ctx.set_tuning("mac_short_cts", 24 - cts_per_wg)  # the other width
        ctx.set_tuning("mac_cycle_c0", fold)
        ctx.set_tuning("mac_cycle_short", one)
        g = up(torch, cts)
        ctx.rotate_sum(g, plan)
        got = down(g)
        for c in range(2):
            assert np.array_equal(got[c], want[c]), (cmin, cts_per_wg, fold, one, c)


def test_rotate_sum_n17_depth3(torch, L, oracle_mod):
    """N = 2^17 (the top of the packing-size sweep) on the depth-3 parameters:
    transforms outside the two-pass range and the key switch's unfused
    conversions, the 3,3,3,3,3,1 plan (cycle walks, short cycles and a single
    rotation); one ciphertext against the oracle."""
    O = oracle_mod
    prm = (17, (50, 40, 40, 40), (48,))
    plan = [3, 3, 3, 3, 3, 1]
    ora0 = O.Oracle(*prm)
    steps = ora0.rotsum_steps(plan)
    ctx, ora, keys = make_pair(L, O, *prm, seed=29, steps=steps)
    cts = synth.uniform_residues(31, ctx.q, (1, 2, ctx.N))
    want = ora.rotate_sum(cts[0], plan, [keys["rot"][k] for k in steps])
    g = up(torch, cts)
    ctx.rotate_sum(g, plan)
    assert np.array_equal(down(g)[0], want)


# ---- the pairwise pipeline -----------------------------------------------------------

def encrypt_workload(O, ora, keys, w, seed):
    upd = synth.client_updates(w)
    scale = 2.0 ** w.scale_log2
    m = np.stack([np.stack([O.encode(ch, w.log_n, scale) for ch in synth.pack(u, w.slots)]) for u in upd])
    n, ln = m.shape[:2]
    cts = ora.encrypt(seed, 0, m.reshape(n * ln, w.N), keys["pk"]).reshape(n, ln, 2, ora.nq, w.N)
    return upd, m, cts


def fp64_dists(upd):
    n = upd.shape[0]
    return np.array([np.sum((upd[i] - upd[j]) ** 2) for i in range(n) for j in range(i + 1, n)])


TINY_W = synth.small_workload(log_n=5, q_bits=(45, 40, 40), p_bits=(45,), n_clients=4, dim=40, scale_log2=30)
TINY_W5 = synth.small_workload(log_n=6, q_bits=(50, 45, 45, 45), p_bits=(50, 50), n_clients=5, dim=100,
                               scale_log2=35, name="tiny5")
TWO_W = synth.small_workload(log_n=6, q_bits=(50, 45, 45), p_bits=(50,), n_clients=2, dim=32, scale_log2=30,
                             name="two-clients-one-ct")
# N = 2^10 (the two-pass NTT), 4 limbs in 2 digits, 3 clients x 2 ciphertexts
KS_W = synth.small_workload(log_n=10, q_bits=(50, 45, 45, 45), p_bits=(50, 50), n_clients=3, dim=700,
                            scale_log2=35, name="ks-tuning")


@pytest.mark.parametrize("w", [TINY_W, TINY_W5, TWO_W, synth.CFG1], ids=lambda w: w.name)
def test_pairwise_pipeline_bitexact(torch, L, oracle_mod, w):
    O = oracle_mod
    ora0 = O.Oracle(w.log_n, w.q_bits, w.p_bits)
    steps = ora0.rotsum_steps(w.rot_plan)
    ctx, ora, keys = make_pair(L, O, w.log_n, w.q_bits, w.p_bits, seed=w.crypto_seed, steps=steps)
    upd, m, cts = encrypt_workload(O, ora, keys, w, w.crypto_seed + 1)
    # GPU encryption of the same plaintexts gives the same ciphertexts
    gcts = ctx.encrypt(torch.from_numpy(m.reshape(-1, w.N)).cuda(), seed=w.crypto_seed + 1)
    assert np.array_equal(down(gcts).reshape(cts.shape), cts)
    res = ora.pairwise(cts, keys["rlk"], list(w.rot_plan), [keys["rot"][k] for k in steps], want_triples=True)
    g = up(torch, cts)
    trip = down(ctx.pair_triples(g))
    assert np.array_equal(trip, res["triples"])
    dist, sumdis = ctx.pairwise_sqdist(g, plan=list(w.rot_plan), sumdis=True)
    assert np.array_equal(down(dist), res["dist"])
    assert np.array_equal(down(sumdis), res["sumdis"])
    # decrypted distances against FP64 (rtol 1e-3 at scale <= 2^35)
    dec = down(ctx.decrypt(dist))
    scale2 = 2.0 ** (2 * w.scale_log2)
    got = ctx.crt_to_double(dec[:, :, 0].T.copy()) / scale2
    assert np.allclose(got, fp64_dists(upd), rtol=1e-3)


@pytest.mark.parametrize("n,ln", [(40, 3), (64, 2), (13, 9)])
def test_pair_triples_many_clients(torch, L, oracle_mod, n, ln):
    """Pair chunking across workgroups and the LDS staging cap (40 and 64
    clients), ragged staging of packed ciphertexts (9 = 2 * 4 + 1)."""
    O = oracle_mod
    prm = (5, (50, 45, 40), (50,))
    ctx = L.Context(*prm, device=0)
    ora = O.Oracle(*prm)
    cts = synth.uniform_residues(31 + n, ctx.q, (n, ln, 2, ctx.N))
    got = down(ctx.pair_triples(up(torch, cts)))
    P = n * (n - 1) // 2
    p = 0
    for i in range(n):
        for j in range(i + 1, n):
            if p % 7 == 0 or p == P - 1:
                assert np.array_equal(got[p], ora.pair_triple(cts, i, j)), (i, j)
            p += 1


@pytest.mark.parametrize("lanes,ppt", [(8, 1), (16, 3), (16, 4), (32, 6), (64, 6)])
def test_pair_tuning_shapes_bitexact(torch, L, oracle_mod, lanes, ppt):
    """Every pair-kernel launch shape gives the oracle's bits (13 clients:
    78 pairs, so more than one pair per lane; 6 ciphertexts: a ragged LDS
    batch)."""
    O = oracle_mod
    prm = (6, (50, 45, 40), (50,))
    ctx = L.Context(*prm, device=0)
    ora = O.Oracle(*prm)
    n, ln = 13, 6
    cts = synth.uniform_residues(77, ctx.q, (n, ln, 2, ctx.N))
    ctx.set_tuning("pair_mfma", 0)  # the per-pair kernel's shapes
    ctx.set_tuning("pair_lanes", lanes)
    ctx.set_tuning("pair_ppt", ppt)
    got = down(ctx.pair_triples(up(torch, cts)))
    p = 0
    for i in range(n):
        for j in range(i + 1, n):
            if p % 5 == 0 or p == n * (n - 1) // 2 - 1:
                assert np.array_equal(got[p], ora.pair_triple(cts, i, j)), (lanes, ppt, i, j)
            p += 1


@pytest.mark.parametrize("log_n", [12, 16])
def test_ntt_sub_batches_bitexact(torch, L, oracle_mod, log_n):
    """Two-pass NTTs run per sub-batch (64 KiB: one limb group at a time) give the same bits as the whole batch and the oracle."""
    O = oracle_mod
    qb, pb = (50, 50, 40), (50, 45)
    ctx = L.Context(log_n, qb, pb, device=0)
    ora = O.Oracle(log_n, qb, pb)
    x = synth.uniform_residues(2000 + log_n, ctx.moduli, (5, 1 << log_n))
    ctx.set_tuning("ntt_sub_kb", 64)
    g = up(torch, x)
    ctx.ntt_fwd(g, nlimb=ctx.ne)
    got = down(g)
    for c in (0, 4):
        want = np.vstack([ora.poly_ntt(x[c][l:l + 1], l) for l in range(ctx.ne)])
        assert np.array_equal(got[c], want), c
    ctx.ntt_inv(g, nlimb=ctx.ne)
    assert np.array_equal(down(g), x)


def test_ks_tuning_bitexact(torch, L, oracle_mod):
    """The pipeline's key switches with one- and three-ciphertext chunks,
    alternating over two streams or all on one, tiny NTT sub-batches (whole
    digit groups with own-digit limbs skipped), the base conversions fused
    into the transforms or not, and XCD-grouped inner-product workgroups give
    the oracle's bits, under a plan of nine blocks (the relinearization writes
    the rotate buffer and the blocks end in the distances) and one of four
    (the relinearization writes the distances)."""
    O = oracle_mod
    w = KS_W
    ora0 = O.Oracle(w.log_n, w.q_bits, w.p_bits)
    plans = (list(w.rot_plan), [3, 3, 2, 1])
    steps = sorted(set(st for pl in plans for st in ora0.rotsum_steps(pl)))
    ctx, ora, keys = make_pair(L, O, w.log_n, w.q_bits, w.p_bits, seed=w.crypto_seed, steps=steps)
    upd, m, cts = encrypt_workload(O, ora, keys, w, w.crypto_seed + 1)
    for plan in plans:
        res = ora.pairwise(cts, keys["rlk"], plan, [keys["rot"][k] for k in ora0.rotsum_steps(plan)])
        for chunk, sub, mac, fuse, streams, xcd in ((1, 64, 8, 1, 2, 0), (3, 64, 16, 0, 2, 1), (64, 0, 16, 1, 2, 1),
                                                    (64, 0, 8, 0, 2, 0), (3, 64, 8, 1, 2, 0), (3, 0, 16, 1, 1, 1),
                                                    (1, 0, 8, 1, 1, 0)):
            ctx.set_tuning("ks_chunk", chunk)
            ctx.set_tuning("ntt_sub_kb", sub)
            ctx.set_tuning("mac_cts", mac)
            ctx.set_tuning("fuse_modup", fuse)
            ctx.set_tuning("ks_streams", streams)
            ctx.set_tuning("mac_xcd", xcd)
            dist = ctx.pairwise_sqdist(up(torch, cts), plan=plan)
            assert np.array_equal(down(dist), res["dist"]), (plan, chunk, sub, mac, fuse, streams, xcd)


def test_set_tuning_rejects_bad_values(L):
    ctx = L.Context(5, (30, 28, 28), (30,), device=0)
    for name, value in (("pair_lanes", 12), ("pair_ppt", 5), ("pair_mfma", 3), ("ks_chunk", 0), ("ntt_sub_kb", -1), ("mac_cts", 4),
                        ("mac_cycle", 2), ("mac_cycle_min", 0), ("fuse_modup", 3), ("ms_shape", 3),
                        ("mac_cycle_cts", 12), ("mac_cycle_c0", 2), ("mac_cycle_short", 2), ("mac_short_cts", 4),
                        ("ks_streams", 3), ("mac_xcd", 2), ("hoist_multi", 2), ("nope", 1)):
        with pytest.raises(L.LancelotError):
            ctx.set_tuning(name, value)


def test_full_round_krum(torch, L, oracle_mod):
    """Algorithm 1 end to end at N = 2^12 (4 clients, one packed ciphertext
    each, client 3 Byzantine x10): device pipeline, KGC decryption and Krum,
    encrypted one-hot mask, lc_mask_aggregate, KGC decryption of the model,
    which equals the chosen client's update within the scheme's noise."""
    from paper_2408_06197_amd import robust
    O = oracle_mod
    w = synth.CFG1
    ora0 = O.Oracle(w.log_n, w.q_bits, w.p_bits)
    steps = ora0.rotsum_steps(w.rot_plan)
    ctx, ora, keys = make_pair(L, O, w.log_n, w.q_bits, w.p_bits, seed=w.crypto_seed, steps=steps)
    upd, m, cts = encrypt_workload(O, ora, keys, w, w.crypto_seed + 1)
    g = up(torch, cts)
    dist = ctx.pairwise_sqdist(g, plan=list(w.rot_plan))
    dec = down(ctx.decrypt(dist))
    scale = 2.0 ** w.scale_log2
    got = ctx.crt_to_double(np.ascontiguousarray(dec[:, :, 0].T)) / scale ** 2
    chosen = robust.select("krum", robust.distance_matrix(got, w.n_clients), w.n_byz)
    assert chosen == robust.select("krum", robust.distance_matrix(fp64_dists(upd), w.n_clients), w.n_byz)
    assert chosen[0] < w.n_clients - w.n_byz
    wts = robust.weights("krum", chosen, w.n_clients)
    mask = ctx.encrypt(torch.from_numpy(robust.mask_plaintexts(wts, ctx.N, scale)).cuda(), seed=9,
                       first_object=1 << 40)
    agg = ctx.mask_aggregate(g, mask)
    z = ctx.decode(down(ctx.decrypt(agg))[0], scale * scale).real
    want = np.zeros(w.slots)
    want[: w.dim] = upd[chosen[0]][: w.slots]
    assert np.max(np.abs(z - want)) < 1e-4


def test_chunked_triples_and_finish(torch, L, oracle_mod):
    """Streaming the packed ciphertexts in chunks of k (accumulating triples)
    then finishing gives the same bits as the one-shot pipeline and the oracle;
    the same work on two streams at once gives the same bits again."""
    O = oracle_mod
    w = TINY_W5
    ora0 = O.Oracle(w.log_n, w.q_bits, w.p_bits)
    steps = ora0.rotsum_steps(w.rot_plan)
    ctx, ora, keys = make_pair(L, O, w.log_n, w.q_bits, w.p_bits, seed=w.crypto_seed, steps=steps)
    upd, m, cts = encrypt_workload(O, ora, keys, w, w.crypto_seed + 1)
    res = ora.pairwise(cts, keys["rlk"], list(w.rot_plan), [keys["rot"][k] for k in steps], want_triples=True)
    g = up(torch, cts)
    n, ln = cts.shape[:2]
    P = n * (n - 1) // 2
    trip = torch.zeros((P, 3, ctx.nq, ctx.N), dtype=torch.int64, device="cuda")
    for k0 in range(0, ln, 1):  # one packed ciphertext per chunk
        ctx.pair_triples_acc(g[:, k0:k0 + 1].contiguous(), trip)
    assert np.array_equal(down(trip), res["triples"])
    dist, sd = ctx.pairwise_finish(trip, n, plan=list(w.rot_plan), sumdis=True)
    assert np.array_equal(down(dist), res["dist"])
    assert np.array_equal(down(sd), res["sumdis"])
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for st in (s1, s2):
        with torch.cuda.stream(st):
            outs.append(ctx.pairwise_sqdist(g, plan=list(w.rot_plan), stream=st))
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(down(o), res["dist"])


def test_cfg2_sampled_pairs(torch, L, oracle_mod):
    """N=2^14, 8 limbs, 10 clients x 13 ciphertexts (ragged last one): all 45
    distances decrypt to FP64 within 1e-4; three pairs are bit-exact against
    the oracle, chosen to cover the first, a middle and the last pair."""
    O = oracle_mod
    w = synth.CFG2
    ora0 = O.Oracle(w.log_n, w.q_bits, w.p_bits)
    steps = ora0.rotsum_steps(w.rot_plan)
    ctx, ora, keys = make_pair(L, O, w.log_n, w.q_bits, w.p_bits, seed=w.crypto_seed, steps=steps)
    upd, m, cts = encrypt_workload(O, ora, keys, w, w.crypto_seed + 1)
    g = up(torch, cts)
    dist = ctx.pairwise_sqdist(g, plan=list(w.rot_plan))
    sample = [0, 22, 44]
    res = ora.pairwise(cts, keys["rlk"], list(w.rot_plan), [keys["rot"][k] for k in steps], want_sumdis=False,
                       pairs=sample)
    gd = down(dist)
    for p in sample:
        assert np.array_equal(gd[p], res["dist"][p]), p
    dec = down(ctx.decrypt(dist))
    got = ctx.crt_to_double(dec[:, :, 0].T.copy()) / 2.0 ** (2 * w.scale_log2)
    assert np.allclose(got, fp64_dists(upd), rtol=1e-4)


# ---- error paths ----------------------------------------------------------------------

def test_error_paths(torch, L, oracle_mod):
    ctx = L.Context(*TINY, device=0)
    srv = L.Context(*TINY, device=0, role=L.ROLE_SERVER)
    with pytest.raises(L.LancelotError) as e:
        srv.keygen(1)
    assert e.value.code == L.LC_EKEY
    ctx.keygen(1)
    ctx.keys_share(srv)
    m = torch.zeros(1, ctx.N, dtype=torch.int64, device="cuda")
    ct = srv.encrypt(m, seed=1)  # a server context can encrypt with the shared pk
    with pytest.raises(L.LancelotError) as e:
        srv.decrypt(ct)
    assert e.value.code == L.LC_EKEY
    with pytest.raises(L.LancelotError) as e:
        srv.rotate_hoisted(ct, [1])
    assert e.value.code == L.LC_EKEY
    with pytest.raises(L.LancelotError) as e:
        srv.rotate_sum(ct, [1, 1, 1, 1])
    assert e.value.code == L.LC_EKEY
    with pytest.raises(L.LancelotError) as e:
        ctx.rotate_sum(ct, [2, 1])  # levels must sum to log_n - 1
    assert e.value.code == L.LC_EINVAL
    t3 = ctx.ct_square(ct)
    with pytest.raises(L.LancelotError) as e:
        ctx.relin(t3, out=t3.view(-1)[: 2 * ctx.nq * ctx.N].view(1, 2, ctx.nq, ctx.N))
    assert e.value.code == L.LC_EINVAL
    with pytest.raises(L.LancelotError) as e:
        ctx.pair_triples(torch.zeros(1, 1, 2, ctx.nq, ctx.N, dtype=torch.int64, device="cuda"))
    assert e.value.code == L.LC_EINVAL
    # the shared keys relinearize identically in both contexts
    a = ctx.relin(t3)
    b = srv.relin(t3)
    assert torch.equal(a, b)
