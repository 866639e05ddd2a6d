"""GPU parity of the boundary calls that take outside keys, mixed ring
degrees and per-client SumDis, against the CPU oracle on the same inputs:

  * lc_key_import: a server context that never ran key generation gets the
    oracle's public, relinearization and rotation keys and then encrypts,
    relinearizes, rotates and runs the whole distance pipeline bit for bit
    as the oracle does with those keys;
  * lc_ntt_fwd_groups / lc_ntt_inv_groups: polynomials of ring degrees
    2^12 .. 2^17 in one launch per pass equal the oracle's transform of each
    degree, and the inverse restores them;
  * lc_sumdis_lazy: per-client SumDis with one relinearization per client
    equals the oracle's composition of pair triples, sums, relinearization
    and rotate-and-sum;
  * lc_footprint: the workspace a resident round grows equals the figure it
    reports.
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


def oracle_keys(O, prm, seed, steps, log_m=None):
    ora = O.Oracle(*prm, log_m=log_m)
    s = ora.secret(seed)
    keys = {"s": s, "pk": ora.pk(seed, s), "rlk": ora.relin_key(seed, s),
            "rot": {k: ora.rot_key(seed, s, k) for k in steps}}
    return ora, keys


def server_with(L, prm, keys):
    """A server-role context holding only imported keys."""
    ctx = L.Context(*prm, device=0, role=L.ROLE_SERVER)
    ctx.key_import(L.KEY_PK, keys["pk"])
    ctx.key_import(L.KEY_RELIN, keys["rlk"])
    for k, v in keys["rot"].items():
        ctx.key_import(L.KEY_ROTATION, v, step=k)
    return ctx


TINY_A2 = (6, (45, 40, 40, 40, 40), (46, 46))
CFG1 = (synth.CFG1.log_n, synth.CFG1.q_bits, synth.CFG1.p_bits)


@pytest.mark.parametrize("prm", [TINY_A2, CFG1], ids=["n64_a2", "n4096"])
def test_imported_keys_pipeline(torch, L, oracle_mod, prm):
    O = oracle_mod
    log_n = prm[0]
    plan = [3] * ((log_n - 1) // 3) + ([(log_n - 1) % 3] if (log_n - 1) % 3 else [])
    extra = [1, -3]
    ora, keys = oracle_keys(O, prm, 515, sorted(set(ora_steps(plan)) | set(extra)))
    ctx = server_with(L, prm, keys)
    assert ora.primes == ctx.moduli
    # encryption with the imported public key
    rng = np.random.default_rng(3)
    n, ln = 5, 3
    m = rng.integers(-(1 << 30), 1 << 30, size=(n * ln, ctx.N), dtype=np.int64)
    cts = ctx.encrypt(torch.from_numpy(m).cuda(), seed=77, first_object=9)
    want_cts = ora.encrypt(77, 9, m, keys["pk"])
    assert np.array_equal(down(cts), want_cts)
    # relinearization and literal hoisted rotations
    t3 = synth.uniform_residues(41, ctx.q, (2, 3, ctx.N))
    got = down(ctx.relin(up(torch, t3)))
    for c in range(2):
        assert np.array_equal(got[c], ora.relin(t3[c], keys["rlk"])), c
    rot = down(ctx.rotate_hoisted(cts[:1].contiguous(), extra))
    assert np.array_equal(rot[0], ora.rotate_hoisted(want_cts[0], extra, [keys["rot"][k] for k in extra]))
    # the whole distance pipeline with SumDis
    cts5 = cts.view(n, ln, 2, ctx.nq, ctx.N)
    dist, sumdis = ctx.pairwise_sqdist(cts5, plan=plan, sumdis=True)
    rks = [keys["rot"][k] for k in ora_steps(plan)]
    res = ora.pairwise(want_cts.reshape(n, ln, 2, ora.nq, ora.N), keys["rlk"], plan, rks)
    assert np.array_equal(down(dist), res["dist"])
    assert np.array_equal(down(sumdis), res["sumdis"])


def ora_steps(plan):
    steps, j0 = [], 0
    for kb in plan:
        steps += [t << j0 for t in range(1, 1 << kb)]
        j0 += kb
    return steps


def test_key_import_rejects(torch, L, oracle_mod):
    ctx = L.Context(*TINY_A2, device=0, role=L.ROLE_SERVER)
    bad = np.zeros((ctx.dnum, 2, ctx.ne, ctx.N), dtype=np.uint64)
    bad[0, 0, 0, 0] = ctx.moduli[0]  # not canonical
    with pytest.raises(L.LancelotError) as e:
        ctx.key_import(L.KEY_RELIN, bad)
    assert e.value.code == L.LC_EINVAL
    with pytest.raises(L.LancelotError) as e:
        ctx.key_import(L.KEY_ROTATION, np.zeros_like(bad), step=ctx.N // 2)  # the identity
    assert e.value.code == L.LC_EINVAL
    with pytest.raises(L.LancelotError) as e:
        ctx.relin(ctx.empty(1, 3, ctx.nq, ctx.N))  # nothing imported yet
    assert e.value.code == L.LC_EKEY


# ---- mixed ring degrees in one launch per pass -----------------------------------

def test_ntt_groups_bitexact(torch, L, oracle_mod):
    """Degrees 2^12 .. 2^16 (ragged counts, limb offsets, a tail group of
    fewer limbs) in one call on a context of degree 2^16 whose primes are
    = 1 mod 2^17, against the oracle's transform of each degree."""
    O = oracle_mod
    qb, pb = (50,) * 24, (50,) * 8
    ctx = L.Context(16, qb, pb, log_m=17, device=0)
    spec = [(12, 3, 3, 0), (13, 2, 2, 5), (14, 2, 6, 0), (12, 1, 1, 30), (15, 1, 4, 20), (16, 2, 3, 1),
            (16, 1, 9, 0)]
    host, dev = [], []
    for k, (log_n, count, nlimb, limb0) in enumerate(spec):
        x = synth.uniform_residues(900 + k, ctx.moduli[limb0:limb0 + nlimb], (count, 1 << log_n))
        host.append(x)
        dev.append(up(torch, x))
    groups = [(t, ln, nl, l0) for t, (ln, _, nl, l0) in zip(dev, spec)]
    ctx.ntt_fwd_groups(groups)
    oras = {}
    for x, t, (log_n, count, nlimb, limb0) in zip(host, dev, spec):
        if log_n not in oras:
            oras[log_n] = O.Oracle(log_n, qb, pb, log_m=17)
            assert oras[log_n].primes == ctx.moduli
        got = down(t)
        for c in range(count):
            for l in range(nlimb):
                want = oras[log_n].poly_ntt(x[c][l:l + 1], limb0 + l)[0]
                assert np.array_equal(got[c][l], want), (log_n, c, l)
    ctx.ntt_inv_groups(groups)
    for x, t in zip(host, dev):
        assert np.array_equal(down(t), x)
    # the same bits as a context of each smaller degree with the same primes
    x = host[2]
    small = L.Context(14, qb, pb, log_m=17, device=0)
    g1, g2 = up(torch, x), up(torch, x)
    small.ntt_fwd(g1, nlimb=6)
    ctx.ntt_fwd_groups([(g2, 14, 6, 0)])
    assert torch.equal(g1, g2)


def test_ntt_groups_degree_2_17(torch, L, oracle_mod):
    """Degrees 2^17 (its second pass has 512-point sub-transforms in three
    register rounds) and 2^12 in one call on a degree-2^17 context."""
    O = oracle_mod
    qb, pb = (50,) * 3, (50,)
    ctx = L.Context(17, qb, pb, device=0)
    host = [synth.uniform_residues(71, ctx.moduli[:3], (2, 1 << 17)),
            synth.uniform_residues(72, ctx.moduli[1:3], (3, 1 << 12))]
    dev = [up(torch, x) for x in host]
    groups = [(dev[0], 17, 3, 0), (dev[1], 12, 2, 1)]
    ctx.ntt_fwd_groups(groups)
    o17, o12 = O.Oracle(17, qb, pb), O.Oracle(12, qb, pb, log_m=18)
    assert o17.primes == ctx.moduli and o12.primes == ctx.moduli
    for c in range(2):
        assert np.array_equal(down(dev[0])[c], o17.poly_ntt(host[0][c]))
    for c in range(3):
        assert np.array_equal(down(dev[1])[c], o12.poly_ntt(host[1][c], 1))
    ctx.ntt_inv_groups(groups)
    assert np.array_equal(down(dev[0]), host[0]) and np.array_equal(down(dev[1]), host[1])


def test_ntt_groups_rejects(torch, L):
    ctx = L.Context(14, (50,) * 3, (50,), log_m=17, device=0)
    x = ctx.empty(1, 1, 1 << 16)
    with pytest.raises(L.LancelotError) as e:
        ctx.ntt_fwd_groups([(x, 16, 1, 0)])  # above the context's degree
    assert e.value.code == L.LC_EUNSUP
    y = ctx.empty(1, 1, 1 << 11)
    with pytest.raises(L.LancelotError) as e:
        ctx.ntt_fwd_groups([(y, 11, 1, 0)])  # below 2^12
    assert e.value.code == L.LC_EUNSUP
    z = ctx.empty(1, 2, 1 << 12)
    with pytest.raises(L.LancelotError) as e:
        ctx.ntt_fwd_groups([(z, 12, 2, 3)])  # limbs past the basis
    assert e.value.code == L.LC_EINVAL


# ---- per-client SumDis -------------------------------------------------------------

@pytest.mark.parametrize("prm,n,ln,plan", [(TINY_A2, 5, 3, (3, 2)), (CFG1, 4, 2, (3, 3, 3, 2))],
                         ids=["n64", "n4096"])
def test_sumdis_lazy_bitexact(torch, L, oracle_mod, prm, n, ln, plan):
    O = oracle_mod
    plan = list(plan)
    ora, keys = oracle_keys(O, prm, 616, ora_steps(plan))
    ctx = server_with(L, prm, keys)
    cts = synth.uniform_residues(617, ctx.q, (n, ln, 2, ctx.N))
    got = down(ctx.sumdis_lazy(up(torch, cts), plan=plan))
    want = ora.sumdis_lazy(cts, keys["rlk"], plan, [keys["rot"][k] for k in ora_steps(plan)])
    assert np.array_equal(got, want)


# ---- memory planning -----------------------------------------------------------------

def test_footprint_matches_workspace(torch, L):
    """A resident round on a fresh stream grows exactly the workspace that
    lc_footprint reports; the round's own buffers are the client and
    distance ciphertexts (and SumDis)."""
    prm = (12, (40, 30, 30), (40,))
    ctx = L.Context(*prm, device=0)
    ctx.keygen(5)
    plan = [3, 3, 3, 2]
    ctx.keygen_rotation(5, ctx.rotsum_steps(plan))
    n, ln = 6, 3
    rb, wb = ctx.footprint(n, ln, 0, L.FP_SUMDIS)
    S = ctx.nq * ctx.N * 8
    P = n * (n - 1) // 2
    assert rb == n * ln * 2 * S + P * 2 * S + n * 2 * S
    cts = up(torch, synth.uniform_residues(8, ctx.q, (n, ln, 2, ctx.N)))
    s = torch.cuda.Stream()
    before = ctx.device_bytes()
    with torch.cuda.stream(s):
        ctx.pairwise_sqdist(cts, plan=plan, sumdis=True, stream=s)
    s.synchronize()
    assert ctx.device_bytes() - before == wb
