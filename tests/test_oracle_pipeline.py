"""End-to-end pins of the oracle's Server Executes pipeline (Algorithm 1):
decrypted pairwise distances against FP64 numpy distances of the same
synthetic updates, and the KGC selection rules against FP64 selections.
"""
import pathlib

import numpy as np
import pytest

import synth

GOLDEN = pathlib.Path(__file__).parent / "golden"


def run_pipeline(O, w, plan=None, want_triples=False):
    ora = O.Oracle(w.log_n, w.q_bits, w.p_bits)
    seed = w.crypto_seed
    s = ora.secret(seed)
    pk = ora.pk(seed, s)
    rlk = ora.relin_key(seed, s)
    plan = list(plan or w.rot_plan)
    rks = [ora.rot_key(seed, s, k) for k in ora.rotsum_steps(plan)]
    upd = synth.client_updates(w)
    scale = 2.0 ** w.scale_log2
    m = np.stack([np.stack([O.encode(chunk, w.log_n, scale) for chunk in synth.pack(u, w.slots)]) for u in upd])
    n, ln = m.shape[0], m.shape[1]
    cts = ora.encrypt(seed + 1, 0, m.reshape(n * ln, w.N), pk).reshape(n, ln, 2, ora.nq, w.N)
    res = ora.pairwise(cts, rlk, plan, rks, want_sumdis=True, want_triples=want_triples)
    return ora, s, upd, cts, res, scale


def fp64_dists(upd):
    n = upd.shape[0]
    return np.array([np.sum((upd[i] - upd[j]) ** 2) for i in range(n) for j in range(i + 1, n)])


TINY = synth.small_workload(log_n=5, q_bits=(45, 40, 40), p_bits=(45,), n_clients=4, dim=40, scale_log2=30)
TINY2 = synth.small_workload(log_n=6, q_bits=(50, 45, 45, 45), p_bits=(50, 50), n_clients=5, dim=100,
                             scale_log2=35, name="tiny2")


@pytest.mark.parametrize("w", [TINY, TINY2])
def test_pairwise_decrypts_to_fp64(oracle_mod, w):
    O = oracle_mod
    ora, s, upd, cts, res, scale = run_pipeline(O, w, want_triples=True)
    want = fp64_dists(upd)
    got = np.array([ora.read_distance(ora.decrypt(d, s), scale * scale) for d in res["dist"]])
    assert np.allclose(got, want, rtol=1e-3), (got, want)
    # the triple before relinearization carries the slot-wise sum: coefficient 0
    # of Dec3 is (2/N) * scale^2 * d (trace of the unrotated sum)
    for p in range(len(want)):
        c0 = ora.crt(ora.decrypt(res["triples"][p], s), [0])[0]
        assert np.isclose(c0 * w.N / 2 / scale**2, want[p], rtol=1e-3)
    # SumDis[i] = sum_j != i Dis[i][j]
    D = O.distance_matrix(want, w.n_clients)
    for i in range(w.n_clients):
        v = ora.read_distance(ora.decrypt(res["sumdis"][i], s), scale * scale)
        assert np.isclose(v, D[i].sum(), rtol=1e-3)


def test_pairwise_subset_matches_full(oracle_mod):
    O = oracle_mod
    w = TINY
    ora, s, upd, cts, res, scale = run_pipeline(O, w)
    seed = w.crypto_seed
    rlk = ora.relin_key(seed, s)
    rks = [ora.rot_key(seed, s, k) for k in ora.rotsum_steps(w.rot_plan)]
    sub = ora.pairwise(cts, rlk, list(w.rot_plan), rks, want_sumdis=False, pairs=[1, 4])
    for p in (1, 4):
        assert np.array_equal(sub["dist"][p], res["dist"][p])


def test_plans_agree_after_decryption(oracle_mod):
    O = oracle_mod
    w = TINY
    L = w.log_n - 1
    _, s, upd, _, r1, scale = run_pipeline(O, w, plan=[1] * L)
    ora, s2, _, _, r2, _ = run_pipeline(O, w, plan=[2, 2])
    for a, b in zip(r1["dist"], r2["dist"]):
        da = ora.read_distance(ora.decrypt(a, s), scale * scale)
        db = ora.read_distance(ora.decrypt(b, s2), scale * scale)
        assert np.isclose(da, db, rtol=1e-4)


def test_selection_rules_fp64(oracle_mod):
    O = oracle_mod
    w = synth.CFG2
    upd = synth.client_updates(w, clients=range(w.n_clients))[:, :5000]
    D = O.distance_matrix(fp64_dists(upd), w.n_clients)
    byz = set(range(w.n_clients - w.n_byz, w.n_clients))
    for rule, l in (("krum", None), ("median", None), ("multikrum", 4)):
        sel = O.select(rule, D, w.n_byz, l)
        assert not (set(sel) & byz), (rule, sel)
    assert len(O.select("multikrum", D, w.n_byz, 4)) == 4
    # Multi-Krum stops once n - |psi| <= 2c + 2
    assert len(O.select("multikrum", D, 3, 10)) == w.n_clients - 8


def test_permutation_mask_example(oracle_mod):
    """The paper's worked mask example (tests/golden/permutation_mask_5clients.txt):
    five clients, the top three are clients 1, 3, 5 (1-based)."""
    O = oracle_mod
    want = np.loadtxt(GOLDEN / "permutation_mask_5clients.txt", comments="#", dtype=np.int64)
    assert want.shape == (5, 5)
    assert np.array_equal(O.permutation_mask(5, [0, 2, 4]), want)


def test_pair_triple_columns_pins(oracle_mod):
    """The column form of the pair triple equals the C oracle's full-array
    pair triple on every limb and coefficient (two implementations, Python
    integers and 128-bit C), and a closed form: constant ciphertexts give
    LEN (a - b)^2 in each slot of the triple."""
    O = oracle_mod
    ora = O.Oracle(5, (50, 45, 40), (50,))
    cts = synth.uniform_residues(91, ora.q, (3, 7, 2, 32))
    for i, j in ((0, 1), (0, 2), (1, 2)):
        full = ora.pair_triple(cts, i, j)
        for l, q in enumerate(ora.q):
            got = O.pair_triple_columns(cts[i, :, :, l, :], cts[j, :, :, l, :], q)
            assert np.array_equal(got, full[:, l, :]), (i, j, l)
    q = int(ora.q[0])
    a = np.zeros((5, 2, 1), dtype=np.uint64)
    b = np.zeros((5, 2, 1), dtype=np.uint64)
    a[:, 0], a[:, 1], b[:, 0], b[:, 1] = 7, q - 3, q - 1, 5  # d0 = 8 - q = 8, d1 = q - 8 = -8 (mod q)
    got = O.pair_triple_columns(a, b, q)
    assert [int(v) for v in got[:, 0]] == [5 * 64 % q, (2 * 5 * -64) % q, 5 * 64 % q]


def test_masked_sum_columns_pins(oracle_mod):
    """The column form of the masked sum equals the C oracle's full-array
    masked sum on every limb and coefficient, and one-hot masks select one
    client's ciphertexts."""
    O = oracle_mod
    ora = O.Oracle(5, (50, 45, 40), (50,))
    n, ln = 5, 3
    cts = synth.uniform_residues(92, ora.q, (n, ln, 2, 32))
    masks = synth.uniform_residues(93, ora.q, (n, 32))
    full = ora.masked_sum(cts, masks)
    for l, q in enumerate(ora.q):
        got = O.masked_sum_columns(cts[:, :, :, l, :], masks[:, l, :], q)
        assert np.array_equal(got, full[:, :, l, :]), l
    hot = np.zeros((n, 32), dtype=np.uint64)
    hot[3] = 1
    assert np.array_equal(O.masked_sum_columns(cts[:, :, :, 0, :], hot, ora.q[0]), cts[3, :, :, 0, :])


def test_sumdis_lazy_pins(oracle_mod):
    """The per-client SumDis (one relinearization per client, Algorithm 1
    SumDis line with Methods, Lazy Relinearization) decrypts to the FP64
    sum of each client's squared distances, and with two clients it reduces
    exactly to the one pair's distance ciphertext (the triple sum of either
    client is the pair's triple)."""
    O = oracle_mod
    w = TINY2
    ora, s, upd, cts, res, scale = run_pipeline(O, w)
    seed = w.crypto_seed
    rlk = ora.relin_key(seed, s)
    plan = list(w.rot_plan)
    rks = [ora.rot_key(seed, s, k) for k in ora.rotsum_steps(plan)]
    got = ora.sumdis_lazy(cts, rlk, plan, rks)
    D = O.distance_matrix(fp64_dists(upd), w.n_clients)
    for i in range(w.n_clients):
        v = ora.read_distance(ora.decrypt(got[i], s), scale * scale)
        assert np.isclose(v, D[i].sum(), rtol=1e-3), (i, v, D[i].sum())
    two = ora.sumdis_lazy(cts[:2], rlk, plan, rks)
    assert np.array_equal(two[0], res["dist"][0]) and np.array_equal(two[1], res["dist"][0])
