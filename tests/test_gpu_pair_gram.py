"""GPU parity of the pair triples in the Gram form on the int8 matrix cores
(a2; the Tensor and Add operations summed lazily over the packed ciphertexts)
against the oracle's per-pair sums of squared differences, bit for bit.

Cases: one, two and three 16-row blocks of the Gram matrix (2, 8, 9, 20, 21
and 24 clients), 4 and 2 coefficients per workgroup, the XCD tile remap on
(N >= 128) and off, ragged chunks of 64 ciphertexts, more than 512
ciphertexts (two launches), accumulation into existing triples, residues
whose balanced digits all sit at the ends of [-128, 127] at the int32
accumulator bound, and the fallback to the per-pair kernel past 24 clients.
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


def check_all(got, ora, cts, every=1):
    n = cts.shape[0]
    p = 0
    for i in range(n):
        for j in range(i + 1, n):
            if p % every == 0 or p == n * (n - 1) // 2 - 1:
                assert np.array_equal(got[p], ora.pair_triple(cts, i, j)), (i, j)
            p += 1


@pytest.mark.parametrize("n,ln,pm,log_n", [(2, 3, 4, 6), (8, 64, 4, 7), (9, 65, 4, 7), (20, 70, 4, 7),
                                           (20, 9, 2, 7), (21, 5, 4, 6), (24, 7, 4, 7), (25, 3, 4, 5)])
def test_pair_gram_bitexact(torch, L, oracle_mod, n, ln, pm, log_n):
    O = oracle_mod
    prm = (log_n, (50, 45, 40), (50,))
    ctx = L.Context(*prm, device=0)
    ora = O.Oracle(*prm)
    cts = synth.uniform_residues(500 + n + ln, ctx.q, (n, ln, 2, ctx.N))
    ctx.set_tuning("pair_mfma", pm)
    got = down(ctx.pair_triples(up(torch, cts)))
    check_all(got, ora, cts, every=1 if n <= 9 else 7)
    # the per-pair kernel gives the same bits
    ctx.set_tuning("pair_mfma", 0)
    assert np.array_equal(down(ctx.pair_triples(up(torch, cts))), got)


def test_pair_gram_long_rows_and_accumulate(torch, L, oracle_mod):
    """600 ciphertexts: two launches (512 + 88) summed; then the chunked form
    adds a second batch into the same triples."""
    O = oracle_mod
    prm = (5, (50, 45), (50,))
    ctx = L.Context(*prm, device=0)
    ora = O.Oracle(*prm)
    n = 3
    cts = synth.uniform_residues(601, ctx.q, (n, 600, 2, ctx.N))
    ctx.set_tuning("pair_mfma", 4)
    trip = ctx.pair_triples(up(torch, cts))
    check_all(down(trip), ora, cts)
    more = synth.uniform_residues(602, ctx.q, (n, 70, 2, ctx.N))
    ctx.pair_triples_acc(up(torch, more), trip)
    both = np.concatenate([cts, more], axis=1)
    check_all(down(trip), ora, both)


@pytest.mark.parametrize("pattern", ["max_digits", "min_digits", "top"])
def test_pair_gram_extreme_digits(torch, L, oracle_mod, pattern):
    """512 ciphertexts (one launch at the accumulator bound) of residues whose
    balanced digits are all +127 or all -128 (below 2^50, then reduced into
    [0, q)), or q - 1 everywhere."""
    O = oracle_mod
    prm = (5, (50, 50), (50,))
    ctx = L.Context(*prm, device=0)
    ora = O.Oracle(*prm)
    n, ln = 4, 512
    cts = np.empty((n, ln, 2, ctx.nq, ctx.N), dtype=np.uint64)
    for l, q in enumerate(ctx.q):
        q = int(q)
        if pattern == "max_digits":  # x + 0x0080..80 = 0x0081ffffffffffff: digits +127 (top digit 1)
            x = 0x00017F7F7F7F7F7F
        elif pattern == "min_digits":  # x + 0x0080..80 = 0x0081000000000000: digits -128 (top digit 1)
            x = 0x00007F7F7F7F7F80
        else:
            x = q - 1
        assert x < q
        cts[:, :, :, l, :] = np.uint64(x)
    cts[1, :, 0] = 0  # one row of zeros, one row alternating
    cts[2, ::2, 1] = np.uint64(1)
    ctx.set_tuning("pair_mfma", 4)
    got = down(ctx.pair_triples(up(torch, cts)))
    check_all(got, ora, cts)


def test_pair_gram_full_shape(torch, L, oracle_mod):
    """The N = 2^16, 24-limb shape of the benchmark workload with 20 clients
    (3 row blocks, the XCD remap over 16384 workgroups per limb) and a ragged
    70-ciphertext row: equal to the per-pair kernel bit for bit, and sampled
    pairs (first, middle, last) equal to the oracle."""
    O = oracle_mod
    prm = (16, (50,) * 24, (50,) * 4)
    ctx = L.Context(*prm, device=0)
    ora = O.Oracle(*prm)
    n, ln = 20, 70
    cts = synth.uniform_residues(777, ctx.q, (n, ln, 2, ctx.N))
    g = up(torch, cts)
    ctx.set_tuning("pair_mfma", 4)
    got = ctx.pair_triples(g)
    ctx.set_tuning("pair_mfma", 0)
    ref = ctx.pair_triples(g)
    assert torch.equal(got, ref)
    got = down(got)
    for p, (i, j) in ((0, (0, 1)), (98, (5, 19)), (189, (18, 19))):
        assert np.array_equal(got[p], ora.pair_triple(cts, i, j)), (i, j)
