"""Parity at the benchmark workload's full size: N = 2^16, 24 limbs, 20 clients
x 342 packed ciphertexts (172 GB resident in HBM, generated on the GPU from a
seeded generator), in the launch shapes the bench times.  The oracle computes
sampled outputs one by one from their definitions on the same residues
(uniform in each limb's whole range), at three limbs and three windows of 32
coefficients (the range's start, middle and end):
  * the pair kernel (a2): the first, a middle and the last pair;
  * the plaintext-mask aggregate (a6): every packed ciphertext and component.
Relinearization (a3), encryption (a1), decryption (a7) and hoisted rotations
(a4, the literal form) at the same ring degree and limb count are checked
whole against the oracle (the hoisted rotate-and-sum at that shape is in
test_gpu_parity.py).
"""
import gc

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

LOG_N, NQ, N_CLIENTS, LEN = 16, 24, 20, 342
SAMPLE_LIMBS = (0, 11, 23)


def windows(N):
    return (0, N // 2 - 16, N - 32)


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


@pytest.fixture(scope="module")
def full(torch, L):
    ctx = L.Context(LOG_N, (50,) * NQ, (50,) * 4, device=0)
    gc.collect()
    torch.cuda.empty_cache()
    need = N_CLIENTS * LEN * 2 * NQ * (8 << LOG_N) + (20 << 30)  # ciphertexts + outputs and workspace
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"the full-size workload needs {need / 2**30:.0f} GiB free on the device, {free / 2**30:.0f} GiB is")
    # every residue uniform in [0, q_l): the top of each limb's range, where
    # the FP64 Barrett bounds are tightest, is exercised
    cts = synth.device_residues_mod(torch, 4242, ctx.q, (N_CLIENTS, LEN, 2, NQ, 1 << LOG_N))
    yield ctx, cts
    del cts
    gc.collect()
    torch.cuda.empty_cache()


def test_pair_triples_full_size_sampled(torch, oracle_mod, full):
    O = oracle_mod
    ctx, cts = full
    ctx.set_tuning("pair_mfma", 0)
    ctx.set_tuning("pair_lanes", 16)
    ctx.set_tuning("pair_ppt", 4)
    trip = ctx.pair_triples(cts)
    torch.cuda.synchronize()
    pairs = {0: (0, 1), 98: (5, 19), 189: (18, 19)}
    try:
        for l in SAMPLE_LIMBS:
            for c0 in windows(ctx.N):
                cols = cts[:, :, :, l, c0:c0 + 32].cpu().numpy().view(np.uint64)  # [n][LEN][2][32]
                got = trip[:, :, l, c0:c0 + 32].cpu().numpy().view(np.uint64)    # [P][3][32]
                for p, (i, j) in pairs.items():
                    want = O.pair_triple_columns(cols[i], cols[j], ctx.q[l])
                    assert np.array_equal(got[p], want), (p, l, c0)
    finally:
        del trip
        torch.cuda.empty_cache()


def test_masked_sum_full_size_sampled(torch, oracle_mod, full):
    O = oracle_mod
    ctx, cts = full
    masks = synth.device_residues_mod(torch, 4343, ctx.q, (N_CLIENTS, NQ, ctx.N))
    ctx.set_tuning("ms_shape", 2)
    out = ctx.masked_sum(cts, masks)
    torch.cuda.synchronize()
    try:
        for l in SAMPLE_LIMBS:
            for c0 in windows(ctx.N):
                cols = cts[:, :, :, l, c0:c0 + 32].cpu().numpy().view(np.uint64)
                w = masks[:, l, c0:c0 + 32].cpu().numpy().view(np.uint64)
                got = out[:, :, l, c0:c0 + 32].cpu().numpy().view(np.uint64)  # [LEN][2][32]
                assert np.array_equal(got, O.masked_sum_columns(cols, w, ctx.q[l])), (l, c0)
    finally:
        del out, masks
        torch.cuda.empty_cache()


def test_relin_full_shape(torch, L, oracle_mod):
    """Relinearization (a3) at N = 2^16 with 24 + 4 limbs (dnum 6) in the
    bench's key-switch configuration (batch of 32, 16 ciphertexts per lane of
    the inner product, fused ModUp / ModDown passes), on two synthetic
    degree-2 ciphertexts with uniform residues, against the oracle's
    relinearization with the same relinearization key."""
    O = oracle_mod
    prm = (LOG_N, (50,) * NQ, (50,) * 4)
    ctx = L.Context(*prm, device=0)
    ctx.keygen(29)
    ora = O.Oracle(*prm)
    assert ora.primes == ctx.moduli
    rlk = ora.relin_key(29, ora.secret(29))
    ctx.set_tuning("ks_chunk", 32)
    ctx.set_tuning("mac_cts", 16)
    t3 = synth.uniform_residues(3131, ctx.q, (2, 3, ctx.N))
    got = ctx.relin(torch.from_numpy(t3.view(np.int64)).cuda()).cpu().numpy().view(np.uint64)
    for c in range(2):
        assert np.array_equal(got[c], ora.relin(t3[c], rlk)), c


def test_encrypt_decrypt_rotate_full_shape(torch, L, oracle_mod):
    """Encryption (a1), decryption of 2- and 3-component ciphertexts (a7) and
    hoisted rotations over several steps sharing one ModUp (a4, the literal
    form) at N = 2^16 with 24 + 4 limbs, against the oracle with the same
    keys and the same counter-based randomness."""
    O = oracle_mod
    prm = (LOG_N, (50,) * NQ, (50,) * 4)
    steps = [1, 64, -5]
    ctx = L.Context(*prm, device=0)
    ctx.keygen(31)
    ctx.keygen_rotation(31, steps)
    ora = O.Oracle(*prm)
    assert ora.primes == ctx.moduli
    s = ora.secret(31)
    pk = ora.pk(31, s)
    rng = np.random.default_rng(12)
    m = rng.integers(-(1 << 40), 1 << 40, size=(2, ctx.N), dtype=np.int64)
    want = ora.encrypt(88, 500, m, pk)
    got = ctx.encrypt(torch.from_numpy(m).cuda(), seed=88, first_object=500)
    assert np.array_equal(got.cpu().numpy().view(np.uint64), want)
    dec = ctx.decrypt(got).cpu().numpy().view(np.uint64)
    for t in range(2):
        assert np.array_equal(dec[t], ora.decrypt(want[t], s)), t
    t3 = ora.mul(want[0], want[1])
    d3 = ctx.decrypt(torch.from_numpy(t3[None].view(np.int64)).cuda(), ncomp=3).cpu().numpy().view(np.uint64)[0]
    assert np.array_equal(d3, ora.decrypt(t3, s))
    rks = [ora.rot_key(31, s, k) for k in steps]
    rot = ctx.rotate_hoisted(got[:1].contiguous(), steps).cpu().numpy().view(np.uint64)
    assert np.array_equal(rot[0], ora.rotate_hoisted(want[0], steps, rks))
