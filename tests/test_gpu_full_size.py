"""Parity of the pair kernel (a2) at the benchmark workload's full size:
N = 2^16, 24 limbs, 20 clients x 342 packed ciphertexts (172 GB of
ciphertexts resident in HBM), in the launch shape the bench times.  The
oracle computes sampled outputs one by one from their definition on the same
residues: the first, a middle and the last pair, at three limbs and three
windows of 32 coefficients (the range's start, middle and end)."""
import gc

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


def test_pair_triples_full_size_sampled(torch, L, oracle_mod):
    O = oracle_mod
    log_n, nq = 16, 24
    ctx = L.Context(log_n, (50,) * nq, (50,) * 4, device=0)
    assert all(int(q) > 1 << 49 for q in ctx.q)  # 49-bit inputs are canonical for every limb
    gc.collect()
    torch.cuda.empty_cache()
    n, ln, N = 20, 342, 1 << log_n
    cts = synth.device_residues(torch, 4242, 49, (n, ln, 2, nq, N))
    ctx.set_tuning("pair_mfma", 0)
    ctx.set_tuning("pair_lanes", 16)
    ctx.set_tuning("pair_ppt", 4)
    trip = ctx.pair_triples(cts)
    torch.cuda.synchronize()
    pairs = {0: (0, 1), 98: (5, 19), 189: (18, 19)}
    try:
        for l in (0, 11, 23):
            for c0 in (0, N // 2 - 16, N - 32):
                cols = cts[:, :, :, l, c0:c0 + 32].cpu().numpy().view(np.uint64)  # [n][ln][2][32]
                got = trip[:, :, l, c0:c0 + 32].cpu().numpy().view(np.uint64)    # [P][3][32]
                for p, (i, j) in pairs.items():
                    want = O.pair_triple_columns(cols[i], cols[j], ctx.q[l])
                    assert np.array_equal(got[p], want), (p, l, c0)
    finally:
        del cts, trip
        gc.collect()
        torch.cuda.empty_cache()
