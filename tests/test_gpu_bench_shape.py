"""The batched distance pipeline at the benchmark's ring degree and limb count,
in the launch configuration the benchmark times, bit for bit against the
oracle.

N = 2^16, 24 + 4 limbs (dnum 6), 20 clients x 8 packed ciphertexts of
residues uniform in each limb's whole range.  Keys are made by the oracle
from its own secret and imported (lc_key_import), so the check does not rest
on the library's key generation.  Launch shapes: pair kernel 16 lanes x 4
pairs, rotate-and-sum plan 3,3,3,3,3 (blocks of 7 hoisted rotations), cycle
walk from 16-tile cycles, key-switch batches of 32 ciphertexts -- the 190
pairs take 6 batches and the key-switch workspace (32 x 148 MiB) has offsets
past 4 GiB.  Pairs 0 and 31 / 32 sit at the ends of the first two batches,
98 in the middle and 189 last; client 0's SumDis sums pairs 0 .. 18.
"""
import concurrent.futures as cf
import sys
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

LOG_N, NQ, NP, N_CLIENTS, LEN = 16, 24, 4, 20, 8
PLAN = [3, 3, 3, 3, 3]
CHECK_PAIRS = [0, 31, 32, 98, 189]


def note(msg):
    print("[bench-shape] " + msg, file=sys.stderr, flush=True)


@pytest.mark.timeout(900)
def test_pairwise_bench_shape_oracle_keys(oracle_mod):
    import torch
    from paper_2408_06197_amd import lancelot as L

    O = oracle_mod
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    prm = (LOG_N, (50,) * NQ, (50,) * NP)
    t0 = time.perf_counter()
    ora = O.Oracle(*prm)
    s = ora.secret(61)
    rlk = ora.relin_key(61, s)
    steps = ora.rotsum_steps(PLAN)
    with cf.ThreadPoolExecutor(max_workers=3) as ex:
        rks = list(ex.map(lambda st: ora.rot_key(61, s, st), steps))
    note(f"oracle keys done ({time.perf_counter() - t0:.0f}s)")
    ctx = L.Context(*prm, device=0, role=L.ROLE_SERVER)
    assert ora.primes == ctx.moduli
    ctx.key_import(L.KEY_RELIN, rlk)
    for st, key in zip(steps, rks):
        ctx.key_import(L.KEY_ROTATION, key, step=st)
    for name, v in (("pair_mfma", 0), ("pair_lanes", 16), ("pair_ppt", 4), ("mac_cycle_min", 16),
                    ("ks_chunk", 32), ("mac_cts", 16)):
        ctx.set_tuning(name, v)
    cts = synth.uniform_residues(6262, ctx.q, (N_CLIENTS, LEN, 2, ctx.N))
    dist, sumdis = ctx.pairwise_sqdist(torch.from_numpy(cts.view(np.int64)).cuda(), plan=PLAN, sumdis=True)
    torch.cuda.synchronize()
    got_dist = dist.cpu().numpy().view(np.uint64)
    got_sumdis0 = sumdis[0].cpu().numpy().view(np.uint64)
    del dist, sumdis
    note(f"GPU pipeline done ({time.perf_counter() - t0:.0f}s); oracle pairs follow")
    # client 0's pairs (0, j) are pair indices 0 .. 18; the oracle's calls
    # release the interpreter lock, so a few pairs run side by side
    pairs = sorted(set(range(N_CLIENTS - 1)) | set(CHECK_PAIRS))
    ij = [(i, j) for i in range(N_CLIENTS) for j in range(i + 1, N_CLIENTS)]
    with cf.ThreadPoolExecutor(max_workers=3) as ex:
        want = dict(zip(pairs, ex.map(lambda p: ora.pair_distance(cts, *ij[p], rlk, PLAN, rks), pairs)))
    note(f"oracle pairs done ({time.perf_counter() - t0:.0f}s)")
    for p in pairs:
        assert np.array_equal(got_dist[p], want[p]), p
    sd = want[0]
    for p in range(1, N_CLIENTS - 1):
        sd = ora.add(sd, want[p])
    assert np.array_equal(got_sumdis0, sd)
