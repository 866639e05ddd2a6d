"""Small fixed GPU cases for hardware-counter runs (rocprofv3 --pmc).

    python -m paper_2408_06197_amd.profile_cases pair       # one pair-triple launch
    python -m paper_2408_06197_amd.profile_cases keyswitch  # one rotate-and-sum of 16 ciphertexts
    python -m paper_2408_06197_amd.profile_cases keyswitch fuse_modup=0   # with lc_set_tuning overrides
    python -m paper_2408_06197_amd.profile_cases ntt        # forward + inverse NTT of 64 ciphertexts' limbs
    python -m paper_2408_06197_amd.profile_cases masked     # one plaintext-mask masked sum (a6)

All run at N = 2^16 with 24 + 4 limbs of 50 bits on random residues, then
copy 4 GiB with a plain device copy so that each counter can be scaled by
what it reads for a copy of known size.  Counter passes each need a run of
their own (rocprofv3 does not split counters over passes).
"""
from __future__ import annotations

import sys

import torch

from . import lancelot as L

NQ, NP, LOG_N = 24, 4, 16


def _calibration_copy():
    src = torch.ones(1 << 29, dtype=torch.int64, device="cuda")  # 4 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def pair(tune, lanes=16, ppt=4, n=20, ln=342):
    """lc_pair_triples over 20 clients x 342 packed ciphertexts (172 GB)."""
    ctx = L.Context(LOG_N, (50,) * NQ, (50,) * NP, device=0)
    for k, v in tune.items():
        ctx.set_tuning(k, v)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    cts = torch.empty((n, ln, 2, NQ, 1 << LOG_N), dtype=torch.int64, device="cuda")
    for i in range(n):
        cts[i].random_(0, 1 << 49, generator=gen)  # below every 50-bit prime
    trip = torch.empty((n * (n - 1) // 2, 3, NQ, 1 << LOG_N), dtype=torch.int64, device="cuda")
    ctx.set_tuning("pair_lanes", tune.get("pair_lanes", lanes))
    ctx.set_tuning("pair_ppt", tune.get("pair_ppt", ppt))
    ctx.pair_triples(cts, out=trip)
    torch.cuda.synchronize()
    del cts
    _calibration_copy()


def keyswitch(tune, count=16, plan=(3, 3, 3, 3, 3)):
    """lc_rotate_sum of `count` ciphertexts with the given hoisting plan."""
    ctx = L.Context(LOG_N, (50,) * NQ, (50,) * NP, device=0)
    ctx.keygen(7)
    ctx.keygen_rotation(7, ctx.rotsum_steps(list(plan)))
    ctx.set_tuning("ks_chunk", count)
    for k, v in tune.items():
        ctx.set_tuning(k, v)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    ct = torch.empty((count, 2, NQ, 1 << LOG_N), dtype=torch.int64, device="cuda")
    ct.random_(0, 1 << 49, generator=gen)
    ctx.rotate_sum(ct, list(plan))
    torch.cuda.synchronize()
    _calibration_copy()


def ntt(tune, count=64, reps=3):
    """Forward then inverse NTT of count x 24 limb-polynomials (residues
    uniform in each limb's range), `reps` times: the transform the
    benchmark's NTT roofline entry times."""
    ctx = L.Context(LOG_N, (50,) * NQ, (50,) * NP, device=0)
    for k, v in tune.items():
        ctx.set_tuning(k, v)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    x = torch.empty((count, NQ, 1 << LOG_N), dtype=torch.int64, device="cuda")
    for l in range(NQ):
        x[:, l].random_(0, int(ctx.q[l]), generator=gen)
    for _ in range(reps):
        ctx.ntt_fwd(x, nlimb=NQ)
        ctx.ntt_inv(x, nlimb=NQ)
    torch.cuda.synchronize()
    del x
    _calibration_copy()


def masked(tune, n=20, ln=342):
    """lc_masked_sum over 20 clients x 342 packed ciphertexts (172 GB) with
    full-range masks, once per masked-sum shape 0, 1, 2 (or the one given)."""
    ctx = L.Context(LOG_N, (50,) * NQ, (50,) * NP, device=0)
    for k, v in tune.items():
        ctx.set_tuning(k, v)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    cts = torch.empty((n, ln, 2, NQ, 1 << LOG_N), dtype=torch.int64, device="cuda")
    masks = torch.empty((n, NQ, 1 << LOG_N), dtype=torch.int64, device="cuda")
    for l in range(NQ):
        cts[:, :, :, l].random_(0, int(ctx.q[l]), generator=gen)
        masks[:, l].random_(0, int(ctx.q[l]), generator=gen)
    out = torch.empty((ln, 2, NQ, 1 << LOG_N), dtype=torch.int64, device="cuda")
    for shape in ([tune["ms_shape"]] if "ms_shape" in tune else [0, 1, 2]):
        ctx.set_tuning("ms_shape", shape)
        ctx.masked_sum(cts, masks, out=out)
    torch.cuda.synchronize()
    del cts
    _calibration_copy()


if __name__ == "__main__":
    case = sys.argv[1] if len(sys.argv) > 1 else "pair"
    cases = {"pair": pair, "keyswitch": keyswitch, "ntt": ntt, "masked": masked}
    if case not in cases:
        sys.exit("cases: " + ", ".join(cases))
    tune = dict((kv.split("=")[0], int(kv.split("=")[1])) for kv in sys.argv[2:])
    torch.cuda.set_device(0)
    cases[case](tune)
    print(f"profile case {case} done", flush=True)
