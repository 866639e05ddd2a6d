"""lc_relin_noalloc, the relinearization for callers that cannot allocate
device memory, against lc_relin through the C ABI: the same residues on two
calls in a row (the second with fewer ciphertexts, so the shared scratch
array holds the first call's contents), no growth of the library's device
memory, batches that fit the fixed array at N = 2^16, and the size limit."""
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


@pytest.mark.parametrize("prm,counts", [((12, (40, 30, 30), (40,)), (7, 3)),
                                        ((14, (50,) * 8, (50,) * 2), (5, 2)),
                                        ((16, (50,) * 24, (50,) * 4), (3, 1))],
                         ids=["n4096", "n16384", "n65536"])
def test_relin_noalloc_matches_relin(torch, L, prm, counts):
    ctx = L.Context(*prm, device=0)
    ctx.keygen(91)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for k, count in enumerate(counts):
            t3 = torch.from_numpy(synth.uniform_residues(300 + k, ctx.q, (count, 3, ctx.N)).view(np.int64)).cuda()
            out = torch.full((count, 2, ctx.nq, ctx.N), -1, dtype=torch.int64, device="cuda")
            before = ctx.device_bytes()
            ctx.relin_noalloc(t3, out, stream=s)
            s.synchronize()
            assert ctx.device_bytes() == before  # no workspace was grown
            want = ctx.relin(t3, stream=s)
            s.synchronize()
            assert torch.equal(out, want), (prm[0], count)


def test_relin_noalloc_rejects_oversize(torch, L):
    # N = 2^17 with 24 + 4 limbs: 310 MB of key-switch scratch per ciphertext
    ctx = L.Context(17, (50,) * 24, (50,) * 4, device=0)
    ctx.keygen(3)
    t3 = ctx.empty(1, 3, ctx.nq, ctx.N)
    out = ctx.empty(1, 2, ctx.nq, ctx.N)
    with pytest.raises(L.LancelotError) as e:
        ctx.relin_noalloc(t3, out)
    assert e.value.code == L.LC_EINVAL and "exceeds" in str(e.value)
