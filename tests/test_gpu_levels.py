"""GPU parity of rescaling and of decryption / decoding at a lower level (f4:
levels of the CKKS Scheme Description) against the oracle's rescale, written
from the definition (CRT to integers, rounded division), bit for bit.
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


# N below, inside and at the top of the two-pass transform range; levels from
# the top down to two limbs; pairs and triples; a ragged count
@pytest.mark.parametrize("log_n,qb", [(5, (30, 28, 28, 28)), (9, (50, 45, 45, 40)), (10, (50, 45, 45, 40, 40)),
                                      (12, (50, 40, 40)), (16, (50, 50, 50))])
def test_rescale_bitexact(torch, L, oracle_mod, log_n, qb):
    O = oracle_mod
    ctx = L.Context(log_n, qb, (50,), device=0)
    ora = O.Oracle(log_n, qb, (50,))
    assert ora.primes == ctx.moduli
    nq, N = len(qb), 1 << log_n
    count = 3 if log_n < 16 else 1
    for nlimb in sorted({nq, 2}):
        for ncomp in (2, 3):
            cts = synth.uniform_residues(40 + nlimb + ncomp, ctx.q[:nlimb], (count, ncomp, N))
            got = down(ctx.rescale(up(torch, cts), nlimb, ncomp=ncomp))
            assert got.shape == (count, ncomp, nlimb - 1, N)
            for c in range(count):
                assert np.array_equal(got[c], ora.rescale(cts[c], nlimb)), (nlimb, ncomp, c)


def test_rescale_rejects_bad_arguments(torch, L):
    ctx = L.Context(5, (30, 28, 28), (30,), device=0)
    ct = torch.zeros((1, 2, 3, 32), dtype=torch.int64, device="cuda")
    for nlimb in (1, 4):
        with pytest.raises(L.LancelotError):
            ctx.rescale(ct, nlimb)
    with pytest.raises(L.LancelotError):  # in place: out overlaps in
        ctx.rescale(ct, 3, out=ct)


def test_square_relin_rescale_decrypts(torch, L, oracle_mod):
    """The paper's depth use: square a ciphertext at scale Delta, relinearize,
    rescale by the last prime, then decrypt and decode at the lower level with
    scale Delta^2 / q_t: the slots hold x^2.  Decryption at the lower level
    equals the oracle's on the same ciphertext, bit for bit."""
    O = oracle_mod
    log_n, qb, pb = 12, (50, 40, 40, 40), (50,)
    scale = 2.0 ** 40
    ctx = L.Context(log_n, qb, pb, device=0)
    ctx.keygen(17)
    ora = O.Oracle(log_n, qb, pb)
    s = ora.secret(17)
    pk = ora.pk(17, s)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1.0, 1.0, size=(2, 1 << (log_n - 1)))
    m = np.stack([O.encode(v, log_n, scale) for v in x])
    cts = ora.encrypt(3, 0, m, pk)
    sq = ctx.relin(ctx.ct_square(up(torch, cts)))
    t = len(qb) - 1
    rs = ctx.rescale(sq, len(qb))
    pt = down(ctx.decrypt_level(rs, t))
    sh = ora.signed_to_ntt(s, t)
    rs_h = down(rs)
    low = [int(q) for q in ora.q[:t]]
    for c in range(2):
        want = ora.poly_intt(np.array([[(int(a) + int(b) * int(d)) % q for a, b, d in
                                        zip(rs_h[c, 0, l], rs_h[c, 1, l], sh[l])] for l, q in enumerate(low)],
                                      dtype=np.uint64))
        assert np.array_equal(pt[c], want)
        z = ctx.decode_level(pt[c], scale * scale / int(ora.q[t])).real
        assert np.max(np.abs(z - x[c] ** 2)) < 1e-6
