"""GPU parity of the device encode (f3: ingest without the host FFT) against
the oracle's encode (numpy FFT of the canonical embedding) and the host
library's, and of device encode + encrypt against the oracle's encryption of
the oracle's plaintexts.

Two FP64 evaluations of the embedding may round a coefficient that lies
within rounding error of a half-integer to neighbouring integers, so the
encodes are compared to within one per coefficient (and must agree on nearly
all coefficients); the decoded slots must match the inputs within the
rounding bound (each coefficient off by at most 1.5 from the exact value
gives at most 1.5 N / scale per slot).
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


def _check_row(O, ctx, z, m_dev, log_n, scale):
    N = 1 << log_n
    want = O.encode(z, log_n, scale)
    host = ctx.encode(z, scale)
    d_or = np.abs(m_dev - want)
    d_host = np.abs(m_dev - host)
    assert d_or.max() <= 1 and d_host.max() <= 1, (d_or.max(), d_host.max())
    assert np.count_nonzero(d_or) <= max(2, N // 1000)
    # the decoded slots recover z within the rounding bound
    back = O.decode(m_dev, log_n, scale)[: len(z)]
    assert np.max(np.abs(back - z)) <= 1.5 * N / scale


@pytest.mark.parametrize("log_n", [5, 6, 9, 10, 12, 13])
def test_encode_device_matches_oracle(torch, L, oracle_mod, log_n):
    O = oracle_mod
    N = 1 << log_n
    ctx = L.Context(log_n, (50, 45), (50,), device=0)
    rng = np.random.default_rng(100 + log_n)
    scale = 2.0 ** 30
    # full, ragged and single-slot rows, one all-zero row (nslots = 0 is its own call)
    for nslots in (N // 2, N // 2 - 3, 1):
        z = rng.normal(0.0, 1.0, size=(5, nslots))
        z[1] *= 1e3
        z[2, :: max(1, nslots // 7)] = 0.0
        m = ctx.encode_device(torch.from_numpy(z).cuda(), scale).cpu().numpy()
        assert m.shape == (5, N)
        for r in range(5):
            _check_row(O, ctx, z[r], m[r], log_n, scale)
    zero = ctx.encode_device(torch.zeros((3, 0), dtype=torch.float64, device="cuda"), scale)
    assert not zero.any()
    empty = ctx.encode_device(torch.zeros((0, N // 2), dtype=torch.float64, device="cuda"), scale)
    assert empty.shape == (0, N)


def test_encode_device_full_size_workload(torch, L, oracle_mod):
    """N = 2^16, scale 2^40: packed model updates of the N=2^16 workload's
    value distribution (the last chunk ragged), against the oracle."""
    O = oracle_mod
    log_n, scale = 16, 2.0 ** 40
    ctx = L.Context(log_n, (50, 50), (50,), device=0)
    w = synth.Workload("encode-full", log_n, (50,) * 2, (50,), 40, 2, 70000, 0.01, 0, "scale10", data_seed=5,
                       crypto_seed=6)
    upd = synth.client_updates(w)
    z = synth.pack(upd[0], 1 << (log_n - 1))  # 3 chunks, the last one ragged
    m = ctx.encode_device(torch.from_numpy(z).cuda(), scale).cpu().numpy()
    for r in range(z.shape[0]):
        _check_row(O, ctx, z[r], m[r], log_n, scale)


def test_encode_device_strided_rows(torch, L, oracle_mod):
    """Rows of a wider tensor (z_stride > nslots) encode as the narrow rows."""
    O = oracle_mod
    log_n, scale = 10, 2.0 ** 35
    ctx = L.Context(log_n, (50, 45), (50,), device=0)
    rng = np.random.default_rng(7)
    wide = torch.from_numpy(rng.normal(size=(4, 512))).cuda()
    narrow = wide[:, :300].contiguous()
    a = ctx.encode_device(wide[:, :300], scale).cpu().numpy()
    b = ctx.encode_device(narrow, scale).cpu().numpy()
    assert np.array_equal(a, b)
    for r in range(4):
        _check_row(O, ctx, narrow[r].cpu().numpy(), a[r], log_n, scale)


def test_encode_device_rejects_bad_arguments(torch, L):
    ctx = L.Context(5, (30, 28, 28), (30,), device=0)
    z = torch.zeros((2, 17), dtype=torch.float64, device="cuda")  # 17 > N/2 = 16
    with pytest.raises(L.LancelotError):
        ctx.encode_device(z, 2.0 ** 20)
    with pytest.raises(L.LancelotError):
        ctx.encode_device(torch.zeros((2, 4), dtype=torch.float64, device="cuda"), -1.0)


def test_device_ingest_encrypts_like_oracle(torch, L, oracle_mod):
    """Device encode, then lc_encrypt, equals the oracle's encryption of the
    device plaintexts bit for bit (the encryption randomness is the shared
    counter-based stream), and decrypts to the input within the noise."""
    O = oracle_mod
    log_n, qb, pb, scale = 12, (50, 40, 40), (50,), 2.0 ** 30
    ctx = L.Context(log_n, qb, pb, device=0)
    ctx.keygen(31)
    ora = O.Oracle(log_n, qb, pb)
    assert ora.primes == ctx.moduli
    pk = ora.pk(31, ora.secret(31))
    rng = np.random.default_rng(3)
    z = rng.normal(0.0, 0.5, size=(3, 1 << (log_n - 1)))
    m = ctx.encode_device(torch.from_numpy(z).cuda(), scale)
    ct = ctx.encrypt(m, seed=9, first_object=4)
    want = ora.encrypt(9, 4, m.cpu().numpy(), pk)
    assert np.array_equal(ct.cpu().numpy().view(np.uint64), want)
    pt = ctx.decrypt(ct).cpu().numpy().view(np.uint64)
    for r in range(3):
        back = ctx.decode(pt[r], scale)[: z.shape[1]].real
        assert np.max(np.abs(back - z[r])) < 1e-4
