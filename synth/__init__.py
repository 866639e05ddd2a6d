"""Seeded synthetic inputs for the encrypted pairwise-distance workloads.

This module holds workload definitions and random draws only: no step of the
method's arithmetic.  Both the CPU oracle's tests and the GPU path's tests and
benchmark take their inputs from here.

The paper's clients send trained LeNet/ResNet updates ("Model Length" column
of Table 1: 61,706 to 23.6M parameters).  No dataset or trained weight is
available, so i.i.d. Gaussian FP64 update vectors stand in for them, with the
lengths, client counts and Byzantine fractions of the workload table below.
Byzantine clients are the last c clients of a round.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    log_n: int
    q_bits: tuple
    p_bits: tuple
    scale_log2: int
    n_clients: int
    dim: int
    std: float
    n_byz: int
    attack: str          # "scale10" | "flip5" | "noise0.1"
    plan: tuple = ()     # rotate-and-sum block plan (levels per block); default all ones
    data_seed: int = 0
    crypto_seed: int = 0

    @property
    def N(self):
        return 1 << self.log_n

    @property
    def slots(self):
        return self.N // 2

    @property
    def n_ct(self):
        """LEN: ciphertexts per client, ceil(dim / slots)."""
        return -(-self.dim // self.slots)

    @property
    def n_pairs(self):
        return self.n_clients * (self.n_clients - 1) // 2

    @property
    def rot_plan(self):
        return tuple(self.plan) if self.plan else tuple([1] * (self.log_n - 1))


# Small case: N=2^12, 3 limbs (one 40-bit, two 30-bit) + one 40-bit special
# prime, scale 2^30, 4 clients x 2048 dims, the last one scaled x10.
CFG1 = Workload("n4096_l3_4clients_2048dim", 12, (40, 30, 30), (40,), 30, 4, 2048, 0.01, 1, "scale10",
                data_seed=1001, crypto_seed=2001)
# N=2^14, 8 x 50-bit limbs + 2 special, scale 2^40, 10 clients x 100,000 dims
# (13 ciphertexts each), the last two sign-flipped x5.
CFG2 = Workload("n16384_l8_10clients_100kdim", 14, (50,) * 8, (50,) * 2, 40, 10, 100_000, 0.01, 2, "flip5",
                data_seed=1002, crypto_seed=2002)
# N=2^16, 24 x 50-bit limbs + 4 special, scale 2^40, 20 clients x 11.2M dims
# (342 ciphertexts each), the last four replaced by N(0, 0.1^2) noise.
CFG3 = Workload("n65536_l24_20clients_11.2Mdim", 16, (50,) * 24, (50,) * 4, 40, 20, 11_200_000, 0.005, 4,
                "noise0.1", data_seed=1003, crypto_seed=2003)

WORKLOADS = {"cfg1": CFG1, "cfg2": CFG2, "cfg3": CFG3}


def client_updates(w: Workload, clients=None) -> np.ndarray:
    """float64 [n][dim] updates ~ N(0, std^2) with the Byzantine transform on the
    last n_byz clients.  Draws are per client (stream i of the seed), so any
    subset of clients can be generated alone and matches the full draw."""
    idx = range(w.n_clients) if clients is None else clients
    out = np.empty((len(list(idx)), w.dim), dtype=np.float64)
    for r, i in enumerate(idx):
        rng = np.random.Generator(np.random.PCG64([w.data_seed, i]))
        x = rng.normal(0.0, w.std, size=w.dim)
        if i >= w.n_clients - w.n_byz:
            if w.attack == "scale10":
                x = 10.0 * x
            elif w.attack == "flip5":
                x = -5.0 * x
            elif w.attack == "noise0.1":
                x = rng.normal(0.0, 0.1, size=w.dim)
            else:
                raise ValueError(w.attack)
        out[r] = x
    return out


def pack(update: np.ndarray, slots: int) -> np.ndarray:
    """[dim] -> [LEN][slots]: slot j of chunk k holds update[k*slots + j]; the
    tail of the last chunk is zero."""
    n_ct = -(-update.shape[-1] // slots)
    out = np.zeros((n_ct, slots), dtype=np.float64)
    out.reshape(-1)[: update.shape[-1]] = update
    return out


def uniform_residues(rng_seed: int, moduli, shape_tail) -> np.ndarray:
    """Uniform residues in [0, q_l) for each limb l: [..., nlimb, N] with the
    limb axis second to last."""
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    moduli = [int(q) for q in moduli]
    *lead, N = shape_tail
    out = np.empty(tuple(lead) + (len(moduli), N), dtype=np.uint64)
    for l, q in enumerate(moduli):
        out[..., l, :] = rng.integers(0, q, size=tuple(lead) + (N,), dtype=np.uint64)
    return out


def small_workload(log_n=5, q_bits=(30, 28, 28), p_bits=(30,), n_clients=4, dim=40, scale_log2=20,
                   name="tiny") -> Workload:
    """A tiny workload for fast CPU tests (parity at several tiles needs larger N)."""
    return Workload(name, log_n, tuple(q_bits), tuple(p_bits), scale_log2, n_clients, dim, 0.01, 1, "scale10",
                    data_seed=77, crypto_seed=88)


def device_residues(torch, rng_seed: int, bits: int, shape):
    """Uniform integers in [0, 2^bits) generated on the GPU from a seeded
    torch generator (int64 storage).  With bits <= 49 they are canonical
    residues of every prime of 50 bits, so full-size inputs never cross the
    host."""
    g = torch.Generator(device="cuda")
    g.manual_seed(rng_seed)
    t = torch.empty(tuple(shape), dtype=torch.int64, device="cuda")
    t.random_(0, 1 << bits, generator=g)
    return t


def device_residues_mod(torch, rng_seed: int, moduli, shape):
    """Uniform residues in [0, q_l) for each limb l, generated on the GPU from
    a seeded torch generator (int64 storage): shape [..., nlimb, N] with the
    limb axis second to last and len(moduli) == nlimb, so full-size inputs
    span each limb's whole range and never cross the host."""
    g = torch.Generator(device="cuda")
    g.manual_seed(rng_seed)
    t = torch.empty(tuple(shape), dtype=torch.int64, device="cuda")
    assert t.shape[-2] == len(moduli)
    for l, q in enumerate(moduli):
        t[..., l, :].random_(0, int(q), generator=g)
    return t
