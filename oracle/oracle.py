"""Python side of the CPU oracle for Lancelot's encrypted pairwise distances.

TEST INFRASTRUCTURE ONLY.  Only tests/, ``__graft_entry__.smoke()`` and
``bench.py``'s cpu_baseline leg may import this module.  It never imports the
HIP package and the HIP package never imports it.

What lives here:
  * a ctypes shim over ``liblancelot_oracle.so`` (plain C, ``% q`` arithmetic,
    textbook transforms), built by ``build()`` below;
  * the FP64 parts of the scheme -- CKKS encode/decode through the canonical
    embedding (Methods, "Batch Encoding and Decoding") using numpy's FFT as a
    library step;
  * exact CRT with Python integers, to read a decrypted polynomial;
  * the KGC-side selection rules applied to decrypted distances (Krum,
    Multi-Krum, Median; Appendix "Descriptions of Aggregation Rules" and
    Algorithm 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblancelot_oracle.so")
SRC_PATH = os.path.join(HERE, "lancelot_oracle.c")

u64 = ctypes.c_uint64
i64 = ctypes.c_int64
P_U64 = ctypes.POINTER(ctypes.c_uint64)
P_I64 = ctypes.POINTER(ctypes.c_int64)
P_INT = ctypes.POINTER(ctypes.c_int)

# PRNG domains of the oracle's stream layout (object ids are per domain).
DOM_SK, DOM_PK_A, DOM_PK_E, DOM_ENC_V, DOM_ENC_E0, DOM_ENC_E1, DOM_KSK_A, DOM_KSK_E = range(1, 9)

_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP over independent limbs)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", LIB_PATH, SRC_PATH]
        subprocess.run(cmd, check=True)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "orc_mulmod": (u64, [u64, u64, u64]),
            "orc_addmod": (u64, [u64, u64, u64]),
            "orc_submod": (u64, [u64, u64, u64]),
            "orc_powmod": (u64, [u64, u64, u64]),
            "orc_invmod": (u64, [u64, u64]),
            "orc_is_prime": (ctypes.c_int, [u64]),
            "orc_find_primes": (ctypes.c_int, [ctypes.c_int, P_INT, ctypes.c_int, P_U64]),
            "orc_min_psi": (u64, [u64, ctypes.c_int]),
            "orc_ntt_direct": (None, [P_U64, P_U64, ctypes.c_int, u64, u64]),
            "orc_ntt": (None, [P_U64, ctypes.c_int, u64, u64]),
            "orc_intt": (None, [P_U64, ctypes.c_int, u64, u64]),
            "orc_negacyclic_mul": (None, [P_U64, P_U64, P_U64, ctypes.c_int, u64]),
            "orc_philox4x64_10": (None, [P_U64, P_U64, P_U64]),
            "orc_draw_word": (u64, [u64, u64, u64, u64]),
            "orc_sample_ternary": (None, [u64, u64, u64, u64, P_I64]),
            "orc_sample_gaussian": (None, [u64, u64, u64, u64, P_I64]),
            "orc_sample_uniform": (None, [u64, u64, u64, u64, u64, P_U64]),
            "orc_cdt_sample": (i64, [u64]),
            "orc_cdt_table": (None, [P_U64]),
            "orc_ctx_new": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_int, ctypes.c_int, P_U64]),
            "orc_ctx_free": (None, [ctypes.c_void_p]),
            "orc_ctx_psi": (u64, [ctypes.c_void_p, ctypes.c_int]),
            "orc_ctx_dnum": (ctypes.c_int, [ctypes.c_void_p]),
            "orc_poly_ntt": (None, [ctypes.c_void_p, P_U64, ctypes.c_int, ctypes.c_int]),
            "orc_poly_intt": (None, [ctypes.c_void_p, P_U64, ctypes.c_int, ctypes.c_int]),
            "orc_signed_to_ntt": (None, [ctypes.c_void_p, P_I64, P_U64, ctypes.c_int]),
            "orc_automorphism_index": (None, [ctypes.c_int, u64, P_U64]),
            "orc_automorphism_coeff": (None, [P_I64, P_I64, ctypes.c_int, u64]),
            "orc_automorphism_ntt": (None, [ctypes.c_void_p, P_U64, P_U64, ctypes.c_int, u64]),
            "orc_galois_elt": (u64, [ctypes.c_int, i64]),
            "orc_sample_secret": (None, [u64, u64, P_I64]),
            "orc_keygen_pk_with": (None, [ctypes.c_void_p, P_I64, P_U64, P_I64, P_U64]),
            "orc_keygen_pk": (None, [ctypes.c_void_p, u64, P_I64, P_U64]),
            "orc_keygen_ksk_with": (None, [ctypes.c_void_p, P_I64, P_I64, P_U64, P_I64, P_U64]),
            "orc_keygen_ksk": (None, [ctypes.c_void_p, u64, u64, P_I64, P_I64, P_U64]),
            "orc_secret_square": (None, [P_I64, P_I64, ctypes.c_int]),
            "orc_encrypt_with": (None, [ctypes.c_void_p, P_I64, P_I64, P_I64, P_I64, P_U64, P_U64]),
            "orc_encrypt": (None, [ctypes.c_void_p, u64, u64, P_I64, u64, P_U64, P_U64]),
            "orc_decrypt": (None, [ctypes.c_void_p, P_U64, ctypes.c_int, P_I64, P_U64]),
            "orc_ct_add": (None, [ctypes.c_void_p, P_U64, P_U64, P_U64, ctypes.c_int]),
            "orc_ct_sub": (None, [ctypes.c_void_p, P_U64, P_U64, P_U64, ctypes.c_int]),
            "orc_ct_mul": (None, [ctypes.c_void_p, P_U64, P_U64, P_U64]),
            "orc_mul_plain": (None, [ctypes.c_void_p, P_U64, P_U64, P_U64]),
            "orc_modup": (None, [ctypes.c_void_p, P_U64, P_U64]),
            "orc_moddown": (None, [ctypes.c_void_p, P_U64, P_U64]),
            "orc_keyswitch": (None, [ctypes.c_void_p, P_U64, P_U64, P_U64]),
            "orc_relin": (None, [ctypes.c_void_p, P_U64, P_U64, P_U64]),
            "orc_rotate_hoisted": (None, [ctypes.c_void_p, P_U64, P_I64, ctypes.c_int,
                                          ctypes.POINTER(P_U64), P_U64]),
            "orc_rotate_sum": (ctypes.c_int, [ctypes.c_void_p, P_U64, P_INT, ctypes.c_int,
                                              ctypes.POINTER(P_U64)]),
            "orc_pair_triple": (None, [ctypes.c_void_p, P_U64, ctypes.c_int, ctypes.c_int, ctypes.c_int, P_U64]),
            "orc_pairwise": (ctypes.c_int, [ctypes.c_void_p, P_U64, ctypes.c_int, ctypes.c_int, P_U64, P_INT,
                                            ctypes.c_int, ctypes.POINTER(P_U64), P_U64, P_U64, P_U64, P_INT,
                                            ctypes.c_int]),
            "orc_masked_sum": (None, [ctypes.c_void_p, P_U64, ctypes.c_int, ctypes.c_int, P_U64, P_U64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _pu(a):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(P_U64)


def _pi(a):
    assert a.dtype == np.int64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(P_I64)


def _u(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def _s(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _key_ptrs(keys):
    arr = (P_U64 * max(1, len(keys)))()
    for t, k in enumerate(keys):
        arr[t] = _pu(k)
    return arr


# --------------------------------------------------------------------------
# Scalar helpers
# --------------------------------------------------------------------------

def mulmod(a, b, q):
    return int(lib().orc_mulmod(a, b, q))


def addmod(a, b, q):
    return int(lib().orc_addmod(a, b, q))


def submod(a, b, q):
    return int(lib().orc_submod(a, b, q))


def powmod(a, e, q):
    return int(lib().orc_powmod(a, e, q))


def invmod(a, q):
    return int(lib().orc_invmod(a, q))


def is_prime(n):
    return bool(lib().orc_is_prime(n))


def find_primes(log_m: int, bits) -> list[int]:
    bits = list(bits)
    arr = (ctypes.c_int * len(bits))(*bits)
    out = np.zeros(len(bits), dtype=np.uint64)
    rc = lib().orc_find_primes(log_m, arr, len(bits), _pu(out))
    if rc != 0:
        raise ValueError("prime search ran out of candidates")
    return [int(x) for x in out]


def min_psi(q: int, log_n: int) -> int:
    return int(lib().orc_min_psi(q, log_n))


def ntt_direct(a, q, psi):
    a = _u(a)
    out = np.zeros_like(a)
    lib().orc_ntt_direct(_pu(a), _pu(out), int(len(a)).bit_length() - 1, q, psi)
    return out


def ntt(a, q, psi):
    a = _u(a).copy()
    lib().orc_ntt(_pu(a), int(len(a)).bit_length() - 1, q, psi)
    return a


def intt(a, q, psi):
    a = _u(a).copy()
    lib().orc_intt(_pu(a), int(len(a)).bit_length() - 1, q, psi)
    return a


def negacyclic_mul(a, b, q):
    a, b = _u(a), _u(b)
    out = np.zeros_like(a)
    lib().orc_negacyclic_mul(_pu(a), _pu(b), _pu(out), int(len(a)).bit_length() - 1, q)
    return out


def philox(ctr, key):
    c = _u(ctr)
    k = _u(key)
    o = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_pu(c), _pu(k), _pu(o))
    return o


def draw_word(seed, domain, obj, w):
    return int(lib().orc_draw_word(seed, domain, obj, w))


def sample_ternary(seed, domain, obj, n):
    out = np.zeros(n, dtype=np.int64)
    lib().orc_sample_ternary(seed, domain, obj, n, _pi(out))
    return out


def sample_gaussian(seed, domain, obj, n):
    out = np.zeros(n, dtype=np.int64)
    lib().orc_sample_gaussian(seed, domain, obj, n, _pi(out))
    return out


def sample_uniform(seed, domain, obj, q, n):
    out = np.zeros(n, dtype=np.uint64)
    lib().orc_sample_uniform(seed, domain, obj, q, n, _pu(out))
    return out


def cdt_sample(w):
    return int(lib().orc_cdt_sample(w))


def cdt_table():
    out = np.zeros(38, dtype=np.uint64)
    lib().orc_cdt_table(_pu(out))
    return out


def automorphism_index(log_n, g):
    out = np.zeros(1 << log_n, dtype=np.uint64)
    lib().orc_automorphism_index(log_n, g, _pu(out))
    return out


def automorphism_coeff(a, g):
    a = _s(a)
    out = np.zeros_like(a)
    lib().orc_automorphism_coeff(_pi(a), _pi(out), int(len(a)).bit_length() - 1, g)
    return out


def galois_elt(log_n, k):
    return int(lib().orc_galois_elt(log_n, k))


def secret_square(s):
    s = _s(s)
    out = np.zeros_like(s)
    lib().orc_secret_square(_pi(s), _pi(out), int(len(s)).bit_length() - 1)
    return out


# --------------------------------------------------------------------------
# FP64 encode / decode (Methods, "Batch Encoding and Decoding").
# Slot j sits at the root zeta_j = xi^(5^j mod 2N), xi = exp(i pi / N), i.e.
# T = <5> (reading of the unnamed order-N/2 subgroup).  Encode rounds half
# away from zero.
# --------------------------------------------------------------------------

def slot_exponents(log_n):
    N = 1 << log_n
    two_n = 2 * N
    e = np.empty(N // 2, dtype=np.int64)
    x = 1
    for j in range(N // 2):
        e[j] = x
        x = (x * 5) % two_n
    return e


def round_half_away(x):
    return np.where(x >= 0, np.floor(x + 0.5), -np.floor(-x + 0.5))


def encode(z, log_n: int, scale: float) -> np.ndarray:
    """m = round(scale * sigma^-1(pi^-1(z))): coefficients of the plaintext."""
    N = 1 << log_n
    half = N // 2
    zz = np.zeros(half, dtype=np.complex128)
    z = np.asarray(z)
    assert z.shape[-1] <= half
    zz[: z.shape[-1]] = z
    e = slot_exponents(log_n)
    u = np.zeros(N, dtype=np.complex128)  # u[t] = value at exponent 2t+1
    u[(e - 1) // 2] = zz
    u[(2 * N - e - 1) // 2] = np.conj(zz)
    F = np.fft.fft(u)
    k = np.arange(N)
    val = (scale / N) * np.real(np.exp(-1j * np.pi * k / N) * F)
    return round_half_away(val).astype(np.int64)


def decode(m, log_n: int, scale: float) -> np.ndarray:
    """z = pi(sigma(m / scale)) for real (float64) coefficients m."""
    N = 1 << log_n
    m = np.asarray(m, dtype=np.float64)
    k = np.arange(N)
    vals = N * np.fft.ifft(m * np.exp(1j * np.pi * k / N))  # vals[t] = m(xi^(2t+1))
    e = slot_exponents(log_n)
    return vals[(e - 1) // 2] / scale


# --------------------------------------------------------------------------
# Exact CRT with Python integers.
# --------------------------------------------------------------------------

def crt_centered(residues, moduli, coeffs=None):
    """residues [nq][N] (uint64) -> list of centred Python ints, one per
    coefficient (or only the listed coefficient indices)."""
    Q = 1
    for q in moduli:
        Q *= int(q)
    basis = []
    for q in moduli:
        q = int(q)
        Qi = Q // q
        basis.append(Qi * pow(Qi % q, -1, q))
    res = np.asarray(residues)
    idx = range(res.shape[1]) if coeffs is None else coeffs
    out = []
    for t in idx:
        x = 0
        for i, b in enumerate(basis):
            x += int(res[i, t]) * b
        x %= Q
        if x > Q // 2:
            x -= Q
        out.append(x)
    return out


# --------------------------------------------------------------------------
# Parameter set and scheme operations
# --------------------------------------------------------------------------

def pair_triple_columns(xi, xj, q) -> np.ndarray:
    """One client pair's tensor-squared differences summed over the packed
    ciphertexts (Methods, Computing the Pairwise Distances: the squared
    difference as a ciphertext-ciphertext product, relinearized once after the
    sum as in Methods, Lazy Relinearization), from the definition, on residue
    columns.  xi, xj: [LEN][2][m] residues of one limb (modulus q) of clients
    i and j at m coefficient positions, in the NTT domain where the tensor
    product is pointwise.  Returns [3][m]: sum_k d0^2, 2 sum_k d0 d1 and
    sum_k d1^2 mod q, with (d0, d1) = ct_i[k] - ct_j[k], in Python integers."""
    q = int(q)
    a = np.asarray(xi, dtype=np.uint64).astype(object)
    b = np.asarray(xj, dtype=np.uint64).astype(object)
    d0, d1 = a[:, 0, :] - b[:, 0, :], a[:, 1, :] - b[:, 1, :]
    out = np.empty((3, a.shape[2]), dtype=np.uint64)
    out[0] = [int(v) % q for v in (d0 * d0).sum(axis=0)]
    out[1] = [(2 * int(v)) % q for v in (d0 * d1).sum(axis=0)]
    out[2] = [int(v) % q for v in (d1 * d1).sum(axis=0)]
    return out


def masked_sum_columns(cols, masks, q) -> np.ndarray:
    """The server's plaintext-mask aggregate (Algorithm 1: the mask products
    summed over clients, Methods, Masked-Based Encrypted Sorting), from the
    definition, on residue columns: cols [n][LEN][2][m] residues of one limb
    (modulus q) of every client's packed ciphertexts at m coefficient
    positions, masks [n][m] the clients' mask plaintexts there, both in the
    NTT domain where the plaintext product is pointwise.  Returns
    [LEN][2][m]: sum_i cols[i] * masks[i] mod q, in Python integers."""
    q = int(q)
    c = np.asarray(cols, dtype=np.uint64).astype(object)
    w = np.asarray(masks, dtype=np.uint64).astype(object)
    acc = (c * w[:, None, None, :]).sum(axis=0)
    return np.vectorize(lambda v: int(v) % q, otypes=[object])(acc).astype(np.uint64)


class Oracle:
    """One RNS-CKKS parameter set: N = 2^log_n, q_0..q_L then p_0..p_{K-1},
    digit size alpha = K, dnum = ceil((L+1)/alpha)."""

    def __init__(self, log_n: int, q_bits, p_bits, log_m: int | None = None, primes=None):
        self.log_n = log_n
        self.N = 1 << log_n
        self.log_m = log_n + 1 if log_m is None else log_m
        self.nq = len(q_bits)
        self.np_ = len(p_bits)
        if primes is None:
            primes = find_primes(self.log_m, list(q_bits) + list(p_bits))
        self.primes = [int(x) for x in primes]
        self.q = self.primes[: self.nq]
        self.p = self.primes[self.nq:]
        arr = np.array(self.primes, dtype=np.uint64)
        self._ctx = lib().orc_ctx_new(log_n, self.nq, self.np_, _pu(arr))
        if not self._ctx:
            raise ValueError("bad parameter set")
        self.alpha = self.np_
        self.dnum = int(lib().orc_ctx_dnum(self._ctx))
        self.psi = [int(lib().orc_ctx_psi(self._ctx, i)) for i in range(len(self.primes))]

    def __del__(self):
        try:
            if self._ctx:
                lib().orc_ctx_free(self._ctx)
        except Exception:
            pass

    # shapes
    @property
    def ne(self):
        return self.nq + self.np_

    def ct_shape(self, ncomp=2):
        return (ncomp, self.nq, self.N)

    # transforms over the basis
    def poly_ntt(self, p, limb0=0):
        p = _u(p).copy()
        lib().orc_poly_ntt(self._ctx, _pu(p), limb0, p.shape[0])
        return p

    def poly_intt(self, p, limb0=0):
        p = _u(p).copy()
        lib().orc_poly_intt(self._ctx, _pu(p), limb0, p.shape[0])
        return p

    def signed_to_ntt(self, s, nlimb=None):
        nlimb = self.nq if nlimb is None else nlimb
        s = _s(s)
        out = np.zeros((nlimb, self.N), dtype=np.uint64)
        lib().orc_signed_to_ntt(self._ctx, _pi(s), _pu(out), nlimb)
        return out

    def automorphism_ntt(self, x, g):
        x = _u(x)
        out = np.zeros_like(x)
        lib().orc_automorphism_ntt(self._ctx, _pu(x), _pu(out), x.size // self.N, g)
        return out

    # keys
    def secret(self, seed):
        s = np.zeros(self.N, dtype=np.int64)
        lib().orc_sample_secret(seed, self.N, _pi(s))
        return s

    def pk(self, seed, s):
        out = np.zeros((2, self.nq, self.N), dtype=np.uint64)
        lib().orc_keygen_pk(self._ctx, seed, _pi(_s(s)), _pu(out))
        return out

    def pk_with(self, s, a_ntt, e):
        out = np.zeros((2, self.nq, self.N), dtype=np.uint64)
        lib().orc_keygen_pk_with(self._ctx, _pi(_s(s)), _pu(_u(a_ntt)), _pi(_s(e)), _pu(out))
        return out

    def ksk(self, seed, key_id, s, s_target):
        out = np.zeros((self.dnum, 2, self.ne, self.N), dtype=np.uint64)
        lib().orc_keygen_ksk(self._ctx, seed, key_id, _pi(_s(s)), _pi(_s(s_target)), _pu(out))
        return out

    def ksk_with(self, s, s_target, a_all, e_all):
        out = np.zeros((self.dnum, 2, self.ne, self.N), dtype=np.uint64)
        lib().orc_keygen_ksk_with(self._ctx, _pi(_s(s)), _pi(_s(s_target)), _pu(_u(a_all)), _pi(_s(e_all)),
                                  _pu(out))
        return out

    def relin_key(self, seed, s):
        return self.ksk(seed, 0, s, secret_square(s))

    def rot_key(self, seed, s, step):
        g = galois_elt(self.log_n, step)
        return self.ksk(seed, g, s, automorphism_coeff(s, g))

    def rotsum_steps(self, plan):
        """Rotation steps used by rotate_sum with block plan, in key order."""
        steps, j0 = [], 0
        for kb in plan:
            steps += [t << j0 for t in range(1, 1 << kb)]
            j0 += kb
        return steps

    # encryption
    def encrypt(self, seed, first_object, m, pk):
        m = _s(np.atleast_2d(m))
        cnt = m.shape[0]
        out = np.zeros((cnt, 2, self.nq, self.N), dtype=np.uint64)
        lib().orc_encrypt(self._ctx, seed, first_object, _pi(m), cnt, _pu(_u(pk)), _pu(out))
        return out

    def encrypt_with(self, m, r, e0, e1, pk):
        out = np.zeros((2, self.nq, self.N), dtype=np.uint64)
        lib().orc_encrypt_with(self._ctx, _pi(_s(m)), _pi(_s(r)), _pi(_s(e0)), _pi(_s(e1)), _pu(_u(pk)), _pu(out))
        return out

    def decrypt(self, ct, s):
        ct = _u(ct)
        ncomp = ct.shape[0]
        out = np.zeros((self.nq, self.N), dtype=np.uint64)
        lib().orc_decrypt(self._ctx, _pu(ct), ncomp, _pi(_s(s)), _pu(out))
        return out

    # evaluation
    def add(self, a, b):
        a, b = _u(a), _u(b)
        out = np.zeros_like(a)
        lib().orc_ct_add(self._ctx, _pu(a), _pu(b), _pu(out), a.shape[0])
        return out

    def sub(self, a, b):
        a, b = _u(a), _u(b)
        out = np.zeros_like(a)
        lib().orc_ct_sub(self._ctx, _pu(a), _pu(b), _pu(out), a.shape[0])
        return out

    def mul(self, a, b):
        out = np.zeros((3, self.nq, self.N), dtype=np.uint64)
        lib().orc_ct_mul(self._ctx, _pu(_u(a)), _pu(_u(b)), _pu(out))
        return out

    def mul_plain(self, ct, pt):
        out = np.zeros((2, self.nq, self.N), dtype=np.uint64)
        lib().orc_mul_plain(self._ctx, _pu(_u(ct)), _pu(_u(pt)), _pu(out))
        return out

    def modup(self, x):
        out = np.zeros((self.dnum, self.ne, self.N), dtype=np.uint64)
        lib().orc_modup(self._ctx, _pu(_u(x)), _pu(out))
        return out

    def moddown(self, u):
        out = np.zeros((self.nq, self.N), dtype=np.uint64)
        lib().orc_moddown(self._ctx, _pu(_u(u)), _pu(out))
        return out

    def keyswitch(self, x, ksk):
        out = np.zeros((2, self.nq, self.N), dtype=np.uint64)
        lib().orc_keyswitch(self._ctx, _pu(_u(x)), _pu(_u(ksk)), _pu(out))
        return out

    def relin(self, ct3, rlk):
        out = np.zeros((2, self.nq, self.N), dtype=np.uint64)
        lib().orc_relin(self._ctx, _pu(_u(ct3)), _pu(_u(rlk)), _pu(out))
        return out

    def rotate_hoisted(self, ct, steps, rks):
        steps_a = np.array(steps, dtype=np.int64)
        rks = [_u(k) for k in rks]
        out = np.zeros((len(steps), 2, self.nq, self.N), dtype=np.uint64)
        lib().orc_rotate_hoisted(self._ctx, _pu(_u(ct)), _pi(steps_a), len(steps), _key_ptrs(rks), _pu(out))
        return out

    def rotate_sum(self, ct, plan, rks):
        ct = _u(ct).copy()
        rks = [_u(k) for k in rks]
        plan_a = (ctypes.c_int * len(plan))(*plan)
        rc = lib().orc_rotate_sum(self._ctx, _pu(ct), plan_a, len(plan), _key_ptrs(rks))
        if rc != 0:
            raise ValueError("malformed rotate-sum plan")
        return ct

    def pair_triple(self, cts, i, j):
        cts = _u(cts)
        out = np.zeros((3, self.nq, self.N), dtype=np.uint64)
        lib().orc_pair_triple(self._ctx, _pu(cts), cts.shape[1], i, j, _pu(out))
        return out

    def pairwise(self, cts, rlk, plan, rks, want_sumdis=True, want_triples=False, pairs=None):
        """cts [n][len][2][nq][N] -> dict(dist=[P][2][nq][N], sumdis=..., triples=...)."""
        cts = _u(cts)
        n, ln = cts.shape[0], cts.shape[1]
        P = n * (n - 1) // 2
        dist = np.zeros((P, 2, self.nq, self.N), dtype=np.uint64)
        sumdis = np.zeros((n, 2, self.nq, self.N), dtype=np.uint64) if (want_sumdis and pairs is None) else None
        triples = np.zeros((P, 3, self.nq, self.N), dtype=np.uint64) if want_triples else None
        rks = [_u(k) for k in rks]
        plan_a = (ctypes.c_int * len(plan))(*plan)
        if pairs is not None:
            pa = (ctypes.c_int * len(pairs))(*pairs)
            npairs = len(pairs)
        else:
            pa, npairs = None, 0
        rc = lib().orc_pairwise(self._ctx, _pu(cts), n, ln, _pu(_u(rlk)), plan_a, len(plan), _key_ptrs(rks),
                                _pu(dist), _pu(sumdis) if sumdis is not None else None,
                                _pu(triples) if triples is not None else None, pa, npairs)
        if rc != 0:
            raise ValueError("pairwise failed")
        return {"dist": dist, "sumdis": sumdis, "triples": triples}

    def pair_distance(self, cts, i, j, rlk, plan, rks):
        """One pair's distance ciphertext (Algorithm 1, Server Executes): the
        lazily accumulated triple of (i, j), one relinearization, then the
        rotate-and-sum with `plan` -- what `pairwise` computes for that pair."""
        return self.rotate_sum(self.relin(self.pair_triple(cts, i, j), rlk), plan, rks)

    def sumdis_lazy(self, cts, rlk, plan, rks, clients=None):
        """SumDis with one relinearization per client (Algorithm 1, the SumDis
        line; Methods, Lazy Relinearization: triples are summed before the
        single relinearization): for client i, the squared-difference triples
        of every pair (i, j), j != i, summed over the packed ciphertexts and
        over j, then relinearized once and rotate-summed with `plan`.
        cts [n][len][2][nq][N] -> [len(clients)][2][nq][N]."""
        n = cts.shape[0]
        out = []
        for i in (range(n) if clients is None else clients):
            acc = None
            for j in range(n):
                if j != i:
                    t = self.pair_triple(cts, min(i, j), max(i, j))
                    acc = t if acc is None else self.add(acc, t)
            out.append(self.rotate_sum(self.relin(acc, rlk), plan, rks))
        return np.stack(out)

    def masked_sum(self, cts, masks_ntt):
        cts = _u(cts)
        n, ln = cts.shape[0], cts.shape[1]
        out = np.zeros((ln, 2, self.nq, self.N), dtype=np.uint64)
        lib().orc_masked_sum(self._ctx, _pu(cts), n, ln, _pu(_u(masks_ntt)), _pu(out))
        return out

    # read-out
    def crt(self, residues, coeffs=None):
        return crt_centered(residues, self.q, coeffs)

    def decode_residues(self, residues, scale):
        vals = np.array([float(x) for x in self.crt(residues)], dtype=np.float64)
        return decode(vals, self.log_n, scale)

    def rescale(self, ct, nlimb=None):
        """CKKS rescaling by the last of `nlimb` Q limbs q_t (levels of the
        CKKS Scheme Description; the operation is the standard one, the paper
        does not spell it out): every coefficient c of every component, as an
        integer modulo Q_t = q_0 ... q_t, becomes the nearest integer to
        c / q_t, reduced modulo q_0 ... q_{t-1}.  ct [ncomp][nlimb][N] in the
        NTT domain -> [ncomp][nlimb - 1][N] in the NTT domain.  Written from
        the definition: inverse transform, CRT to Python integers, exact
        rounded division, reduction, forward transform (q_t is odd, so
        c / q_t is never a tie)."""
        ct = _u(ct)
        nlimb = ct.shape[-2] if nlimb is None else nlimb
        t = nlimb - 1
        mods = [int(q) for q in self.q[:nlimb]]
        qt = mods[t]
        out = np.zeros(ct.shape[:-2] + (t, self.N), dtype=np.uint64)
        for comp in range(ct.shape[0]):
            coef = self.poly_intt(ct[comp, :nlimb])
            vals = crt_centered(coef, mods)
            rounded = [(2 * v + qt) // (2 * qt) for v in vals]  # floor(v / qt + 1/2)
            low = np.array([[r % q for r in rounded] for q in mods[:t]], dtype=np.uint64)
            out[comp] = self.poly_ntt(low)
        return out

    def decode_level(self, residues, nlimb, scale):
        """Decode a coefficient-domain plaintext with residues for the first
        `nlimb` Q limbs."""
        vals = np.array([float(x) for x in crt_centered(residues[:nlimb], self.q[:nlimb])], dtype=np.float64)
        return decode(vals, self.log_n, scale)

    def read_distance(self, coeff_residues, scale):
        """Distance from a decrypted rotate-summed ciphertext: after the slot
        sum every slot holds the total, so coefficient 0 equals scale * d."""
        return float(self.crt(coeff_residues, [0])[0]) / scale


# --------------------------------------------------------------------------
# KGC-side selection on decrypted FP64 distances (Appendix, Descriptions of
# Aggregation Rules; Algorithm 2).  Ties go to the lower client index.
# --------------------------------------------------------------------------

def distance_matrix(pair_values, n):
    D = np.zeros((n, n))
    p = 0
    for i in range(n):
        for j in range(i + 1, n):
            D[i, j] = D[j, i] = pair_values[p]
            p += 1
    return D


def krum_scores(D, c):
    """s_i = sum of the n - c - 2 smallest distances from client i."""
    n = D.shape[0]
    m = n - c - 2
    scores = np.zeros(n)
    for i in range(n):
        others = np.sort(np.delete(D[i], i), kind="stable")
        scores[i] = others[: max(m, 0)].sum()
    return scores


def select(rule, D, c, l=None):
    """Selected client indices (0-based) for rule in {krum, multikrum, median}."""
    n = D.shape[0]
    scores = krum_scores(D, c)
    order = list(np.argsort(scores, kind="stable"))
    if rule == "krum":
        return [int(order[0])]
    if rule == "median":
        # Reading of Algorithm 2's index rule as 1-based: position ceil(n/2).
        return [int(order[(n + 1) // 2 - 1])]
    if rule == "multikrum":
        chosen = []
        while len(chosen) < l and n - len(chosen) > 2 * c + 2:
            chosen.append(int(order.pop(0)))
        return chosen
    raise ValueError(rule)


def permutation_mask(n, selected):
    """P_pi with rows e_{pi(j)} for selected positions and zero rows otherwise
    (Methods, Masked-based Encrypted Sorting)."""
    P = np.zeros((n, n), dtype=np.int64)
    for row, j in enumerate(selected):
        P[row, j] = 1
    return P
