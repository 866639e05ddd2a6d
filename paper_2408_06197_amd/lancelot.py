"""Thin ctypes binding of liblancelot.so (the C ABI in include/lancelot.h).

Argument marshalling only: every step of the distance path runs in the HIP
library.  Device buffers are torch tensors on the context's device, of dtype
int64 (residues are < 2^50, so the bits equal the ABI's uint64) or uint64;
streams are torch's current stream unless one is passed.  If the library has
not been built this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblancelot.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lancelot.h")

LC_OK, LC_EINVAL, LC_ENOMEM, LC_EKEY, LC_EHIP, LC_EUNSUP = 0, -1, -2, -3, -4, -5
ROLE_SERVER, ROLE_KGC = 0, 1

_c = ctypes
VP = _c.c_void_p
U64 = _c.c_uint64
PU64 = _c.POINTER(_c.c_uint64)
PI64 = _c.POINTER(_c.c_int64)
PINT = _c.POINTER(_c.c_int)
PD = _c.POINTER(_c.c_double)
SZ = _c.c_size_t
INT = _c.c_int


class LcParams(_c.Structure):
    _fields_ = [("log_n", INT), ("n_q", INT), ("n_p", INT), ("q_bits", PINT), ("p_bits", PINT), ("log_m", INT)]


class LcPolyGroup(_c.Structure):
    _fields_ = [("data", VP), ("count", SZ), ("log_n", INT), ("nlimb", INT), ("limb0", INT)]


KEY_PK, KEY_RELIN, KEY_ROTATION = 0, 1, 2
FP_SUMDIS, FP_PLAINTEXTS, FP_DECRYPT = 1, 2, 4


_SIGS = {
    "lc_ctx_create": [_c.POINTER(LcParams), INT, INT, _c.POINTER(VP)],
    "lc_ctx_destroy": [VP],
    "lc_last_error": [VP],
    "lc_ctx_moduli": [VP, PU64],
    "lc_ctx_info": [VP, PINT, PINT, PINT, PINT],
    "lc_sync": [VP, VP],
    "lc_ctx_device_bytes": [VP, _c.POINTER(SZ)],
    "lc_keygen": [VP, U64],
    "lc_keygen_rotation": [VP, U64, PINT, INT],
    "lc_keys_share": [VP, VP],
    "lc_secret_export": [VP, PI64],
    "lc_pk_export": [VP, PU64],
    "lc_ksk_export": [VP, INT, INT, PU64],
    "lc_key_import": [VP, INT, INT, PU64],
    "lc_encode": [VP, PD, PD, SZ, _c.c_double, PI64],
    "lc_encode_device": [VP, VP, SZ, SZ, SZ, _c.c_double, VP, VP],
    "lc_decode": [VP, PU64, _c.c_double, PD, PD],
    "lc_decode_level": [VP, PU64, INT, _c.c_double, PD, PD],
    "lc_crt_to_double": [VP, PU64, SZ, SZ, PD],
    "lc_gaussian_table": [VP, PU64],
    "lc_encrypt": [VP, VP, SZ, U64, U64, VP, VP],
    "lc_decrypt": [VP, VP, INT, SZ, VP, VP],
    "lc_decrypt_level": [VP, VP, INT, INT, SZ, VP, VP],
    "lc_rescale": [VP, VP, SZ, INT, INT, VP, VP],
    "lc_ct_sub": [VP, VP, VP, VP, SZ, INT, VP],
    "lc_ct_add": [VP, VP, VP, VP, SZ, INT, VP],
    "lc_ct_mul": [VP, VP, VP, VP, SZ, VP],
    "lc_ct_square": [VP, VP, VP, SZ, VP],
    "lc_relin": [VP, VP, VP, SZ, VP],
    "lc_relin_noalloc": [VP, VP, VP, SZ, VP],
    "lc_rotate_hoisted": [VP, VP, SZ, PINT, INT, VP, VP],
    "lc_rotate_sum": [VP, VP, SZ, PINT, INT, VP],
    "lc_mul_plain": [VP, VP, VP, VP, SZ, VP],
    "lc_masked_sum": [VP, VP, INT, INT, VP, VP, VP],
    "lc_mask_aggregate": [VP, VP, INT, INT, VP, VP, VP],
    "lc_release_workspace": [VP],
    "lc_pair_triples": [VP, VP, INT, INT, VP, VP],
    "lc_pair_triples_acc": [VP, VP, INT, INT, VP, VP],
    "lc_pairwise_finish": [VP, VP, INT, PINT, INT, VP, VP, VP],
    "lc_pairwise_sqdist": [VP, VP, INT, INT, PINT, INT, VP, VP, VP],
    "lc_sumdis_lazy": [VP, VP, INT, INT, PINT, INT, VP, VP],
    "lc_ntt_fwd_groups": [VP, VP, INT, VP],
    "lc_ntt_inv_groups": [VP, VP, INT, VP],
    "lc_footprint": [VP, INT, INT, INT, INT, _c.POINTER(SZ), _c.POINTER(SZ)],
    "lc_ntt_fwd": [VP, VP, SZ, INT, INT, VP],
    "lc_ntt_inv": [VP, VP, SZ, INT, INT, VP],
    "lc_workspace_query": [VP, INT, INT, _c.POINTER(SZ)],
    "lc_set_workspace_limit": [VP, SZ],
    "lc_set_tuning": [VP, _c.c_char_p, INT],
}

_lib = None


class LancelotError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lancelot error {code}: {msg}")
        self.code = code


def header_symbols():
    """Function names declared in include/lancelot.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lc_\w+)\s*\(", txt, re.M)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblancelot.so is not built; run `python -m paper_2408_06197_amd.build`")
        L = _c.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _c.c_char_p if name == "lc_last_error" else INT
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        assert t.is_contiguous(), "tensor must be contiguous"
        return VP(t.data_ptr())
    raise TypeError("expected a torch tensor")


def _stream(stream):
    if stream is not None:
        return VP(stream if isinstance(stream, int) else stream.cuda_stream)
    import torch
    return VP(torch.cuda.current_stream().cuda_stream)


def _ints(vals):
    vals = list(vals)
    return (INT * max(1, len(vals)))(*vals), len(vals)


class Context:
    """One parameter set on one device (device=-1: host-only context)."""

    def __init__(self, log_n, q_bits, p_bits, log_m=0, device=0, role=ROLE_KGC):
        qb, _ = _ints(q_bits)
        pb, _ = _ints(p_bits)
        prm = LcParams(log_n, len(q_bits), len(p_bits), qb, pb, log_m)
        h = VP()
        rc = lib().lc_ctx_create(_c.byref(prm), device, role, _c.byref(h))
        if rc != LC_OK:
            raise LancelotError(rc, "lc_ctx_create failed")
        self._h = h
        self.device = device
        li, nq, np_, dn = INT(), INT(), INT(), INT()
        lib().lc_ctx_info(h, _c.byref(li), _c.byref(nq), _c.byref(np_), _c.byref(dn))
        self.log_n, self.nq, self.np, self.dnum = li.value, nq.value, np_.value, dn.value
        self.N = 1 << self.log_n
        self.ne = self.nq + self.np
        m = np.zeros(self.ne, dtype=np.uint64)
        lib().lc_ctx_moduli(h, m.ctypes.data_as(PU64))
        self.moduli = [int(x) for x in m]
        self.q = self.moduli[: self.nq]
        self.p = self.moduli[self.nq:]

    def close(self):
        if getattr(self, "_h", None):
            lib().lc_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != LC_OK:
            msg = lib().lc_last_error(self._h)
            raise LancelotError(rc, msg.decode() if msg else "")

    # ---- shapes / allocation helpers (torch) ----
    def empty(self, *shape, dtype=None):
        import torch
        return torch.empty(*shape, dtype=dtype or torch.int64, device=f"cuda:{self.device}")

    def ct_words(self, ncomp=2):
        return ncomp * self.nq * self.N

    # ---- keys ----
    def keygen(self, seed):
        self._check(lib().lc_keygen(self._h, seed))

    def keygen_rotation(self, seed, steps):
        a, n = _ints(steps)
        self._check(lib().lc_keygen_rotation(self._h, seed, a, n))

    def keys_share(self, dst: "Context"):
        self._check(lib().lc_keys_share(self._h, dst._h))

    def secret(self):
        out = np.zeros(self.N, dtype=np.int64)
        self._check(lib().lc_secret_export(self._h, out.ctypes.data_as(PI64)))
        return out

    def pk(self):
        out = np.zeros((2, self.nq, self.N), dtype=np.uint64)
        self._check(lib().lc_pk_export(self._h, out.ctypes.data_as(PU64)))
        return out

    def ksk(self, which=0, step=0):
        out = np.zeros((self.dnum, 2, self.ne, self.N), dtype=np.uint64)
        self._check(lib().lc_ksk_export(self._h, which, step, out.ctypes.data_as(PU64)))
        return out

    def rotsum_steps(self, plan):
        steps, j0 = [], 0
        for kb in plan:
            steps += [t << j0 for t in range(1, 1 << kb)]
            j0 += kb
        return steps

    def key_import(self, kind, blob, step=0):
        """Install a host key (numpy uint64: pk [2][nq][N] or a key-switching
        key [dnum][2][ne][N]) made outside the library."""
        b = np.ascontiguousarray(blob, dtype=np.uint64)
        want = (2, self.nq, self.N) if kind == KEY_PK else (self.dnum, 2, self.ne, self.N)
        if b.shape != want:
            raise ValueError(f"key shape {b.shape}, expected {want}")
        self._check(lib().lc_key_import(self._h, kind, step, b.ctypes.data_as(PU64)))

    # ---- host encode / decode ----
    def encode(self, z, scale):
        z = np.asarray(z)
        re_ = np.ascontiguousarray(z.real, dtype=np.float64)
        im_ = np.ascontiguousarray(z.imag, dtype=np.float64) if np.iscomplexobj(z) else None
        out = np.zeros(self.N, dtype=np.int64)
        self._check(lib().lc_encode(self._h, re_.ctypes.data_as(PD), im_.ctypes.data_as(PD) if im_ is not None
                                    else None, len(re_), scale, out.ctypes.data_as(PI64)))
        return out

    def decode(self, residues, scale):
        r = np.ascontiguousarray(residues, dtype=np.uint64)
        re_ = np.zeros(self.N // 2)
        im_ = np.zeros(self.N // 2)
        self._check(lib().lc_decode(self._h, r.ctypes.data_as(PU64), scale, re_.ctypes.data_as(PD),
                                    im_.ctypes.data_as(PD)))
        return re_ + 1j * im_

    def decode_level(self, residues, scale):
        """residues [nlimb][N] of the first nlimb Q limbs (coefficient domain)."""
        r = np.ascontiguousarray(residues, dtype=np.uint64)
        re_ = np.zeros(self.N // 2)
        im_ = np.zeros(self.N // 2)
        self._check(lib().lc_decode_level(self._h, r.ctypes.data_as(PU64), r.shape[0], scale,
                                          re_.ctypes.data_as(PD), im_.ctypes.data_as(PD)))
        return re_ + 1j * im_

    def crt_to_double(self, residues):
        """residues [nq][ncoeff] -> centred values as float64."""
        r = np.ascontiguousarray(residues, dtype=np.uint64)
        out = np.zeros(r.shape[1])
        self._check(lib().lc_crt_to_double(self._h, r.ctypes.data_as(PU64), r.shape[1], r.shape[1],
                                           out.ctypes.data_as(PD)))
        return out

    def gaussian_table(self):
        out = np.zeros(38, dtype=np.uint64)
        self._check(lib().lc_gaussian_table(self._h, out.ctypes.data_as(PU64)))
        return out

    # ---- device ops ----
    def encode_device(self, z, scale, out=None, stream=None):
        """z: float64 device tensor [count, nslots] (real slots, nslots <= N/2,
        rows contiguous) -> int64 device tensor [count, N] of plaintext
        coefficients, as `encode` computes them."""
        import torch
        if z.dtype != torch.float64 or z.dim() != 2 or z.stride(1) != 1:
            raise ValueError("z must be a float64 [count, nslots] tensor with contiguous rows")
        count, nslots = z.shape
        out = torch.empty((count, self.N), dtype=torch.int64, device=z.device) if out is None else out
        zp = VP(z.data_ptr()) if z.numel() else None  # rows may be strided (stride(1) == 1 checked above)
        self._check(lib().lc_encode_device(self._h, zp, count, nslots, z.stride(0) if count > 1 else nslots, scale,
                                           _ptr(out), _stream(stream)))
        return out

    def encrypt(self, m, seed, first_object=0, out=None, stream=None):
        count = m.shape[0]
        out = self.empty(count, 2, self.nq, self.N) if out is None else out
        self._check(lib().lc_encrypt(self._h, _ptr(m), count, seed, first_object, _ptr(out), _stream(stream)))
        return out

    def decrypt(self, ct, ncomp=None, out=None, stream=None):
        ncomp = ncomp or ct.shape[-3]
        count = ct.numel() // (ncomp * self.nq * self.N)
        out = self.empty(count, self.nq, self.N) if out is None else out
        self._check(lib().lc_decrypt(self._h, _ptr(ct), ncomp, count, _ptr(out), _stream(stream)))
        return out

    def decrypt_level(self, ct, nlimb, ncomp=2, out=None, stream=None):
        """ct [count][ncomp][nlimb][N] -> coefficient-domain [count][nlimb][N]."""
        count = ct.numel() // (ncomp * nlimb * self.N)
        out = self.empty(count, nlimb, self.N) if out is None else out
        self._check(lib().lc_decrypt_level(self._h, _ptr(ct), ncomp, nlimb, count, _ptr(out), _stream(stream)))
        return out

    def rescale(self, ct, nlimb, ncomp=2, out=None, stream=None):
        """ct [count][ncomp][nlimb][N] (NTT domain) -> [count][ncomp][nlimb - 1][N]."""
        count = ct.numel() // (ncomp * nlimb * self.N)
        out = self.empty(count, ncomp, nlimb - 1, self.N) if out is None else out
        self._check(lib().lc_rescale(self._h, _ptr(ct), count, ncomp, nlimb, _ptr(out), _stream(stream)))
        return out

    def ct_sub(self, a, b, out=None, ncomp=2, stream=None):
        out = self.empty(*a.shape) if out is None else out
        count = a.numel() // self.ct_words(ncomp)
        self._check(lib().lc_ct_sub(self._h, _ptr(a), _ptr(b), _ptr(out), count, ncomp, _stream(stream)))
        return out

    def ct_add(self, a, b, out=None, ncomp=2, stream=None):
        out = self.empty(*a.shape) if out is None else out
        count = a.numel() // self.ct_words(ncomp)
        self._check(lib().lc_ct_add(self._h, _ptr(a), _ptr(b), _ptr(out), count, ncomp, _stream(stream)))
        return out

    def ct_mul(self, a, b, out=None, stream=None):
        count = a.numel() // self.ct_words(2)
        out = self.empty(count, 3, self.nq, self.N) if out is None else out
        self._check(lib().lc_ct_mul(self._h, _ptr(a), _ptr(b), _ptr(out), count, _stream(stream)))
        return out

    def ct_square(self, a, out=None, stream=None):
        count = a.numel() // self.ct_words(2)
        out = self.empty(count, 3, self.nq, self.N) if out is None else out
        self._check(lib().lc_ct_square(self._h, _ptr(a), _ptr(out), count, _stream(stream)))
        return out

    def relin(self, ct3, out=None, stream=None):
        count = ct3.numel() // self.ct_words(3)
        out = self.empty(count, 2, self.nq, self.N) if out is None else out
        self._check(lib().lc_relin(self._h, _ptr(ct3), _ptr(out), count, _stream(stream)))
        return out

    def relin_noalloc(self, ct3, out, stream=None):
        """lc_relin_noalloc: relinearization with the library's fixed scratch
        array (no device allocation; `out` must be given)."""
        count = ct3.numel() // self.ct_words(3)
        self._check(lib().lc_relin_noalloc(self._h, _ptr(ct3), _ptr(out), count, _stream(stream)))
        return out

    def rotate_hoisted(self, ct, steps, out=None, stream=None):
        count = ct.numel() // self.ct_words(2)
        a, n = _ints(steps)
        out = self.empty(count, n, 2, self.nq, self.N) if out is None else out
        self._check(lib().lc_rotate_hoisted(self._h, _ptr(ct), count, a, n, _ptr(out), _stream(stream)))
        return out

    def rotate_sum(self, ct, plan=None, stream=None):
        count = ct.numel() // self.ct_words(2)
        if plan is None:
            pa, n = None, 0
        else:
            pa, n = _ints(plan)
        self._check(lib().lc_rotate_sum(self._h, _ptr(ct), count, pa, n, _stream(stream)))
        return ct

    def mul_plain(self, ct, pt, out=None, stream=None):
        count = ct.numel() // self.ct_words(2)
        out = self.empty(*ct.shape) if out is None else out
        self._check(lib().lc_mul_plain(self._h, _ptr(ct), _ptr(pt), _ptr(out), count, _stream(stream)))
        return out

    def masked_sum(self, cts, masks, out=None, stream=None):
        n, ln = cts.shape[0], cts.shape[1]
        out = self.empty(ln, 2, self.nq, self.N) if out is None else out
        self._check(lib().lc_masked_sum(self._h, _ptr(cts), n, ln, _ptr(masks), _ptr(out), _stream(stream)))
        return out

    def mask_aggregate(self, cts, mask_cts, out=None, stream=None):
        """sum_i cts[i][k] (x) mask_cts[i], relinearized: [len][2][n_q][N]."""
        n, ln = cts.shape[0], cts.shape[1]
        out = self.empty(ln, 2, self.nq, self.N) if out is None else out
        self._check(lib().lc_mask_aggregate(self._h, _ptr(cts), n, ln, _ptr(mask_cts), _ptr(out), _stream(stream)))
        return out

    def pair_triples(self, cts, out=None, stream=None):
        n, ln = cts.shape[0], cts.shape[1]
        P = n * (n - 1) // 2
        out = self.empty(P, 3, self.nq, self.N) if out is None else out
        self._check(lib().lc_pair_triples(self._h, _ptr(cts), n, ln, _ptr(out), _stream(stream)))
        return out

    def pair_triples_acc(self, cts, triples, stream=None):
        n, ln = cts.shape[0], cts.shape[1]
        self._check(lib().lc_pair_triples_acc(self._h, _ptr(cts), n, ln, _ptr(triples), _stream(stream)))
        return triples

    def pairwise_finish(self, triples, n, plan=None, sumdis=False, out=None, sumdis_out=None, stream=None):
        P = n * (n - 1) // 2
        out = self.empty(P, 2, self.nq, self.N) if out is None else out
        if sumdis and sumdis_out is None:
            sumdis_out = self.empty(n, 2, self.nq, self.N)
        pa, nb = (None, 0) if plan is None else _ints(plan)
        self._check(lib().lc_pairwise_finish(self._h, _ptr(triples), n, pa, nb, _ptr(out),
                                             _ptr(sumdis_out) if sumdis else None, _stream(stream)))
        return (out, sumdis_out) if sumdis else out

    def pairwise_sqdist(self, cts, plan=None, sumdis=False, out=None, sumdis_out=None, stream=None):
        n, ln = cts.shape[0], cts.shape[1]
        P = n * (n - 1) // 2
        out = self.empty(P, 2, self.nq, self.N) if out is None else out
        if sumdis and sumdis_out is None:
            sumdis_out = self.empty(n, 2, self.nq, self.N)
        if plan is None:
            pa, nb = None, 0
        else:
            pa, nb = _ints(plan)
        self._check(lib().lc_pairwise_sqdist(self._h, _ptr(cts), n, ln, pa, nb, _ptr(out),
                                             _ptr(sumdis_out) if sumdis else None, _stream(stream)))
        return (out, sumdis_out) if sumdis else out

    def sumdis_lazy(self, cts, plan=None, out=None, stream=None):
        """Per-client SumDis with one relinearization and rotate-and-sum per
        client: [n][2][n_q][N]."""
        n, ln = cts.shape[0], cts.shape[1]
        out = self.empty(n, 2, self.nq, self.N) if out is None else out
        pa, nb = (None, 0) if plan is None else _ints(plan)
        self._check(lib().lc_sumdis_lazy(self._h, _ptr(cts), n, ln, pa, nb, _ptr(out), _stream(stream)))
        return out

    def _groups(self, groups):
        arr = (LcPolyGroup * max(1, len(groups)))()
        for k, (t, log_n, nlimb, limb0) in enumerate(groups):
            count = t.numel() // (nlimb << log_n)
            arr[k] = LcPolyGroup(_ptr(t), count, log_n, nlimb, limb0)
        return arr, len(groups)

    def ntt_fwd_groups(self, groups, stream=None):
        """groups: [(tensor [count][nlimb][2^log_n], log_n, nlimb, limb0)],
        transformed in place, one launch per pass for all of them."""
        arr, n = self._groups(groups)
        self._check(lib().lc_ntt_fwd_groups(self._h, arr, n, _stream(stream)))

    def ntt_inv_groups(self, groups, stream=None):
        arr, n = self._groups(groups)
        self._check(lib().lc_ntt_inv_groups(self._h, arr, n, _stream(stream)))

    def footprint(self, n, len_, k_chunk=0, flags=0):
        """(round bytes, workspace bytes) of a pairwise-distance round."""
        rb, wb = SZ(), SZ()
        self._check(lib().lc_footprint(self._h, n, len_, k_chunk, flags, _c.byref(rb), _c.byref(wb)))
        return rb.value, wb.value

    def ntt_fwd(self, polys, nlimb, limb0=0, stream=None):
        count = polys.numel() // (nlimb * self.N)
        self._check(lib().lc_ntt_fwd(self._h, _ptr(polys), count, nlimb, limb0, _stream(stream)))
        return polys

    def ntt_inv(self, polys, nlimb, limb0=0, stream=None):
        count = polys.numel() // (nlimb * self.N)
        self._check(lib().lc_ntt_inv(self._h, _ptr(polys), count, nlimb, limb0, _stream(stream)))
        return polys

    def sync(self, stream=None):
        self._check(lib().lc_sync(self._h, _stream(stream)))

    def workspace_query(self, n, len_):
        b = SZ()
        self._check(lib().lc_workspace_query(self._h, n, len_, _c.byref(b)))
        return b.value

    def release_workspace(self):
        self._check(lib().lc_release_workspace(self._h))

    def set_tuning(self, name, value):
        self._check(lib().lc_set_tuning(self._h, name.encode(), int(value)))

    def set_workspace_limit(self, nbytes):
        self._check(lib().lc_set_workspace_limit(self._h, nbytes))

    def device_bytes(self):
        b = SZ()
        self._check(lib().lc_ctx_device_bytes(self._h, _c.byref(b)))
        return b.value
