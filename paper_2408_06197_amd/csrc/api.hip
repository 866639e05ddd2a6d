// The C ABI declared in include/lancelot.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lc_internal.h"

struct lc_ctx {
    lc::Ctx c;
};

namespace lc {

typedef unsigned __int128 u128;

int fail(Ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

int hip_fail(Ctx *c, hipError_t e, const char *what)
{
    return fail(c, LC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

u64 *ws_get(Ctx *c, int slot, size_t bytes, hipStream_t s)
{
    Ctx::Workspace &w = c->ws[s];
    if (w.bytes[slot] >= bytes && w.slot[slot]) return (u64 *)w.slot[slot];
    if (w.slot[slot]) {
        // a HIP graph captured on this stream may still name the old buffer:
        // retire it (freed with the context) rather than free it now
        c->retired.push_back(w.slot[slot]);
        c->retired_bytes += w.bytes[slot];
        w.slot[slot] = nullptr;
        w.bytes[slot] = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        hipGetLastError();
        c->err = "workspace allocation of " + std::to_string(bytes) + " bytes failed";
        return nullptr;
    }
    w.slot[slot] = p;
    w.bytes[slot] = bytes;
    return (u64 *)p;
}

static std::vector<u64> shoup_host(const std::vector<u64> &v, const std::vector<u64> &mod, int nlimb, u64 N)
{
    std::vector<u64> out(v.size());
    for (size_t i = 0; i < v.size(); i++) {
        int l = (int)((i / N) % (u64)nlimb);
        out[i] = (u64)(((u128)v[i] << 64) / mod[l]);
    }
    return out;
}

static int upload_shoup(Ctx *c, const u64 *dev, u64 *dev_sh, int nlimb, u64 count)
{
    size_t n = (size_t)count * nlimb * c->N;
    std::vector<u64> h(n);
    LC_HIP(c, hipMemcpy(h.data(), dev, n * 8, hipMemcpyDeviceToHost));
    std::vector<u64> sh = shoup_host(h, c->mod, nlimb, c->N);
    LC_HIP(c, hipMemcpy(dev_sh, sh.data(), n * 8, hipMemcpyHostToDevice));
    return LC_OK;
}

// Key-switching key from s to target t (NTT domain over all ne limbs).
static int gen_ksk(Ctx *c, u64 seed, u64 key_id, const u64 *t_ntt, u64 *ksk)
{
    const int ne = c->ne, nq = c->nq, alpha = c->alpha;
    const u64 N = c->N, NE = (u64)ne * N;
    u64 *tmp = ws_get(c, WS_KEYGEN, (NE + N + ne) * 8, 0);
    if (!tmp) return LC_ENOMEM;
    u64 *e_ntt = tmp;
    i64 *e_coef = (i64 *)(tmp + NE);
    u64 *gadget = tmp + NE + N;
    std::vector<u64> pmod(nq);
    LC_HIP(c, hipMemcpy(pmod.data(), c->dp.pmod, nq * 8, hipMemcpyDeviceToHost));
    int rc;
    for (int d = 0; d < c->dnum; d++) {
        u64 *k0 = ksk + (u64)d * 2 * NE, *k1 = k0 + NE;
        if ((rc = launch_uniform_limbs(c, seed, 7, (key_id << 32) | ((u64)d << 16), k1, ne, 0))) return rc;
        if ((rc = launch_gaussian(c, seed, 8, (key_id << 32) | (u64)d, e_coef, 0))) return rc;
        if ((rc = launch_signed_to_limbs(c, e_coef, e_ntt, ne, 1, 0))) return rc;
        if ((rc = launch_ntt_fwd(c, PolyBatch{e_ntt, 1, ne, (u64)ne, 0, 0}, 0))) return rc;
        std::vector<u64> g(ne, 0);
        for (int l = 0; l < nq; l++)
            if (l / alpha == d) g[l] = pmod[l];
        LC_HIP(c, hipMemcpy(gadget, g.data(), ne * 8, hipMemcpyHostToDevice));
        if ((rc = launch_keycombine(c, k1, e_ntt, c->sk_ntt, t_ntt, gadget, k0, k1, ne, 0))) return rc;
    }
    LC_HIP(c, hipDeviceSynchronize());
    return LC_OK;
}

static bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

// Overlap other than the same range: element-wise kernels that read each
// element before writing the same element may run in place, never shifted.
static bool partial_overlap(const void *a, size_t na, const void *b, size_t nb)
{
    return overlap(a, na, b, nb) && !(a == b && na == nb);
}

// Scratch of lc_relin_noalloc: a fixed device array (every GPU the library
// runs on holds its own copy from module load until the process ends).  In
// host code `scratch` names a host-side stand-in, never device memory: the
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current (scratch_init, called by lc_ctx_create) and kept in
// g_scratch.  Only those addresses are passed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)LC_NOALLOC_SCRATCH_MIB << 20;
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) u64 scratch[NOALLOC_SCRATCH_BYTES / sizeof(u64)];
static std::mutex g_scratch_mu;
static u64 *g_scratch[MAX_DEVICES] = {};

static int scratch_init(Ctx *c)
{
    if (c->device < 0 || c->device >= MAX_DEVICES) return fail(c, LC_EUNSUP, "device index outside 0..63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[c->device]) return LC_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(c, LC_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch[c->device] = (u64 *)p;
    return LC_OK;
}

static u64 *scratch_of(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return device >= 0 && device < MAX_DEVICES ? g_scratch[device] : nullptr;
}

static Ctx *C(lc_ctx *x) { return x ? &x->c : nullptr; }
static const Ctx *C(const lc_ctx *x) { return x ? &x->c : nullptr; }

static bool set_device(Ctx *c)
{
    return hipSetDevice(c->device) == hipSuccess;
}

}  // namespace lc

using namespace lc;

#define CHECK_CTX(x)                                                              \
    if (!(x)) return LC_EINVAL;                                                   \
    Ctx *c = C(x);                                                                \
    if (c->device < 0) return fail(c, LC_EUNSUP, "host-only context (device -1)"); \
    if (!set_device(c)) return fail(c, LC_EHIP, "hipSetDevice failed");

extern "C" {

int lc_ctx_create(const lc_params *prm, int device, int role, lc_ctx **out)
{
    if (!out) return LC_EINVAL;
    *out = nullptr;
    if (role != LC_ROLE_SERVER && role != LC_ROLE_KGC) return LC_EINVAL;
    if (device >= 0) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return LC_EHIP;
    } else if (device != -1) {
        return LC_EINVAL;
    }
    lc_ctx *x = new (std::nothrow) lc_ctx();
    if (!x) return LC_ENOMEM;
    x->c.device = device;
    x->c.role = role;
    if (device >= 0 && hipSetDevice(device) != hipSuccess) {
        delete x;
        return LC_EHIP;
    }
    int rc = build_params(&x->c, prm);
    if (!rc && device >= 0) rc = scratch_init(&x->c);  // with the device current
    if (rc) {
        lc_ctx_destroy(x);
        return rc;
    }
    *out = x;
    return LC_OK;
}

int lc_ctx_destroy(lc_ctx *x)
{
    if (!x) return LC_EINVAL;
    Ctx *c = &x->c;
    if (c->device >= 0) {
        hipSetDevice(c->device);
        hipDeviceSynchronize();
        for (void *p : c->allocs) hipFree(p);
        for (void *p : c->retired) hipFree(p);
        for (auto &kv : c->ws)
            for (int i = 0; i < 8; i++)
                if (kv.second.slot[i]) hipFree(kv.second.slot[i]);
        for (auto &kv : c->aux) {
            hipStreamDestroy(kv.second.stream);
            hipEventDestroy(kv.second.fork);
            hipEventDestroy(kv.second.join);
        }
    }
    delete x;
    return LC_OK;
}

const char *lc_last_error(const lc_ctx *x) { return x ? x->c.err.c_str() : "null context"; }

int lc_ctx_moduli(const lc_ctx *x, uint64_t *out)
{
    if (!x || !out) return LC_EINVAL;
    std::memcpy(out, x->c.mod.data(), x->c.mod.size() * 8);
    return LC_OK;
}

int lc_ctx_info(const lc_ctx *x, int *log_n, int *n_q, int *n_p, int *dnum)
{
    if (!x) return LC_EINVAL;
    if (log_n) *log_n = x->c.log_n;
    if (n_q) *n_q = x->c.nq;
    if (n_p) *n_p = x->c.np;
    if (dnum) *dnum = x->c.dnum;
    return LC_OK;
}

int lc_sync(lc_ctx *x, void *stream)
{
    CHECK_CTX(x);
    LC_HIP(c, hipStreamSynchronize((hipStream_t)stream));
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

int lc_release_workspace(lc_ctx *x)
{
    CHECK_CTX(x);
    if (c->device < 0) return LC_OK;
    LC_HIP(c, hipDeviceSynchronize());
    for (void *p : c->retired) hipFree(p);
    c->retired.clear();
    c->retired_bytes = 0;
    for (auto &kv : c->ws)
        for (int i = 0; i < 8; i++)
            if (kv.second.slot[i]) {
                hipFree(kv.second.slot[i]);
                kv.second.slot[i] = nullptr;
                kv.second.bytes[i] = 0;
            }
    c->ws.clear();
    return LC_OK;
}

int lc_ctx_device_bytes(const lc_ctx *x, size_t *bytes)
{
    if (!x || !bytes) return LC_EINVAL;
    size_t b = x->c.table_bytes + x->c.key_bytes + x->c.retired_bytes;
    for (auto &kv : x->c.ws)
        for (int i = 0; i < 8; i++) b += kv.second.bytes[i];
    *bytes = b;
    return LC_OK;
}

// ---- keys --------------------------------------------------------------------

int lc_keygen(lc_ctx *x, uint64_t seed)
{
    CHECK_CTX(x);
    if (c->role != LC_ROLE_KGC) return fail(c, LC_EKEY, "key generation needs a KGC-role context");
    const int ne = c->ne, nq = c->nq;
    const u64 N = c->N, NE = (u64)ne * N, S = (u64)nq * N;
    if (!c->sk_coeff) {
        c->sk_coeff = (i64 *)dev_alloc(c, N * 8);
        c->sk_ntt = (u64 *)dev_alloc(c, NE * 8);
        c->sk_ntt_sh = (u64 *)dev_alloc(c, NE * 8);
        c->sk2_ntt = (u64 *)dev_alloc(c, S * 8);
        c->sk2_ntt_sh = (u64 *)dev_alloc(c, S * 8);
        c->pk = (u64 *)dev_alloc(c, 2 * S * 8);
        c->pk_sh = (u64 *)dev_alloc(c, 2 * S * 8);
        c->rlk = (u64 *)dev_alloc(c, (u64)c->dnum * 2 * NE * 8);
        if (!c->sk_coeff || !c->sk_ntt || !c->sk_ntt_sh || !c->sk2_ntt || !c->sk2_ntt_sh || !c->pk || !c->pk_sh ||
            !c->rlk)
            return fail(c, LC_ENOMEM, "key allocation failed");
        c->key_bytes += (N + 2 * NE + 2 * S + 4 * S + (u64)c->dnum * 2 * NE) * 8;
    }
    int rc;
    // secret
    if ((rc = launch_sample_ternary(c, seed, 1, 0, c->sk_coeff, 0))) return rc;
    if ((rc = launch_signed_to_limbs(c, c->sk_coeff, c->sk_ntt, ne, 1, 0))) return rc;
    if ((rc = launch_ntt_fwd(c, PolyBatch{c->sk_ntt, 1, ne, (u64)ne, 0, 0}, 0))) return rc;
    if ((rc = launch_pointwise_sq(c, c->sk_ntt, c->sk2_ntt, nq, 0))) return rc;
    LC_HIP(c, hipDeviceSynchronize());
    if ((rc = upload_shoup(c, c->sk_ntt, c->sk_ntt_sh, ne, 1))) return rc;
    if ((rc = upload_shoup(c, c->sk2_ntt, c->sk2_ntt_sh, nq, 1))) return rc;
    // public key: a uniform (NTT domain), e Gaussian
    u64 *tmp = ws_get(c, WS_KEYGEN, (NE + N + ne) * 8, 0);
    if (!tmp) return LC_ENOMEM;
    u64 *e_ntt = tmp;
    i64 *e_coef = (i64 *)(tmp + NE);
    if ((rc = launch_uniform_limbs(c, seed, 2, 0, c->pk + S, nq, 0))) return rc;
    if ((rc = launch_gaussian(c, seed, 3, 0, e_coef, 0))) return rc;
    if ((rc = launch_signed_to_limbs(c, e_coef, e_ntt, nq, 1, 0))) return rc;
    if ((rc = launch_ntt_fwd(c, PolyBatch{e_ntt, 1, nq, (u64)nq, 0, 0}, 0))) return rc;
    if ((rc = launch_keycombine(c, c->pk + S, e_ntt, c->sk_ntt, nullptr, nullptr, c->pk, c->pk + S, nq, 0))) return rc;
    LC_HIP(c, hipDeviceSynchronize());
    if ((rc = upload_shoup(c, c->pk, c->pk_sh, nq, 2))) return rc;
    // relinearization key: target s^2 over all ne limbs
    u64 *t = ws_get(c, WS_TMP, NE * 8, 0);
    if (!t) return LC_ENOMEM;
    if ((rc = launch_pointwise_sq(c, c->sk_ntt, t, ne, 0))) return rc;
    if ((rc = gen_ksk(c, seed, 0, t, c->rlk))) return rc;
    // rotation keys made before a re-keygen are stale
    c->rot.clear();
    return LC_OK;
}

int lc_keygen_rotation(lc_ctx *x, uint64_t seed, const int *steps, int nsteps)
{
    CHECK_CTX(x);
    if (c->role != LC_ROLE_KGC) return fail(c, LC_EKEY, "key generation needs a KGC-role context");
    if (!c->sk_ntt) return fail(c, LC_EKEY, "call lc_keygen first");
    if (nsteps < 0 || (nsteps && !steps)) return fail(c, LC_EINVAL, "bad steps");
    const u64 NE = (u64)c->ne * c->N;
    u64 *t = ws_get(c, WS_TMP, NE * 8, 0);
    if (!t) return LC_ENOMEM;
    for (int i = 0; i < nsteps; i++) {
        u64 g = galois_of_step(c->log_n, steps[i]);
        if (g == 1 || c->rot.count(g)) continue;
        u32 *perm = get_perm(c, g);
        u64 *k = (u64 *)dev_alloc(c, (u64)c->dnum * 2 * NE * 8);
        if (!perm || !k) return fail(c, LC_ENOMEM, "rotation key allocation failed");
        c->key_bytes += (u64)c->dnum * 2 * NE * 8;
        int rc;
        if ((rc = launch_permute(c, c->sk_ntt, t, perm, c->ne, 0))) return rc;
        if ((rc = gen_ksk(c, seed, g, t, k))) return rc;
        c->rot[g] = RotKey{k, perm, g};
        if ((rc = build_cycle_table(c, g))) return rc;
    }
    return LC_OK;
}

int lc_keys_share(const lc_ctx *xs, lc_ctx *xd)
{
    if (!xs || !xd) return LC_EINVAL;
    const Ctx *s = &xs->c;
    Ctx *c = &xd->c;
    if (s->mod != c->mod || s->log_n != c->log_n || s->device != c->device)
        return fail(c, LC_EINVAL, "contexts differ in parameters or device");
    if (!s->pk) return fail(c, LC_EKEY, "source has no keys");
    if (!set_device(c)) return LC_EHIP;
    const u64 S = (u64)c->nq * c->N, NE = (u64)c->ne * c->N, K = (u64)c->dnum * 2 * NE;
    if (!c->pk) {
        c->pk = (u64 *)dev_alloc(c, 2 * S * 8);
        c->pk_sh = (u64 *)dev_alloc(c, 2 * S * 8);
        c->rlk = (u64 *)dev_alloc(c, K * 8);
        if (!c->pk || !c->pk_sh || !c->rlk) return fail(c, LC_ENOMEM, "key allocation failed");
        c->key_bytes += (4 * S + K) * 8;
    }
    LC_HIP(c, hipMemcpy(c->pk, s->pk, 2 * S * 8, hipMemcpyDeviceToDevice));
    LC_HIP(c, hipMemcpy(c->pk_sh, s->pk_sh, 2 * S * 8, hipMemcpyDeviceToDevice));
    LC_HIP(c, hipMemcpy(c->rlk, s->rlk, K * 8, hipMemcpyDeviceToDevice));
    for (auto &kv : s->rot) {
        if (c->rot.count(kv.first)) continue;
        u64 *k = (u64 *)dev_alloc(c, K * 8);
        u32 *perm = get_perm(c, kv.first);
        if (!k || !perm) return fail(c, LC_ENOMEM, "key allocation failed");
        c->key_bytes += K * 8;
        LC_HIP(c, hipMemcpy(k, kv.second.ksk, K * 8, hipMemcpyDeviceToDevice));
        c->rot[kv.first] = RotKey{k, perm, kv.first};
        int rc = build_cycle_table(c, kv.first);
        if (rc) return rc;
    }
    return LC_OK;
}

int lc_secret_export(const lc_ctx *x, int64_t *s_host)
{
    if (!x || !s_host) return LC_EINVAL;
    Ctx *c = const_cast<Ctx *>(&x->c);
    if (c->role != LC_ROLE_KGC || !c->sk_coeff) return fail(c, LC_EKEY, "no secret key in this context");
    if (!set_device(c)) return LC_EHIP;
    LC_HIP(c, hipMemcpy(s_host, c->sk_coeff, c->N * 8, hipMemcpyDeviceToHost));
    return LC_OK;
}

int lc_pk_export(const lc_ctx *x, uint64_t *pk_host)
{
    if (!x || !pk_host) return LC_EINVAL;
    Ctx *c = const_cast<Ctx *>(&x->c);
    if (!c->pk) return fail(c, LC_EKEY, "no public key");
    if (!set_device(c)) return LC_EHIP;
    LC_HIP(c, hipMemcpy(pk_host, c->pk, 2 * (u64)c->nq * c->N * 8, hipMemcpyDeviceToHost));
    return LC_OK;
}

int lc_ksk_export(const lc_ctx *x, int which, int step, uint64_t *out)
{
    if (!x || !out) return LC_EINVAL;
    Ctx *c = const_cast<Ctx *>(&x->c);
    if (!set_device(c)) return LC_EHIP;
    const u64 K = (u64)c->dnum * 2 * c->ne * c->N;
    const u64 *src = nullptr;
    if (which == 0) src = c->rlk;
    else if (which == 1) {
        auto it = c->rot.find(galois_of_step(c->log_n, step));
        if (it != c->rot.end()) src = it->second.ksk;
    } else return fail(c, LC_EINVAL, "which must be 0 or 1");
    if (!src) return fail(c, LC_EKEY, "key not present");
    LC_HIP(c, hipMemcpy(out, src, K * 8, hipMemcpyDeviceToHost));
    return LC_OK;
}

static bool canonical_limbs(const Ctx *c, const u64 *h, u64 count, int nlimb)
{
    for (u64 o = 0; o < count; o++)
        for (int l = 0; l < nlimb; l++) {
            const u64 m = c->mod[l], *p = h + (o * nlimb + l) * c->N;
            for (u64 j = 0; j < c->N; j++)
                if (p[j] >= m) return false;
        }
    return true;
}

int lc_key_import(lc_ctx *x, int kind, int step, const uint64_t *blob)
{
    CHECK_CTX(x);
    if (!blob) return fail(c, LC_EINVAL, "null key");
    const u64 S = (u64)c->nq * c->N, NE = (u64)c->ne * c->N, K = (u64)c->dnum * 2 * NE;
    if (kind == LC_KEY_PK) {
        if (!canonical_limbs(c, blob, 2, c->nq)) return fail(c, LC_EINVAL, "key residues must be canonical");
        if (!c->pk) {
            c->pk = (u64 *)dev_alloc(c, 2 * S * 8);
            c->pk_sh = (u64 *)dev_alloc(c, 2 * S * 8);
            if (!c->pk || !c->pk_sh) return fail(c, LC_ENOMEM, "key allocation failed");
            c->key_bytes += 4 * S * 8;
        }
        LC_HIP(c, hipDeviceSynchronize());
        LC_HIP(c, hipMemcpy(c->pk, blob, 2 * S * 8, hipMemcpyHostToDevice));
        return upload_shoup(c, c->pk, c->pk_sh, c->nq, 2);
    }
    if (kind != LC_KEY_RELIN && kind != LC_KEY_ROTATION) return fail(c, LC_EINVAL, "unknown key kind");
    if (!canonical_limbs(c, blob, (u64)c->dnum * 2, c->ne)) return fail(c, LC_EINVAL, "key residues must be canonical");
    u64 *dst;
    if (kind == LC_KEY_RELIN) {
        if (!c->rlk) {
            c->rlk = (u64 *)dev_alloc(c, K * 8);
            if (!c->rlk) return fail(c, LC_ENOMEM, "key allocation failed");
            c->key_bytes += K * 8;
        }
        dst = c->rlk;
    } else {
        const u64 g = galois_of_step(c->log_n, step);
        if (g == 1) return fail(c, LC_EINVAL, "step is a multiple of N/2: no rotation");
        auto it = c->rot.find(g);
        if (it == c->rot.end()) {
            u32 *perm = get_perm(c, g);
            u64 *k = (u64 *)dev_alloc(c, K * 8);
            if (!perm || !k) return fail(c, LC_ENOMEM, "rotation key allocation failed");
            c->key_bytes += K * 8;
            c->rot[g] = RotKey{k, perm, g};
            int rc = build_cycle_table(c, g);
            if (rc) return rc;
            it = c->rot.find(g);
        }
        dst = it->second.ksk;
    }
    // work queued on any stream may still read the key being replaced
    LC_HIP(c, hipDeviceSynchronize());
    LC_HIP(c, hipMemcpy(dst, blob, K * 8, hipMemcpyHostToDevice));
    return LC_OK;
}

// ---- encode / decode ------------------------------------------------------------

int lc_encode(const lc_ctx *x, const double *re, const double *im, size_t nslots, double scale, int64_t *m)
{
    if (!x || !re || !m) return LC_EINVAL;
    if (nslots > x->c.N / 2) return LC_EINVAL;
    encode_host(x->c.log_n, re, im, nslots, scale, m);
    return LC_OK;
}

int lc_encode_device(lc_ctx *x, const double *z_dev, size_t count, size_t nslots, size_t z_stride, double scale,
                     int64_t *m_dev, void *stream)
{
    CHECK_CTX(x);
    if (nslots > c->N / 2 || z_stride < nslots) return fail(c, LC_EINVAL, "need nslots <= N/2 and z_stride >= nslots");
    if (count && ((!z_dev && nslots) || !m_dev)) return fail(c, LC_EINVAL, "null buffer");
    if (!(scale > 0.0)) return fail(c, LC_EINVAL, "scale must be positive");
    return launch_encode(c, z_dev, count, nslots, z_stride, scale, m_dev, (hipStream_t)stream);
}

int lc_decode_level(const lc_ctx *x, const uint64_t *res, int nlimb, double scale, double *re, double *im)
{
    if (!x || !res || !re) return LC_EINVAL;
    const Ctx *c = &x->c;
    if (nlimb < 1 || nlimb > c->nq) return LC_EINVAL;
    std::vector<u64> q(c->mod.begin(), c->mod.begin() + nlimb);
    std::vector<double> coeff(c->N);
    crt_to_double(q, res, c->N, c->N, coeff.data());
    decode_host(c->log_n, coeff.data(), scale, re, im);
    return LC_OK;
}

int lc_decode(const lc_ctx *x, const uint64_t *res, double scale, double *re, double *im)
{
    if (!x || !res || !re) return LC_EINVAL;
    const Ctx *c = &x->c;
    std::vector<u64> q(c->mod.begin(), c->mod.begin() + c->nq);
    std::vector<double> coeff(c->N);
    crt_to_double(q, res, c->N, c->N, coeff.data());
    decode_host(c->log_n, coeff.data(), scale, re, im);
    return LC_OK;
}

int lc_crt_to_double(const lc_ctx *x, const uint64_t *res, size_t ncoeff, size_t stride, double *out)
{
    if (!x || !res || !out || ncoeff > stride) return LC_EINVAL;
    const Ctx *c = &x->c;
    std::vector<u64> q(c->mod.begin(), c->mod.begin() + c->nq);
    crt_to_double(q, res, ncoeff, stride, out);
    return LC_OK;
}

// ---- encryption / decryption -----------------------------------------------------

int lc_encrypt(lc_ctx *x, const int64_t *m, size_t count, uint64_t seed, uint64_t first_object, uint64_t *ct,
               void *stream)
{
    CHECK_CTX(x);
    if (!c->pk) return fail(c, LC_EKEY, "no public key");
    if ((!m || !ct) && count) return fail(c, LC_EINVAL, "null buffer");
    hipStream_t s = (hipStream_t)stream;
    const u64 S = (u64)c->nq * c->N;
    u64 chunk = std::min<u64>(count, std::max<u64>(1, (1ull << 31) / (3 * S * 8)));
    u64 *tmp = ws_get(c, WS_ENC, chunk * 3 * S * 8, s);
    if (!tmp) return LC_ENOMEM;
    for (u64 t0 = 0; t0 < count; t0 += chunk) {
        u64 B = std::min<u64>(chunk, count - t0);
        int rc;
        if ((rc = launch_enc_sample(c, m + t0 * c->N, B, seed, first_object + t0, tmp, s))) return rc;
        if ((rc = launch_ntt_fwd(c, PolyBatch{tmp, B * 3, c->nq, (u64)c->nq, 0, 0}, s))) return rc;
        if ((rc = launch_enc_combine(c, tmp, B, ct + t0 * 2 * S, s))) return rc;
    }
    return LC_OK;
}

int lc_decrypt_level(lc_ctx *x, const uint64_t *ct, int ncomp, int nlimb, size_t count, uint64_t *pt, void *stream)
{
    CHECK_CTX(x);
    if (c->role != LC_ROLE_KGC || !c->sk_ntt) return fail(c, LC_EKEY, "decryption needs the secret key (KGC role)");
    if (ncomp != 2 && ncomp != 3) return fail(c, LC_EINVAL, "ncomp must be 2 or 3");
    if (nlimb < 1 || nlimb > c->nq) return fail(c, LC_EINVAL, "need 1 <= nlimb <= n_q");
    if (!count) return LC_OK;
    if (!ct || !pt) return fail(c, LC_EINVAL, "null buffer");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = launch_dec_combine(c, ct, ncomp, nlimb, count, pt, s))) return rc;
    return launch_ntt_inv(c, PolyBatch{pt, count, nlimb, (u64)nlimb, 0, 0}, s);
}

int lc_decrypt(lc_ctx *x, const uint64_t *ct, int ncomp, size_t count, uint64_t *pt, void *stream)
{
    return lc_decrypt_level(x, ct, ncomp, x ? x->c.nq : 0, count, pt, stream);
}

int lc_rescale(lc_ctx *x, const uint64_t *ct, size_t count, int ncomp, int nlimb, uint64_t *out, void *stream)
{
    CHECK_CTX(x);
    if (ncomp < 1 || ncomp > 3) return fail(c, LC_EINVAL, "ncomp must be 1..3");
    if (nlimb < 2 || nlimb > c->nq) return fail(c, LC_EINVAL, "need 2 <= nlimb <= n_q");
    if (!count) return LC_OK;
    if (!ct || !out) return fail(c, LC_EINVAL, "null buffer");
    const u64 in_bytes = (u64)count * ncomp * nlimb * c->N * 8, out_bytes = (u64)count * ncomp * (nlimb - 1) * c->N * 8;
    if (overlap(ct, in_bytes, out, out_bytes)) return fail(c, LC_EINVAL, "out must not overlap the input");
    return launch_rescale(c, ct, count, ncomp, nlimb, out, (hipStream_t)stream);
}

// ---- homomorphic operations -------------------------------------------------------

int lc_ct_sub(lc_ctx *x, const uint64_t *a, const uint64_t *b, uint64_t *out, size_t count, int ncomp, void *stream)
{
    CHECK_CTX(x);
    if (ncomp < 1 || ncomp > 3) return fail(c, LC_EINVAL, "ncomp must be 1..3");
    if (count && (!a || !b || !out)) return fail(c, LC_EINVAL, "null buffer");
    const size_t bytes = count * ncomp * c->nq * c->N * 8;
    if (partial_overlap(a, bytes, out, bytes) || partial_overlap(b, bytes, out, bytes))
        return fail(c, LC_EINVAL, "out must equal an input or not overlap it");
    return launch_add_sub(c, a, b, out, count, ncomp, 1, (hipStream_t)stream);
}

int lc_ct_add(lc_ctx *x, const uint64_t *a, const uint64_t *b, uint64_t *out, size_t count, int ncomp, void *stream)
{
    CHECK_CTX(x);
    if (ncomp < 1 || ncomp > 3) return fail(c, LC_EINVAL, "ncomp must be 1..3");
    if (count && (!a || !b || !out)) return fail(c, LC_EINVAL, "null buffer");
    const size_t bytes = count * ncomp * c->nq * c->N * 8;
    if (partial_overlap(a, bytes, out, bytes) || partial_overlap(b, bytes, out, bytes))
        return fail(c, LC_EINVAL, "out must equal an input or not overlap it");
    return launch_add_sub(c, a, b, out, count, ncomp, 0, (hipStream_t)stream);
}

int lc_ct_mul(lc_ctx *x, const uint64_t *a, const uint64_t *b, uint64_t *out3, size_t count, void *stream)
{
    CHECK_CTX(x);
    if (count && (!a || !b || !out3)) return fail(c, LC_EINVAL, "null buffer");
    const size_t S8 = (size_t)c->nq * c->N * 8;
    if (count && (overlap(a, count * 2 * S8, out3, count * 3 * S8) || overlap(b, count * 2 * S8, out3, count * 3 * S8)))
        return fail(c, LC_EINVAL, "out3 must not overlap the inputs");
    return launch_tensor(c, a, b, out3, count, (hipStream_t)stream);
}

int lc_ct_square(lc_ctx *x, const uint64_t *a, uint64_t *out3, size_t count, void *stream)
{
    CHECK_CTX(x);
    if (count && (!a || !out3)) return fail(c, LC_EINVAL, "null buffer");
    const size_t S8 = (size_t)c->nq * c->N * 8;
    if (count && overlap(a, count * 2 * S8, out3, count * 3 * S8))
        return fail(c, LC_EINVAL, "out3 must not overlap the input");
    return launch_tensor(c, a, nullptr, out3, count, (hipStream_t)stream);
}


int lc_relin(lc_ctx *x, const uint64_t *ct3, uint64_t *ct2, size_t count, void *stream)
{
    CHECK_CTX(x);
    if (!c->rlk) return fail(c, LC_EKEY, "no relinearization key");
    if (!count) return LC_OK;
    if (!ct3 || !ct2) return fail(c, LC_EINVAL, "null buffer");
    const u64 S = (u64)c->nq * c->N;
    if (overlap(ct3, count * 3 * S * 8, ct2, count * 2 * S * 8))
        return fail(c, LC_EINVAL, "lc_relin output must not overlap its input");
    KsGroup g{};
    g.keys[0] = c->rlk;
    g.n = 1;
    g.base = ct3;
    g.base_stride = 3 * S;
    g.out = ct2;
    g.out_stride = 2 * S;
    return keyswitch_hoisted(c, ct3 + 2 * S, 3 * S, count, &g, 1, (hipStream_t)stream);
}

int lc_relin_noalloc(lc_ctx *x, const uint64_t *ct3, uint64_t *ct2, size_t count, void *stream)
{
    CHECK_CTX(x);
    if (!c->rlk) return fail(c, LC_EKEY, "no relinearization key");
    const u64 per_ct = ks_words_per_ct(c);
    if (per_ct * sizeof(u64) > NOALLOC_SCRATCH_BYTES)
        return fail(c, LC_EINVAL, "one ciphertext's key-switch scratch (" + std::to_string(per_ct * sizeof(u64)) +
                                      " bytes) exceeds the fixed " + std::to_string(NOALLOC_SCRATCH_BYTES) +
                                      "-byte array of lc_relin_noalloc");
    if (!count) return LC_OK;
    if (!ct3 || !ct2) return fail(c, LC_EINVAL, "null buffer");
    const u64 S = (u64)c->nq * c->N;
    if (overlap(ct3, count * 3 * S * 8, ct2, count * 2 * S * 8))
        return fail(c, LC_EINVAL, "lc_relin_noalloc output must not overlap its input");
    u64 *ws = scratch_of(c->device);
    if (!ws) return fail(c, LC_EHIP, "no scratch address for this device");
    KsGroup g{};
    g.keys[0] = c->rlk;
    g.n = 1;
    g.base = ct3;
    g.base_stride = 3 * S;
    g.out = ct2;
    g.out_stride = 2 * S;
    return keyswitch_hoisted_ws(c, ct3 + 2 * S, 3 * S, count, &g, 1, ws, NOALLOC_SCRATCH_BYTES / sizeof(u64),
                                (hipStream_t)stream);
}

int lc_rotate_hoisted(lc_ctx *x, const uint64_t *ct, size_t count, const int *steps, int nsteps, uint64_t *outs,
                      void *stream)
{
    CHECK_CTX(x);
    if (nsteps < 1 || nsteps > 64 || !steps) return fail(c, LC_EINVAL, "1..64 steps");
    if (!count) return LC_OK;
    if (!ct || !outs) return fail(c, LC_EINVAL, "null buffer");
    const u64 S = (u64)c->nq * c->N;
    if (overlap(ct, count * 2 * S * 8, outs, count * nsteps * 2 * S * 8))
        return fail(c, LC_EINVAL, "output must not overlap the input");
    // the source-major inner product when every key's automorphism acts on
    // tiles and the key switch takes the fused transforms
    bool multi = c->tune.hoist_multi && c->tune.mac_cycle_c0 && c->tune.fuse_modup && c->log_n >= 10 &&
                 c->log_n <= 17 && c->np <= MAX_NP && c->dnum <= 8;
    std::vector<const u64 *> mkeys(nsteps);
    std::vector<const u32 *> mperms(nsteps), minv(nsteps);
    for (int t = 0; t < nsteps && multi; t++) {
        auto it = c->rot.find(galois_of_step(c->log_n, steps[t]));
        if (it == c->rot.end()) break;  // reported below
        auto cy = c->cycles.find(it->first);
        if (!it->second.perm || cy == c->cycles.end() || !cy->second.inv_tile) {
            multi = false;
            break;
        }
        mkeys[t] = it->second.ksk;
        mperms[t] = it->second.perm;
        minv[t] = cy->second.inv_tile;
    }
    std::vector<KsGroup> groups(nsteps);
    for (int t = 0; t < nsteps; t++) {
        u64 g = galois_of_step(c->log_n, steps[t]);
        auto it = c->rot.find(g);
        if (it == c->rot.end()) return fail(c, LC_EKEY, "no rotation key for step " + std::to_string(steps[t]));
        KsGroup &G = groups[t];
        G = KsGroup{};
        G.keys[0] = it->second.ksk;
        G.perms[0] = it->second.perm;
        G.n = 1;
        G.c0src = ct;
        G.c0_stride = 2 * S;
        G.out = outs + (u64)t * 2 * S;
        G.out_stride = (u64)nsteps * 2 * S;
    }
    if (multi)
        return keyswitch_rotations(c, ct, count, mkeys.data(), mperms.data(), minv.data(), nsteps, outs,
                                   (u64)nsteps * 2 * S, (hipStream_t)stream);
    return keyswitch_hoisted(c, ct + S, 2 * S, count, groups.data(), nsteps, (hipStream_t)stream);
}

// The key groups of a rotate-and-sum plan (Methods, Dynamic Hoisting): block
// b starting at level j0 holds the keys of rot_{t 2^j0}, t = 1 .. 2^plan[b] - 1.
// With blocks null the plan is only checked.
static int rotsum_blocks(Ctx *c, const int *plan, int nblocks, std::vector<KsGroup> *blocks)
{
    std::vector<int> pl;
    if (!plan) pl.assign(c->log_n - 1, 1);
    else pl.assign(plan, plan + nblocks);
    int total = 0;
    for (int k : pl) {
        if (k < 1 || k > 3) return fail(c, LC_EINVAL, "plan blocks must have 1..3 levels");
        total += k;
    }
    if (total != c->log_n - 1) return fail(c, LC_EINVAL, "plan levels must sum to log_n - 1");
    if (!blocks) return LC_OK;
    blocks->clear();
    int j0 = 0;
    for (int k : pl) {
        KsGroup G{};
        G.n = (1 << k) - 1;
        for (int t = 1; t <= G.n; t++) {
            u64 g = galois_of_step(c->log_n, (long long)t << j0);
            auto it = c->rot.find(g);
            if (it == c->rot.end())
                return fail(c, LC_EKEY, "no rotation key for step " + std::to_string((long long)t << j0));
            G.keys[t - 1] = it->second.ksk;
            G.perms[t - 1] = it->second.perm;
        }
        // keys t 2^j0 = powers of the step-2^j0 automorphism: the cycle walk applies
        auto cy = c->cycles.find(galois_of_step(c->log_n, 1ll << j0));
        if (G.n > 1 && cy != c->cycles.end() && cy->second.nseg > 0) G.cyc = &cy->second;
        blocks->push_back(G);
        j0 += k;
    }
    return LC_OK;
}

// Rotate-and-sum of B ciphertexts.  Each block reads one of `io` and `tmp`
// (B ciphertexts each) and writes the other; the first block reads `tmp`
// when from_tmp is set, else `io`.  The result is left in `io`, with one copy
// when the blocks end in `tmp` (from_tmp and an even number of blocks, or an
// odd number without it).
static int rotsum_run(Ctx *c, const std::vector<KsGroup> &blocks, u64 *io, u64 *tmp, bool from_tmp, u64 B,
                      hipStream_t s)
{
    const u64 S = (u64)c->nq * c->N;
    u64 *y = from_tmp ? tmp : io, *z = from_tmp ? io : tmp;
    for (KsGroup G : blocks) {
        G.base = y;
        G.base_stride = 2 * S;
        G.c0src = y;
        G.c0_stride = 2 * S;
        G.out = z;
        G.out_stride = 2 * S;
        int rc = keyswitch_hoisted(c, y + S, 2 * S, B, &G, 1, s);
        if (rc) return rc;
        std::swap(y, z);
    }
    if (y != io) return launch_copy(c, y, io, B * 2 * S, s);
    return LC_OK;
}

int lc_rotate_sum(lc_ctx *x, uint64_t *ct, size_t count, const int *plan, int nblocks, void *stream)
{
    CHECK_CTX(x);
    std::vector<KsGroup> blocks;
    int rc = rotsum_blocks(c, plan, nblocks, nullptr);
    if (rc || !count) return rc;
    if (!ct) return fail(c, LC_EINVAL, "null buffer");
    if ((rc = rotsum_blocks(c, plan, nblocks, &blocks))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const u64 S = (u64)c->nq * c->N;
    u64 chunk = std::min<u64>(count, (u64)c->tune.ks_chunk);
    u64 *other = ws_get(c, WS_ROT, chunk * 2 * S * 8, s);
    if (!other) return LC_ENOMEM;
    for (u64 b0 = 0; b0 < count; b0 += chunk) {
        u64 B = std::min<u64>(chunk, count - b0);
        if ((rc = rotsum_run(c, blocks, ct + b0 * 2 * S, other, false, B, s))) return rc;
    }
    return LC_OK;
}

int lc_mul_plain(lc_ctx *x, const uint64_t *ct, const uint64_t *pt, uint64_t *out, size_t count, void *stream)
{
    CHECK_CTX(x);
    if (count && (!ct || !pt || !out)) return fail(c, LC_EINVAL, "null buffer");
    const size_t S8 = (size_t)c->nq * c->N * 8;
    if (count && (partial_overlap(ct, count * 2 * S8, out, count * 2 * S8) || overlap(pt, count * S8, out, count * 2 * S8)))
        return fail(c, LC_EINVAL, "out must equal ct or not overlap it, and must not overlap pt");
    return launch_mul_plain(c, ct, pt, out, count, (hipStream_t)stream);
}

int lc_masked_sum(lc_ctx *x, const uint64_t *cts, int n, int len, const uint64_t *masks, uint64_t *out, void *stream)
{
    CHECK_CTX(x);
    if (n < 1 || n > 4096 || len < 1) return fail(c, LC_EINVAL, "need 1 <= n <= 4096 and len >= 1");
    if (!cts || !masks || !out) return fail(c, LC_EINVAL, "null buffer");
    const u64 S = (u64)c->nq * c->N;
    if (overlap(cts, (u64)n * len * 2 * S * 8, out, (u64)len * 2 * S * 8) ||
        overlap(masks, (u64)n * S * 8, out, (u64)len * 2 * S * 8))
        return fail(c, LC_EINVAL, "out must not overlap the inputs");
    return launch_masked_sum(c, cts, n, len, masks, out, (hipStream_t)stream);
}

int lc_mask_aggregate(lc_ctx *x, const uint64_t *cts, int n, int len, const uint64_t *mask_cts, uint64_t *out,
                      void *stream)
{
    CHECK_CTX(x);
    if (n < 1 || n > 4096 || len < 1) return fail(c, LC_EINVAL, "need 1 <= n <= 4096 and len >= 1");
    if (!cts || !mask_cts || !out) return fail(c, LC_EINVAL, "null buffer");
    if (!c->rlk) return fail(c, LC_EKEY, "no relinearization key");
    const u64 S = (u64)c->nq * c->N;
    if (overlap(cts, (u64)n * len * 2 * S * 8, out, (u64)len * 2 * S * 8) ||
        overlap(mask_cts, (u64)n * 2 * S * 8, out, (u64)len * 2 * S * 8))
        return fail(c, LC_EINVAL, "out must not overlap the inputs");
    hipStream_t s = (hipStream_t)stream;
    // triples of a chunk of packed ciphertexts, then one relinearization each
    const int chunk = std::min(len, std::max(1, c->tune.ks_chunk));
    u64 *trip = ws_get(c, WS_PIPE, (u64)chunk * 3 * S * 8, s);
    if (!trip) return LC_ENOMEM;
    for (int k0 = 0; k0 < len; k0 += chunk) {
        const int kc = std::min(chunk, len - k0);
        int rc = launch_mask_mul_acc(c, cts + (u64)k0 * 2 * S, n, kc, len, mask_cts, trip, s);
        if (rc) return rc;
        KsGroup g{};
        g.keys[0] = c->rlk;
        g.n = 1;
        g.base = trip;
        g.base_stride = 3 * S;
        g.out = out + (u64)k0 * 2 * S;
        g.out_stride = 2 * S;
        if ((rc = keyswitch_hoisted(c, trip + 2 * S, 3 * S, kc, &g, 1, s))) return rc;
    }
    return LC_OK;
}

int lc_pair_triples(lc_ctx *x, const uint64_t *cts, int n, int len, uint64_t *triples, void *stream)
{
    CHECK_CTX(x);
    if (!cts || !triples) return fail(c, LC_EINVAL, "null buffer");
    const u64 S = (u64)c->nq * c->N;
    if (n >= 2 && len >= 1 && overlap(cts, (u64)n * len * 2 * S * 8, triples, (u64)n * (n - 1) / 2 * 3 * S * 8))
        return fail(c, LC_EINVAL, "triples must not overlap the client ciphertexts");
    return launch_pair_triples(c, cts, n, len, triples, 3 * S, triples + 2 * S, 3 * S, 0, (hipStream_t)stream);
}

int lc_pair_triples_acc(lc_ctx *x, const uint64_t *cts, int n, int len, uint64_t *triples, void *stream)
{
    CHECK_CTX(x);
    if (!cts || !triples) return fail(c, LC_EINVAL, "null buffer");
    const u64 S = (u64)c->nq * c->N;
    if (n >= 2 && len >= 1 && overlap(cts, (u64)n * len * 2 * S * 8, triples, (u64)n * (n - 1) / 2 * 3 * S * 8))
        return fail(c, LC_EINVAL, "triples must not overlap the client ciphertexts");
    return launch_pair_triples(c, cts, n, len, triples, 3 * S, triples + 2 * S, 3 * S, 1, (hipStream_t)stream);
}

// relinearize the triples whose (d0, d1) sit at `d01` (stride 2S, becoming
// the distances in place) and whose d2 sit at `d2` (stride d2_stride), then
// rotate-and-sum and SumDis.
// The second stream of caller stream s (made on first use: not inside a
// HIP graph capture).
static Ctx::Aux *aux_for(Ctx *c, hipStream_t s)
{
    auto it = c->aux.find(s);
    if (it != c->aux.end()) return &it->second;
    Ctx::Aux a;
    if (hipStreamCreateWithFlags(&a.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&a.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&a.join, hipEventDisableTiming) != hipSuccess) {
        hipGetLastError();
        if (a.stream) hipStreamDestroy(a.stream);
        if (a.fork) hipEventDestroy(a.fork);
        c->err = "could not create the pipeline's second stream";
        return nullptr;
    }
    return &(c->aux[s] = a);
}

// Relinearization and rotate-and-sum of the P triples, a key-switch batch of
// ks_chunk pairs at a time.  Batches touch disjoint pairs and their own
// stream's workspace, so with ks_streams = 2 they alternate between the
// caller's stream and a second one and overlap on the device (the kernels of
// one batch are half VALU-bound, half waiting on memory); the second stream
// forks from the caller's after the triples and joins it before SumDis.
static int pairwise_finish(lc_ctx *x, Ctx *c, const u64 *d01_base, u64 d01_stride, const u64 *d2, u64 d2_stride,
                           int n, const int *plan, int nblocks, uint64_t *dist, uint64_t *sumdis, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const u64 S = (u64)c->nq * c->N;
    const u64 P = (u64)n * (n - 1) / 2;
    const u64 chunk = std::max<u64>(1, std::min<u64>(P, (u64)c->tune.ks_chunk));
    std::vector<KsGroup> blocks;
    int rc = rotsum_blocks(c, plan, nblocks, &blocks);
    if (rc) return rc;
    // With an odd number of blocks the relinearization writes the rotate
    // buffer, so that the blocks' ping-pong ends in dist without a copy.
    const bool from_tmp = blocks.size() % 2 == 1;
    KsGroup g{};
    g.keys[0] = c->rlk;
    g.n = 1;
    g.base_stride = d01_stride;
    g.out_stride = 2 * S;
    Ctx::Aux *ax = nullptr;
    if (c->tune.ks_streams > 1 && P > chunk) {
        if (!(ax = aux_for(c, s))) return LC_EHIP;
        LC_HIP(c, hipEventRecord(ax->fork, s));
        LC_HIP(c, hipStreamWaitEvent(ax->stream, ax->fork, 0));
    }
    u64 k = 0;
    for (u64 p0 = 0; p0 < P; p0 += chunk, k++) {
        const u64 B = std::min(chunk, P - p0);
        hipStream_t st = (ax && (k & 1)) ? ax->stream : s;
        u64 *tmp = ws_get(c, WS_ROT, chunk * 2 * S * 8, st);  // the stream's own rotate buffer
        if (!tmp) return LC_ENOMEM;
        u64 *io = dist + p0 * 2 * S;
        g.base = d01_base + p0 * d01_stride;
        g.out = from_tmp ? tmp : io;
        if ((rc = keyswitch_hoisted(c, d2 + p0 * d2_stride, d2_stride, B, &g, 1, st))) return rc;
        if ((rc = rotsum_run(c, blocks, io, tmp, from_tmp, B, st))) return rc;
    }
    if (ax) {
        LC_HIP(c, hipEventRecord(ax->join, ax->stream));
        LC_HIP(c, hipStreamWaitEvent(s, ax->join, 0));
    }
    if (sumdis) return launch_sumdis(c, dist, 2 * S, n, 2, sumdis, s);
    return LC_OK;
}

int lc_pairwise_finish(lc_ctx *x, const uint64_t *triples, int n, const int *plan, int nblocks, uint64_t *dist,
                       uint64_t *sumdis, void *stream)
{
    CHECK_CTX(x);
    if (!triples || !dist) return fail(c, LC_EINVAL, "null buffer");
    if (!c->rlk) return fail(c, LC_EKEY, "no relinearization key");
    if (n < 2 || n > 64) return fail(c, LC_EINVAL, "pairwise kernels take 2..64 clients");
    const u64 S = (u64)c->nq * c->N;
    const u64 P = (u64)n * (n - 1) / 2;
    if (overlap(triples, P * 3 * S * 8, dist, P * 2 * S * 8))
        return fail(c, LC_EINVAL, "dist must not overlap the triples");
    return pairwise_finish(x, c, triples, 3 * S, triples + 2 * S, 3 * S, n, plan, nblocks, dist, sumdis, stream);
}

int lc_pairwise_sqdist(lc_ctx *x, const uint64_t *cts, int n, int len, const int *plan, int nblocks, uint64_t *dist,
                       uint64_t *sumdis, void *stream)
{
    CHECK_CTX(x);
    if (!cts || !dist) return fail(c, LC_EINVAL, "null buffer");
    if (!c->rlk) return fail(c, LC_EKEY, "no relinearization key");
    if (n < 2 || n > 64) return fail(c, LC_EINVAL, "pairwise kernels take 2..64 clients");
    hipStream_t s = (hipStream_t)stream;
    const u64 S = (u64)c->nq * c->N;
    const u64 P = (u64)n * (n - 1) / 2;
    u64 *d2 = ws_get(c, WS_PIPE, P * S * 8, s);
    if (!d2) return LC_ENOMEM;
    int rc;
    if ((rc = launch_pair_triples(c, cts, n, len, dist, 2 * S, d2, S, 0, s))) return rc;
    return pairwise_finish(x, c, dist, 2 * S, d2, S, n, plan, nblocks, dist, sumdis, stream);
}

int lc_sumdis_lazy(lc_ctx *x, const uint64_t *cts, int n, int len, const int *plan, int nblocks, uint64_t *sumdis,
                   void *stream)
{
    CHECK_CTX(x);
    if (!cts || !sumdis) return fail(c, LC_EINVAL, "null buffer");
    if (!c->rlk) return fail(c, LC_EKEY, "no relinearization key");
    if (n < 2 || n > 64) return fail(c, LC_EINVAL, "pairwise kernels take 2..64 clients");
    if (len < 1) return fail(c, LC_EINVAL, "need len >= 1");
    hipStream_t s = (hipStream_t)stream;
    const u64 S = (u64)c->nq * c->N;
    const u64 P = (u64)n * (n - 1) / 2;
    if (overlap(cts, (u64)n * len * 2 * S * 8, sumdis, (u64)n * 2 * S * 8))
        return fail(c, LC_EINVAL, "sumdis must not overlap the client ciphertexts");
    // pair triples, then each client's sum of its n - 1 triples
    u64 *trip = ws_get(c, WS_PIPE, (P + (u64)n) * 3 * S * 8, s);
    if (!trip) return LC_ENOMEM;
    u64 *sums = trip + P * 3 * S;
    int rc;
    if ((rc = launch_pair_triples(c, cts, n, len, trip, 3 * S, trip + 2 * S, 3 * S, 0, s))) return rc;
    if ((rc = launch_sumdis(c, trip, 3 * S, n, 3, sums, s))) return rc;
    KsGroup g{};
    g.keys[0] = c->rlk;
    g.n = 1;
    g.base = sums;
    g.base_stride = 3 * S;
    g.out = sumdis;
    g.out_stride = 2 * S;
    if ((rc = keyswitch_hoisted(c, sums + 2 * S, 3 * S, (u64)n, &g, 1, s))) return rc;
    return lc_rotate_sum(x, sumdis, (size_t)n, plan, nblocks, stream);
}

static int ntt_groups(lc_ctx *x, const lc_poly_group *groups, int ngroups, void *stream, bool inverse)
{
    CHECK_CTX(x);
    if (ngroups < 1 || ngroups > MAX_MIXED || !groups) return fail(c, LC_EINVAL, "1..16 polynomial groups");
    MixedArgs ma{};
    for (int d = MIXED_LOG_MIN; d <= MIXED_LOG_MAX && d <= c->log_n; d++) {
        DegreeTables t;
        bool used = false;
        for (int g = 0; g < ngroups; g++) used |= groups[g].log_n == d && groups[g].count > 0;
        if (!used) continue;
        int rc = degree_tables(c, d, &t);
        if (rc) return rc;
        ma.tw[d - MIXED_LOG_MIN] = inverse ? t.itwd : t.twd;
        ma.ninv[d - MIXED_LOG_MIN] = t.ninv;
    }
    for (int g = 0; g < ngroups; g++) {
        const lc_poly_group &G = groups[g];
        if (G.log_n < MIXED_LOG_MIN || G.log_n > std::min(MIXED_LOG_MAX, c->log_n))
            return fail(c, LC_EUNSUP, "group ring degrees must lie in 2^12 .. min(2^17, N)");
        if (G.nlimb < 1 || G.limb0 < 0 || G.limb0 + G.nlimb > c->ne) return fail(c, LC_EINVAL, "limb range outside the basis");
        if (G.count && !G.data) return fail(c, LC_EINVAL, "null buffer");
        if (!G.count) continue;
        MixedGroup &M = ma.g[ma.ng++];
        M.base = G.data;
        M.npoly = (u64)G.count * G.nlimb;
        M.nlimb = G.nlimb;
        M.limb0 = G.limb0;
        M.log_n = G.log_n;
    }
    if (!ma.ng) return LC_OK;
    return launch_ntt_mixed(c, ma, inverse, (hipStream_t)stream);
}

int lc_ntt_fwd_groups(lc_ctx *x, const lc_poly_group *groups, int ngroups, void *stream)
{
    return ntt_groups(x, groups, ngroups, stream, false);
}

int lc_ntt_inv_groups(lc_ctx *x, const lc_poly_group *groups, int ngroups, void *stream)
{
    return ntt_groups(x, groups, ngroups, stream, true);
}

int lc_ntt_fwd(lc_ctx *x, uint64_t *polys, size_t count, int nlimb, int limb0, void *stream)
{
    CHECK_CTX(x);
    if (nlimb < 1 || limb0 < 0 || limb0 + nlimb > c->ne) return fail(c, LC_EINVAL, "limb range outside the basis");
    if (count && !polys) return fail(c, LC_EINVAL, "null buffer");
    return launch_ntt_fwd(c, PolyBatch{polys, count, nlimb, (u64)nlimb, limb0, 0}, (hipStream_t)stream);
}

int lc_ntt_inv(lc_ctx *x, uint64_t *polys, size_t count, int nlimb, int limb0, void *stream)
{
    CHECK_CTX(x);
    if (nlimb < 1 || limb0 < 0 || limb0 + nlimb > c->ne) return fail(c, LC_EINVAL, "limb range outside the basis");
    if (count && !polys) return fail(c, LC_EINVAL, "null buffer");
    return launch_ntt_inv(c, PolyBatch{polys, count, nlimb, (u64)nlimb, limb0, 0}, (hipStream_t)stream);
}

int lc_gaussian_table(const lc_ctx *x, uint64_t *out38)
{
    if (!x || !out38) return LC_EINVAL;
    std::memcpy(out38, x->c.cdt_host.data(), 38 * 8);
    return LC_OK;
}

int lc_workspace_query(const lc_ctx *x, int n, int len, size_t *bytes)
{
    if (!x || !bytes || n < 2) return LC_EINVAL;
    (void)len;
    const Ctx *c = &x->c;
    const u64 S = (u64)c->nq * c->N, P = (u64)n * (n - 1) / 2;
    u64 chunk = std::min<u64>(P, (u64)c->tune.ks_chunk);
    *bytes = (P * S + chunk * ks_words_per_ct(c) + chunk * 2 * S) * 8;
    return LC_OK;
}

int lc_footprint(const lc_ctx *x, int n, int len, int k_chunk, int flags, size_t *round_bytes, size_t *workspace_bytes)
{
    if (!x || n < 2 || len < 1 || k_chunk < 0) return LC_EINVAL;
    const Ctx *c = &x->c;
    const u64 S = (u64)c->nq * c->N, P = (u64)n * (n - 1) / 2;
    const u64 k = k_chunk ? std::min<u64>((u64)k_chunk, (u64)len) : (u64)len;
    // caller-held buffers of the round
    u64 words = (u64)n * k * 2 * S + P * 2 * S;      // client ciphertexts (a chunk of k), distances
    if (k < (u64)len) words += P * 3 * S;             // streamed: the lazy triples accumulate in a buffer
    if (flags & LC_FP_SUMDIS) words += (u64)n * 2 * S;
    if (flags & LC_FP_PLAINTEXTS) words += (u64)n * k * c->N;
    if (flags & LC_FP_DECRYPT) words += P * S;
    // library workspace on the round's stream: the pipeline's d2 (resident
    // form), the key-switch batch, the rotate-and-sum ping-pong buffer and
    // (streamed form) the encryption staging of one chunk
    const u64 kc = std::min<u64>(P, (u64)c->tune.ks_chunk);
    u64 ws = kc * ks_words_per_ct(c) + kc * 2 * S;
    if (c->tune.ks_streams > 1 && P > kc) ws *= 2;  // the second stream's batches
    if (k < (u64)len) ws += std::min<u64>((u64)n * k, std::max<u64>(1, (1ull << 31) / (3 * S * 8))) * 3 * S;
    else ws += P * S;
    if (round_bytes) *round_bytes = words * 8;
    if (workspace_bytes) *workspace_bytes = ws * 8;
    return LC_OK;
}

int lc_set_tuning(lc_ctx *x, const char *name, int value)
{
    if (!x || !name) return LC_EINVAL;
    Ctx *c = &x->c;
    std::string k(name);
    if (k == "pair_lanes") {
        if (value != 8 && value != 16 && value != 32 && value != 64) return fail(c, LC_EINVAL, "pair_lanes: 8/16/32/64");
        c->tune.pair_lanes = value;
    } else if (k == "pair_mfma") {
        if (value != 0 && value != 2 && value != 4) return fail(c, LC_EINVAL, "pair_mfma: 0/2/4");
        c->tune.pair_mfma = value;
    } else if (k == "pair_ppt") {
        if (value != 1 && value != 3 && value != 4 && value != 6) return fail(c, LC_EINVAL, "pair_ppt: 1/3/4/6");
        c->tune.pair_ppt = value;
    } else if (k == "ks_chunk") {
        if (value < 1 || value > 256) return fail(c, LC_EINVAL, "ks_chunk: 1..256");
        c->tune.ks_chunk = value;
    } else if (k == "mac_cts") {
        if (value != 8 && value != 16) return fail(c, LC_EINVAL, "mac_cts: 8/16");
        c->tune.mac_cts = value;
    } else if (k == "mac_cycle") {
        if (value != 0 && value != 1) return fail(c, LC_EINVAL, "mac_cycle: 0/1");
        c->tune.mac_cycle = value;
    } else if (k == "mac_short_cts") {
        if (value != 8 && value != 16) return fail(c, LC_EINVAL, "mac_short_cts: 8/16");
        c->tune.mac_short_cts = value;
    } else if (k == "mac_cycle_cts") {
        if (value != 8 && value != 16) return fail(c, LC_EINVAL, "mac_cycle_cts: 8/16");
        c->tune.mac_cycle_cts = value;
    } else if (k == "mac_cycle_short") {
        if (value != 0 && value != 1) return fail(c, LC_EINVAL, "mac_cycle_short: 0/1");
        c->tune.mac_cycle_short = value;
    } else if (k == "mac_cycle_c0") {
        if (value != 0 && value != 1) return fail(c, LC_EINVAL, "mac_cycle_c0: 0/1");
        c->tune.mac_cycle_c0 = value;
    } else if (k == "ms_shape") {
        if (value < 0 || value > 2) return fail(c, LC_EINVAL, "ms_shape: 0/1/2");
        c->tune.ms_shape = value;
    } else if (k == "fuse_modup") {
        if (value != 0 && value != 1) return fail(c, LC_EINVAL, "fuse_modup: 0/1");
        c->tune.fuse_modup = value;
    } else if (k == "mac_cycle_min") {
        if (value < 1) return fail(c, LC_EINVAL, "mac_cycle_min: >= 1");
        c->tune.mac_cycle_min = value;
    } else if (k == "ks_streams") {
        if (value != 1 && value != 2) return fail(c, LC_EINVAL, "ks_streams: 1/2");
        c->tune.ks_streams = value;
    } else if (k == "hoist_multi") {
        if (value != 0 && value != 1) return fail(c, LC_EINVAL, "hoist_multi: 0/1");
        c->tune.hoist_multi = value;
    } else if (k == "mac_xcd") {
        if (value != 0 && value != 1) return fail(c, LC_EINVAL, "mac_xcd: 0/1");
        c->tune.mac_xcd = value;
    } else if (k == "ntt_sub_kb") {
        if (value < 0 || value > (1 << 22)) return fail(c, LC_EINVAL, "ntt_sub_kb: 0..4194304");
        c->tune.ntt_sub_kb = value;
    } else {
        return fail(c, LC_EINVAL, "unknown tuning parameter " + k);
    }
    return LC_OK;
}

int lc_set_workspace_limit(lc_ctx *x, size_t bytes)
{
    if (!x) return LC_EINVAL;
    x->c.ws_limit = bytes;
    return LC_OK;
}

}  // extern "C"
