// Host-side construction of a parameter set: primes, NTT roots and twiddles,
// base-conversion constants, automorphism index maps.  All device tables are
// built here once per context and uploaded.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "lc_internal.h"

namespace lc {

typedef unsigned __int128 u128;

static u64 mulm(u64 a, u64 b, u64 m) { return (u64)((u128)a * b % m); }
static u64 powm(u64 a, u64 e, u64 m)
{
    u64 r = 1 % m;
    a %= m;
    for (; e; e >>= 1) {
        if (e & 1) r = mulm(r, a, m);
        a = mulm(a, a, m);
    }
    return r;
}
static u64 invm(u64 a, u64 m) { return powm(a, m - 2, m); }
static u64 shoup_of(u64 w, u64 m) { return (u64)(((u128)w << 64) / m); }

// Strong-probable-prime test with the seven bases of Jaeschke/Sinclair that
// decide primality for every n < 2^64.
static bool is_prime64(u64 n)
{
    if (n < 4) return n >= 2;
    if ((n & 1) == 0) return false;
    for (u64 p : {3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull})
        if (n % p == 0) return n == p;
    u64 d = n - 1;
    int s = 0;
    while (!(d & 1)) d >>= 1, s++;
    for (u64 a : {2ull, 325ull, 9375ull, 28178ull, 450775ull, 9780504ull, 1795265022ull}) {
        u64 b = a % n;
        if (b == 0) continue;
        u64 x = powm(b, d, n);
        if (x == 1 || x == n - 1) continue;
        bool witness = true;
        for (int r = 1; r < s && witness; r++) {
            x = mulm(x, x, n);
            if (x == n - 1) witness = false;
        }
        if (witness) return false;
    }
    return true;
}

static u64 bit_reverse(u64 x, int bits)
{
    u64 r = 0;
    for (int i = 0; i < bits; i++, x >>= 1) r = (r << 1) | (x & 1);
    return r;
}

// Smallest primitive 2N-th root of unity mod q.
static u64 smallest_psi(u64 q, int log_n)
{
    u64 two_n = 2ull << log_n;
    if ((q - 1) % two_n) return 0;
    u64 root = 0;
    for (u64 h = 2; h < 1000000 && !root; h++) {
        u64 x = powm(h, (q - 1) / two_n, q);
        if (powm(x, two_n / 2, q) == q - 1) root = x;  // order exactly 2N
    }
    if (!root) return 0;
    u64 step = mulm(root, root, q), best = root, y = root;
    for (u64 k = 1; k < two_n / 2; k++) {
        y = mulm(y, step, q);
        if (y < best) best = y;
    }
    return best;
}

u64 galois_of_step(int log_n, long long step)
{
    long long half = 1ll << (log_n - 1);  // order of 5 in (Z/2N)^*
    long long e = ((step % half) + half) % half;
    return powm(5, (u64)e, 2ull << log_n);
}

std::vector<u32> automorphism_perm(int log_n, u64 g)
{
    u64 N = 1ull << log_n, two_n = 2 * N;
    std::vector<u32> p(N);
    for (u64 i = 0; i < N; i++) {
        u64 e = (2 * bit_reverse(i, log_n) + 1) * (g % two_n) % two_n;
        p[i] = (u32)bit_reverse((e - 1) / 2, log_n);
    }
    return p;
}

void *dev_alloc(Ctx *c, size_t bytes)
{
    void *p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 8) != hipSuccess) return nullptr;
    c->allocs.push_back(p);
    return p;
}

u32 *get_perm(Ctx *c, u64 g)
{
    auto it = c->perms.find(g);
    if (it != c->perms.end()) return it->second;
    std::vector<u32> h = automorphism_perm(c->log_n, g);
    u32 *d = (u32 *)dev_alloc(c, h.size() * sizeof(u32));
    if (!d) return nullptr;
    if (hipMemcpy(d, h.data(), h.size() * sizeof(u32), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    c->table_bytes += h.size() * sizeof(u32);
    c->perms[g] = d;
    return d;
}

template <class T>
static const T *upload(Ctx *c, const std::vector<T> &h)
{
    if (c->device < 0) return nullptr;  // host-only context
    T *d = (T *)dev_alloc(c, h.size() * sizeof(T));
    if (!d) return nullptr;
    if (hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    c->table_bytes += h.size() * sizeof(T);
    return d;
}

int degree_tables(Ctx *c, int log_n, DegreeTables *out)
{
    if (log_n == c->log_n) {
        *out = DegreeTables{c->dp.twd, c->dp.itwd, c->dp.ninv};
        return LC_OK;
    }
    if (log_n < 1 || log_n > c->log_n) return fail(c, LC_EINVAL, "ring degree above the context's");
    auto it = c->degree_tabs.find(log_n);
    if (it != c->degree_tabs.end()) {
        *out = it->second;
        return LC_OK;
    }
    // the same construction as the context's own tables, with the smallest
    // primitive 2^(log_n + 1)-th root of each modulus
    const int ne = c->ne;
    const u64 N = 1ull << log_n;
    std::vector<double> twd(ne * N), itwd(ne * N);
    std::vector<u64> ninv(ne);
    for (int l = 0; l < ne; l++) {
        const u64 m = c->mod[l], psi = smallest_psi(m, log_n);
        if (!psi) return fail(c, LC_EINVAL, "a modulus has no root of unity of that order");
        const u64 ipsi = invm(psi, m);
        std::vector<u64> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (u64 k = 1; k < N; k++) {
            pw[k] = mulm(pw[k - 1], psi, m);
            ipw[k] = mulm(ipw[k - 1], ipsi, m);
        }
        for (u64 k = 0; k < N; k++) {
            const u64 r = bit_reverse(k, log_n);
            twd[l * N + k] = (double)pw[r];
            itwd[l * N + k] = (double)ipw[r];
        }
        ninv[l] = invm(N % m, m);
    }
    DegreeTables t{upload(c, twd), upload(c, itwd), upload(c, ninv)};
    if (!t.twd || !t.itwd || !t.ninv) return fail(c, LC_ENOMEM, "could not upload twiddle tables");
    c->degree_tabs[log_n] = t;
    *out = t;
    return LC_OK;
}

int build_params(Ctx *c, const lc_params *prm)
{
    if (!prm) return fail(c, LC_EINVAL, "params is NULL");
    if (prm->log_n < 3 || prm->log_n > 17) return fail(c, LC_EUNSUP, "log_n must lie in [3, 17]");
    if (prm->n_q < 1 || prm->n_q > 48 || prm->n_p < 1 || prm->n_p > MAX_NP)
        return fail(c, LC_EUNSUP, "need 1 <= n_q <= 48 and 1 <= n_p <= 8");
    if (!prm->q_bits || !prm->p_bits) return fail(c, LC_EINVAL, "bit-size arrays are NULL");
    c->log_n = prm->log_n;
    c->N = 1ull << prm->log_n;
    c->nq = prm->n_q;
    c->np = prm->n_p;
    c->ne = c->nq + c->np;
    c->alpha = c->np;
    c->dnum = (c->nq + c->alpha - 1) / c->alpha;
    c->log_m = prm->log_m ? prm->log_m : prm->log_n + 1;
    if (c->log_m < c->log_n + 1 || c->log_m > 40) return fail(c, LC_EINVAL, "log_m must be >= log_n + 1");

    // primes
    std::vector<int> bits;
    for (int i = 0; i < c->nq; i++) bits.push_back(prm->q_bits[i]);
    for (int i = 0; i < c->np; i++) bits.push_back(prm->p_bits[i]);
    u64 M = 1ull << c->log_m;
    for (int b : bits) {
        if (b < 20 || b > 50) return fail(c, LC_EUNSUP, "modulus bit sizes must lie in [20, 50]");
        u64 lo = 1ull << (b - 1);
        u64 k = ((1ull << b) - 1) / M;
        u64 found = 0;
        for (; k >= 1; k--) {
            u64 cand = k * M + 1;
            if (cand < lo) break;
            bool taken = false;
            for (u64 x : c->mod) taken |= (x == cand);
            if (!taken && is_prime64(cand)) { found = cand; break; }
        }
        if (!found) return fail(c, LC_EINVAL, "ran out of NTT-friendly primes of " + std::to_string(b) + " bits");
        c->mod.push_back(found);
    }
    for (u64 q : c->mod) {
        u64 psi = smallest_psi(q, c->log_n);
        if (!psi) return fail(c, LC_EINVAL, "no 2N-th root of unity");
        c->psi.push_back(psi);
    }

    const int ne = c->ne, nq = c->nq, np = c->np, alpha = c->alpha, dnum = c->dnum;
    const u64 N = c->N;
    DevParams &d = c->dp;
    d.log_n = c->log_n;
    d.N = (u32)N;
    d.nq = nq;
    d.np = np;
    d.ne = ne;
    d.alpha = alpha;
    d.dnum = dnum;

    std::vector<ModConst> mc(ne);
    for (int l = 0; l < ne; l++) {
        u64 m = c->mod[l];
        mc[l].m = m;
        mc[l].c50 = (u64)(((u128)1 << 50) % m);
        mc[l].c50sh = shoup_of(mc[l].c50, m);
        mc[l].c25 = (u64)(((u128)1 << 25) % m);
        mc[l].c25sh = shoup_of(mc[l].c25, m);
        mc[l].one_sh = shoup_of(1, m);
        mc[l].qd = (double)m;
        mc[l].qinv = 1.0 / (double)m;
    }
    d.mc = upload(c, mc);

    // twiddles: tw[l][k] = psi^brev(k) for k in [0, N); itw = inverses
    std::vector<u64> tw(ne * N), tws(ne * N), itw(ne * N), itws(ne * N), ninv(ne), ninvs(ne);
    std::vector<double> twd(ne * N), itwd(ne * N);
    for (int l = 0; l < ne; l++) {
        u64 m = c->mod[l], psi = c->psi[l], ipsi = invm(psi, m);
        std::vector<u64> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (u64 k = 1; k < N; k++) {
            pw[k] = mulm(pw[k - 1], psi, m);
            ipw[k] = mulm(ipw[k - 1], ipsi, m);
        }
        for (u64 k = 0; k < N; k++) {
            u64 r = bit_reverse(k, c->log_n);
            tw[l * N + k] = pw[r];
            tws[l * N + k] = shoup_of(pw[r], m);
            itw[l * N + k] = ipw[r];
            itws[l * N + k] = shoup_of(ipw[r], m);
            twd[l * N + k] = (double)pw[r];
            itwd[l * N + k] = (double)ipw[r];
        }
        ninv[l] = invm(N % m, m);
        ninvs[l] = shoup_of(ninv[l], m);
    }
    d.tw = upload(c, tw);
    d.tw_sh = upload(c, tws);
    d.itw = upload(c, itw);
    d.itw_sh = upload(c, itws);
    d.ninv = upload(c, ninv);
    d.ninv_sh = upload(c, ninvs);
    d.twd = upload(c, twd);
    d.itwd = upload(c, itwd);

    // ModUp constants per digit
    std::vector<u64> upi(dnum * alpha, 0), upis(dnum * alpha, 0), upf((size_t)dnum * alpha * ne, 0);
    for (int dg = 0; dg < dnum; dg++) {
        int a0 = dg * alpha, a1 = std::min(nq, a0 + alpha);
        for (int a = a0; a < a1; a++) {
            u64 qa = c->mod[a];
            u64 prod = 1;
            for (int b = a0; b < a1; b++)
                if (b != a) prod = mulm(prod, c->mod[b] % qa, qa);
            upi[dg * alpha + (a - a0)] = invm(prod, qa);
            upis[dg * alpha + (a - a0)] = shoup_of(upi[dg * alpha + (a - a0)], qa);
            for (int l = 0; l < ne; l++) {
                u64 m = c->mod[l], f = 1;
                for (int b = a0; b < a1; b++)
                    if (b != a) f = mulm(f, c->mod[b] % m, m);
                upf[((size_t)dg * alpha + (a - a0)) * ne + l] = f;
            }
        }
    }
    std::vector<u64> ups(ne);
    for (int l = 0; l < nq; l++) ups[l] = mulm(ninv[l], upi[(size_t)(l / alpha) * alpha + l % alpha], c->mod[l]);
    d.up_inv = upload(c, upi);
    d.up_inv_sh = upload(c, upis);
    d.up_fac = upload(c, upf);
    d.up_inv_d = upload(c, std::vector<double>(upi.begin(), upi.end()));
    d.up_fac_d = upload(c, std::vector<double>(upf.begin(), upf.end()));

    // ModDown constants
    std::vector<u64> dni(np), dnis(np), dnf((size_t)np * nq), pinv(nq), pinvs(nq), pmod(nq);
    for (int k = 0; k < np; k++) {
        u64 pk = c->mod[nq + k], prod = 1;
        for (int j = 0; j < np; j++)
            if (j != k) prod = mulm(prod, c->mod[nq + j] % pk, pk);
        dni[k] = invm(prod, pk);
        dnis[k] = shoup_of(dni[k], pk);
        for (int l = 0; l < nq; l++) {
            u64 m = c->mod[l], f = 1;
            for (int j = 0; j < np; j++)
                if (j != k) f = mulm(f, c->mod[nq + j] % m, m);
            dnf[(size_t)k * nq + l] = f;
        }
    }
    for (int l = 0; l < nq; l++) {
        u64 m = c->mod[l], P = 1;
        for (int k = 0; k < np; k++) P = mulm(P, c->mod[nq + k] % m, m);
        pmod[l] = P;
        pinv[l] = invm(P, m);
        pinvs[l] = shoup_of(pinv[l], m);
    }
    for (int k = 0; k < np; k++) ups[nq + k] = mulm(ninv[nq + k], dni[k], c->mod[nq + k]);
    d.ks_scale = upload(c, ups);
    d.dn_inv = upload(c, dni);
    d.dn_inv_sh = upload(c, dnis);
    d.dn_fac = upload(c, dnf);
    d.dn_inv_d = upload(c, std::vector<double>(dni.begin(), dni.end()));
    d.dn_fac_d = upload(c, std::vector<double>(dnf.begin(), dnf.end()));
    d.pinv = upload(c, pinv);
    d.pinv_sh = upload(c, pinvs);
    d.pmod = upload(c, pmod);
    // rescaling by q_t: q_t^-1 mod q_i for every pair i < t of Q limbs
    std::vector<u64> rsi((size_t)nq * nq, 0), rsis((size_t)nq * nq, 0);
    for (int t = 1; t < nq; t++)
        for (int i = 0; i < t; i++) {
            const u64 m = c->mod[i];
            rsi[(size_t)t * nq + i] = invm(c->mod[t] % m, m);
            rsis[(size_t)t * nq + i] = shoup_of(rsi[(size_t)t * nq + i], m);
        }
    d.rs_inv = upload(c, rsi);
    d.rs_inv_sh = upload(c, rsis);

    std::vector<u64> cdt(38);
    cdt_thresholds(cdt.data());
    d.cdt = upload(c, cdt);
    c->cdt_host = cdt;

    if (c->device < 0) return LC_OK;
    if (!d.twd || !d.itwd || !d.up_inv_d || !d.up_fac_d || !d.dn_inv_d || !d.dn_fac_d || !d.ks_scale)
        return fail(c, LC_ENOMEM, "could not upload parameter tables");
    if (!d.mc || !d.tw || !d.tw_sh || !d.itw || !d.itw_sh || !d.ninv || !d.ninv_sh || !d.up_inv || !d.up_inv_sh ||
        !d.up_fac || !d.dn_inv || !d.dn_inv_sh || !d.dn_fac || !d.pinv || !d.pinv_sh || !d.pmod || !d.cdt ||
        !d.rs_inv || !d.rs_inv_sh)
        return fail(c, LC_ENOMEM, "could not upload parameter tables");
    return LC_OK;
}

}  // namespace lc
