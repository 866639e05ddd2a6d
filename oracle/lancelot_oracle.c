/*
 * lancelot_oracle.c -- plain, slow, obviously-correct CPU RNS-CKKS used as the
 * test oracle for the encrypted pairwise-distance path of Lancelot
 * (arXiv 2408.06197).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file.  Only tests/, __graft_entry__.smoke() and bench.py's
 * cpu_baseline leg use it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * Arithmetic style: every modular product is (unsigned __int128)a*b % q;
 * every transform is a textbook one.  No Montgomery, Barrett or Shoup form
 * appears here on purpose.
 *
 * Conventions (readings of places where the paper is silent are stated next
 * to each function):
 *   - Residues are canonical, in [0, q).
 *   - A polynomial over the RNS basis is laid out limb-major: [limb][N].
 *   - A ciphertext is [comp][limb][N], kept in the NTT domain (double-CRT,
 *     Appendix "Hardware Acceleration on Homomorphic Multiplication": no NTT is
 *     needed around the tensor product).
 *   - The extended basis is q_0..q_L followed by p_0..p_{K-1}.
 *
 * Parity status: every function here is pinned by tests/test_oracle_*.py
 * against brute force, closed forms, library routines or invariants.  The
 * bit patterns that follow from conventions the paper leaves open are pinned
 * too: the PRNG stream layout against numpy's Philox4x64-10, the gadget by
 * the key-structure identity, and fast base conversion, ModUp, ModDown, key
 * switching, hoisted rotations and rotate-and-sum (for several plans) bit for
 * bit against an independent Python big-integer computation at N = 16
 * (tests/test_oracle_bigint.py).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "cdt_sigma3_2.h"

typedef uint64_t u64;
typedef int64_t i64;
typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* Modular arithmetic.  Paper: Methods, "Private Distance Evaluation": R_Q is  */
/* handled limb by limb in the residue number system of the chain q_i.       */
/* ------------------------------------------------------------------------ */

static u64 add_mod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + b) % q); }
static u64 sub_mod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + q - b) % q); }
static u64 mul_mod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 neg_mod(u64 a, u64 q) { return a == 0 ? 0 : q - a; }

u64 orc_mulmod(u64 a, u64 b, u64 q) { return mul_mod(a % q, b % q, q); }
u64 orc_addmod(u64 a, u64 b, u64 q) { return add_mod(a % q, b % q, q); }
u64 orc_submod(u64 a, u64 b, u64 q) { return sub_mod(a % q, b % q, q); }

u64 orc_powmod(u64 a, u64 e, u64 q)
{
    u64 r = 1 % q, b = a % q;
    while (e) {
        if (e & 1) r = mul_mod(r, b, q);
        b = mul_mod(b, b, q);
        e >>= 1;
    }
    return r;
}

/* Inverse by Fermat's little theorem (q prime). */
u64 orc_invmod(u64 a, u64 q) { return orc_powmod(a, q - 2, q); }

/* Reduce a signed integer into [0, q). */
static u64 from_signed(i64 v, u64 q)
{
    if (v >= 0) return (u64)v % q;
    u64 m = (u64)(-(v + 1)) % q; /* -(v+1) >= 0 avoids overflow at INT64_MIN */
    return q - 1 - m;
}

/* ------------------------------------------------------------------------ */
/* Primes of the modulus chain (paper: "Q is ... a chain of prime integers",  */
/* Methods, Private Distance Evaluation; special modulus p, CKKS scheme       */
/* description).  The paper does not say which primes; reading: for each     */
/* requested bit size b in order, the largest b-bit prime of the form         */
/* c = k*M + 1 (M = 2^log_m) not already chosen.                              */
/* ------------------------------------------------------------------------ */

/* Deterministic Miller-Rabin; the first twelve primes as bases decide every */
/* n < 3.3e24, which covers all 64-bit n.                                     */
int orc_is_prime(u64 n)
{
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    u64 d = n - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; r++; }
    for (int i = 0; i < 12; i++) {
        u64 x = orc_powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int composite = 1;
        for (int j = 1; j < r; j++) {
            x = mul_mod(x, x, n);
            if (x == n - 1) { composite = 0; break; }
        }
        if (composite) return 0;
    }
    return 1;
}

/* Returns 0 on success, -1 if some bit size runs out of candidates. */
int orc_find_primes(int log_m, const int *bits, int count, u64 *out)
{
    u64 M = (u64)1 << log_m;
    for (int i = 0; i < count; i++) {
        int b = bits[i];
        if (b < 2 || b > 62) return -1;
        u64 lo = (u64)1 << (b - 1);
        u64 top = (((u64)1 << b) - 1) / M; /* largest k with k*M + 1 < 2^b */
        int found = 0;
        for (u64 k = top; k >= 1; k--) {
            u64 c = k * M + 1;
            if (c < lo) break;
            if (!orc_is_prime(c)) continue;
            int dup = 0;
            for (int j = 0; j < i; j++)
                if (out[j] == c) dup = 1;
            if (dup) continue;
            out[i] = c;
            found = 1;
            break;
        }
        if (!found) return -1;
    }
    return 0;
}

/* psi_q = the smallest x in [2, q) with x^N = -1 mod q, i.e. the smallest    */
/* primitive 2N-th root of unity (reading of the unspecified NTT root).       */
u64 orc_min_psi(u64 q, int log_n)
{
    u64 N = (u64)1 << log_n, two_n = 2 * N;
    if ((q - 1) % two_n != 0) return 0;
    u64 g = 0;
    for (u64 h = 2; h < q; h++) {
        u64 x = orc_powmod(h, (q - 1) / two_n, q);
        if (orc_powmod(x, N, q) == q - 1) { g = x; break; }
    }
    if (!g) return 0;
    /* The primitive 2N-th roots are exactly g^k for odd k. */
    u64 g2 = mul_mod(g, g, q), y = g, best = g;
    for (u64 k = 1; k < N; k++) {
        y = mul_mod(y, g2, q);
        if (y < best) best = y;
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Negacyclic NTT ("NWT", Appendix, Descriptions of Hardware Acceleration).   */
/* Definition adopted: NTT(a)[i] = sum_j a_j psi^((2 brev(i) + 1) j) mod q,   */
/* i.e. evaluation of a at the odd powers of psi in bit-reversed order.      */
/* iNTT is the exact inverse (it carries the 1/N factor).                    */
/* ------------------------------------------------------------------------ */

static u64 brev(u64 x, int bits)
{
    u64 r = 0;
    for (int i = 0; i < bits; i++) r |= ((x >> i) & 1) << (bits - 1 - i);
    return r;
}

/* O(N^2) evaluation straight from the definition. */
void orc_ntt_direct(const u64 *a, u64 *out, int log_n, u64 q, u64 psi)
{
    u64 N = (u64)1 << log_n, two_n = 2 * N;
    u64 *pw = (u64 *)malloc(two_n * sizeof(u64));
    pw[0] = 1;
    for (u64 k = 1; k < two_n; k++) pw[k] = mul_mod(pw[k - 1], psi, q);
    for (u64 i = 0; i < N; i++) {
        u64 e = 2 * brev(i, log_n) + 1, acc = 0;
        for (u64 j = 0; j < N; j++) acc = add_mod(acc, mul_mod(a[j], pw[(e * j) % two_n], q), q);
        out[i] = acc;
    }
    free(pw);
}

static void bitrev_permute(u64 *a, int log_n)
{
    u64 N = (u64)1 << log_n;
    for (u64 i = 0; i < N; i++) {
        u64 j = brev(i, log_n);
        if (j > i) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
    }
}

/* Textbook iterative radix-2 cyclic DFT over Z_q with root w (order N).     */
/* Input in natural order; output A[k] = sum_j a_j w^(jk) in natural order.  */
static void cyclic_dft(u64 *a, int log_n, u64 q, u64 w)
{
    u64 N = (u64)1 << log_n;
    bitrev_permute(a, log_n);
    for (u64 len = 2; len <= N; len <<= 1) {
        u64 wl = orc_powmod(w, N / len, q);
        for (u64 s = 0; s < N; s += len) {
            u64 t = 1;
            for (u64 j = 0; j < len / 2; j++) {
                u64 u = a[s + j], v = mul_mod(a[s + j + len / 2], t, q);
                a[s + j] = add_mod(u, v, q);
                a[s + j + len / 2] = sub_mod(u, v, q);
                t = mul_mod(t, wl, q);
            }
        }
    }
}

/* Forward negacyclic NTT in place: twist by psi^j, cyclic DFT with psi^2,   */
/* then put index k = brev(i) at position i.                                  */
void orc_ntt(u64 *a, int log_n, u64 q, u64 psi)
{
    u64 N = (u64)1 << log_n, t = 1;
    for (u64 j = 0; j < N; j++) { a[j] = mul_mod(a[j], t, q); t = mul_mod(t, psi, q); }
    cyclic_dft(a, log_n, q, mul_mod(psi, psi, q));
    bitrev_permute(a, log_n);
}

/* Inverse of orc_ntt. */
void orc_intt(u64 *a, int log_n, u64 q, u64 psi)
{
    u64 N = (u64)1 << log_n;
    u64 psi_inv = orc_invmod(psi, q), n_inv = orc_invmod(N % q, q);
    bitrev_permute(a, log_n);
    cyclic_dft(a, log_n, q, mul_mod(psi_inv, psi_inv, q));
    u64 t = n_inv;
    for (u64 j = 0; j < N; j++) { a[j] = mul_mod(a[j], t, q); t = mul_mod(t, psi_inv, q); }
}

/* Schoolbook product in Z_q[X]/(X^N + 1) (a pin for the NTT). */
void orc_negacyclic_mul(const u64 *a, const u64 *b, u64 *out, int log_n, u64 q)
{
    u64 N = (u64)1 << log_n;
    for (u64 k = 0; k < N; k++) out[k] = 0;
    for (u64 i = 0; i < N; i++)
        for (u64 j = 0; j < N; j++) {
            u64 p = mul_mod(a[i], b[j], q);
            u64 k = i + j;
            if (k < N) out[k] = add_mod(out[k], p, q);
            else out[k - N] = sub_mod(out[k - N], p, q);
        }
}

/* ------------------------------------------------------------------------ */
/* Counter-based generator: Philox4x64-10 (Salmon, Moraes, Dror, Shaw,        */
/* "Parallel random numbers: as easy as 1, 2, 3", SC 2011).  The paper only   */
/* names "a pseudo-random generator" (Appendix); this counter-based one makes */
/* every coefficient's draw a pure function of its position.                  */
/* ------------------------------------------------------------------------ */

void orc_philox4x64_10(const u64 ctr_in[4], const u64 key_in[2], u64 out[4])
{
    const u64 M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const u64 W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    u64 c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    u64 k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += W0; k1 += W1; }
        u128 p0 = (u128)M0 * c0, p1 = (u128)M1 * c2;
        u64 hi0 = (u64)(p0 >> 64), lo0 = (u64)p0;
        u64 hi1 = (u64)(p1 >> 64), lo1 = (u64)p1;
        u64 n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream layout: word number w of (seed, domain, object) is lane w % 4 of    */
/* Philox(counter = (w / 4, object, domain, 0), key = (seed, 0)).             */
static u64 draw_word(u64 seed, u64 domain, u64 object, u64 w)
{
    u64 ctr[4] = {w / 4, object, domain, 0}, key[2] = {seed, 0}, o[4];
    orc_philox4x64_10(ctr, key, o);
    return o[w % 4];
}

u64 orc_draw_word(u64 seed, u64 domain, u64 object, u64 w) { return draw_word(seed, domain, object, w); }

/* Ternary coefficients in {-1, 0, 1}: word mod 3, minus 1 (X_key, uniform). */
void orc_sample_ternary(u64 seed, u64 domain, u64 object, u64 n, i64 *out)
{
    for (u64 c = 0; c < n; c++) out[c] = (i64)(draw_word(seed, domain, object, c) % 3) - 1;
}

/* Rounded Gaussian, sigma 3.2, by inversion of the stored cumulative table.  */
i64 orc_cdt_sample(u64 w)
{
    for (int k = 0; k < 2 * ORC_CDT_TAIL; k++)
        if (w < ORC_CDT[k]) return (i64)k - ORC_CDT_TAIL;
    return ORC_CDT_TAIL;
}

void orc_sample_gaussian(u64 seed, u64 domain, u64 object, u64 n, i64 *out)
{
    for (u64 c = 0; c < n; c++) out[c] = orc_cdt_sample(draw_word(seed, domain, object, c));
}

/* Uniform residue mod q from two words: (hi * 2^64 + lo) mod q, where hi, lo */
/* are words 2c and 2c + 1 of the stream.                                     */
void orc_sample_uniform(u64 seed, u64 domain, u64 object, u64 q, u64 n, u64 *out)
{
    for (u64 c = 0; c < n; c++) {
        u64 hi = draw_word(seed, domain, object, 2 * c), lo = draw_word(seed, domain, object, 2 * c + 1);
        out[c] = (u64)((((u128)hi << 64) | lo) % q);
    }
}

void orc_cdt_table(u64 *out)
{
    for (int k = 0; k < 2 * ORC_CDT_TAIL; k++) out[k] = ORC_CDT[k];
}

/* ------------------------------------------------------------------------ */
/* Parameter context.                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int log_n;
    u64 n;
    int nq, np, alpha, dnum;
    u64 mod[64];  /* q_0..q_{nq-1}, p_0..p_{np-1} */
    u64 psi[64];
} orc_ctx;

orc_ctx *orc_ctx_new(int log_n, int nq, int np, const u64 *primes)
{
    if (nq < 1 || np < 1 || nq + np > 64) return NULL;
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    c->log_n = log_n;
    c->n = (u64)1 << log_n;
    c->nq = nq;
    c->np = np;
    c->alpha = np; /* digit size alpha = K (hybrid key switching) */
    c->dnum = (nq + np - 1) / np;
    for (int i = 0; i < nq + np; i++) {
        c->mod[i] = primes[i];
        c->psi[i] = orc_min_psi(primes[i], log_n);
        if (!c->psi[i]) { free(c); return NULL; }
    }
    return c;
}

void orc_ctx_free(orc_ctx *c) { free(c); }
u64 orc_ctx_psi(const orc_ctx *c, int i) { return c->psi[i]; }
int orc_ctx_dnum(const orc_ctx *c) { return c->dnum; }

/* NTT / iNTT over the first `nlimb` limbs of basis positions `limb0..`.      */
void orc_poly_ntt(const orc_ctx *c, u64 *p, int limb0, int nlimb)
{
#pragma omp parallel for schedule(static)
    for (int l = 0; l < nlimb; l++) orc_ntt(p + (u64)l * c->n, c->log_n, c->mod[limb0 + l], c->psi[limb0 + l]);
}

void orc_poly_intt(const orc_ctx *c, u64 *p, int limb0, int nlimb)
{
#pragma omp parallel for schedule(static)
    for (int l = 0; l < nlimb; l++) orc_intt(p + (u64)l * c->n, c->log_n, c->mod[limb0 + l], c->psi[limb0 + l]);
}

/* Signed integer coefficients -> NTT-domain residues on basis positions      */
/* 0..nlimb-1 (optionally the full extended basis).                           */
static void signed_to_ntt(const orc_ctx *c, const i64 *s, u64 *out, int nlimb)
{
    for (int l = 0; l < nlimb; l++) {
        u64 q = c->mod[l];
        u64 *o = out + (u64)l * c->n;
        for (u64 j = 0; j < c->n; j++) o[j] = from_signed(s[j], q);
    }
    orc_poly_ntt(c, out, 0, nlimb);
}

void orc_signed_to_ntt(const orc_ctx *c, const i64 *s, u64 *out, int nlimb) { signed_to_ntt(c, s, out, nlimb); }

/* ------------------------------------------------------------------------ */
/* Automorphism phi_g : X -> X^g (Methods, Dynamic Hoisting: "Automorphism"). */
/* In the NTT domain it is a permutation: output slot i holds the value at    */
/* the evaluation point psi^(e_i g) where e_i = 2 brev(i) + 1.               */
/* ------------------------------------------------------------------------ */

void orc_automorphism_index(int log_n, u64 g, u64 *idx)
{
    u64 N = (u64)1 << log_n, two_n = 2 * N;
    for (u64 i = 0; i < N; i++) {
        u64 e = (2 * brev(i, log_n) + 1) * (g % two_n) % two_n;
        idx[i] = brev((e - 1) / 2, log_n);
    }
}

/* Coefficient-domain form: X^j -> X^(jg mod 2N) = +-X^(jg mod N).            */
void orc_automorphism_coeff(const i64 *in, i64 *out, int log_n, u64 g)
{
    u64 N = (u64)1 << log_n, two_n = 2 * N;
    for (u64 j = 0; j < N; j++) {
        u64 e = j * (g % two_n) % two_n;
        if (e < N) out[e] = in[j];
        else out[e - N] = -in[j];
    }
}

static void automorphism_ntt(const orc_ctx *c, const u64 *in, u64 *out, int nlimb, u64 g)
{
    u64 *idx = (u64 *)malloc(c->n * sizeof(u64));
    orc_automorphism_index(c->log_n, g, idx);
    for (int l = 0; l < nlimb; l++) {
        const u64 *a = in + (u64)l * c->n;
        u64 *o = out + (u64)l * c->n;
        for (u64 i = 0; i < c->n; i++) o[i] = a[idx[i]];
    }
    free(idx);
}

void orc_automorphism_ntt(const orc_ctx *c, const u64 *in, u64 *out, int nlimb, u64 g)
{
    automorphism_ntt(c, in, out, nlimb, g);
}

/* Galois element of a slot rotation by k: g = 5^k mod 2N (T = <5>).          */
u64 orc_galois_elt(int log_n, i64 k)
{
    u64 two_n = (u64)2 << log_n;
    u64 half = two_n / 4; /* order of 5 modulo 2N is N/2 */
    u64 e = (u64)(((k % (i64)half) + (i64)half) % (i64)half);
    return orc_powmod(5, e, two_n);
}

/* ------------------------------------------------------------------------ */
/* Keys (Methods, CKKS scheme description: key generation).                  */
/* ------------------------------------------------------------------------ */

enum { DOM_SK = 1, DOM_PK_A = 2, DOM_PK_E = 3, DOM_ENC_V = 4, DOM_ENC_E0 = 5, DOM_ENC_E1 = 6,
       DOM_KSK_A = 7, DOM_KSK_E = 8 };

/* Secret s: ternary coefficients. */
void orc_sample_secret(u64 seed, u64 n, i64 *s) { orc_sample_ternary(seed, DOM_SK, 0, n, s); }

/* pk = ([-a s + e]_Q, a): a uniform, drawn directly in the NTT domain per    */
/* limb; e Gaussian.  pk layout [2][nq][N], NTT domain.                       */
void orc_keygen_pk_with(const orc_ctx *c, const i64 *s, const u64 *a_ntt, const i64 *e, u64 *pk)
{
    u64 N = c->n;
    u64 *sh = (u64 *)malloc((u64)c->nq * N * sizeof(u64));
    u64 *eh = (u64 *)malloc((u64)c->nq * N * sizeof(u64));
    signed_to_ntt(c, s, sh, c->nq);
    signed_to_ntt(c, e, eh, c->nq);
    for (int l = 0; l < c->nq; l++) {
        u64 q = c->mod[l];
        for (u64 j = 0; j < N; j++) {
            u64 k = (u64)l * N + j;
            pk[k] = add_mod(neg_mod(mul_mod(a_ntt[k], sh[k], q), q), eh[k], q);
            pk[(u64)c->nq * N + k] = a_ntt[k];
        }
    }
    free(sh);
    free(eh);
}

void orc_keygen_pk(const orc_ctx *c, u64 seed, const i64 *s, u64 *pk)
{
    u64 N = c->n;
    u64 *a = (u64 *)malloc((u64)c->nq * N * sizeof(u64));
    i64 *e = (i64 *)malloc(N * sizeof(i64));
    for (int l = 0; l < c->nq; l++) orc_sample_uniform(seed, DOM_PK_A, (u64)l, c->mod[l], N, a + (u64)l * N);
    orc_sample_gaussian(seed, DOM_PK_E, 0, N, e);
    orc_keygen_pk_with(c, s, a, e, pk);
    free(a);
    free(e);
}

/* Hybrid key-switching key from s' (signed coefficients) to s, with dnum    */
/* digits of alpha = K limbs each (Methods, Dynamic Hoisting, RNS decompose;  */
/* the evaluation key of the scheme description is the dnum = 1 case).       */
/*   ksk_d = ([-a_d s + e_d + G_d s']_{PQ}, a_d),                             */
/*   G_d = P mod q_i for limbs i of digit d, 0 on every other limb.           */
/* Layout [dnum][2][nq + np][N], NTT domain.  a_d is drawn in the NTT domain. */
void orc_keygen_ksk_with(const orc_ctx *c, const i64 *s, const i64 *s_target, const u64 *a_all,
                         const i64 *e_all, u64 *ksk)
{
    u64 N = c->n;
    int ne = c->nq + c->np;
    u64 *sh = (u64 *)malloc((u64)ne * N * sizeof(u64));
    u64 *th = (u64 *)malloc((u64)ne * N * sizeof(u64));
    u64 *eh = (u64 *)malloc((u64)ne * N * sizeof(u64));
    signed_to_ntt(c, s, sh, ne);
    signed_to_ntt(c, s_target, th, ne);
    for (int d = 0; d < c->dnum; d++) {
        const u64 *a = a_all + (u64)d * ne * N;
        signed_to_ntt(c, e_all + (u64)d * N, eh, ne);
        u64 *k0 = ksk + (u64)d * 2 * ne * N, *k1 = k0 + (u64)ne * N;
        for (int l = 0; l < ne; l++) {
            u64 m = c->mod[l];
            u64 g = 0;
            if (l < c->nq && l / c->alpha == d) {
                g = 1;
                for (int k = 0; k < c->np; k++) g = mul_mod(g, c->mod[c->nq + k] % m, m);
            }
            for (u64 j = 0; j < N; j++) {
                u64 x = (u64)l * N + j;
                u64 v = add_mod(neg_mod(mul_mod(a[x], sh[x], m), m), eh[x], m);
                v = add_mod(v, mul_mod(g, th[x], m), m);
                k0[x] = v;
                k1[x] = a[x];
            }
        }
    }
    free(sh);
    free(th);
    free(eh);
}

/* key_id names the key in the PRNG stream: 0 for relinearization, the Galois */
/* element g for a rotation key.                                              */
void orc_keygen_ksk(const orc_ctx *c, u64 seed, u64 key_id, const i64 *s, const i64 *s_target, u64 *ksk)
{
    u64 N = c->n;
    int ne = c->nq + c->np;
    u64 *a = (u64 *)malloc((u64)c->dnum * ne * N * sizeof(u64));
    i64 *e = (i64 *)malloc((u64)c->dnum * N * sizeof(i64));
    for (int d = 0; d < c->dnum; d++) {
        for (int l = 0; l < ne; l++)
            orc_sample_uniform(seed, DOM_KSK_A, (key_id << 32) | ((u64)d << 16) | (u64)l, c->mod[l], N,
                               a + ((u64)d * ne + l) * N);
        orc_sample_gaussian(seed, DOM_KSK_E, (key_id << 32) | (u64)d, N, e + (u64)d * N);
    }
    orc_keygen_ksk_with(c, s, s_target, a, e, ksk);
    free(a);
    free(e);
}

/* s^2 in Z[X]/(X^N + 1), exact over the integers (|coeff| <= N).           */
void orc_secret_square(const i64 *s, i64 *out, int log_n)
{
    u64 N = (u64)1 << log_n;
    for (u64 k = 0; k < N; k++) out[k] = 0;
    for (u64 i = 0; i < N; i++) {
        if (!s[i]) continue;
        for (u64 j = 0; j < N; j++) {
            i64 p = s[i] * s[j];
            if (i + j < N) out[i + j] += p;
            else out[i + j - N] -= p;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Encryption and decryption (CKKS scheme description).                       */
/* ------------------------------------------------------------------------ */

/* ct = ([m + r u0 + e0]_Q, [r u1 + e1]_Q) with pk = (u0, u1).  All inputs   */
/* are signed coefficient polynomials except pk (NTT domain).  Output [2][nq][N] NTT. */
void orc_encrypt_with(const orc_ctx *c, const i64 *m, const i64 *r, const i64 *e0, const i64 *e1,
                      const u64 *pk, u64 *ct)
{
    u64 N = c->n, S = (u64)c->nq * N;
    u64 *mh = (u64 *)malloc(S * sizeof(u64)), *rh = (u64 *)malloc(S * sizeof(u64));
    u64 *e0h = (u64 *)malloc(S * sizeof(u64)), *e1h = (u64 *)malloc(S * sizeof(u64));
    signed_to_ntt(c, m, mh, c->nq);
    signed_to_ntt(c, r, rh, c->nq);
    signed_to_ntt(c, e0, e0h, c->nq);
    signed_to_ntt(c, e1, e1h, c->nq);
    for (int l = 0; l < c->nq; l++) {
        u64 q = c->mod[l];
        for (u64 j = 0; j < N; j++) {
            u64 x = (u64)l * N + j;
            ct[x] = add_mod(add_mod(mh[x], mul_mod(rh[x], pk[x], q), q), e0h[x], q);
            ct[S + x] = add_mod(mul_mod(rh[x], pk[S + x], q), e1h[x], q);
        }
    }
    free(mh); free(rh); free(e0h); free(e1h);
}

/* Encrypt `count` plaintexts; plaintext t uses PRNG object first_object + t. */
void orc_encrypt(const orc_ctx *c, u64 seed, u64 first_object, const i64 *m, u64 count, const u64 *pk, u64 *ct)
{
    u64 N = c->n;
#pragma omp parallel for schedule(dynamic)
    for (i64 t = 0; t < (i64)count; t++) {
        i64 *r = (i64 *)malloc(3 * N * sizeof(i64));
        u64 obj = first_object + (u64)t;
        orc_sample_ternary(seed, DOM_ENC_V, obj, N, r);
        orc_sample_gaussian(seed, DOM_ENC_E0, obj, N, r + N);
        orc_sample_gaussian(seed, DOM_ENC_E1, obj, N, r + 2 * N);
        orc_encrypt_with(c, m + (u64)t * N, r, r + N, r + 2 * N, pk, ct + (u64)t * 2 * c->nq * N);
        free(r);
    }
}

/* Dec = [c0 + c1 s (+ c2 s^2)]_Q, returned in the coefficient domain.       */
/* ncomp = 2 for a ciphertext, 3 for a triple (reading: the s^2 term is       */
/* needed to read a lazily accumulated triple).                               */
void orc_decrypt(const orc_ctx *c, const u64 *ct, int ncomp, const i64 *s, u64 *out)
{
    u64 N = c->n, S = (u64)c->nq * N;
    u64 *sh = (u64 *)malloc(S * sizeof(u64));
    signed_to_ntt(c, s, sh, c->nq);
    for (int l = 0; l < c->nq; l++) {
        u64 q = c->mod[l];
        for (u64 j = 0; j < N; j++) {
            u64 x = (u64)l * N + j;
            u64 v = add_mod(ct[x], mul_mod(ct[S + x], sh[x], q), q);
            if (ncomp == 3) v = add_mod(v, mul_mod(ct[2 * S + x], mul_mod(sh[x], sh[x], q), q), q);
            out[x] = v;
        }
    }
    orc_poly_intt(c, out, 0, c->nq);
    free(sh);
}

/* ------------------------------------------------------------------------ */
/* Homomorphic add / sub / tensor (CKKS scheme description, evaluation).     */
/* ------------------------------------------------------------------------ */

void orc_ct_add(const orc_ctx *c, const u64 *a, const u64 *b, u64 *out, int ncomp)
{
    u64 N = c->n;
    for (int k = 0; k < ncomp; k++)
        for (int l = 0; l < c->nq; l++)
            for (u64 j = 0; j < N; j++) {
                u64 x = ((u64)k * c->nq + l) * N + j;
                out[x] = add_mod(a[x], b[x], c->mod[l]);
            }
}

void orc_ct_sub(const orc_ctx *c, const u64 *a, const u64 *b, u64 *out, int ncomp)
{
    u64 N = c->n;
    for (int k = 0; k < ncomp; k++)
        for (int l = 0; l < c->nq; l++)
            for (u64 j = 0; j < N; j++) {
                u64 x = ((u64)k * c->nq + l) * N + j;
                out[x] = sub_mod(a[x], b[x], c->mod[l]);
            }
}

/* (c0 c0', c0 c1' + c1 c0', c1 c1'): the triple of CKKS.Mult. */
void orc_ct_mul(const orc_ctx *c, const u64 *a, const u64 *b, u64 *out3)
{
    u64 N = c->n, S = (u64)c->nq * N;
    for (int l = 0; l < c->nq; l++) {
        u64 q = c->mod[l];
        for (u64 j = 0; j < N; j++) {
            u64 x = (u64)l * N + j;
            out3[x] = mul_mod(a[x], b[x], q);
            out3[S + x] = add_mod(mul_mod(a[x], b[S + x], q), mul_mod(a[S + x], b[x], q), q);
            out3[2 * S + x] = mul_mod(a[S + x], b[S + x], q);
        }
    }
}

/* Plaintext multiply: each component times pt (NTT domain, [nq][N]). */
void orc_mul_plain(const orc_ctx *c, const u64 *ct, const u64 *pt, u64 *out)
{
    u64 N = c->n, S = (u64)c->nq * N;
    for (int k = 0; k < 2; k++)
        for (int l = 0; l < c->nq; l++)
            for (u64 j = 0; j < N; j++) {
                u64 x = (u64)l * N + j;
                out[k * S + x] = mul_mod(ct[k * S + x], pt[x], c->mod[l]);
            }
}

/* ------------------------------------------------------------------------ */
/* Key switching (Methods, Dynamic Hoisting: RNS decompose, ModUp, switch    */
/* key, ModDown).  Fast base conversion without overflow correction and a    */
/* ModDown without rounding offset (reading of the unspecified BConv type).  */
/* ------------------------------------------------------------------------ */

/* Fast base conversion of the residues {x_i : i in src} to modulus r:        */
/* sum_i [x_i (Qs/q_i)^-1]_{q_i} (Qs/q_i) mod r, Qs = prod of src moduli.     */
/* bconv_consts fills, for each source a, inv[a] = (Qs/q_a)^-1 mod q_a and    */
/* fac[a] = (Qs/q_a) mod r; bconv_one then evaluates the sum.                 */
static void bconv_consts(const orc_ctx *c, const int *src, int ns, u64 r, u64 *inv, u64 *fac)
{
    for (int a = 0; a < ns; a++) {
        u64 qa = c->mod[src[a]];
        u64 prod_a = 1, prod_r = 1;
        for (int b = 0; b < ns; b++) {
            if (b == a) continue;
            u64 qb = c->mod[src[b]];
            prod_a = mul_mod(prod_a, qb % qa, qa);
            prod_r = mul_mod(prod_r, qb % r, r);
        }
        inv[a] = orc_invmod(prod_a, qa);
        fac[a] = prod_r;
    }
}

static u64 bconv_one(const orc_ctx *c, const int *src, int ns, const u64 *inv, const u64 *fac, const u64 *xi_hat,
                     u64 r)
{
    u64 acc = 0;
    for (int a = 0; a < ns; a++) {
        u64 y = mul_mod(xi_hat[a], inv[a], c->mod[src[a]]);
        acc = add_mod(acc, mul_mod(y % r, fac[a], r), r);
    }
    return acc;
}

/* Raise x (NTT domain, [nq][N]) into dnum digits over the extended basis:   */
/* out [dnum][nq + np][N] NTT domain.  Digit d keeps x's own limbs; every    */
/* other limb is the fast base conversion of the digit, then NTT.            */
void orc_modup(const orc_ctx *c, const u64 *x, u64 *out)
{
    u64 N = c->n;
    int ne = c->nq + c->np;
    u64 *xc = (u64 *)malloc((u64)c->nq * N * sizeof(u64));
    memcpy(xc, x, (u64)c->nq * N * sizeof(u64));
    orc_poly_intt(c, xc, 0, c->nq);
    for (int d = 0; d < c->dnum; d++) {
        int src[64], ns = 0;
        for (int i = d * c->alpha; i < c->nq && i < (d + 1) * c->alpha; i++) src[ns++] = i;
        u64 *X = out + (u64)d * ne * N;
#pragma omp parallel for schedule(static)
        for (int l = 0; l < ne; l++) {
            int own = (l < c->nq && l / c->alpha == d);
            u64 *o = X + (u64)l * N;
            if (own) { memcpy(o, x + (u64)l * N, N * sizeof(u64)); continue; }
            u64 xi[64], inv[64], fac[64];
            bconv_consts(c, src, ns, c->mod[l], inv, fac);
            for (u64 j = 0; j < N; j++) {
                for (int a = 0; a < ns; a++) xi[a] = xc[(u64)src[a] * N + j];
                o[j] = bconv_one(c, src, ns, inv, fac, xi, c->mod[l]);
            }
            orc_ntt(o, c->log_n, c->mod[l], c->psi[l]);
        }
    }
    free(xc);
}

/* ModDown of u (NTT domain over the extended basis, [nq + np][N]) to Q:      */
/* (u_Q - BConv_{P->Q}(iNTT(u_P))) * P^-1 mod q_i, result NTT domain [nq][N]. */
void orc_moddown(const orc_ctx *c, const u64 *u, u64 *out)
{
    u64 N = c->n;
    int src[64];
    for (int k = 0; k < c->np; k++) src[k] = c->nq + k;
    u64 *up = (u64 *)malloc((u64)c->np * N * sizeof(u64));
    memcpy(up, u + (u64)c->nq * N, (u64)c->np * N * sizeof(u64));
    orc_poly_intt(c, up, c->nq, c->np);
#pragma omp parallel for schedule(static)
    for (int l = 0; l < c->nq; l++) {
        u64 q = c->mod[l];
        u64 *o = out + (u64)l * N;
        u64 xi[64], inv[64], fac[64];
        bconv_consts(c, src, c->np, q, inv, fac);
        for (u64 j = 0; j < N; j++) {
            for (int k = 0; k < c->np; k++) xi[k] = up[(u64)k * N + j];
            o[j] = bconv_one(c, src, c->np, inv, fac, xi, q);
        }
        orc_ntt(o, c->log_n, q, c->psi[l]);
        u64 pinv = 1;
        for (int k = 0; k < c->np; k++) pinv = mul_mod(pinv, c->mod[c->nq + k] % q, q);
        pinv = orc_invmod(pinv, q);
        for (u64 j = 0; j < N; j++) o[j] = mul_mod(sub_mod(u[(u64)l * N + j], o[j], q), pinv, q);
    }
    free(up);
}

/* Inner product of raised digits (optionally passed through phi_g first)    */
/* with a key: acc[k] += sum_d phi_g(X_d) * ksk_d[k], k = 0, 1.  acc is       */
/* [2][nq + np][N]; g = 1 means no automorphism.                              */
static void ks_inner(const orc_ctx *c, const u64 *X, const u64 *ksk, u64 g, u64 *acc)
{
    u64 N = c->n;
    int ne = c->nq + c->np;
    u64 *idx = (u64 *)malloc(N * sizeof(u64));
    orc_automorphism_index(c->log_n, g, idx);
    for (int d = 0; d < c->dnum; d++) {
        const u64 *Xd = X + (u64)d * ne * N;
        const u64 *k0 = ksk + (u64)d * 2 * ne * N, *k1 = k0 + (u64)ne * N;
#pragma omp parallel for schedule(static)
        for (int l = 0; l < ne; l++) {
            u64 m = c->mod[l];
            for (u64 j = 0; j < N; j++) {
                u64 x = (u64)l * N + j;
                u64 v = Xd[(u64)l * N + idx[j]];
                acc[x] = add_mod(acc[x], mul_mod(v, k0[x], m), m);
                acc[(u64)ne * N + x] = add_mod(acc[(u64)ne * N + x], mul_mod(v, k1[x], m), m);
            }
        }
    }
    free(idx);
}

/* Key switch of x (NTT domain [nq][N]) with ksk: out [2][nq][N]. */
void orc_keyswitch(const orc_ctx *c, const u64 *x, const u64 *ksk, u64 *out)
{
    u64 N = c->n;
    int ne = c->nq + c->np;
    u64 *X = (u64 *)malloc((u64)c->dnum * ne * N * sizeof(u64));
    u64 *acc = (u64 *)calloc((u64)2 * ne * N, sizeof(u64));
    orc_modup(c, x, X);
    ks_inner(c, X, ksk, 1, acc);
    orc_moddown(c, acc, out);
    orc_moddown(c, acc + (u64)ne * N, out + (u64)c->nq * N);
    free(X);
    free(acc);
}

/* Relinearization of a triple: (d0 + KS0(d2), d1 + KS1(d2)), key for s^2.  */
void orc_relin(const orc_ctx *c, const u64 *ct3, const u64 *rlk, u64 *out)
{
    u64 S = (u64)c->nq * c->n;
    u64 *ks = (u64 *)malloc(2 * S * sizeof(u64));
    orc_keyswitch(c, ct3 + 2 * S, rlk, ks);
    orc_ct_add(c, ct3, ks, out, 2);
    free(ks);
}

/* Hoisted rotations (Methods, Dynamic Hoisting, reversed order): raise c1    */
/* once, then for each step t: Y_t = sum_d phi_{g_t}(X_d) * rk_t,d, ModDown,  */
/* out_t = (phi_{g_t}(c0) + Y_t,0, Y_t,1).  rks[t] is the key of step t.      */
/* outs: [nsteps][2][nq][N].                                                  */
void orc_rotate_hoisted(const orc_ctx *c, const u64 *ct, const i64 *steps, int nsteps, const u64 *const *rks,
                        u64 *outs)
{
    u64 N = c->n, S = (u64)c->nq * N;
    int ne = c->nq + c->np;
    u64 *X = (u64 *)malloc((u64)c->dnum * ne * N * sizeof(u64));
    u64 *acc = (u64 *)malloc((u64)2 * ne * N * sizeof(u64));
    u64 *tmp = (u64 *)malloc(S * sizeof(u64));
    orc_modup(c, ct + S, X);
    for (int t = 0; t < nsteps; t++) {
        u64 g = orc_galois_elt(c->log_n, steps[t]);
        u64 *o = outs + (u64)t * 2 * S;
        memset(acc, 0, (u64)2 * ne * N * sizeof(u64));
        ks_inner(c, X, rks[t], g, acc);
        orc_moddown(c, acc, o);
        orc_moddown(c, acc + (u64)ne * N, o + S);
        automorphism_ntt(c, ct, tmp, c->nq, g);
        for (int l = 0; l < c->nq; l++)
            for (u64 j = 0; j < N; j++) {
                u64 x = (u64)l * N + j;
                o[x] = add_mod(o[x], tmp[x], c->mod[l]);
            }
    }
    free(X);
    free(acc);
    free(tmp);
}

/* Rotate-and-sum (Methods, Dynamic Hoisting; the recurrence                 */
/* y <- y + HRot(y) over log2(N/2) levels), with a block plan: block b covers */
/* k_b consecutive levels starting at level j0 and does                       */
/*   y <- y + sum_{t=1}^{2^k_b - 1} rot_{t 2^j0}(y)                           */
/* with one raise of y.c1, all key products summed in PQ and ONE ModDown.    */
/* rks holds, block after block, the keys of the steps t 2^j0 in order of t. */
/* ct is [2][nq][N], updated in place.  Returns -1 if the plan is malformed. */
int orc_rotate_sum(const orc_ctx *c, u64 *ct, const int *plan, int nblocks, const u64 *const *rks)
{
    u64 N = c->n, S = (u64)c->nq * N;
    int ne = c->nq + c->np;
    int total = 0;
    for (int b = 0; b < nblocks; b++) total += plan[b];
    if (total != c->log_n - 1) return -1;
    u64 *X = (u64 *)malloc((u64)c->dnum * ne * N * sizeof(u64));
    u64 *acc = (u64 *)malloc((u64)2 * ne * N * sizeof(u64));
    u64 *ks = (u64 *)malloc(2 * S * sizeof(u64));
    u64 *rot0 = (u64 *)malloc(S * sizeof(u64));
    u64 *c0sum = (u64 *)malloc(S * sizeof(u64));
    int j0 = 0, key = 0;
    for (int b = 0; b < nblocks; b++) {
        int kb = plan[b];
        int nt = (1 << kb) - 1;
        orc_modup(c, ct + S, X);
        memset(acc, 0, (u64)2 * ne * N * sizeof(u64));
        memset(c0sum, 0, S * sizeof(u64));
        for (int t = 1; t <= nt; t++) {
            u64 g = orc_galois_elt(c->log_n, (i64)t << j0);
            ks_inner(c, X, rks[key++], g, acc);
            automorphism_ntt(c, ct, rot0, c->nq, g);
            for (int l = 0; l < c->nq; l++)
                for (u64 j = 0; j < N; j++) {
                    u64 x = (u64)l * N + j;
                    c0sum[x] = add_mod(c0sum[x], rot0[x], c->mod[l]);
                }
        }
        orc_moddown(c, acc, ks);
        orc_moddown(c, acc + (u64)ne * N, ks + S);
        for (int l = 0; l < c->nq; l++)
            for (u64 j = 0; j < N; j++) {
                u64 x = (u64)l * N + j;
                u64 q = c->mod[l];
                ct[x] = add_mod(add_mod(ct[x], c0sum[x], q), ks[x], q);
                ct[S + x] = add_mod(ct[S + x], ks[S + x], q);
            }
        j0 += kb;
    }
    free(X); free(acc); free(ks); free(rot0); free(c0sum);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Server Executes (Algorithm 1): for each pair i < j, sum over the LEN       */
/* packed ciphertexts of (ct_i[k] - ct_j[k])^2 kept as triples (lazy          */
/* relinearization, Methods), relinearize once, then rotate-and-sum.         */
/* Reading: j runs over j > i and the accumulator restarts for every pair.    */
/* ------------------------------------------------------------------------ */

/* Accumulated triple of one pair: out3 [3][nq][N]. */
void orc_pair_triple(const orc_ctx *c, const u64 *cts, int len, int i, int j, u64 *out3)
{
    u64 N = c->n, S = (u64)c->nq * N;
    memset(out3, 0, 3 * S * sizeof(u64));
#pragma omp parallel for schedule(static)
    for (int l = 0; l < c->nq; l++) {
        u64 q = c->mod[l];
        for (int k = 0; k < len; k++) {
            const u64 *a = cts + ((u64)i * len + k) * 2 * S;
            const u64 *b = cts + ((u64)j * len + k) * 2 * S;
            for (u64 t = 0; t < N; t++) {
                u64 x = (u64)l * N + t;
                u64 d0 = sub_mod(a[x], b[x], q), d1 = sub_mod(a[S + x], b[S + x], q);
                out3[x] = add_mod(out3[x], mul_mod(d0, d0, q), q);
                out3[S + x] = add_mod(out3[S + x], mul_mod(2, mul_mod(d0, d1, q), q), q);
                out3[2 * S + x] = add_mod(out3[2 * S + x], mul_mod(d1, d1, q), q);
            }
        }
    }
}

/* Full pairwise pipeline.  cts [n][len][2][nq][N]; dist [P][2][nq][N] in    */
/* row-major upper-triangle pair order; sumdis [n][2][nq][N] or NULL (reading: */
/* SumDis[i] = sum over j != i of Dis[i][j]); triples [P][3][nq][N] or NULL.  */
/* pairs_only: if non-NULL, an array of npairs pair indices to compute (others */
/* left untouched); sumdis must be NULL then.                                 */
int orc_pairwise(const orc_ctx *c, const u64 *cts, int n, int len, const u64 *rlk, const int *plan, int nblocks,
                 const u64 *const *rks, u64 *dist, u64 *sumdis, u64 *triples, const int *pairs_only, int npairs)
{
    u64 S = (u64)c->nq * c->n;
    int P = n * (n - 1) / 2;
    int pi[4096], pj[4096];
    if (P > 4096) return -1;
    for (int i = 0, p = 0; i < n; i++)
        for (int j = i + 1; j < n; j++, p++) { pi[p] = i; pj[p] = j; }
    int cnt = pairs_only ? npairs : P;
    if (pairs_only && sumdis) return -1;
    u64 *t3 = (u64 *)malloc(3 * S * sizeof(u64));
    for (int w = 0; w < cnt; w++) {
        int p = pairs_only ? pairs_only[w] : w;
        if (p < 0 || p >= P) { free(t3); return -1; }
        orc_pair_triple(c, cts, len, pi[p], pj[p], t3);
        if (triples) memcpy(triples + (u64)p * 3 * S, t3, 3 * S * sizeof(u64));
        u64 *d = dist + (u64)p * 2 * S;
        orc_relin(c, t3, rlk, d);
        if (orc_rotate_sum(c, d, plan, nblocks, rks) != 0) { free(t3); return -1; }
    }
    free(t3);
    if (sumdis) {
        memset(sumdis, 0, (u64)n * 2 * S * sizeof(u64));
        for (int p = 0; p < P; p++) {
            const u64 *d = dist + (u64)p * 2 * S;
            orc_ct_add(c, sumdis + (u64)pi[p] * 2 * S, d, sumdis + (u64)pi[p] * 2 * S, 2);
            orc_ct_add(c, sumdis + (u64)pj[p] * 2 * S, d, sumdis + (u64)pj[p] * 2 * S, 2);
        }
    }
    return 0;
}

/* ServerUpdate (Algorithm 1): agg[k] = sum_i ct_i[k] * mask_i, plaintext    */
/* masks in the NTT domain [n][nq][N]; out [len][2][nq][N].                   */
void orc_masked_sum(const orc_ctx *c, const u64 *cts, int n, int len, const u64 *masks, u64 *out)
{
    u64 N = c->n, S = (u64)c->nq * N;
    memset(out, 0, (u64)len * 2 * S * sizeof(u64));
    u64 *tmp = (u64 *)malloc(2 * S * sizeof(u64));
    for (int k = 0; k < len; k++)
        for (int i = 0; i < n; i++) {
            orc_mul_plain(c, cts + ((u64)i * len + k) * 2 * S, masks + (u64)i * S, tmp);
            orc_ct_add(c, out + (u64)k * 2 * S, tmp, out + (u64)k * 2 * S, 2);
        }
    free(tmp);
}
