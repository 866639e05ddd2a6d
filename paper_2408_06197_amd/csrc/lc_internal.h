// Internal declarations shared by the HIP translation units of the engine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/lancelot.h"
#include "modarith.h"

namespace lc {

typedef int64_t i64;

constexpr int MAX_LIMBS = 56;
constexpr int MAX_NP = 8;

// Everything a kernel needs to know about the parameter set; passed by value.
struct DevParams {
    int log_n;
    u32 N;
    int nq, np, ne, alpha, dnum;
    const ModConst *mc;  // [ne]
    const u64 *tw, *tw_sh;    // [ne][N]: psi^brev(k) and Shoup companions
    const u64 *itw, *itw_sh;  // [ne][N]: inverses of the above
    const u64 *ninv, *ninv_sh;  // [ne]: N^-1 mod m
    const double *twd, *itwd;   // [ne][N]: the twiddles above as doubles (FP64 butterflies)
    const u64 *up_inv, *up_inv_sh;  // [dnum][alpha]: (Q_d / q_a)^-1 mod q_a
    const u64 *up_fac;              // [dnum][alpha][ne]: (Q_d / q_a) mod m_l
    const u64 *dn_inv, *dn_inv_sh;  // [np]: (P / p_k)^-1 mod p_k
    const u64 *dn_fac;              // [np][nq]: (P / p_k) mod q_l
    const u64 *ks_scale;            // [ne]: scale of a key switch's last inverse pass: N^-1 (Q_d / q_a)^-1
                                    // mod q_a for limb a of digit d, N^-1 (P / p_k)^-1 mod p_k for P limb k
    const double *up_inv_d, *up_fac_d, *dn_inv_d, *dn_fac_d;  // the four tables above as doubles
    const u64 *pinv, *pinv_sh;      // [nq]: P^-1 mod q_l
    const u64 *pmod;                // [nq]: P mod q_l (gadget)
    const u64 *rs_inv, *rs_inv_sh;  // [nq][nq]: q_t^-1 mod q_i at [t][i] (i < t), for rescaling by q_t
    const u64 *cdt;                 // [38]: Gaussian thresholds
};

// Cycle walk of an automorphism's tile map (the cycle-walking key-switch
// inner product): with tiles of KS_CYC_TILE coefficients, the NTT-domain
// permutation of a Galois element maps every aligned tile onto one aligned
// tile.  `walk` lists the tiles cycle by cycle in map order; segment s covers
// output positions m0 .. m0 + cnt - 1 of the cycle at walk[base .. base + len).
constexpr int KS_CYC_TILE = 32;
constexpr int KS_CYC_SEG = 32;
constexpr int MULTI_KEYS = 8;  // keys per source-major inner product (literal hoisted rotations)
struct CycleSeg {
    int base, len, m0, cnt;
};
struct CycleTable {
    const CycleSeg *segs = nullptr;
    const u32 *walk = nullptr;
    int nseg = 0;     // 0: the map does not act on tiles (N below the tile size)
    int min_len = 0;  // shortest cycle (all cycles have one length for a power of 5)
    int max_len = 0;  // longest cycle
    const u32 *inv_tile = nullptr;  // [N / KS_CYC_TILE]: source tile -> output tile (the inverse tile map)
};

struct RotKey {
    u64 *ksk = nullptr;    // [dnum][2][ne][N]
    u32 *perm = nullptr;   // [N]: NTT-domain index map of the automorphism
    u64 galois = 0;
};

// Twiddles (forward and inverse, as doubles, [ne][N]) and N^-1 mod m of one
// ring degree.
struct DegreeTables {
    const double *twd = nullptr, *itwd = nullptr;
    const u64 *ninv = nullptr;
};

struct Ctx {
    int device = 0, role = 0;
    int log_n = 0;
    u64 N = 0;
    int nq = 0, np = 0, ne = 0, alpha = 0, dnum = 0, log_m = 0;
    std::vector<u64> mod, psi;
    std::vector<u64> cdt_host;
    std::string err;

    // device tables (one allocation each, freed at destroy)
    std::vector<void *> allocs;
    DevParams dp{};

    // keys
    u64 *pk = nullptr;       // [2][nq][N]
    u64 *pk_sh = nullptr;    // Shoup companions of pk
    u64 *rlk = nullptr;      // [dnum][2][ne][N]
    std::map<u64, RotKey> rot;   // galois element -> key
    std::map<u64, u32 *> perms;  // galois element -> permutation (also for keyless uses)
    i64 *sk_coeff = nullptr;     // [N] (KGC only)
    u64 *sk_ntt = nullptr;       // [ne][N]
    u64 *sk_ntt_sh = nullptr;
    u64 *sk2_ntt = nullptr;      // [nq][N]: s^2
    u64 *sk2_ntt_sh = nullptr;

    // workspace: independent slots grown on demand, one set per stream so
    // that work queued on different streams never shares scratch memory
    struct Workspace {
        void *slot[8] = {};
        size_t bytes[8] = {};
    };
    std::map<hipStream_t, Workspace> ws;
    std::vector<void *> retired;  // outgrown workspace buffers, freed with the context
    size_t retired_bytes = 0;
    std::map<u64, CycleTable> cycles;  // by Galois element
    // device encode tables (built on first use): exp(-2 pi i j / N),
    // exp(-i pi k / N) as (re, im) doubles, and the slot of each odd exponent
    void *enc_w = nullptr, *enc_twist = nullptr;
    int *enc_slot = nullptr;
    size_t ws_limit = 0;
    size_t gram_lds_allowed[2] = {0, 0};  // dynamic LDS granted to the Gram-form pair kernel (2 / 4 coefficients)

    // launch-shape tuning (lc_set_tuning)
    struct Tuning {
        int pair_lanes = 16;  // coefficients per workgroup of the pair-triple kernel
        int pair_ppt = 4;     // pairs per lane (1, 3, 4 or 6)
        int pair_mfma = 0;    // Gram form on the int8 MFMA with 4 or 2 coefficients per workgroup (0: per-pair form)
        int ks_chunk = 64;    // ciphertexts per key-switch batch
        int ntt_sub_kb = 0;   // two-pass NTTs run per sub-batch of this many KiB (0: whole batch)
        int mac_cts = 8;      // ciphertexts per lane of the key-switch inner product (8 or 16)
        int mac_cycle = 1;    // hoisted blocks of 3 or 7 keys use the cycle-walking inner product ...
        int mac_cycle_min = 16;  // ... when the tile cycles are at least this long
        int mac_cycle_cts = 8;   // ciphertexts per cycle-walk workgroup (8 or 16)
        int mac_short_cts = 16;  // ciphertexts per short-cycle workgroup (8 or 16)
        int mac_cycle_c0 = 1;    // the inner product (walk or gather) also folds sum_t phi_t(c0) into the accumulator
        int mac_cycle_short = 1; // blocks whose tile cycles are at most 2 tiles long skip the walk
        int fuse_modup = 1;   // ModUp conversion fused into the first forward-NTT pass (N >= 2^10)
        int ms_shape = 2;     // masked-sum lane shape: 0 = 1 coefficient x 16 rows, 1 = 2 x 8, 2 = 2 x 16
        int ks_streams = 2;   // streams the batches of a pairwise finish alternate over (1 or 2)
        int hoist_multi = 1;  // literal hoisted rotations stage each source tile once for up to 8 keys
        int mac_xcd = 1;      // cycle-walk / short-cycle workgroups sharing key tiles run on one XCD
    } tune;
    size_t table_bytes = 0, key_bytes = 0;
    std::map<int, DegreeTables> degree_tabs;  // by log_n, below the context's degree
    // a second stream per caller stream (created on first use, default
    // priority), so that independent key-switch batches of one call overlap
    // on the device, and the events that fork it from and join it back to
    // the caller's stream
    struct Aux {
        hipStream_t stream = nullptr;
        hipEvent_t fork = nullptr, join = nullptr;
    };
    std::map<hipStream_t, Aux> aux;
};

// error helpers (set ctx->err and return the code)
int fail(Ctx *c, int code, const std::string &msg);
int hip_fail(Ctx *c, hipError_t e, const char *what);

#define LC_HIP(ctx, call)                                  \
    do {                                                   \
        hipError_t _e = (call);                            \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #call); \
    } while (0)

// device memory owned by the context
void *dev_alloc(Ctx *c, size_t bytes);
enum { WS_KS = 0, WS_PIPE = 1, WS_ROT = 2, WS_ENC = 3, WS_TMP = 4, WS_KEYGEN = 5, WS_ENCODE = 6, WS_RESCALE = 7 };
// Pointer to workspace slot `slot` of stream `s` holding at least `bytes`;
// NULL (with ctx->err set) if it cannot be allocated.  Growing a slot waits
// for the work already queued on `s`.
u64 *ws_get(Ctx *c, int slot, size_t bytes, hipStream_t s);

// host-side parameter setup (params.cpp)
int build_params(Ctx *c, const lc_params *prm);
u64 galois_of_step(int log_n, long long step);
std::vector<u32> automorphism_perm(int log_n, u64 g);
u32 *get_perm(Ctx *c, u64 g);
void cdt_thresholds(u64 out[38]);  // cdt.cpp (quad precision)

// host FP64 encode/decode (encode.cpp)
void encode_host(int log_n, const double *re, const double *im, size_t nslots, double scale, i64 *m);
int launch_encode(Ctx *c, const double *z, u64 count, u64 nslots, u64 z_stride, double scale, i64 *m, hipStream_t s);
int launch_rescale(Ctx *c, const u64 *ct, u64 count, int ncomp, int nlimb, u64 *out, hipStream_t s);
void decode_host(int log_n, const double *coeff, double scale, double *re, double *im);
void crt_to_double(const std::vector<u64> &q, const u64 *res, size_t ncoeff, size_t stride, double *out);

// ---- kernel launchers ----------------------------------------------------
// A batch of limb-polynomials for the NTT: polynomial p (0 <= p < count*nlimb)
// lives at base + ((p / nlimb) * gstride + (p % nlimb)) * N and uses modulus
// limb0 + p % nlimb.  If skip_own_digit, group g = p / nlimb belongs to digit
// g % dnum and limbs l < nq with l / alpha == digit are skipped.
struct PolyBatch {
    u64 *base;
    u64 count;     // groups
    int nlimb;
    u64 gstride;   // in polynomials
    int limb0;
    int skip_own_digit;
    // inverse only: per-limb scale of the last pass (by absolute limb; NULL = N^-1)
    const u64 *iscale = nullptr;
    // the last pass writes canonical residues as doubles (bit patterns)
    // instead of uint64: the form the fused conversions below read
    int out_f64 = 0;
    // forward only, two-pass transforms: the first pass computes its input
    // as a base conversion (conv = 1: ModUp, 2: ModDown) of canonical
    // residues in conv_y, stored as doubles (out_f64), instead of reading
    // base.
    //   ModUp: groups = (ciphertext, digit) of raised limbs; conv_y is
    //     [count / dnum][nq][N] (conv_stride words per ciphertext), limb a of
    //     digit d already scaled by (Q_d / q_a)^-1.
    //   ModDown: groups = (ciphertext, component) of nq limbs; conv_y holds
    //     each group's np limbs (conv_stride words per group), limb k
    //     already scaled by (P / p_k)^-1.
    int conv = 0;
    const u64 *conv_y = nullptr;
    u64 conv_stride = 0;
    // forward only, two-pass transforms, groups = (ciphertext, component)
    // of nq limbs: the last pass writes the ModDown result
    //   comb_out = (comb_acc - this transform) P^-1 (+ comb_add)
    // instead of base.  comb_acc: comb_acc_stride words per group;
    // comb_add / comb_out: stride words per ciphertext, component 1 at +nq N.
    const u64 *comb_acc = nullptr;
    u64 comb_acc_stride = 0;
    const u64 *comb_add = nullptr;
    u64 comb_add_stride = 0;
    u64 *comb_out = nullptr;
    u64 comb_out_stride = 0;
    // two-pass transforms (2^10 <= N <= 2^17) only: the first pass reads
    // group g, limb l from in_base + (g in_gstride + l) N instead of base
    // (an out-of-place transform; in_base is not written)
    const u64 *in_base = nullptr;
    u64 in_gstride = 0;  // in polynomials
};
// Polynomials of mixed ring degree 2^MIXED_LOG_MIN .. 2^17 in one launch per
// pass: group g is npoly limb-polynomials of degree 2^log_n contiguous at
// base, polynomial p using modulus limb0 + p % nlimb; tw / ninv hold each
// degree's twiddles (inverse ones for inverse transforms) and N^-1, by
// log_n - MIXED_LOG_MIN.  block0 is filled in by the launcher.
constexpr int MIXED_LOG_MIN = 12, MIXED_LOG_MAX = 17, MAX_MIXED = 16;
struct MixedGroup {
    u64 *base;
    u64 npoly;
    u64 block0;
    int nlimb, limb0, log_n;
};
struct MixedArgs {
    MixedGroup g[MAX_MIXED];
    int ng;
    const double *tw[MIXED_LOG_MAX - MIXED_LOG_MIN + 1];
    const u64 *ninv[MIXED_LOG_MAX - MIXED_LOG_MIN + 1];
};
int launch_ntt_mixed(Ctx *c, const MixedArgs &ma, bool inverse, hipStream_t s);
// Twiddle tables of ring degree 2^log_n for the mixed launches (below the
// context's degree: built on first use, synchronous upload).
int degree_tables(Ctx *c, int log_n, DegreeTables *out);
int launch_ntt_fwd(Ctx *c, const PolyBatch &b, hipStream_t s);
int launch_ntt_inv(Ctx *c, const PolyBatch &b, hipStream_t s);

// elementwise (ops.hip)
int launch_add_sub(Ctx *c, const u64 *a, const u64 *b, u64 *out, u64 count, int ncomp, int sub, hipStream_t s);
int launch_tensor(Ctx *c, const u64 *a, const u64 *b, u64 *out3, u64 count, hipStream_t s);  // b NULL: square
int launch_mul_plain(Ctx *c, const u64 *ct, const u64 *pt, u64 *out, u64 count, hipStream_t s);
int launch_masked_sum(Ctx *c, const u64 *cts, int n, int len, const u64 *masks, u64 *out, hipStream_t s);
// trip[k] = sum_i cts[i][k] (x) masks[i] for k < len; client i's row starts
// at cts + i row_len 2 S (row_len >= len packed ciphertexts)
int launch_mask_mul_acc(Ctx *c, const u64 *cts, int n, int len, int row_len, const u64 *masks, u64 *trip,
                        hipStream_t s);
int pair_gram_positions(Ctx *c, int n, int want);
int launch_pair_gram(Ctx *c, int pm, const u64 *cts, int n, int len, u64 *d01, u64 d01_stride, u64 *d2,
                     u64 d2_stride, int accumulate, hipStream_t s);
int launch_pair_triples(Ctx *c, const u64 *cts, int n, int len, u64 *d01, u64 d01_stride, u64 *d2, u64 d2_stride,
                        int accumulate, hipStream_t s);
// out[i] = sum over j != i of in[pair (i, j)], ncomp components per object,
// in_stride words between pairs; out [n][ncomp][nq][N]
int launch_sumdis(Ctx *c, const u64 *dist, u64 in_stride, int n, int ncomp, u64 *sumdis, hipStream_t s);
int launch_copy(Ctx *c, const u64 *src, u64 *dst, u64 words, hipStream_t s);

// keys / rng (rng.hip)
int launch_sample_ternary(Ctx *c, u64 seed, u64 domain, u64 object, i64 *out, hipStream_t s);
int launch_signed_to_limbs(Ctx *c, const i64 *in, u64 *out, int nlimb, u64 count, hipStream_t s);
int launch_uniform_limbs(Ctx *c, u64 seed, u64 domain, u64 obj_base, u64 *out, int nlimb, hipStream_t s);
int launch_gaussian(Ctx *c, u64 seed, u64 domain, u64 object, i64 *out, hipStream_t s);
int launch_keycombine(Ctx *c, const u64 *a, const u64 *e, const u64 *s_ntt, const u64 *t_ntt, const u64 *gadget,
                      u64 *k0, u64 *k1, int nlimb, hipStream_t s);
int launch_pointwise_sq(Ctx *c, const u64 *a, u64 *out, int nlimb, hipStream_t s);
int launch_permute(Ctx *c, const u64 *in, u64 *out, const u32 *perm, u64 npoly, hipStream_t s);
int launch_enc_sample(Ctx *c, const i64 *m, u64 count, u64 seed, u64 first_object, u64 *tmp, hipStream_t s);
int launch_enc_combine(Ctx *c, const u64 *tmp, u64 count, u64 *ct, hipStream_t s);
int launch_dec_combine(Ctx *c, const u64 *ct, int ncomp, int nlimb, u64 count, u64 *out, hipStream_t s);

// key switching (keyswitch.hip)
// One output of a hoisted key switch: the key products of all keys in the
// group are summed in PQ before a single ModDown.
struct KsGroup {
    const u64 *keys[8];
    const u32 *perms[8];  // NULL = identity
    int n;
    const CycleTable *cyc;  // optional: keys t = 1..n are the powers phi^t of one automorphism with this walk
    const u64 *base;      // optional [2][nq][N] added to the output (stride per ct)
    u64 base_stride;
    const u64 *c0src;     // optional: sum_t phi_t(c0src) added to component 0
    u64 c0_stride;
    u64 *out;
    u64 out_stride;
};
// Raises each x (stride x_stride, nq limbs, NTT domain) once and evaluates
// every group on it.
int keyswitch_hoisted(Ctx *c, const u64 *x, u64 x_stride, u64 count, const KsGroup *groups, int ngroups,
                      hipStream_t s);
// The same with caller-provided scratch of ws_words words (at least
// ks_words_per_ct); batches are sized to fit it.  Allocates nothing.
int keyswitch_hoisted_ws(Ctx *c, const u64 *x, u64 x_stride, u64 count, const KsGroup *groups, int ngroups,
                         u64 *ws, u64 ws_words, hipStream_t s);
u64 ks_words_per_ct(const Ctx *c);
// Builds (once, at key set-up: it copies to the device synchronously) the
// tile-cycle walk of Galois element g.
int build_cycle_table(Ctx *c, u64 g);
// Literal hoisted rotations of count ciphertexts (ct, [count][2][nq][N])
// through the source-major inner product; needs the fused key-switch path
// and tile tables for every key.
int keyswitch_rotations(Ctx *c, const u64 *ct, u64 count, const u64 *const *keys, const u32 *const *perms,
                        const u32 *const *inv, int nsteps, u64 *out, u64 out_stride, hipStream_t s);

}  // namespace lc
