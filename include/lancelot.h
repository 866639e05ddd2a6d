/*
 * lancelot.h -- C ABI of the MI355X (gfx950) engine for Lancelot's encrypted
 * pairwise squared distances (arXiv 2408.06197): RNS-CKKS over
 * Z_Q[X]/(X^N + 1) with hand-written HIP kernels.
 *
 * Conventions shared by every call
 * --------------------------------
 * Moduli.  A context holds the chain q_0..q_L (n_q = L+1 limbs) and the
 *   special primes p_0..p_{K-1} (n_p = K) of hybrid key switching.  Digit
 *   size alpha = K, dnum = ceil((L+1)/alpha).  Every modulus has at most 50
 *   bits.  Prime rule: for each requested bit size b, in order, the largest
 *   b-bit prime k*2^log_m + 1 not already chosen.
 * Layouts.  Device buffers of uint64 residues in [0, q_l), limb-major:
 *   plaintext [n_q][N], ciphertext [2][n_q][N], triple [3][n_q][N].  A batch
 *   of `count` objects is contiguous: [count][comp][n_q][N].  Ciphertexts and
 *   triples are in the NTT domain: entry i of a limb is the value at
 *   psi^(2 brev(i) + 1), psi the smallest primitive 2N-th root mod q_l.
 * Ownership.  The caller allocates and frees every buffer it passes; a
 *   pointer argument named *_dev is device memory on the context's device,
 *   *_host is host memory.  The library owns its parameter tables, resident
 *   keys and a workspace per stream that it grows on demand (hipMalloc);
 *   an outgrown workspace buffer is kept until lc_ctx_destroy, so work
 *   captured into a HIP graph earlier keeps valid memory.
 * Streams.  `stream` is a hipStream_t (NULL: the default stream).  Device
 *   calls are asynchronous on it; lc_sync waits and reports asynchronous
 *   errors.  Calls on one context must come from one host thread at a time.
 *   Once a stream's workspace has grown to a call's size, that call on that
 *   stream allocates, copies and synchronizes nothing (it can be captured
 *   into a HIP graph; replays share the stream's workspace).
 * Errors.  Every call returns LC_OK (0) or a negative code; lc_last_error
 *   gives text.  Nothing is written to outputs when a call returns an error
 *   before launching work.
 * Roles.  A LC_ROLE_KGC context may hold the secret key; a LC_ROLE_SERVER
 *   context holds only public and evaluation keys (the server of the threat
 *   model is semi-honest, Methods, Threat Model).  Decryption and key
 *   generation need LC_ROLE_KGC (else LC_EKEY).
 */
#ifndef LANCELOT_H
#define LANCELOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LC_OK 0
#define LC_EINVAL (-1)  /* bad argument: shape, size, level, plan        */
#define LC_ENOMEM (-2)  /* device allocation failed                       */
#define LC_EKEY (-3)    /* missing key, or secret-key use in server role  */
#define LC_EHIP (-4)    /* HIP runtime error                              */
#define LC_EUNSUP (-5)  /* parameters outside what the kernels support    */

#define LC_ROLE_SERVER 0
#define LC_ROLE_KGC 1

typedef struct lc_ctx lc_ctx;

/* Parameter set (Methods, CKKS Scheme Description: N, Q = prod q_i, special
 * modulus p; hybrid decomposition of Dynamic Hoisting).  log_n in [3, 17];
 * 1 <= n_q <= 48, 1 <= n_p <= 8; bit sizes in [20, 50]; log_m = 0 means
 * log_n + 1, otherwise log_m >= log_n + 1. */
typedef struct lc_params {
    int log_n;
    int n_q;
    int n_p;
    const int *q_bits;
    const int *p_bits;
    int log_m;
} lc_params;

/* ---- context ------------------------------------------------------------ */

/* Builds primes, NTT twiddles and base-conversion tables on `device`.
 * device = -1 makes a host-only context: primes, encode/decode, CRT and the
 * Gaussian table work; every device call returns LC_EUNSUP. */
int lc_ctx_create(const lc_params *prm, int device, int role, lc_ctx **out);
int lc_ctx_destroy(lc_ctx *ctx);
const char *lc_last_error(const lc_ctx *ctx);
/* Copies the n_q + n_p moduli (q's then p's) to host memory. */
int lc_ctx_moduli(const lc_ctx *ctx, uint64_t *moduli_host);
/* Any pointer may be NULL. */
int lc_ctx_info(const lc_ctx *ctx, int *log_n, int *n_q, int *n_p, int *dnum);
int lc_sync(lc_ctx *ctx, void *stream);
/* Waits for the device and frees every workspace of the context (outgrown
 * ones included); later calls grow them again.  HIP graphs captured before
 * must not be replayed afterwards. */
int lc_release_workspace(lc_ctx *ctx);
/* Bytes of library-owned device memory (tables, keys, workspace). */
int lc_ctx_device_bytes(const lc_ctx *ctx, size_t *bytes);

/* ---- keys (KGC role) ----------------------------------------------------- */

/* Secret s (ternary), public key pk = ([-a s + e]_Q, a) and the
 * relinearization key for s^2 (CKKS Scheme Description, key generation, in
 * the hybrid dnum-digit form).  Draws come from Philox4x64-10 keyed
 * (seed, 0): word w of (domain, object) is lane w % 4 of the block at counter
 * (w / 4, object, domain, 0).  Domains: 1 secret, 2 pk.a (object = limb),
 * 3 pk.e, 4/5/6 encryption r/e0/e1 (object = plaintext id), 7 key a (object =
 * key_id << 32 | digit << 16 | limb), 8 key e (object = key_id << 32 | digit);
 * key_id is 0 for the relinearization key and the Galois element of a
 * rotation key.  Ternary = word mod 3 - 1; Gaussian = smallest t in
 * [-19, 19] with word < T[t] (sigma 3.2 cumulative table); uniform mod q =
 * (word[2c] * 2^64 + word[2c+1]) mod q.  Synchronous. */
int lc_keygen(lc_ctx *ctx, uint64_t seed);
/* Rotation keys for slot rotations by steps[t] (Galois element 5^step). */
int lc_keygen_rotation(lc_ctx *ctx, uint64_t seed, const int *steps, int nsteps);
/* Copies pk, relin and rotation keys (never the secret) into `dst`, which
 * must have identical parameters and device. */
int lc_keys_share(const lc_ctx *src, lc_ctx *dst);
/* Secret coefficients in {-1, 0, 1} to host int64[N] (KGC role only). */
int lc_secret_export(const lc_ctx *ctx, int64_t *s_host);
/* Public key [2][n_q][N] to host. */
int lc_pk_export(const lc_ctx *ctx, uint64_t *pk_host);
/* Key-switching key [dnum][2][n_q+n_p][N] to host: which = 0 relin key,
 * which = 1 rotation key for `step`. */
int lc_ksk_export(const lc_ctx *ctx, int which, int step, uint64_t *ksk_host);

/* Imports a key made outside the library, for instance by an independent
 * implementation from the same secret, so that every server operation can be
 * checked without relying on lc_keygen (CKKS Scheme Description, key
 * generation; Methods, Dynamic Hoisting for the digit form).  kind:
 *   LC_KEY_PK        host_blob = pk [2][n_q][N];
 *   LC_KEY_RELIN     host_blob = relinearization key [dnum][2][n_q + n_p][N];
 *   LC_KEY_ROTATION  host_blob = key of slot rotation `step` (Galois element
 *                    5^step mod 2N), same layout as the relinearization key.
 * NTT domain, residues canonical (checked on the host: LC_EINVAL).  Any role;
 * a key already present is replaced (the device is synchronized first).
 * `step` is ignored unless kind is LC_KEY_ROTATION.  Synchronous; the caller
 * keeps ownership of host_blob. */
#define LC_KEY_PK 0
#define LC_KEY_RELIN 1
#define LC_KEY_ROTATION 2
int lc_key_import(lc_ctx *ctx, int kind, int step, const uint64_t *host_blob);

/* ---- encode / decode (host, FP64; Methods, Batch Encoding and Decoding) -- */

/* m = round(scale * sigma^-1(pi^-1(z))), z real (z_im NULL) or complex with
 * nslots <= N/2 slots (missing slots are zero).  m_host: int64[N]. */
int lc_encode(const lc_ctx *ctx, const double *z_re, const double *z_im, size_t nslots, double scale,
              int64_t *m_host);
/* Device encode of `count` real vectors (the f3 ingest path): z_dev is
 * double[count][z_stride] on the device, of which the first nslots <= N/2
 * values of each vector are the slots (the rest are zero); m_dev int64[count][N]
 * receives round(scale * sigma^-1(pi^-1(z))) exactly as lc_encode computes it,
 * in FP64 on the device (a coefficient within rounding error of a
 * half-integer may differ by one from lc_encode).  Asynchronous on `stream`.
 * The first call on a context uploads its transform tables (synchronous).
 * Scratch: the stream's workspace (up to 256 MiB).  Errors: LC_EINVAL for
 * nslots > N/2, z_stride < nslots, null buffers or scale <= 0. */
int lc_encode_device(lc_ctx *ctx, const double *z_dev, size_t count, size_t nslots, size_t z_stride, double scale,
                     int64_t *m_dev, void *stream);
/* Decode a coefficient-domain plaintext given as residues [n_q][N] (host):
 * exact CRT to centred integers, then z = pi(sigma(m)) / scale. */
int lc_decode(const lc_ctx *ctx, const uint64_t *res_host, double scale, double *z_re, double *z_im);
/* lc_decode for a plaintext at a lower level: residues [nlimb][N] of the
 * first nlimb Q limbs (1 <= nlimb <= n_q). */
int lc_decode_level(const lc_ctx *ctx, const uint64_t *res_host, int nlimb, double scale, double *z_re,
                    double *z_im);
/* Exact CRT of `ncoeff` coefficients: res_host is [n_q][stride], coefficient
 * t of limb l at res_host[l * stride + t]; out[t] = centred value as double. */
int lc_crt_to_double(const lc_ctx *ctx, const uint64_t *res_host, size_t ncoeff, size_t stride, double *out);
/* The 38 thresholds of the sigma = 3.2 error sampler (entry k belongs to
 * t = k - 19) to host memory. */
int lc_gaussian_table(const lc_ctx *ctx, uint64_t *out38);

/* ---- encryption / decryption ---------------------------------------------- */

/* ct = ([m + r u0 + e0]_Q, [r u1 + e1]_Q) (CKKS Scheme Description,
 * encryption) for `count` plaintexts m_dev int64[count][N] (coefficients,
 * |m| < 2^62).  r ternary, e Gaussian sigma 3.2; plaintext t draws from PRNG
 * object first_object + t.  ct_dev [count][2][n_q][N]. */
int lc_encrypt(lc_ctx *ctx, const int64_t *m_dev, size_t count, uint64_t seed, uint64_t first_object,
               uint64_t *ct_dev, void *stream);
/* [c0 + c1 s (+ c2 s^2)]_Q in the coefficient domain (CKKS Scheme
 * Description, decryption; ncomp 3 reads a triple).  in [count][ncomp][n_q][N],
 * out [count][n_q][N].  KGC role. */
int lc_decrypt(lc_ctx *ctx, const uint64_t *ct_dev, int ncomp, size_t count, uint64_t *pt_dev, void *stream);
/* lc_decrypt of ciphertexts at a lower level: their first nlimb Q limbs
 * (1 <= nlimb <= n_q; in [count][ncomp][nlimb][N], out [count][nlimb][N]). */
int lc_decrypt_level(lc_ctx *ctx, const uint64_t *ct_dev, int ncomp, int nlimb, size_t count, uint64_t *pt_dev,
                     void *stream);
/* CKKS rescaling (levels Q_l of the CKKS Scheme Description; the paper uses
 * the standard operation without spelling it out): for ciphertexts with nlimb
 * Q limbs q_0 .. q_t (t = nlimb - 1, 2 <= nlimb <= n_q), every coefficient c
 * of every component becomes the nearest integer to c / q_t modulo
 * q_0 .. q_{t-1}; the scale drops by the factor q_t.  in [count][ncomp][nlimb][N]
 * and out [count][ncomp][nlimb - 1][N], NTT domain, ncomp 1..3; out must not
 * overlap in (LC_EINVAL).  Scratch: the stream's workspace (up to ~1 GiB). */
int lc_rescale(lc_ctx *ctx, const uint64_t *ct_dev, size_t count, int ncomp, int nlimb, uint64_t *out_dev,
               void *stream);

/* ---- homomorphic operations (CKKS Scheme Description, evaluation; Methods,
 * Private Distance Evaluation) --------------------------------------------- */

/* out = a -/+ b limb-wise for count ciphertexts of ncomp components.  out
 * may be a or b itself (in place); any other overlap gives LC_EINVAL. */
int lc_ct_sub(lc_ctx *ctx, const uint64_t *a_dev, const uint64_t *b_dev, uint64_t *out_dev, size_t count,
              int ncomp, void *stream);
int lc_ct_add(lc_ctx *ctx, const uint64_t *a_dev, const uint64_t *b_dev, uint64_t *out_dev, size_t count,
              int ncomp, void *stream);
/* Triple (a0 b0, a0 b1 + a1 b0, a1 b1) without relinearization; out3
 * [count][3][n_q][N] must not overlap a or b (LC_EINVAL). */
int lc_ct_mul(lc_ctx *ctx, const uint64_t *a_dev, const uint64_t *b_dev, uint64_t *out3_dev, size_t count,
              void *stream);
/* Triple (a0^2, 2 a0 a1, a1^2); out3 must not overlap a (LC_EINVAL). */
int lc_ct_square(lc_ctx *ctx, const uint64_t *a_dev, uint64_t *out3_dev, size_t count, void *stream);
/* Relinearization of triples with the s^2 key: out = (d0 + KS0(d2),
 * d1 + KS1(d2)), hybrid key switching (Methods, Lazy Relinearization and
 * Dynamic Hoisting).  in [count][3][n_q][N], out [count][2][n_q][N]; out must
 * not overlap in (LC_EINVAL). */
int lc_relin(lc_ctx *ctx, const uint64_t *ct3_dev, uint64_t *ct2_dev, size_t count, void *stream);
/* lc_relin for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments and bits as lc_relin, but the key-switching scratch is a fixed
 * device array of LC_NOALLOC_SCRATCH_MIB MiB that every GPU the library runs
 * on holds from module load until the process ends; the call allocates
 * nothing and runs in batches of as many ciphertexts as fit it.  LC_EINVAL
 * when one ciphertext's scratch, (n_q + dnum (n_q + n_p) + 2 (n_q + n_p)
 * + 2 n_q) N words (N = 2^16 with 24 + 4 limbs: 155 MB), exceeds the array.
 * Every call on one GPU (any context, any stream) shares the array and keeps
 * the last call's contents: calls that overlap on a GPU race, so the caller
 * serializes them.  No word of it needs to start at zero. */
#define LC_NOALLOC_SCRATCH_MIB 256
int lc_relin_noalloc(lc_ctx *ctx, const uint64_t *ct3_dev, uint64_t *ct2_dev, size_t count, void *stream);
/* Hoisted rotations (Methods, Dynamic Hoisting): one decomposition/ModUp of
 * c1 shared by all steps, then per step the automorphism on the raised
 * digits, the key inner product and ModDown.  outs [count][nsteps][2][n_q][N],
 * not overlapping ct; 1 <= nsteps <= 64; a missing key gives LC_EKEY.  With
 * "hoist_multi" (default) the stream's key-switch workspace holds the
 * accumulators of up to 8 steps per ciphertext of a batch, and batches are
 * sized to at most 12 GiB (or the workspace limit):
 * (n_q + dnum (n_q + n_p) + 2 min(nsteps, 8) (n_q + n_p) + 2 n_q) N words
 * per ciphertext. */
int lc_rotate_hoisted(lc_ctx *ctx, const uint64_t *ct_dev, size_t count, const int *steps, int nsteps,
                      uint64_t *outs_dev, void *stream);
/* Rotate-and-sum in place (Methods, Dynamic Hoisting): after it every slot
 * holds the sum of all N/2 slots.  plan[b] = levels of block b (sum =
 * log_n - 1); block b starting at level j0 adds rot_{t 2^j0} for t = 1 ..
 * 2^plan[b] - 1 with one ModUp and one ModDown.  plan NULL = all ones. */
int lc_rotate_sum(lc_ctx *ctx, uint64_t *ct_dev, size_t count, const int *plan, int nblocks, void *stream);
/* out = ct * pt per component, pt [n_q][N] NTT domain, one pt per ct.  out
 * may be ct itself; any other overlap with ct or pt gives LC_EINVAL. */
int lc_mul_plain(lc_ctx *ctx, const uint64_t *ct_dev, const uint64_t *pt_dev, uint64_t *out_dev, size_t count,
                 void *stream);
/* ServerUpdate (Algorithm 1): out[k] = sum_i ct_i[k] * mask_i, client_cts
 * [n][len][2][n_q][N], masks [n][n_q][N] (NTT domain), out [len][2][n_q][N]
 * (must not overlap the inputs: LC_EINVAL). */
int lc_masked_sum(lc_ctx *ctx, const uint64_t *client_cts_dev, int n, int len, const uint64_t *masks_dev,
                  uint64_t *out_dev, void *stream);

/* ---- the pairwise-distance pipeline (Algorithm 1, Server Executes) ------- */

/* Lazy triples only: for pairs i < j in row-major order, sum over k < len of
 * (ct_i[k] - ct_j[k])^2 as triples.  triples [P][3][n_q][N], P = n(n-1)/2,
 * 2 <= n <= 64; triples must not overlap the client ciphertexts (LC_EINVAL). */
int lc_pair_triples(lc_ctx *ctx, const uint64_t *client_cts_dev, int n, int len, uint64_t *triples_dev,
                    void *stream);
/* Same, adding into triples (which must hold canonical residues): lets a
 * round stream its packed ciphertexts in chunks of k (Methods, Lazy
 * Relinearization: triples of all k are summed before one relinearization). */
int lc_pair_triples_acc(lc_ctx *ctx, const uint64_t *client_cts_dev, int n, int len, uint64_t *triples_dev,
                        void *stream);
/* The rest of the pipeline on accumulated triples [P][3][n_q][N]: one
 * relinearization per pair, rotate-and-sum with `plan`, SumDis (may be NULL).
 * dist [P][2][n_q][N] must not overlap the triples. */
int lc_pairwise_finish(lc_ctx *ctx, const uint64_t *triples_dev, int n, const int *plan, int nblocks,
                       uint64_t *dist_dev, uint64_t *sumdis_dev, void *stream);
/* Full batched pipeline: lazy triples, one relinearization per pair,
 * rotate-and-sum with `plan`; dist [P][2][n_q][N].  sumdis (may be NULL)
 * [n][2][n_q][N] gets sum over j != i of Dis[i][j]. */
int lc_pairwise_sqdist(lc_ctx *ctx, const uint64_t *client_cts_dev, int n, int len, const int *plan, int nblocks,
                       uint64_t *dist_dev, uint64_t *sumdis_dev, void *stream);

/* SumDis with one relinearization and one rotate-and-sum per client instead
 * of per pair (Algorithm 1, the SumDis line; Methods, Lazy Relinearization:
 * all squared-difference triples are summed before the single
 * relinearization): sumdis[i] = RotSum(Relin(sum_{j != i} sum_{k < len}
 * (ct_i[k] - ct_j[k])^2)).  It decrypts to the same value as the SumDis of
 * lc_pairwise_sqdist (within the key-switching noise) with n instead of
 * n(n-1)/2 key-switching chains.  client_cts [n][len][2][n_q][N],
 * sumdis [n][2][n_q][N] (must not overlap the input); 2 <= n <= 64; plan as
 * for lc_rotate_sum.  Scratch: the stream's workspace ((P + n) triples plus
 * the key-switch batch). */
int lc_sumdis_lazy(lc_ctx *ctx, const uint64_t *client_cts_dev, int n, int len, const int *plan, int nblocks,
                   uint64_t *sumdis_dev, void *stream);

/* ServerUpdate with an encrypted mask (Algorithm 1, ServerUpdate; Methods,
 * Masked-based Encrypted Sorting): out[k] = relin(sum_i ct_i[k] (x) M_i),
 * the client ciphertexts [n][len][2][n_q][N] times each client's mask
 * ciphertext M_i = Enc_pk(weight_i) ([n][2][n_q][N], NTT domain), summed
 * over clients before one relinearization per packed ciphertext (lazy).
 * out [len][2][n_q][N] must not overlap the inputs (LC_EINVAL); needs the
 * relinearization key (LC_EKEY).  The result is at the product of the two
 * scales. */
int lc_mask_aggregate(lc_ctx *ctx, const uint64_t *client_cts_dev, int n, int len, const uint64_t *mask_cts_dev,
                      uint64_t *out_dev, void *stream);

/* ---- transforms ------------------------------------------------------------ */

/* In-place negacyclic NTT / inverse NTT of count polynomials of nlimb limbs
 * each ([count][nlimb][N]); limb l of each uses modulus limb0 + l of the
 * extended basis (q's then p's). */
int lc_ntt_fwd(lc_ctx *ctx, uint64_t *polys_dev, size_t count, int nlimb, int limb0, void *stream);
int lc_ntt_inv(lc_ctx *ctx, uint64_t *polys_dev, size_t count, int nlimb, int limb0, void *stream);

/* A group of limb-polynomials for the mixed-degree transforms: count
 * polynomials of nlimb limbs of ring degree 2^log_n each, [count][nlimb][2^log_n]
 * contiguous at data (device memory); limb l of each uses modulus limb0 + l
 * of the extended basis. */
typedef struct lc_poly_group {
    uint64_t *data;
    size_t count;
    int log_n;
    int nlimb;
    int limb0;
} lc_poly_group;
/* In-place forward / inverse negacyclic NTTs of polynomials of mixed ring
 * degree, all groups in one launch per pass (two passes per direction;
 * Appendix, Descriptions of Hardware Acceleration: the batched NTT).  A
 * degree-2^k polynomial is transformed with psi_k, the smallest primitive
 * 2^(k+1)-th root of unity of its modulus, so its result equals lc_ntt_fwd /
 * lc_ntt_inv of a context of degree 2^k with the same moduli.  Needs
 * 12 <= log_n <= min(17, the context's log_n) (LC_EUNSUP) and 1 <= ngroups
 * <= 16 (LC_EINVAL); every modulus of the context is = 1 mod 2N, hence also
 * mod 2^(k+1).  The first call with a degree below the context's uploads that
 * degree's twiddle tables (synchronous). */
int lc_ntt_fwd_groups(lc_ctx *ctx, const lc_poly_group *groups, int ngroups, void *stream);
int lc_ntt_inv_groups(lc_ctx *ctx, const lc_poly_group *groups, int ngroups, void *stream);

/* ---- memory planning ------------------------------------------------------- */

/* Workspace bytes that lc_pairwise_sqdist needs for n clients. */
int lc_workspace_query(const lc_ctx *ctx, int n, int len, size_t *bytes);
/* HBM footprint of one pairwise-distance round of n clients x len packed
 * ciphertexts (Methods, Dynamic Hoisting, on the memory a batch needs), for
 * admission control.  k_chunk = 0: the client ciphertexts are resident and
 * the round runs lc_pairwise_sqdist; 0 < k_chunk < len: they arrive in chunks
 * of k_chunk that lc_pair_triples_acc folds into a triple buffer, then
 * lc_pairwise_finish.  *round_bytes (may be NULL): the buffers the caller
 * holds for the round -- client ciphertexts (all, or one chunk), distance
 * ciphertexts, the triple buffer when streamed, and with flags
 * LC_FP_SUMDIS the SumDis ciphertexts, LC_FP_PLAINTEXTS one chunk of int64
 * plaintexts to encrypt, LC_FP_DECRYPT the decrypted distances [P][n_q][N].
 * *workspace_bytes (may be NULL): the library workspace those calls grow on
 * the round's stream and its second stream (kept by them afterwards).  LC_EINVAL for n < 2
 * or len < 1. */
#define LC_FP_SUMDIS 1
#define LC_FP_PLAINTEXTS 2
#define LC_FP_DECRYPT 4
int lc_footprint(const lc_ctx *ctx, int n, int len, int k_chunk, int flags, size_t *round_bytes,
                 size_t *workspace_bytes);
/* Caps the workspace the library may hold (0 = no cap); calls that would
 * need more run in smaller batches, or fail with LC_ENOMEM. */
int lc_set_workspace_limit(lc_ctx *ctx, size_t bytes);

/* Launch-shape tuning, results unchanged (every shape computes the same
 * residues): "pair_lanes" (8/16/32/64 coefficients per workgroup of the pair
 * kernel), "pair_ppt" (1/3/4/6 pairs per lane), "pair_mfma" (0 = per-pair
 * kernel; 4 or 2 = for n <= 24 clients the triples are read off exact
 * modular Gram products of the 2n (client, component) rows on the int8
 * matrix cores, 4 or 2 coefficients per workgroup), "ks_chunk" (1..256
 * ciphertexts per key-switch batch), "ntt_sub_kb" (0..4194304: two-pass NTTs
 * run both passes per sub-batch of about this many KiB; 0 = whole batch),
 * "mac_cts" (8/16 ciphertexts per lane of the key-switch inner product),
 * "mac_cycle" (1 = hoisted blocks of 3 or 7 rotations use the cycle-walking
 * inner product that reads each raised digit once; 0 = one gather per key),
 * "mac_cycle_min" (>= 1: shortest tile cycle for which the walk is used),
 * "mac_cycle_cts" (8/16 ciphertexts per walking workgroup), "mac_short_cts"
 * (8/16 ciphertexts per short-cycle workgroup), "mac_cycle_c0"
 * (1 = the inner product, walk or per-key gather, also adds the group's
 * permuted c0 terms, so that ModDown's last transform pass does the whole
 * combine; 0 = a combine kernel adds them),
 * "mac_cycle_short" (1 = blocks whose tile cycles are at most 2 tiles long,
 * such as rotations that keep every tile in place, stage each cycle once
 * instead of walking it),
 * "fuse_modup" (1 = for 2^10 <= N the ModUp base conversion runs inside the
 * first forward-NTT pass of the raised digits; 0 = a kernel of its own),
 * "ms_shape" (masked-sum lanes: 0 = 1 coefficient x 16 rows, 1 = 2 x 8,
 * 2 = 2 x 16, the default), "ks_streams" (2 = the relinearization / rotate-and-sum
 * batches of lc_pairwise_sqdist and lc_pairwise_finish alternate between the
 * caller's stream and a second stream of the library's, made on the first
 * such call on that caller stream, forked after the triples and joined
 * before SumDis, so that batches overlap; 1 = all on the caller's stream),
 * "hoist_multi" (1 = lc_rotate_hoisted from N = 2^10 on stages each
 * source tile of the raised digits once for up to 8 keys; 0 = one gather per
 * key), "mac_xcd" (1 = the walking and short-cycle inner-product workgroups that
 * read the same key tiles for different ciphertexts are dispatched to one
 * XCD back to back, so the keys come from that XCD's L2 after the first
 * read; 0 = plain grid order).
 * LC_EINVAL for unknown names/values. */
int lc_set_tuning(lc_ctx *ctx, const char *name, int value);

#ifdef __cplusplus
}
#endif
#endif
