// Hybrid key switching (Methods, Dynamic Hoisting: RNS decompose, ModUp,
// switch key, ModDown), batched over ciphertexts and hoisted over keys.
//
// For each input x (NTT domain, n_q limbs):
//   1. x^ = iNTT(x);
//   2. digit d (limbs D_d, alpha of them): for every limb l outside D_d,
//      X_d[l] = sum_{a in D_d} [x^_a (Q_d/q_a)^-1]_{q_a} (Q_d/q_a) mod m_l
//      (fast base conversion, no overflow correction); NTT of those limbs.
//      Limbs inside D_d reuse x itself;
//   3. acc_k = sum_t sum_d phi_t(X_d) * key_{t,d,k} over the n_q + n_p limbs,
//      phi_t a permutation in the NTT domain (identity for relinearization);
//      one raise serves every key t: hoisting;
//   4. ModDown: (acc_Q - BConv_{P->Q}(iNTT(acc_P)))^ * P^-1 mod q_l;
//   5. out0 = base0 + sum_t phi_t(c0src) + ModDown(acc_0), out1 = base1 +
//      ModDown(acc_1).
#include <numeric>

#include "lc_internal.h"

namespace lc {

constexpr int KS_THREADS = 256;

static inline u32 blocks_for(u64 n) { return (u32)((n + KS_THREADS - 1) / KS_THREADS); }

// count blocks of `words` from src (stride sstride) to dst (stride dstride)
__global__ void __launch_bounds__(KS_THREADS)
strided_copy_kernel(const u64 *src, u64 sstride, u64 *dst, u64 dstride, u64 words, u64 count)
{
    u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= words * count) return;
    u64 b = e / words, r = e % words;
    dst[b * dstride + r] = src[b * sstride + r];
}

// raised[b][d][l][j] for l outside digit d, coefficient domain.
//
// FP64 Barrett form: y_a = [x^_a (Q_d/q_a)^-1]_{q_a} is taken to its
// canonical representative (the conversion is defined on it), then each
// product y_a (Q_d/q_a mod m_l) < q_a m_l comes back with |r| <= 0.875 m_l;
// at most MAX_NP of them are summed before the canonical read-out.
__global__ void __launch_bounds__(KS_THREADS)
modup_bconv_kernel(DevParams dp, const u64 *xhat, u64 *raised)
{
    // grid (N / blockDim.x, count * dnum): the digit and ciphertext are
    // uniform over the workgroup, so the conversion constants are scalar loads
    const u64 j = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    const int d = (int)(blockIdx.y % (u32)dp.dnum);
    const u64 b = blockIdx.y / (u32)dp.dnum;
    const int a0 = d * dp.alpha, na = min(dp.alpha, dp.nq - a0);
    double y[MAX_NP];
    for (int a = 0; a < na; a++) {
        const ModConst &mc = dp.mc[a0 + a];
        double v = u64_to_d(xhat[(b * dp.nq + a0 + a) * dp.N + j]);
        y[a] = canon_d(mulmod_d(v, dp.up_inv_d[d * dp.alpha + a], mc.qd, mc.qinv), mc.qd, mc.qinv);
    }
    u64 *out = raised + (b * dp.dnum + d) * (u64)dp.ne * dp.N + j;
    const double *fac = dp.up_fac_d + (u64)d * dp.alpha * dp.ne;
    for (int l = 0; l < dp.ne; l++) {
        if (l >= a0 && l < a0 + na) continue;
        const double q = dp.mc[l].qd, qinv = dp.mc[l].qinv;
        double s = 0.0;
        for (int a = 0; a < na; a++) s += mulmod_d(y[a], fac[(u64)a * dp.ne + l], q, qinv);
        out[(u64)l * dp.N] = d_to_canonical(s, q, qinv);
    }
}

struct KeySet {
    const u64 *key[8];
    const u32 *perm[8];  // NULL = identity
    int n;
};

// ks.key[r] / ks.perm[r] for a per-lane r < R go through LDS: indexing the
// argument struct with a lane value would load the pointer from memory and
// stall the wave on every load in flight.  One lane copies them (scalar
// reads of the arguments); a barrier must follow before they are read.
typedef const u64 __attribute__((address_space(1))) gu64;  // global memory: loads are not flat
typedef const u32 __attribute__((address_space(1))) gu32;

template <int R>
__device__ __forceinline__ void stage_key_ptrs(const KeySet &ks, const u64 **kp, const u32 **pp)
{
    if (threadIdx.x == 0 && threadIdx.y == 0) {
#pragma unroll
        for (int k = 0; k < R; k++) {
            kp[k] = ks.key[k];
            pp[k] = ks.perm[k];
        }
    }
}

// acc[b][k][l][j] = sum_t sum_d X_d[l][perm_t(j)] key_t[d][k][l][j]
//
// A lane owns one coefficient (l, j) of MAC_B ciphertexts: each key value is
// read once and used for all MAC_B of them (the key of a block is read once per
// MAC_B ciphertexts instead of once per ciphertext; MAC_B = 8 or 16 is a
// tuning choice).  Products use the FP64 Barrett form (|x key| reduced to at
// most 0.8125 q); the two accumulators per ciphertext are reduced after every
// 8 products, so they stay below 7 q.
// With FOLD, c0 is given and the Q limbs of accumulator 0 also take
// sum_t phi_t(c0) times P mod q (one more product per key, counted like the
// others): ModDown divides it by P exactly, so the output gets the permuted
// c0 terms without a combine kernel, as in the cycle walk.
template <int MAC_B, bool FOLD>
__global__ void __launch_bounds__(KS_THREADS)
mac_kernel(DevParams dp, const u64 *x, u64 x_stride, const u64 *raised, const u64 *c0, u64 c0_stride, KeySet ks,
           u64 *acc, u64 count)
{
    u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // over ne * N
    u64 b0 = (u64)blockIdx.y * MAC_B;
    if (e >= (u64)dp.ne * dp.N) return;
    int l = (int)(e >> dp.log_n);
    u64 j = e & (dp.N - 1);
    const u64 NE = (u64)dp.ne * dp.N;
    const double q = dp.mc[l].qd, qinv = dp.mc[l].qinv;
    const int nb = (int)min<u64>(MAC_B, count - b0);
    const bool own_limb = l < dp.nq;
    const int own_digit = own_limb ? l / dp.alpha : -1;
    double a0[MAC_B], a1[MAC_B];
#pragma unroll
    for (int b = 0; b < MAC_B; b++) a0[b] = a1[b] = 0.0;
    int since = 0;
    for (int t = 0; t < ks.n; t++) {
        u64 src = ks.perm[t] ? ks.perm[t][j] : j;
        const u64 *key = ks.key[t];
        for (int d = 0; d < dp.dnum; d++) {
            // all MAC_B loads issued before any is used (a ragged group
            // re-reads its last ciphertext; those sums are not stored)
            const bool own = d == own_digit;
            const u64 *xb = own ? x + b0 * x_stride + (u64)l * dp.N + src
                                : raised + ((b0 * dp.dnum + d) * dp.ne + l) * (u64)dp.N + src;
            const u64 bstride = own ? x_stride : (u64)dp.dnum * dp.ne * dp.N;
            const u64 kv0 = key[((u64)d * 2) * NE + e], kv1 = key[((u64)d * 2 + 1) * NE + e];
            u64 v[MAC_B];
#pragma unroll
            for (int b = 0; b < MAC_B; b++) v[b] = xb[(u64)min(b, nb - 1) * bstride];
            const double k0 = u64_to_d(kv0), k1 = u64_to_d(kv1);
#pragma unroll
            for (int b = 0; b < MAC_B; b++) {
                const double xv = u64_to_d(v[b]);
                a0[b] += mulmod_d(xv, k0, q, qinv);
                a1[b] += mulmod_d(xv, k1, q, qinv);
            }
            if (++since == 8) {
                since = 0;
#pragma unroll
                for (int b = 0; b < MAC_B; b++) {
                    a0[b] = reduce_d(a0[b], q, qinv);
                    a1[b] = reduce_d(a1[b], q, qinv);
                }
            }
        }
        if (FOLD && own_limb) {
            const double pq = u64_to_d(dp.pmod[l]);
            const u64 *cb = c0 + b0 * c0_stride + (u64)l * dp.N + src;
            u64 v[MAC_B];
#pragma unroll
            for (int b = 0; b < MAC_B; b++) v[b] = cb[(u64)min(b, nb - 1) * c0_stride];
#pragma unroll
            for (int b = 0; b < MAC_B; b++) a0[b] += mulmod_d(u64_to_d(v[b]), pq, q, qinv);
            if (++since == 8) {
                since = 0;
#pragma unroll
                for (int b = 0; b < MAC_B; b++) {
                    a0[b] = reduce_d(a0[b], q, qinv);
                    a1[b] = reduce_d(a1[b], q, qinv);
                }
            }
        }
    }
#pragma unroll
    for (int b = 0; b < MAC_B; b++) {
        if (b >= nb) break;
        u64 bb = b0 + b;
        acc[(bb * 2) * NE + e] = d_to_canonical(reduce_d(a0[b], q, qinv), q, qinv);
        acc[(bb * 2 + 1) * NE + e] = d_to_canonical(reduce_d(a1[b], q, qinv), q, qinv);
    }
}

// Workgroups are dealt to the 8 XCDs round-robin in dispatch order (x
// fastest).  With remap set (the launch pads gx so that gx * gy is a
// multiple of 8; workgroups with x past the real count return at once), the
// gz workgroups that share (x, y) -- the same key tiles, for different
// ciphertexts -- are made consecutive on one XCD, so all but the first find
// the keys in its L2.
__device__ __forceinline__ void mac_block_ids(int remap, u32 &bx, u32 &by, u32 &bz)
{
    bx = blockIdx.x;
    by = blockIdx.y;
    bz = blockIdx.z;
    if (!remap) return;
    const u32 gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
    const u32 lin = bx + gx * (by + gy * bz);
    const u32 j = lin >> 3, xy = (j / gz) * 8 + (lin & 7);
    bz = j % gz;
    bx = xy % gx;
    by = xy / gx;
}

// ---- cycle-walking inner product for a hoisted block ------------------------
//
// The keys of a rotate-and-sum block are the powers phi^1 .. phi^R of one
// automorphism phi (rotations t 2^j0).  In the NTT domain phi permutes
// coefficients so that every aligned tile of KS_CYC_TILE coefficients lands
// inside one aligned tile; call that tile map tau.  Output tile o of key t
// reads source tile tau^t(o).  Walking a cycle c_0, c_1 = tau(c_0), ... of
// tau, output c_m reads c_{m+1} .. c_{m+R}, so a workgroup that walks the
// cycle needs one new source tile per step: it stages source tile c_p (all
// digits of 8 or 16 ciphertexts, as doubles) and the keys of the R outputs
// that read it (c_{p-1} with key 1 ... c_{p-R} with key R) in LDS, adds the
// contributions, and writes c_{p-R}, which is then complete.  Accumulators
// live in registers by age.  The raised digits are read about
// (1 + (R - 1) / KS_CYC_SEG) times instead of R times, every key value once
// per 8 or 16 ciphertexts.  Short cycles re-stage the same tiles, which the
// caches serve.  Same FP64 Barrett products as mac_kernel, so the same
// residues.  An accumulator enters a step reduced (|a| <= q/2 + 2) and takes
// at most 8 products of magnitude <= 7q/8 before the next reduction, so it
// stays below 7.5 q + 2 < 2^53 (q < 2^50) and every sum is exact: one
// reduction per key, and one more midway only when a key brings 9 products
// (8 digits and the folded c0).
// With c0 given, the block's sum_t phi_t(c0) rides along: its tiles are the
// same source tiles, so it is staged with the digits and added to the Q
// limbs of accumulator 0 times P mod q (exact after ModDown, which divides
// by P), and the combine kernel skips its per-key gathers of c0.
template <int R, int D, int CB, bool FOLD>
__global__ void __launch_bounds__(KS_CYC_TILE * CB, CB == 8 ? 3 : 1)
mac_cycle_kernel(DevParams dp, const u64 *x, u64 x_stride, const u64 *raised, const u64 *c0, u64 c0_stride,
                 KeySet ks, const CycleSeg *segs, const u32 *walk, u64 *acc, u64 count, int remap, u32 nx)
{
    constexpr int TT = KS_CYC_TILE;
    constexpr int XD = FOLD ? D + 1 : D;     // staged rows per ciphertext: D digits (and c0)
    __shared__ double xt[CB * XD * TT];      // [CB][XD][TT]: source tile c_p
    // [R][D][TT][2]: keys of the outputs c_{p-1} .. c_{p-R}
    __shared__ __attribute__((aligned(16))) double kt[R * 2 * D * TT];
    const int u = threadIdx.x, bl = threadIdx.y;
    u32 bx, by, bz;
    mac_block_ids(remap, bx, by, bz);
    if (bx >= nx) return;  // launch padding
    const CycleSeg sg = segs[bx];
    const int l = (int)by;
    const u64 b = (u64)bz * CB + bl;
    const bool live = b < count;
    const u64 N = dp.N, NE = (u64)dp.ne * N, lN = (u64)l * N;
    const double q = dp.mc[l].qd, qinv = dp.mc[l].qinv;
    const int own = l < dp.nq ? l / dp.alpha : -1;
    const bool fold = FOLD && l < dp.nq;
    const double pq = fold ? u64_to_d(dp.pmod[l]) : 0.0;

    // The segment's tiles, positions m0 .. m0 + cnt + R - 1, in LDS: the
    // addresses of every step are then known without a dependent global load.
    __shared__ u32 tl[KS_CYC_SEG + 8];
    __shared__ const u64 *kp[R];
    __shared__ const u32 *pp[R];
    const int tid = bl * TT + u;
    for (int k = tid; k < sg.cnt + R; k += TT * CB) tl[k] = walk[sg.base + (sg.m0 + k) % sg.len];
    stage_key_ptrs<R>(ks, kp, pp);
    __syncthreads();

    // Staging roles: thread row bl stages its ciphertext's D digit values
    // (and c0) at lane u, and (for bl < R) the 2 D key values of key bl + 1
    // for the output that key serves at this step, with that output's
    // in-tile source index.  The loads of step p + 1 are in flight while
    // step p computes: nothing waits on them before the next step's staging.
    const u64 *xraised = raised + (b * D * dp.ne + l) * N + u;
    const u64 *xown = x + b * x_stride + lN + u;
    const u64 *xc0 = fold ? c0 + b * c0_stride + lN + u : nullptr;
    gu64 *ksrc = bl < R ? (gu64 *)kp[bl] + lN + u : nullptr;
    gu32 *psrc = bl < R ? (gu32 *)pp[bl] + u : nullptr;
    __shared__ u32 pt[R * TT];  // [R][TT]: in-tile source index of the output key t serves
    u64 xv[XD], kv[2 * D];
    u32 pk = 0;
    auto fetch = [&](int p) {
        const u64 src = (u64)tl[p - sg.m0] * TT;
#pragma unroll
        for (int d = 0; d < D; d++)
            xv[d] = live ? (d == own ? xown[src] : xraised[(u64)d * dp.ne * N + src]) : 0;
        if (FOLD) xv[XD - 1] = (live && fold) ? xc0[src] : 0;
        const int m = p - 1 - bl;  // output served by key bl + 1
        const bool kl = bl < R && m >= sg.m0 && m < sg.m0 + sg.cnt;
        const u64 dst = kl ? (u64)tl[m - sg.m0] * TT : 0;
#pragma unroll
        for (int dk = 0; dk < 2 * D; dk++) kv[dk] = kl ? ksrc[(u64)dk * NE + dst] : 0;
        if (bl < R) pk = psrc[dst];  // in bounds also when !kl (dst = 0); unused then
    };
    auto store = [&]() {
#pragma unroll
        for (int d = 0; d < XD; d++) xt[(bl * XD + d) * TT + u] = u64_to_d(xv[d]);
        if (bl < R) {
#pragma unroll
            for (int d = 0; d < D; d++)  // both components of a digit in one 16-byte word
                reinterpret_cast<double2 *>(kt)[(bl * D + d) * TT + u] =
                    make_double2(u64_to_d(kv[2 * d]), u64_to_d(kv[2 * d + 1]));
            pt[bl * TT + u] = pk & (TT - 1);
        }
    };

    double A[R][2];  // A[t - 1]: output position p - t
#pragma unroll
    for (int t = 0; t < R; t++) A[t][0] = A[t][1] = 0.0;
    const int pend = sg.m0 + sg.cnt + R;
    fetch(sg.m0 + 1);
    for (int p = sg.m0 + 1; p < pend; p++) {
        store();
        __syncthreads();
        if (p + 1 < pend) fetch(p + 1);
#pragma unroll
        for (int t = 1; t <= R; t++) {
            const int m = p - t;
            if (m >= sg.m0 && m < sg.m0 + sg.cnt) {
                const double *xs = xt + bl * XD * TT + pt[(t - 1) * TT + u];
                const double2 *kk = reinterpret_cast<const double2 *>(kt) + (t - 1) * D * TT + u;
                double a0 = A[t - 1][0], a1 = A[t - 1][1];
#pragma unroll
                for (int d = 0; d < D; d++) {
                    const double xd = xs[d * TT];
                    const double2 kd = kk[d * TT];
                    a0 += mulmod_d(xd, kd.x, q, qinv);
                    a1 += mulmod_d(xd, kd.y, q, qinv);
                    if (XD > 8 && d == 3) {
                        a0 = reduce_d(a0, q, qinv);
                        a1 = reduce_d(a1, q, qinv);
                    }
                }
                if (FOLD && fold) a0 += mulmod_d(xs[(XD - 1) * TT], pq, q, qinv);
                A[t - 1][0] = reduce_d(a0, q, qinv);
                A[t - 1][1] = reduce_d(a1, q, qinv);
            }
        }
        const int mo = p - R;  // complete: its key-R contribution was just added
        if (mo >= sg.m0 && live) {
            const u64 j = (u64)tl[mo - sg.m0] * TT + u;
            acc[(b * 2) * NE + lN + j] = d_to_canonical(A[R - 1][0], q, qinv);
            acc[(b * 2 + 1) * NE + lN + j] = d_to_canonical(A[R - 1][1], q, qinv);
        }
#pragma unroll
        for (int t = R - 1; t > 0; t--) {
            A[t][0] = A[t - 1][0];
            A[t][1] = A[t - 1][1];
        }
        A[0][0] = A[0][1] = 0.0;
        __syncthreads();  // the tile is rewritten next step
    }
}

// Blocks whose tile map has only short cycles (at most LM tiles; one tile:
// the automorphisms keep every tile in place) need no walk: a workgroup
// stages all source tiles of its cycle (digits, and c0 when folded) once,
// then for each output tile of the cycle stages that tile's R keys and adds
// all R contributions.  Same products and reductions as the walk.
template <int R, int D, int CB, bool FOLD, int LM>
__global__ void __launch_bounds__(KS_CYC_TILE * CB)
mac_short_kernel(DevParams dp, const u64 *x, u64 x_stride, const u64 *raised, const u64 *c0, u64 c0_stride,
                 KeySet ks, const CycleSeg *segs, const u32 *walk, u64 *acc, u64 count, int remap, u32 nx)
{
    constexpr int TT = KS_CYC_TILE;
    constexpr int XD = FOLD ? D + 1 : D;
    __shared__ double xt[LM * CB * XD * TT];  // [LM][CB][XD][TT]: the cycle's source tiles
    __shared__ __attribute__((aligned(16))) double kt[R * 2 * D * TT];  // [R][D][TT][2]: keys of one output tile
    const int u = threadIdx.x, bl = threadIdx.y;
    u32 bx, by, bz;
    mac_block_ids(remap, bx, by, bz);
    if (bx >= nx) return;  // launch padding
    // With one-tile cycles the walk is the identity (tile i is segment i), so
    // the tables are not read.
    int L = 1, base = (int)bx;
    if (LM > 1) {
        const CycleSeg sg = segs[bx];
        L = sg.len;  // <= LM (checked when the kernel is chosen)
        base = sg.base;
    }
    auto tile = [&](int i) -> u64 { return LM == 1 ? (u64)bx : (u64)walk[base + i]; };
    const int l = (int)by;
    const u64 b = (u64)bz * CB + bl;
    const bool live = b < count;
    const u64 N = dp.N, NE = (u64)dp.ne * N, lN = (u64)l * N;
    const double q = dp.mc[l].qd, qinv = dp.mc[l].qinv;
    const int own = l < dp.nq ? l / dp.alpha : -1;
    const bool fold = FOLD && l < dp.nq;
    const double pq = fold ? u64_to_d(dp.pmod[l]) : 0.0;

    // Rows bl < R stage key bl + 1 (2 D values) and its in-tile source
    // indices for one output tile; the next output's are loaded while this
    // one computes.
    static_assert(R < CB, "one key per staging row");
    __shared__ const u64 *kp[R];
    __shared__ const u32 *pp[R];
    stage_key_ptrs<R>(ks, kp, pp);
    __syncthreads();
    gu64 *ksrc = bl < R ? (gu64 *)kp[bl] + lN + u : nullptr;
    gu32 *psrc = bl < R ? (gu32 *)pp[bl] + u : nullptr;
    __shared__ u32 pt[R * TT];
    u64 kv[2 * D];
    u32 pk = 0;
    auto fetch_keys = [&](int m) {
        if (bl < R) {
            const u64 dst = tile(m) * TT;
#pragma unroll
            for (int dk = 0; dk < 2 * D; dk++) kv[dk] = ksrc[(u64)dk * NE + dst];
            pk = psrc[dst];
        }
    };
    auto store_keys = [&]() {
        if (bl < R) {
#pragma unroll
            for (int d = 0; d < D; d++)  // both components of a digit in one 16-byte word
                reinterpret_cast<double2 *>(kt)[(bl * D + d) * TT + u] =
                    make_double2(u64_to_d(kv[2 * d]), u64_to_d(kv[2 * d + 1]));
            pt[bl * TT + u] = pk & (TT - 1);
        }
    };
    // all loads of the cycle's source tiles in flight before any is used
    const u64 *xraised = raised + (b * D * dp.ne + l) * N + u;
    const u64 *xown = x + b * x_stride + lN + u;
    const u64 *xc0 = fold ? c0 + b * c0_stride + lN + u : nullptr;
    u64 xv[LM][XD];
    fetch_keys(0);
#pragma unroll
    for (int i = 0; i < LM; i++) {
        const u64 src = tile(i < L ? i : 0) * TT;
#pragma unroll
        for (int d = 0; d < D; d++) xv[i][d] = live ? (d == own ? xown[src] : xraised[(u64)d * dp.ne * N + src]) : 0;
        if (FOLD) xv[i][XD - 1] = (live && fold) ? xc0[src] : 0;
    }
#pragma unroll
    for (int i = 0; i < LM; i++) {  // (slots past the cycle's length are written, never read)
        double *xs = xt + (i * CB + bl) * XD * TT + u;
#pragma unroll
        for (int d = 0; d < XD; d++) xs[d * TT] = u64_to_d(xv[i][d]);
    }
    store_keys();
    __syncthreads();
#pragma unroll
    for (int m = 0; m < LM; m++) {
        if (m >= L) break;
        if (m > 0) {
            __syncthreads();  // the previous output's keys are consumed
            store_keys();
            __syncthreads();
        }
        if (m + 1 < L) fetch_keys(m + 1);
        const u64 j = tile(m) * TT + u;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll 1
        for (int t = 1; t <= R; t++) {
            const int i = LM == 1 ? 0 : (m + t) % L;  // output c_m reads source tile c_{m+t}
            const double *xs = xt + (i * CB + bl) * XD * TT + pt[(t - 1) * TT + u];
            const double2 *kk = reinterpret_cast<const double2 *>(kt) + (t - 1) * D * TT + u;
#pragma unroll
            for (int d = 0; d < D; d++) {
                const double xd = xs[d * TT];
                const double2 kd = kk[d * TT];
                a0 += mulmod_d(xd, kd.x, q, qinv);
                a1 += mulmod_d(xd, kd.y, q, qinv);
                if (XD > 8 && d == 3) {
                    a0 = reduce_d(a0, q, qinv);
                    a1 = reduce_d(a1, q, qinv);
                }
            }
            if (FOLD && fold) a0 += mulmod_d(xs[(XD - 1) * TT], pq, q, qinv);
            a0 = reduce_d(a0, q, qinv);
            a1 = reduce_d(a1, q, qinv);
        }
        if (live) {
            acc[(b * 2) * NE + lN + j] = d_to_canonical(a0, q, qinv);
            acc[(b * 2 + 1) * NE + lN + j] = d_to_canonical(a1, q, qinv);
        }
    }
}

template <int R, int CB, bool FOLD>
static void launch_mac_cycle_cb(int short_lm, int dnum, dim3 grid, hipStream_t s, const DevParams &dp, const u64 *x, u64 x_stride,
                                const u64 *raised, const u64 *c0, u64 c0_stride, const KeySet &ks,
                                const CycleTable *cyc, u64 *acc, u64 count, int remap, u32 nx)
{
    dim3 block(KS_CYC_TILE, CB);
    if (short_lm == 1 || short_lm == 2) {
#define LC_SHORT(DD, LMV)                                                                                        \
    hipLaunchKernelGGL((mac_short_kernel<R, DD, CB, FOLD, LMV>), grid, block, 0, s, dp, x, x_stride, raised, c0, \
                       c0_stride, ks, cyc->segs, cyc->walk, acc, count, remap, nx)
        if (short_lm == 1) {
            if (dnum == 3) LC_SHORT(3, 1); else if (dnum == 4) LC_SHORT(4, 1); else LC_SHORT(6, 1);
        } else {
            if (dnum == 3) LC_SHORT(3, 2); else if (dnum == 4) LC_SHORT(4, 2); else LC_SHORT(6, 2);
        }
#undef LC_SHORT
        return;
    }
    switch (dnum) {
    case 3: hipLaunchKernelGGL((mac_cycle_kernel<R, 3, CB, FOLD>), grid, block, 0, s, dp, x, x_stride, raised, c0,
                               c0_stride, ks, cyc->segs, cyc->walk, acc, count, remap, nx); break;
    case 4: hipLaunchKernelGGL((mac_cycle_kernel<R, 4, CB, FOLD>), grid, block, 0, s, dp, x, x_stride, raised, c0,
                               c0_stride, ks, cyc->segs, cyc->walk, acc, count, remap, nx); break;
    default: hipLaunchKernelGGL((mac_cycle_kernel<R, 6, CB, FOLD>), grid, block, 0, s, dp, x, x_stride, raised, c0,
                                c0_stride, ks, cyc->segs, cyc->walk, acc, count, remap, nx); break;
    }
}

template <int R, bool FOLD>
static void launch_mac_cycle_r(int short_lm, int cb, int dnum, dim3 grid, hipStream_t s, const DevParams &dp, const u64 *x,
                               u64 x_stride, const u64 *raised, const u64 *c0, u64 c0_stride, const KeySet &ks,
                               const CycleTable *cyc, u64 *acc, u64 count, int remap, u32 nx)
{
    if (cb == 16) launch_mac_cycle_cb<R, 16, FOLD>(short_lm, dnum, grid, s, dp, x, x_stride, raised, c0, c0_stride, ks, cyc, acc, count, remap, nx);
    else launch_mac_cycle_cb<R, 8, FOLD>(short_lm, dnum, grid, s, dp, x, x_stride, raised, c0, c0_stride, ks, cyc, acc, count, remap, nx);
}

// ciphertexts per workgroup: 8 or 16 (tuning "mac_cycle_cts" for walks,
// "mac_short_cts" for short cycles)
static void launch_mac_cycle(const Ctx *c, int R, u64 nseg, hipStream_t s, const u64 *x, u64 x_stride,
                             const u64 *raised, const u64 *c0, u64 c0_stride, const KeySet &ks, const CycleTable *cyc,
                             u64 *acc, u64 count)
{
    // cycles of at most 2 tiles: no walk (0 = walk)
    const int short_lm = c->tune.mac_cycle_short && cyc->max_len <= 2 ? cyc->max_len : 0;
    const int cb = (short_lm ? c->tune.mac_short_cts : c->tune.mac_cycle_cts) == 16 ? 16 : 8;
    dim3 grid((u32)nseg, (u32)c->ne, (u32)((count + cb - 1) / cb));
    const u32 nx = (u32)nseg;
    const int remap = c->tune.mac_xcd && grid.z > 1;
    if (remap) {  // pad x so that x * y is a multiple of 8
        const u32 m = 8u / std::gcd(grid.y, 8u);
        grid.x = (grid.x + m - 1) / m * m;
    }
    if (R == 3) {
        if (c0) launch_mac_cycle_r<3, true>(short_lm, cb, c->dnum, grid, s, c->dp, x, x_stride, raised, c0, c0_stride, ks, cyc, acc, count, remap, nx);
        else launch_mac_cycle_r<3, false>(short_lm, cb, c->dnum, grid, s, c->dp, x, x_stride, raised, c0, c0_stride, ks, cyc, acc, count, remap, nx);
    } else {
        if (c0) launch_mac_cycle_r<7, true>(short_lm, cb, c->dnum, grid, s, c->dp, x, x_stride, raised, c0, c0_stride, ks, cyc, acc, count, remap, nx);
        else launch_mac_cycle_r<7, false>(short_lm, cb, c->dnum, grid, s, c->dp, x, x_stride, raised, c0, c0_stride, ks, cyc, acc, count, remap, nx);
    }
}

// ---- literal hoisted rotations: one staging of each source tile for all keys --
//
// Every key of the call maps aligned tiles of KS_CYC_TILE coefficients onto
// aligned tiles (checked at key set-up), and output tile o of key t reads
// source tile tau_t(o) at the in-tile positions of its permutation.  A
// workgroup owns one source tile s of one limb for CB ciphertexts: it stages
// the tile's digits (and c0) in LDS once, then for each key t computes output
// tile tau_t^-1(s) of that key from it (the next key's values and indices
// load while the current key multiplies).  acc is [key][ct][2][ne][N].  Same
// FP64 Barrett products as the other inner products, and with FOLD the
// permuted c0 times P mod q joins accumulator 0 of the Q limbs.
struct MultiKeys {
    const u64 *key[MULTI_KEYS];
    const u32 *perm[MULTI_KEYS];
    const u32 *inv[MULTI_KEYS];  // source tile -> output tile of the key
    int n;
};

template <int D, int CB, bool FOLD>
__global__ void __launch_bounds__(KS_CYC_TILE * CB)
mac_multi_kernel(DevParams dp, const u64 *x, u64 x_stride, const u64 *raised, const u64 *c0, u64 c0_stride,
                 MultiKeys mk, u64 *acc, u64 count, int remap, u32 nx)
{
    constexpr int TT = KS_CYC_TILE;
    constexpr int XD = FOLD ? D + 1 : D;
    __shared__ double xt[CB * XD * TT];  // [CB][XD][TT]: the source tile
    const int u = threadIdx.x, bl = threadIdx.y;
    u32 bx, by, bz;
    mac_block_ids(remap, bx, by, bz);
    if (bx >= nx) return;  // launch padding
    const u32 st = bx;     // source tile
    const int l = (int)by;
    const u64 b = (u64)bz * CB + bl;
    const bool live = b < count;
    const u64 N = dp.N, NE = (u64)dp.ne * N, lN = (u64)l * N;
    const double q = dp.mc[l].qd, qinv = dp.mc[l].qinv;
    const int own = l < dp.nq ? l / dp.alpha : -1;
    const bool fold = FOLD && l < dp.nq;
    const double pq = fold ? u64_to_d(dp.pmod[l]) : 0.0;
    {
        const u64 src = (u64)st * TT + u;
        u64 xv[XD];
#pragma unroll
        for (int d = 0; d < D; d++)
            xv[d] = live ? (d == own ? x[b * x_stride + lN + src] : raised[((b * D + d) * dp.ne + l) * N + src]) : 0;
        if (FOLD) xv[XD - 1] = (live && fold) ? c0[b * c0_stride + lN + src] : 0;
#pragma unroll
        for (int d = 0; d < XD; d++) xt[(bl * XD + d) * TT + u] = u64_to_d(xv[d]);
    }
    __syncthreads();
    const double *xs0 = xt + bl * XD * TT;
    u64 kv[2 * D];
    u32 pin = 0;
    u64 j = 0;
    auto fetch = [&](int t) {
        const u64 o = ((const gu32 *)mk.inv[t])[st];  // uniform over the workgroup
        j = o * TT + u;
        pin = ((const gu32 *)mk.perm[t])[j] & (TT - 1);
        const gu64 *kp = (const gu64 *)mk.key[t] + lN + j;
#pragma unroll
        for (int dk = 0; dk < 2 * D; dk++) kv[dk] = kp[(u64)dk * NE];
    };
    fetch(0);
    for (int t = 0; t < mk.n; t++) {
        double k[2 * D];
#pragma unroll
        for (int dk = 0; dk < 2 * D; dk++) k[dk] = u64_to_d(kv[dk]);
        const u32 p0 = pin;
        const u64 j0 = j;
        if (t + 1 < mk.n) fetch(t + 1);
        const double *xs = xs0 + p0;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int d = 0; d < D; d++) {
            const double xd = xs[d * TT];
            a0 += mulmod_d(xd, k[2 * d], q, qinv);
            a1 += mulmod_d(xd, k[2 * d + 1], q, qinv);
        }
        if (FOLD && fold) a0 += mulmod_d(xs[(XD - 1) * TT], pq, q, qinv);
        if (live) {
            u64 *o = acc + (((u64)t * count + b) * 2) * NE + lN + j0;
            o[0] = d_to_canonical(reduce_d(a0, q, qinv), q, qinv);
            o[NE] = d_to_canonical(reduce_d(a1, q, qinv), q, qinv);
        }
    }
}

int build_cycle_table(Ctx *c, u64 g)
{
    if (c->cycles.count(g)) return LC_OK;
    CycleTable tab;
    const u64 N = c->N, TT = KS_CYC_TILE;
    if (c->device >= 0 && N >= TT) {
        const std::vector<u32> perm = automorphism_perm(c->log_n, g);
        const u64 nt = N / TT;
        std::vector<u32> tau(nt);
        bool tiles = true;
        for (u64 o = 0; o < nt && tiles; o++) {
            tau[o] = perm[o * TT] / (u32)TT;
            for (u64 v = 1; v < TT; v++)
                if (perm[o * TT + v] / TT != tau[o]) tiles = false;
        }
        if (tiles) {
            std::vector<u32> walk;
            std::vector<CycleSeg> segs;
            std::vector<char> seen(nt, 0);
            int min_len = (int)nt, max_len = 0;
            for (u64 o = 0; o < nt; o++) {
                if (seen[o]) continue;
                const int base = (int)walk.size();
                for (u32 t = (u32)o; !seen[t]; t = tau[t]) {
                    seen[t] = 1;
                    walk.push_back(t);
                }
                const int len = (int)walk.size() - base;
                min_len = std::min(min_len, len);
                max_len = std::max(max_len, len);
                for (int m0 = 0; m0 < len; m0 += KS_CYC_SEG)
                    segs.push_back(CycleSeg{base, len, m0, std::min(KS_CYC_SEG, len - m0)});
            }
            if (walk.size() == nt) {  // tau is a permutation of the tiles
                std::vector<u32> inv(nt);
                for (u64 o = 0; o < nt; o++) inv[tau[o]] = (u32)o;
                u32 *dw = (u32 *)dev_alloc(c, walk.size() * sizeof(u32));
                CycleSeg *ds = (CycleSeg *)dev_alloc(c, segs.size() * sizeof(CycleSeg));
                u32 *di = (u32 *)dev_alloc(c, nt * sizeof(u32));
                if (!dw || !ds || !di) return fail(c, LC_ENOMEM, "cycle table allocation failed");
                LC_HIP(c, hipMemcpy(dw, walk.data(), walk.size() * sizeof(u32), hipMemcpyHostToDevice));
                LC_HIP(c, hipMemcpy(ds, segs.data(), segs.size() * sizeof(CycleSeg), hipMemcpyHostToDevice));
                LC_HIP(c, hipMemcpy(di, inv.data(), nt * sizeof(u32), hipMemcpyHostToDevice));
                c->table_bytes += walk.size() * sizeof(u32) + segs.size() * sizeof(CycleSeg) + nt * sizeof(u32);
                tab.inv_tile = di;
                tab.walk = dw;
                tab.segs = ds;
                tab.nseg = (int)segs.size();
                tab.min_len = min_len;
                tab.max_len = max_len;  // 1: walk[i] = i, which the short-cycle kernel relies on
            }
        }
    }
    c->cycles[g] = tab;
    return LC_OK;
}

// v[b][k][l][j] = BConv_{P->Q} of the (coefficient-domain) P limbs of acc,
// in the same FP64 form as the ModUp conversion.
__global__ void __launch_bounds__(KS_THREADS)
moddown_bconv_kernel(DevParams dp, const u64 *acc, u64 *v, u64 count)
{
    u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // over count * 2 * N
    if (e >= count * 2 * (u64)dp.N) return;
    u64 j = e & (dp.N - 1), bk = e >> dp.log_n;
    const u64 *A = acc + bk * (u64)dp.ne * dp.N;
    double y[MAX_NP];
    for (int k = 0; k < dp.np; k++) {
        const ModConst &mc = dp.mc[dp.nq + k];
        double a = u64_to_d(A[(u64)(dp.nq + k) * dp.N + j]);
        y[k] = canon_d(mulmod_d(a, dp.dn_inv_d[k], mc.qd, mc.qinv), mc.qd, mc.qinv);
    }
    u64 *out = v + bk * (u64)dp.nq * dp.N + j;
    for (int l = 0; l < dp.nq; l++) {
        const double q = dp.mc[l].qd, qinv = dp.mc[l].qinv;
        double s = 0.0;
        for (int k = 0; k < dp.np; k++) s += mulmod_d(y[k], dp.dn_fac_d[(u64)k * dp.nq + l], q, qinv);
        out[(u64)l * dp.N] = d_to_canonical(s, q, qinv);
    }
}

// out0 = base0 + sum_t phi_t(c0src) + (acc0_Q - v0) P^-1, out1 = base1 + (acc1_Q - v1) P^-1
__global__ void __launch_bounds__(KS_THREADS)
ks_combine_kernel(DevParams dp, const u64 *acc, const u64 *v, const u64 *base, u64 base_stride, const u64 *c0src,
                  u64 c0_stride, KeySet ks, u64 *out, u64 out_stride, u64 count)
{
    u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // over nq * N
    u64 b = blockIdx.y;
    const u64 S = (u64)dp.nq * dp.N;
    if (e >= S || b >= count) return;
    int l = (int)(e >> dp.log_n);
    u64 j = e & (dp.N - 1);
    u64 q = dp.mc[l].m, pi = dp.pinv[l], pish = dp.pinv_sh[l];
    const u64 NE = (u64)dp.ne * dp.N;
    u64 r0 = mul_shoup(acc[(b * 2) * NE + e] + q - v[(b * 2) * S + e], pi, pish, q);
    u64 r1 = mul_shoup(acc[(b * 2 + 1) * NE + e] + q - v[(b * 2 + 1) * S + e], pi, pish, q);
    if (base) {
        r0 = add_mod(r0, base[b * base_stride + e], q);
        r1 = add_mod(r1, base[b * base_stride + S + e], q);
    }
    if (c0src) {
        for (int t = 0; t < ks.n; t++) {
            u64 src = ks.perm[t] ? ks.perm[t][j] : j;
            r0 = add_mod(r0, c0src[b * c0_stride + (u64)l * dp.N + src], q);
        }
    }
    out[b * out_stride + e] = r0;
    out[b * out_stride + S + e] = r1;
}

u64 ks_words_per_ct(const Ctx *c)
{
    return ((u64)c->nq + (u64)c->dnum * c->ne + 2ull * c->ne + 2ull * c->nq) * c->N;
}

int keyswitch_hoisted(Ctx *c, const u64 *x, u64 x_stride, u64 count, const KsGroup *groups, int ngroups,
                      hipStream_t s)
{
    for (int g = 0; g < ngroups; g++)
        if (groups[g].n < 1 || groups[g].n > 8) return fail(c, LC_EINVAL, "1..8 keys per hoisted group");
    const u64 per_ct = ks_words_per_ct(c);
    u64 chunk = std::min<u64>(count, (u64)c->tune.ks_chunk);
    if (c->ws_limit) chunk = std::max<u64>(1, std::min<u64>(chunk, c->ws_limit / (per_ct * 8)));
    u64 *ws = ws_get(c, WS_KS, per_ct * 8 * chunk, s);
    if (!ws) return LC_ENOMEM;
    return keyswitch_hoisted_ws(c, x, x_stride, count, groups, ngroups, ws, per_ct * chunk, s);
}

// ModUp of B inputs (limbs at x, stride x_stride, NTT domain) into the raised
// digits: the inverse transform reads the input limbs in place (out of place
// into xhat); its last pass scales limb a by N^-1 (Q_d/q_a)^-1, leaving the
// ModUp digits y_a; the forward transform of the raised limbs computes their
// base conversion in its first pass.
static int modup_fused(Ctx *c, const u64 *xb, u64 x_stride, u64 B, u64 *xhat, u64 *raised, hipStream_t s)
{
    const u64 N = c->N;
    PolyBatch ib{xhat, B, c->nq, (u64)c->nq, 0, 0};
    ib.iscale = c->dp.ks_scale;
    ib.out_f64 = 1;
    ib.in_base = xb;
    ib.in_gstride = x_stride / N;
    int rc = launch_ntt_inv(c, ib, s);
    if (rc) return rc;
    PolyBatch fb{raised, B * c->dnum, c->ne, (u64)c->ne, 0, 1};
    fb.conv = 1;
    fb.conv_y = xhat;
    fb.conv_stride = (u64)c->nq * N;
    return launch_ntt_fwd(c, fb, s);
}

// ModDown of B accumulators acc [B][2][ne][N] in two transforms: the inverse
// one scales P limb k by N^-1 (P / p_k)^-1 (in place in acc); the forward one
// of v computes the conversion to the Q limbs in its first pass (K products
// below 0.875 q each: the sum stays below 7 q for K <= 8) and, when out is
// given, the combine out = (acc - v) P^-1 (+ base) in its last pass.
static int moddown_fused(Ctx *c, u64 *acc, u64 B, u64 *v, const u64 *base, u64 base_stride, u64 *out,
                         u64 out_stride, hipStream_t s)
{
    const u64 N = c->N;
    PolyBatch ib{acc + (u64)c->nq * N, B * 2, c->np, (u64)c->ne, c->nq, 0};
    ib.iscale = c->dp.ks_scale;
    ib.out_f64 = 1;
    int rc = launch_ntt_inv(c, ib, s);
    if (rc) return rc;
    PolyBatch fb{v, B * 2, c->nq, (u64)c->nq, 0, 0};
    fb.conv = 2;
    fb.conv_y = acc + (u64)c->nq * N;
    fb.conv_stride = (u64)c->ne * N;
    if (out) {
        fb.comb_acc = acc;
        fb.comb_acc_stride = (u64)c->ne * N;
        fb.comb_add = base;
        fb.comb_add_stride = base_stride;
        fb.comb_out = out;
        fb.comb_out_stride = out_stride;
    }
    return launch_ntt_fwd(c, fb, s);
}

int keyswitch_hoisted_ws(Ctx *c, const u64 *x, u64 x_stride, u64 count, const KsGroup *groups, int ngroups,
                         u64 *ws, u64 ws_words, hipStream_t s)
{
    const u64 N = c->N;
    const int nq = c->nq, np = c->np, ne = c->ne, dnum = c->dnum;
    for (int g = 0; g < ngroups; g++)
        if (groups[g].n < 1 || groups[g].n > 8) return fail(c, LC_EINVAL, "1..8 keys per hoisted group");
    const u64 per_ct = ks_words_per_ct(c);
    if (ws_words < per_ct) return fail(c, LC_EINVAL, "key-switch scratch smaller than one ciphertext's");
    const u64 chunk = std::min<u64>(std::min<u64>(count, (u64)c->tune.ks_chunk), ws_words / per_ct);
    int rc;
    for (u64 b0 = 0; b0 < count; b0 += chunk) {
        u64 B = std::min(chunk, count - b0);
        u64 *xhat = ws;
        u64 *raised = xhat + B * nq * N;
        u64 *acc = raised + B * dnum * ne * N;
        u64 *v = acc + B * 2 * ne * N;
        const u64 *xb = x + b0 * x_stride;
        u64 words = (u64)nq * N;
        const bool fused = c->tune.fuse_modup && c->log_n >= 10 && c->log_n <= 17 && x_stride % N == 0;
        if (!fused) {
            hipLaunchKernelGGL(strided_copy_kernel, dim3(blocks_for(words * B)), dim3(KS_THREADS), 0, s, xb, x_stride,
                               xhat, words, words, B);
            LC_HIP(c, hipGetLastError());
        }
        if (fused) {
            if ((rc = modup_fused(c, xb, x_stride, B, xhat, raised, s))) return rc;
        } else {
            if ((rc = launch_ntt_inv(c, PolyBatch{xhat, B, nq, (u64)nq, 0, 0}, s))) return rc;
            const u32 tpb = (u32)std::min<u64>(N, KS_THREADS);
            hipLaunchKernelGGL(modup_bconv_kernel, dim3((u32)(N / tpb), (u32)(B * dnum)), dim3(tpb), 0, s, c->dp,
                               xhat, raised);
            LC_HIP(c, hipGetLastError());
            if ((rc = launch_ntt_fwd(c, PolyBatch{raised, B * dnum, ne, (u64)ne, 0, 1}, s))) return rc;
        }
        for (int g = 0; g < ngroups; g++) {
            const KsGroup &G = groups[g];
            KeySet ks{};
            ks.n = G.n;
            for (int t = 0; t < G.n; t++) {
                ks.key[t] = G.keys[t];
                ks.perm[t] = G.perms[t];
            }
            // the walk pays off on long cycles; on short ones the per-key gathers
            // of mac_kernel hit the same few tiles in cache
            const bool cyc = c->tune.mac_cycle && G.cyc && G.cyc->nseg > 0 && (G.n == 3 || G.n == 7) &&
                             (dnum == 3 || dnum == 4 || dnum == 6) &&
                             (G.cyc->min_len >= c->tune.mac_cycle_min ||
                              (G.cyc->max_len <= 2 && c->tune.mac_cycle_short));
            // the inner product folds sum_t phi_t(c0) into the accumulator
            // (then ModDown's last pass does the whole combine)
            const u64 *c0_fold = c->tune.mac_cycle_c0 && G.c0src ? G.c0src + b0 * G.c0_stride : nullptr;
            if (cyc) {
                launch_mac_cycle(c, G.n, (u64)G.cyc->nseg, s, xb, x_stride, raised, c0_fold, G.c0_stride, ks, G.cyc,
                                 acc, B);
            } else {
                const dim3 grid(blocks_for((u64)ne * N), (u32)((B + c->tune.mac_cts - 1) / c->tune.mac_cts));
                if (c->tune.mac_cts == 16 && c0_fold)
                    hipLaunchKernelGGL((mac_kernel<16, true>), grid, dim3(KS_THREADS), 0, s, c->dp, xb, x_stride,
                                       raised, c0_fold, G.c0_stride, ks, acc, B);
                else if (c->tune.mac_cts == 16)
                    hipLaunchKernelGGL((mac_kernel<16, false>), grid, dim3(KS_THREADS), 0, s, c->dp, xb, x_stride,
                                       raised, nullptr, 0, ks, acc, B);
                else if (c0_fold)
                    hipLaunchKernelGGL((mac_kernel<8, true>), grid, dim3(KS_THREADS), 0, s, c->dp, xb, x_stride,
                                       raised, c0_fold, G.c0_stride, ks, acc, B);
                else
                    hipLaunchKernelGGL((mac_kernel<8, false>), grid, dim3(KS_THREADS), 0, s, c->dp, xb, x_stride,
                                       raised, nullptr, 0, ks, acc, B);
            }
            LC_HIP(c, hipGetLastError());
            const u64 *c0rest = (G.c0src && !c0_fold) ? G.c0src + b0 * G.c0_stride : nullptr;
            if (fused && np <= MAX_NP) {
                // unless permuted c0 terms remain, the combine runs in the
                // ModDown's last pass
                if ((rc = moddown_fused(c, acc, B, v, G.base ? G.base + b0 * G.base_stride : nullptr, G.base_stride,
                                        c0rest ? nullptr : G.out + b0 * G.out_stride, G.out_stride, s)))
                    return rc;
                if (!c0rest) continue;
            } else {
                if ((rc = launch_ntt_inv(c, PolyBatch{acc + (u64)nq * N, B * 2, np, (u64)ne, nq, 0}, s))) return rc;
                hipLaunchKernelGGL(moddown_bconv_kernel, dim3(blocks_for(B * 2 * N)), dim3(KS_THREADS), 0, s, c->dp,
                                   acc, v, B);
                LC_HIP(c, hipGetLastError());
                if ((rc = launch_ntt_fwd(c, PolyBatch{v, B * 2, nq, (u64)nq, 0, 0}, s))) return rc;
            }
            hipLaunchKernelGGL(ks_combine_kernel, dim3(blocks_for((u64)nq * N), (u32)B), dim3(KS_THREADS), 0, s,
                               c->dp, acc, v, G.base ? G.base + b0 * G.base_stride : nullptr, G.base_stride, c0rest,
                               G.c0_stride, ks, G.out + b0 * G.out_stride, G.out_stride, B);
            LC_HIP(c, hipGetLastError());
        }
    }
    return LC_OK;
}

// Literal hoisted rotations through the source-major inner product: per
// batch one ModUp, then per group of up to MULTI_KEYS keys one inner product
// that stages each source tile once, and one fused ModDown per key (the
// permuted c0 is folded into the inner product, so its last pass writes the
// rotated ciphertext).  keys / perms / inv are per step; outs[t] of ct b is at
// out + b * out_stride + t * 2 S.
int keyswitch_rotations(Ctx *c, const u64 *ct, u64 count, const u64 *const *keys, const u32 *const *perms,
                        const u32 *const *inv, int nsteps, u64 *out, u64 out_stride, hipStream_t s)
{
    const u64 N = c->N, S = (u64)c->nq * N;
    const int nq = c->nq, ne = c->ne, dnum = c->dnum;
    if (dnum > 8 || nsteps < 1) return fail(c, LC_EINVAL, "source-major rotations need 1 <= dnum <= 8 and a step");
    const int rk = std::min(nsteps, MULTI_KEYS);
    const u64 per_ct = ((u64)nq + (u64)dnum * ne + (u64)rk * 2 * ne + 2ull * nq) * N;
    // batches sized to at most 12 GiB of workspace (the accumulators of 8
    // keys make a ciphertext's workspace about 2.3 times that of one key
    // switch): all of a small ring's ciphertexts in one batch, whose
    // launches are then few and large; 35 ciphertexts at N = 2^16 with
    // 24 + 4 limbs
    const u64 cap = ((u64)12 << 30) / (per_ct * 8);
    u64 chunk = std::max<u64>(1, std::min<u64>(count, cap));
    if (c->ws_limit) chunk = std::max<u64>(1, std::min<u64>(chunk, c->ws_limit / (per_ct * 8)));
    u64 *ws = ws_get(c, WS_KS, per_ct * 8 * chunk, s);
    if (!ws) return LC_ENOMEM;
    constexpr int CB = 8;
    int rc;
    for (u64 b0 = 0; b0 < count; b0 += chunk) {
        const u64 B = std::min(chunk, count - b0);
        u64 *xhat = ws;
        u64 *raised = xhat + B * nq * N;
        u64 *acc = raised + B * dnum * ne * N;
        u64 *v = acc + (u64)rk * B * 2 * ne * N;
        const u64 *cb = ct + b0 * 2 * S;
        if ((rc = modup_fused(c, cb + S, 2 * S, B, xhat, raised, s))) return rc;
        for (int t0 = 0; t0 < nsteps; t0 += rk) {
            MultiKeys mk{};
            mk.n = std::min(rk, nsteps - t0);
            for (int t = 0; t < mk.n; t++) {
                mk.key[t] = keys[t0 + t];
                mk.perm[t] = perms[t0 + t];
                mk.inv[t] = inv[t0 + t];
            }
            dim3 grid((u32)(N / KS_CYC_TILE), (u32)ne, (u32)((B + CB - 1) / CB));
            const u32 nx = grid.x;
            const int remap = c->tune.mac_xcd && grid.z > 1;
            if (remap) {
                const u32 m = 8u / std::gcd(grid.y, 8u);
                grid.x = (grid.x + m - 1) / m * m;
            }
            const dim3 block(KS_CYC_TILE, CB);
#define LC_MULTI(DD)                                                                                              \
    hipLaunchKernelGGL((mac_multi_kernel<DD, CB, true>), grid, block, 0, s, c->dp, cb + S, 2 * S, raised, cb, 2 * S, \
                       mk, acc, B, remap, nx)
            switch (dnum) {
            case 1: LC_MULTI(1); break;
            case 2: LC_MULTI(2); break;
            case 3: LC_MULTI(3); break;
            case 4: LC_MULTI(4); break;
            case 5: LC_MULTI(5); break;
            case 6: LC_MULTI(6); break;
            case 7: LC_MULTI(7); break;
            default: LC_MULTI(8); break;
            }
#undef LC_MULTI
            LC_HIP(c, hipGetLastError());
            for (int t = 0; t < mk.n; t++) {
                u64 *o = out + b0 * out_stride + (u64)(t0 + t) * 2 * S;
                if ((rc = moddown_fused(c, acc + (u64)t * B * 2 * ne * N, B, v, nullptr, 0, o, out_stride, s)))
                    return rc;
            }
        }
    }
    return LC_OK;
}

}  // namespace lc
