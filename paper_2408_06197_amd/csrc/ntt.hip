// Batched negacyclic NTT / inverse NTT over RNS limbs (the paper's "NWT",
// Appendix, Descriptions of Hardware Acceleration).
//
// Forward transform: merged Cooley-Tukey with psi-twisted twiddles, natural
// order in, bit-reversed evaluation order out; stage s pairs elements at
// distance N / 2^(s+1) inside group i = j >> (log_n - s) with twiddle
// psi^brev(2^s + i).  Inverse: Gentleman-Sande with inverse twiddles, stages
// in reverse order, N^-1 applied on the way out.  Butterflies are lazy
// (Harvey): forward values stay in [0, 4q), inverse values in [0, 2q); the
// last pass returns canonical residues.
//
// A transform of size N is split into passes; a pass covers LOG_S
// consecutive stages, i.e. independent sub-transforms of size S = 2^LOG_S
// over elements j = hi * S * stride + a * stride + lo (a in [0, S)).  One
// workgroup loads a tile of C such sub-transforms into LDS -- C adjacent `lo`
// values when stride >= C, C adjacent blocks when stride == 1 -- so global
// accesses are coalesced, runs its stages out of LDS and writes the tile back.
#include "lc_internal.h"

namespace lc {

constexpr int NTT_TILE = 4096;  // u64 elements per workgroup tile (32 KiB LDS)
constexpr int NTT_THREADS = 256;

struct PassArgs {
    int s0;      // first global stage of the pass
    int log_s;   // stages in the pass
    int cols;    // sub-transforms per workgroup
    int final_;  // last pass of the transform: canonicalize (and scale by N^-1 when inverse)
};

__device__ __forceinline__ bool poly_of_block(const DevParams &dp, const PolyBatch &pb, u64 p, u64 *&ptr, int &mi,
                                              const u64 **in = nullptr)
{
    u64 g = p / (u64)pb.nlimb;
    int l = (int)(p % (u64)pb.nlimb);
    mi = pb.limb0 + l;
    if (pb.skip_own_digit && mi < dp.nq && (int)(g % (u64)dp.dnum) == mi / dp.alpha) return false;
    ptr = pb.base + (g * pb.gstride + (u64)l) * dp.N;
    if (in) *in = pb.in_base ? pb.in_base + (g * pb.in_gstride + (u64)l) * dp.N : ptr;
    return true;
}

__device__ __forceinline__ u64 elem_index(u32 a, u32 c, u32 tile, u32 stride, int log_s, int cols, int log_n)
{
    u32 S = 1u << log_s;
    if (stride == 1) return ((u64)tile * cols + c) * S + a;
    u32 lo_tiles = stride / cols;
    u64 hi = tile / lo_tiles, lo0 = (u64)(tile % lo_tiles) * cols;
    (void)log_n;
    return hi * S * stride + (u64)a * stride + lo0 + c;
}

template <bool INVERSE>
__global__ void __launch_bounds__(NTT_THREADS) ntt_pass_kernel(DevParams dp, PolyBatch pb, PassArgs pa)
{
    __shared__ u64 lds[NTT_TILE];
    u64 *poly;
    int mi;
    if (!poly_of_block(dp, pb, blockIdx.x, poly, mi)) return;
    const u64 q = dp.mc[mi].m, q2 = 2 * q;
    const u32 S = 1u << pa.log_s;
    const u32 stride = dp.N >> (pa.s0 + pa.log_s);
    const u32 cols = (u32)pa.cols;
    const u32 tile = blockIdx.y;
    const u32 nel = S * cols;
    const u64 *tw = (INVERSE ? dp.itw : dp.tw) + (u64)mi * dp.N;
    const u64 *tws = (INVERSE ? dp.itw_sh : dp.tw_sh) + (u64)mi * dp.N;

    for (u32 idx = threadIdx.x; idx < nel; idx += blockDim.x) {
        u32 a, c;
        if (stride == 1) { c = idx / S; a = idx % S; }
        else { a = idx / cols; c = idx % cols; }
        lds[a * cols + c] = poly[elem_index(a, c, tile, stride, pa.log_s, pa.cols, dp.log_n)];
    }
    __syncthreads();

    const u32 nbf = (S / 2) * cols;
    for (int t = 0; t < pa.log_s; t++) {
        int tl = INVERSE ? (pa.log_s - 1 - t) : t;  // local stage
        int s = pa.s0 + tl;                         // global stage
        u32 half = S >> (tl + 1);
        for (u32 b = threadIdx.x; b < nbf; b += blockDim.x) {
            u32 c = b % cols, k = b / cols;
            u32 a1 = (k / half) * 2 * half + (k % half), a2 = a1 + half;
            u64 j1 = elem_index(a1, c, tile, stride, pa.log_s, pa.cols, dp.log_n);
            u64 ti = (1ull << s) + (j1 >> (dp.log_n - s));
            u64 w = tw[ti], wsh = tws[ti];
            u64 X = lds[a1 * cols + c], Y = lds[a2 * cols + c];
            if (!INVERSE) {
                X = csub(X, q2);
                u64 T = mul_shoup_lazy(Y, w, wsh, q);
                lds[a1 * cols + c] = X + T;
                lds[a2 * cols + c] = X - T + q2;
            } else {
                lds[a1 * cols + c] = csub(X + Y, q2);
                lds[a2 * cols + c] = mul_shoup_lazy(X - Y + q2, w, wsh, q);
            }
        }
        __syncthreads();
    }

    const u64 ni = dp.ninv[mi], nish = dp.ninv_sh[mi];
    for (u32 idx = threadIdx.x; idx < nel; idx += blockDim.x) {
        u32 a, c;
        if (stride == 1) { c = idx / S; a = idx % S; }
        else { a = idx / cols; c = idx % cols; }
        u64 v = lds[a * cols + c];
        if (pa.final_) {
            if (INVERSE) v = mul_shoup(v, ni, nish, q);
            else v = csub(csub(v, q2), q);
        }
        poly[elem_index(a, c, tile, stride, pa.log_s, pa.cols, dp.log_n)] = v;
    }
}

// ---- register-radix pass kernel (N >= 2^10) ---------------------------------
//
// Same passes, faster execution: LOG_S in [5, 9] is a compile-time constant
// and each lane owns 16 elements of one sub-transform.  The tile is staged in
// LDS with coalesced global accesses; the pass then runs as register rounds
// separated by LDS exchanges.  Round r (forward order) does stages 4r ..
// min(4r + 3, LOG_S - 1), which pair on bits of a inside [pos, pos + 4),
// pos = max(0, LOG_S - 4 - 4r); lane t holds the 16 elements whose bits
// [pos, pos + 4) are h = 0..15 and whose other bits are t:
//   a = ((t >> pos) << (pos + 4)) | (h << pos) | (t & (2^pos - 1)).
// LOG_S <= 8 takes two rounds (top: a = (h << (LOG_S-4)) | t; bottom:
// a = (t << 4) | h, the remaining LOG_S - 4 stages), LOG_S = 9 three (the
// last does stage 8 alone).  Forward passes run the rounds in order, inverse
// passes in reverse.

// LDS layout of a tile: sub-transform c holds its S elements with one pad
// word per 16.  A 16-lane group of a wave accesses LDS in one go over 32
// banks of 4 bytes.  The rounds read and write 16 consecutive pad-free runs
// of one or two sub-transforms, which never conflict.  The coalesced staging
// of a column pass (and its read-out) instead touches the same element a of
// 8 to 16 sub-transforms at once, which with a stride of S + S / 16 words
// (a multiple of 16 doubles for S >= 256) all fall in the same two banks.
// So column tiles get a sub-transform stride one (S = 256) or two (S = 512)
// doubles longer, and below 256 points, where one 16-lane group of a round
// spans several sub-transforms and the stride has to stay, the element
// index is XORed with bits of c (a permutation inside each run of 16, so
// the pad words stay put).  Block tiles keep the plain layout: their staging
// is already conflict-free.
template <int LOG_S, bool BLOCKS>
constexpr u32 lds_stride()
{
    return (1u << LOG_S) + (1u << LOG_S) / 16 + (BLOCKS ? 0u : LOG_S == 8 ? 1u : LOG_S == 9 ? 2u : 0u);
}

template <int LOG_S, bool BLOCKS>
__device__ __forceinline__ u32 lds_idx(u32 c, u32 a)
{
    if (!BLOCKS && LOG_S < 8) a ^= (c >> (8 - LOG_S)) & 15u;
    return c * lds_stride<LOG_S, BLOCKS>() + a + (a >> 4);
}

// LDS bytes of a tile (4096 elements), host side
static size_t fast_lds_bytes(int log_s, bool blocks)
{
    const size_t S = (size_t)1 << log_s;
    const size_t extra = blocks ? 0 : log_s == 8 ? 1 : log_s == 9 ? 2 : 0;
    return (4096 / S) * (S + S / 16 + extra) * sizeof(double);
}

template <int LOG_S>
constexpr int round_count() { return (LOG_S + 3) / 4; }
template <int LOG_S>
constexpr int round_pos(int r) { return LOG_S - 4 - 4 * r > 0 ? LOG_S - 4 - 4 * r : 0; }

// element index a of entry h of lane t in round r
template <int LOG_S>
__device__ __forceinline__ u32 round_elem(int r, u32 t, u32 h)
{
    const int pos = round_pos<LOG_S>(r);
    return ((t >> pos) << (pos + 4)) | (h << pos) | (t & ((1u << pos) - 1));
}

template <int LOG_S, bool INVERSE>
__device__ __forceinline__ void ntt_round(double (&x)[16], int r, u32 t, u64 hi, int s0, const double *tw,
                                          double q, double qinv)
{
    const int pos = round_pos<LOG_S>(r);
    // local stages of this round, in execution order
    const int first = 4 * r, last = 4 * r + 3 < LOG_S - 1 ? 4 * r + 3 : LOG_S - 1;
#pragma unroll
    for (int it = 0; it < 4; it++) {
        int sl = INVERSE ? (last - it) : (first + it);
        if (sl < first || sl > last) continue;
        int bit = LOG_S - 1 - sl;                  // bit of a this stage pairs on
        int hb = bit - pos;                        // the same bit inside h
        u64 base = (1ull << (s0 + sl)) + (hi << sl);
#pragma unroll
        for (int h = 0; h < 16; h++) {
            if (h & (1 << hb)) continue;
            u32 a1 = round_elem<LOG_S>(r, t, (u32)h);
            double w = tw[base + (a1 >> (LOG_S - sl))];
            double X = x[h], Y = x[h | (1 << hb)];
            if (!INVERSE) {
                // X is reduced only on every other stage, counted back from
                // the pass's last one (which always reduces).  With q < 2^50
                // the Barrett estimate of T = Y w mod q is off by at most
                // 1/2 + 3 |Y| 2^-53 <= 1/2 + 0.375 |Y| / q, so |T| <= (1/2 +
                // 0.375 b) q for |Y| <= b q.  A lazy stage takes entries
                // <= 2.46 q to <= 1.375 * 2.46 q + q/2 <= 3.89 q, a reducing
                // stage takes those back to <= q/2 + 1 + (1/2 + 0.375 * 3.89) q
                // <= 2.46 q: every mulmod input stays below 4 q and every value
                // below 2^52, so all of it is exact.  Pass inputs (canonical, or
                // a reduced conversion sum) and outputs (after a reducing
                // stage) lie within 2.46 q.
                double T = mulmod_d(Y, w, q, qinv);
                if (((LOG_S - 1 - sl) & 1) == 0) X = reduce_d(X, q, qinv);  // |X| <= q/2 + 1
                x[h] = X + T;
                x[h | (1 << hb)] = X - T;
            } else {
                // invariant: |X|, |Y| <= 2q on entry and exit
                double S = reduce_d(X + Y, q, qinv);
                x[h | (1 << hb)] = mulmod_d(X - Y, w, q, qinv);
                x[h] = S;
            }
        }
    }
}

// first_: the pass reads uint64 residues (else doubles left by the other pass);
// final_: the pass writes canonical uint64 residues (times N^-1 when inverse).
// MODE (forward only): 1 / 2 = first pass with the ModUp / ModDown base
// conversion (PolyBatch::conv), 3 = last pass with the ModDown combine
// (PolyBatch::comb_*).
// One workgroup's pass over one tile of polynomial `poly` (ring degree
// N_, modulus index mi, double twiddles tw of that degree and modulus;
// ntab[mi] is the inverse pass's final scale unless pb.iscale is set).  src
// is what a first pass reads; pidx is the polynomial's index in pb (used by
// the fused conversion and combine modes).
template <int LOG_S, bool INVERSE, bool BLOCKS, int MODE>
__device__ __forceinline__ void ntt_fast_body(const DevParams &dp, const PolyBatch &pb, u64 pidx, u64 *poly,
                                              const u64 *src, int mi, u32 tile, u32 N_, const double *tw,
                                              const u64 *ntab, int s0, int cols, int final_, double *lds)
{
    constexpr u32 S = 1u << LOG_S;
    constexpr u32 TPC = S / 16;  // lanes per sub-transform
    const double q = dp.mc[mi].qd, qinv = dp.mc[mi].qinv;
    const bool first_ = !final_;
    if (!first_) src = poly;
    const u32 stride = N_ >> (s0 + LOG_S);
    const u32 nthreads = blockDim.x;
    const u32 tid = threadIdx.x;
    const u32 nel = S * (u32)cols;
    // tile geometry
    u64 hi_col = 0, lo0 = 0;
    if (!BLOCKS) {
        u32 lo_tiles = stride / (u32)cols;
        hi_col = tile / lo_tiles;
        lo0 = (u64)(tile % lo_tiles) * (u32)cols;
    }
    // coalesced load into LDS: every lane issues its eight 16-byte loads
    // (element pairs e, e+1 with e even) before writing any of them
    double v[16];
    if (MODE == 1 || MODE == 2) {  // forward, first pass, base conversion
        // the limb's input is the base conversion sum_a y_a F_a mod m over
        // the source limbs a of conv_y, each y_a already scaled by its
        // inverse factor (ModUp: the digit's limbs, F_a = Q_d / q_a; ModDown:
        // the P limbs, F_k = P / p_k); the sum (|s| <= 7 m) is reduced to
        // |s| <= m / 2 + 1, a valid input of the transform
        const u64 grp = pidx / (u64)pb.nlimb;
        const u64 *yb;
        const double *fac;
        u64 fstride;
        int na;
        if (MODE == 1) {
            const int d = (int)(grp % (u64)dp.dnum);
            const int a0 = d * dp.alpha;
            na = min(dp.alpha, dp.nq - a0);
            yb = pb.conv_y + (grp / (u64)dp.dnum) * pb.conv_stride + (u64)a0 * dp.N;
            fac = dp.up_fac_d + (u64)d * dp.alpha * dp.ne + mi;
            fstride = (u64)dp.ne;
        } else {
            na = dp.np;
            yb = pb.conv_y + grp * pb.conv_stride;
            fac = dp.dn_fac_d + mi;
            fstride = (u64)dp.nq;
        }
#pragma unroll
        for (int i = 0; i < 16; i++) v[i] = 0.0;
        for (int a = 0; a < na; a++) {
            const double f = fac[(u64)a * fstride];
            ulonglong2 y2[8];
#pragma unroll
            for (int i = 0; i < 8; i++) {
                u32 e = 2 * (tid + (u32)i * nthreads);
                u64 g;
                if (BLOCKS) g = ((u64)tile * cols + (e >> LOG_S)) * S + (e & (S - 1));
                else g = (hi_col * S + e / (u32)cols) * stride + lo0 + e % (u32)cols;
                y2[i] = *reinterpret_cast<const ulonglong2 *>(yb + (u64)a * dp.N + g);
            }
#pragma unroll
            for (int i = 0; i < 8; i++) {
                v[2 * i] += mulmod_d(__longlong_as_double((long long)y2[i].x), f, q, qinv);
                v[2 * i + 1] += mulmod_d(__longlong_as_double((long long)y2[i].y), f, q, qinv);
            }
        }
#pragma unroll
        for (int i = 0; i < 16; i++) v[i] = reduce_d(v[i], q, qinv);
    } else {
        // all eight loads are issued before any value is used: a conversion
        // between them would make each load wait for the one before
        ulonglong2 p2[8];
#pragma unroll
        for (int i = 0; i < 8; i++) {
            u32 e = 2 * (tid + (u32)i * nthreads);
            u64 g;
            if (BLOCKS) g = ((u64)tile * cols + (e >> LOG_S)) * S + (e & (S - 1));
            else g = (hi_col * S + e / (u32)cols) * stride + lo0 + e % (u32)cols;
            p2[i] = *reinterpret_cast<const ulonglong2 *>(src + g);
        }
        if (first_) {
#pragma unroll
            for (int i = 0; i < 8; i++) {
                v[2 * i] = u64_to_d(p2[i].x);
                v[2 * i + 1] = u64_to_d(p2[i].y);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; i++) {
                v[2 * i] = __longlong_as_double((long long)p2[i].x);
                v[2 * i + 1] = __longlong_as_double((long long)p2[i].y);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 8; i++) {
        u32 e = 2 * (tid + (u32)i * nthreads);
        u32 a, c;
        if (BLOCKS) { c = e >> LOG_S; a = e & (S - 1); }
        else { a = e / (u32)cols; c = e % (u32)cols; }
        // BLOCKS: (c, a), (c, a+1); columns: (c, a), (c+1, a)
        u32 i0 = lds_idx<LOG_S, BLOCKS>(c, a), i1 = BLOCKS ? lds_idx<LOG_S, BLOCKS>(c, a + 1) : lds_idx<LOG_S, BLOCKS>(c + 1, a);
        lds[i0] = v[2 * i];
        lds[i1] = v[2 * i + 1];
    }
    __syncthreads();
    const u32 c = tid / TPC, t = tid % TPC;
    const u64 hi = BLOCKS ? ((u64)tile * cols + c) : hi_col;
    double x[16];
    constexpr int NR = round_count<LOG_S>();
#pragma unroll
    for (int k = 0; k < NR; k++) {
        const int r = INVERSE ? NR - 1 - k : k;
#pragma unroll
        for (int h = 0; h < 16; h++) x[h] = lds[lds_idx<LOG_S, BLOCKS>(c, round_elem<LOG_S>(r, t, (u32)h))];
        ntt_round<LOG_S, INVERSE>(x, r, t, hi, s0, tw, q, qinv);
#pragma unroll
        for (int h = 0; h < 16; h++) lds[lds_idx<LOG_S, BLOCKS>(c, round_elem<LOG_S>(r, t, (u32)h))] = x[h];
        __syncthreads();
    }
    const double ni = (double)(pb.iscale ? pb.iscale[mi] : ntab[mi]);
    if (MODE == 3) {  // forward, last pass: the ModDown combine
        // out = (acc - v) P^-1 (+ add) with v this transform's output:
        // |acc - v| < 4 q, so the product and the sum stay exact
        const u64 grp = pidx / (u64)pb.nlimb, lN = (u64)mi * dp.N, half = (u64)dp.nq * dp.N;
        const u64 *accp = pb.comb_acc + grp * pb.comb_acc_stride + lN;
        const u64 *addp = pb.comb_add ? pb.comb_add + (grp >> 1) * pb.comb_add_stride + (grp & 1) * half + lN
                                      : nullptr;
        u64 *outp = pb.comb_out + (grp >> 1) * pb.comb_out_stride + (grp & 1) * half + lN;
        const double pinv = u64_to_d(dp.pinv[mi]);
        ulonglong2 a2[8], b2[8];
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const u32 e = 2 * (tid + (u32)i * nthreads);
            const u64 g = ((u64)tile * cols + (e >> LOG_S)) * S + (e & (S - 1));
            a2[i] = *reinterpret_cast<const ulonglong2 *>(accp + g);
            if (addp) b2[i] = *reinterpret_cast<const ulonglong2 *>(addp + g);
        }
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const u32 e = 2 * (tid + (u32)i * nthreads);
            const u32 cc = e >> LOG_S, a = e & (S - 1);
            const u64 g = ((u64)tile * cols + cc) * S + a;
            double r0 = mulmod_d(u64_to_d(a2[i].x) - lds[lds_idx<LOG_S, BLOCKS>(cc, a)], pinv, q, qinv);
            double r1 = mulmod_d(u64_to_d(a2[i].y) - lds[lds_idx<LOG_S, BLOCKS>(cc, a + 1)], pinv, q, qinv);
            if (addp) {
                r0 += u64_to_d(b2[i].x);
                r1 += u64_to_d(b2[i].y);
            }
            ulonglong2 o;
            o.x = d_to_canonical(r0, q, qinv);
            o.y = d_to_canonical(r1, q, qinv);
            *reinterpret_cast<ulonglong2 *>(outp + g) = o;
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < 8; i++) {
        u32 e = 2 * (tid + (u32)i * nthreads);
        u32 a, cc;
        u64 g;
        if (BLOCKS) { cc = e >> LOG_S; a = e & (S - 1); g = ((u64)tile * cols + cc) * S + a; }
        else { a = e / (u32)cols; cc = e % (u32)cols; g = (hi_col * S + a) * stride + lo0 + cc; }
        double d0 = lds[lds_idx<LOG_S, BLOCKS>(cc, a)];
        double d1 = BLOCKS ? lds[lds_idx<LOG_S, BLOCKS>(cc, a + 1)] : lds[lds_idx<LOG_S, BLOCKS>(cc + 1, a)];
        ulonglong2 o;
        if (final_) {
            if (INVERSE) {
                d0 = mulmod_d(d0, ni, q, qinv);
                d1 = mulmod_d(d1, ni, q, qinv);
            }
            if (pb.out_f64) {
                o.x = (u64)__double_as_longlong(canon_d(d0, q, qinv));
                o.y = (u64)__double_as_longlong(canon_d(d1, q, qinv));
            } else {
                o.x = d_to_canonical(d0, q, qinv);
                o.y = d_to_canonical(d1, q, qinv);
            }
        } else {
            o.x = (u64)__double_as_longlong(d0);
            o.y = (u64)__double_as_longlong(d1);
        }
        *reinterpret_cast<ulonglong2 *>(poly + g) = o;
    }
}

template <int LOG_S, bool INVERSE, bool BLOCKS, int MODE = 0>
__global__ void __launch_bounds__(256) ntt_fast_kernel(DevParams dp, PolyBatch pb, int s0, int cols, int final_)
{
    extern __shared__ double lds[];
    u64 *poly;
    int mi;
    u64 pidx = blockIdx.x;
    if ((MODE == 1 || MODE == 2) && (pb.count & 7) == 0) {
        // workgroups are dealt to the 8 XCDs round-robin: remap so that the
        // limbs of one group run on one XCD and share its L2 copy of the
        // group's conversion inputs
        const u64 j = blockIdx.x >> 3, nl = (u64)pb.nlimb;
        pidx = ((j / nl) * 8 + (blockIdx.x & 7)) * nl + j % nl;
    }
    const u64 *src;  // what the first pass reads
    if (!poly_of_block(dp, pb, pidx, poly, mi, &src)) return;
    const double *tw = (INVERSE ? dp.itwd : dp.twd) + (u64)mi * dp.N;
    ntt_fast_body<LOG_S, INVERSE, BLOCKS, MODE>(dp, pb, pidx, poly, src, mi, blockIdx.y, dp.N, tw, dp.ninv, s0,
                                                cols, final_, lds);
}

struct FastPass {
    int s0, log_s, blocks, cols;
};

// Two passes for 2^10 <= N <= 2^17: columns of the top half of the stages,
// then contiguous blocks.  At most 4096 elements per workgroup.
static int plan_fast(int log_n, FastPass *p)
{
    if (log_n < 10 || log_n > 17) return 0;
    int k1 = log_n / 2, k2 = log_n - k1;  // k1 <= k2, both in [5, 8]
    u32 stride1 = 1u << k2;
    p[0] = {0, k1, 0, (int)std::min<u32>(4096u >> k1, stride1)};
    p[1] = {k1, k2, 1, (int)std::min<u32>(4096u >> k2, 1u << k1)};
    return 2;
}

template <bool INV, bool BLOCKS, int MODE = 0>
static void launch_fast_one(int log_s, dim3 grid, dim3 block, size_t lds, hipStream_t s, const DevParams &dp,
                            const PolyBatch &b, int s0, int cols, int final_)
{
    switch (log_s) {
    case 5: hipLaunchKernelGGL((ntt_fast_kernel<5, INV, BLOCKS, MODE>), grid, block, lds, s, dp, b, s0, cols, final_); break;
    case 6: hipLaunchKernelGGL((ntt_fast_kernel<6, INV, BLOCKS, MODE>), grid, block, lds, s, dp, b, s0, cols, final_); break;
    case 7: hipLaunchKernelGGL((ntt_fast_kernel<7, INV, BLOCKS, MODE>), grid, block, lds, s, dp, b, s0, cols, final_); break;
    case 8: hipLaunchKernelGGL((ntt_fast_kernel<8, INV, BLOCKS, MODE>), grid, block, lds, s, dp, b, s0, cols, final_); break;
    default: hipLaunchKernelGGL((ntt_fast_kernel<9, INV, BLOCKS, MODE>), grid, block, lds, s, dp, b, s0, cols, final_); break;
    }
}

// ---- mixed ring degrees in one launch per pass ------------------------------
//
// For 2^12 <= N <= 2^17 both passes of the two-pass plan have 4096-element
// tiles and 256-lane workgroups (columns: LOG_S = floor(log N / 2), 4096 /
// 2^LOG_S sub-transforms per tile; blocks: LOG_S = ceil(log N / 2)), so one
// launch can hold polynomials of several degrees: workgroup b finds its group
// (uniform over the workgroup), its polynomial and tile, and runs the pass
// body of that degree with that degree's twiddles.

template <bool INVERSE, bool BLOCKS, int LOG_S>
__device__ __forceinline__ void mixed_body(const DevParams &dp, const PolyBatch &pb, u64 *poly, int mi, u32 tile,
                                           u32 N_, const double *tw, const u64 *ntab, int final_, double *lds)
{
    const int log_n = 31 - __clz((int)N_);
    const int s0 = BLOCKS ? log_n - LOG_S : 0;
    ntt_fast_body<LOG_S, INVERSE, BLOCKS, 0>(dp, pb, 0, poly, poly, mi, tile, N_, tw, ntab, s0, 4096 >> LOG_S,
                                             final_, lds);
}

template <bool INVERSE, bool BLOCKS>
__global__ void __launch_bounds__(256) ntt_mixed_kernel(DevParams dp, MixedArgs ma, int final_)
{
    extern __shared__ double lds[];
    const u64 b = blockIdx.x;
    int gi = 0;
    while (gi + 1 < ma.ng && b >= ma.g[gi + 1].block0) gi++;
    const MixedGroup &G = ma.g[gi];
    const u32 N_ = 1u << G.log_n;
    const u32 tiles = N_ / 4096u;
    const u64 local = b - G.block0;
    const u64 p = local / tiles;
    const u32 tile = (u32)(local % tiles);
    const int mi = G.limb0 + (int)(p % (u64)G.nlimb);
    u64 *poly = G.base + p * N_;
    const int di = G.log_n - MIXED_LOG_MIN;
    const double *tw = ma.tw[di] + (u64)mi * N_;
    const u64 *ntab = ma.ninv[di];
    const PolyBatch pb{};
    const int ls = BLOCKS ? G.log_n - G.log_n / 2 : G.log_n / 2;
    if (ls == 6) mixed_body<INVERSE, BLOCKS, 6>(dp, pb, poly, mi, tile, N_, tw, ntab, final_, lds);
    else if (ls == 7) mixed_body<INVERSE, BLOCKS, 7>(dp, pb, poly, mi, tile, N_, tw, ntab, final_, lds);
    else if (ls == 8) mixed_body<INVERSE, BLOCKS, 8>(dp, pb, poly, mi, tile, N_, tw, ntab, final_, lds);
    else mixed_body<INVERSE, BLOCKS, 9>(dp, pb, poly, mi, tile, N_, tw, ntab, final_, lds);
}

int launch_ntt_mixed(Ctx *c, const MixedArgs &ma0, bool inverse, hipStream_t s)
{
    MixedArgs ma = ma0;
    u64 blocks = 0;
    for (int g = 0; g < ma.ng; g++) {
        ma.g[g].block0 = blocks;
        blocks += ma.g[g].npoly * ((1ull << ma.g[g].log_n) / 4096);
    }
    if (blocks == 0) return LC_OK;
    if (blocks > 0x7fffffffull) return fail(c, LC_EINVAL, "too many polynomials in one NTT launch");
    const size_t lds = fast_lds_bytes(8, false);  // the largest tile layout of the degrees 2^12 .. 2^17
    const dim3 grid((u32)blocks), block(256);
    if (!inverse) {
        hipLaunchKernelGGL((ntt_mixed_kernel<false, false>), grid, block, lds, s, c->dp, ma, 0);
        LC_HIP(c, hipGetLastError());
        hipLaunchKernelGGL((ntt_mixed_kernel<false, true>), grid, block, lds, s, c->dp, ma, 1);
    } else {
        hipLaunchKernelGGL((ntt_mixed_kernel<true, true>), grid, block, lds, s, c->dp, ma, 0);
        LC_HIP(c, hipGetLastError());
        hipLaunchKernelGGL((ntt_mixed_kernel<true, false>), grid, block, lds, s, c->dp, ma, 1);
    }
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// Pass plan of the generic kernel: one pass up to N = 4096, two passes above.
static int plan_passes(int log_n, PassArgs *pass)
{
    if (log_n <= 12) {
        pass[0] = {0, log_n, 1, 1};
        return 1;
    }
    int k1 = log_n / 2, k2 = log_n - k1;
    pass[0] = {0, k1, NTT_TILE >> k1, 0};
    pass[1] = {k1, k2, NTT_TILE >> k2, 1};
    return 2;
}

static int launch_fast(Ctx *c, const PolyBatch &b, const FastPass *fp, hipStream_t s, bool inverse)
{
    const u64 npoly = b.count * (u64)b.nlimb;
    for (int k = 0; k < 2; k++) {
        int i = inverse ? 1 - k : k;
        const FastPass &P = fp[i];
        int final_ = inverse ? (i == 0) : (i == 1);
        u32 S = 1u << P.log_s;
        u32 tiles = (u32)(c->N >> P.log_s) / (u32)P.cols;
        dim3 grid((u32)npoly, tiles), block((u32)P.cols * (S / 16));
        size_t lds = fast_lds_bytes(P.log_s, P.blocks);
        if (inverse) {
            if (P.blocks) launch_fast_one<true, true>(P.log_s, grid, block, lds, s, c->dp, b, P.s0, P.cols, final_);
            else launch_fast_one<true, false>(P.log_s, grid, block, lds, s, c->dp, b, P.s0, P.cols, final_);
        } else if (k == 0 && b.conv == 1) {  // first forward pass (columns) with the ModUp conversion
            launch_fast_one<false, false, 1>(P.log_s, grid, block, lds, s, c->dp, b, P.s0, P.cols, final_);
        } else if (k == 0 && b.conv == 2) {  // ... with the ModDown conversion
            launch_fast_one<false, false, 2>(P.log_s, grid, block, lds, s, c->dp, b, P.s0, P.cols, final_);
        } else if (k == 1 && b.comb_out) {  // last forward pass (blocks) with the ModDown combine
            launch_fast_one<false, true, 3>(P.log_s, grid, block, lds, s, c->dp, b, P.s0, P.cols, final_);
        } else {
            if (P.blocks) launch_fast_one<false, true>(P.log_s, grid, block, lds, s, c->dp, b, P.s0, P.cols, final_);
            else launch_fast_one<false, false>(P.log_s, grid, block, lds, s, c->dp, b, P.s0, P.cols, final_);
        }
        LC_HIP(c, hipGetLastError());
    }
    return LC_OK;
}

static int launch(Ctx *c, const PolyBatch &b, hipStream_t s, bool inverse)
{
    u64 npoly = b.count * (u64)b.nlimb;
    if (npoly == 0) return LC_OK;
    if (npoly > 0x7fffffffull) return fail(c, LC_EINVAL, "too many polynomials in one NTT batch");
    FastPass fp[2];
    if (plan_fast(c->log_n, fp)) {
        // Both passes run over one sub-batch of about ntt_sub_kb KiB before the
        // next, so that the first pass's output can still sit in the
        // memory-side cache when the second pass reads it.  Sub-batches hold
        // whole digit groups when own-digit limbs are skipped.
        u64 gsub = b.count;
        if (c->tune.ntt_sub_kb > 0) {
            const u64 group_bytes = (u64)b.nlimb * c->N * sizeof(u64);
            gsub = std::max<u64>(1, ((u64)c->tune.ntt_sub_kb << 10) / group_bytes);
            if (b.skip_own_digit) gsub = std::max<u64>((u64)c->dnum, gsub / c->dnum * c->dnum);
            if (b.comb_out) gsub = std::max<u64>(2, gsub / 2 * 2);  // whole ciphertexts
        }
        for (u64 g0 = 0; g0 < b.count; g0 += gsub) {
            PolyBatch sb = b;
            sb.base = b.base + g0 * b.gstride * c->N;
            if (b.in_base) sb.in_base = b.in_base + g0 * b.in_gstride * c->N;
            sb.count = std::min(gsub, b.count - g0);
            if (b.conv == 1) sb.conv_y = b.conv_y + (g0 / (u64)c->dnum) * b.conv_stride;  // g0 % dnum == 0
            if (b.conv == 2) sb.conv_y = b.conv_y + g0 * b.conv_stride;
            if (b.comb_out) {  // groups are (ciphertext, component): g0 is even
                sb.comb_acc = b.comb_acc + g0 * b.comb_acc_stride;
                if (b.comb_add) sb.comb_add = b.comb_add + g0 / 2 * b.comb_add_stride;
                sb.comb_out = b.comb_out + g0 / 2 * b.comb_out_stride;
            }
            int rc = launch_fast(c, sb, fp, s, inverse);
            if (rc) return rc;
        }
        return LC_OK;
    }
    if (b.conv || b.comb_out || b.out_f64) return fail(c, LC_EINVAL, "fused key-switch transforms need 2^10 <= N <= 2^17");
    if (b.in_base) return fail(c, LC_EINVAL, "an out-of-place transform needs 2^10 <= N <= 2^17");
    PassArgs pass[2];
    int np = plan_passes(c->log_n, pass);
    for (int k = 0; k < np; k++) {
        int i = inverse ? np - 1 - k : k;
        PassArgs pa = pass[i];
        pa.final_ = inverse ? (i == 0) : (i == np - 1);
        u32 tiles = (u32)(c->N >> pa.log_s) / (u32)pa.cols;
        dim3 grid((u32)npoly, tiles);
        if (inverse)
            hipLaunchKernelGGL(ntt_pass_kernel<true>, grid, dim3(NTT_THREADS), 0, s, c->dp, b, pa);
        else
            hipLaunchKernelGGL(ntt_pass_kernel<false>, grid, dim3(NTT_THREADS), 0, s, c->dp, b, pa);
        LC_HIP(c, hipGetLastError());
    }
    return LC_OK;
}

int launch_ntt_fwd(Ctx *c, const PolyBatch &b, hipStream_t s) { return launch(c, b, s, false); }
int launch_ntt_inv(Ctx *c, const PolyBatch &b, hipStream_t s) { return launch(c, b, s, true); }

}  // namespace lc
