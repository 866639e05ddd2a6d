// Element-wise homomorphic operations and the fused lazy-triple kernel of
// the pairwise distances (Algorithm 1, Server Executes; Methods, Lazy
// Relinearization).  All operate in the NTT domain, one lane per coefficient.
#include "lc_internal.h"

namespace lc {

constexpr int EW_THREADS = 256;

static inline dim3 grid_for(u64 n, int threads)
{
    u64 b = (n + threads - 1) / threads;
    return dim3((u32)b);
}

// ---- add / sub -------------------------------------------------------------

__global__ void __launch_bounds__(EW_THREADS)
add_sub_kernel(DevParams dp, const u64 *a, const u64 *b, u64 *out, u64 total, int sub)
{
    u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int l = (int)((e >> dp.log_n) % (u64)dp.nq);
    u64 q = dp.mc[l].m;
    out[e] = sub ? sub_mod(a[e], b[e], q) : add_mod(a[e], b[e], q);
}

int launch_add_sub(Ctx *c, const u64 *a, const u64 *b, u64 *out, u64 count, int ncomp, int sub, hipStream_t s)
{
    u64 total = count * (u64)ncomp * c->nq * c->N;
    if (!total) return LC_OK;
    hipLaunchKernelGGL(add_sub_kernel, grid_for(total, EW_THREADS), dim3(EW_THREADS), 0, s, c->dp, a, b, out,
                       total, sub);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// ---- tensor product (CKKS.Mult without relinearization) --------------------

__global__ void __launch_bounds__(EW_THREADS)
tensor_kernel(DevParams dp, const u64 *a, const u64 *b, u64 *out3, u64 total)
{
    u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // over count * nq * N
    if (e >= total) return;
    u64 S = (u64)dp.nq << dp.log_n;
    u64 ct = e / S, r = e % S;
    int l = (int)(r >> dp.log_n);
    const ModConst &mc = dp.mc[l];
    const u64 *A = a + ct * 2 * S;
    u64 a0 = A[r], a1 = A[S + r];
    u64 *O = out3 + ct * 3 * S;
    Split3 s0, s1, s2;
    split_zero(s0);
    split_zero(s1);
    split_zero(s2);
    if (b) {
        const u64 *B = b + ct * 2 * S;
        u64 b0 = B[r], b1 = B[S + r];
        split_mac(s0, a0, b0);
        split_mac(s1, a0, b1);
        split_mac(s1, a1, b0);
        split_mac(s2, a1, b1);
        O[r] = reduce_split(s0, mc);
        O[S + r] = reduce_split(s1, mc);
        O[2 * S + r] = reduce_split(s2, mc);
    } else {
        split_sq(s0, a0);
        split_mac(s1, a0, a1);
        split_sq(s2, a1);
        O[r] = reduce_split_sq(s0, mc);
        u64 x = reduce_split(s1, mc);
        O[S + r] = add_mod(x, x, mc.m);
        O[2 * S + r] = reduce_split_sq(s2, mc);
    }
}

int launch_tensor(Ctx *c, const u64 *a, const u64 *b, u64 *out3, u64 count, hipStream_t s)
{
    u64 total = count * c->nq * c->N;
    if (!total) return LC_OK;
    hipLaunchKernelGGL(tensor_kernel, grid_for(total, EW_THREADS), dim3(EW_THREADS), 0, s, c->dp, a, b, out3, total);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// ---- plaintext multiply and masked aggregation (ServerUpdate) -------------

__global__ void __launch_bounds__(EW_THREADS)
mul_plain_kernel(DevParams dp, const u64 *ct, const u64 *pt, u64 *out, u64 total)
{
    u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // over count * nq * N
    if (e >= total) return;
    u64 S = (u64)dp.nq << dp.log_n;
    u64 k = e / S, r = e % S;
    int l = (int)(r >> dp.log_n);
    const ModConst &mc = dp.mc[l];
    u64 p = pt[k * S + r];
    out[k * 2 * S + r] = mul_mod(ct[k * 2 * S + r], p, mc);
    out[k * 2 * S + S + r] = mul_mod(ct[k * 2 * S + S + r], p, mc);
}

int launch_mul_plain(Ctx *c, const u64 *ct, const u64 *pt, u64 *out, u64 count, hipStream_t s)
{
    u64 total = count * c->nq * c->N;
    if (!total) return LC_OK;
    hipLaunchKernelGGL(mul_plain_kernel, grid_for(total, EW_THREADS), dim3(EW_THREADS), 0, s, c->dp, ct, pt, out,
                       total);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// out[k][comp][l][j] = sum_i cts[i][k][comp][l][j] * masks[i][l][j]
//
// Workgroup = (256 x COEF consecutive coefficients of one (limb, position)
// range, ROWS consecutive (k, comp) rows).  A lane owns COEF adjacent
// coefficients (COEF = 2: 16-byte accesses) and their ROWS row accumulators;
// clients go in groups of 8 whose mask values are loaded once into
// registers and used for every row, so the masks cost 1 / ROWS of a read
// per output instead of one (the client ciphertexts are read exactly once).
// The row tiles of one coefficient window are the grid's fastest index, so
// the workgroups that re-read a window's masks run back to back and find
// them in L2 rather than HBM.
// FP64 Barrett products of residues below q come back with |r| < q; a
// reduction follows every 4 products, so the accumulators stay below
// 4.5 q < 2^53.  The shape (COEF, ROWS) is a tuning choice ("ms_shape").
constexpr int MS_TILE = 256;

template <int COEF, int ROWS>
__global__ void __launch_bounds__(MS_TILE)
masked_sum_kernel(DevParams dp, const u64 *__restrict__ cts, int n, int len, const u64 *__restrict__ masks,
                  u64 *__restrict__ out)
{
    const u64 S = (u64)dp.nq << dp.log_n;
    const u64 r = ((u64)blockIdx.y * MS_TILE + threadIdx.x) * COEF;  // (limb, coefficient), COEF | N
    if (r >= S) return;
    const int rows = 2 * len, row0 = blockIdx.x * ROWS;
    const int l = (int)(r >> dp.log_n);
    const double q = dp.mc[l].qd, qinv = dp.mc[l].qinv;
    const u64 client_stride = (u64)len * 2 * S;
    double acc[ROWS][COEF];
#pragma unroll
    for (int t = 0; t < ROWS; t++)
#pragma unroll
        for (int e = 0; e < COEF; e++) acc[t][e] = 0.0;
    // Every load is unconditional, from a clamped client and row: a load
    // under a condition makes the wave wait for all loads in flight where
    // the branches join.  A client past n gets mask 0, so its (re-read)
    // ciphertext adds nothing; rows past the end are computed, not stored.
    for (int i0 = 0; i0 < n; i0 += 8) {
        double m[8][COEF];
        const u64 *cbase[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int iu = min(i0 + u, n - 1);
            const bool live = i0 + u < n;
            cbase[u] = cts + (u64)iu * client_stride + r;
            if (COEF == 2) {
                const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(masks + (u64)iu * S + r);
                m[u][0] = live ? u64_to_d(v.x) : 0.0;
                m[u][COEF - 1] = live ? u64_to_d(v.y) : 0.0;
            } else {
                const u64 v = masks[(u64)iu * S + r];
                m[u][0] = live ? u64_to_d(v) : 0.0;
            }
        }
#pragma unroll
        for (int t = 0; t < ROWS; t++) {
            const u64 rt = (u64)min(row0 + t, rows - 1);
            double c[8][COEF];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const u64 *src = cbase[u] + rt * S;
                if (COEF == 2) {
                    const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(src);
                    c[u][0] = u64_to_d(v.x);
                    c[u][COEF - 1] = u64_to_d(v.y);
                } else {
                    c[u][0] = u64_to_d(*src);
                }
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
#pragma unroll
                for (int e = 0; e < COEF; e++) {
                    acc[t][e] += mulmod_d(c[u][e], m[u][e], q, qinv);
                    if (u == 3 || u == 7) acc[t][e] = reduce_d(acc[t][e], q, qinv);
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < ROWS; t++) {
        if (row0 + t < rows) {
            u64 *o = out + (u64)(row0 + t) * S + r;
            if (COEF == 2) {
                ulonglong2 v;
                v.x = d_to_canonical(acc[t][0], q, qinv);
                v.y = d_to_canonical(acc[t][COEF - 1], q, qinv);
                *reinterpret_cast<ulonglong2 *>(o) = v;
            } else {
                *o = d_to_canonical(acc[t][0], q, qinv);
            }
        }
    }
}

template <int COEF, int ROWS>
static void launch_ms(hipStream_t s, const DevParams &dp, u64 S, const u64 *cts, int n, int len, const u64 *masks,
                      u64 *out)
{
    // x: row tiles, y: coefficient windows (at most 48 limbs x 2^17 / 256 = 24576)
    dim3 grid((u32)((2 * len + ROWS - 1) / ROWS), (u32)((S / COEF + MS_TILE - 1) / MS_TILE));
    hipLaunchKernelGGL((masked_sum_kernel<COEF, ROWS>), grid, dim3(MS_TILE), 0, s, dp, cts, n, len, masks, out);
}

int launch_masked_sum(Ctx *c, const u64 *cts, int n, int len, const u64 *masks, u64 *out, hipStream_t s)
{
    const u64 S = (u64)c->nq * c->N;
    if (len < 1 || n < 1) return LC_OK;
    switch (c->tune.ms_shape) {  // COEF x ROWS
    case 0: launch_ms<1, 16>(s, c->dp, S, cts, n, len, masks, out); break;
    case 1: launch_ms<2, 8>(s, c->dp, S, cts, n, len, masks, out); break;
    default: launch_ms<2, 16>(s, c->dp, S, cts, n, len, masks, out); break;
    }
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// ---- ServerUpdate with an encrypted mask --------------------------------------
//
// trip[k] = sum_i ct_i[k] (x) mask_i: the tensor product (a0 m0, a0 m1 + a1 m0,
// a1 m1) of every client's packed ciphertext with that client's encrypted
// mask (Enc_pk of its weight), summed over clients before one
// relinearization per k.  Same structure as the masked sum: a lane owns one
// coefficient and MA_ROWS packed ciphertexts, clients go in pairs whose mask
// components sit in registers, every client ciphertext is read once, and a
// coefficient window's row tiles run back to back (the grid's fastest index)
// so that their re-reads of the masks come from L2.  FP64 Barrett products
// below q (|r| < q), a reduction after every 4 products per accumulator.
constexpr int MA_TILE = 256;
constexpr int MA_ROWS = 8;

__global__ void __launch_bounds__(MA_TILE)
mask_mul_acc_kernel(DevParams dp, const u64 *__restrict__ cts, int n, int len, int row_len,
                    const u64 *__restrict__ masks, u64 *__restrict__ trip)
{
    const u64 S = (u64)dp.nq << dp.log_n;
    const u64 r = (u64)blockIdx.y * MA_TILE + threadIdx.x;  // (limb, coefficient)
    if (r >= S) return;
    const int k0 = blockIdx.x * MA_ROWS;
    const int l = (int)(r >> dp.log_n);
    const double q = dp.mc[l].qd, qinv = dp.mc[l].qinv;
    const u64 client_stride = (u64)row_len * 2 * S;  // a client's row holds row_len ciphertexts, of which len are used
    double acc[MA_ROWS][3];
#pragma unroll
    for (int t = 0; t < MA_ROWS; t++) acc[t][0] = acc[t][1] = acc[t][2] = 0.0;
    for (int i0 = 0; i0 < n; i0 += 2) {
        // every load of the round is issued before any is used: rows past len
        // re-read row len - 1 (their sums are not stored), a missing second
        // client re-reads the first with a zero mask
        u64 mv[2][2], cv[2][MA_ROWS][2];
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const u64 i = (u64)min(i0 + u, n - 1);
            mv[u][0] = masks[i * 2 * S + r];
            mv[u][1] = masks[i * 2 * S + S + r];
#pragma unroll
            for (int t = 0; t < MA_ROWS; t++) {
                const u64 *c = cts + i * client_stride + (u64)min(k0 + t, len - 1) * 2 * S + r;
                cv[u][t][0] = c[0];
                cv[u][t][1] = c[S];
            }
        }
        double m[2][2];
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const bool live = i0 + u < n;
            m[u][0] = live ? u64_to_d(mv[u][0]) : 0.0;
            m[u][1] = live ? u64_to_d(mv[u][1]) : 0.0;
        }
#pragma unroll
        for (int t = 0; t < MA_ROWS; t++) {
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const double a0 = u64_to_d(cv[u][t][0]), a1 = u64_to_d(cv[u][t][1]);
                acc[t][0] += mulmod_d(a0, m[u][0], q, qinv);
                acc[t][1] += mulmod_d(a0, m[u][1], q, qinv) + mulmod_d(a1, m[u][0], q, qinv);
                acc[t][2] += mulmod_d(a1, m[u][1], q, qinv);
            }
            acc[t][0] = reduce_d(acc[t][0], q, qinv);
            acc[t][1] = reduce_d(acc[t][1], q, qinv);
            acc[t][2] = reduce_d(acc[t][2], q, qinv);
        }
    }
#pragma unroll
    for (int t = 0; t < MA_ROWS; t++) {
        if (k0 + t < len) {
            u64 *o = trip + (u64)(k0 + t) * 3 * S + r;
            o[0] = d_to_canonical(acc[t][0], q, qinv);
            o[S] = d_to_canonical(acc[t][1], q, qinv);
            o[2 * S] = d_to_canonical(acc[t][2], q, qinv);
        }
    }
}

int launch_mask_mul_acc(Ctx *c, const u64 *cts, int n, int len, int row_len, const u64 *masks, u64 *trip,
                        hipStream_t s)
{
    const u64 S = (u64)c->nq * c->N;
    if (len < 1 || n < 1) return LC_OK;
    if (len > row_len) return fail(c, LC_EINVAL, "chunk longer than the client row");
    // x: row tiles, y: coefficient windows (at most 48 limbs x 2^17 / 256 = 24576)
    dim3 grid((u32)((len + MA_ROWS - 1) / MA_ROWS), (u32)((S + MA_TILE - 1) / MA_TILE));
    hipLaunchKernelGGL(mask_mul_acc_kernel, grid, dim3(MA_TILE), 0, s, c->dp, cts, n, len, row_len, masks, trip);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// ---- fused subtract / square / lazy accumulate over all pairs --------------
//
// Workgroup = (tile of T coefficients, limb l, chunk of pairs).  PT_KB packed
// ciphertexts at a time, the tiles of all n clients (both components) are
// staged in LDS once -- as exact doubles -- and every pair of the chunk reads
// them from there.  A lane owns one coefficient of PPT pairs and keeps their
// triple accumulators in registers across all k.  T and PPT are tuning
// parameters (lc_set_tuning); the defaults come from measurements on MI355X.
//
// LDS layout is [client * 2 + comp][PT_KB][T], so with T and PT_KB known at
// compile time a lane reads all of its operands at one base address per
// client plus immediate offsets.  Ciphertexts past len are staged as zeros
// and pair slots past P compute on clients (0, 1) and are not stored, so the
// inner loop carries no branches and the compiler can issue every LDS read of
// a k-step before the arithmetic that waits on them.  (Issuing a batch's
// staging loads together, or double buffering the tile through registers,
// measured no faster on MI355X: the staging is hidden by the second
// workgroup on each CU.)
//
// Arithmetic is the FP64 Barrett form of modarith.h: differences x = a - b
// lie in (-q, q), so |x y / q| < q < 2^50; the quotient estimate rint(fl(fl(x
// y) fl(1/q))) is off by at most 1/2 + 3 2^-53 |x y / q| < 7/8, giving each
// product as an integer r with |r| < 7q/8.  The accumulators (|acc| <= q/2 +
// 1 after a reduction) take two batches of PT_KB = 4 such products before the
// next reduction (the cross term is accumulated once and doubled at the end),
// so they stay below 7.5 q + 1 < 2^53 and every value is exact; the last
// batch always reduces.  The canonical residue is taken once at the end.

constexpr int PT_MAXN = 64;     // clients per call
constexpr int PT_KB = 4;        // packed ciphertexts staged per barrier
constexpr size_t PT_LDS = 64 * 1024;
constexpr int PT_BUF = (int)(PT_LDS / 2 / sizeof(double));  // most doubles per tile buffer
constexpr int PT_NC = 4;        // most wave copies per wave and batch

__device__ __forceinline__ void pair_of_index(int p, int n, int &i, int &j)
{
    int row = 0, base = 0;
    while (base + (n - 1 - row) <= p) {
        base += n - 1 - row;
        row++;
    }
    i = row;
    j = row + 1 + (p - base);
}

__host__ __device__ inline int pair_index(int n, int i, int j) { return i * (2 * n - i - 1) / 2 + (j - i - 1); }

template <int T, int PPT>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(PPT <= 4 ? 6 : 4)))
pair_triples_kernel(DevParams dp, const u64 *__restrict__ cts, int n, int len, int P, u64 *d01, u64 d01_stride,
                    u64 *d2, u64 d2_stride, int accumulate)
{
    // two tile buffers, each [n * 2][PT_KB][T] (rows of T coefficients,
    // rounded up to whole wave copies: bufsz doubles)
    extern __shared__ __attribute__((aligned(16))) double tile0[];
    constexpr int ROW = PT_KB * T;    // doubles per (client, comp)
    const int G = blockDim.y;         // pair groups
    const int lane = threadIdx.x, g = threadIdx.y;
    const int tid = g * T + lane;
    const int nthreads = T * G;
    const int l = blockIdx.y;
    const u64 N = dp.N;
    const u64 S = (u64)dp.nq * N;
    const double q = dp.mc[l].qd, qinv = dp.mc[l].qinv;
    const int staged = n * 2 * ROW;

    // pair r of this lane is p = pbase + r G; its two clients' tile offsets
    const int pbase = blockIdx.z * (G * PPT) + g;
    int oa[PPT], ob[PPT];
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        int p = pbase + r * G, i = 0, j = 1;
        if (p < P) pair_of_index(p, n, i, j);
        oa[r] = i * 2 * ROW + lane;
        ob[r] = j * 2 * ROW + lane;
    }
    double acc[PPT][3];
#pragma unroll
    for (int r = 0; r < PPT; r++) acc[r][0] = acc[r][1] = acc[r][2] = 0.0;

    // Staging of a batch of PT_KB packed ciphertexts.  Row rw = (client * 2 +
    // comp) * PT_KB + kk of a buffer holds the T coefficients of the tile.
    // When the thread count is a whole number of waves, each wave copies
    // groups of 128 / T rows straight from HBM into LDS (16 bytes per lane,
    // lane i landing 16 i bytes past the group's start: no registers, and the
    // copy of the next batch runs while this one computes); each lane then
    // turns the 16 bytes it copied into doubles in place, zeroing packed
    // ciphertexts past len.  Otherwise each thread stages elements one by one.
    const u64 client_stride = (u64)len * 2 * S;
    const u64 off = (u64)l * N + (u64)blockIdx.x * T;
    const int nrows = n * 2 * PT_KB;
    constexpr int RPI = 128 / T;  // rows per wave copy
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), nwaves = nthreads >> 6;
    const int wl = tid & 63, ncopy = (nrows + RPI - 1) / RPI;
    const bool dma = nthreads % 64 == 0 && (ncopy + nwaves - 1) / nwaves <= PT_NC;
    double *const tile1 = tile0 + ncopy * RPI * T;
    auto row_src = [&](int rw, int k0) -> const u64 * {
        rw = min(rw, nrows - 1);  // rows past the last of a copy group re-read it
        const int cc = rw / PT_KB, k = min(k0 + rw % PT_KB, len - 1);
        return cts + (u64)(cc >> 1) * client_stride + (u64)k * 2 * S + (u64)(cc & 1) * S + off;
    };
    // a wave's copies (at most PT_NC, else the thread stages one by one):
    // their source addresses without the ciphertext index, computed once
    const int nmine = dma ? (ncopy - wave + nwaves - 1) / nwaves : 0;
    const u64 *cbase[PT_NC];
    int ckk[PT_NC];
#pragma unroll
    for (int i = 0; i < PT_NC; i++) {
        const int rw = min((wave + i * nwaves) * RPI + wl / (T / 2), nrows - 1);
        const int cc = rw / PT_KB;
        ckk[i] = rw % PT_KB;
        cbase[i] = cts + (u64)(cc >> 1) * client_stride + (u64)(cc & 1) * S + off + (wl % (T / 2)) * 2;
    }
    auto issue = [&](int k0, double *buf) {
        if (!dma) return;
#pragma unroll
        for (int i = 0; i < PT_NC; i++) {
            if (i >= nmine) break;
            const u64 *src = cbase[i] + (u64)min(k0 + ckk[i], len - 1) * 2 * S;
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                             (__attribute__((address_space(3))) void *)(buf + (wave + i * nwaves) * RPI * T),
                                             16, 0, 0);
        }
    };
    auto finish = [&](int k0, double *buf) {
        if (dma) {
            __builtin_amdgcn_s_waitcnt(0);  // this wave's copies have landed
#pragma unroll
            for (int i = 0; i < PT_NC; i++) {
                if (i >= nmine) break;
                double *d = buf + (wave + i * nwaves) * RPI * T + wl * 2;
                const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(d);
                const bool live = k0 + ckk[i] < len;
                // a residue x < 2^52 with the exponent bits of 2^52 set is the
                // double 2^52 + x: one OR instead of a conversion, and the
                // offset cancels in every difference of two clients' values
                // (exact: both lie in [2^52, 2^53))
                d[0] = live ? __longlong_as_double((long long)(v.x | 0x4330000000000000ull)) : 0.0;
                d[1] = live ? __longlong_as_double((long long)(v.y | 0x4330000000000000ull)) : 0.0;
            }
        } else {
            for (int e = tid; e < staged; e += nthreads) {
                const int rw = e / T;
                buf[e] = k0 + rw % PT_KB < len ? u64_to_d(row_src(rw, k0)[e % T]) : 0.0;
            }
        }
    };
    auto compute = [&](const double *tb) {
#pragma unroll
        for (int kk = 0; kk < PT_KB; kk++) {
#pragma unroll
            for (int r = 0; r < PPT; r++) {
                double x0 = tb[oa[r] + kk * T] - tb[ob[r] + kk * T];
                double x1 = tb[oa[r] + ROW + kk * T] - tb[ob[r] + ROW + kk * T];
                acc[r][0] += mulmod_d(x0, x0, q, qinv);
                acc[r][1] += mulmod_d(x0, x1, q, qinv);
                acc[r][2] += mulmod_d(x1, x1, q, qinv);
            }
            // keep the compiler from hoisting every LDS read of the batch
            // (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    auto reduce_all = [&]() {
#pragma unroll
        for (int r = 0; r < PPT; r++) {
            acc[r][0] = reduce_d(acc[r][0], q, qinv);
            acc[r][1] = reduce_d(acc[r][1], q, qinv);
            acc[r][2] = reduce_d(acc[r][2], q, qinv);
        }
    };
    // Batch b computes from buffer b % 2 while batch b + 1 is copied into
    // the other.  One barrier per batch: after it every wave has finished
    // the conversion of batch b and the compute of batch b - 1, whose buffer
    // the copies of batch b + 1 then overwrite.
    issue(0, tile0);
    for (int k0 = 0, cur = 0; k0 < len; k0 += PT_KB, cur ^= 1) {
        double *tb = cur ? tile1 : tile0, *nb = cur ? tile0 : tile1;
        finish(k0, tb);
        __syncthreads();
        if (k0 + PT_KB < len) issue(k0 + PT_KB, nb);
        compute(tb);
        if (cur == 1 || k0 + PT_KB >= len) reduce_all();  // every second batch, and the last
    }
    const u64 o = (u64)l * N + (u64)blockIdx.x * T + lane;
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        const u64 p = (u64)(pbase + r * G);
        if (p < (u64)P) {
            u64 *o0 = d01 + p * d01_stride + o, *o1 = o0 + S, *o2 = d2 + p * d2_stride + o;
            double c1 = acc[r][1] + acc[r][1];  // |2 acc| <= q + 2
            if (accumulate) {  // previous values in [0, q): the sums stay below 2q + 2
                acc[r][0] += u64_to_d(*o0);
                c1 += u64_to_d(*o1);
                acc[r][2] += u64_to_d(*o2);
            }
            *o0 = d_to_canonical(acc[r][0], q, qinv);
            *o1 = d_to_canonical(c1, q, qinv);
            *o2 = d_to_canonical(acc[r][2], q, qinv);
        }
    }
}

template <int T>
static void launch_pt(int ppt, dim3 grid, dim3 block, size_t lds, hipStream_t s, const DevParams &dp, const u64 *cts,
                      int n, int len, int P, u64 *d01, u64 d01_stride, u64 *d2, u64 d2_stride, int accumulate)
{
    switch (ppt) {
    case 1: hipLaunchKernelGGL((pair_triples_kernel<T, 1>), grid, block, lds, s, dp, cts, n, len, P, d01, d01_stride,
                               d2, d2_stride, accumulate); break;
    case 3: hipLaunchKernelGGL((pair_triples_kernel<T, 3>), grid, block, lds, s, dp, cts, n, len, P, d01, d01_stride,
                               d2, d2_stride, accumulate); break;
    case 4: hipLaunchKernelGGL((pair_triples_kernel<T, 4>), grid, block, lds, s, dp, cts, n, len, P, d01, d01_stride,
                               d2, d2_stride, accumulate); break;
    default: hipLaunchKernelGGL((pair_triples_kernel<T, 6>), grid, block, lds, s, dp, cts, n, len, P, d01,
                                d01_stride, d2, d2_stride, accumulate); break;
    }
}

int launch_pair_triples(Ctx *c, const u64 *cts, int n, int len, u64 *d01, u64 d01_stride, u64 *d2, u64 d2_stride,
                        int accumulate, hipStream_t s)
{
    if (n < 2 || n > PT_MAXN) return fail(c, LC_EINVAL, "pairwise kernels take 2..64 clients");
    if (len < 1) return fail(c, LC_EINVAL, "len must be >= 1");
    if (c->tune.pair_mfma) {  // the Gram form on the matrix cores, where its LDS fits
        const int pm = pair_gram_positions(c, n, c->tune.pair_mfma);
        if (pm) return launch_pair_gram(c, pm, cts, n, len, d01, d01_stride, d2, d2_stride, accumulate, s);
    }
    int P = n * (n - 1) / 2;
    int ppt = c->tune.pair_ppt;
    if (P <= 64) ppt = 1;  // few pairs: one per lane
    // coefficient lanes: the tuned value, at most N, and small enough that the
    // staged tiles of all n clients fit the LDS budget
    int T = c->tune.pair_lanes;
    // (wave copies move 128 / T rows: a buffer holds whole copy groups)
    auto buf_doubles = [&](int t) { return ((size_t)n * 2 * PT_KB * t + 127) / 128 * 128; };
    while (T > 8 && ((u64)T > c->N || buf_doubles(T) > (size_t)PT_BUF)) T >>= 1;
    int G = std::max(1, std::min((P + ppt - 1) / ppt, 1024 / T));
    int chunks = (P + G * ppt - 1) / (G * ppt);
    dim3 grid((u32)(c->N / T), (u32)c->nq, (u32)chunks), block(T, G);
    size_t lds = 2 * buf_doubles(T) * sizeof(double);  // two tile buffers
    switch (T) {
    case 8: launch_pt<8>(ppt, grid, block, lds, s, c->dp, cts, n, len, P, d01, d01_stride, d2, d2_stride, accumulate); break;
    case 16: launch_pt<16>(ppt, grid, block, lds, s, c->dp, cts, n, len, P, d01, d01_stride, d2, d2_stride, accumulate); break;
    case 32: launch_pt<32>(ppt, grid, block, lds, s, c->dp, cts, n, len, P, d01, d01_stride, d2, d2_stride, accumulate); break;
    default: launch_pt<64>(ppt, grid, block, lds, s, c->dp, cts, n, len, P, d01, d01_stride, d2, d2_stride, accumulate); break;
    }
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// ---- SumDis[i] = sum_{j != i} Dis[i][j] -------------------------------------
// (also the per-client sums of pair triples: ncomp 3, in_stride 3 n_q N)

__global__ void __launch_bounds__(EW_THREADS)
sumdis_kernel(DevParams dp, const u64 *dist, u64 in_stride, int n, int ncomp, u64 *sumdis, u64 total)
{
    u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // over n * ncomp * nq * N
    if (e >= total) return;
    u64 SC = (u64)ncomp * ((u64)dp.nq << dp.log_n);
    int i = (int)(e / SC);
    u64 r = e % SC;
    int l = (int)((r >> dp.log_n) % (u64)dp.nq);
    u64 q = dp.mc[l].m, acc = 0;
    for (int j = 0; j < n; j++) {
        if (j == i) continue;
        int a = i < j ? i : j, b = i < j ? j : i;
        int p = pair_index(n, a, b);
        acc = add_mod(acc, dist[(u64)p * in_stride + r], q);
    }
    sumdis[e] = acc;
}

int launch_sumdis(Ctx *c, const u64 *dist, u64 in_stride, int n, int ncomp, u64 *sumdis, hipStream_t s)
{
    u64 total = (u64)n * ncomp * c->nq * c->N;
    hipLaunchKernelGGL(sumdis_kernel, grid_for(total, EW_THREADS), dim3(EW_THREADS), 0, s, c->dp, dist, in_stride, n,
                       ncomp, sumdis, total);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

__global__ void __launch_bounds__(EW_THREADS) copy_kernel(const u64 *src, u64 *dst, u64 words)
{
    u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < words) dst[e] = src[e];
}

int launch_copy(Ctx *c, const u64 *src, u64 *dst, u64 words, hipStream_t s)
{
    if (!words) return LC_OK;
    hipLaunchKernelGGL(copy_kernel, grid_for(words, EW_THREADS), dim3(EW_THREADS), 0, s, src, dst, words);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

}  // namespace lc
