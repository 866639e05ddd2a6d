// Fused subtract / square / lazy accumulate over all client pairs as exact
// modular Gram products on the int8 matrix cores (Methods, Computing the
// Pairwise Distances; the Tensor and Add operations of the CKKS Scheme
// Description, accumulated lazily before one relinearization per pair).
//
// For one coefficient position (limb l, coefficient c) let row r = 2 i + comp
// hold ct_i[k][comp][l][c] over the packed ciphertexts k.  With the Gram
// matrix G[r][r'] = sum_k x_r[k] x_r'[k], the pair triple of (i, j) is
//   d0^2   = G[2i][2i]     + G[2j][2j]     - 2 G[2i][2j]
//   d1^2   = G[2i+1][2i+1] + G[2j+1][2j+1] - 2 G[2i+1][2j+1]
//   2 d0d1 = 2 (G[2i][2i+1] + G[2j][2j+1] - G[2i][2j+1] - G[2j][2i+1])
// (all mod q_l), i.e. the same sums of squared differences as the
// per-pair form, read off n (2n + 1) Gram entries instead of computed per pair.
//
// Exactness.  A residue x < q < 2^50 is written in balanced base-256 digits
// x = sum_{s<7} d_s 256^s with d_s in [-128, 127]: the bytes of
// x + 0x0080808080808080 with 0x80 subtracted.  For each digit sum m = s + t
// the int8 MFMA accumulates G_m = sum_k sum_{s+t=m} d_s(x_r) d_t(x_r') in int32;
// |G_m| <= len * 7 * 2^14 < 2^26 for len <= 512 ciphertexts per launch, so
// nothing wraps.  G mod q = sum_m G_m (256^m mod q), taken in FP64 as four
// exact partial sums of four digit groups (each below 2^51) times 2^{32 g} mod q
// with the Barrett form of modarith.h.  Every step is exact, so the output is
// the canonical residue, bit for bit the same as the per-pair kernel's.
//
// Work split.  A workgroup owns PM consecutive coefficients of one limb and all
// 2n rows.  Per chunk of 64 ciphertexts its waves copy the rows straight from
// HBM into LDS (PM * 8 bytes per row and ciphertext), turn them into seven
// digit planes (byte transposes; one 16-byte MFMA operand per lane), and run
// the 16x16x64 MFMAs: one item = (coefficient, 16x16 tile of the upper
// triangle of G), 49 digit pairs per item and chunk, 13 int32 accumulator
// tiles per item kept across all chunks.  At the end the items are reduced mod
// q into an LDS copy of G and the pair triples read off it.  The copy of chunk
// k + 1 runs while chunk k is multiplied.
//
// Status: an option (tuning "pair_mfma").  The 13 accumulator tiles per item
// limit a CU to a few coefficients in flight, so each client row is read 16 or
// 32 bytes at a time; on MI355X at N = 2^16 with 20 clients this measured
// slower than the per-pair FP64 kernel, which stays the default.
#include "lc_internal.h"

namespace lc {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int PG_KC = 64;     // ciphertexts per chunk: the MFMA's K
constexpr int PG_KMAX = 512;  // ciphertexts per launch: |G_m| < 2^26
constexpr int PG_IPW = 3;     // (coefficient, tile) items per wave
constexpr int PG_ND = 7;      // balanced base-256 digits of a residue < 2^50
constexpr int PG_MAXR = 48;   // rows 2n: at most 3 row blocks of 16

template <int PM>
struct PgShape {
    static constexpr int SEG = PM * 8;                 // bytes per (row, ciphertext) in the copy buffer
    static constexpr int RS = PG_KC * SEG + 16;        // bytes per copy-buffer row (padded to spread rows over banks)
    static constexpr int SPL = 1024 / SEG;             // segments per wave copy (16 bytes per lane)
    static constexpr int LPS = SEG / 16;               // lanes per segment
    static constexpr int IPR = PG_KC / SPL;            // wave copies per row
    static constexpr int TPL = 128 / SEG;              // workgroups per 128-byte line of a row
    static size_t lds_bytes(int R) { return (size_t)R * RS + (size_t)PG_ND * PM * R * 64; }
};

__device__ __forceinline__ void pg_pair_of_index(int p, int n, int &i, int &j)
{
    int row = 0, base = 0;
    while (base + (n - 1 - row) <= p) {
        base += n - 1 - row;
        row++;
    }
    i = row;
    j = row + 1 + (p - base);
}

// upper-triangle tile t of an nrb x nrb block grid, row-major: (I, J), I <= J
__device__ __forceinline__ void pg_tile(int t, int nrb, int &I, int &J)
{
    I = 0;
    while (t >= nrb - I) {
        t -= nrb - I;
        I++;
    }
    J = I + t;
}

template <int PM>
__global__ void __launch_bounds__(512)
pair_gram_kernel(DevParams dp, const u64 *__restrict__ cts, u64 client_stride, int n, int len, int P, u64 *d01,
                 u64 d01_stride, u64 *d2, u64 d2_stride, int accumulate, int xcd_remap)
{
    using SH = PgShape<PM>;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int R = 2 * n, nrb = (R + 15) >> 4, ntile = nrb * (nrb + 1) / 2, nitems = PM * ntile;
    const int tid = threadIdx.x, lane = tid & 63, nthreads = blockDim.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), nwaves = nthreads >> 6;
    const int l = blockIdx.y;
    const u64 N = dp.N, S = (u64)dp.nq * N;

    // Coefficient tile.  Workgroups are dealt to the 8 XCDs round-robin; the
    // remap puts the TPL tiles that share a 128-byte line of every row on one
    // XCD, dispatched together, so its L2 fetches each line once.
    u32 bx = blockIdx.x;
    if (xcd_remap) {
        const u32 x = bx & 7, slot = bx >> 3;
        bx = (slot / SH::TPL) * (8 * SH::TPL) + x * SH::TPL + slot % SH::TPL;
    }
    const u64 c0 = (u64)bx * PM;
    unsigned char *const raw = smem;                  // [R][RS]: row r, ciphertext k at k * SEG
    unsigned char *const dig = smem + (size_t)R * SH::RS;  // [7][PM][R][64]: digit planes
    const int plane = PM * R * 64;

    // ---- copy of a chunk: R * IPR wave copies of 16 bytes per lane ----
    const int kl = lane / SH::LPS, sub = lane % SH::LPS;
    auto issue = [&](int k0) {
        for (int g = wave; g < R * SH::IPR; g += nwaves) {
            const int r = g / SH::IPR, h = g % SH::IPR;
            const int k = min(k0 + h * SH::SPL + kl, len - 1);  // past len: re-read, zeroed below
            const u64 *src = cts + (u64)(r >> 1) * client_stride + (u64)k * 2 * S + (u64)(r & 1) * S +
                             (u64)l * N + c0 + sub * 2;
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                             (__attribute__((address_space(3))) void *)(raw + r * SH::RS + h * 1024),
                                             16, 0, 0);
        }
    };

    // ---- digit planes: unit (r, p, j) turns ciphertexts 8j .. 8j+7 of row r,
    // coefficient p into 7 plane words of 8 bytes (byte t = ciphertext 8j + t).
    // Within a plane row the 16-byte group kb of ciphertexts sits at slot
    // kb ^ ((r >> 2) & 3), so that a wave's operand reads hit distinct banks.
    auto convert = [&](int k0) {
        const int nunits = R * PM * (PG_KC / 8);
        for (int u = tid; u < nunits; u += nthreads) {
            const int r = u % R, p = (u / R) % PM, j = u / (R * PM);
            const unsigned char *src = raw + r * SH::RS + j * 8 * SH::SEG + p * 8;
            u32 lo[8], hi[8];
#pragma unroll
            for (int t = 0; t < 8; t++) {
                u64 x = *reinterpret_cast<const u64 *>(src + t * SH::SEG);
                if (k0 + j * 8 + t >= len) x = 0;  // zero digits
                x += 0x0080808080808080ull;
                lo[t] = (u32)x;
                hi[t] = (u32)(x >> 32);
            }
            // bytes (s, s+1) of ciphertext pairs (2w, 2w+1): [s:2w s:2w+1 s+1:2w s+1:2w+1]
            u32 qv[4][4];
#pragma unroll
            for (int w = 0; w < 4; w++) {
                qv[w][0] = __builtin_amdgcn_perm(lo[2 * w + 1], lo[2 * w], 0x05010400u);
                qv[w][1] = __builtin_amdgcn_perm(lo[2 * w + 1], lo[2 * w], 0x07030602u);
                qv[w][2] = __builtin_amdgcn_perm(hi[2 * w + 1], hi[2 * w], 0x05010400u);
                qv[w][3] = __builtin_amdgcn_perm(hi[2 * w + 1], hi[2 * w], 0x07030602u);
            }
            const int kb = j >> 1;
            const int off = (p * R + r) * 64 + ((kb ^ ((r >> 2) & 3)) << 4) + (j & 1) * 8;
#pragma unroll
            for (int sg = 0; sg < 4; sg++) {  // digit pair (2 sg, 2 sg + 1)
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    const int s = 2 * sg + e;
                    if (s >= PG_ND) continue;
                    const u32 sel = e ? 0x07060302u : 0x05040100u;
                    const u32 w0 = __builtin_amdgcn_perm(qv[1][sg], qv[0][sg], sel) ^ 0x80808080u;
                    const u32 w1 = __builtin_amdgcn_perm(qv[3][sg], qv[2][sg], sel) ^ 0x80808080u;
                    *reinterpret_cast<u64 *>(dig + s * plane + off) = ((u64)w1 << 32) | w0;
                }
            }
        }
    };

    // ---- MFMA: item it = (p, tile), 13 accumulator tiles each ----
    v4i acc[PG_IPW][2 * PG_ND - 1];
#pragma unroll
    for (int u = 0; u < PG_IPW; u++)
#pragma unroll
        for (int m = 0; m < 2 * PG_ND - 1; m++) acc[u][m] = v4i{0, 0, 0, 0};
    const int kb = lane >> 4;
    auto operands = [&](int p, int rb, v4i *x) {
        const int r = 16 * rb + (lane & 15);
        const int off = (p * R + r) * 64 + ((kb ^ ((r >> 2) & 3)) << 4);
#pragma unroll
        for (int s = 0; s < PG_ND; s++)
            x[s] = r < R ? *reinterpret_cast<const v4i *>(dig + s * plane + off) : v4i{0, 0, 0, 0};
    };
    auto multiply = [&]() {
#pragma unroll
        for (int u = 0; u < PG_IPW; u++) {
            const int it = wave * PG_IPW + u;
            if (it >= nitems) break;
            int I, J;
            pg_tile(it % ntile, nrb, I, J);
            v4i a[PG_ND], b[PG_ND];
            operands(it / ntile, I, a);
            if (I == J) {
#pragma unroll
                for (int s = 0; s < PG_ND; s++) b[s] = a[s];
            } else {
                operands(it / ntile, J, b);
            }
            // consecutive MFMAs go to different accumulators
#pragma unroll
            for (int t = 0; t < PG_ND; t++)
#pragma unroll
                for (int s = 0; s < PG_ND; s++)
                    acc[u][s + t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[s], b[t], acc[u][s + t], 0, 0, 0);
        }
    };

    issue(0);
    for (int k0 = 0; k0 < len; k0 += PG_KC) {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies have landed
        __syncthreads();                // everyone's have; the digit planes are free
        convert(k0);
        __syncthreads();                // planes ready; the copy buffer is free
        if (k0 + PG_KC < len) issue(k0 + PG_KC);
        multiply();
    }
    __syncthreads();  // the copy buffer becomes G

    // ---- G mod q into LDS: Gm[p][r][r'] ----
    const double q = dp.mc[l].qd, qinv = dp.mc[l].qinv;
    const double w1 = canon_d(reduce_d(4294967296.0, q, qinv), q, qinv);  // 2^32 mod q
    const double w2 = canon_d(mulmod_d(w1, w1, q, qinv), q, qinv);       // 2^64 mod q
    const double w3 = canon_d(mulmod_d(w2, w1, q, qinv), q, qinv);       // 2^96 mod q
    double *const Gm = reinterpret_cast<double *>(smem);
#pragma unroll
    for (int u = 0; u < PG_IPW; u++) {
        const int it = wave * PG_IPW + u;
        if (it >= nitems) break;
        const int p = it / ntile;
        int I, J;
        pg_tile(it % ntile, nrb, I, J);
#pragma unroll
        for (int e = 0; e < 4; e++) {
            // C layout of the 16x16 MFMA: lane holds column lane % 16, rows 4 (lane / 16) + e
            const int ra = 16 * I + 4 * (lane >> 4) + e, rb = 16 * J + (lane & 15);
            double v[4];
#pragma unroll
            for (int g = 0; g < 4; g++) {
                double x = 0.0;
#pragma unroll
                for (int h = 3; h >= 0; h--) {
                    const int m = 4 * g + h;
                    if (m < 2 * PG_ND - 1) x = x * 256.0 + (double)acc[u][m][e];
                }
                v[g] = x;  // |x| < 2^26 * (1 + 2^8 + 2^16 + 2^24) < 2^51, exact
            }
            double gv = reduce_d(v[0], q, qinv) + mulmod_d(v[1], w1, q, qinv) + mulmod_d(v[2], w2, q, qinv) +
                        mulmod_d(v[3], w3, q, qinv);
            gv = reduce_d(gv, q, qinv);  // |gv| <= q/2 + 1
            if (ra < R && rb < R) {
                Gm[(p * R + ra) * R + rb] = gv;
                Gm[(p * R + rb) * R + ra] = gv;
            }
        }
    }
    __syncthreads();

    // ---- pair triples ----
    for (int u = tid; u < P * PM; u += nthreads) {
        const int p = u % PM, pp = u / PM;
        int i, j;
        pg_pair_of_index(pp, n, i, j);
        const double *g = Gm + p * R * R;
        const int a0 = 2 * i, a1 = a0 + 1, b0 = 2 * j, b1 = b0 + 1;
        double s00 = g[a0 * R + a0] + g[b0 * R + b0] - 2.0 * g[a0 * R + b0];  // |.| <= 2q + 4
        double s11 = g[a1 * R + a1] + g[b1 * R + b1] - 2.0 * g[a1 * R + b1];
        double s01 = 2.0 * (g[a0 * R + a1] + g[b0 * R + b1] - g[a0 * R + b1] - g[b0 * R + a1]);  // <= 4q + 8
        const u64 o = (u64)l * N + c0 + p;
        u64 *o0 = d01 + (u64)pp * d01_stride + o, *o1 = o0 + S, *o2 = d2 + (u64)pp * d2_stride + o;
        if (accumulate) {  // previous values in [0, q)
            s00 += u64_to_d(*o0);
            s01 += u64_to_d(*o1);
            s11 += u64_to_d(*o2);
        }
        *o0 = d_to_canonical(s00, q, qinv);
        *o1 = d_to_canonical(s01, q, qinv);
        *o2 = d_to_canonical(s11, q, qinv);
    }
}

// Coefficients per workgroup for n clients: PM = want (4 or 2) if its LDS fits,
// else 2 if that fits, else 0 (the per-pair kernel runs).
int pair_gram_positions(Ctx *c, int n, int want)
{
    if (n < 2 || 2 * n > PG_MAXR || c->N < 4) return 0;
    int dev_lds = 0;
    if (hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess) return 0;
    const int R = 2 * n;
    if (want >= 4 && PgShape<4>::lds_bytes(R) <= (size_t)dev_lds) return 4;
    if (PgShape<2>::lds_bytes(R) <= (size_t)dev_lds) return 2;
    return 0;
}

template <int PM>
static int launch_pg(Ctx *c, const u64 *cts, int n, int len, u64 *d01, u64 d01_stride, u64 *d2, u64 d2_stride,
                     int accumulate, hipStream_t s)
{
    using SH = PgShape<PM>;
    const int R = 2 * n, nrb = (R + 15) / 16, ntile = nrb * (nrb + 1) / 2;
    const int nwaves = (PM * ntile + PG_IPW - 1) / PG_IPW;
    const size_t lds = SH::lds_bytes(R);
    // dynamic LDS beyond 64 KiB must be asked for; tracked per context (one device)
    size_t &allowed = c->gram_lds_allowed[PM == 4 ? 1 : 0];
    if (lds > allowed) {
        LC_HIP(c, hipFuncSetAttribute((const void *)pair_gram_kernel<PM>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds));
        allowed = lds;
    }
    const u64 S = (u64)c->nq * c->N, client_stride = (u64)len * 2 * S;
    const int P = n * (n - 1) / 2;
    const u32 gx = (u32)(c->N / PM);
    const int remap = gx % (8 * SH::TPL) == 0;
    for (int k0 = 0; k0 < len; k0 += PG_KMAX) {
        const int kl = std::min(PG_KMAX, len - k0);
        hipLaunchKernelGGL((pair_gram_kernel<PM>), dim3(gx, (u32)c->nq), dim3(64 * nwaves), lds, s, c->dp,
                           cts + (u64)k0 * 2 * S, client_stride, n, kl, P, d01, d01_stride, d2, d2_stride,
                           k0 ? 1 : accumulate, remap);
        LC_HIP(c, hipGetLastError());
    }
    return LC_OK;
}

int launch_pair_gram(Ctx *c, int pm, const u64 *cts, int n, int len, u64 *d01, u64 d01_stride, u64 *d2,
                     u64 d2_stride, int accumulate, hipStream_t s)
{
    if (pm == 4) return launch_pg<4>(c, cts, n, len, d01, d01_stride, d2, d2_stride, accumulate, s);
    return launch_pg<2>(c, cts, n, len, d01, d01_stride, d2, d2_stride, accumulate, s);
}

}  // namespace lc
