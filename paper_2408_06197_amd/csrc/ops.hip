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
// Two adjacent coefficients per lane (16-byte accesses), four clients' loads
// in flight; FP64 Barrett products (|r| <= 0.875 q) summed with a reduction
// after at most 8 clients.
__global__ void __launch_bounds__(EW_THREADS)
masked_sum_kernel(DevParams dp, const u64 *cts, int n, int len, const u64 *masks, u64 *out, u64 total2)
{
    u64 e2 = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // over len * 2 * nq * N / 2
    if (e2 >= total2) return;
    u64 e = 2 * e2;
    u64 S = (u64)dp.nq << dp.log_n;
    u64 r = e % S;
    int l = (int)(r >> dp.log_n);
    const double q = dp.mc[l].qd, qinv = dp.mc[l].qinv;
    u64 client_stride = (u64)len * 2 * S;
    double a0 = 0.0, a1 = 0.0;
    for (int i0 = 0; i0 < n; i0 += 4) {
        ulonglong2 c2[4], m2[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            int i = min(i0 + u, n - 1);
            c2[u] = *reinterpret_cast<const ulonglong2 *>(cts + (u64)i * client_stride + e);
            m2[u] = *reinterpret_cast<const ulonglong2 *>(masks + (u64)i * S + r);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if (i0 + u < n) {
                a0 += mulmod_d(u64_to_d(c2[u].x), u64_to_d(m2[u].x), q, qinv);
                a1 += mulmod_d(u64_to_d(c2[u].y), u64_to_d(m2[u].y), q, qinv);
            }
        }
        if ((i0 & 7) == 4 || i0 + 4 >= n) {  // at most 8 products between reductions
            a0 = reduce_d(a0, q, qinv);
            a1 = reduce_d(a1, q, qinv);
        }
    }
    ulonglong2 o;
    o.x = d_to_canonical(reduce_d(a0, q, qinv), q, qinv);
    o.y = d_to_canonical(reduce_d(a1, q, qinv), q, qinv);
    *reinterpret_cast<ulonglong2 *>(out + e) = o;
}

int launch_masked_sum(Ctx *c, const u64 *cts, int n, int len, const u64 *masks, u64 *out, hipStream_t s)
{
    u64 total2 = (u64)len * c->nq * c->N;  // pairs of coefficients (N is even)
    if (!total2) return LC_OK;
    hipLaunchKernelGGL(masked_sum_kernel, grid_for(total2, EW_THREADS), dim3(EW_THREADS), 0, s, c->dp, cts, n, len,
                       masks, out, total2);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// ---- fused subtract / square / lazy accumulate over all pairs --------------
//
// Workgroup = (tile of T coefficients, limb l, chunk of pairs).  KB packed
// ciphertexts at a time, the tiles of all n clients (both components) are
// staged in LDS once -- as exact doubles -- and every pair of the chunk reads
// them from there.  A lane owns one coefficient of PPT pairs and keeps their
// triple accumulators in registers across all k.  T and PPT are tuning
// parameters (lc_set_tuning); the defaults come from measurements on MI355X.
//
// Arithmetic is the FP64 Barrett form of modarith.h: differences x = a - b
// lie in (-q, q); each product comes back as an integer r with |r| <= 0.875 q;
// the accumulators (|acc| <= q/2 + 1 after a reduction) take at most
// KB * 1.75 q <= 7 q before the next reduction, so they stay below 2^53 and
// every value is exact.  The canonical residue is taken once at the end.

constexpr int PT_MAXN = 64;     // clients per call
constexpr int PT_KB = 4;        // packed ciphertexts staged per barrier (at most)
constexpr size_t PT_LDS = 64 * 1024;

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

template <int PPT>
__global__ void __launch_bounds__(1024)
pair_triples_kernel(DevParams dp, const u64 *__restrict__ cts, int n, int len, int P, u64 *d01, u64 d01_stride,
                    u64 *d2, u64 d2_stride, int KB, int accumulate)
{
    extern __shared__ double tile[];  // [KB][n][2][T]
    const int T = blockDim.x;         // coefficient lanes
    const int G = blockDim.y;         // pair groups
    const int lane = threadIdx.x, g = threadIdx.y;
    const int tid = g * T + lane;
    const int nthreads = T * G;
    const int l = blockIdx.y;
    const u64 N = dp.N;
    const u64 S = (u64)dp.nq * N;
    const double q = dp.mc[l].qd, qinv = dp.mc[l].qinv;
    const int per_k = n * 2 * T;

    // pair r of this lane is p = pbase + r G; its two clients' LDS offsets
    // are packed into one register
    const int pbase = blockIdx.z * (G * PPT) + g;
    int offs[PPT];
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        int p = pbase + r * G, i = 0, j = 1;
        if (p < P) pair_of_index(p, n, i, j);
        offs[r] = ((i * 2) * T + lane) | (((j * 2) * T + lane) << 16);
    }
    double acc[PPT][3];
#pragma unroll
    for (int r = 0; r < PPT; r++) acc[r][0] = acc[r][1] = acc[r][2] = 0.0;

    const u64 client_stride = (u64)len * 2 * S;
    const u64 off = (u64)l * N + (u64)blockIdx.x * T;
    for (int k0 = 0; k0 < len; k0 += KB) {
        const int kb = min(KB, len - k0);
        for (int idx = tid; idx < kb * per_k; idx += nthreads) {
            int row = idx / T, t = idx - row * T;
            int kk = row / (2 * n), rr = row - kk * 2 * n;  // rr = client * 2 + comp
            tile[idx] = u64_to_d(cts[(u64)(rr >> 1) * client_stride + (u64)(k0 + kk) * 2 * S + (u64)(rr & 1) * S +
                                     off + t]);
        }
        __syncthreads();
        for (int kk = 0; kk < kb; kk++) {
            const double *tl = tile + kk * per_k;
#pragma unroll
            for (int r = 0; r < PPT; r++) {
                if (pbase + r * G < P) {
                    const int oa = offs[r] & 0xffff, ob = offs[r] >> 16;
                    double x0 = tl[oa] - tl[ob];
                    double x1 = tl[oa + T] - tl[ob + T];
                    double m = mulmod_d(x0, x1, q, qinv);
                    acc[r][0] += mulmod_d(x0, x0, q, qinv);
                    acc[r][1] += m + m;
                    acc[r][2] += mulmod_d(x1, x1, q, qinv);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < PPT; r++) {
            acc[r][0] = reduce_d(acc[r][0], q, qinv);
            acc[r][1] = reduce_d(acc[r][1], q, qinv);
            acc[r][2] = reduce_d(acc[r][2], q, qinv);
        }
        __syncthreads();
    }
    const u64 o = (u64)l * N + (u64)blockIdx.x * T + lane;
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        const u64 p = (u64)(pbase + r * G);
        if (p < (u64)P) {
            u64 *o0 = d01 + p * d01_stride + o, *o1 = o0 + S, *o2 = d2 + p * d2_stride + o;
            if (accumulate) {  // |acc| <= q/2 + 1, previous value in [0, q): the sum stays within 2q
                acc[r][0] += u64_to_d(*o0);
                acc[r][1] += u64_to_d(*o1);
                acc[r][2] += u64_to_d(*o2);
            }
            *o0 = d_to_canonical(acc[r][0], q, qinv);
            *o1 = d_to_canonical(acc[r][1], q, qinv);
            *o2 = d_to_canonical(acc[r][2], q, qinv);
        }
    }
}

int launch_pair_triples(Ctx *c, const u64 *cts, int n, int len, u64 *d01, u64 d01_stride, u64 *d2, u64 d2_stride,
                        int accumulate, hipStream_t s)
{
    if (n < 2 || n > PT_MAXN) return fail(c, LC_EINVAL, "pairwise kernels take 2..64 clients");
    if (len < 1) return fail(c, LC_EINVAL, "len must be >= 1");
    int P = n * (n - 1) / 2;
    int ppt = c->tune.pair_ppt, T = c->tune.pair_lanes;
    if (P <= 64) ppt = 1;  // few pairs: one per lane
    T = (int)std::min<u64>((u64)T, c->N);
    int G = std::max(1, std::min((P + ppt - 1) / ppt, 1024 / T));
    int chunks = (P + G * ppt - 1) / (G * ppt);
    dim3 grid((u32)(c->N / T), (u32)c->nq, (u32)chunks), block(T, G);
    size_t per_k = (size_t)n * 2 * T * sizeof(double);
    int kb = (int)std::max<size_t>(1, std::min<size_t>(PT_KB, PT_LDS / per_k));
    size_t lds = (size_t)kb * per_k;
    switch (ppt) {
    case 1: hipLaunchKernelGGL((pair_triples_kernel<1>), grid, block, lds, s, c->dp, cts, n, len, P, d01, d01_stride,
                               d2, d2_stride, kb, accumulate); break;
    case 3: hipLaunchKernelGGL((pair_triples_kernel<3>), grid, block, lds, s, c->dp, cts, n, len, P, d01, d01_stride,
                               d2, d2_stride, kb, accumulate); break;
    default: hipLaunchKernelGGL((pair_triples_kernel<6>), grid, block, lds, s, c->dp, cts, n, len, P, d01,
                                d01_stride, d2, d2_stride, kb, accumulate); break;
    }
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// ---- SumDis[i] = sum_{j != i} Dis[i][j] -------------------------------------

__global__ void __launch_bounds__(EW_THREADS)
sumdis_kernel(DevParams dp, const u64 *dist, int n, u64 *sumdis, u64 total)
{
    u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // over n * 2 * nq * N
    if (e >= total) return;
    u64 S2 = 2 * ((u64)dp.nq << dp.log_n);
    int i = (int)(e / S2);
    u64 r = e % S2;
    int l = (int)((r >> dp.log_n) % (u64)dp.nq);
    u64 q = dp.mc[l].m, acc = 0;
    for (int j = 0; j < n; j++) {
        if (j == i) continue;
        int a = i < j ? i : j, b = i < j ? j : i;
        int p = pair_index(n, a, b);
        acc = add_mod(acc, dist[(u64)p * S2 + r], q);
    }
    sumdis[e] = acc;
}

int launch_sumdis(Ctx *c, const u64 *dist, int n, u64 *sumdis, hipStream_t s)
{
    u64 total = (u64)n * 2 * c->nq * c->N;
    hipLaunchKernelGGL(sumdis_kernel, grid_for(total, EW_THREADS), dim3(EW_THREADS), 0, s, c->dp, dist, n, sumdis,
                       total);
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
