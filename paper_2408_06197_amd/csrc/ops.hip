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
__global__ void __launch_bounds__(EW_THREADS)
masked_sum_kernel(DevParams dp, const u64 *cts, int n, int len, const u64 *masks, u64 *out, u64 total)
{
    u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // over len * 2 * nq * N
    if (e >= total) return;
    u64 S = (u64)dp.nq << dp.log_n;
    u64 r = e % S;
    int l = (int)(r >> dp.log_n);
    u64 client_stride = (u64)len * 2 * S;
    Split3 acc;
    split_zero(acc);
    for (int i = 0; i < n; i++) split_mac(acc, cts[(u64)i * client_stride + e], masks[(u64)i * S + r]);
    out[e] = reduce_split(acc, dp.mc[l]);
}

int launch_masked_sum(Ctx *c, const u64 *cts, int n, int len, const u64 *masks, u64 *out, hipStream_t s)
{
    u64 total = (u64)len * 2 * c->nq * c->N;
    if (!total) return LC_OK;
    hipLaunchKernelGGL(masked_sum_kernel, grid_for(total, EW_THREADS), dim3(EW_THREADS), 0, s, c->dp, cts, n, len,
                       masks, out, total);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// ---- fused subtract / square / lazy accumulate over all pairs --------------
//
// Workgroup = (coefficient tile of T lanes, limb l, chunk of pairs).  KB
// packed ciphertexts at a time, the tiles of all n clients (both components)
// are staged in LDS and every pair of the chunk reads them from there; each
// lane keeps PPT pairs' accumulators (three split sums per triple component,
// 18 VGPRs per pair) in registers across all k, and reduces once at the end.

constexpr int PT_T = 16;        // coefficients per workgroup
constexpr int PT_MAXN = 64;     // clients per call
constexpr int PT_PPT = 3;       // pairs per lane
constexpr int PT_KB = 4;        // packed ciphertexts staged per barrier

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

template <int PPT, int KB>
__global__ void __launch_bounds__(1024)
pair_triples_kernel(DevParams dp, const u64 *__restrict__ cts, int n, int len, int P, u64 *d01, u64 d01_stride,
                    u64 *d2, u64 d2_stride)
{
    extern __shared__ u64 tile[];  // [KB][n][2][T]
    const int T = blockDim.x;      // coefficient lanes
    const int G = blockDim.y;      // pair groups
    const int lane = threadIdx.x, g = threadIdx.y;
    const int tid = g * T + lane;
    const int nthreads = T * G;
    const int l = blockIdx.y;
    const u64 N = dp.N;
    const u64 S = (u64)dp.nq * N;
    const ModConst mc = dp.mc[l];
    const u64 q = mc.m;
    const int per_k = n * 2 * T;

    int offa[PPT], offb[PPT], pp[PPT];
    bool live[PPT];
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        int p = blockIdx.z * (G * PPT) + r * G + g;
        live[r] = p < P;
        pp[r] = p;
        int i = 0, j = 1;
        if (live[r]) pair_of_index(p, n, i, j);
        offa[r] = (i * 2) * T + lane;
        offb[r] = (j * 2) * T + lane;
    }
    Split3 acc[PPT][3];
#pragma unroll
    for (int r = 0; r < PPT; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) split_zero(acc[r][c]);

    const u64 client_stride = (u64)len * 2 * S;
    const u64 off = (u64)l * N + (u64)blockIdx.x * T;
    for (int k0 = 0; k0 < len; k0 += KB) {
        const int kb = min(KB, len - k0);
        for (int idx = tid; idx < kb * per_k; idx += nthreads) {
            int kk = idx / per_k, rem = idx - kk * per_k;
            int t = rem % T, ic = rem / T;  // ic = i * 2 + comp
            int i = ic >> 1, comp = ic & 1;
            tile[idx] = cts[(u64)i * client_stride + (u64)(k0 + kk) * 2 * S + (u64)comp * S + off + t];
        }
        __syncthreads();
        for (int kk = 0; kk < kb; kk++) {
            const u64 *tl = tile + kk * per_k;
#pragma unroll
            for (int r = 0; r < PPT; r++) {
                if (!live[r]) continue;
                u64 x0 = sub_mod(tl[offa[r]], tl[offb[r]], q);
                u64 x1 = sub_mod(tl[offa[r] + T], tl[offb[r] + T], q);
                split_sq(acc[r][0], x0);
                split_mac(acc[r][1], x0, x1);
                split_sq(acc[r][2], x1);
            }
        }
        __syncthreads();
    }
    const u64 o = (u64)l * N + (u64)blockIdx.x * T + lane;
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        if (!live[r]) continue;
        u64 v0 = reduce_split_sq(acc[r][0], mc);
        u64 v1 = reduce_split(acc[r][1], mc);
        v1 = add_mod(v1, v1, q);
        u64 v2 = reduce_split_sq(acc[r][2], mc);
        d01[(u64)pp[r] * d01_stride + o] = v0;
        d01[(u64)pp[r] * d01_stride + S + o] = v1;
        d2[(u64)pp[r] * d2_stride + o] = v2;
    }
}

int launch_pair_triples(Ctx *c, const u64 *cts, int n, int len, u64 *d01, u64 d01_stride, u64 *d2, u64 d2_stride,
                        hipStream_t s)
{
    if (n < 2 || n > PT_MAXN) return fail(c, LC_EINVAL, "pairwise kernels take 2..64 clients");
    if (len < 1 || len > 4096) return fail(c, LC_EINVAL, "len must lie in [1, 4096]");
    int P = n * (n - 1) / 2;
    int T = (int)std::min<u64>(PT_T, c->N);
    int groups_needed = (P + PT_PPT - 1) / PT_PPT;
    int G = std::min(groups_needed, 1024 / T);
    int chunks = (P + G * PT_PPT - 1) / (G * PT_PPT);
    dim3 grid((u32)(c->N / T), (u32)c->nq, (u32)chunks), block(T, G);
    size_t lds = (size_t)PT_KB * n * 2 * T * sizeof(u64);
    hipLaunchKernelGGL((pair_triples_kernel<PT_PPT, PT_KB>), grid, block, lds, s, c->dp, cts, n, len, P, d01,
                       d01_stride, d2, d2_stride);
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
        int p = a * (2 * n - a - 1) / 2 + (b - a - 1);
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
