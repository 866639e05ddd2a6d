// Counter-based randomness and the kernels of key generation, encryption and
// decryption (Methods, CKKS Scheme Description).
//
// Generator: Philox4x64-10 (Salmon et al., SC 2011).  Word w of the stream
// (seed, domain, object) is lane w % 4 of Philox(counter = (w / 4, object,
// domain, 0), key = (seed, 0)), so every coefficient's draw is a pure
// function of its position and any lane can produce it.
#include "lc_internal.h"

namespace lc {

constexpr int RNG_THREADS = 256;

__device__ __forceinline__ void philox4x64_10(u64 ctr[4], u64 k0, u64 k1)
{
    const u64 M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const u64 W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        u64 lo0 = M0 * ctr[0], hi0 = __umul64hi(M0, ctr[0]);
        u64 lo1 = M1 * ctr[2], hi1 = __umul64hi(M1, ctr[2]);
        u64 n0 = hi1 ^ ctr[1] ^ k0, n2 = hi0 ^ ctr[3] ^ k1;
        ctr[0] = n0;
        ctr[1] = lo1;
        ctr[2] = n2;
        ctr[3] = lo0;
    }
}

// Four consecutive words 4*blk .. 4*blk+3 of a stream.
__device__ __forceinline__ void stream_block(u64 seed, u64 domain, u64 object, u64 blk, u64 w[4])
{
    w[0] = blk;
    w[1] = object;
    w[2] = domain;
    w[3] = 0;
    philox4x64_10(w, seed, 0);
}

__device__ __forceinline__ int64_t ternary_of(u64 w) { return (int64_t)(w % 3) - 1; }

// Smallest t in [-19, 19] with w < T[t]: the number of thresholds <= w, minus 19.
__device__ __forceinline__ int64_t gaussian_of(u64 w, const u64 *cdt)
{
    int lo = 0, hi = 38;  // count of k with cdt[k] <= w lies in [lo, hi]
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cdt[mid] <= w) lo = mid + 1;
        else hi = mid;
    }
    return (int64_t)lo - 19;
}

// (hi 2^64 + lo) mod m.
__device__ __forceinline__ u64 wide_mod(u64 hi, u64 lo, const ModConst &mc)
{
    u64 h = csub(mul_shoup_lazy(hi, 1, mc.one_sh, mc.m), mc.m);
    u64 l = csub(mul_shoup_lazy(lo, 1, mc.one_sh, mc.m), mc.m);
    u64 c64 = mul_mod(mc.c50, 1ull << 14, mc);  // 2^64 mod m
    return add_mod(mul_mod(h, c64, mc), l, mc.m);
}

// ---- samplers --------------------------------------------------------------

__global__ void __launch_bounds__(RNG_THREADS)
ternary_kernel(u64 seed, u64 domain, u64 object, int64_t *out, u64 n)
{
    u64 blk = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (blk * 4 >= n) return;
    u64 w[4];
    stream_block(seed, domain, object, blk, w);
    for (int k = 0; k < 4 && blk * 4 + k < n; k++) out[blk * 4 + k] = ternary_of(w[k]);
}

__global__ void __launch_bounds__(RNG_THREADS)
gaussian_kernel(const u64 *cdt, u64 seed, u64 domain, u64 object, int64_t *out, u64 n)
{
    u64 blk = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (blk * 4 >= n) return;
    u64 w[4];
    stream_block(seed, domain, object, blk, w);
    for (int k = 0; k < 4 && blk * 4 + k < n; k++) out[blk * 4 + k] = gaussian_of(w[k], cdt);
}

// Uniform residues for limbs 0..nlimb-1 (object obj_base | limb), directly in
// the NTT domain: out [nlimb][N].
__global__ void __launch_bounds__(RNG_THREADS)
uniform_kernel(DevParams dp, u64 seed, u64 domain, u64 obj_base, u64 *out, int nlimb)
{
    u64 blk = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // two coefficients per block
    int l = blockIdx.y;
    if (blk * 2 >= dp.N || l >= nlimb) return;
    u64 w[4];
    stream_block(seed, domain, obj_base | (u64)l, blk, w);
    const ModConst &mc = dp.mc[l];
    out[(u64)l * dp.N + blk * 2] = wide_mod(w[0], w[1], mc);
    out[(u64)l * dp.N + blk * 2 + 1] = wide_mod(w[2], w[3], mc);
}

int launch_sample_ternary(Ctx *c, u64 seed, u64 domain, u64 object, i64 *out, hipStream_t s)
{
    u64 blocks = c->N / 4;
    hipLaunchKernelGGL(ternary_kernel, dim3((u32)((blocks + RNG_THREADS - 1) / RNG_THREADS)), dim3(RNG_THREADS), 0,
                       s, seed, domain, object, out, c->N);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

int launch_gaussian(Ctx *c, u64 seed, u64 domain, u64 object, i64 *out, hipStream_t s)
{
    u64 blocks = c->N / 4;
    hipLaunchKernelGGL(gaussian_kernel, dim3((u32)((blocks + RNG_THREADS - 1) / RNG_THREADS)), dim3(RNG_THREADS), 0,
                       s, c->dp.cdt, seed, domain, object, out, c->N);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

int launch_uniform_limbs(Ctx *c, u64 seed, u64 domain, u64 obj_base, u64 *out, int nlimb, hipStream_t s)
{
    u64 blocks = c->N / 2;
    dim3 grid((u32)((blocks + RNG_THREADS - 1) / RNG_THREADS), (u32)nlimb);
    hipLaunchKernelGGL(uniform_kernel, grid, dim3(RNG_THREADS), 0, s, c->dp, seed, domain, obj_base, out, nlimb);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// ---- small polynomial helpers ----------------------------------------------

// out[t][l][j] = in[t][j] mod m_l for l < nlimb.
__global__ void __launch_bounds__(RNG_THREADS)
signed_to_limbs_kernel(DevParams dp, const int64_t *in, u64 *out, int nlimb, u64 total)
{
    u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // over count * N
    if (e >= total) return;
    u64 t = e >> dp.log_n, j = e & (dp.N - 1);
    int64_t v = in[e];
    for (int l = 0; l < nlimb; l++) out[(t * nlimb + l) * dp.N + j] = from_signed(v, dp.mc[l]);
}

int launch_signed_to_limbs(Ctx *c, const i64 *in, u64 *out, int nlimb, u64 count, hipStream_t s)
{
    u64 total = count * c->N;
    hipLaunchKernelGGL(signed_to_limbs_kernel, dim3((u32)((total + RNG_THREADS - 1) / RNG_THREADS)),
                       dim3(RNG_THREADS), 0, s, c->dp, in, out, nlimb, total);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// Key-switching key row: k0 = -a s + e + g_l t, k1 = a (g_l = gadget[l] or 0).
__global__ void __launch_bounds__(RNG_THREADS)
keycombine_kernel(DevParams dp, const u64 *a, const u64 *e, const u64 *s_ntt, const u64 *t_ntt,
                  const u64 *gadget, u64 *k0, u64 *k1, int nlimb)
{
    u64 idx = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (u64)nlimb * dp.N) return;
    int l = (int)(idx >> dp.log_n);
    const ModConst &mc = dp.mc[l];
    u64 v = sub_mod(e[idx], mul_mod(a[idx], s_ntt[idx], mc), mc.m);
    if (gadget && gadget[l]) v = add_mod(v, mul_mod(gadget[l], t_ntt[idx], mc), mc.m);
    k0[idx] = v;
    k1[idx] = a[idx];
}

int launch_keycombine(Ctx *c, const u64 *a, const u64 *e, const u64 *s_ntt, const u64 *t_ntt, const u64 *gadget,
                      u64 *k0, u64 *k1, int nlimb, hipStream_t s)
{
    u64 total = (u64)nlimb * c->N;
    hipLaunchKernelGGL(keycombine_kernel, dim3((u32)((total + RNG_THREADS - 1) / RNG_THREADS)), dim3(RNG_THREADS),
                       0, s, c->dp, a, e, s_ntt, t_ntt, gadget, k0, k1, nlimb);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

__global__ void __launch_bounds__(RNG_THREADS) pointwise_sq_kernel(DevParams dp, const u64 *a, u64 *out, int nlimb)
{
    u64 idx = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (u64)nlimb * dp.N) return;
    int l = (int)(idx >> dp.log_n);
    out[idx] = mul_mod(a[idx], a[idx], dp.mc[l]);
}

int launch_pointwise_sq(Ctx *c, const u64 *a, u64 *out, int nlimb, hipStream_t s)
{
    u64 total = (u64)nlimb * c->N;
    hipLaunchKernelGGL(pointwise_sq_kernel, dim3((u32)((total + RNG_THREADS - 1) / RNG_THREADS)),
                       dim3(RNG_THREADS), 0, s, c->dp, a, out, nlimb);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// out[p][i] = in[p][perm[i]]: an automorphism in the NTT domain.
__global__ void __launch_bounds__(RNG_THREADS)
permute_kernel(const u64 *in, u64 *out, const u32 *perm, u64 N, u64 total)
{
    u64 idx = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    u64 p = idx / N, i = idx % N;
    out[idx] = in[p * N + perm[i]];
}

int launch_permute(Ctx *c, const u64 *in, u64 *out, const u32 *perm, u64 npoly, hipStream_t s)
{
    u64 total = npoly * c->N;
    hipLaunchKernelGGL(permute_kernel, dim3((u32)((total + RNG_THREADS - 1) / RNG_THREADS)), dim3(RNG_THREADS), 0,
                       s, in, out, perm, c->N, total);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// ---- encryption --------------------------------------------------------------
// tmp [count][3][nq][N] (coefficient domain, to be NTT'd): (m + e0, r, e1).

__global__ void __launch_bounds__(RNG_THREADS)
enc_sample_kernel(DevParams dp, const int64_t *m, u64 count, u64 seed, u64 first_object, u64 *tmp)
{
    u64 idx = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // over count * N / 4
    u64 per = dp.N / 4;
    if (idx >= count * per) return;
    u64 t = idx / per, blk = idx % per;
    u64 obj = first_object + t;
    u64 wr[4], we0[4], we1[4];
    stream_block(seed, 4, obj, blk, wr);
    stream_block(seed, 5, obj, blk, we0);
    stream_block(seed, 6, obj, blk, we1);
    const u64 S = (u64)dp.nq * dp.N;
    u64 *base = tmp + t * 3 * S;
    for (int k = 0; k < 4; k++) {
        u64 j = blk * 4 + k;
        int64_t r = ternary_of(wr[k]);
        int64_t e0 = gaussian_of(we0[k], dp.cdt), e1 = gaussian_of(we1[k], dp.cdt);
        int64_t me = m[t * dp.N + j] + e0;
        for (int l = 0; l < dp.nq; l++) {
            const ModConst &mc = dp.mc[l];
            base[(u64)l * dp.N + j] = from_signed(me, mc);
            base[S + (u64)l * dp.N + j] = from_signed(r, mc);
            base[2 * S + (u64)l * dp.N + j] = from_signed(e1, mc);
        }
    }
}

int launch_enc_sample(Ctx *c, const i64 *m, u64 count, u64 seed, u64 first_object, u64 *tmp, hipStream_t s)
{
    u64 total = count * c->N / 4;
    hipLaunchKernelGGL(enc_sample_kernel, dim3((u32)((total + RNG_THREADS - 1) / RNG_THREADS)), dim3(RNG_THREADS), 0,
                       s, c->dp, m, count, seed, first_object, tmp);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// ct0 = (m + e0)^ + r^ pk0, ct1 = r^ pk1 + e1^
__global__ void __launch_bounds__(RNG_THREADS)
enc_combine_kernel(DevParams dp, const u64 *tmp, u64 count, const u64 *pk, const u64 *pk_sh, u64 *ct)
{
    u64 idx = (u64)blockIdx.x * blockDim.x + threadIdx.x;  // over count * nq * N
    const u64 S = (u64)dp.nq * dp.N;
    if (idx >= count * S) return;
    u64 t = idx / S, r = idx % S;
    int l = (int)(r >> dp.log_n);
    u64 q = dp.mc[l].m;
    const u64 *T = tmp + t * 3 * S;
    u64 me = T[r], rr = T[S + r], e1 = T[2 * S + r];
    u64 c0 = add_mod(me, mul_shoup(rr, pk[r], pk_sh[r], q), q);
    u64 c1 = add_mod(e1, mul_shoup(rr, pk[S + r], pk_sh[S + r], q), q);
    ct[t * 2 * S + r] = c0;
    ct[t * 2 * S + S + r] = c1;
}

int launch_enc_combine(Ctx *c, const u64 *tmp, u64 count, u64 *ct, hipStream_t s)
{
    u64 total = count * c->nq * c->N;
    hipLaunchKernelGGL(enc_combine_kernel, dim3((u32)((total + RNG_THREADS - 1) / RNG_THREADS)), dim3(RNG_THREADS),
                       0, s, c->dp, tmp, count, c->pk, c->pk_sh, ct);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

// ---- decryption: c0 + c1 s (+ c2 s^2), NTT domain ---------------------------

__global__ void __launch_bounds__(RNG_THREADS)
dec_combine_kernel(DevParams dp, const u64 *ct, int ncomp, int nlimb, u64 count, const u64 *s, const u64 *s_sh,
                   const u64 *s2, const u64 *s2_sh, u64 *out)
{
    u64 idx = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    const u64 S = (u64)nlimb * dp.N;  // the ciphertext's first nlimb Q limbs
    if (idx >= count * S) return;
    u64 t = idx / S, r = idx % S;
    int l = (int)(r >> dp.log_n);
    u64 q = dp.mc[l].m;
    const u64 *C = ct + t * (u64)ncomp * S;
    u64 v = add_mod(C[r], mul_shoup(C[S + r], s[r], s_sh[r], q), q);
    if (ncomp == 3) v = add_mod(v, mul_shoup(C[2 * S + r], s2[r], s2_sh[r], q), q);
    out[idx] = v;
}

int launch_dec_combine(Ctx *c, const u64 *ct, int ncomp, int nlimb, u64 count, u64 *out, hipStream_t s)
{
    u64 total = count * (u64)nlimb * c->N;
    hipLaunchKernelGGL(dec_combine_kernel, dim3((u32)((total + RNG_THREADS - 1) / RNG_THREADS)), dim3(RNG_THREADS),
                       0, s, c->dp, ct, ncomp, nlimb, count, c->sk_ntt, c->sk_ntt_sh, c->sk2_ntt, c->sk2_ntt_sh, out);
    LC_HIP(c, hipGetLastError());
    return LC_OK;
}

}  // namespace lc
