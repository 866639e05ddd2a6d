// CKKS rescaling by the last Q limb of a ciphertext (levels of the CKKS
// Scheme Description): ct' = round(ct / q_t) modulo q_0 ... q_{t-1}, for a
// ciphertext with nlimb = t + 1 limbs in the NTT domain.  In RNS form,
// limb i of the result is (c_i - r) q_t^-1 mod q_i, where r is the centred
// residue of c modulo q_t (|r| < q_t / 2): (c - r) / q_t is then the nearest
// integer to c / q_t, whatever representative of c modulo Q_t is taken.  r
// lives in the coefficient domain, so the last limb goes through one inverse
// transform and its centred value, reduced modulo each q_i, through a forward
// transform per remaining limb.
#include "lc_internal.h"

namespace lc {

constexpr int RS_THREADS = 256;

// dst[g][j] = src[g * sstride + j], j < N
__global__ void __launch_bounds__(RS_THREADS) rs_copy_kernel(const u64 *src, u64 sstride, u64 *dst, u64 N, u64 total)
{
    const u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    dst[e] = src[(e / N) * sstride + e % N];
}

// lift[g][i][j] = centred(r[g][j] mod q_t) mod q_i, i < t
__global__ void __launch_bounds__(RS_THREADS)
rs_lift_kernel(DevParams dp, const u64 *r, int t, u64 total, u64 *lift)
{
    const u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const u64 N = dp.N, j = e % N, gi = e / N;
    const int i = (int)(gi % (u64)t);
    const u64 g = gi / (u64)t;
    const u64 qt = dp.mc[t].m, v = r[g * N + j];
    const i64 centred = v > qt / 2 ? (i64)v - (i64)qt : (i64)v;
    lift[e] = from_signed(centred, dp.mc[i]);
}

// out[g][i][j] = (ct[g][i][j] - lift[g][i][j]) q_t^-1 mod q_i
__global__ void __launch_bounds__(RS_THREADS)
rs_combine_kernel(DevParams dp, const u64 *ct, int nlimb, const u64 *lift, u64 total, u64 *out)
{
    const u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int t = nlimb - 1;
    const u64 N = dp.N, j = e % N, gi = e / N;
    const int i = (int)(gi % (u64)t);
    const u64 g = gi / (u64)t;
    const u64 q = dp.mc[i].m;
    const u64 d = sub_mod(ct[(g * nlimb + i) * N + j], lift[e], q);
    out[e] = mul_shoup(d, dp.rs_inv[t * dp.nq + i], dp.rs_inv_sh[t * dp.nq + i], q);
}

static u32 rs_blocks(u64 total) { return (u32)((total + RS_THREADS - 1) / RS_THREADS); }

int launch_rescale(Ctx *c, const u64 *ct, u64 count, int ncomp, int nlimb, u64 *out, hipStream_t s)
{
    const u64 N = c->N;
    const int t = nlimb - 1;
    const u64 groups = count * (u64)ncomp;
    if (!groups) return LC_OK;
    // workspace: the last limbs [G][N] and their lifts [G][t][N], in chunks of at most ~1 GiB
    const u64 per_group = (1 + (u64)t) * N * sizeof(u64);
    const u64 chunk = std::min<u64>(groups, std::max<u64>(1, (1ull << 30) / per_group));
    u64 *ws = ws_get(c, WS_RESCALE, chunk * per_group, s);
    if (!ws) return LC_ENOMEM;
    const bool two_pass = c->log_n >= 10 && c->log_n <= 17;
    int rc;
    for (u64 g0 = 0; g0 < groups; g0 += chunk) {
        const u64 G = std::min(chunk, groups - g0);
        u64 *r = ws, *lift = ws + G * N;
        const u64 *src = ct + g0 * (u64)nlimb * N;
        // r = INTT(last limb)
        PolyBatch ib{r, G, 1, 1, t, 0};
        if (two_pass) {
            ib.in_base = src + (u64)t * N;
            ib.in_gstride = (u64)nlimb;
        } else {
            hipLaunchKernelGGL(rs_copy_kernel, dim3(rs_blocks(G * N)), dim3(RS_THREADS), 0, s, src + (u64)t * N,
                               (u64)nlimb * N, r, N, G * N);
            LC_HIP(c, hipGetLastError());
        }
        if ((rc = launch_ntt_inv(c, ib, s))) return rc;
        hipLaunchKernelGGL(rs_lift_kernel, dim3(rs_blocks(G * t * N)), dim3(RS_THREADS), 0, s, c->dp, r, t,
                           G * (u64)t * N, lift);
        LC_HIP(c, hipGetLastError());
        if ((rc = launch_ntt_fwd(c, PolyBatch{lift, G, t, (u64)t, 0, 0}, s))) return rc;
        hipLaunchKernelGGL(rs_combine_kernel, dim3(rs_blocks(G * t * N)), dim3(RS_THREADS), 0, s, c->dp, src, nlimb,
                           lift, G * (u64)t * N, out + g0 * (u64)t * N);
        LC_HIP(c, hipGetLastError());
    }
    return LC_OK;
}

}  // namespace lc
