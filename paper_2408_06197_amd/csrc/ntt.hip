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

__device__ __forceinline__ bool poly_of_block(const DevParams &dp, const PolyBatch &pb, u64 p, u64 *&ptr, int &mi)
{
    u64 g = p / (u64)pb.nlimb;
    int l = (int)(p % (u64)pb.nlimb);
    mi = pb.limb0 + l;
    if (pb.skip_own_digit && mi < dp.nq && (int)(g % (u64)dp.dnum) == mi / dp.alpha) return false;
    ptr = pb.base + (g * pb.gstride + (u64)l) * dp.N;
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

// Pass plan: one pass up to N = 4096, two passes above.
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

static int launch(Ctx *c, const PolyBatch &b, hipStream_t s, bool inverse)
{
    PassArgs pass[2];
    int np = plan_passes(c->log_n, pass);
    u64 npoly = b.count * (u64)b.nlimb;
    if (npoly == 0) return LC_OK;
    if (npoly > 0x7fffffffull) return fail(c, LC_EINVAL, "too many polynomials in one NTT batch");
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
