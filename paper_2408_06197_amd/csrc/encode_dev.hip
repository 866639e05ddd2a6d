// Device FP64 encode of real vectors (Methods, Batch Encoding and Decoding):
// the same computation as encode_host in encode.cpp, batched on the GPU.
//
// Slot j of z sits at the odd exponent e = 5^j mod 2N and, conjugated, at
// -5^j; over t = (e - 1) / 2 this gives a length-N vector u (real for real
// z), and m_k = round((scale / N) Re(xi^-k X_k)) with X_k = sum_t u_t w^-tk,
// w = exp(2 pi i / N), xi = exp(i pi / N).  The length-N transform is done
// as N = N1 N2 in two passes through HBM (t = t1 + N1 t2, k = k2 + N2 k1):
//   pass A, per column t1: N2-point transforms over t2, then the twiddle
//          w^-(t1 k2), stored as Y[k2][t1];
//   pass B, per row k2:    N1-point transforms over t1, giving X at
//          k = k2 + N2 k1, then the twist, scale and rounding.
// Sub-transforms are radix-2 decimation in time in LDS (bit-reversed load).
// Rounding is half away from zero as on the host; a coefficient may differ by
// one from another FP64 evaluation order when its value lies within rounding
// error of a half-integer.
#include "lc_internal.h"

namespace lc {

constexpr int ENC_THREADS = 256;
constexpr int ENC_LDS = 2048;  // complex values per workgroup (32 KiB)

struct Cplx {
    double re, im;
};

__device__ __forceinline__ Cplx cmul(Cplx a, Cplx b)
{
    return Cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

__device__ __forceinline__ u32 bitrev(u32 x, int bits) { return __brev(x) >> (32 - bits); }

// In-place radix-2 DIT transforms of `rows` sequences of length 2^lg in LDS
// (input in bit-reversed order, output in natural order), sign -1:
// X_k = sum_t x_t exp(-2 pi i t k / 2^lg).  W[j] = exp(-2 pi i j / N).
__device__ void lds_dft(Cplx *a, int rows, int lg, const Cplx *W, int log_n)
{
    const int len = 1 << lg, half_total = rows * (len >> 1);
    for (int s = 1; s <= lg; s++) {
        const int h = 1 << (s - 1);
        __syncthreads();
        for (int b = threadIdx.x; b < half_total; b += blockDim.x) {
            const int r = b >> (lg - 1), q = b & ((len >> 1) - 1);
            const int j = q & (h - 1), g = q >> (s - 1);
            Cplx *x = a + r * len + g * 2 * h + j;
            const Cplx w = W[(u64)j << (log_n - s)];  // exp(-2 pi i j / 2h)
            const Cplx v = cmul(x[h], w), u = x[0];
            x[0] = Cplx{u.re + v.re, u.im + v.im};
            x[h] = Cplx{u.re - v.re, u.im - v.im};
        }
    }
    __syncthreads();
}

// Pass A: workgroup = (ca columns t1, vector).  Y[v][k2][t1].
__global__ void __launch_bounds__(ENC_THREADS)
enc_pass_a(const double *z, u64 z_stride, u64 nslots, const int *slot, const Cplx *W, int log_n, int lg1, int lg2,
           int ca, Cplx *Y)
{
    __shared__ Cplx a[ENC_LDS];
    const u64 N = (u64)1 << log_n, N1 = (u64)1 << lg1, N2 = (u64)1 << lg2;
    const u64 v = blockIdx.y;
    const int c0 = blockIdx.x * ca;
    const double *zv = z + v * z_stride;
    for (int e = threadIdx.x; e < ca * (int)N2; e += blockDim.x) {
        const int c = e >> lg2, t2 = e & (int)(N2 - 1);
        const u64 t = (u64)(c0 + c) + N1 * (u64)t2;
        const int j = slot[t];
        const double re = (u64)j < nslots ? zv[j] : 0.0;
        a[c * N2 + bitrev((u32)t2, lg2)] = Cplx{re, 0.0};
    }
    lds_dft(a, ca, lg2, W, log_n);
    Cplx *Yv = Y + v * N;
    for (int e = threadIdx.x; e < ca * (int)N2; e += blockDim.x) {
        const int c = e & (ca - 1), k2 = e / ca;  // consecutive threads: consecutive t1
        const u64 t1 = (u64)(c0 + c);
        const Cplx y = cmul(a[c * N2 + k2], W[(t1 * (u64)k2) & (N - 1)]);
        Yv[(u64)k2 * N1 + t1] = y;
    }
}

// Pass B: workgroup = (rb rows k2, vector).  m[v][k] for k = k2 + N2 k1.
__global__ void __launch_bounds__(ENC_THREADS)
enc_pass_b(const Cplx *Y, const Cplx *W, const Cplx *twist, int log_n, int lg1, int lg2, int rb, double scale,
           i64 *m)
{
    __shared__ Cplx a[ENC_LDS];
    const u64 N = (u64)1 << log_n, N1 = (u64)1 << lg1, N2 = (u64)1 << lg2;
    const u64 v = blockIdx.y;
    const int r0 = blockIdx.x * rb;
    const Cplx *Yv = Y + v * N;
    for (int e = threadIdx.x; e < rb * (int)N1; e += blockDim.x) {
        const int r = e >> lg1, t1 = e & (int)(N1 - 1);
        a[r * N1 + bitrev((u32)t1, lg1)] = Yv[(u64)(r0 + r) * N1 + t1];
    }
    lds_dft(a, rb, lg1, W, log_n);
    const double f = scale / (double)N;
    i64 *mv = m + v * N;
    for (int e = threadIdx.x; e < rb * (int)N1; e += blockDim.x) {
        const int r = e % rb, k1 = e / rb;  // consecutive threads: consecutive k
        const u64 k = (u64)(r0 + r) + N2 * (u64)k1;
        const Cplx x = a[r * N1 + k1], tw = twist[k];
        const double val = f * (x.re * tw.re - x.im * tw.im);
        mv[k] = (i64)(val >= 0 ? floor(val + 0.5) : -floor(-val + 0.5));
    }
}

// Tables on the device, built on first use: W[j] = exp(-2 pi i j / N),
// twist[k] = exp(-i pi k / N), slot[t] = j with 5^j = +-(2t + 1) mod 2N.
static int encode_tables(Ctx *c)
{
    if (c->enc_w) return LC_OK;
    const u64 N = c->N, two_n = 2 * N;
    std::vector<Cplx> w(N), tw(N);
    for (u64 k = 0; k < N; k++) {
        w[k] = Cplx{std::cos(-2.0 * M_PI * (double)k / (double)N), std::sin(-2.0 * M_PI * (double)k / (double)N)};
        tw[k] = Cplx{std::cos(-M_PI * (double)k / (double)N), std::sin(-M_PI * (double)k / (double)N)};
    }
    std::vector<int> slot(N, -1);
    u64 e = 1;
    for (u64 j = 0; j < N / 2; j++) {
        slot[(e - 1) / 2] = (int)j;
        slot[(two_n - e - 1) / 2] = (int)j;
        e = e * 5 % two_n;
    }
    Cplx *dw = (Cplx *)dev_alloc(c, N * sizeof(Cplx));
    Cplx *dt = (Cplx *)dev_alloc(c, N * sizeof(Cplx));
    int *ds = (int *)dev_alloc(c, N * sizeof(int));
    if (!dw || !dt || !ds) return fail(c, LC_ENOMEM, "encode table allocation failed");
    LC_HIP(c, hipMemcpy(dw, w.data(), N * sizeof(Cplx), hipMemcpyHostToDevice));
    LC_HIP(c, hipMemcpy(dt, tw.data(), N * sizeof(Cplx), hipMemcpyHostToDevice));
    LC_HIP(c, hipMemcpy(ds, slot.data(), N * sizeof(int), hipMemcpyHostToDevice));
    c->table_bytes += N * (2 * sizeof(Cplx) + sizeof(int));
    c->enc_w = dw;
    c->enc_twist = dt;
    c->enc_slot = ds;
    return LC_OK;
}

int launch_encode(Ctx *c, const double *z, u64 count, u64 nslots, u64 z_stride, double scale, i64 *m, hipStream_t s)
{
    if (c->log_n < 2 || c->log_n > 20) return fail(c, LC_EUNSUP, "device encode needs 4 <= N <= 2^20");
    int rc;
    if ((rc = encode_tables(c))) return rc;
    if (!count) return LC_OK;
    const int lg1 = c->log_n / 2, lg2 = c->log_n - lg1;
    const u64 N = c->N, N1 = (u64)1 << lg1, N2 = (u64)1 << lg2;
    const int ca = (int)std::min<u64>(N1, ENC_LDS / N2), rb = (int)std::min<u64>(N2, ENC_LDS / N1);
    if (ca < 1 || rb < 1) return fail(c, LC_EUNSUP, "device encode: transform too long for one workgroup");
    const u64 chunk = std::min<u64>(count, std::max<u64>(1, (256ull << 20) / (N * sizeof(Cplx))));
    Cplx *Y = (Cplx *)ws_get(c, WS_ENCODE, chunk * N * sizeof(Cplx), s);
    if (!Y) return LC_ENOMEM;
    const Cplx *W = (const Cplx *)c->enc_w, *T = (const Cplx *)c->enc_twist;
    for (u64 v0 = 0; v0 < count; v0 += chunk) {
        const u64 B = std::min(chunk, count - v0);
        hipLaunchKernelGGL(enc_pass_a, dim3((u32)(N1 / ca), (u32)B), dim3(ENC_THREADS), 0, s, z + v0 * z_stride,
                           z_stride, nslots, c->enc_slot, W, c->log_n, lg1, lg2, ca, Y);
        LC_HIP(c, hipGetLastError());
        hipLaunchKernelGGL(enc_pass_b, dim3((u32)(N2 / rb), (u32)B), dim3(ENC_THREADS), 0, s, Y, W, T, c->log_n, lg1,
                           lg2, rb, scale, m + v0 * N);
        LC_HIP(c, hipGetLastError());
    }
    return LC_OK;
}

}  // namespace lc
