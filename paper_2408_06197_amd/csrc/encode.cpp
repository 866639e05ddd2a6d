// Host FP64 encode/decode through the canonical embedding (Methods, Batch
// Encoding and Decoding) and exact CRT to centred integers.
//
// Slot j sits at zeta_j = xi^(5^j mod 2N), xi = exp(i pi / N).  With u the
// vector over odd exponents e = 2t + 1 (u_e = z_j at e = 5^j, conj(z_j) at
// -5^j), the inverse embedding is m_k = (scale / N) Re(xi^-k sum_t u_t w^-tk),
// w = exp(2 pi i / N): one length-N complex DFT.  Decoding evaluates
// sum_k (m_k xi^k) w^tk, the conjugate DFT.
#include <cmath>
#include <complex>
#include <map>
#include <mutex>
#include <vector>

#include "lc_internal.h"

namespace lc {

typedef std::complex<double> cd;

// Twiddle tables per transform size, built once: root[k] = exp(-2 pi i k / n)
// for k < n/2, and the twist xi^-k = exp(-i pi k / N) for k < N.
struct FftTables {
    std::vector<cd> root, twist;
};

static const FftTables &tables(size_t n)
{
    static std::mutex mu;
    static std::map<size_t, FftTables> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(n);
    if (it != cache.end()) return it->second;
    FftTables t;
    t.root.resize(n / 2);
    for (size_t k = 0; k < n / 2; k++) t.root[k] = std::polar(1.0, -2.0 * M_PI * (double)k / (double)n);
    t.twist.resize(n);
    for (size_t k = 0; k < n; k++) t.twist[k] = std::polar(1.0, -M_PI * (double)k / (double)n);
    return cache.emplace(n, std::move(t)).first->second;
}

// In-place iterative radix-2 DFT: sign -1 computes sum_t a_t w^-tk, sign +1
// the conjugate transform (w = exp(2 pi i / n)).
static void dft(std::vector<cd> &a, int sign)
{
    size_t n = a.size();
    const FftTables &T = tables(n);
    for (size_t i = 1, j = 0; i < n; i++) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        size_t step = n / len;
        for (size_t s = 0; s < n; s += len)
            for (size_t k = 0; k < len / 2; k++) {
                cd w = T.root[k * step];
                if (sign > 0) w = std::conj(w);
                cd u = a[s + k], v = a[s + k + len / 2] * w;
                a[s + k] = u + v;
                a[s + k + len / 2] = u - v;
            }
    }
}

void encode_host(int log_n, const double *re, const double *im, size_t nslots, double scale, i64 *m)
{
    size_t N = (size_t)1 << log_n, two_n = 2 * N;
    std::vector<cd> u(N, cd(0, 0));
    size_t e = 1;
    for (size_t j = 0; j < N / 2; j++) {
        cd z(0, 0);
        if (j < nslots) z = cd(re[j], im ? im[j] : 0.0);
        u[(e - 1) / 2] = z;
        u[(two_n - e - 1) / 2] = std::conj(z);
        e = (e * 5) % two_n;
    }
    dft(u, -1);
    const FftTables &T = tables(N);
    for (size_t k = 0; k < N; k++) {
        double v = scale / (double)N * (u[k] * T.twist[k]).real();
        m[k] = (i64)(v >= 0 ? std::floor(v + 0.5) : -std::floor(-v + 0.5));
    }
}

void decode_host(int log_n, const double *coeff, double scale, double *re, double *im)
{
    size_t N = (size_t)1 << log_n, two_n = 2 * N;
    std::vector<cd> a(N);
    const FftTables &T = tables(N);
    for (size_t k = 0; k < N; k++) a[k] = coeff[k] * std::conj(T.twist[k]);
    dft(a, +1);
    size_t e = 1;
    for (size_t j = 0; j < N / 2; j++) {
        cd v = a[(e - 1) / 2] / scale;
        re[j] = v.real();
        if (im) im[j] = v.imag();
        e = (e * 5) % two_n;
    }
}

// ---- exact CRT with little-endian multiword integers ------------------------

typedef unsigned __int128 u128;

static void mw_mul_small(std::vector<u64> &x, u64 f)  // x *= f
{
    u64 carry = 0;
    for (auto &w : x) {
        u128 t = (u128)w * f + carry;
        w = (u64)t;
        carry = (u64)(t >> 64);
    }
    if (carry) x.push_back(carry);
}

static void mw_addmul(std::vector<u64> &acc, const std::vector<u64> &x, u64 f)  // acc += x * f
{
    if (acc.size() < x.size() + 1) acc.resize(x.size() + 1, 0);
    u64 carry = 0;
    size_t i = 0;
    for (; i < x.size(); i++) {
        u128 t = (u128)x[i] * f + acc[i] + carry;
        acc[i] = (u64)t;
        carry = (u64)(t >> 64);
    }
    for (; carry && i < acc.size(); i++) {
        u128 t = (u128)acc[i] + carry;
        acc[i] = (u64)t;
        carry = (u64)(t >> 64);
    }
    if (carry) acc.push_back(carry);
}

static int mw_cmp(const std::vector<u64> &a, const std::vector<u64> &b)
{
    size_t n = std::max(a.size(), b.size());
    for (size_t i = n; i-- > 0;) {
        u64 x = i < a.size() ? a[i] : 0, y = i < b.size() ? b[i] : 0;
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}

static void mw_sub(std::vector<u64> &a, const std::vector<u64> &b)  // a -= b, a >= b
{
    u64 borrow = 0;
    for (size_t i = 0; i < a.size(); i++) {
        u64 y = i < b.size() ? b[i] : 0;
        u128 t = (u128)a[i] - y - borrow;
        a[i] = (u64)t;
        borrow = (u64)(t >> 127) & 1;
    }
}

// Correctly rounded conversion: the top two non-zero words carry at least 65
// significant bits; any non-zero word below them sets a sticky bit.
static double mw_to_double(const std::vector<u64> &a)
{
    size_t top = a.size();
    while (top > 0 && a[top - 1] == 0) top--;
    if (top == 0) return 0.0;
    if (top <= 2) return (double)(((u128)(top == 2 ? a[1] : 0) << 64) | a[0]);
    u128 hi = ((u128)a[top - 1] << 64) | a[top - 2];
    bool sticky = false;
    for (size_t i = 0; i + 2 < top; i++) sticky |= a[i] != 0;
    if (sticky) hi |= 1;
    return std::ldexp((double)hi, (int)(64 * (top - 2)));
}

void crt_to_double(const std::vector<u64> &q, const u64 *res, size_t ncoeff, size_t stride, double *out)
{
    size_t L = q.size();
    std::vector<u64> Q{1};
    for (u64 qi : q) mw_mul_small(Q, qi);
    std::vector<u64> half = Q;  // Q / 2
    for (size_t i = 0; i < half.size(); i++) {
        half[i] >>= 1;
        if (i + 1 < half.size()) half[i] |= half[i + 1] << 63;
    }
    std::vector<std::vector<u64>> Qi(L);
    std::vector<u64> inv(L);
    for (size_t i = 0; i < L; i++) {
        Qi[i] = {1};
        u64 r = 1;
        for (size_t j = 0; j < L; j++)
            if (j != i) {
                mw_mul_small(Qi[i], q[j]);
                r = (u64)((u128)r * (q[j] % q[i]) % q[i]);
            }
        // inverse of r mod q_i by Fermat
        u64 e = q[i] - 2, b = r, acc = 1;
        for (; e; e >>= 1) {
            if (e & 1) acc = (u64)((u128)acc * b % q[i]);
            b = (u64)((u128)b * b % q[i]);
        }
        inv[i] = acc;
    }
    for (size_t t = 0; t < ncoeff; t++) {
        std::vector<u64> acc(Q.size() + 1, 0);
        for (size_t i = 0; i < L; i++) {
            u64 y = (u64)((u128)(res[i * stride + t] % q[i]) * inv[i] % q[i]);
            mw_addmul(acc, Qi[i], y);
        }
        while (mw_cmp(acc, Q) >= 0) mw_sub(acc, Q);
        if (mw_cmp(acc, half) > 0) {
            std::vector<u64> neg = Q;
            mw_sub(neg, acc);
            out[t] = -mw_to_double(neg);
        } else {
            out[t] = mw_to_double(acc);
        }
    }
}

}  // namespace lc
