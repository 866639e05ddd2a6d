// Device-side 64-bit modular arithmetic for moduli below 2^50 on gfx950.
//
// gfx950 has no 64-bit integer multiplier; v_mad_u64_u32 (32x32 + 64 -> 64)
// is the widest integer multiply.  Two forms are used:
//   * Shoup multiplication by a constant w with precomputed
//     w' = floor(w 2^64 / m): for any x < 2^64, x w - mulhi(x, w') m lies in
//     [0, 2m).  Used for NTT twiddles and per-limb constants.
//   * Split products for variable operands: a, b < 2^50 are cut into 25-bit
//     halves, a = ah 2^25 + al, and the three partial sums
//     hh = sum ah bh, hl = sum (ah bl + al bh), ll = sum al bl are kept in
//     plain 64-bit registers; every partial product is one v_mad_u64_u32 that
//     also does the accumulation, and no carry ever appears for up to 2^12
//     terms (each term < 2^51).  The sum is reduced once at the end.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lc {

typedef uint64_t u64;
typedef uint32_t u32;

constexpr u64 MASK25 = (1ull << 25) - 1;

__device__ __forceinline__ u64 csub(u64 x, u64 m) { return x >= m ? x - m : x; }
__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 m) { return csub(a + b, m); }
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 m) { return a >= b ? a - b : a + m - b; }

// x * w mod m in [0, 2m), for any x < 2^64, w < m, wsh = floor(w 2^64 / m).
__device__ __forceinline__ u64 mul_shoup_lazy(u64 x, u64 w, u64 wsh, u64 m)
{
    u64 qh = __umul64hi(x, wsh);
    return x * w - qh * m;
}
__device__ __forceinline__ u64 mul_shoup(u64 x, u64 w, u64 wsh, u64 m) { return csub(mul_shoup_lazy(x, w, wsh, m), m); }

// Per-modulus constants for the end of a split accumulation.
struct ModConst {
    u64 m;
    double qd, qinv;  // q and fl(1/q) for the FP64 Barrett form
    u64 c50, c50sh;  // 2^50 mod m and its Shoup companion
    u64 c25, c25sh;  // 2^25 mod m
    u64 one_sh;      // floor(2^64 / m): Shoup companion of 1 (Barrett reduction)
};

struct Split3 {
    u64 hh, hl, ll;
};

__device__ __forceinline__ void split_zero(Split3 &s) { s.hh = s.hl = s.ll = 0; }

// s += a * b, a, b < 2^50.
__device__ __forceinline__ void split_mac(Split3 &s, u64 a, u64 b)
{
    u32 ah = (u32)(a >> 25), al = (u32)(a & MASK25);
    u32 bh = (u32)(b >> 25), bl = (u32)(b & MASK25);
    s.hh += (u64)ah * bh;
    s.hl += (u64)ah * bl;
    s.hl += (u64)al * bh;
    s.ll += (u64)al * bl;
}

// s += a * a (the cross term counted once; reduce_split_sq doubles it).
__device__ __forceinline__ void split_sq(Split3 &s, u64 a)
{
    u32 ah = (u32)(a >> 25), al = (u32)(a & MASK25);
    s.hh += (u64)ah * ah;
    s.hl += (u64)ah * al;
    s.ll += (u64)al * al;
}

// (hh 2^50 + hl 2^25 + ll) mod m, canonical.
__device__ __forceinline__ u64 reduce_split(const Split3 &s, const ModConst &c)
{
    u64 a = mul_shoup_lazy(s.hh, c.c50, c.c50sh, c.m);
    u64 b = mul_shoup_lazy(s.hl, c.c25, c.c25sh, c.m);
    u64 d = mul_shoup_lazy(s.ll, 1, c.one_sh, c.m);
    u64 r = csub(a + b, 2 * c.m);  // < 2m
    r = csub(r + d, 2 * c.m);      // < 2m
    return csub(r, c.m);
}

// (hh 2^50 + 2 hl 2^25 + ll) mod m: the accumulation of squares.
__device__ __forceinline__ u64 reduce_split_sq(const Split3 &s, const ModConst &c)
{
    u64 a = mul_shoup_lazy(s.hh, c.c50, c.c50sh, c.m);
    u64 b = mul_shoup_lazy(s.hl, c.c25, c.c25sh, c.m);
    u64 d = mul_shoup_lazy(s.ll, 1, c.one_sh, c.m);
    b = csub(b, c.m);
    b = csub(b + b, c.m);  // 2 hl 2^25 mod m
    u64 r = csub(a + b, 2 * c.m);
    r = csub(r + d, 2 * c.m);
    return csub(r, c.m);
}

// a * b mod m for a, b < 2^50.
__device__ __forceinline__ u64 mul_mod(u64 a, u64 b, const ModConst &c)
{
    Split3 s;
    split_zero(s);
    split_mac(s, a, b);
    return reduce_split(s, c);
}

// Signed 64-bit integer reduced into [0, m).
__device__ __forceinline__ u64 from_signed(int64_t v, const ModConst &c)
{
    if (v >= 0) return csub(mul_shoup_lazy((u64)v, 1, c.one_sh, c.m), c.m);
    u64 r = csub(mul_shoup_lazy((u64)(-(v + 1)), 1, c.one_sh, c.m), c.m);  // (-v-1) mod m
    return c.m - 1 - r;
}

// ---- FP64 Barrett form (NTT butterflies) ----------------------------------
//
// gfx950 runs FP64 FMA at full rate and 32-bit integer multiplies at about
// half rate, so the NTT keeps its values as exactly-representable signed
// integers in doubles while a pass runs.  For q < 2^50, |y| <= 4q, w < q:
//   p = fl(y w),  e = fma(y, w, -p)       (y w = p + e exactly, |e| <= 2^-53 |p|)
//   k = rint(p * fl(1/q))                  (Barrett quotient estimate, |k - yw/q| <= 2)
//   r = fma(-k, q, p) + e                  (both steps exact: the values are
//                                           integers of magnitude < 2^53)
// gives r = y w - k q, an integer with |r| <= 2q.  reduce_d brings any |x| < 2^52
// to |x| <= q/2 + 1 the same way.  Every quantity stays exact, so the canonical
// residue read out at the end is the same as with integer arithmetic.
#pragma clang fp contract(off)
__device__ __forceinline__ double mulmod_d(double y, double w, double q, double qinv)
{
    double p = y * w;
    double e = __fma_rn(y, w, -p);
    double k = __builtin_rint(p * qinv);
    return __fma_rn(-k, q, p) + e;
}

__device__ __forceinline__ double reduce_d(double x, double q, double qinv)
{
    double k = __builtin_rint(x * qinv);
    return __fma_rn(-k, q, x);
}

// u64 residue (< 2^53) to double, exactly.
__device__ __forceinline__ double u64_to_d(u64 v)
{
    return __fma_rn((double)(u32)(v >> 32), 4294967296.0, (double)(u32)v);
}

// integer-valued double with |x| < 2^52 to the canonical residue in [0, q),
// still as a double.
__device__ __forceinline__ double canon_d(double x, double q, double qinv)
{
    double r = reduce_d(x, q, qinv);   // |r| <= q/2 + 1
    if (r < 0) r += q;
    if (r >= q) r -= q;
    return r;
}

// integer-valued double with |x| < 2^52 to the canonical residue in [0, q).
__device__ __forceinline__ u64 d_to_canonical(double x, double q, double qinv)
{
    double r = reduce_d(x, q, qinv);   // |r| <= q/2 + 1
    if (r < 0) r += q;
    if (r >= q) r -= q;
    u32 hi = (u32)(r * (1.0 / 4294967296.0));
    u32 lo = (u32)__fma_rn(-(double)hi, 4294967296.0, r);
    return ((u64)hi << 32) | lo;
}
#pragma clang fp contract(on)

}  // namespace lc
