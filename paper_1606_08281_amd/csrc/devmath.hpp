// devmath.hpp -- device-side random streams and elementary functions.
//
// Every decision of the particle filter (when an interval ends, which
// reaction fires, which ancestor a slot takes) depends on these values, so
// they are built only from correctly rounded IEEE-754 operations (+ - * /,
// fma, exact scalings) in a fixed order.  The library is compiled with
// -ffp-contract=off; fused multiply-adds appear only where written.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

namespace lik {

// ---------------------------------------------------------------------------
// Lanes of a wavefront.  lane_id() is the lane index behind an empty asm
// statement, so the compiler recomputes what it derives from it (LDS and
// exchange addresses) where it is used instead of keeping those values in
// registers across a whole persistent loop.  Exchanges go through
// ds_bpermute with addresses from that index.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() {
    int l = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    asm volatile("" : "+v"(l));
    return l;
}
__device__ __forceinline__ uint32_t lane_read(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}
__device__ __forceinline__ uint64_t lane_read(uint64_t v, int src) {
    const uint32_t lo = lane_read((uint32_t)v, src), hi = lane_read((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double lane_read(double v, int src) {
    return __longlong_as_double((long long)lane_read((uint64_t)__double_as_longlong(v), src));
}
__device__ __forceinline__ float lane_read(float v, int src) {
    return __uint_as_float(lane_read(__float_as_uint(v), src));
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): per round two
// 32x32->64-bit products, the high halves xor'ed with the other words and
// the round key; the key advances by the Weyl constants between rounds.
struct Block4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Block4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        // three-input exclusive or in one gfx950 instruction (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Block4{c0, c1, c2, c3};
}

// The same generator for an event's counter (n, j, c2, c3) whose last two
// words and key are wave-uniform: the exclusive-or of two uniform words in
// rounds 1 and 2 is formed once, on the scalar unit (a vector instruction
// reads one scalar operand, so the general form copies the other into a
// vector register for every event).  Same block as philox4x32_10.
__device__ __forceinline__ Block4 philox4x32_10_event(uint32_t n, uint32_t j, uint32_t c2,
                                                      uint32_t c3, uint32_t k0, uint32_t k1) {
    const uint64_t q1 = (uint64_t)c2 * 0xCD9E8D57u;  // uniform
    uint32_t a1 = (uint32_t)(q1 >> 32) ^ k0;         // round 1: hi(c2 M1) ^ key
    uint32_t b1 = c3 ^ k1;
    uint32_t a2 = (uint32_t)q1 ^ (k0 + 0x9E3779B9u);  // round 2: c1 ^ key
    asm("" : "+s"(a1), "+s"(b1), "+s"(a2));
    // round 1
    const uint64_t p0 = (uint64_t)n * 0xD2511F53u;
    uint32_t c0 = j ^ a1;
    uint32_t w2 = (uint32_t)(p0 >> 32) ^ b1;
    uint32_t w3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    // round 2 (its c1 is lo(c2 M1), folded into a2)
    {
        const uint64_t r0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t r1 = (uint64_t)w2 * 0xCD9E8D57u;
        c0 = (uint32_t)(r1 >> 32) ^ a2;
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(r0 >> 32), w3, k1, 0x96);
        w3 = (uint32_t)r0;
        const uint32_t c1 = (uint32_t)r1;
        w2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
        uint32_t c1r = c1;
#pragma unroll
        for (int round = 2; round < 10; ++round) {
            const uint64_t s0 = (uint64_t)c0 * 0xD2511F53u;
            const uint64_t s1 = (uint64_t)w2 * 0xCD9E8D57u;
            const uint32_t m0 = __builtin_amdgcn_bitop3_b32((uint32_t)(s1 >> 32), c1r, k0, 0x96);
            const uint32_t m2 = __builtin_amdgcn_bitop3_b32((uint32_t)(s0 >> 32), w3, k1, 0x96);
            c1r = (uint32_t)s1;
            w3 = (uint32_t)s0;
            c0 = m0;
            w2 = m2;
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        return Block4{c0, c1r, w2, w3};
    }
}

// ln 2 split: 32 leading significant bits (so e * LN2_HI is exact for any
// binary64 exponent) and the binary64 nearest to the remainder.
constexpr double kLn2Hi = 0x1.62e42feep-1;
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
constexpr double kInvLn2 = 0x1.71547652b82fep+0;
constexpr double kHalfSqrt2 = 0x1.6a09e667f3bcdp-1;  // (nearest sqrt 2) / 2, exact halving

// a * b + c with one rounding, as one three-operand v_fma_f64.  In a loop the
// compiler keeps each Horner coefficient in registers and, choosing the
// two-operand v_fmac_f64, copies it into the accumulator before every step;
// this form takes the coefficient as a plain source (one instruction per
// step instead of two).  Same operation as fma(): IEEE fused multiply-add.
__device__ __forceinline__ double fma_f64(double a, double b, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// a * k + k with one rounding, k taken once from scalar registers (one
// v_fma_f64; the two-operand form would first copy k into the accumulator).
__device__ __forceinline__ double fma_f64_s(double a, double k) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %2" : "=v"(r) : "v"(a), "s"(k));
    return r;
}

// n / d correctly rounded, for operands the division sequence needs neither
// to scale nor to fix up: d normal in [1, 4], n zero or with |n| in
// [2^-60, 4] (the log's f / (2 + f)).  These are the steps of the IEEE
// division sequence -- reciprocal estimate, two Newton steps, one residual
// correction -- whose range scaling and special-case fix-up are the identity
// on such operands: the same quotient, bit for bit, in three fewer
// instructions.
__device__ __forceinline__ double div_inrange(double n, double d) {
    double y = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-d, y, 1.0);
    y = __builtin_fma(y, e, y);
    const double q = n * y;
    const double r = __builtin_fma(-d, q, n);
    return __builtin_fma(r, y, q);
}

// The binary32 counterpart (one Newton step, two residual corrections, as
// the binary32 division sequence takes them).
__device__ __forceinline__ float divf_inrange(float n, float d) {
    float y = __builtin_amdgcn_rcpf(d);
    const float e = __builtin_fmaf(-d, y, 1.0f);
    y = __builtin_fmaf(e, y, y);
    float q = n * y;
    float r = __builtin_fmaf(-d, q, n);
    q = __builtin_fmaf(r, y, q);
    r = __builtin_fmaf(-d, q, n);
    return __builtin_fmaf(r, y, q);
}

// Natural logarithm of x > 0 (x = 0 -> -inf).  Reduction x = 2^e m,
// m in [sqrt(1/2), sqrt(2)]; with f = m - 1 and s = f / (2 + f),
// log m = 2 atanh s = t + t z Q(z), t = 2s, z = s^2,
// Q(z) = 1/3 + z/5 + ... + z^9/21; log x = e ln2_hi + (e ln2_lo + log m).
__device__ __forceinline__ double dlog_pos(double x);
__device__ __forceinline__ double dlog(double x) {
    if (x == 0.0) return -__builtin_inf();
    return dlog_pos(x);
}

// The same for x > 0 (no test for zero: the SSA's uniforms are in (0, 1]).
__device__ __forceinline__ double dlog_pos(double x) {
    const double mant = __builtin_amdgcn_frexp_mant(x);  // [1/2, 1), exact, subnormals too
    int e = __builtin_amdgcn_frexp_exp(x);
    double m;
    if (mant > kHalfSqrt2) {
        m = mant;
    } else {
        m = mant * 2.0;
        e = e - 1;
    }
    const double f = m - 1.0;
    const double s = div_inrange(f, 2.0 + f);  // f in [-0.293, 0.415]
    const double z = s * s;
    double q = 1.0 / 21.0;
    q = fma_f64(q, z, 1.0 / 19.0);
    q = fma_f64(q, z, 1.0 / 17.0);
    q = fma_f64(q, z, 1.0 / 15.0);
    q = fma_f64(q, z, 1.0 / 13.0);
    q = fma_f64(q, z, 1.0 / 11.0);
    q = fma_f64(q, z, 1.0 / 9.0);
    q = fma_f64(q, z, 1.0 / 7.0);
    q = fma_f64(q, z, 1.0 / 5.0);
    q = fma_f64(q, z, 1.0 / 3.0);
    const double t = 2.0 * s;
    const double w = t * z;
    const double lm = __builtin_fma(w, q, t);
    const double ed = (double)e;
    return ed * kLn2Hi + (ed * kLn2Lo + lm);
}

// exp(d) for d <= 0 (d < -708 or -inf -> 0): k = floor(d/ln2 + 1/2),
// r = (d - k ln2_hi) - k ln2_lo, exp r = sum_{i<=13} r^i / i! (Horner),
// result exp(r) 2^k (always a normal number in this range).
__device__ __forceinline__ double dexp_nonpos(double d) {
    if (!(d >= -708.0)) return 0.0;
    const double kd = __builtin_floor(d * kInvLn2 + 0.5);
    const double r = (d - kd * kLn2Hi) - kd * kLn2Lo;
    double p = 1.0 / 6227020800.0;  // 1/13!
    p = __builtin_fma(p, r, 1.0 / 479001600.0);
    p = __builtin_fma(p, r, 1.0 / 39916800.0);
    p = __builtin_fma(p, r, 1.0 / 3628800.0);
    p = __builtin_fma(p, r, 1.0 / 362880.0);
    p = __builtin_fma(p, r, 1.0 / 40320.0);
    p = __builtin_fma(p, r, 1.0 / 5040.0);
    p = __builtin_fma(p, r, 1.0 / 720.0);
    p = __builtin_fma(p, r, 1.0 / 120.0);
    p = __builtin_fma(p, r, 1.0 / 24.0);
    p = __builtin_fma(p, r, 1.0 / 6.0);
    p = __builtin_fma(p, r, 1.0 / 2.0);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_amdgcn_ldexp(p, (int)kd);
}

// binary32 logarithm (FP32-mixed event times): the same reduction, series
// to z^4/11, ln 2 split as 16 significant bits + remainder.
constexpr float kLn2HiF = 0x1.62e4p-1f;
constexpr float kLn2LoF = 0x1.7f7d1cp-20f;
constexpr float kHalfSqrt2F = 0x1.6a09e6p-1f;

__device__ __forceinline__ float flog_pos(float x);
__device__ __forceinline__ float flog(float x) {
    if (x == 0.0f) return -__builtin_inff();
    return flog_pos(x);
}

// The same for x > 0.
__device__ __forceinline__ float flog_pos(float x) {
    const float mant = __builtin_amdgcn_frexp_mantf(x);
    int e = __builtin_amdgcn_frexp_expf(x);
    float m;
    if (mant > kHalfSqrt2F) {
        m = mant;
    } else {
        m = mant * 2.0f;
        e = e - 1;
    }
    const float f = m - 1.0f;
    const float s = divf_inrange(f, 2.0f + f);
    const float z = s * s;
    float q = 1.0f / 11.0f;
    q = __builtin_fmaf(q, z, 1.0f / 9.0f);
    q = __builtin_fmaf(q, z, 1.0f / 7.0f);
    q = __builtin_fmaf(q, z, 1.0f / 5.0f);
    q = __builtin_fmaf(q, z, 1.0f / 3.0f);
    const float t = 2.0f * s;
    const float w = t * z;
    const float lm = __builtin_fmaf(w, q, t);
    const float ef = (float)e;
    return ef * kLn2HiF + (ef * kLn2LoF + lm);
}

// A value equal on every lane, moved to scalar registers.
__device__ __forceinline__ double wave_uniform(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float wave_uniform(float v) {
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}
__device__ __forceinline__ uint32_t wave_uniform(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t wave_uniform(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
template <class T>
__device__ __forceinline__ T *wave_uniform(T *p) {
    return reinterpret_cast<T *>(wave_uniform((uint64_t)reinterpret_cast<unsigned long long>(p)));
}

}  // namespace lik
