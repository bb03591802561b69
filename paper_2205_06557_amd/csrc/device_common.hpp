// device_common.hpp -- shared device helpers of libodust: the counter-based
// generator, uniform and normal draws, fixed-point accumulation and wave
// reductions.  Units inside the kernels are dimensionless: lengths in the
// electron Debye length r_De, times in 1/omega_pi, velocities in
// c_s = r_De omega_pi, charges in e.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace odk {

constexpr int kMaxDust = 32;
constexpr double kPi = 3.14159265358979323846;

// Random-stream purposes (third counter word).
enum : uint64_t { kInitPos = 0, kInitVel = 1, kColl = 2, kReinj = 3 };

// Per-ion event byte.
enum : uint8_t { kEvNone = 0, kEvExit = 1, kEvAbsBase = 2, kEvCollBit = 0x80 };

// Device status bits.
enum : int { kStNaN = 1, kStPlace = 2, kStOverflow = 4 };

// Fixed-point scales of the integer accumulators (two's-complement int64
// sums are associative, so the totals do not depend on the order in which
// blocks add them).
constexpr double kForceScale = 4294967296.0;    // 2^32: Eq. (1) sums, dimensionless
constexpr double kMomScale = 4294967296.0;      // 2^32: absorbed velocity sums, c_s

// Counters that every block adds to are spread over kSlots addresses (slot =
// block index mod kSlots): device-scope atomics on one address serialise, and
// thousands of blocks adding to one word would take tens of microseconds.
// Each slot of a counter has a 128-byte cache line of its own (the memory
// side performs atomics on a line one at a time), so a counter's slots are
// kPad64 (8-byte) or kPad32 (4-byte) words apart.
constexpr int kSlots = 64;
constexpr int kPad64 = 16, kPad32 = 32;

// Layout of one system's control block (device memory, int64/double words).
struct alignas(128) Ctl {
    unsigned long long acc[kMaxDust][8];   // [3] absorbed count, [4..6] sum v ([0..2], [7] unused)
    unsigned long long part[kSlots][kMaxDust][3];  // Eq.(1) sums, per slot (block index mod kSlots)
    unsigned long long n_exit[kSlots][kPad64];     // exits, per slot ([s][0])
    unsigned long long n_coll[kSlots][kPad64];     // collisions, per slot ([s][0])
    unsigned int ticket_slot[kSlots][kPad32];      // tail blocks of the slot that have finished ([s][0])
    unsigned int lost_seg[kSlots * kPad32];        // lost-list segment lengths (single system), [s * kPad32]
    double Q[kMaxDust];                    // charge, e
    double last[kMaxDust][16];             // [0] Q^n, [1..12] F parts (SI), [13] absorbed count
    double sums[kMaxDust][16];             // running sums over recorded steps
    long long step;                        // step counter n
    long long nrec;                        // recorded steps
    long long last_exit, last_coll;
    int status;
    unsigned int ticket;                   // slots of the tail whose blocks have all finished
    unsigned int lost_ticket;              // reinjection blocks that have finished
    int pad[5];
};
static_assert(offsetof(Ctl, n_exit) % 128 == 0 && offsetof(Ctl, n_coll) % 128 == 0 &&
                  offsetof(Ctl, ticket_slot) % 128 == 0 && offsetof(Ctl, lost_seg) % 128 == 0,
              "slot counters start on cache lines");

// ---------------------------------------------------------------------------
// Philox4x64 with 10 rounds (Salmon et al., SC'11): per round two 64x64->128
// products; the words are permuted and the high halves mixed with the key;
// the key advances by two Weyl increments between rounds.
struct U64x4 {
    uint64_t w[4];
};

__host__ __device__ inline void mul128(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo)
{
#if defined(__HIP_DEVICE_COMPILE__)
    lo = a * b;
    hi = __umul64hi(a, b);
#else
    unsigned __int128 p = (unsigned __int128)a * b;
    lo = (uint64_t)p;
    hi = (uint64_t)(p >> 64);
#endif
}

__host__ __device__ inline U64x4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                        uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t h0, l0, h1, l1;
        mul128(M0, c0, h0, l0);
        mul128(M1, c2, h1, l1);
        const uint64_t t0 = h1 ^ c1 ^ k0;
        const uint64_t t2 = h0 ^ c3 ^ k1;
        c0 = t0;
        c1 = l1;
        c2 = t2;
        c3 = l0;
        k0 += W0;
        k1 += W1;
    }
    U64x4 o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

// Uniform strictly inside (0,1): 52 high bits plus one half, over 2^52.
__host__ __device__ inline double unit(uint64_t w)
{
    return ((double)(w >> 12) + 0.5) * 2.220446049250313080847e-16;
}

// Box-Muller: two standard normals from two uniforms.
__device__ inline void gauss2(double ua, double ub, double& g1, double& g2)
{
    const double m = sqrt(-2.0 * log(ua));
    double s, c;
    sincos(2.0 * kPi * ub, &s, &c);
    g1 = m * c;
    g2 = m * s;
}

// ---------------------------------------------------------------------------
// FP64 pieces of the screened pair term without a division.
//
// 1/sqrt(x), x > 0: the hardware estimate (about 24 correct bits) and one
// third-order Newton-Raphson correction, y (1 + e/2 + 3e^2/8) with
// e = 1 - x y^2 (the series of (1 - e)^(-1/2)), which triples the correct
// bits (measured on gfx950 within 1.3 ulp).
__device__ inline double rsq_f64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// e^(-r) for r >= 0 (large r clamped, where the result is 0 in FP64):
// Cody-Waite reduction r = n ln2 - f with ln 2 split into a 32-bit head
// (n * head exact) and its remainder, |f| <= ln2 / 2, then the Taylor
// polynomial of e^f to degree 13 (remainder below 1e-17) by Horner, scaled
// by 2^n (measured on gfx950 within 1.3 ulp).
__device__ inline double exp_neg_f64(double r)
{
    const double kLog2e = 1.4426950408889634;
    const double kLn2Hi = 0.6931471803691238;         // ln 2 to 32 significant bits
    const double kLn2Lo = 1.9082149292705877e-10;     // ln 2 - kLn2Hi
    const double x = -fmin(r, 800.0);
    const double n = rint(x * kLog2e);
    const double f = fma(-n, kLn2Lo, fma(-n, kLn2Hi, x));
    double p = 1.6059043836821613e-10;                // 1/13!
    p = fma(p, f, 2.08767569878681e-09);              // 1/12!
    p = fma(p, f, 2.505210838544172e-08);             // 1/11!
    p = fma(p, f, 2.755731922398589e-07);             // 1/10!
    p = fma(p, f, 2.7557319223985893e-06);            // 1/9!
    p = fma(p, f, 2.48015873015873e-05);              // 1/8!
    p = fma(p, f, 0.0001984126984126984);             // 1/7!
    p = fma(p, f, 0.001388888888888889);              // 1/6!
    p = fma(p, f, 0.008333333333333333);              // 1/5!
    p = fma(p, f, 0.041666666666666664);              // 1/4!
    p = fma(p, f, 0.16666666666666666);               // 1/3!
    p = fma(p, f, 0.5);
    p = fma(p, f, 1.0);
    p = fma(p, f, 1.0);
    return ldexp(p, (int)n);
}

// ---------------------------------------------------------------------------
// Wave64 reduction of a double (butterfly over xor masks).
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ inline unsigned long long to_fixed(double v, double scale, int* status)
{
    double s = v * scale;
    const double lim = 4.0e18;
    if (!(s < lim && s > -lim)) {   // also catches NaN
        atomicOr(status, (s != s) ? kStNaN : kStOverflow);
        s = 0.0;
    }
    return (unsigned long long)__double2ll_rn(s);
}

__host__ __device__ inline double from_fixed(unsigned long long v, double scale)
{
    return (double)(long long)v / scale;
}

}  // namespace odk
