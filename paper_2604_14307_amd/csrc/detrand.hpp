// detrand.hpp -- device-side deterministic primitives for the MPCD step.
//
// Counter-based random numbers (Philox4x64-10, Salmon et al., SC'11), a
// project-written natural log (atanh series) and sin/cos (Taylor series after a
// two-part pi/2 reduction), and the samplers built on them: the random grid
// shift, Box-Muller normals for the site velocities, and a cell's random
// unit axis (Archimedes) with its Marsaglia-Tsang (2000) gamma variate (on
// Box-Muller normals) drawn from one stream.
// With contraction disabled (-ffp-contract=off) every + - * / sqrt below is
// one correctly rounded IEEE operation in the order written, so a host
// implementation of the same definitions draws bit-identical numbers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpcd {

// purposes of the streams (2, an earlier thermostat stream, is unused)
enum : uint64_t { RNG_SHIFT = 0, RNG_CELL = 1, RNG_SITE = 3 };
constexpr int RNG_MAX_CALLS = 64;

constexpr uint32_t ST_NONFINITE = 1u, ST_ESCAPE = 2u, ST_FIXOVF = 4u, ST_RNGLOOP = 8u, ST_BINERR = 16u,
                   ST_REACH = 32u, ST_CROWD = 64u;

struct Words {
    uint64_t w[4];
};

// The 128-bit product a * b as (hi, lo), from four 32 x 32 -> 64-bit products
// (the 32-bit halves of a and b); exact, so equal to (__umul64hi(a, b), a * b),
// in four multiply-adds instead of the seven or eight of the two separately.
__device__ __forceinline__ void mul128(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo)
{
    const uint64_t aL = (uint32_t)a, aH = a >> 32, bL = (uint32_t)b, bH = b >> 32;
    const uint64_t p0 = aL * bL;
    const uint64_t p1 = aH * bL + (p0 >> 32);        // < 2^64: (2^32 - 1)^2 + 2^32 - 1
    const uint64_t p2 = aL * bH + (uint32_t)p1;
    hi = aH * bH + (p1 >> 32) + (p2 >> 32);
    lo = (p2 << 32) | (uint32_t)p0;
}

// Philox4x64-10: counter (c0..c3), key (k0, k1).
__device__ __forceinline__ Words philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        uint64_t lo0, hi0, lo1, hi1;
        mul128(M0, c0, hi0, lo0);
        mul128(M1, c2, hi1, lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    Words r;
    r.w[0] = c0; r.w[1] = c1; r.w[2] = c2; r.w[3] = c3;
    return r;
}

// Stream of (seed, purpose) at (step, entity, replica), call index `call`.
__device__ __forceinline__ Words rng_draw(uint64_t seed, uint64_t purpose, uint64_t step,
                                          uint64_t entity, uint64_t replica, uint64_t call)
{
    return philox4x64(step, entity, replica, call, seed, purpose);
}


// ln x = e ln2 + 2 atanh(t), x = f 2^e with f in (sqrt(2)/2, sqrt(2)], t = (f-1)/(f+1).
__device__ inline double det_log(double x)
{
    if (x != x) return x;
    if (x < 0.0) return __builtin_nan("");
    if (x == 0.0) return -__builtin_inf();
    if (x == __builtin_inf()) return x;
    int adj = 0;
    if (x < 0x1p-1022) {
        x = x * 0x1p54;
        adj = -54;
    }
    uint64_t bits = (uint64_t)__double_as_longlong(x);
    int e = (int)((bits >> 52) & 0x7ffu) - 1023 + adj;
    bits = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
    double f = __longlong_as_double((long long)bits);
    if (f > 0x1.6a09e667f3bcdp+0) {
        f = 0.5 * f;
        e = e + 1;
    }
    const double t = (f - 1.0) / (f + 1.0);
    const double t2 = t * t;
    double p = 1.0 / 21.0;
    p = p * t2 + 1.0 / 19.0;
    p = p * t2 + 1.0 / 17.0;
    p = p * t2 + 1.0 / 15.0;
    p = p * t2 + 1.0 / 13.0;
    p = p * t2 + 1.0 / 11.0;
    p = p * t2 + 1.0 / 9.0;
    p = p * t2 + 1.0 / 7.0;
    p = p * t2 + 1.0 / 5.0;
    p = p * t2 + 1.0 / 3.0;
    p = p * t2 + 1.0;
    const double de = (double)e;
    const double ln2_hi = 0x1.62e42fee00000p-1, ln2_lo = 0x1.a39ef35793c76p-33;
    return de * ln2_hi + ((2.0 * t) * p + de * ln2_lo);
}

// sin and cos of th.
__device__ inline void det_sincos(double th, double *s_out, double *c_out)
{
    const double pio2_hi = 0x1.921fb54400000p+0, pio2_lo = 0x1.0b4611a626331p-34;
    const double kf = rint(th * 0x1.45f306dc9c883p-1);
    const long long k = (long long)kf;
    const double r = (th - kf * pio2_hi) - kf * pio2_lo;
    const double r2 = r * r;
    double ps = 1.0 / 355687428096000.0;
    ps = ps * r2 - 1.0 / 1307674368000.0;
    ps = ps * r2 + 1.0 / 6227020800.0;
    ps = ps * r2 - 1.0 / 39916800.0;
    ps = ps * r2 + 1.0 / 362880.0;
    ps = ps * r2 - 1.0 / 5040.0;
    ps = ps * r2 + 1.0 / 120.0;
    ps = ps * r2 - 1.0 / 6.0;
    const double sn = r + (r * r2) * ps;
    double pc = 1.0 / 6402373705728000.0;
    pc = pc * r2 - 1.0 / 20922789888000.0;
    pc = pc * r2 + 1.0 / 87178291200.0;
    pc = pc * r2 - 1.0 / 479001600.0;
    pc = pc * r2 + 1.0 / 3628800.0;
    pc = pc * r2 - 1.0 / 40320.0;
    pc = pc * r2 + 1.0 / 720.0;
    pc = pc * r2 - 1.0 / 24.0;
    pc = pc * r2 + 1.0 / 2.0;
    const double cs = 1.0 - r2 * pc;
    switch ((int)(k & 3)) {
    case 0: *s_out = sn; *c_out = cs; break;
    case 1: *s_out = cs; *c_out = -sn; break;
    case 2: *s_out = -sn; *c_out = -cs; break;
    default: *s_out = -cs; *c_out = sn; break;
    }
}

// Grid shift component k in [-a/2, a/2) on a 2^-24 a grid.
__device__ __forceinline__ double shift_component(uint64_t w, double a)
{
    const double q = (double)(int64_t)(w >> 40) - 8388608.0;
    return (q * 0x1p-24) * a;
}

constexpr double TWO_PI = 0x1.921fb54442d18p+2;

// (w >> 12 + 1/2) 2^-52: exact, in (0, 1).
__device__ __forceinline__ double unit52(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1p-52; }

// Three standard normals from one call without rejection: Box-Muller (1958)
// pairs rho (cos, sin)(2 pi u) with rho = sqrt(-2 ln u'), from words
// (w0, w1) and (w2, w3); the sine of the second pair is dropped.
__device__ inline uint32_t site_normals(uint64_t seed, uint64_t step, uint64_t site, uint64_t replica, double z[3])
{
    const Words w = rng_draw(seed, RNG_SITE, step, site, replica, 0);
    double sn, cs;
    const double rho1 = sqrt(-2.0 * det_log(unit52(w.w[0])));
    det_sincos(TWO_PI * unit52(w.w[1]), &sn, &cs);
    z[0] = rho1 * cs;
    z[1] = rho1 * sn;
    const double rho2 = sqrt(-2.0 * det_log(unit52(w.w[2])));
    det_sincos(TWO_PI * unit52(w.w[3]), &sn, &cs);
    z[2] = rho2 * cs;
    return 0;
}

// 32-bit half i (0..7) of a call's words, the high half of each word first.
__device__ __forceinline__ uint32_t half32(const Words &w, int i)
{
    return (i & 1) ? (uint32_t)w.w[i >> 1] : (uint32_t)(w.w[i >> 1] >> 32);
}

// (h + 1/2) 2^-31 - 1: exact, symmetric, in (-1, 1), never 0.
__device__ __forceinline__ double sym32(uint32_t h) { return ((double)h + 0.5) * 0x1p-31 - 1.0; }

// (h + 1/2) 2^-32: exact, in (0, 1).
__device__ __forceinline__ double unit32(uint32_t h) { return ((double)h + 0.5) * 0x1p-32; }

// Uniform random unit vector without rejection (Archimedes: on the unit sphere
// z is uniform in (-1, 1) and the azimuth phi uniform in [0, 2 pi)):
// n = (sqrt(1 - z^2) cos phi, sqrt(1 - z^2) sin phi, z).
__device__ __forceinline__ void axis_from(uint32_t hz, uint32_t hphi, double n[3])
{
    const double z = sym32(hz);
    const double r = sqrt(1.0 - z * z);
    double sn, cs;
    det_sincos(TWO_PI * unit32(hphi), &sn, &cs);
    n[0] = r * cs;
    n[1] = r * sn;
    n[2] = z;
}

// One Marsaglia-Tsang (2000) test for Gamma(k), d = k - 1/3, c = 1/sqrt(9d),
// of the standard normal z with the uniform u.
__device__ __forceinline__ bool mt_try(double z, double u, double d, double c, double *g)
{
    double v = 1.0 + c * z;
    if (v <= 0.0) return false;
    v = (v * v) * v;
    const double z2 = z * z;
    if (u < 1.0 - 0.0331 * (z2 * z2) || det_log(u) < (0.5 * z) * z + d * ((1.0 - v) + det_log(v))) {
        *g = d * v;
        return true;
    }
    return false;
}

// Two Marsaglia-Tsang tests on one call's halves: the Box-Muller (1958) pair
// z1 = rho cos(2 pi u2), z2 = rho sin(2 pi u2), rho = sqrt(-2 ln u1), from
// (h1, h2), tested with the uniforms from h3 and then h4.
__device__ __forceinline__ bool gamma_try2(uint32_t h1, uint32_t h2, uint32_t h3, uint32_t h4, double d, double c,
                                           double *g)
{
    const double rho = sqrt(-2.0 * det_log(unit32(h1)));
    double sn, cs;
    det_sincos(TWO_PI * unit32(h2), &sn, &cs);
    return mt_try(rho * cs, unit32(h3), d, c, g) || mt_try(rho * sn, unit32(h4), d, c, g);
}

// A cell's random axis and (want_gamma) thermostat Gamma variate from its one
// stream.  Call 0's halves 0 and 1 give the axis (no rejection); while the
// variate is pending, each call's halves 2-5 give two Marsaglia-Tsang tests;
// calls go on until the variate is accepted.  The axis does not depend on
// whether the variate is wanted.  Neither draw rejects often, so the lanes of
// a wave rarely need a second call.  State per call, for a caller that
// interleaves calls of several cells: see cell_draw_call.
struct CellDraw {
    double n[3], g, d, c;
    bool have_axis, have_gamma;
};

__device__ __forceinline__ void cell_draw_begin(CellDraw &D, bool want_gamma, double k)
{
    D.have_axis = false;
    D.have_gamma = !want_gamma;
    D.g = 0.0;
    if (want_gamma) {
        D.d = k - 1.0 / 3.0;
        D.c = 1.0 / sqrt(9.0 * D.d);
    }
}

// One call's draws; true when both are done.
__device__ __forceinline__ bool cell_draw_call(CellDraw &D, const Words &w)
{
    if (!D.have_axis) {
        axis_from(half32(w, 0), half32(w, 1), D.n);
        D.have_axis = true;
    }
    if (!D.have_gamma)
        D.have_gamma = gamma_try2(half32(w, 2), half32(w, 3), half32(w, 4), half32(w, 5), D.d, D.c, &D.g);
    return D.have_axis && D.have_gamma;
}

// Fallback after RNG_MAX_CALLS calls without acceptance (flagged).
__device__ __forceinline__ uint32_t cell_draw_end(CellDraw &D)
{
    uint32_t st = 0;
    if (!D.have_axis) {
        D.n[0] = 0.0; D.n[1] = 0.0; D.n[2] = 1.0;
        st |= ST_RNGLOOP;
    }
    if (!D.have_gamma) {
        D.g = D.d;
        st |= ST_RNGLOOP;
    }
    return st;
}

// cell_draw in two parts, for a caller that knows the cell's member count
// only later: cell_draw_pre takes call 0 and forms everything of it that does
// not depend on the count (the axis, the Box-Muller pair and the two test
// uniforms); cell_draw_post runs the Marsaglia-Tsang tests on them and, when
// both reject, continues with calls 1, 2, ... exactly as cell_draw does.  The
// pair gives cell_draw's values bit for bit.
struct CellDrawPre {
    double n[3], z1, z2, u1, u2;
};

__device__ inline void cell_draw_pre(uint64_t seed, uint64_t step, uint64_t cell, uint64_t replica, CellDrawPre &P)
{
    const Words w = rng_draw(seed, RNG_CELL, step, cell, replica, 0);
    axis_from(half32(w, 0), half32(w, 1), P.n);
    const double rho = sqrt(-2.0 * det_log(unit32(half32(w, 2))));
    double sn, cs;
    det_sincos(TWO_PI * unit32(half32(w, 3)), &sn, &cs);
    P.z1 = rho * cs;
    P.z2 = rho * sn;
    P.u1 = unit32(half32(w, 4));
    P.u2 = unit32(half32(w, 5));
}

// cell_draw_post's first part alone: the axis and call 0's two
// Marsaglia-Tsang tests; false when both reject (cell_draw_post then
// continues from the same state).
__device__ inline bool cell_draw_first(const CellDrawPre &P, bool want_gamma, double k, CellDraw &D)
{
    cell_draw_begin(D, want_gamma, k);
    D.n[0] = P.n[0];
    D.n[1] = P.n[1];
    D.n[2] = P.n[2];
    D.have_axis = true;
    if (!D.have_gamma) D.have_gamma = mt_try(P.z1, P.u1, D.d, D.c, &D.g) || mt_try(P.z2, P.u2, D.d, D.c, &D.g);
    return D.have_gamma;
}

__device__ inline uint32_t cell_draw_post(uint64_t seed, uint64_t step, uint64_t cell, uint64_t replica,
                                          const CellDrawPre &P, bool want_gamma, double k, CellDraw &D)
{
    if (cell_draw_first(P, want_gamma, k, D)) return 0u;
    for (int call = 1; !D.have_gamma && call < RNG_MAX_CALLS; ++call)
        cell_draw_call(D, rng_draw(seed, RNG_CELL, step, cell, replica, (uint64_t)call));
    return D.have_gamma ? 0u : cell_draw_end(D);
}

__device__ inline uint32_t cell_draw(uint64_t seed, uint64_t step, uint64_t cell, uint64_t replica, bool want_gamma,
                                     double k, CellDraw &D)
{
    cell_draw_begin(D, want_gamma, k);
    for (int call = 0; call < RNG_MAX_CALLS; ++call)
        if (cell_draw_call(D, rng_draw(seed, RNG_CELL, step, cell, replica, (uint64_t)call))) return 0;
    return cell_draw_end(D);
}

}  // namespace mpcd
