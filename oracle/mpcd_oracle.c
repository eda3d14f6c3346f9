/*
 * mpcd_oracle.c -- plain, slow CPU FP64 oracle for one step of multiparticle
 * collision dynamics (MPCD, stochastic rotation dynamics collision rule) with
 * colloids represented as rigid bodies of discrete surface sites.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
 * GPU library is compared against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no source with the
 * GPU library: every primitive below (Philox, log, sin/cos, samplers) is
 * written here a second time from its published definition.
 *
 * Paper: Bush, Palmer, Howard, "Simulating hydrodynamic interactions in
 * colloidal suspensions using multiparticle collision dynamics with rigid-body
 * constraints" (arXiv 2604.14307).
 *   - Solvent: Sec. II.A (streaming, cell sorting, SRD rotation about a random
 *     axis by a fixed angle, random grid shift, cell thermostat).
 *   - Rigid body kinematics: Sec. II.B.2, Eqs. (3)-(5).
 *   - Site thermalization before the collision: Sec. II.B.2, Eq. (7).
 *   - Momentum transfer to the body and reset to rigid motion: Sec. II.B.2,
 *     the paragraphs around Eq. (5) and after Eq. (7).
 *   - Colloid repulsion: core-shifted WCA, Eq. (1).
 *   - Rigid-body integrator: quaternion velocity Verlet of Miller et al.
 *     (NO_SQUISH splitting), cited in Sec. II.B.2.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no -march, no fast-math),
 * so that every + - * / sqrt is one IEEE-754 correctly rounded operation in the
 * order written.  Parentheses below fix the evaluation order exactly.
 *
 * Every random number is drawn from Philox4x64-10 keyed by (seed, purpose)
 * with counter (step, entity, replica, call), so the GPU path can draw the
 * identical numbers.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Status bits (also returned by the GPU library, same meaning).              */
#define ORC_NONFINITE 1u
#define ORC_ESCAPE 2u
#define ORC_FIXOVF 4u
#define ORC_RNGLOOP 8u

/* Philox purposes (second key word). */
#define PURPOSE_SHIFT 0u
#define PURPOSE_CELL 1u /* a cell's collision axis and thermostat variate */
#define PURPOSE_SITE 3u

#define MAX_RNG_CALLS 64

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two      */
/* 64x64->128 multiplies, key bumped by the Weyl constants between rounds.   */
void orc_philox(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        unsigned __int128 prod0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * c0;
        unsigned __int128 prod1 = (unsigned __int128)0xCA5A826395121157ULL * c2;
        uint64_t hi0 = (uint64_t)(prod0 >> 64), lo0 = (uint64_t)prod0;
        uint64_t hi1 = (uint64_t)(prod1 >> 64), lo1 = (uint64_t)prod1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint64_t purpose, uint64_t step, uint64_t entity,
                 uint64_t replica, uint64_t call, uint64_t w[4])
{
    uint64_t ctr[4] = {step, entity, replica, call};
    uint64_t key[2] = {seed, purpose};
    orc_philox(ctr, key, w);
}

/* ------------------------------------------------------------------------- */
/* Natural logarithm from the atanh series:                                   */
/*   x = f 2^e, f in (sqrt2/2, sqrt2],  ln x = e ln2 + 2 atanh((f-1)/(f+1)).  */
/* ln2 is split (Cody and Waite) so that e*LN2_HI is exact.                   */
static const double LN2_HI = 0x1.62e42fee00000p-1;
static const double LN2_LO = 0x1.a39ef35793c76p-33;
static const double SQRT2_D = 0x1.6a09e667f3bcdp+0;

double orc_dlog(double x)
{
    if (x != x) return x;
    if (x < 0.0) return NAN;
    if (x == 0.0) return -INFINITY;
    if (x == INFINITY) return x;
    int adj = 0;
    if (x < 0x1p-1022) { /* subnormal: scale into the normal range */
        x = x * 0x1p54;
        adj = -54;
    }
    uint64_t bits;
    memcpy(&bits, &x, sizeof bits);
    int e = (int)((bits >> 52) & 0x7ffu) - 1023 + adj;
    bits = (bits & 0x000FFFFFFFFFFFFFULL) | 0x3FF0000000000000ULL;
    double f;
    memcpy(&f, &bits, sizeof f);
    if (f > SQRT2_D) {
        f = 0.5 * f;
        e = e + 1;
    }
    double t = (f - 1.0) / (f + 1.0);
    double t2 = t * t;
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
    double de = (double)e;
    return de * LN2_HI + ((2.0 * t) * p + de * LN2_LO);
}

/* ------------------------------------------------------------------------- */
/* sin and cos: reduce by the nearest multiple of pi/2 (two-part pi/2), then  */
/* Taylor series in r^2 (through r^17 for sin, r^18 for cos), then quadrant.  */
static const double PIO2_HI = 0x1.921fb54400000p+0;
static const double PIO2_LO = 0x1.0b4611a626331p-34;
static const double TWO_OVER_PI = 0x1.45f306dc9c883p-1;

void orc_dsincos(double th, double *s_out, double *c_out)
{
    double kf = rint(th * TWO_OVER_PI);
    long long k = (long long)kf;
    double r = (th - kf * PIO2_HI) - kf * PIO2_LO;
    double r2 = r * r;
    double ps = 1.0 / 355687428096000.0;          /* 1/17! */
    ps = ps * r2 - 1.0 / 1307674368000.0;         /* 1/15! */
    ps = ps * r2 + 1.0 / 6227020800.0;            /* 1/13! */
    ps = ps * r2 - 1.0 / 39916800.0;              /* 1/11! */
    ps = ps * r2 + 1.0 / 362880.0;                /* 1/9!  */
    ps = ps * r2 - 1.0 / 5040.0;                  /* 1/7!  */
    ps = ps * r2 + 1.0 / 120.0;                   /* 1/5!  */
    ps = ps * r2 - 1.0 / 6.0;                     /* 1/3!  */
    double sn = r + (r * r2) * ps;
    double pc = 1.0 / 6402373705728000.0;         /* 1/18! */
    pc = pc * r2 - 1.0 / 20922789888000.0;        /* 1/16! */
    pc = pc * r2 + 1.0 / 87178291200.0;           /* 1/14! */
    pc = pc * r2 - 1.0 / 479001600.0;             /* 1/12! */
    pc = pc * r2 + 1.0 / 3628800.0;               /* 1/10! */
    pc = pc * r2 - 1.0 / 40320.0;                 /* 1/8!  */
    pc = pc * r2 + 1.0 / 720.0;                   /* 1/6!  */
    pc = pc * r2 - 1.0 / 24.0;                    /* 1/4!  */
    pc = pc * r2 + 1.0 / 2.0;                     /* 1/2!, sign applied below */
    double cs = 1.0 - r2 * pc;
    switch ((int)(k & 3)) {
    case 0: *s_out = sn; *c_out = cs; break;
    case 1: *s_out = cs; *c_out = -sn; break;
    case 2: *s_out = -sn; *c_out = -cs; break;
    default: *s_out = -cs; *c_out = sn; break;
    }
}

/* ------------------------------------------------------------------------- */
/* Samplers.                                                                  */

/* Random grid shift, uniform in [-a/2, a/2) per axis, on a 2^-24 a grid so   */
/* that it is exact in single and double precision (Sec. II.A).               */
void orc_shift(uint64_t seed, uint64_t step, uint64_t replica, double a, double s[3])
{
    uint64_t w[4];
    draw(seed, PURPOSE_SHIFT, step, 0, replica, 0, w);
    for (int k = 0; k < 3; ++k) {
        double q = (double)(int64_t)(w[k] >> 40) - 8388608.0;
        s[k] = (q * 0x1p-24) * a;
    }
}

#define TWO_PI 0x1.921fb54442d18p+2

/* (w >> 12 + 1/2) 2^-52: a uniform in (0, 1), exact in double.                */
static double u52(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1p-52; }

/* Three standard normals for a site by Box-Muller (1958): the pairs           */
/* rho (cos 2 pi u1, sin 2 pi u1), rho = sqrt(-2 ln u0), from words (w0, w1)   */
/* and (w2, w3) of call 0; the sine of the second pair is dropped.  Never      */
/* rejects.                                                                    */
uint32_t orc_site_normals(uint64_t seed, uint64_t step, uint64_t site, uint64_t replica,
                          double z[3])
{
    uint64_t w[4];
    draw(seed, PURPOSE_SITE, step, site, replica, 0, w);
    double sn, cs;
    double rho1 = sqrt(-2.0 * orc_dlog(u52(w[0])));
    orc_dsincos(TWO_PI * u52(w[1]), &sn, &cs);
    z[0] = rho1 * cs;
    z[1] = rho1 * sn;
    double rho2 = sqrt(-2.0 * orc_dlog(u52(w[2])));
    orc_dsincos(TWO_PI * u52(w[3]), &sn, &cs);
    z[2] = rho2 * cs;
    return 0;
}

/* The 32-bit halves of a call's four words, high half of each word first.   */
static void halves(const uint64_t w[4], uint32_t h[8])
{
    for (int i = 0; i < 4; ++i) {
        h[2 * i] = (uint32_t)(w[i] >> 32);
        h[2 * i + 1] = (uint32_t)(w[i] & 0xffffffffu);
    }
}

/* A half as a uniform in (-1, 1) and in (0, 1): (h + 1/2) 2^-31 - 1 and      */
/* (h + 1/2) 2^-32, both exact in double.                                     */
static double sym_u32(uint32_t h) { return ((double)h + 0.5) * 0x1p-31 - 1.0; }
static double unit_u32(uint32_t h) { return ((double)h + 0.5) * 0x1p-32; }

/* Uniform random unit vector without rejection (Archimedes' theorem: on the   */
/* unit sphere z is uniform in (-1, 1) and the azimuth uniform in [0, 2 pi)).  */
static void axis_from_halves(uint32_t hz, uint32_t hphi, double n[3])
{
    double z = sym_u32(hz);
    double r = sqrt(1.0 - z * z);
    double sn, cs;
    orc_dsincos(TWO_PI * unit_u32(hphi), &sn, &cs);
    n[0] = r * cs;
    n[1] = r * sn;
    n[2] = z;
}

/* The Marsaglia-Tsang (2000) test for Gamma(shape k >= 1, scale 1) of the    */
/* standard normal z with the uniform u; d = k - 1/3, c = 1/sqrt(9 d).         */
static int mt_accept(double z, double u, double d, double c, double *g)
{
    double v = 1.0 + c * z;
    if (v <= 0.0) return 0;
    v = (v * v) * v;
    double z2 = z * z;
    if (u < 1.0 - 0.0331 * (z2 * z2)) {
        *g = d * v;
        return 1;
    }
    if (orc_dlog(u) < (0.5 * z) * z + d * ((1.0 - v) + orc_dlog(v))) {
        *g = d * v;
        return 1;
    }
    return 0;
}

/* A cell's random collision axis and, when want_gamma, its thermostat        */
/* Gamma(k) variate, both from the cell's one stream (purpose PURPOSE_CELL).  */
/* Call 0's halves 0 and 1 give the axis.  While the variate is pending, call  */
/* i's halves 2 and 3 give the Box-Muller (1958) pair                          */
/* z1 = rho cos(2 pi u3), z2 = rho sin(2 pi u3), rho = sqrt(-2 ln u2), tested  */
/* by Marsaglia-Tsang with the uniform of half 4 and then z2 with half 5;      */
/* calls 0, 1, ... continue until one test accepts.  The axis is the same      */
/* whether or not the variate is wanted.                                       */
uint32_t orc_cell_draws(uint64_t seed, uint64_t step, uint64_t cell, uint64_t replica, int want_gamma, double k,
                        double n[3], double *g)
{
    int have_axis = 0, have_gamma = !want_gamma;
    double d = 0.0, c = 0.0;
    if (want_gamma) {
        d = k - 1.0 / 3.0;
        c = 1.0 / sqrt(9.0 * d);
    }
    *g = 0.0;
    for (uint64_t call = 0; call < MAX_RNG_CALLS && !(have_axis && have_gamma); ++call) {
        uint64_t w[4];
        uint32_t h[8];
        draw(seed, PURPOSE_CELL, step, cell, replica, call, w);
        halves(w, h);
        if (!have_axis) {
            axis_from_halves(h[0], h[1], n);
            have_axis = 1;
        }
        if (!have_gamma) {
            double rho = sqrt(-2.0 * orc_dlog(unit_u32(h[2])));
            double sn, cs;
            orc_dsincos(TWO_PI * unit_u32(h[3]), &sn, &cs);
            have_gamma = mt_accept(rho * cs, unit_u32(h[4]), d, c, g) || mt_accept(rho * sn, unit_u32(h[5]), d, c, g);
        }
    }
    uint32_t flags = 0;
    if (!have_gamma) {
        *g = d;
        flags |= ORC_RNGLOOP;
    }
    return flags;
}

/* The axis alone, and the variate alone, of a cell's draws.                  */
uint32_t orc_cell_axis(uint64_t seed, uint64_t step, uint64_t cell, uint64_t replica, double n[3])
{
    double g;
    return orc_cell_draws(seed, step, cell, replica, 0, 0.0, n, &g);
}

uint32_t orc_gamma(uint64_t seed, uint64_t step, uint64_t cell, uint64_t replica, double k, double *g)
{
    double n[3];
    return orc_cell_draws(seed, step, cell, replica, 1, k, n, g);
}

/* ------------------------------------------------------------------------- */
/* Small vector helpers with a fixed evaluation order.                        */

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Body-to-space rotation matrix of the quaternion q = (w, x, y, z). */
static void quat_to_mat(const double q[4], double A[3][3])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    A[0][0] = (w * w + x * x) - (y * y + z * z);
    A[0][1] = 2.0 * (x * y - w * z);
    A[0][2] = 2.0 * (x * z + w * y);
    A[1][0] = 2.0 * (x * y + w * z);
    A[1][1] = (w * w - x * x) + (y * y - z * z);
    A[1][2] = 2.0 * (y * z - w * x);
    A[2][0] = 2.0 * (x * z - w * y);
    A[2][1] = 2.0 * (y * z + w * x);
    A[2][2] = (w * w - x * x) - (y * y - z * z);
}

static void mat_vec(const double A[3][3], const double v[3], double out[3])
{
    for (int i = 0; i < 3; ++i) out[i] = (A[i][0] * v[0] + A[i][1] * v[1]) + A[i][2] * v[2];
}

static void mat_t_vec(const double A[3][3], const double v[3], double out[3])
{
    for (int i = 0; i < 3; ++i) out[i] = (A[0][i] * v[0] + A[1][i] * v[1]) + A[2][i] * v[2];
}

/* q (x) (0, a): the quaternion product with a pure quaternion, i.e. the      */
/* matrix S(q) of Miller et al. applied to (0, a).                            */
static void quat_times_pure(const double q[4], const double a[3], double out[4])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    out[0] = ((-x) * a[0] + (-y) * a[1]) + (-z) * a[2];
    out[1] = (w * a[0] + (-z) * a[1]) + y * a[2];
    out[2] = (z * a[0] + w * a[1]) + (-x) * a[2];
    out[3] = ((-y) * a[0] + x * a[1]) + w * a[2];
}

/* Body-frame angular momentum from the conjugate quaternion momentum:        */
/* Lhat_k = (1/2) p . P_k q with the permutations P_k of Miller et al.        */
static void perm_k(int k, const double q[4], double out[4])
{
    if (k == 1) { out[0] = -q[1]; out[1] = q[0]; out[2] = q[3]; out[3] = -q[2]; }
    else if (k == 2) { out[0] = -q[2]; out[1] = -q[3]; out[2] = q[0]; out[3] = q[1]; }
    else { out[0] = -q[3]; out[1] = q[2]; out[2] = -q[1]; out[3] = q[0]; }
}

static double dot4(const double a[4], const double b[4])
{
    return ((a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]) + a[3] * b[3];
}

static void body_frame_angmom(const double q[4], const double p[4], double Lh[3])
{
    for (int k = 1; k <= 3; ++k) {
        double Pq[4];
        perm_k(k, q, Pq);
        Lh[k - 1] = 0.5 * dot4(p, Pq);
    }
}

/* Periodic wrap into [0, L) by at most one period. */
static double wrap1(double y, double L, uint32_t *flags)
{
    if (y >= L) y = y - L;
    else if (y < 0.0) y = y + L;
    if (!(y >= 0.0 && y <= L)) *flags |= (y != y) ? ORC_NONFINITE : ORC_ESCAPE;
    return y;
}

/* ------------------------------------------------------------------------- */
/* System description (host arrays, component-major [3][n] layout).           */
typedef struct {
    int32_t n[3];
    double a;
    int64_t N;        /* solvent particles */
    double m;         /* solvent mass */
    double *x, *v;    /* [3N] */
    int64_t B;        /* rigid bodies */
    double *R;        /* [3B] centre of mass, wrapped into the box */
    int32_t *img;     /* [3B] periodic image counters */
    double *q;        /* [4B] orientation quaternion (w,x,y,z) */
    double *P;        /* [3B] linear momentum */
    double *p;        /* [4B] conjugate quaternion momentum */
    double *F;        /* [3B] force from the last evaluation */
    double *T;        /* [3B] torque (space frame) from the last evaluation */
    const double *M;  /* [B] body mass */
    const double *I;  /* [3B] principal moments of inertia */
    int64_t S;        /* surface sites */
    const int64_t *site_off; /* [B+1] sites of body b: site_off[b] .. site_off[b+1]-1 */
    const double *dhat;      /* [3S] body-frame site positions relative to R */
    const double *sm;        /* [S] site masses */
    double *xs, *vs, *vpre, *d; /* [3S] site positions, velocities, pre-collision velocities, space-frame offsets */
} orc_sys;

typedef struct {
    double dt;
    double cos_a, sin_a; /* SRD rotation angle */
    double kT;           /* site thermalization temperature */
    double kT_cell;      /* cell thermostat temperature; <= 0 turns it off */
    uint64_t seed;
    uint64_t replica;
    int32_t thermalize;  /* 1: Eq. (7); 0: naive scheme (rigid velocities only) */
    int32_t wca_mode;    /* 0 off, 1 between body centres, 2 between sites of different bodies */
    double eps, sigma, delta;
    double g[3];         /* constant acceleration of every solvent particle      */
    double f_ext[3];     /* constant force on every body, at its centre          */
} orc_par;

static int forced(const double a[3]) { return a[0] != 0.0 || a[1] != 0.0 || a[2] != 0.0; }

static double box_len(const orc_sys *s, int k) { return (double)s->n[k] * s->a; }

/* ------------------------------------------------------------------------- */
/* (a1) Site positions and thermalized velocities, Eqs. (5) and (7).          */
/* vt_in (optional, [3S]) replaces the Maxwell-Boltzmann draws.               */
uint32_t orc_sites_thermalize(orc_sys *s, const orc_par *par, uint64_t step, const double *vt_in)
{
    uint32_t flags = 0;
    int64_t S = s->S;
    for (int64_t b = 0; b < s->B; ++b) {
        double q[4], p[4], A[3][3];
        for (int r = 0; r < 4; ++r) { q[r] = s->q[r * s->B + b]; p[r] = s->p[r * s->B + b]; }
        quat_to_mat(q, A);
        double Mb = s->M[b];
        double V[3], Lh[3], wh[3], w[3];
        for (int k = 0; k < 3; ++k) V[k] = s->P[k * s->B + b] / Mb;
        body_frame_angmom(q, p, Lh);
        for (int k = 0; k < 3; ++k) {
            double Ik = s->I[k * s->B + b];
            wh[k] = (Ik == 0.0) ? 0.0 : Lh[k] / Ik;
        }
        mat_vec(A, wh, w);

        int64_t j0 = s->site_off[b], j1 = s->site_off[b + 1];
        /* site offsets, positions and random velocities */
        double Vt[3] = {0.0, 0.0, 0.0}, Lt[3] = {0.0, 0.0, 0.0};
        for (int64_t j = j0; j < j1; ++j) {
            double dh[3] = {s->dhat[j], s->dhat[S + j], s->dhat[2 * S + j]}, d[3];
            mat_vec(A, dh, d);
            for (int k = 0; k < 3; ++k) {
                s->d[k * S + j] = d[k];
                s->xs[k * S + j] = wrap1(s->R[k * s->B + b] + d[k], box_len(s, k), &flags);
            }
            double vt[3] = {0.0, 0.0, 0.0};
            if (par->thermalize) {
                if (vt_in) {
                    for (int k = 0; k < 3; ++k) vt[k] = vt_in[k * S + j];
                } else {
                    double z[3];
                    flags |= orc_site_normals(par->seed, step, (uint64_t)j, par->replica, z);
                    double sig = sqrt(par->kT / s->sm[j]);
                    for (int k = 0; k < 3; ++k) vt[k] = sig * z[k];
                }
            }
            /* keep the draw in vs for the second pass */
            for (int k = 0; k < 3; ++k) s->vs[k * S + j] = vt[k];
            double pv[3], c[3];
            for (int k = 0; k < 3; ++k) pv[k] = s->sm[j] * vt[k];
            for (int k = 0; k < 3; ++k) Vt[k] = Vt[k] + pv[k];
            cross3(d, pv, c);
            for (int k = 0; k < 3; ++k) Lt[k] = Lt[k] + c[k];
        }
        double Lth[3], wth[3], wt[3], dV[3], dw[3];
        for (int k = 0; k < 3; ++k) Vt[k] = Vt[k] / Mb;
        mat_t_vec(A, Lt, Lth);
        for (int k = 0; k < 3; ++k) {
            double Ik = s->I[k * s->B + b];
            wth[k] = (Ik == 0.0) ? 0.0 : Lth[k] / Ik;
        }
        mat_vec(A, wth, wt);
        for (int k = 0; k < 3; ++k) { dV[k] = V[k] - Vt[k]; dw[k] = w[k] - wt[k]; }
        for (int64_t j = j0; j < j1; ++j) {
            double d[3] = {s->d[j], s->d[S + j], s->d[2 * S + j]}, c[3];
            cross3(dw, d, c);
            for (int k = 0; k < 3; ++k) {
                double vt = s->vs[k * S + j];
                double vj = (dV[k] + c[k]) + vt;
                s->vs[k * S + j] = vj;
                s->vpre[k * S + j] = vj;
                if (!isfinite(vj)) flags |= ORC_NONFINITE;
            }
        }
    }
    return flags;
}

/* ------------------------------------------------------------------------- */
/* (a2) Cell of every particle (solvent 0..N-1, then sites N..N+S-1) for the  */
/* shifted grid, and per-cell member lists in ascending particle index.       */
static int64_t cell_of(const orc_sys *s, const double s3[3], double x0, double x1, double x2)
{
    double xx[3] = {x0, x1, x2};
    int64_t j[3];
    for (int k = 0; k < 3; ++k) {
        double g = xx[k] - s3[k];
        int64_t jk = (int64_t)floor(g / s->a);
        if (jk < 0) jk += s->n[k];
        else if (jk >= s->n[k]) jk -= s->n[k];
        j[k] = jk;
    }
    return (j[2] * s->n[1] + j[1]) * s->n[0] + j[0];
}

uint32_t orc_bin(const orc_sys *s, const double shift[3], int32_t *cell, int64_t *cell_start,
                 int64_t *members)
{
    uint32_t flags = 0;
    int64_t C = (int64_t)s->n[0] * s->n[1] * s->n[2];
    int64_t NT = s->N + s->S;
    for (int64_t c = 0; c <= C; ++c) cell_start[c] = 0;
    for (int64_t k = 0; k < NT; ++k) {
        int64_t c;
        if (k < s->N) c = cell_of(s, shift, s->x[k], s->x[s->N + k], s->x[2 * s->N + k]);
        else {
            int64_t j = k - s->N;
            c = cell_of(s, shift, s->xs[j], s->xs[s->S + j], s->xs[2 * s->S + j]);
        }
        if (c < 0 || c >= C) { flags |= ORC_ESCAPE; c = 0; }
        cell[k] = (int32_t)c;
        cell_start[c + 1] += 1;
    }
    for (int64_t c = 0; c < C; ++c) cell_start[c + 1] += cell_start[c];
    int64_t *fill = (int64_t *)calloc((size_t)(C > 0 ? C : 1), sizeof(int64_t));
    for (int64_t k = 0; k < NT; ++k) {
        int64_t c = cell[k];
        members[cell_start[c] + fill[c]] = k;
        fill[c] += 1;
    }
    free(fill);
    return flags;
}

/* ------------------------------------------------------------------------- */
/* (a3) SRD collision with optional cell thermostat (Sec. II.A).  Sums run    */
/* over each cell's members in ascending particle index.  axis_in (optional,  */
/* [3C]) replaces the random axes.                                            */
static double *pvel(orc_sys *s, int64_t k, int comp)
{
    if (k < s->N) return &s->v[comp * s->N + k];
    return &s->vs[comp * s->S + (k - s->N)];
}

static double pmass(const orc_sys *s, int64_t k) { return (k < s->N) ? s->m : s->sm[k - s->N]; }

uint32_t orc_collide(orc_sys *s, const orc_par *par, uint64_t step, const int64_t *cell_start,
                     const int64_t *members, const double *axis_in)
{
    uint32_t flags = 0;
    int64_t C = (int64_t)s->n[0] * s->n[1] * s->n[2];
    double ca = par->cos_a, sa = par->sin_a;
    for (int64_t c = 0; c < C; ++c) {
        int64_t b = cell_start[c], e = cell_start[c + 1], nc = e - b;
        if (nc < 2) continue;
        double Mc = 0.0, Pc[3] = {0.0, 0.0, 0.0};
        for (int64_t i = b; i < e; ++i) {
            int64_t k = members[i];
            double mk = pmass(s, k);
            Mc = Mc + mk;
            for (int d = 0; d < 3; ++d) Pc[d] = Pc[d] + mk * (*pvel(s, k, d));
        }
        double u[3];
        for (int d = 0; d < 3; ++d) u[d] = Pc[d] / Mc;

        /* the cell's axis and, with the thermostat, its Gamma(3(nc-1)/2)      */
        /* variate, from the cell's one stream                                 */
        double n[3], g = 0.0;
        double shape = 0.5 * (double)(3 * (nc - 1));
        if (axis_in) {
            n[0] = axis_in[c]; n[1] = axis_in[C + c]; n[2] = axis_in[2 * C + c];
            if (par->kT_cell > 0.0) flags |= orc_gamma(par->seed, step, (uint64_t)c, par->replica, shape, &g);
        } else {
            flags |= orc_cell_draws(par->seed, step, (uint64_t)c, par->replica, par->kT_cell > 0.0, shape, n, &g);
        }

        /* R = cos(a) I + sin(a) [n]x + (1 - cos(a)) n n^T (right-hand rule) */
        double omc = 1.0 - ca, R[3][3];
        R[0][0] = (omc * n[0]) * n[0] + ca;
        R[0][1] = (omc * n[0]) * n[1] - sa * n[2];
        R[0][2] = (omc * n[0]) * n[2] + sa * n[1];
        R[1][0] = (omc * n[1]) * n[0] + sa * n[2];
        R[1][1] = (omc * n[1]) * n[1] + ca;
        R[1][2] = (omc * n[1]) * n[2] - sa * n[0];
        R[2][0] = (omc * n[2]) * n[0] - sa * n[1];
        R[2][1] = (omc * n[2]) * n[1] + sa * n[0];
        R[2][2] = (omc * n[2]) * n[2] + ca;

        double lam = 1.0;
        if (par->kT_cell > 0.0) {
            double Es = 0.0;
            for (int64_t i = b; i < e; ++i) {
                int64_t k = members[i];
                double d0 = *pvel(s, k, 0) - u[0];
                double d1 = *pvel(s, k, 1) - u[1];
                double d2 = *pvel(s, k, 2) - u[2];
                Es = Es + pmass(s, k) * ((d0 * d0 + d1 * d1) + d2 * d2);
            }
            double E = 0.5 * Es;
            if (E > 0.0) {
                double Enew = par->kT_cell * g;
                lam = sqrt(Enew / E);
            }
        }
        for (int64_t i = b; i < e; ++i) {
            int64_t k = members[i];
            double dl[3], r[3];
            for (int d = 0; d < 3; ++d) dl[d] = *pvel(s, k, d) - u[d];
            for (int d = 0; d < 3; ++d) r[d] = (R[d][0] * dl[0] + R[d][1] * dl[1]) + R[d][2] * dl[2];
            for (int d = 0; d < 3; ++d) {
                double vn = u[d] + lam * r[d];
                if (!isfinite(vn)) flags |= ORC_NONFINITE;
                *pvel(s, k, d) = vn;
            }
        }
    }
    return flags;
}

/* ------------------------------------------------------------------------- */
/* (a4) Net momentum change of each body's sites over the collision:          */
/* J = sum m (v - v_pre), K = sum d x m (v - v_pre), in site order.           */
uint32_t orc_sites_to_body(const orc_sys *s, double *J, double *K)
{
    int64_t S = s->S;
    for (int64_t b = 0; b < s->B; ++b) {
        double Jb[3] = {0.0, 0.0, 0.0}, Kb[3] = {0.0, 0.0, 0.0};
        for (int64_t j = s->site_off[b]; j < s->site_off[b + 1]; ++j) {
            double mdv[3], d[3], c[3];
            for (int k = 0; k < 3; ++k) {
                double dv = s->vs[k * S + j] - s->vpre[k * S + j];
                mdv[k] = s->sm[j] * dv;
                d[k] = s->d[k * S + j];
            }
            for (int k = 0; k < 3; ++k) Jb[k] = Jb[k] + mdv[k];
            cross3(d, mdv, c);
            for (int k = 0; k < 3; ++k) Kb[k] = Kb[k] + c[k];
        }
        for (int k = 0; k < 3; ++k) { J[k * s->B + b] = Jb[k]; K[k * s->B + b] = Kb[k]; }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Colloid forces: core-shifted WCA between body centres, Eq. (1), minimum    */
/* image, summed over partners in ascending index.  Central forces exert no   */
/* torque.                                                                    */
/* Core-shifted WCA of Eq. (1) at separation dr (|dr|^2 = r2 within the
 * cutoff): adds the force on the first particle, -u'(r) dr / r, to f.
 * Returns ORC_NONFINITE (and adds nothing) when r <= delta. */
static uint32_t wca_pair(const orc_par *par, const double dr[3], double r2, double f[3])
{
    double r = sqrt(r2);
    double sh = r - par->delta;
    if (!(sh > 0.0)) return ORC_NONFINITE;
    double is = par->sigma / sh;
    double is2 = is * is;
    double is6 = (is2 * is2) * is2;
    double is12 = is6 * is6;
    double fr = ((24.0 * par->eps) * (2.0 * is12 - is6)) / sh;
    double fo = fr / r;
    for (int k = 0; k < 3; ++k) f[k] = f[k] + fo * dr[k];
    return 0;
}

/* Space-frame site offsets d_j = A(q_b) dhat_j and unwrapped site positions
 * R_b + d_j of every site (arrays [3S]). */
static void site_frames(const orc_sys *s, double *off, double *pos)
{
    int64_t B = s->B, S = s->S;
    for (int64_t b = 0; b < B; ++b) {
        double q[4], A[3][3];
        for (int r = 0; r < 4; ++r) q[r] = s->q[r * B + b];
        quat_to_mat(q, A);
        for (int64_t j = s->site_off[b]; j < s->site_off[b + 1]; ++j) {
            double dh[3] = {s->dhat[j], s->dhat[S + j], s->dhat[2 * S + j]}, d[3];
            mat_vec(A, dh, d);
            for (int k = 0; k < 3; ++k) {
                off[k * S + j] = d[k];
                pos[k * S + j] = s->R[k * B + b] + d[k];
            }
        }
    }
}

/* Minimum image of a site-site separation: t - L rint(t / L). */
static double min_image(double t, double L) { return t - L * rint(t / L); }

/* Site-site WCA force and torque of body i (mode 2): for each of its sites j
 * in order, f_j sums the pair forces of the sites of every other body (bodies
 * in ascending index, their sites in ascending index); then F = sum_j f_j,
 * T = sum_j d_j x f_j. */
static uint32_t site_wca_body(const orc_sys *s, const orc_par *par, const double *off, const double *pos,
                              int64_t i, double rc2, double F[3], double T[3])
{
    uint32_t flags = 0;
    int64_t B = s->B, S = s->S;
    for (int k = 0; k < 3; ++k) { F[k] = 0.0; T[k] = 0.0; }
    for (int64_t j = s->site_off[i]; j < s->site_off[i + 1]; ++j) {
        double f[3] = {0.0, 0.0, 0.0};
        for (int64_t b = 0; b < B; ++b) {
            if (b == i) continue;
            for (int64_t k2 = s->site_off[b]; k2 < s->site_off[b + 1]; ++k2) {
                double dr[3];
                for (int k = 0; k < 3; ++k) dr[k] = min_image(pos[k * S + j] - pos[k * S + k2], box_len(s, k));
                double r2 = (dr[0] * dr[0] + dr[1] * dr[1]) + dr[2] * dr[2];
                if (!(r2 <= rc2)) continue;
                flags |= wca_pair(par, dr, r2, f);
            }
        }
        double d[3] = {off[j], off[S + j], off[2 * S + j]}, c[3];
        cross3(d, f, c);
        for (int k = 0; k < 3; ++k) {
            F[k] = F[k] + f[k];
            T[k] = T[k] + c[k];
        }
    }
    return flags;
}

/* Colloid forces and torques.  Mode 1: WCA between body centres (Sec. II.B),
 * partners in ascending index.  Mode 2: WCA between sites of different
 * bodies; the force on site j is summed over the other bodies in ascending
 * index and their sites in ascending index, then F = sum_j f_j and
 * T = sum_j d_j x f_j in site order. */
static uint32_t wca_forces(orc_sys *s, const orc_par *par);

uint32_t orc_body_forces(orc_sys *s, const orc_par *par)
{
    uint32_t flags = 0;
    int64_t B = s->B;
    for (int64_t i = 0; i < B; ++i)
        for (int k = 0; k < 3; ++k) { s->F[k * B + i] = 0.0; s->T[k * B + i] = 0.0; }
    if (par->wca_mode == 1 || par->wca_mode == 2) flags = wca_forces(s, par);
    /* a constant external force at the body centre (no torque), Sec. III.B */
    if (forced(par->f_ext))
        for (int64_t i = 0; i < B; ++i)
            for (int k = 0; k < 3; ++k) s->F[k * B + i] = s->F[k * B + i] + par->f_ext[k];
    return flags;
}

static uint32_t wca_forces(orc_sys *s, const orc_par *par)
{
    uint32_t flags = 0;
    int64_t B = s->B, S = s->S;
    double rc = par->delta + 0x1.1f59ac3c7d6c0p+0 * par->sigma;
    double rc2 = rc * rc;
    if (par->wca_mode == 1) {
        for (int64_t i = 0; i < B; ++i) {
            double f[3] = {0.0, 0.0, 0.0};
            for (int64_t j = 0; j < B; ++j) {
                if (j == i) continue;
                double dr[3];
                for (int k = 0; k < 3; ++k) {
                    double L = box_len(s, k);
                    double t = s->R[k * B + i] - s->R[k * B + j];
                    if (t > 0.5 * L) t = t - L;
                    else if (t < -0.5 * L) t = t + L;
                    dr[k] = t;
                }
                double r2 = (dr[0] * dr[0] + dr[1] * dr[1]) + dr[2] * dr[2];
                if (!(r2 <= rc2)) continue;
                flags |= wca_pair(par, dr, r2, f);
            }
            for (int k = 0; k < 3; ++k) s->F[k * B + i] = f[k];
        }
        return flags;
    }
    double *off = (double *)malloc(sizeof(double) * 3 * (size_t)(S > 0 ? S : 1));
    double *pos = (double *)malloc(sizeof(double) * 3 * (size_t)(S > 0 ? S : 1));
    site_frames(s, off, pos);
    for (int64_t i = 0; i < B; ++i) {
        double F[3], T[3];
        flags |= site_wca_body(s, par, off, pos, i, rc2, F, T);
        for (int k = 0; k < 3; ++k) {
            s->F[k * B + i] = F[k];
            s->T[k * B + i] = T[k];
        }
    }
    free(off);
    free(pos);
    return flags;
}

/* Mode 2 force and torque of the n listed bodies only (the same sums as
 * orc_body_forces; F, T are [3][n]). */
uint32_t orc_site_wca_bodies(const orc_sys *s, const orc_par *par, const int64_t *idx, int64_t n, double *F,
                             double *T)
{
    uint32_t flags = 0;
    int64_t S = s->S;
    double rc = par->delta + 0x1.1f59ac3c7d6c0p+0 * par->sigma;
    double rc2 = rc * rc;
    double *off = (double *)malloc(sizeof(double) * 3 * (size_t)(S > 0 ? S : 1));
    double *pos = (double *)malloc(sizeof(double) * 3 * (size_t)(S > 0 ? S : 1));
    site_frames(s, off, pos);
    for (int64_t u = 0; u < n; ++u) {
        double Fi[3], Ti[3];
        flags |= site_wca_body(s, par, off, pos, idx[u], rc2, Fi, Ti);
        for (int k = 0; k < 3; ++k) {
            F[k * n + u] = Fi[k];
            T[k * n + u] = Ti[k];
        }
    }
    free(off);
    free(pos);
    return flags;
}

/* Total WCA potential energy, Eq. (1), summed over interacting pairs (body
 * centres in mode 1, sites of different bodies in mode 2).  Used to check
 * forces and torques as derivatives of the potential. */
double orc_wca_energy(const orc_sys *s, const orc_par *par)
{
    int64_t B = s->B, S = s->S;
    double rc = par->delta + 0x1.1f59ac3c7d6c0p+0 * par->sigma;
    double U = 0.0;
    double *off = NULL, *pos = NULL;
    if (par->wca_mode == 2) {
        off = (double *)malloc(sizeof(double) * 3 * (size_t)(S > 0 ? S : 1));
        pos = (double *)malloc(sizeof(double) * 3 * (size_t)(S > 0 ? S : 1));
        site_frames(s, off, pos);
    }
    for (int64_t i = 0; i < B; ++i)
        for (int64_t b = i + 1; b < B; ++b) {
            int64_t n1 = par->wca_mode == 2 ? s->site_off[i + 1] - s->site_off[i] : 1;
            int64_t n2 = par->wca_mode == 2 ? s->site_off[b + 1] - s->site_off[b] : 1;
            for (int64_t u = 0; u < n1; ++u)
                for (int64_t w = 0; w < n2; ++w) {
                    double r2 = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        double L = box_len(s, k);
                        double t = par->wca_mode == 2
                                       ? pos[k * S + s->site_off[i] + u] - pos[k * S + s->site_off[b] + w]
                                       : s->R[k * B + i] - s->R[k * B + b];
                        t = t - L * rint(t / L);
                        r2 += t * t;
                    }
                    double r = sqrt(r2);
                    if (r > rc || r <= par->delta) continue;
                    double x = par->sigma / (r - par->delta);
                    double x6 = pow(x, 6.0);
                    U += 4.0 * par->eps * (x6 * x6 - x6) + par->eps;
                }
        }
    free(off);
    free(pos);
    return U;
}

/* One NO_SQUISH free rotation about body axis k for time delta. */
static void nosquish_rot(int k, double delta, double Ik, double q[4], double p[4])
{
    if (Ik == 0.0) return;
    double Pq[4], Pp[4];
    perm_k(k, q, Pq);
    double zeta = (delta * dot4(p, Pq)) / (4.0 * Ik);
    double sn, cs;
    orc_dsincos(zeta, &sn, &cs);
    perm_k(k, p, Pp);
    for (int r = 0; r < 4; ++r) {
        q[r] = cs * q[r] + sn * Pq[r];
        p[r] = cs * p[r] + sn * Pp[r];
    }
}

/* ------------------------------------------------------------------------- */
/* (a5) Apply the collision impulse (J, K) to each body, then one velocity    */
/* Verlet step of the Miller et al. quaternion scheme: half kick, drift,      */
/* NO_SQUISH rotation (axes 3,2,1,2,3), new forces, half kick.                */
uint32_t orc_body_integrate(orc_sys *s, const orc_par *par, const double *J, const double *K)
{
    uint32_t flags = 0;
    int64_t B = s->B;
    double dt = par->dt, hdt = 0.5 * par->dt;
    for (int64_t b = 0; b < B; ++b) {
        double q[4], p[4], A[3][3], Kv[3], Kh[3], Tv[3], Th[3], dq[4];
        for (int r = 0; r < 4; ++r) { q[r] = s->q[r * B + b]; p[r] = s->p[r * B + b]; }
        quat_to_mat(q, A);
        /* impulse from the collision */
        for (int k = 0; k < 3; ++k) s->P[k * B + b] = s->P[k * B + b] + J[k * B + b];
        for (int k = 0; k < 3; ++k) Kv[k] = K[k * B + b];
        mat_t_vec(A, Kv, Kh);
        quat_times_pure(q, Kh, dq);
        for (int r = 0; r < 4; ++r) p[r] = p[r] + 2.0 * dq[r];
        /* first half kick */
        for (int k = 0; k < 3; ++k) s->P[k * B + b] = s->P[k * B + b] + hdt * s->F[k * B + b];
        for (int k = 0; k < 3; ++k) Tv[k] = s->T[k * B + b];
        mat_t_vec(A, Tv, Th);
        quat_times_pure(q, Th, dq);
        for (int r = 0; r < 4; ++r) p[r] = p[r] + dt * dq[r];
        /* drift */
        for (int k = 0; k < 3; ++k) {
            double L = box_len(s, k);
            double y = s->R[k * B + b] + dt * (s->P[k * B + b] / s->M[b]);
            if (y >= L) { y = y - L; s->img[k * B + b] += 1; }
            else if (y < 0.0) { y = y + L; s->img[k * B + b] -= 1; }
            if (!(y >= 0.0 && y <= L)) flags |= (y != y) ? ORC_NONFINITE : ORC_ESCAPE;
            s->R[k * B + b] = y;
        }
        /* free rotation */
        double I1 = s->I[b], I2 = s->I[B + b], I3 = s->I[2 * B + b];
        nosquish_rot(3, hdt, I3, q, p);
        nosquish_rot(2, hdt, I2, q, p);
        nosquish_rot(1, dt, I1, q, p);
        nosquish_rot(2, hdt, I2, q, p);
        nosquish_rot(3, hdt, I3, q, p);
        for (int r = 0; r < 4; ++r) { s->q[r * B + b] = q[r]; s->p[r * B + b] = p[r]; }
    }
    flags |= orc_body_forces(s, par);
    for (int64_t b = 0; b < B; ++b) {
        double q[4], A[3][3], Tv[3], Th[3], dq[4];
        for (int r = 0; r < 4; ++r) q[r] = s->q[r * B + b];
        quat_to_mat(q, A);
        for (int k = 0; k < 3; ++k) s->P[k * B + b] = s->P[k * B + b] + hdt * s->F[k * B + b];
        for (int k = 0; k < 3; ++k) Tv[k] = s->T[k * B + b];
        mat_t_vec(A, Tv, Th);
        quat_times_pure(q, Th, dq);
        for (int r = 0; r < 4; ++r) s->p[r * B + b] = s->p[r * B + b] + dt * dq[r];
        for (int k = 0; k < 3; ++k)
            if (!isfinite(s->P[k * B + b])) flags |= ORC_NONFINITE;
    }
    return flags;
}

/* ------------------------------------------------------------------------- */
/* (a7) Ballistic streaming of the solvent with periodic wrap (Sec. II.A).    */
/* With a constant acceleration g (forced flow, Sec. III.B), Newton's
 * equations over dt give x + v dt + g dt^2 / 2 and v + g dt, evaluated as
 * (x + v dt) + h with h = (dt / 2)(g dt), then v + g dt. */
uint32_t orc_stream_forced(orc_sys *s, double dt, const double g[3])
{
    uint32_t flags = 0;
    int on = forced(g);
    for (int k = 0; k < 3; ++k) {
        double L = box_len(s, k);
        double gdt = g[k] * dt;
        double h = (0.5 * dt) * gdt;
        for (int64_t i = 0; i < s->N; ++i) {
            double y = s->x[k * s->N + i] + s->v[k * s->N + i] * dt;
            if (on) {
                y = y + h;
                s->v[k * s->N + i] = s->v[k * s->N + i] + gdt;
            }
            s->x[k * s->N + i] = wrap1(y, L, &flags);
        }
    }
    return flags;
}

uint32_t orc_stream(orc_sys *s, double dt)
{
    const double zero[3] = {0.0, 0.0, 0.0};
    return orc_stream_forced(s, dt, zero);
}

/* ------------------------------------------------------------------------- */
/* Harmonic-bond comparator (Sec. II.B.1).  Each colloid is a centre site plus */
/* surface sites; every surface site is bonded to its nearest surface         */
/* neighbours and to the centre by u_b = (k_b / 2)(r - r_b)^2, Eq. (2).  All  */
/* sites move by velocity Verlet with a small step; the surface sites collide */
/* like heavy solvent (the orc_sys site arrays xs, vs, sm, with B = 0); the   */
/* centre sites carry the colloid WCA of Eq. (1) and do not collide.          */
typedef struct {
    int64_t B;               /* colloids (one centre site each) */
    double *xc, *vc;         /* [3B] centre sites (wrapped), velocities */
    int32_t *imgc, *imgs;    /* [3B], [3S] periodic images */
    double mc;               /* centre site mass */
    double kb;               /* spring constant */
    const int64_t *site_off; /* [B+1] surface sites of colloid b */
    const int32_t *site_body;/* [S] colloid of each surface site */
    const int64_t *adj_off;  /* [S+1] bonds of surface site j to other surface sites */
    const int32_t *adj;      /* partner (ascending within each site's range) */
    const double *adj_r0;    /* rest length of each bond */
    const double *rc0;       /* [S] rest length of the bond of site j to its centre */
    double *fs, *fc;         /* [3S], [3B] forces at the current positions */
} orc_harm;

/* Force on the first end of a bond with separation d = x_1 - x_2 (minimum
 * image): -k_b (r - r0) d / r, added to f. */
static void bond_add(double kb, double r0, const double d[3], double f[3])
{
    double r = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    double fo = (-kb * (r - r0)) / r;
    for (int k = 0; k < 3; ++k) f[k] = f[k] + fo * d[k];
}

/* Forces on every site: a surface site sums its surface bonds in ascending
 * partner index, then its centre bond; a centre sums its bonds in site order,
 * then the WCA of Eq. (1) with the other centres in ascending index. */
uint32_t orc_harm_forces(const orc_sys *s, orc_harm *h, const orc_par *par)
{
    uint32_t flags = 0;
    int64_t S = s->S, B = h->B;
    for (int64_t j = 0; j < S; ++j) {
        double f[3] = {0.0, 0.0, 0.0}, d[3];
        for (int64_t e = h->adj_off[j]; e < h->adj_off[j + 1]; ++e) {
            int64_t k2 = h->adj[e];
            for (int k = 0; k < 3; ++k) d[k] = min_image(s->xs[k * S + j] - s->xs[k * S + k2], box_len(s, k));
            bond_add(h->kb, h->adj_r0[e], d, f);
        }
        int64_t b = h->site_body[j];
        for (int k = 0; k < 3; ++k) d[k] = min_image(s->xs[k * S + j] - h->xc[k * B + b], box_len(s, k));
        bond_add(h->kb, h->rc0[j], d, f);
        for (int k = 0; k < 3; ++k) h->fs[k * S + j] = f[k];
    }
    double rc = par->delta + 0x1.1f59ac3c7d6c0p+0 * par->sigma;
    double rc2 = rc * rc;
    for (int64_t b = 0; b < B; ++b) {
        double f[3] = {0.0, 0.0, 0.0}, d[3];
        for (int64_t j = h->site_off[b]; j < h->site_off[b + 1]; ++j) {
            for (int k = 0; k < 3; ++k) d[k] = min_image(h->xc[k * B + b] - s->xs[k * S + j], box_len(s, k));
            bond_add(h->kb, h->rc0[j], d, f);
        }
        if (par->wca_mode == 1)
            for (int64_t b2 = 0; b2 < B; ++b2) {
                if (b2 == b) continue;
                double dr[3];
                for (int k = 0; k < 3; ++k) {
                    double L = box_len(s, k);
                    double t = h->xc[k * B + b] - h->xc[k * B + b2];
                    if (t > 0.5 * L) t = t - L;
                    else if (t < -0.5 * L) t = t + L;
                    dr[k] = t;
                }
                double r2 = (dr[0] * dr[0] + dr[1] * dr[1]) + dr[2] * dr[2];
                if (!(r2 <= rc2)) continue;
                flags |= wca_pair(par, dr, r2, f);
            }
        for (int k = 0; k < 3; ++k) h->fc[k * B + b] = f[k];
    }
    return flags;
}

/* Velocity Verlet for all sites, nsub steps of dt: v += (dt/2)(f/m),
 * x += v dt (wrapped, image counted), new forces, v += (dt/2)(f/m). */
uint32_t orc_harm_md(orc_sys *s, orc_harm *h, const orc_par *par, double dt, int64_t nsub)
{
    uint32_t flags = 0;
    int64_t S = s->S, B = h->B;
    double hdt = 0.5 * dt;
    for (int64_t n = 0; n < nsub; ++n) {
        for (int k = 0; k < 3; ++k) {
            double L = box_len(s, k);
            for (int64_t j = 0; j < S; ++j) {
                double v = s->vs[k * S + j] + hdt * (h->fs[k * S + j] / s->sm[j]);
                s->vs[k * S + j] = v;
                double y = s->xs[k * S + j] + v * dt;
                if (y >= L) { y = y - L; h->imgs[k * S + j] += 1; }
                else if (y < 0.0) { y = y + L; h->imgs[k * S + j] -= 1; }
                if (!(y >= 0.0 && y <= L)) flags |= (y != y) ? ORC_NONFINITE : ORC_ESCAPE;
                s->xs[k * S + j] = y;
            }
            for (int64_t b = 0; b < B; ++b) {
                double v = h->vc[k * B + b] + hdt * (h->fc[k * B + b] / h->mc);
                h->vc[k * B + b] = v;
                double y = h->xc[k * B + b] + v * dt;
                if (y >= L) { y = y - L; h->imgc[k * B + b] += 1; }
                else if (y < 0.0) { y = y + L; h->imgc[k * B + b] -= 1; }
                if (!(y >= 0.0 && y <= L)) flags |= (y != y) ? ORC_NONFINITE : ORC_ESCAPE;
                h->xc[k * B + b] = y;
            }
        }
        flags |= orc_harm_forces(s, h, par);
        for (int k = 0; k < 3; ++k) {
            for (int64_t j = 0; j < S; ++j) s->vs[k * S + j] = s->vs[k * S + j] + hdt * (h->fs[k * S + j] / s->sm[j]);
            for (int64_t b = 0; b < B; ++b) h->vc[k * B + b] = h->vc[k * B + b] + hdt * (h->fc[k * B + b] / h->mc);
        }
    }
    return flags;
}

/* Bond and WCA potential energy of the harmonic colloids. */
double orc_harm_energy(const orc_sys *s, const orc_harm *h, const orc_par *par)
{
    int64_t S = s->S, B = h->B;
    double U = 0.0;
    for (int64_t j = 0; j < S; ++j) {
        for (int64_t e = h->adj_off[j]; e < h->adj_off[j + 1]; ++e) {
            int64_t k2 = h->adj[e];
            if (k2 < j) continue; /* each bond once */
            double r2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                double t = min_image(s->xs[k * S + j] - s->xs[k * S + k2], box_len(s, k));
                r2 += t * t;
            }
            double x = sqrt(r2) - h->adj_r0[e];
            U += 0.5 * h->kb * x * x;
        }
        int64_t b = h->site_body[j];
        double r2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            double t = min_image(s->xs[k * S + j] - h->xc[k * B + b], box_len(s, k));
            r2 += t * t;
        }
        double x = sqrt(r2) - h->rc0[j];
        U += 0.5 * h->kb * x * x;
    }
    if (par->wca_mode == 1) {
        double rc = par->delta + 0x1.1f59ac3c7d6c0p+0 * par->sigma;
        for (int64_t i = 0; i < B; ++i)
            for (int64_t b = i + 1; b < B; ++b) {
                double r2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    double t = min_image(h->xc[k * B + i] - h->xc[k * B + b], box_len(s, k));
                    r2 += t * t;
                }
                double r = sqrt(r2);
                if (r > rc || r <= par->delta) continue;
                double x6 = pow(par->sigma / (r - par->delta), 6.0);
                U += 4.0 * par->eps * (x6 * x6 - x6) + par->eps;
            }
    }
    return U;
}

/* One collision period of the harmonic model: shift, bin solvent and surface
 * sites, collide (the sites as heavy solvent), stream the solvent over the
 * period, then nsub velocity-Verlet steps of dt_md for the sites. */
uint32_t orc_harm_step(orc_sys *s, orc_harm *h, const orc_par *par, uint64_t step, double dt_md, int64_t nsub)
{
    uint32_t flags = 0;
    int64_t C = (int64_t)s->n[0] * s->n[1] * s->n[2];
    int64_t NT = s->N + s->S;
    double sh[3];
    orc_shift(par->seed, step, par->replica, s->a, sh);
    int32_t *cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(NT > 0 ? NT : 1));
    int64_t *cs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    int64_t *mem = (int64_t *)malloc(sizeof(int64_t) * (size_t)(NT > 0 ? NT : 1));
    flags |= orc_bin(s, sh, cell, cs, mem);
    flags |= orc_collide(s, par, step, cs, mem, NULL);
    free(cell);
    free(cs);
    free(mem);
    flags |= orc_stream_forced(s, par->dt, par->g);
    flags |= orc_harm_md(s, h, par, dt_md, nsub);
    return flags;
}

/* ------------------------------------------------------------------------- */
/* Reverse nonequilibrium shear (Sec. III.B, viscosity).  The solvent in the  */
/* lower slab y0 <= y < y0 + dy whose v_x is closest to +target and in the     */
/* upper slab y1 <= y < y1 + dy closest to -target are ranked by |v_x -+      */
/* target| (ties: lower identity first); the first min(npairs, n_lower,       */
/* n_upper) of each list exchange v_x pairwise.  *dp accumulates the          */
/* x-momentum moved from the lower to the upper slab, m (v_lower - v_upper)   */
/* per pair, in rank order.  tag (optional) gives the identities.            */
typedef struct {
    double key;
    int64_t id, k;
} rn_item;

static int rn_cmp(const void *a, const void *b)
{
    const rn_item *x = (const rn_item *)a, *y = (const rn_item *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->id < y->id) ? -1 : (x->id > y->id);
}

uint32_t orc_rnemd(orc_sys *s, const int32_t *tag, double y0, double y1, double dy, double target,
                   int64_t npairs, double *dp, int64_t *nswapped)
{
    int64_t N = s->N;
    rn_item *lo = (rn_item *)malloc(sizeof(rn_item) * (size_t)(N > 0 ? N : 1));
    rn_item *up = (rn_item *)malloc(sizeof(rn_item) * (size_t)(N > 0 ? N : 1));
    int64_t nl = 0, nu = 0;
    for (int64_t k = 0; k < N; ++k) {
        double y = s->x[N + k], vx = s->v[k];
        int64_t id = tag ? (int64_t)tag[k] : k;
        if (y >= y0 && y < y0 + dy) {
            lo[nl].key = fabs(vx - target); lo[nl].id = id; lo[nl].k = k; ++nl;
        } else if (y >= y1 && y < y1 + dy) {
            up[nu].key = fabs(vx + target); up[nu].id = id; up[nu].k = k; ++nu;
        }
    }
    qsort(lo, (size_t)nl, sizeof(rn_item), rn_cmp);
    qsort(up, (size_t)nu, sizeof(rn_item), rn_cmp);
    int64_t np = npairs;
    if (nl < np) np = nl;
    if (nu < np) np = nu;
    double acc = *dp;
    for (int64_t i = 0; i < np; ++i) {
        double vl = s->v[lo[i].k], vu = s->v[up[i].k];
        acc = acc + s->m * (vl - vu);
        s->v[lo[i].k] = vu;
        s->v[up[i].k] = vl;
    }
    *dp = acc;
    *nswapped = np;
    free(lo);
    free(up);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* One full step n: thermalize sites, shift, bin, collide, transfer to the    */
/* bodies, stream the solvent, integrate the bodies.                          */
uint32_t orc_step(orc_sys *s, const orc_par *par, uint64_t step)
{
    uint32_t flags = 0;
    int64_t C = (int64_t)s->n[0] * s->n[1] * s->n[2];
    int64_t NT = s->N + s->S;
    int32_t *cell = (int32_t *)malloc((size_t)(NT > 0 ? NT : 1) * sizeof(int32_t));
    int64_t *cell_start = (int64_t *)malloc((size_t)(C + 1) * sizeof(int64_t));
    int64_t *members = (int64_t *)malloc((size_t)(NT > 0 ? NT : 1) * sizeof(int64_t));
    double *J = (double *)calloc((size_t)(3 * s->B + 1), sizeof(double));
    double *K = (double *)calloc((size_t)(3 * s->B + 1), sizeof(double));
    double shift[3];

    flags |= orc_sites_thermalize(s, par, step, NULL);
    orc_shift(par->seed, step, par->replica, s->a, shift);
    flags |= orc_bin(s, shift, cell, cell_start, members);
    flags |= orc_collide(s, par, step, cell_start, members, NULL);
    flags |= orc_sites_to_body(s, J, K);
    flags |= orc_stream_forced(s, par->dt, par->g);
    flags |= orc_body_integrate(s, par, J, K);

    free(cell); free(cell_start); free(members); free(J); free(K);
    return flags;
}

/* Run nsteps steps starting at step0; returns the OR of the status bits. */
uint32_t orc_run(orc_sys *s, const orc_par *par, uint64_t step0, int64_t nsteps)
{
    uint32_t flags = 0;
    for (int64_t i = 0; i < nsteps; ++i) flags |= orc_step(s, par, step0 + (uint64_t)i);
    return flags;
}

/* ------------------------------------------------------------------------- */
/* Array helpers for the statistical pins of the samplers.                    */
void orc_dlog_n(const double *x, double *y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = orc_dlog(x[i]);
}

void orc_dsincos_n(const double *x, double *s, double *c, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) orc_dsincos(x[i], &s[i], &c[i]);
}

uint32_t orc_site_normals_n(uint64_t seed, uint64_t step, uint64_t replica, int64_t n, double *z)
{
    uint32_t flags = 0;
    for (int64_t j = 0; j < n; ++j) flags |= orc_site_normals(seed, step, (uint64_t)j, replica, &z[3 * j]);
    return flags;
}

uint32_t orc_cell_axis_n(uint64_t seed, uint64_t step, uint64_t replica, int64_t n, double *ax)
{
    uint32_t flags = 0;
    for (int64_t c = 0; c < n; ++c) flags |= orc_cell_axis(seed, step, (uint64_t)c, replica, &ax[3 * c]);
    return flags;
}

uint32_t orc_gamma_n(uint64_t seed, uint64_t step, uint64_t replica, double k, int64_t n, double *g)
{
    uint32_t flags = 0;
    for (int64_t c = 0; c < n; ++c) flags |= orc_gamma(seed, step, (uint64_t)c, replica, k, &g[c]);
    return flags;
}

uint32_t orc_cell_draws_n(uint64_t seed, uint64_t step, uint64_t replica, double k, int64_t n, double *ax, double *g)
{
    uint32_t flags = 0;
    for (int64_t c = 0; c < n; ++c) flags |= orc_cell_draws(seed, step, (uint64_t)c, replica, 1, k, &ax[3 * c], &g[c]);
    return flags;
}
