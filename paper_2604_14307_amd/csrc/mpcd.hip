// mpcd.hip -- HIP kernels (gfx950) and the C ABI of libmpcd.so.
//
// One MPCD step with rigid-body discrete-particle colloids (Bush, Palmer,
// Howard, arXiv 2604.14307): site thermalization (Eqs. 5, 7), random grid
// shift and counting-sort binning, SRD collision with an optional cell
// thermostat (Sec. II.A), momentum transfer to the bodies (Sec. II.B.2),
// quaternion velocity-Verlet body update (Miller et al., cited in Sec. II.B.2)
// and ballistic streaming.
//
// Design (MI355X): SoA arrays with coalesced grid-stride passes over particles;
// cells are sorted by an atomic counting sort (count, exclusive scan, scatter)
// into a permutation; the collision runs one lane per cell over its segment of
// the permutation.  The FP64 form sums each cell's members in ascending
// identity (ordered in LDS), so it reproduces a sequential host sum bit for
// bit.  The FP32 form sums m v exactly in int64 fixed point (2^-32), so its
// cell sums are exact and independent of order.  Body-level sums run in FP64
// in site order.  Everything is built with -ffp-contract=off.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "../../include/mpcd.h"
#include "detrand.hpp"

using namespace mpcd;

namespace {

// ---------------------------------------------------------------------------
// Kernel-side views of the C-ABI structs

struct SysDev {
    int32_t nsys;
    double a;
    double m;
    int64_t N, S, B, C;
    uint64_t replica0;
    const int32_t *ncell;
    const int64_t *solv_off, *cell_off, *body_off;
};

struct BodyDev {
    double *pos;
    int32_t *image;
    double *quat, *mom, *angmom, *force, *torque;
    const double *mass, *inertia;
    const int64_t *site_off;
    const int32_t *site_body;
    const double *site_d, *site_m;
};

SysDev make_sysdev(const mpcd_sys *s)
{
    SysDev d;
    d.nsys = s->nsys;
    d.a = s->a;
    d.m = s->m_solvent;
    d.N = s->n_solvent;
    d.S = s->n_sites;
    d.B = s->n_bodies;
    d.C = s->n_cells;
    d.replica0 = s->replica0;
    d.ncell = s->ncell;
    d.solv_off = s->solv_off;
    d.cell_off = s->cell_off;
    d.body_off = s->body_off;
    return d;
}

BodyDev make_bodydev(const mpcd_bodies *b)
{
    BodyDev d;
    memset(&d, 0, sizeof d);
    if (!b) return d;
    d.pos = b->pos; d.image = b->image; d.quat = b->quat; d.mom = b->mom; d.angmom = b->angmom;
    d.force = b->force; d.torque = b->torque; d.mass = b->mass; d.inertia = b->inertia;
    d.site_off = b->site_off; d.site_body = b->site_body; d.site_d = b->site_d; d.site_m = b->site_m;
    return d;
}

// Largest r in [0, nsys) with off[r] <= i.
__device__ __forceinline__ int find_sys(const int64_t *off, int nsys, int64_t i)
{
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void flag(uint32_t *status, uint32_t bits)
{
    if (bits) atomicOr(status, bits);
}

// ---------------------------------------------------------------------------
// Small fixed-order vector algebra (FP64)

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Body-to-space rotation matrix of the quaternion (w, x, y, z).
__device__ __forceinline__ void quat_matrix(const double q[4], double A[3][3])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
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

__device__ __forceinline__ void matvec(const double A[3][3], const double v[3], double o[3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i) o[i] = (A[i][0] * v[0] + A[i][1] * v[1]) + A[i][2] * v[2];
}

__device__ __forceinline__ void matTvec(const double A[3][3], const double v[3], double o[3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i) o[i] = (A[0][i] * v[0] + A[1][i] * v[1]) + A[2][i] * v[2];
}

// q (x) (0, a): S(q) of Miller et al. applied to the pure quaternion (0, a).
__device__ __forceinline__ void qmul_pure(const double q[4], const double a[3], double o[4])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    o[0] = ((-x) * a[0] + (-y) * a[1]) + (-z) * a[2];
    o[1] = (w * a[0] + (-z) * a[1]) + y * a[2];
    o[2] = (z * a[0] + w * a[1]) + (-x) * a[2];
    o[3] = ((-y) * a[0] + x * a[1]) + w * a[2];
}

// Permutations P_k of Miller et al.
__device__ __forceinline__ void perm_q(int k, const double q[4], double o[4])
{
    if (k == 1) { o[0] = -q[1]; o[1] = q[0]; o[2] = q[3]; o[3] = -q[2]; }
    else if (k == 2) { o[0] = -q[2]; o[1] = -q[3]; o[2] = q[0]; o[3] = q[1]; }
    else { o[0] = -q[3]; o[1] = q[2]; o[2] = -q[1]; o[3] = q[0]; }
}

__device__ __forceinline__ double dot4(const double a[4], const double b[4])
{
    return ((a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]) + a[3] * b[3];
}

// Space-frame angular velocity omega = A (Lhat / I), Lhat_k = p . P_k q / 2.
__device__ __forceinline__ void body_omega(const double q[4], const double p[4], const double A[3][3],
                                           const double I[3], double w[3])
{
    double wh[3];
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        double Pq[4];
        perm_q(k, q, Pq);
        const double Lk = 0.5 * dot4(p, Pq);
        wh[k - 1] = (I[k - 1] == 0.0) ? 0.0 : Lk / I[k - 1];
    }
    matvec(A, wh, w);
}

__device__ __forceinline__ double wrap_d(double y, double L, uint32_t &st)
{
    if (y >= L) y = y - L;
    else if (y < 0.0) y = y + L;
    if (!(y >= 0.0 && y <= L)) st |= (y != y) ? ST_NONFINITE : ST_ESCAPE;
    return y;
}

__device__ __forceinline__ float wrap_f(float y, float L, uint32_t &st)
{
    if (y >= L) y = y - L;
    else if (y < 0.0f) y = y + L;
    if (!(y >= 0.0f && y <= L)) st |= (y != y) ? ST_NONFINITE : ST_ESCAPE;
    return y;
}

template <typename Real> struct Prec;
template <> struct Prec<double> {
    __device__ static double wrap(double y, double L, uint32_t &st) { return wrap_d(y, L, st); }
};
template <> struct Prec<float> {
    __device__ static float wrap(float y, float L, uint32_t &st) { return wrap_f(y, L, st); }
};

// Cell index along one axis for the shifted grid: floor((x - s)/a) mod n.
__device__ __forceinline__ int axis_cell(double x, double s, double a, int n, uint32_t &st)
{
    const double g = x - s;
    const double jf = floor(g / a);
    if (!(jf >= -1.0 && jf <= (double)n)) {
        st |= (g != g) ? ST_NONFINITE : ST_ESCAPE;
        return 0;
    }
    int j = (int)jf;
    if (j < 0) j += n;
    else if (j >= n) j -= n;
    return j;
}

__device__ __forceinline__ int axis_cell(float x, double s, double a, int n, uint32_t &st)
{
    const float g = x - (float)s;
    const float jf = floorf(g / (float)a);
    if (!(jf >= -1.0f && jf <= (float)n)) {
        st |= (g != g) ? ST_NONFINITE : ST_ESCAPE;
        return 0;
    }
    int j = (int)jf;
    if (j < 0) j += n;
    else if (j >= n) j -= n;
    return j;
}

inline unsigned grid_for(int64_t n, int block, int64_t cap = 1 << 20)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// ---------------------------------------------------------------------------
// Workspace layout (identical for every call with the same sizes)

struct Layout {
    size_t status, shift, counts, cell_start, cellid, slot, perm, partial, site_d, vpre, body_dv,
        body_dw, total;
};

constexpr int SCAN_T = 1024, SCAN_V = 4, SCAN_TILE = SCAN_T * SCAN_V;

Layout layout_of(const mpcd_sys *s)
{
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const int64_t NT = s->n_solvent + s->n_sites;
    const int64_t nb = (s->n_cells + SCAN_TILE - 1) / SCAN_TILE;
    L.status = take(256);
    L.shift = take(sizeof(double) * 3 * (size_t)s->nsys);
    L.counts = take(sizeof(int32_t) * (size_t)s->n_cells);
    L.cell_start = take(sizeof(int32_t) * (size_t)(s->n_cells + 1));
    L.cellid = take(sizeof(int32_t) * (size_t)NT);
    L.slot = take(sizeof(int32_t) * (size_t)NT);
    L.perm = take(sizeof(int32_t) * (size_t)NT);
    L.partial = take(sizeof(int32_t) * (size_t)(nb + 1));
    L.site_d = take(sizeof(double) * 3 * (size_t)s->n_sites);
    L.vpre = take(sizeof(double) * 3 * (size_t)s->n_sites);
    L.body_dv = take(sizeof(double) * 3 * (size_t)s->n_bodies);
    L.body_dw = take(sizeof(double) * 3 * (size_t)s->n_bodies);
    L.total = off;
    return L;
}

template <typename T> T *at(void *ws, size_t off) { return (T *)((char *)ws + off); }

// ---------------------------------------------------------------------------
// Utility kernels

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t val)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t val)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

__global__ void k_advance(uint64_t *d_step)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *d_step = *d_step + 1;
}

// ---------------------------------------------------------------------------
// (a7) streaming

template <typename Real>
__global__ void k_stream(SysDev s, Real *x, const Real *v, double dt, uint32_t *status)
{
    uint32_t st = 0;
    const Real dtr = (Real)dt;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int r = find_sys(s.solv_off, s.nsys, i);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const Real L = (Real)((double)s.ncell[3 * r + k] * s.a);
            const Real y = x[k * s.N + i] + v[k * s.N + i] * dtr;
            x[k * s.N + i] = Prec<Real>::wrap(y, L, st);
        }
    }
    flag(status, st);
}

// ---------------------------------------------------------------------------
// (a2) grid shift and counting sort

__global__ void k_shift(SysDev s, uint64_t seed, const uint64_t *d_step, double *shift)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= s.nsys) return;
    const Words w = rng_draw(seed, RNG_SHIFT, *d_step, 0, s.replica0 + (uint64_t)r, 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) shift[3 * r + k] = shift_component(w.w[k], s.a);
}

template <typename Real>
__global__ void k_bin_count(SysDev s, const Real *x, const Real *xs, const int32_t *site_body,
                            const double *shift, int32_t *counts, int32_t *cellid, int32_t *slot,
                            uint32_t *status)
{
    uint32_t st = 0;
    const int64_t NT = s.N + s.S;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < NT;
         k += (int64_t)gridDim.x * blockDim.x) {
        int r;
        Real p0, p1, p2;
        if (k < s.N) {
            r = find_sys(s.solv_off, s.nsys, k);
            p0 = x[k]; p1 = x[s.N + k]; p2 = x[2 * s.N + k];
        } else {
            const int64_t j = k - s.N;
            r = find_sys(s.body_off, s.nsys, (int64_t)site_body[j]);
            p0 = xs[j]; p1 = xs[s.S + j]; p2 = xs[2 * s.S + j];
        }
        const int nx = s.ncell[3 * r], ny = s.ncell[3 * r + 1], nz = s.ncell[3 * r + 2];
        const int jx = axis_cell(p0, shift[3 * r], s.a, nx, st);
        const int jy = axis_cell(p1, shift[3 * r + 1], s.a, ny, st);
        const int jz = axis_cell(p2, shift[3 * r + 2], s.a, nz, st);
        const int64_t gc = s.cell_off[r] + ((int64_t)jz * ny + jy) * nx + jx;
        slot[k] = atomicAdd(&counts[gc], 1);
        cellid[k] = (int32_t)gc;
    }
    flag(status, st);
}

// Block-wide exclusive scan of one value per thread (SCAN_T threads, wave64).
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *total)
{
    __shared__ int32_t wsum[SCAN_T / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        int32_t w = (lane < SCAN_T / 64) ? wsum[lane] : 0;
        int32_t wi = w;
#pragma unroll
        for (int d = 1; d < SCAN_T / 64; d <<= 1) {
            const int32_t y = __shfl_up(wi, d, 64);
            if (lane >= d) wi += y;
        }
        if (lane < SCAN_T / 64) wsum[lane] = wi - w;
        if (lane == SCAN_T / 64 - 1) *total = wi;
    }
    __syncthreads();
    const int32_t res = wsum[wid] + inc - v;
    __syncthreads();
    return res;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const int32_t *counts, int64_t C, int32_t *partial)
{
    __shared__ int32_t tot;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_V;
    int32_t v = 0;
#pragma unroll
    for (int i = 0; i < SCAN_V; ++i)
        if (base + i < C) v += counts[base + i];
    (void)block_exclusive_scan(v, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_partials(int32_t *partial, int64_t nb)
{
    __shared__ int32_t tot;
    int32_t carry = 0;
    for (int64_t base = 0; base < nb; base += SCAN_T) {
        const int64_t i = base + threadIdx.x;
        const int32_t v = (i < nb) ? partial[i] : 0;
        const int32_t ex = block_exclusive_scan(v, &tot);
        if (i < nb) partial[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(SCAN_T) void k_scan_down(int32_t *counts, int64_t C, const int32_t *partial,
                                                      int32_t *cell_start, int32_t total)
{
    __shared__ int32_t tot;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_V;
    int32_t c[SCAN_V];
    int32_t v = 0;
#pragma unroll
    for (int i = 0; i < SCAN_V; ++i) {
        c[i] = (base + i < C) ? counts[base + i] : 0;
        v += c[i];
    }
    int32_t run = partial[blockIdx.x] + block_exclusive_scan(v, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_V; ++i) {
        if (base + i < C) {
            cell_start[base + i] = run;
            counts[base + i] = 0;
        }
        run += c[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) cell_start[C] = total;
}

__global__ void k_bin_scatter(int64_t NT, const int32_t *cellid, const int32_t *slot,
                              const int32_t *cell_start, int32_t *perm)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < NT;
         k += (int64_t)gridDim.x * blockDim.x)
        perm[cell_start[cellid[k]] + slot[k]] = (int32_t)k;
}

// ---------------------------------------------------------------------------
// (a3) collision

struct Rot {
    double R[3][3];
};

__device__ __forceinline__ Rot rotation(const double n[3], double ca, double sa)
{
    Rot o;
    const double omc = 1.0 - ca;
    o.R[0][0] = (omc * n[0]) * n[0] + ca;
    o.R[0][1] = (omc * n[0]) * n[1] - sa * n[2];
    o.R[0][2] = (omc * n[0]) * n[2] + sa * n[1];
    o.R[1][0] = (omc * n[1]) * n[0] + sa * n[2];
    o.R[1][1] = (omc * n[1]) * n[1] + ca;
    o.R[1][2] = (omc * n[1]) * n[2] - sa * n[0];
    o.R[2][0] = (omc * n[2]) * n[0] - sa * n[1];
    o.R[2][1] = (omc * n[2]) * n[1] + sa * n[0];
    o.R[2][2] = (omc * n[2]) * n[2] + ca;
    return o;
}

constexpr int COL_T = 128;   // cells per block (one lane per cell)
constexpr int COL_MAXK = 32; // members ordered in LDS; larger cells use a slower path

struct CollideArgs {
    SysDev s;
    const double *site_m;
    const int32_t *tag;
    const int32_t *cell_start, *perm;
    double cos_a, sin_a, kT_cell, dt;
    uint64_t seed;
    const uint64_t *d_step;
    uint32_t *status;
};

// FP64: cell sums in ascending identity (tag for solvent, N_total + site index
// for sites), exactly as a sequential host loop.
__global__ __launch_bounds__(COL_T) void k_collide_f64(CollideArgs A, double *v, double *vs, double *xstream)
{
    __shared__ uint64_t skey[COL_MAXK * COL_T];
    const SysDev &s = A.s;
    const int t = threadIdx.x;
    const int64_t gc = (int64_t)blockIdx.x * COL_T + t;
    if (gc >= s.C) return;
    const int b = A.cell_start[gc], e = A.cell_start[gc + 1], n = e - b;
    if (n == 0) return;
    uint32_t st = 0;
    const int r = find_sys(s.cell_off, s.nsys, gc);
    const int64_t N = s.N, S = s.S;

    auto key_of = [&](int32_t k) -> uint64_t {
        const uint32_t tg = (k < N && A.tag) ? (uint32_t)A.tag[k] : (uint32_t)k;
        return ((uint64_t)tg << 32) | (uint32_t)k;
    };
    auto mass = [&](int32_t k) -> double { return k < N ? s.m : A.site_m[k - N]; };
    auto vel = [&](int32_t k, int d) -> double & { return k < N ? v[d * N + k] : vs[d * S + (k - N)]; };

    const bool fast = n <= COL_MAXK;
    if (fast && n >= 2) {
        // insertion into a sorted column of LDS (members arrive nearly ordered)
        for (int i = 0; i < n; ++i) {
            const uint64_t kk = key_of(A.perm[b + i]);
            int pos = i;
            while (pos > 0 && skey[(pos - 1) * COL_T + t] > kk) {
                skey[pos * COL_T + t] = skey[(pos - 1) * COL_T + t];
                --pos;
            }
            skey[pos * COL_T + t] = kk;
        }
    }
    auto canonical = [&](auto &&fn) {
        if (fast) {
            for (int i = 0; i < n; ++i) fn((int32_t)(uint32_t)(skey[i * COL_T + t] & 0xffffffffu));
        } else {
            uint64_t lo = 0;
            for (int i = 0; i < n; ++i) {
                uint64_t best = ~0ull;
                for (int j = b; j < e; ++j) {
                    const uint64_t kk = key_of(A.perm[j]);
                    if (kk >= lo && kk < best) best = kk;
                }
                lo = best + 1;
                fn((int32_t)(uint32_t)(best & 0xffffffffu));
            }
        }
    };

    if (n >= 2) {
        double M = 0.0, P0 = 0.0, P1 = 0.0, P2 = 0.0;
        canonical([&](int32_t k) {
            const double mk = mass(k);
            M = M + mk;
            P0 = P0 + mk * vel(k, 0);
            P1 = P1 + mk * vel(k, 1);
            P2 = P2 + mk * vel(k, 2);
        });
        const double u0 = P0 / M, u1 = P1 / M, u2 = P2 / M;
        const uint64_t step = *A.d_step;
        const uint64_t cl = (uint64_t)(gc - s.cell_off[r]);
        const uint64_t rep = s.replica0 + (uint64_t)r;
        double nax[3];
        st |= cell_axis(A.seed, step, cl, rep, nax);
        const Rot R = rotation(nax, A.cos_a, A.sin_a);
        double lam = 1.0;
        if (A.kT_cell > 0.0) {
            double Es = 0.0;
            canonical([&](int32_t k) {
                const double d0 = vel(k, 0) - u0, d1 = vel(k, 1) - u1, d2 = vel(k, 2) - u2;
                Es = Es + mass(k) * ((d0 * d0 + d1 * d1) + d2 * d2);
            });
            const double E = 0.5 * Es;
            if (E > 0.0) {
                double g;
                const double shape = 0.5 * (double)(3 * (n - 1));
                st |= gamma_variate(A.seed, step, cl, rep, shape, &g);
                const double Enew = A.kT_cell * g;
                lam = sqrt(Enew / E);
            }
        }
        for (int i = b; i < e; ++i) {
            const int32_t k = A.perm[i];
            const double d0 = vel(k, 0) - u0, d1 = vel(k, 1) - u1, d2 = vel(k, 2) - u2;
            const double dl[3] = {d0, d1, d2};
            const double uu[3] = {u0, u1, u2};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double rr = (R.R[d][0] * dl[0] + R.R[d][1] * dl[1]) + R.R[d][2] * dl[2];
                const double vn = uu[d] + lam * rr;
                if (!(vn - vn == 0.0)) st |= ST_NONFINITE;
                vel(k, d) = vn;
            }
        }
    }
    if (xstream) {
        for (int i = b; i < e; ++i) {
            const int32_t k = A.perm[i];
            if (k >= N) continue;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double L = (double)s.ncell[3 * r + d] * s.a;
                const double y = xstream[d * N + k] + v[d * N + k] * A.dt;
                xstream[d * N + k] = wrap_d(y, L, st);
            }
        }
    }
    flag(A.status, st);
}

// FP32: exact int64 fixed-point cell sums (scale 2^32) of m, m v and m |v|^2;
// per-cell quantities in FP64; per-particle rotation in FP32.
__global__ __launch_bounds__(COL_T) void k_collide_f32(CollideArgs A, float *v, float *vs, float *xstream)
{
    const SysDev &s = A.s;
    const int64_t gc = (int64_t)blockIdx.x * COL_T + threadIdx.x;
    if (gc >= s.C) return;
    const int b = A.cell_start[gc], e = A.cell_start[gc + 1], n = e - b;
    if (n == 0) return;
    uint32_t st = 0;
    const int r = find_sys(s.cell_off, s.nsys, gc);
    const int64_t N = s.N, S = s.S;
    auto vel = [&](int32_t k, int d) -> float & { return k < N ? v[d * N + k] : vs[d * S + (k - N)]; };

    if (n >= 2) {
        const double SC = 0x1p32, LIM = 0x1p62;
        long long Mf = 0, P0 = 0, P1 = 0, P2 = 0, Kf = 0;
        for (int i = b; i < e; ++i) {
            const int32_t k = A.perm[i];
            const double mk = k < N ? s.m : A.site_m[k - N];
            const double v0 = (double)vel(k, 0), v1 = (double)vel(k, 1), v2 = (double)vel(k, 2);
            const double q0 = (mk * v0) * SC, q1 = (mk * v1) * SC, q2 = (mk * v2) * SC;
            const double qk = (mk * ((v0 * v0 + v1 * v1) + v2 * v2)) * SC;
            if (!(fabs(q0) < LIM && fabs(q1) < LIM && fabs(q2) < LIM && qk < LIM)) st |= ST_FIXOVF;
            Mf += __double2ll_rn(mk * SC);
            P0 += __double2ll_rn(q0);
            P1 += __double2ll_rn(q1);
            P2 += __double2ll_rn(q2);
            Kf += __double2ll_rn(qk);
        }
        const double Md = (double)Mf;
        const double u0 = (double)P0 / Md, u1 = (double)P1 / Md, u2 = (double)P2 / Md;
        const uint64_t step = *A.d_step;
        const uint64_t cl = (uint64_t)(gc - s.cell_off[r]);
        const uint64_t rep = s.replica0 + (uint64_t)r;
        double nax[3];
        st |= cell_axis(A.seed, step, cl, rep, nax);
        const Rot R = rotation(nax, A.cos_a, A.sin_a);
        double lam = 1.0;
        if (A.kT_cell > 0.0) {
            const double Pd0 = (double)P0 * 0x1p-32, Pd1 = (double)P1 * 0x1p-32, Pd2 = (double)P2 * 0x1p-32;
            const double E = 0.5 * ((double)Kf * 0x1p-32 - ((Pd0 * Pd0 + Pd1 * Pd1) + Pd2 * Pd2) / (Md * 0x1p-32));
            if (E > 0.0) {
                double g;
                const double shape = 0.5 * (double)(3 * (n - 1));
                st |= gamma_variate(A.seed, step, cl, rep, shape, &g);
                lam = sqrt((A.kT_cell * g) / E);
            }
        }
        float Rf[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Rf[i][j] = (float)(lam * R.R[i][j]);
        const float uf[3] = {(float)u0, (float)u1, (float)u2};
        for (int i = b; i < e; ++i) {
            const int32_t k = A.perm[i];
            const float dl[3] = {vel(k, 0) - uf[0], vel(k, 1) - uf[1], vel(k, 2) - uf[2]};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const float vn = uf[d] + ((Rf[d][0] * dl[0] + Rf[d][1] * dl[1]) + Rf[d][2] * dl[2]);
                if (!(vn - vn == 0.0f)) st |= ST_NONFINITE;
                vel(k, d) = vn;
            }
        }
    }
    if (xstream) {
        const float dtf = (float)A.dt;
        for (int i = b; i < e; ++i) {
            const int32_t k = A.perm[i];
            if (k >= N) continue;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const float L = (float)((double)s.ncell[3 * r + d] * s.a);
                const float y = xstream[d * N + k] + v[d * N + k] * dtf;
                xstream[d * N + k] = wrap_f(y, L, st);
            }
        }
    }
    flag(A.status, st);
}

// ---------------------------------------------------------------------------
// (a1) site thermalization: one block per body; per-body sums in site order.

constexpr int BODY_T = 128;

template <typename Real>
__global__ __launch_bounds__(BODY_T) void k_sites_thermalize(SysDev s, BodyDev bd, double kT, int thermalize,
                                                             uint64_t seed, const uint64_t *d_step,
                                                             Real *xs, Real *vs, double *site_d,
                                                             double *vpre, uint32_t *status)
{
    __shared__ double sh[6][BODY_T];
    __shared__ double dvw[6];
    const int64_t b = blockIdx.x;
    if (b >= s.B) return;
    const int t = threadIdx.x;
    const int64_t B = s.B, S = s.S;
    uint32_t st = 0;
    const int r = find_sys(s.body_off, s.nsys, b);
    double q[4], p[4], A[3][3], I[3], V[3], w[3], R[3], Lbox[3];
#pragma unroll
    for (int i = 0; i < 4; ++i) { q[i] = bd.quat[i * B + b]; p[i] = bd.angmom[i * B + b]; }
    quat_matrix(q, A);
    const double Mb = bd.mass[b];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        I[k] = bd.inertia[k * B + b];
        V[k] = bd.mom[k * B + b] / Mb;
        R[k] = bd.pos[k * B + b];
        Lbox[k] = (double)s.ncell[3 * r + k] * s.a;
    }
    body_omega(q, p, A, I, w);
    const int64_t j0 = bd.site_off[b], j1 = bd.site_off[b + 1];
    const int64_t sbase = bd.site_off[s.body_off[r]];
    const uint64_t step = *d_step;
    const uint64_t rep = s.replica0 + (uint64_t)r;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t c0 = j0; c0 < j1; c0 += BODY_T) {
        const int64_t j = c0 + t;
        if (j < j1) {
            const double dh[3] = {bd.site_d[j], bd.site_d[S + j], bd.site_d[2 * S + j]};
            double d[3];
            matvec(A, dh, d);
            double vt[3] = {0.0, 0.0, 0.0};
            if (thermalize) {
                double z[3];
                st |= site_normals(seed, step, (uint64_t)(j - sbase), rep, z);
                const double sig = sqrt(kT / bd.site_m[j]);
#pragma unroll
                for (int k = 0; k < 3; ++k) vt[k] = sig * z[k];
            }
            const double mj = bd.site_m[j];
            double pv[3], c[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                site_d[k * S + j] = d[k];
                xs[k * S + j] = (Real)wrap_d(R[k] + d[k], Lbox[k], st);
                vpre[k * S + j] = vt[k];
                pv[k] = mj * vt[k];
            }
            cross3(d, pv, c);
#pragma unroll
            for (int k = 0; k < 3; ++k) { sh[k][t] = pv[k]; sh[3 + k][t] = c[k]; }
        }
        __syncthreads();
        if (t == 0) {
            const int cnt = (int)((j1 - c0) < BODY_T ? (j1 - c0) : BODY_T);
            for (int i = 0; i < cnt; ++i) {
#pragma unroll
                for (int k = 0; k < 6; ++k) acc[k] = acc[k] + sh[k][i];
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        double Vt[3], Lt[3], Lth[3], wth[3], wt[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) { Vt[k] = acc[k] / Mb; Lt[k] = acc[3 + k]; }
        matTvec(A, Lt, Lth);
#pragma unroll
        for (int k = 0; k < 3; ++k) wth[k] = (I[k] == 0.0) ? 0.0 : Lth[k] / I[k];
        matvec(A, wth, wt);
#pragma unroll
        for (int k = 0; k < 3; ++k) { dvw[k] = V[k] - Vt[k]; dvw[3 + k] = w[k] - wt[k]; }
    }
    __syncthreads();
    const double dV[3] = {dvw[0], dvw[1], dvw[2]}, dw[3] = {dvw[3], dvw[4], dvw[5]};
    for (int64_t j = j0 + t; j < j1; j += BODY_T) {
        const double d[3] = {site_d[j], site_d[S + j], site_d[2 * S + j]};
        double c[3];
        cross3(dw, d, c);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double vj = (dV[k] + c[k]) + vpre[k * S + j];
            const Real vr = (Real)vj;
            if (!(vj - vj == 0.0)) st |= ST_NONFINITE;
            vs[k * S + j] = vr;
            vpre[k * S + j] = (double)vr;
        }
    }
    flag(status, st);
}

// (a4) J = sum m (v - v_pre), K = sum d x m (v - v_pre), site order.
template <typename Real>
__global__ __launch_bounds__(BODY_T) void k_sites_to_body(SysDev s, BodyDev bd, const Real *vs,
                                                          const double *site_d, const double *vpre,
                                                          double *J, double *K)
{
    __shared__ double sh[6][BODY_T];
    const int64_t b = blockIdx.x;
    if (b >= s.B) return;
    const int t = threadIdx.x;
    const int64_t B = s.B, S = s.S;
    const int64_t j0 = bd.site_off[b], j1 = bd.site_off[b + 1];
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t c0 = j0; c0 < j1; c0 += BODY_T) {
        const int64_t j = c0 + t;
        if (j < j1) {
            double mdv[3], d[3], c[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double dv = (double)vs[k * S + j] - vpre[k * S + j];
                mdv[k] = bd.site_m[j] * dv;
                d[k] = site_d[k * S + j];
            }
            cross3(d, mdv, c);
#pragma unroll
            for (int k = 0; k < 3; ++k) { sh[k][t] = mdv[k]; sh[3 + k][t] = c[k]; }
        }
        __syncthreads();
        if (t == 0) {
            const int cnt = (int)((j1 - c0) < BODY_T ? (j1 - c0) : BODY_T);
            for (int i = 0; i < cnt; ++i) {
#pragma unroll
                for (int k = 0; k < 6; ++k) acc[k] = acc[k] + sh[k][i];
            }
        }
        __syncthreads();
    }
    if (t == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) { J[k * B + b] = acc[k]; K[k * B + b] = acc[3 + k]; }
    }
}

// ---------------------------------------------------------------------------
// (a5) rigid bodies

__device__ __forceinline__ void nosquish(int k, double delta, double Ik, double q[4], double p[4])
{
    if (Ik == 0.0) return;
    double Pq[4], Pp[4];
    perm_q(k, q, Pq);
    const double zeta = (delta * dot4(p, Pq)) / (4.0 * Ik);
    double sn, cs;
    det_sincos(zeta, &sn, &cs);
    perm_q(k, p, Pp);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        q[i] = cs * q[i] + sn * Pq[i];
        p[i] = cs * p[i] + sn * Pp[i];
    }
}

__global__ void k_body_first(SysDev s, BodyDev bd, const double *J, const double *K, double dt,
                             uint32_t *status)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= s.B) return;
    const int64_t B = s.B;
    uint32_t st = 0;
    const int r = find_sys(s.body_off, s.nsys, b);
    const double hdt = 0.5 * dt;
    double q[4], p[4], A[3][3], P[3], v3[3], h3[3], dq[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) { q[i] = bd.quat[i * B + b]; p[i] = bd.angmom[i * B + b]; }
    quat_matrix(q, A);
#pragma unroll
    for (int k = 0; k < 3; ++k) P[k] = bd.mom[k * B + b];
    if (J) {
#pragma unroll
        for (int k = 0; k < 3; ++k) P[k] = P[k] + J[k * B + b];
    }
    if (K) {
#pragma unroll
        for (int k = 0; k < 3; ++k) v3[k] = K[k * B + b];
        matTvec(A, v3, h3);
        qmul_pure(q, h3, dq);
#pragma unroll
        for (int i = 0; i < 4; ++i) p[i] = p[i] + 2.0 * dq[i];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) P[k] = P[k] + hdt * bd.force[k * B + b];
#pragma unroll
    for (int k = 0; k < 3; ++k) v3[k] = bd.torque[k * B + b];
    matTvec(A, v3, h3);
    qmul_pure(q, h3, dq);
#pragma unroll
    for (int i = 0; i < 4; ++i) p[i] = p[i] + dt * dq[i];
    const double Mb = bd.mass[b];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double L = (double)s.ncell[3 * r + k] * s.a;
        double y = bd.pos[k * B + b] + dt * (P[k] / Mb);
        if (y >= L) { y = y - L; bd.image[k * B + b] += 1; }
        else if (y < 0.0) { y = y + L; bd.image[k * B + b] -= 1; }
        if (!(y >= 0.0 && y <= L)) st |= (y != y) ? ST_NONFINITE : ST_ESCAPE;
        bd.pos[k * B + b] = y;
        bd.mom[k * B + b] = P[k];
    }
    const double I1 = bd.inertia[b], I2 = bd.inertia[B + b], I3 = bd.inertia[2 * B + b];
    nosquish(3, hdt, I3, q, p);
    nosquish(2, hdt, I2, q, p);
    nosquish(1, dt, I1, q, p);
    nosquish(2, hdt, I2, q, p);
    nosquish(3, hdt, I3, q, p);
#pragma unroll
    for (int i = 0; i < 4; ++i) { bd.quat[i * B + b] = q[i]; bd.angmom[i * B + b] = p[i]; }
    flag(status, st);
}

// Core-shifted WCA between body centres, Eq. (1), partners in ascending index.
__global__ void k_body_forces(SysDev s, BodyDev bd, mpcd_wca wca, uint32_t *status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.B) return;
    const int64_t B = s.B;
    uint32_t st = 0;
    double f[3] = {0.0, 0.0, 0.0};
    if (wca.mode == 1) {
        const int r = find_sys(s.body_off, s.nsys, i);
        const double rc = wca.delta + 0x1.1f59ac3c7d6c0p+0 * wca.sigma;
        const double rc2 = rc * rc;
        double Lb[3], Ri[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Lb[k] = (double)s.ncell[3 * r + k] * s.a;
            Ri[k] = bd.pos[k * B + i];
        }
        for (int64_t j = s.body_off[r]; j < s.body_off[r + 1]; ++j) {
            if (j == i) continue;
            double dr[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double t = Ri[k] - bd.pos[k * B + j];
                if (t > 0.5 * Lb[k]) t = t - Lb[k];
                else if (t < -0.5 * Lb[k]) t = t + Lb[k];
                dr[k] = t;
            }
            const double r2 = (dr[0] * dr[0] + dr[1] * dr[1]) + dr[2] * dr[2];
            if (!(r2 <= rc2)) continue;
            const double rr = sqrt(r2);
            const double sh = rr - wca.delta;
            if (!(sh > 0.0)) { st |= ST_NONFINITE; continue; }
            const double is = wca.sigma / sh;
            const double is2 = is * is;
            const double is6 = (is2 * is2) * is2;
            const double is12 = is6 * is6;
            const double fr = ((24.0 * wca.eps) * (2.0 * is12 - is6)) / sh;
            const double fo = fr / rr;
#pragma unroll
            for (int k = 0; k < 3; ++k) f[k] = f[k] + fo * dr[k];
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) { bd.force[k * B + i] = f[k]; bd.torque[k * B + i] = 0.0; }
    flag(status, st);
}

__global__ void k_body_second(SysDev s, BodyDev bd, double dt, uint32_t *status)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= s.B) return;
    const int64_t B = s.B;
    uint32_t st = 0;
    const double hdt = 0.5 * dt;
    double q[4], A[3][3], v3[3], h3[3], dq[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = bd.quat[i * B + b];
    quat_matrix(q, A);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double Pk = bd.mom[k * B + b] + hdt * bd.force[k * B + b];
        if (!(Pk - Pk == 0.0)) st |= ST_NONFINITE;
        bd.mom[k * B + b] = Pk;
        v3[k] = bd.torque[k * B + b];
    }
    matTvec(A, v3, h3);
    qmul_pure(q, h3, dq);
#pragma unroll
    for (int i = 0; i < 4; ++i) bd.angmom[i * B + b] = bd.angmom[i * B + b] + dt * dq[i];
    flag(status, st);
}

// ---------------------------------------------------------------------------
// Host-side validation and launch helpers

thread_local int g_last_hip = 0;

int hip_check(hipError_t e)
{
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        return MPCD_EHIP;
    }
    return MPCD_OK;
}

int launch_check() { return hip_check(hipGetLastError()); }

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

int check_sizes(const mpcd_sys *s)
{
    if (!s) return MPCD_EINVAL;
    if (s->nsys < 1 || !(s->a > 0.0) || !(s->m_solvent > 0.0)) return MPCD_EINVAL;
    if (s->prec != MPCD_F64 && s->prec != MPCD_F32) return MPCD_ENOTSUP;
    if (s->n_solvent < 0 || s->n_sites < 0 || s->n_bodies < 0 || s->n_cells < 1) return MPCD_EINVAL;
    if (s->n_solvent + s->n_sites >= ((int64_t)1 << 31) || s->n_cells >= ((int64_t)1 << 31))
        return MPCD_EINVAL;
    return MPCD_OK;
}

int check_sys(const mpcd_sys *s)
{
    if (!s) return MPCD_EINVAL;
    if (s->nsys < 1 || !(s->a > 0.0) || !(s->m_solvent > 0.0)) return MPCD_EINVAL;
    if (s->prec != MPCD_F64 && s->prec != MPCD_F32) return MPCD_ENOTSUP;
    if (s->n_solvent < 0 || s->n_sites < 0 || s->n_bodies < 0 || s->n_cells < 1) return MPCD_EINVAL;
    if (s->n_solvent + s->n_sites >= ((int64_t)1 << 31) || s->n_cells >= ((int64_t)1 << 31))
        return MPCD_EINVAL;
    if (!s->ncell || !s->solv_off || !s->cell_off || !s->body_off) return MPCD_EINVAL;
    return MPCD_OK;
}

int check_ws(const mpcd_sys *s, const void *ws, size_t ws_bytes)
{
    if (!ws || !aligned(ws, 256)) return MPCD_EINVAL;
    if (ws_bytes < layout_of(s).total) return MPCD_EWORKSPACE;
    return MPCD_OK;
}

size_t esize(const mpcd_sys *s) { return s->prec == MPCD_F64 ? sizeof(double) : sizeof(float); }

bool ok_arr(const void *p, int64_t n, size_t elem)
{
    return n == 0 || (p != nullptr && aligned(p, elem));
}

int check_bodies(const mpcd_sys *s, const mpcd_bodies *b)
{
    if (s->n_bodies == 0 && s->n_sites == 0) return MPCD_OK;
    if (!b) return MPCD_EINVAL;
    const int64_t B = s->n_bodies, S = s->n_sites;
    if (!ok_arr(b->pos, B, 8) || !ok_arr(b->image, B, 4) || !ok_arr(b->quat, B, 8) ||
        !ok_arr(b->mom, B, 8) || !ok_arr(b->angmom, B, 8) || !ok_arr(b->force, B, 8) ||
        !ok_arr(b->torque, B, 8) || !ok_arr(b->mass, B, 8) || !ok_arr(b->inertia, B, 8) ||
        !ok_arr(b->site_off, B + 1, 8) || !ok_arr(b->site_body, S, 4) || !ok_arr(b->site_d, S, 8) ||
        !ok_arr(b->site_m, S, 8))
        return MPCD_EINVAL;
    return MPCD_OK;
}

#define TRY(x)                         \
    do {                               \
        int _rc = (x);                 \
        if (_rc != MPCD_OK) return _rc; \
    } while (0)

}  // namespace

// ===========================================================================
// C ABI

extern "C" {

size_t mpcd_workspace_bytes(const mpcd_sys *sys)
{
    if (check_sizes(sys) != MPCD_OK) return 0;
    return layout_of(sys).total;
}

int mpcd_last_hip_error(void) { return g_last_hip; }

int mpcd_workspace_offsets(const mpcd_sys *sys, int64_t out[8])
{
    TRY(check_sizes(sys));
    if (!out) return MPCD_EINVAL;
    const Layout L = layout_of(sys);
    out[0] = (int64_t)L.status;
    out[1] = (int64_t)L.shift;
    out[2] = (int64_t)L.cell_start;
    out[3] = (int64_t)L.perm;
    out[4] = (int64_t)L.cellid;
    out[5] = (int64_t)L.slot;
    out[6] = (int64_t)L.site_d;
    out[7] = (int64_t)L.vpre;
    return MPCD_OK;
}

int mpcd_ws_init(void *stream, const mpcd_sys *sys, void *ws, size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    const Layout L = layout_of(sys);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, at<uint32_t>(ws, L.status), (int64_t)64, 0u);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(sys->n_cells, 256)), dim3(256), 0, st,
                       at<int32_t>(ws, L.counts), sys->n_cells, 0);
    return launch_check();
}

int mpcd_stream(void *stream, const mpcd_sys *sys, void *x, const void *v, double dt, void *ws,
                size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    if (!ok_arr(x, sys->n_solvent, esize(sys)) || !ok_arr(v, sys->n_solvent, esize(sys)) || !(dt > 0.0))
        return MPCD_EINVAL;
    if (sys->n_solvent == 0) return MPCD_OK;
    const Layout L = layout_of(sys);
    const SysDev sd = make_sysdev(sys);
    hipStream_t st = (hipStream_t)stream;
    const unsigned g = grid_for(sys->n_solvent, 256);
    if (sys->prec == MPCD_F64)
        hipLaunchKernelGGL(k_stream<double>, dim3(g), dim3(256), 0, st, sd, (double *)x, (const double *)v, dt,
                           at<uint32_t>(ws, L.status));
    else
        hipLaunchKernelGGL(k_stream<float>, dim3(g), dim3(256), 0, st, sd, (float *)x, (const float *)v, dt,
                           at<uint32_t>(ws, L.status));
    return launch_check();
}

int mpcd_bin(void *stream, const mpcd_sys *sys, const void *x, const void *xs, const mpcd_bodies *bodies,
             uint64_t seed, const uint64_t *d_step, void *ws, size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    if (!ok_arr(x, sys->n_solvent, esize(sys)) || !ok_arr(xs, sys->n_sites, esize(sys)) || !d_step)
        return MPCD_EINVAL;
    if (sys->n_sites > 0 && (!bodies || !bodies->site_body)) return MPCD_EINVAL;
    const Layout L = layout_of(sys);
    const SysDev sd = make_sysdev(sys);
    hipStream_t st = (hipStream_t)stream;
    const int64_t NT = sys->n_solvent + sys->n_sites, C = sys->n_cells;
    const int64_t nb = (C + SCAN_TILE - 1) / SCAN_TILE;
    double *shift = at<double>(ws, L.shift);
    int32_t *counts = at<int32_t>(ws, L.counts), *cs = at<int32_t>(ws, L.cell_start);
    int32_t *cellid = at<int32_t>(ws, L.cellid), *slot = at<int32_t>(ws, L.slot), *perm = at<int32_t>(ws, L.perm);
    int32_t *partial = at<int32_t>(ws, L.partial);
    uint32_t *status = at<uint32_t>(ws, L.status);
    const int32_t *site_body = bodies ? bodies->site_body : nullptr;

    hipLaunchKernelGGL(k_shift, dim3(grid_for(sys->nsys, 64)), dim3(64), 0, st, sd, seed, d_step, shift);
    if (NT > 0) {
        const unsigned g = grid_for(NT, 256);
        if (sys->prec == MPCD_F64)
            hipLaunchKernelGGL(k_bin_count<double>, dim3(g), dim3(256), 0, st, sd, (const double *)x,
                               (const double *)xs, site_body, shift, counts, cellid, slot, status);
        else
            hipLaunchKernelGGL(k_bin_count<float>, dim3(g), dim3(256), 0, st, sd, (const float *)x,
                               (const float *)xs, site_body, shift, counts, cellid, slot, status);
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_T), 0, st, counts, C, partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_T), 0, st, partial, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SCAN_T), 0, st, counts, C, partial, cs, (int32_t)NT);
    if (NT > 0)
        hipLaunchKernelGGL(k_bin_scatter, dim3(grid_for(NT, 256)), dim3(256), 0, st, NT, cellid, slot, cs, perm);
    return launch_check();
}

int mpcd_collide(void *stream, const mpcd_sys *sys, void *v, const int32_t *tag, void *vs,
                 const mpcd_bodies *bodies, double cos_a, double sin_a, double kT_cell, uint64_t seed,
                 const uint64_t *d_step, void *ws, size_t ws_bytes, void *x_stream, double dt)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    if (!ok_arr(v, sys->n_solvent, esize(sys)) || !ok_arr(vs, sys->n_sites, esize(sys)) || !d_step)
        return MPCD_EINVAL;
    if (tag && !aligned(tag, 4)) return MPCD_EINVAL;
    if (sys->n_sites > 0 && (!bodies || !bodies->site_m)) return MPCD_EINVAL;
    if (x_stream && (!aligned(x_stream, esize(sys)) || !(dt > 0.0))) return MPCD_EINVAL;
    const Layout L = layout_of(sys);
    CollideArgs A;
    A.s = make_sysdev(sys);
    A.site_m = bodies ? bodies->site_m : nullptr;
    A.tag = tag;
    A.cell_start = at<int32_t>(ws, L.cell_start);
    A.perm = at<int32_t>(ws, L.perm);
    A.cos_a = cos_a;
    A.sin_a = sin_a;
    A.kT_cell = kT_cell;
    A.dt = dt;
    A.seed = seed;
    A.d_step = d_step;
    A.status = at<uint32_t>(ws, L.status);
    hipStream_t st = (hipStream_t)stream;
    const unsigned g = (unsigned)((sys->n_cells + COL_T - 1) / COL_T);
    if (sys->prec == MPCD_F64)
        hipLaunchKernelGGL(k_collide_f64, dim3(g), dim3(COL_T), 0, st, A, (double *)v, (double *)vs,
                           (double *)x_stream);
    else
        hipLaunchKernelGGL(k_collide_f32, dim3(g), dim3(COL_T), 0, st, A, (float *)v, (float *)vs,
                           (float *)x_stream);
    return launch_check();
}

int sites_thermalize(void *stream, const mpcd_sys *sys, const mpcd_bodies *bodies, double kT,
                     int32_t thermalize, uint64_t seed, const uint64_t *d_step, void *xs, void *vs, void *ws,
                     size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    TRY(check_bodies(sys, bodies));
    if (!ok_arr(xs, sys->n_sites, esize(sys)) || !ok_arr(vs, sys->n_sites, esize(sys)) || !d_step)
        return MPCD_EINVAL;
    if (thermalize && !(kT > 0.0)) return MPCD_EINVAL;
    if (sys->n_bodies == 0) return MPCD_OK;
    const Layout L = layout_of(sys);
    const SysDev sd = make_sysdev(sys);
    const BodyDev bd = make_bodydev(bodies);
    hipStream_t st = (hipStream_t)stream;
    const dim3 g((unsigned)sys->n_bodies);
    if (sys->prec == MPCD_F64)
        hipLaunchKernelGGL(k_sites_thermalize<double>, g, dim3(BODY_T), 0, st, sd, bd, kT, (int)thermalize, seed,
                           d_step, (double *)xs, (double *)vs, at<double>(ws, L.site_d), at<double>(ws, L.vpre),
                           at<uint32_t>(ws, L.status));
    else
        hipLaunchKernelGGL(k_sites_thermalize<float>, g, dim3(BODY_T), 0, st, sd, bd, kT, (int)thermalize, seed,
                           d_step, (float *)xs, (float *)vs, at<double>(ws, L.site_d), at<double>(ws, L.vpre),
                           at<uint32_t>(ws, L.status));
    return launch_check();
}

int sites_to_body(void *stream, const mpcd_sys *sys, const mpcd_bodies *bodies, const void *vs, void *ws,
                  size_t ws_bytes, double *J, double *K)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    TRY(check_bodies(sys, bodies));
    if (!ok_arr(vs, sys->n_sites, esize(sys)) || !ok_arr(J, sys->n_bodies, 8) || !ok_arr(K, sys->n_bodies, 8))
        return MPCD_EINVAL;
    if (sys->n_bodies == 0) return MPCD_OK;
    const Layout L = layout_of(sys);
    const SysDev sd = make_sysdev(sys);
    const BodyDev bd = make_bodydev(bodies);
    hipStream_t st = (hipStream_t)stream;
    const dim3 g((unsigned)sys->n_bodies);
    if (sys->prec == MPCD_F64)
        hipLaunchKernelGGL(k_sites_to_body<double>, g, dim3(BODY_T), 0, st, sd, bd, (const double *)vs,
                           at<double>(ws, L.site_d), at<double>(ws, L.vpre), J, K);
    else
        hipLaunchKernelGGL(k_sites_to_body<float>, g, dim3(BODY_T), 0, st, sd, bd, (const float *)vs,
                           at<double>(ws, L.site_d), at<double>(ws, L.vpre), J, K);
    return launch_check();
}

int body_forces(void *stream, const mpcd_sys *sys, const mpcd_bodies *bodies, const mpcd_wca *wca, void *ws,
                size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    TRY(check_bodies(sys, bodies));
    if (!wca || (wca->mode != 0 && wca->mode != 1)) return MPCD_EINVAL;
    if (wca->mode == 1 && !(wca->sigma > 0.0 && wca->eps >= 0.0 && wca->delta >= 0.0)) return MPCD_EINVAL;
    if (sys->n_bodies == 0) return MPCD_OK;
    const Layout L = layout_of(sys);
    hipLaunchKernelGGL(k_body_forces, dim3(grid_for(sys->n_bodies, 64)), dim3(64), 0, (hipStream_t)stream,
                       make_sysdev(sys), make_bodydev(bodies), *wca, at<uint32_t>(ws, L.status));
    return launch_check();
}

int body_integrate(void *stream, const mpcd_sys *sys, const mpcd_bodies *bodies, const double *J,
                   const double *K, const mpcd_wca *wca, double dt, void *ws, size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    TRY(check_bodies(sys, bodies));
    if (!(dt > 0.0) || !wca || (wca->mode != 0 && wca->mode != 1)) return MPCD_EINVAL;
    if ((J && !aligned(J, 8)) || (K && !aligned(K, 8))) return MPCD_EINVAL;
    if (sys->n_bodies == 0) return MPCD_OK;
    const Layout L = layout_of(sys);
    const SysDev sd = make_sysdev(sys);
    const BodyDev bd = make_bodydev(bodies);
    hipStream_t st = (hipStream_t)stream;
    const unsigned g = grid_for(sys->n_bodies, 64);
    uint32_t *status = at<uint32_t>(ws, L.status);
    hipLaunchKernelGGL(k_body_first, dim3(g), dim3(64), 0, st, sd, bd, J, K, dt, status);
    TRY(launch_check());
    TRY(body_forces(stream, sys, bodies, wca, ws, ws_bytes));
    hipLaunchKernelGGL(k_body_second, dim3(g), dim3(64), 0, st, sd, bd, dt, status);
    return launch_check();
}

int mpcd_advance_step(void *stream, uint64_t *d_step)
{
    if (!d_step || !aligned(d_step, 8)) return MPCD_EINVAL;
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, (hipStream_t)stream, d_step);
    return launch_check();
}

int mpcd_step(void *stream, const mpcd_step_args *a)
{
    if (!a || !a->sys) return MPCD_EINVAL;
    const mpcd_sys *s = a->sys;
    const mpcd_params &p = a->par;
    TRY(sites_thermalize(stream, s, &a->bodies, p.kT, p.thermalize, p.seed, a->d_step, a->xs, a->vs, a->ws,
                         a->ws_bytes));
    TRY(mpcd_bin(stream, s, a->x, a->xs, &a->bodies, p.seed, a->d_step, a->ws, a->ws_bytes));
    TRY(mpcd_collide(stream, s, a->v, a->tag, a->vs, &a->bodies, p.cos_a, p.sin_a, p.kT_cell, p.seed,
                     a->d_step, a->ws, a->ws_bytes, p.fuse_stream ? a->x : nullptr, p.dt));
    TRY(sites_to_body(stream, s, &a->bodies, a->vs, a->ws, a->ws_bytes, a->J, a->K));
    if (!p.fuse_stream) TRY(mpcd_stream(stream, s, a->x, a->v, p.dt, a->ws, a->ws_bytes));
    TRY(body_integrate(stream, s, &a->bodies, a->J, a->K, &p.wca, p.dt, a->ws, a->ws_bytes));
    return mpcd_advance_step(stream, a->d_step);
}

int mpcd_graph_create(void *stream, const mpcd_step_args *args, int32_t nsteps, void **graph_exec)
{
    if (!stream || !args || nsteps < 1 || !graph_exec) return MPCD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    TRY(hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)));
    int rc = MPCD_OK;
    for (int i = 0; i < nsteps && rc == MPCD_OK; ++i) rc = mpcd_step(stream, args);
    hipGraph_t graph = nullptr;
    const int rc_end = hip_check(hipStreamEndCapture(st, &graph));
    if (rc != MPCD_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    TRY(rc_end);
    hipGraphExec_t exec = nullptr;
    rc = hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    TRY(rc);
    *graph_exec = (void *)exec;
    return MPCD_OK;
}

int mpcd_graph_launch(void *stream, void *graph_exec)
{
    if (!graph_exec) return MPCD_EINVAL;
    return hip_check(hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream));
}

int mpcd_graph_destroy(void *graph_exec)
{
    if (!graph_exec) return MPCD_EINVAL;
    return hip_check(hipGraphExecDestroy((hipGraphExec_t)graph_exec));
}

int mpcd_status(void *stream, const void *ws, size_t ws_bytes, uint32_t *flags)
{
    if (!ws || !flags || ws_bytes < 256) return MPCD_EINVAL;
    uint32_t h = 0;
    TRY(hip_check(hipMemcpyAsync(&h, ws, sizeof h, hipMemcpyDeviceToHost, (hipStream_t)stream)));
    TRY(hip_check(hipStreamSynchronize((hipStream_t)stream)));
    *flags = h;
    return MPCD_OK;
}

}  // extern "C"
