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

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "../../include/mpcd.h"
#include "detrand.hpp"

using namespace mpcd;

namespace {

// ---------------------------------------------------------------------------
// Kernel-side views of the C-ABI structs

struct SysDev {
    int32_t nsys;
    double a;
    double inv_a;  // 1/a when a is a power of two (x/a == x*inv_a exactly, in FP32 too), else 0
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
    int e = 0;
    const double f = frexp(s->a, &e);
    d.inv_a = (f == 0.5 && s->a > 0x1p-120 && s->a < 0x1p120) ? ldexp(1.0, 1 - e) : 0.0;
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
__device__ __forceinline__ int find_sys_in(const int64_t *off, int lo, int hi, int64_t i)
{
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

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

// find_sys by a whole wave (all 64 lanes take part, each gets the result):
// each round the lanes probe 64 evenly spaced offsets of the remaining range,
// so 512 systems take two dependent loads instead of nine.
__device__ __forceinline__ int find_sys_wave(const int64_t *off, int nsys, int64_t i)
{
    const int lane = threadIdx.x & 63;
    int lo = 0, n = nsys;  // off[lo] <= i, and i < off[lo + n] when lo + n < nsys
    while (n > 1) {
        const int stride = (n + 63) >> 6;
        const int idx = lane * stride;
        const unsigned long long m = __ballot(idx < n && off[lo + idx] <= i);
        const int last = m ? 63 - __clzll(m) : 0;
        lo += last * stride;
        n = min(stride, n - last * stride);
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
// inv_a != 0: a is a power of two and g * inv_a is the same correctly rounded
// quotient as g / a (both round the exact value g 2^-k), without the division.
__device__ __forceinline__ int axis_cell(double x, double s, double a, double inv_a, int n, uint32_t &st)
{
    const double g = x - s;
    const double jf = floor(inv_a != 0.0 ? g * inv_a : g / a);
    if (!(jf >= -1.0 && jf <= (double)n)) {
        st |= (g != g) ? ST_NONFINITE : ST_ESCAPE;
        return 0;
    }
    int j = (int)jf;
    if (j < 0) j += n;
    else if (j >= n) j -= n;
    return j;
}

__device__ __forceinline__ int axis_cell(float x, double s, double a, double inv_a, int n, uint32_t &st)
{
    const float g = x - (float)s;
    const float jf = floorf(inv_a != 0.0 ? g * (float)inv_a : g / (float)a);
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

// Collision tiles: a block owns cpb consecutive cells (a power of two, at
// most one per thread), sized so that a tile holds on average at most a
// fraction `fill` of the block's LDS member capacity (TILE_T * items).  The
// items per thread and the fill are launch-shape choices (mpcd_tune); they
// change the split of work, never the results.
constexpr int TILE_T = 256;
constexpr int ITEMS_F64 = 2, ITEMS_F32 = 4;  // defaults

struct TileCfg {
    int items, cpb, cpb_shift, cap, ntiles;
};

static bool tune_ok(const mpcd_tune &tu, bool f64)
{
    const int it = tu.tile_items;
    const bool items_ok = it == 0 || (f64 ? (it == 1 || it == 2 || it == 4) : (it == 2 || it == 4 || it == 8));
    return items_ok && (tu.tile_fill == 0 || (tu.tile_fill >= 10 && tu.tile_fill <= 100)) &&
           tu.draw_cells >= 0 && tu.draw_cells <= 16 && (tu.draws_inline == 0 || tu.draws_inline == 1) &&
           (tu.overlap >= 0 && tu.overlap <= 3);
}

TileCfg tile_config(const mpcd_sys *s, const mpcd_tune &tu)
{
    TileCfg T;
    const bool f64 = s->prec == MPCD_F64;
    T.items = tu.tile_items ? tu.tile_items : (f64 ? ITEMS_F64 : ITEMS_F32);
    T.cap = TILE_T * T.items;
    const double fill = (tu.tile_fill ? tu.tile_fill : 70) / 100.0;
    const double per_cell = (double)(s->n_solvent + s->n_sites) / (double)s->n_cells;
    int cpb = TILE_T, sh = 8;
    while (cpb > 8 && (double)cpb * per_cell > fill * T.cap) {
        cpb >>= 1;
        --sh;
    }
    T.cpb = cpb;
    T.cpb_shift = sh;
    T.ntiles = (int)((s->n_cells + cpb - 1) / cpb);
    return T;
}

struct Layout {
    size_t status, shift, counts, partial, cell_start, site_start, cellid, slot, perm, draws, site_d, vpre, rtmp,
        grid_count, grid_body, wpos, woff, step_next, scan_ctl, scan_d0, scan_d1, rn_hist, rn_bcnt, rn_ctl, rn_key,
        rn_id, rn_k, total;
    uint32_t grid_mask;
};

// Scan blocks of SCAN_T threads, each thread SCAN_V counters (4 up to
// SCAN_BIG_C cells, else 16: fewer tiles, fewer tickets on one address);
// SCAN_TILE, the smaller tile, sizes the per-tile arrays.
constexpr int SCAN_T = 1024, SCAN_V = 4, SCAN_TILE = SCAN_T * SCAN_V;
constexpr int64_t SCAN_BIG_C = 1 << 19;
constexpr int scan_v(int64_t C) { return C > SCAN_BIG_C ? 16 : 4; }

// Slots per bucket of the body-centre grid: at one or two bodies per cell on
// average a bucket of 32 practically never overflows (a body whose 27
// neighbouring buckets include a full one takes the all-pairs loop).
constexpr int GRID_K = 32;

// Reverse nonequilibrium exchange: key histogram bins over [0, RN_KMAX) (the
// last bin also takes larger keys), candidate capacity per slab, pair limit.
constexpr int RN_BINS = 4096, RN_CAP = 2048, RN_MAXPAIRS = 1024;
constexpr int RN_HBLOCKS = 1024;  // blocks of the histogram pass (grid-stride)
constexpr double RN_KMAX = 0.4096;

// Binning and reorder chunks: BIN_T threads x BIN_ITEMS entries per block.
constexpr int BIN_T = 256, BIN_ITEMS = 4, BIN_CHUNK = BIN_T * BIN_ITEMS;
// Binning of the step's first kernel and of mpcd_bin: PREP_ITEMS per thread.
constexpr int PREP_ITEMS = 8, PREP_CHUNK = BIN_T * PREP_ITEMS;

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
    const int64_t nbc = (s->n_cells + SCAN_TILE - 1) / SCAN_TILE, nbp = (NT + BIN_CHUNK - 1) / BIN_CHUNK;
    const int64_t nb = nbc > nbp ? nbc : nbp;
    L.status = take(256);
    L.shift = take(sizeof(double) * 3 * (size_t)s->nsys);
    L.counts = take(sizeof(uint64_t) * (size_t)s->n_cells);  // packed: solvent (low 32 bits), sites (high)
    L.partial = take(sizeof(uint64_t) * (size_t)(nb + 1));
    L.cell_start = take(sizeof(int32_t) * (size_t)(s->n_cells + 1));
    L.site_start = take(sizeof(int32_t) * (size_t)(s->n_cells + 1));
    L.cellid = take(sizeof(int32_t) * (size_t)NT);
    L.slot = take(sizeof(int32_t) * (size_t)NT);
    L.perm = take(sizeof(int32_t) * (size_t)NT);
    L.draws = take(sizeof(double) * 4 * (size_t)s->n_cells);
    L.site_d = take(sizeof(double) * 3 * (size_t)s->n_sites);
    L.vpre = take(sizeof(double) * 3 * (size_t)s->n_sites);
    // reorder staging: positions and velocities (prec) and tags of the solvent
    const size_t es = s->prec == MPCD_F64 ? sizeof(double) : sizeof(float);
    L.rtmp = take(6 * es * (size_t)s->n_solvent + sizeof(int32_t) * (size_t)s->n_solvent);
    // hashed grid of body centres for the WCA neighbour search: a power of two
    // >= 4 B buckets of GRID_K slots
    uint64_t G = 64;
    while (G < 4 * (uint64_t)s->n_bodies) G <<= 1;
    L.grid_mask = (uint32_t)(G - 1);
    L.grid_count = take(sizeof(int32_t) * (size_t)G);
    L.grid_body = take(sizeof(int32_t) * (size_t)G * GRID_K);
    // site frames for the site-site WCA (offsets and unwrapped positions)
    L.wpos = take(sizeof(double) * 3 * (size_t)s->n_sites);
    L.woff = take(sizeof(double) * 3 * (size_t)s->n_sites);
    // the next step's index, stored by the collision for a binning of the next
    // step that runs beside this step's body update
    L.step_next = take(sizeof(uint64_t));
    // single-pass scan: tile ticket counter and two descriptor words per tile
    L.scan_ctl = take(sizeof(uint64_t));
    L.scan_d0 = take(sizeof(uint64_t) * (size_t)nbc);
    L.scan_d1 = take(sizeof(uint64_t) * (size_t)nbc);
    // reverse nonequilibrium exchange: key histograms, control words and
    // candidate lists of the two slabs
    L.rn_hist = take(sizeof(int32_t) * 2 * RN_BINS);
    L.rn_bcnt = take(sizeof(int32_t) * 2 * RN_HBLOCKS);
    L.rn_ctl = take(sizeof(int32_t) * 16);
    L.rn_key = take(sizeof(double) * 2 * RN_CAP);
    L.rn_id = take(sizeof(int32_t) * 2 * RN_CAP);
    L.rn_k = take(sizeof(int32_t) * 2 * RN_CAP);
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

// Constant solvent acceleration g over one streaming interval (forced flow,
// Sec. III.B): x + v dt + h with h = (dt / 2)(g dt), then v + g dt.
struct Forcing {
    double gdt[3], h[3];
    int on;
};

Forcing make_forcing(const double *g, double dt)
{
    Forcing F;
    F.on = g && (g[0] != 0.0 || g[1] != 0.0 || g[2] != 0.0);
    for (int k = 0; k < 3; ++k) {
        F.gdt[k] = F.on ? g[k] * dt : 0.0;
        F.h[k] = (0.5 * dt) * F.gdt[k];
    }
    return F;
}

// A constant force at every body centre (no torque).
struct ExtForce {
    double f[3];
    int on;
};

ExtForce make_ext(const double *f)
{
    ExtForce E;
    E.on = f && (f[0] != 0.0 || f[1] != 0.0 || f[2] != 0.0);
    for (int k = 0; k < 3; ++k) E.f[k] = E.on ? f[k] : 0.0;
    return E;
}

template <typename Real>
__global__ void k_stream(SysDev s, Real *x, Real *v, double dt, Forcing F, uint32_t *status)
{
    uint32_t st = 0;
    const Real dtr = (Real)dt;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int r = find_sys(s.solv_off, s.nsys, i);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const Real L = (Real)((double)s.ncell[3 * r + k] * s.a);
            Real y = x[k * s.N + i] + v[k * s.N + i] * dtr;
            if (F.on) {
                y = y + (Real)F.h[k];
                v[k * s.N + i] = v[k * s.N + i] + (Real)F.gdt[k];
            }
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

// Blocks are remapped so that each of the 8 XCDs (own L2 each) works on a
// contiguous range of tiles/chunks.
constexpr int NXCD = 8;

__device__ __forceinline__ int tile_of_block(int ntiles)
{
    const int per = (ntiles + NXCD - 1) / NXCD;
    return (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
}

inline unsigned xcd_grid(int64_t ntiles)
{
    const int64_t per = (ntiles + NXCD - 1) / NXCD;
    return (unsigned)(per * NXCD);
}

// Binning: atomic counting sort by cell.
//  1. k_bin_count (and the solvent blocks of k_prep): cell of every particle
//     and its slot in the cell.  A block covers PREP_CHUNK consecutive
//     particles, counts them per cell in an LDS hash table and takes one
//     device-scope atomic per distinct cell (bin_chunk); with storage in
//     brick order that is about 0.3 atomics per particle.  The sites of a
//     body take one atomic per run of equal cells within a wave (run_slots).
//     A cell's counter is 64 bits: solvent particles take slots from the low
//     32 bits and sites from the high 32 bits, so one scan yields both.
//  2. k_scan: single-pass exclusive scan of the packed counters ->
//     cell_start (all members) and site_start (sites in earlier cells); each
//     block takes the earlier tiles' prefix by look-back and clears the
//     counters.
//  3. k_bin_scatter: perm[cell_start[cell] + slot] = particle, solvent first
//     within each cell, then its sites.  A solvent particle at permutation
//     position p of cell c is therefore solvent number p - site_start[c] in
//     cell order, the position the out-of-place collision writes it to.

// Grid shift of system r at a step: a pure function of (seed, step, replica).
__device__ __forceinline__ void shift_of(const SysDev &s, uint64_t seed, uint64_t step, int r, double sh[3])
{
    const Words w = rng_draw(seed, RNG_SHIFT, step, 0, s.replica0 + (uint64_t)r, 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) sh[k] = shift_component(w.w[k], s.a);
}

// Shifts for a block: taken from `arr` when given; otherwise lane 0 draws the
// shifts of systems ra and rb into LDS, and a particle of any other system
// (a chunk spanning three or more systems) draws its own.
struct BlockShift {
    const double *arr;
    const double *lds;  // [2][3]
    const int *sys;     // [2]: ra, rb in LDS, or nullptr (systems unknown)
    uint64_t seed, step;
    __device__ int ra() const { return sys ? sys[0] : -1; }
    __device__ int rb() const { return sys ? sys[1] : -1; }
    __device__ void get(const SysDev &s, int r, double sh[3]) const
    {
        if (arr) { sh[0] = arr[3 * r]; sh[1] = arr[3 * r + 1]; sh[2] = arr[3 * r + 2]; }
        else if (r == sys[0]) { sh[0] = lds[0]; sh[1] = lds[1]; sh[2] = lds[2]; }
        else if (r == sys[1]) { sh[0] = lds[3]; sh[1] = lds[4]; sh[2] = lds[5]; }
        else shift_of(s, seed, step, r, sh);
    }
};

// Storage order of a system's cells (the order of the cell lists and of the
// out-of-place solvent): bricks of BRX x BRY x BRZ cells, narrower at the far
// faces when the box is not a multiple, the bricks x-fastest and the cells of
// a brick x-fastest.  Consecutive cells are then a compact region, so the
// particles of a run of storage land in few cells of the next grid and the
// binning aggregates their counts per block.  The canonical index
// (jz n_y + j_y) n_x + j_x keys the random streams.
constexpr int BRX = 8, BRY = 8, BRZ = 4;

__host__ __device__ __forceinline__ int32_t brick_index(int nx, int ny, int nz, int jx, int jy, int jz)
{
    const int bz = jz / BRZ, lz = jz - bz * BRZ, ez = min(BRZ, nz - bz * BRZ);
    const int by = jy / BRY, ly = jy - by * BRY, ey = min(BRY, ny - by * BRY);
    const int bx = jx / BRX, lx = jx - bx * BRX, ex = min(BRX, nx - bx * BRX);
    return bz * BRZ * ny * nx + ez * (by * BRY) * nx + ez * ey * (bx * BRX) + (lz * ey + ly) * ex + lx;
}

// Inverse of brick_index: the canonical local index of storage position q.
__host__ __device__ __forceinline__ int32_t brick_canonical(int nx, int ny, int nz, int32_t q)
{
    const uint32_t slab = (uint32_t)(BRZ * ny * nx);
    const int bz = (int)((uint32_t)q / slab);
    uint32_t rem = (uint32_t)q - (uint32_t)bz * slab;
    const int ez = min(BRZ, nz - bz * BRZ);
    const uint32_t row = (uint32_t)(ez * BRY * nx);
    const int by = (int)(rem / row);
    rem -= (uint32_t)by * row;
    const int ey = min(BRY, ny - by * BRY);
    const uint32_t brick = (uint32_t)(ez * ey * BRX);
    const int bx = (int)(rem / brick);
    rem -= (uint32_t)bx * brick;
    const int ex = min(BRX, nx - bx * BRX);
    const int lz = (int)(rem / (uint32_t)(ey * ex));
    rem -= (uint32_t)(lz * ey * ex);
    const int ly = (int)(rem / (uint32_t)ex);
    const int lx = (int)(rem - (uint32_t)(ly * ex));
    return ((bz * BRZ + lz) * ny + (by * BRY + ly)) * nx + (bx * BRX + lx);
}

template <typename Real>
__device__ __forceinline__ int32_t cell_of_pos(const SysDev &s, int r, Real p0, Real p1, Real p2, const double sh[3],
                                               uint32_t &st)
{
    const int nx = s.ncell[3 * r], ny = s.ncell[3 * r + 1], nz = s.ncell[3 * r + 2];
    const int jx = axis_cell(p0, sh[0], s.a, s.inv_a, nx, st);
    const int jy = axis_cell(p1, sh[1], s.a, s.inv_a, ny, st);
    const int jz = axis_cell(p2, sh[2], s.a, s.inv_a, nz, st);
    return (int32_t)(s.cell_off[r] + brick_index(nx, ny, nz, jx, jy, jz));
}

// Slots for one group of 64 lanes: one atomic per run of equal cells.
// A run is a stretch of lanes with the same cell and kind (solvent or site).
__device__ __forceinline__ void run_slots(int32_t gc, bool site, unsigned long long *counts, int &hl, int &base)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const int32_t key = (site && gc >= 0) ? (int32_t)((uint32_t)gc | 0x80000000u) : gc;
    const int32_t prev = __shfl_up(key, 1, 64);
    const bool head = (lane == 0) || (prev != key);
    const unsigned long long heads = __ballot(head);
    hl = 63 - __clzll(heads & le);
    const unsigned long long above = heads & ~le;
    const int nh = above ? (__ffsll((long long)above) - 1) : 64;
    base = 0;
    if (head && gc >= 0) {
        const int sh = site ? 32 : 0;
        const unsigned long long old = atomicAdd(&counts[gc], (unsigned long long)(nh - hl) << sh);
        base = (int)((old >> sh) & 0xffffffffull);
    }
}

// One chunk of PREP_CHUNK particles starting at kbase (< k1).  The block counts
// its particles per (cell, kind) in an LDS hash table (each particle's rank
// among its key's particles), then takes one global atomic per distinct key
// for the key's base slot; slot = base + rank.  With cells in brick order a
// chunk is a compact region and lands in about a third as many cells as it
// has particles.
constexpr int BIN_HT_BITS = 12, BIN_HT = 1 << BIN_HT_BITS;  // hash slots: at most half full
static_assert(BIN_HT >= 2 * PREP_CHUNK, "hash load");
constexpr uint32_t BIN_EMPTY = 0xffffffffu;

struct BinLds {
    uint32_t key[BIN_HT];
    int32_t cnt[BIN_HT];  // particles per key, then the key's base slot
};

template <typename Real, bool SITES, typename PreBarrier>
__device__ void bin_chunk(const SysDev &s, const Real *x, const Real *xs, const int32_t *site_body,
                          const BlockShift &bs, unsigned long long *counts, int32_t *cellid, int32_t *slot,
                          int64_t kbase, int64_t k1, BinLds &H, uint32_t &st, PreBarrier pre_barrier)
{
    uint32_t *hkey = H.key;
    int32_t *hcnt = H.cnt;
    for (int i = threadIdx.x; i < BIN_HT; i += BIN_T) {
        hkey[i] = BIN_EMPTY;
        hcnt[i] = 0;
    }
    // positions first: their loads are in flight while the block draws its
    // grid shifts (pre_barrier) and until the barrier
    Real p[PREP_ITEMS][3];
#pragma unroll
    for (int j = 0; j < PREP_ITEMS; ++j) {
        const int64_t k = kbase + (int64_t)j * BIN_T + threadIdx.x;
        p[j][0] = p[j][1] = p[j][2] = (Real)0;
        if (k < k1) {
            if (!SITES || k < s.N) {
                p[j][0] = x[k]; p[j][1] = x[s.N + k]; p[j][2] = x[2 * s.N + k];
            } else {
                const int64_t q = k - s.N;
                p[j][0] = xs[q]; p[j][1] = xs[s.S + q]; p[j][2] = xs[2 * s.S + q];
            }
        }
    }
    pre_barrier();
    __syncthreads();  // hash table cleared; the block's shifts and systems in LDS
    const int ra = bs.ra(), rb = bs.rb();
    int32_t gc[PREP_ITEMS];
#pragma unroll
    for (int j = 0; j < PREP_ITEMS; ++j) {
        const int64_t k = kbase + (int64_t)j * BIN_T + threadIdx.x;
        gc[j] = -1;
        if (k < k1) {
            int r;
            if (!SITES || k < s.N)  // the chunk's first and last systems, when known, bound the search
                r = ra < 0 ? find_sys(s.solv_off, s.nsys, k) : (ra == rb ? ra : find_sys_in(s.solv_off, ra, rb, k));
            else
                r = find_sys(s.body_off, s.nsys, (int64_t)site_body[k - s.N]);
            double sh[3];
            bs.get(s, r, sh);
            gc[j] = cell_of_pos<Real>(s, r, p[j][0], p[j][1], p[j][2], sh, st);
        }
    }
    int hs[PREP_ITEMS], rank[PREP_ITEMS];
#pragma unroll
    for (int j = 0; j < PREP_ITEMS; ++j) {
        hs[j] = 0;
        rank[j] = 0;
        if (gc[j] < 0) continue;
        const bool site = SITES && (kbase + (int64_t)j * BIN_T + threadIdx.x) >= s.N;
        const uint32_t key = (uint32_t)gc[j] | (site ? 0x80000000u : 0u);
        uint32_t h = (key * 2654435761u) >> (32 - BIN_HT_BITS);
        while (true) {  // ends: fewer distinct keys than slots
            const uint32_t old = atomicCAS(&hkey[h], BIN_EMPTY, key);
            if (old == BIN_EMPTY || old == key) break;
            h = (h + 1) & (BIN_HT - 1);
        }
        hs[j] = (int)h;
        rank[j] = atomicAdd(&hcnt[h], 1);
    }
    __syncthreads();
    // one device atomic per distinct key; unrolled with the returned bases in
    // registers, so a lane's atomics are all in flight before it waits
    constexpr int HT_PER_T = BIN_HT / BIN_T;
    static_assert(BIN_HT % BIN_T == 0, "hash slots per thread");
    unsigned long long old[HT_PER_T];
    uint32_t keys[HT_PER_T];
#pragma unroll
    for (int it = 0; it < HT_PER_T; ++it) {
        const int i = threadIdx.x + it * BIN_T;
        keys[it] = hkey[i];
        old[it] = 0ull;
        if (keys[it] != BIN_EMPTY) {
            const int sh = (keys[it] & 0x80000000u) ? 32 : 0;
            old[it] = atomicAdd(&counts[keys[it] & 0x7fffffffu], (unsigned long long)hcnt[i] << sh);
        }
    }
#pragma unroll
    for (int it = 0; it < HT_PER_T; ++it) {
        if (keys[it] == BIN_EMPTY) continue;
        const int sh = (keys[it] & 0x80000000u) ? 32 : 0;
        hcnt[threadIdx.x + it * BIN_T] = (int)((old[it] >> sh) & 0xffffffffull);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PREP_ITEMS; ++j) {
        const int64_t k = kbase + (int64_t)j * BIN_T + threadIdx.x;
        if (k < k1) {
            slot[k] = hcnt[hs[j]] + rank[j];
            cellid[k] = gc[j];
        }
    }
}

template <typename Real>
__global__ __launch_bounds__(BIN_T) void k_bin_count(SysDev s, const Real *x, const Real *xs,
                                                     const int32_t *site_body, const double *shift,
                                                     unsigned long long *counts, int32_t *cellid, int32_t *slot,
                                                     uint32_t *status, int64_t k0, int64_t k1)
{
    __shared__ BinLds H;
    uint32_t st = 0;
    BlockShift bs;
    bs.arr = shift; bs.lds = nullptr; bs.sys = nullptr; bs.seed = 0; bs.step = 0;
    bin_chunk<Real, true>(s, x, xs, site_body, bs, counts, cellid, slot, k0 + (int64_t)blockIdx.x * PREP_CHUNK, k1, H,
                          st, [] {});
    flag(status, st);
}

// Block-wide exclusive scan of one value per thread (blockDim = NTHR, wave64).
template <int NTHR = SCAN_T, typename T = int32_t>
__device__ __forceinline__ T block_exclusive_scan(T v, T *total)
{
    constexpr int NW = NTHR / 64;
    __shared__ T wsum[NW];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        T w = (lane < NW) ? wsum[lane] : (T)0;
        T wi = w;
#pragma unroll
        for (int d = 1; d < NW; d <<= 1) {
            const T y = __shfl_up(wi, d, 64);
            if (lane >= d) wi += y;
        }
        if (lane < NW) wsum[lane] = wi - w;
        if (lane == NW - 1) *total = wi;
    }
    __syncthreads();
    const T res = wsum[wid] + inc - v;
    __syncthreads();
    return res;
}

using u64 = unsigned long long;

// Single-pass exclusive scan of the packed cell counters (decoupled
// look-back, Merrill & Garland 2016) into cell_start (solvent + sites) and
// site_start (sites), clearing the counters for the next step.  Packed sums
// cannot carry from the low half into the high half: the solvent total is
// below 2^31.  A block takes its tile from a ticket counter, so every tile it
// waits for belongs to a block that started before it; each block publishes
// its tile's aggregate at once and its inclusive prefix when known.  A tile's
// descriptor is two 64-bit words, each a 32-bit flag (launch generation,
// ticket / tiles + 1, above a two-bit state) beside one 32-bit half of the
// value, written and read with relaxed device-scope atomics: a reader takes
// them only when both flags match the current generation and each other, so
// no fence (and no cache write-back or invalidation) is needed, flags of
// earlier launches read as not ready, and nothing is cleared between launches.
// Wave 0 looks back over 64 earlier tiles at a time.  The waits end because
// the tiles waited for publish without waiting; a spin limit turns a stall
// into ST_BINERR instead of a hang.
struct ScanWs {
    u64 *ctl, *d0, *d1;
};
constexpr uint32_t SCAN_AGG = 1, SCAN_INCL = 2;
constexpr int SCAN_SPIN_LIMIT = 1 << 22;

__device__ __forceinline__ u64 load_relaxed(const u64 *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_relaxed(u64 *p, u64 v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void scan_publish(const ScanWs &W, int64_t j, uint32_t fl, u64 val)
{
    store_relaxed(&W.d0[j], ((u64)fl << 32) | (val & 0xffffffffull));
    store_relaxed(&W.d1[j], ((u64)fl << 32) | (val >> 32));
}

template <int V>
__global__ __launch_bounds__(SCAN_T) void k_scan(u64 *counts, int64_t C, int64_t ntiles, ScanWs W,
                                                 int32_t *cell_start, int32_t *site_start, int32_t total,
                                                 int32_t total_sites, uint32_t *status)
{
    __shared__ u64 s_ticket, tot, pre;
    if (threadIdx.x == 0) s_ticket = atomicAdd((unsigned long long *)W.ctl, 1ull);
    __syncthreads();
    const u64 ticket = s_ticket;
    const int64_t j = (int64_t)(ticket % (u64)ntiles);
    const uint32_t gen = (uint32_t)((ticket / (u64)ntiles + 1) & 0x3fffffffull);
    static_assert(V % 4 == 0, "vector loads and stores of a scan thread's counters");
    const int64_t base = j * (int64_t)(SCAN_T * V) + (int64_t)threadIdx.x * V;
    const bool full = base + V <= C;  // whole vectors (the arrays are 256-byte aligned)
    u64 c[V];
    u64 v = 0;
    if (full) {
        const ulonglong2 *src = (const ulonglong2 *)(counts + base);
#pragma unroll
        for (int i = 0; i < V / 2; ++i) {
            const ulonglong2 w = src[i];
            c[2 * i] = w.x;
            c[2 * i + 1] = w.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) c[i] = (base + i < C) ? counts[base + i] : 0ull;
    }
#pragma unroll
    for (int i = 0; i < V; ++i) v += c[i];
    u64 run = block_exclusive_scan<SCAN_T, u64>(v, &tot);
    const u64 agg = tot;
    uint32_t st = 0;
    if (threadIdx.x == 0) {
        scan_publish(W, j, (gen << 2) | (j == 0 ? SCAN_INCL : SCAN_AGG), agg);
        if (j == 0) pre = 0;
    }
    if (j > 0 && threadIdx.x < 64) {
        const int lane = threadIdx.x;
        u64 excl = 0;
        int64_t look = j - 1;
        int spins = 0;
        while (true) {
            const int64_t q = look - lane;  // lane 0: the nearest earlier tile
            uint32_t state = SCAN_INCL;     // before tile 0 there is nothing: an inclusive zero
            u64 val = 0;
            if (q >= 0) {
                const u64 w0 = load_relaxed(&W.d0[q]), w1 = load_relaxed(&W.d1[q]);
                const uint32_t f0 = (uint32_t)(w0 >> 32), f1 = (uint32_t)(w1 >> 32);
                state = (f0 == f1 && (f0 >> 2) == gen) ? (f0 & 3u) : 0u;
                val = (w0 & 0xffffffffull) | (w1 << 32);
            }
            const unsigned long long incl_mask = __ballot(state == SCAN_INCL);
            const int first = incl_mask ? __ffsll((long long)incl_mask) - 1 : 63;
            const unsigned long long upto = (first == 63) ? ~0ull : ((2ull << first) - 1ull);
            if (__ballot(state == 0u) & upto) {  // a tile this window needs has not published
                if (++spins > SCAN_SPIN_LIMIT) {
                    st |= ST_BINERR;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            if (lane > first) val = 0;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) val += __shfl_down(val, d, 64);
            excl += __shfl(val, 0, 64);
            if (incl_mask) break;
            look -= 64;
        }
        if (lane == 0) {
            scan_publish(W, j, (gen << 2) | SCAN_INCL, excl + agg);
            pre = excl;
        }
    }
    __syncthreads();
    run += pre;
    int32_t cs[V], ss[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const uint32_t ns = (uint32_t)(run & 0xffffffffull), nq = (uint32_t)(run >> 32);
        cs[i] = (int32_t)(ns + nq);
        ss[i] = (int32_t)nq;
        run += c[i];
    }
    if (full) {
        int4 *dc = (int4 *)(cell_start + base), *ds = (int4 *)(site_start + base);
        ulonglong2 *dz = (ulonglong2 *)(counts + base);
#pragma unroll
        for (int i = 0; i < V / 4; ++i) {
            dc[i] = make_int4(cs[4 * i], cs[4 * i + 1], cs[4 * i + 2], cs[4 * i + 3]);
            ds[i] = make_int4(ss[4 * i], ss[4 * i + 1], ss[4 * i + 2], ss[4 * i + 3]);
        }
#pragma unroll
        for (int i = 0; i < V / 2; ++i) dz[i] = make_ulonglong2(0ull, 0ull);
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) {
            if (base + i < C) {
                cell_start[base + i] = cs[i];
                site_start[base + i] = ss[i];
                counts[base + i] = 0;
            }
        }
    }
    if (j == 0 && threadIdx.x == 0) {
        cell_start[C] = total;
        site_start[C] = total_sites;
    }
    flag(status, st);
}

// The scatter of BIN_ITEMS entries per thread, k = kb + j BIN_T + t, each to
// its position in the permutation: its cell's start plus its slot, the
// solvent first and then the cell's sites.  Every entry's cell and slot loads
// are issued before the first dependent load (its cell's start), so a thread
// waits for two round trips, not two per entry.
__device__ __forceinline__ void scatter_items(int64_t kb, int64_t NT, int64_t N, const int32_t *cellid,
                                              const int32_t *slot, const int32_t *cell_start,
                                              const int32_t *site_start, int32_t *perm, uint32_t &st)
{
    int32_t gc[BIN_ITEMS], sl[BIN_ITEMS], b[BIN_ITEMS];
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j) {
        const int64_t k = kb + (int64_t)j * BIN_T + threadIdx.x;
        gc[j] = -1;
        sl[j] = 0;
        if (k < NT) {
            gc[j] = cellid[k];
            sl[j] = slot[k];
        }
    }
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j) b[j] = gc[j] >= 0 ? cell_start[gc[j]] : 0;
    // every position before the first store (a store would otherwise count
    // in the waits for the later entries' loads)
    int64_t pos[BIN_ITEMS];
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j) {
        const int64_t k = kb + (int64_t)j * BIN_T + threadIdx.x;
        pos[j] = -1;
        if (k >= NT) continue;
        if (gc[j] < 0) {  // only with a corrupted binning
            st |= ST_BINERR;
            continue;
        }
        pos[j] = (int64_t)b[j] + sl[j];
        if (k >= N)  // sites follow the cell's solvent
            pos[j] += (cell_start[gc[j] + 1] - b[j]) - (site_start[gc[j] + 1] - site_start[gc[j]]);
        if (pos[j] < 0 || pos[j] >= NT) {
            st |= ST_BINERR;
            pos[j] = -1;
        }
    }
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j)
        if (pos[j] >= 0) perm[pos[j]] = (int32_t)(kb + (int64_t)j * BIN_T + threadIdx.x);
}

// grid_count (when set): the body-centre grid, cleared here for the step's
// insertions when the step's first kernel did not run (fused schedule).
__global__ __launch_bounds__(BIN_T) void k_bin_scatter(int64_t NT, int64_t N, const int32_t *cellid,
                                                       const int32_t *slot, const int32_t *cell_start,
                                                       const int32_t *site_start, int32_t *perm, int32_t *grid_count,
                                                       int64_t grid_n, uint32_t *status)
{
    uint32_t st = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; grid_count && q < grid_n;
         q += (int64_t)gridDim.x * blockDim.x)
        grid_count[q] = 0;
    scatter_items((int64_t)blockIdx.x * BIN_CHUNK, NT, N, cellid, slot, cell_start, site_start, perm, st);
    flag(status, st);
}

// ---------------------------------------------------------------------------
// Storage reorder: solvent particles into the order of the last binning (cell
// order), carrying their identity tags.  Keeps gathers and atomics local as
// the solvent diffuses; identities keep the FP64 summation order unchanged.

// Solvent count per BIN_CHUNK entries of the permutation.
__global__ __launch_bounds__(BIN_T) void k_reorder_count(const int32_t *perm, int64_t NT, int64_t N, int32_t *partial)
{
    __shared__ int32_t tot;
    const int64_t base = (int64_t)blockIdx.x * BIN_CHUNK;
    int32_t v = 0;
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * BIN_T + threadIdx.x;
        if (i < NT && perm[i] < N) v += 1;
    }
    (void)block_exclusive_scan<BIN_T>(v, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One block: exclusive scan of nb partial sums in place.
__global__ __launch_bounds__(SCAN_T) void k_partials_scan(int32_t *partial, int64_t nb)
{
    __shared__ int32_t tot;
    int32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_T) {
        const int64_t i = b0 + threadIdx.x;
        const int32_t v = (i < nb) ? partial[i] : 0;
        const int32_t ex = block_exclusive_scan(v, &tot);
        if (i < nb) partial[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

// Gather the solvent in permutation order into the staging buffers.
template <typename Real>
__global__ __launch_bounds__(BIN_T) void k_reorder_gather(const int32_t *perm, int64_t NT, int64_t N,
                                                          const int32_t *partial, const Real *x, const Real *v,
                                                          const int32_t *tag, Real *tx, Real *tv, int32_t *ttag)
{
    __shared__ int32_t tot;
    const int64_t base = (int64_t)blockIdx.x * BIN_CHUNK + (int64_t)threadIdx.x * BIN_ITEMS;
    int32_t k[BIN_ITEMS];
    int32_t cnt = 0;
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j) {
        k[j] = (base + j < NT) ? perm[base + j] : -1;
        if (k[j] >= 0 && k[j] < N) cnt += 1;
    }
    int32_t dst = partial[blockIdx.x] + block_exclusive_scan<BIN_T>(cnt, &tot);
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j) {
        if (k[j] >= 0 && k[j] < N) {
            if (dst < N) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    tx[d * N + dst] = x[d * N + k[j]];
                    tv[d * N + dst] = v[d * N + k[j]];
                }
                ttag[dst] = tag[k[j]];
            }
            dst += 1;
        }
    }
}

template <typename Real>
__global__ void k_reorder_copy(int64_t N, Real *x, Real *v, int32_t *tag, const Real *tx, const Real *tv,
                               const int32_t *ttag)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[d * N + i] = tx[d * N + i];
            v[d * N + i] = tv[d * N + i];
        }
        tag[i] = ttag[i];
    }
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

struct CollideArgs {
    SysDev s;
    const double *site_m;
    const int32_t *tag;
    const int32_t *cell_start, *site_start, *perm;
    const double *draws; // [4][C]: random axis (3) and thermostat gamma variate of each cell
    double cos_a, sin_a, kT_cell, dt;
    uint64_t seed;
    const uint64_t *d_step;
    uint32_t *status;
    uint64_t *advance_step;  // when set, block 0 advances the step counter (graph schedule)
    uint64_t *step_next;     // when set, block 0 stores the step index + 1 there
    Forcing F;               // solvent acceleration applied by the fused streaming
    int inline_draws;        // 1: the collision draws each cell's axis and gamma itself
    // binning of the new solvent for the next step (kernels with BIN): packed
    // per-cell counters (solvent in the low 32 bits) and the cell and slot of
    // each new solvent particle
    unsigned long long *bin_counts;
    int32_t *bin_cellid, *bin_slot;
};

// Identity order key of particle k: solvent tag (or index), sites N_total + j.
__device__ __forceinline__ uint32_t ident(const CollideArgs &A, int32_t k)
{
    return (k < A.s.N && A.tag) ? (uint32_t)A.tag[k] : (uint32_t)k;
}

// Per-cell random draws: the collision axis and, with the thermostat, the
// Gamma(3(n-1)/2) variate for the cell's member count n, stored as
// draws[0..2][C] and draws[3][C] (cells with fewer than two members draw no
// gamma variate).  Both come from the cell's one stream (cell_draw).
//
// Lane g of nlanes takes cells g, g + nlanes, ...; each loop iteration makes
// one Philox call for the lane's current cell and moves on as soon as both
// draws are accepted, so the rejections of a wave share one loop.  Each cell
// uses calls 0, 1, ... of its stream in order, exactly as cell_draw does.
// One cell per lane measured best: the Philox call is a long dependent chain,
// and longer queues per lane leave too few waves to hide it.
struct DrawLane {
    int64_t cell;
    uint64_t cl, rep;
    int call;
    bool want_gamma;
    CellDraw D;
};

__device__ __forceinline__ void draw_lane_start(const CollideArgs &A, DrawLane &L, int r_lo, int r_hi)
{
    const SysDev &s = A.s;
    const int r = r_lo == r_hi ? r_lo : find_sys_in(s.cell_off, r_lo, r_hi, L.cell);
    L.cl = (uint64_t)brick_canonical(s.ncell[3 * r], s.ncell[3 * r + 1], s.ncell[3 * r + 2],
                                     (int32_t)(L.cell - s.cell_off[r]));
    L.rep = s.replica0 + (uint64_t)r;
    L.call = 0;
    const int n = A.cell_start[L.cell + 1] - A.cell_start[L.cell];
    L.want_gamma = A.kT_cell > 0.0 && n >= 2;
    cell_draw_begin(L.D, L.want_gamma, 0.5 * (double)(3 * (n - 1)));
}

__device__ void draw_cells(const CollideArgs &A, double *draws, int64_t g, int64_t nlanes, uint32_t &st)
{
    const int64_t C = A.s.C;
    const uint64_t step = *A.d_step;
    DrawLane L;
    L.cell = g;
    // the wave's first cells are consecutive: two wave-wide searches bound
    // their systems (every lane of the wave is here)
    const int64_t w0 = g - (threadIdx.x & 63);
    int r_lo = 0, r_hi = 0;
    if (w0 < C) {
        r_lo = find_sys_wave(A.s.cell_off, A.s.nsys, w0);
        r_hi = find_sys_wave(A.s.cell_off, A.s.nsys, (w0 + 63 < C) ? w0 + 63 : C - 1);
    }
    if (L.cell < C) draw_lane_start(A, L, r_lo, r_hi);
    while (L.cell < C) {
        bool done = cell_draw_call(L.D, rng_draw(A.seed, RNG_CELL, step, L.cl, L.rep, (uint64_t)L.call));
        L.call += 1;
        if (!done && L.call == RNG_MAX_CALLS) {
            st |= cell_draw_end(L.D);
            done = true;
        }
        if (done) {
            draws[L.cell] = L.D.n[0];
            draws[C + L.cell] = L.D.n[1];
            draws[2 * C + L.cell] = L.D.n[2];
            if (L.want_gamma) draws[3 * C + L.cell] = L.D.g;
            L.cell += nlanes;
            if (L.cell < C) draw_lane_start(A, L, 0, A.s.nsys - 1);
        }
    }
}

// Standalone per-cell draws (axis and gamma variate of every cell; the gamma
// variates need this step's cell counts).
constexpr int DRAW_CELLS_PER_LANE = 1;

__global__ __launch_bounds__(BIN_T) void k_cell_draws(CollideArgs A, double *draws)
{
    uint32_t st = 0;
    draw_cells(A, draws, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x, st);
    flag(A.status, st);
}

// Per-cell draws (blocks [0, ndraw)) fused with the scatter (the other
// blocks): independent work, one launch.  The draw blocks come first so their
// ALU work starts early and overlaps the scatter's memory traffic.
__global__ __launch_bounds__(BIN_T) void k_scatter_draws(int64_t NT, const int32_t *cellid, const int32_t *slot,
                                                         int32_t *perm, int ndraw, CollideArgs A, double *draws,
                                                         int32_t *grid_count, int64_t grid_n)
{
    uint32_t st = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; grid_count && q < grid_n;
         q += (int64_t)gridDim.x * blockDim.x)
        grid_count[q] = 0;
    if ((int)blockIdx.x >= ndraw) {
        // one entry after the other here: issuing all loads first (scatter_items)
        // measured slower beside the draw blocks of this launch
        const int64_t b = (int64_t)blockIdx.x - ndraw;
#pragma unroll
        for (int j = 0; j < BIN_ITEMS; ++j) {
            const int64_t k = b * BIN_CHUNK + (int64_t)j * BIN_T + threadIdx.x;
            if (k < NT) {
                const int32_t gc = cellid[k];
                const int32_t c0 = A.cell_start[gc];
                int64_t pos = (int64_t)c0 + slot[k];
                if (k >= A.s.N)  // sites follow the cell's solvent
                    pos += (A.cell_start[gc + 1] - c0) - (A.site_start[gc + 1] - A.site_start[gc]);
                if (pos >= 0 && pos < NT) perm[pos] = (int32_t)k;
                else st |= ST_BINERR;
            }
        }
    } else {
        draw_cells(A, draws, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)ndraw * blockDim.x, st);
    }
    flag(A.status, st);
}

__device__ __forceinline__ void read_axis(const CollideArgs &A, int64_t gc, double nax[3])
{
    const int64_t C = A.s.C;
    nax[0] = A.draws[gc];
    nax[1] = A.draws[C + gc];
    nax[2] = A.draws[2 * C + gc];
}

// lambda = sqrt(kT_cell g / E) when E > 0 (cell thermostat), else 1; g is the
// cell's gamma variate.
__device__ __forceinline__ double thermostat_factor(const CollideArgs &A, double g, double E)
{
    if (!(E > 0.0)) return 1.0;
    const double Enew = A.kT_cell * g;
    return sqrt(Enew / E);
}

// The cell's random axis and, with the thermostat, its gamma variate (n: the
// cell's member count).  Read from the draws pass, or (A.inline_draws) drawn
// here by the same calls of the cell's streams as the draws pass makes, so
// the values are the same either way; inside the collision the ALU work of
// the draws overlaps the tile's gathers.
template <int INL = -1>  // 0 or 1: known at compile time; -1: A.inline_draws
__device__ __forceinline__ void cell_axis_gamma(const CollideArgs &A, int64_t gc, int r, int n, double nax[3],
                                                double &gvar, uint32_t &st)
{
    const SysDev &s = A.s;
    gvar = 0.0;
    if (INL == 0 || (INL < 0 && !A.inline_draws)) {
        read_axis(A, gc, nax);
        if (A.kT_cell > 0.0) gvar = A.draws[3 * s.C + gc];
        return;
    }
    const uint64_t cl = (uint64_t)brick_canonical(s.ncell[3 * r], s.ncell[3 * r + 1], s.ncell[3 * r + 2],
                                                  (int32_t)(gc - s.cell_off[r]));
    CellDraw D;
    st |= cell_draw(A.seed, *A.d_step, cl, s.replica0 + (uint64_t)r, A.kT_cell > 0.0 && n >= 2,
                    0.5 * (double)(3 * (n - 1)), D);
    nax[0] = D.n[0];
    nax[1] = D.n[1];
    nax[2] = D.n[2];
    if (A.kT_cell > 0.0 && n >= 2) gvar = D.g;
}

// ---- fallback: one lane per cell, members read from global memory ----------
// (tiles whose member count exceeds the LDS capacity)

template <typename Real> struct RealOps;
template <> struct RealOps<double> {
    __device__ static double wrap(double y, double L, uint32_t &st) { return wrap_d(y, L, st); }
};
template <> struct RealOps<float> {
    __device__ static float wrap(float y, float L, uint32_t &st) { return wrap_f(y, L, st); }
};

// Out-of-place solvent output: the new state of the solvent in cell order
// (v == nullptr: the collision works in place).
template <typename Real> struct SolvOut {
    Real *x, *v;
    int32_t *tag;
};

// Velocity of the member at permutation position i (particle k): sites in
// place; solvent in place, or at its cell-order slot of the output.
template <typename Real> struct MemberVel {
    Real *v, *vs, *vo;
    int64_t N, S, ss;  // ss: sites in the cells before this one
    __device__ Real &operator()(int i, int32_t k, int d) const
    {
        if (k >= N) return vs[d * S + (k - N)];
        return vo ? vo[d * N + (i - ss)] : v[d * N + k];
    }
};

// Cell gc with global-memory traffic only (a tile above the LDS capacity).
// Out of place, the cell's solvent is first copied to its output slots and
// collides there; the input arrays are not written.
// Returns false (and the cell is skipped) when a solvent member's output slot
// falls outside [0, N), which only a corrupted permutation can cause.
template <typename Real>
__device__ bool cell_out_prepare(const CollideArgs &A, int64_t gc, const Real *v, const SolvOut<Real> &O,
                                 uint32_t &st)
{
    if (!O.v) return true;
    const int64_t N = A.s.N, ss = A.site_start[gc];
    for (int i = A.cell_start[gc]; i < A.cell_start[gc + 1]; ++i) {
        const int64_t dst = i - ss;
        if (A.perm[i] < N && (dst < 0 || dst >= N)) {
            st |= ST_BINERR;
            return false;
        }
    }
    for (int i = A.cell_start[gc]; i < A.cell_start[gc + 1]; ++i) {
        const int32_t k = A.perm[i];
        if (k >= N) continue;
        const int64_t dst = i - ss;
#pragma unroll
        for (int d = 0; d < 3; ++d) O.v[d * N + dst] = v[d * N + k];
        O.tag[dst] = A.tag ? A.tag[k] : k;
    }
    return true;
}

template <typename Real>
__device__ void cell_stream_global(const CollideArgs &A, int64_t gc, const MemberVel<Real> &vel, Real *x,
                                   const SolvOut<Real> &O, uint32_t &st)
{
    if (!x) return;
    const SysDev &s = A.s;
    const int64_t N = s.N;
    const int r = find_sys(s.cell_off, s.nsys, gc);
    const Real dtr = (Real)A.dt;
    for (int i = A.cell_start[gc]; i < A.cell_start[gc + 1]; ++i) {
        const int32_t k = A.perm[i];
        if (k >= N) continue;
        Real *xd = O.v ? O.x + (i - vel.ss) : x + k;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const Real L = (Real)((double)s.ncell[3 * r + d] * s.a);
            Real y = x[d * N + k] + vel(i, k, d) * dtr;
            if (A.F.on) {
                y = y + (Real)A.F.h[d];
                vel(i, k, d) = vel(i, k, d) + (Real)A.F.gdt[d];
            }
            xd[d * N] = RealOps<Real>::wrap(y, L, st);
        }
    }
}

template <int INL>
__device__ void collide_cell_f64_global(const CollideArgs &A, int64_t gc, double *v, double *vs, double *x,
                                        const SolvOut<double> &O, uint32_t &st)
{
    const SysDev &s = A.s;
    const int b = A.cell_start[gc], e = A.cell_start[gc + 1], n = e - b;
    if (n == 0) return;
    const int64_t N = s.N, S = s.S;
    if (!cell_out_prepare<double>(A, gc, v, O, st)) return;
    const MemberVel<double> vel{v, vs, O.v, N, S, A.site_start[gc]};
    // the canonical ordering below is quadratic in the members: a cell far
    // beyond any physical occupancy (a corrupted state) is streamed, not collided
    constexpr int MAX_CELL_F64 = 1 << 14;
    if (n > MAX_CELL_F64) {
        st |= ST_CROWD;
        cell_stream_global<double>(A, gc, vel, x, O, st);
        return;
    }
    // identity key in the high word, permutation position in the low word
    auto key_at = [&](int i) -> uint64_t { return ((uint64_t)ident(A, A.perm[i]) << 32) | (uint32_t)i; };
    auto mass = [&](int32_t k) -> double { return k < N ? s.m : A.site_m[k - N]; };
    // members in ascending identity by repeated selection of the next key
    auto canonical = [&](auto &&fn) {
        uint64_t lo = 0;
        for (int c = 0; c < n; ++c) {
            uint64_t best = ~0ull;
            for (int j = b; j < e; ++j) {
                const uint64_t kk = key_at(j);
                if (kk >= lo && kk < best) best = kk;
            }
            lo = best + 1;
            const int i = (int)(uint32_t)(best & 0xffffffffu);
            fn(i, A.perm[i]);
        }
    };
    if (n >= 2) {
        double M = 0.0, P0 = 0.0, P1 = 0.0, P2 = 0.0;
        canonical([&](int i, int32_t k) {
            const double mk = mass(k);
            M = M + mk;
            P0 = P0 + mk * vel(i, k, 0);
            P1 = P1 + mk * vel(i, k, 1);
            P2 = P2 + mk * vel(i, k, 2);
        });
        const double u[3] = {P0 / M, P1 / M, P2 / M};
        double nax[3], gvar;
        cell_axis_gamma<INL>(A, gc, find_sys(A.s.cell_off, A.s.nsys, gc), n, nax, gvar, st);
        const Rot R = rotation(nax, A.cos_a, A.sin_a);
        double lam = 1.0;
        if (A.kT_cell > 0.0) {
            double Es = 0.0;
            canonical([&](int i, int32_t k) {
                const double d0 = vel(i, k, 0) - u[0], d1 = vel(i, k, 1) - u[1], d2 = vel(i, k, 2) - u[2];
                Es = Es + mass(k) * ((d0 * d0 + d1 * d1) + d2 * d2);
            });
            lam = thermostat_factor(A, gvar, 0.5 * Es);
        }
        for (int i = b; i < e; ++i) {
            const int32_t k = A.perm[i];
            const double dl[3] = {vel(i, k, 0) - u[0], vel(i, k, 1) - u[1], vel(i, k, 2) - u[2]};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double rr = (R.R[d][0] * dl[0] + R.R[d][1] * dl[1]) + R.R[d][2] * dl[2];
                const double vn = u[d] + lam * rr;
                if (!(vn - vn == 0.0)) st |= ST_NONFINITE;
                vel(i, k, d) = vn;
            }
        }
    }
    cell_stream_global<double>(A, gc, vel, x, O, st);
}

// FP32 form: per-member fixed-point terms m, m v (3) and m |v|^2, each formed
// in double and rounded once to the nearest multiple of 2^-32 (ties to even)
// into int64, so that the per-cell sums are exact and independent of order.
// The fine unit matters for the thermostat: a cell's relative kinetic energy
// is the difference of two sums, and in a cell of nearly equal velocities it
// is small.  A member whose term reaches 2^51 units (|m v| or m |v|^2 of
// 2^19) adds nothing and sets FIXOVF.
constexpr double FIX_SCALE = 0x1p32, FIX_UNIT = 0x1p-32, FIX_LIM = 0x1p51;

// Nearest integer (ties to even) of |a| < 2^51: adding 1.5 2^52 rounds a to
// an integer within the sum's mantissa (the sum's unit in the last place is
// 1, and 1.5 2^52 is even, so ties go the same way), and the difference of
// the two bit patterns is that integer.  One add and one subtraction, the
// same value as a general double-to-int64 rounding.
__device__ __forceinline__ long long fix_round(double a)
{
    const double m = 0x1.8p52;
    return __double_as_longlong(a + m) - __double_as_longlong(m);
}

// The same for any a in the int64 range (a species' mass term, once).
__device__ __forceinline__ long long fix_round_any(double a) { return __double2ll_rn(a); }

// The terms from mS = m 2^32 and q0 = its rounding, which a caller can form
// once per species: (m 2^32) v equals (m v) 2^32 exactly (scaling by a power
// of two commutes with rounding; neither product can underflow or overflow).
__device__ __forceinline__ void fixed_terms_scaled(double mS, long long q0, float fv0, float fv1, float fv2,
                                                   long long q[5], uint32_t &st)
{
    const double v0 = (double)fv0, v1 = (double)fv1, v2 = (double)fv2;
    const double a0 = mS * v0, a1 = mS * v1, a2 = mS * v2;
    const double ak = mS * ((v0 * v0 + v1 * v1) + v2 * v2);
    if (!(fabs(a0) < FIX_LIM && fabs(a1) < FIX_LIM && fabs(a2) < FIX_LIM && ak < FIX_LIM)) {
        st |= ST_FIXOVF;
        q[0] = q[1] = q[2] = q[3] = q[4] = 0;
        return;
    }
    q[0] = q0;
    q[1] = fix_round(a0);
    q[2] = fix_round(a1);
    q[3] = fix_round(a2);
    q[4] = fix_round(ak);
}

__device__ __forceinline__ void fixed_terms(double mk, float fv0, float fv1, float fv2, long long q[5],
                                            uint32_t &st)
{
    const double mS = mk * FIX_SCALE;
    fixed_terms_scaled(mS, fix_round_any(mS), fv0, fv1, fv2, q, st);
}

// Relative kinetic energy of a cell, 1/2 (sum m |v|^2 - |sum m v|^2 / sum m),
// from its fixed-point sums.
__device__ __forceinline__ double fixed_energy(const long long q[5])
{
    const double Mu = (double)q[0] * FIX_UNIT;
    const double P0 = (double)q[1] * FIX_UNIT, P1 = (double)q[2] * FIX_UNIT, P2 = (double)q[3] * FIX_UNIT;
    return 0.5 * ((double)q[4] * FIX_UNIT - ((P0 * P0 + P1 * P1) + P2 * P2) / Mu);
}

// Per-cell FP32 collision parameters from exact fixed-point sums: u and
// lambda R rounded to float.
template <int INL>
__device__ __forceinline__ void f32_cell_params(const CollideArgs &A, int64_t gc, int n, const long long q[5],
                                                float uf[3], float Rf[3][3], uint32_t &st)
{
    const double Md = (double)q[0];
    const double u0 = (double)q[1] / Md, u1 = (double)q[2] / Md, u2 = (double)q[3] / Md;
    double nax[3], gvar;
    cell_axis_gamma<INL>(A, gc, find_sys(A.s.cell_off, A.s.nsys, gc), n, nax, gvar, st);
    const Rot R = rotation(nax, A.cos_a, A.sin_a);
    double lam = 1.0;
    if (A.kT_cell > 0.0) {
        const double E = fixed_energy(q);
        lam = thermostat_factor(A, gvar, E);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Rf[i][j] = (float)(lam * R.R[i][j]);
    uf[0] = (float)u0; uf[1] = (float)u1; uf[2] = (float)u2;
}

template <int INL>
__device__ void collide_cell_f32_global(const CollideArgs &A, int64_t gc, float *v, float *vs, float *x,
                                        const SolvOut<float> &O, uint32_t &st)
{
    const SysDev &s = A.s;
    const int b = A.cell_start[gc], e = A.cell_start[gc + 1], n = e - b;
    if (n == 0) return;
    const int64_t N = s.N, S = s.S;
    if (!cell_out_prepare<float>(A, gc, v, O, st)) return;
    const MemberVel<float> vel{v, vs, O.v, N, S, A.site_start[gc]};
    if (n >= 2) {
        long long acc[5] = {0, 0, 0, 0, 0};
        for (int i = b; i < e; ++i) {
            const int32_t k = A.perm[i];
            long long q[5];
            fixed_terms(k < N ? s.m : A.site_m[k - N], vel(i, k, 0), vel(i, k, 1), vel(i, k, 2), q, st);
#pragma unroll
            for (int j = 0; j < 5; ++j) acc[j] += q[j];
        }
        float uf[3], Rf[3][3];
        f32_cell_params<INL>(A, gc, n, acc, uf, Rf, st);
        for (int i = b; i < e; ++i) {
            const int32_t k = A.perm[i];
            const float dl[3] = {vel(i, k, 0) - uf[0], vel(i, k, 1) - uf[1], vel(i, k, 2) - uf[2]};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const float vn = uf[d] + ((Rf[d][0] * dl[0] + Rf[d][1] * dl[1]) + Rf[d][2] * dl[2]);
                if (!(vn - vn == 0.0f)) st |= ST_NONFINITE;
                vel(i, k, d) = vn;
            }
        }
    }
    cell_stream_global<float>(A, gc, vel, x, O, st);
}

// ---- tiled collision: a block owns cpb consecutive cells -------------------
//
// The tile's members are a contiguous range of the permutation.  Each thread
// owns ITEMS members (register-batched, so all of its gathers are in flight at
// once) and, while those loads are outstanding, draws its cell's random axis
// and thermostat gamma variate (they depend only on the step, the cell and its
// member count).  Phase 2, one lane per cell: FP64 orders the cell's keys in
// LDS and sums in ascending identity; FP32 reads exact int64 fixed-point sums
// accumulated with LDS atomics in phase 1.  Phase 3 rotates each member and
// streams the solvent.  Blocks are remapped so that each XCD (8 per MI355X,
// each with its own L2) processes a contiguous range of tiles.


__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS layout: offsets of s_cs, s_idx, s_cl, s_v, s_key|s_acc, s_par, s_r, end.
struct TileLayout {
    size_t cs, idx, cl, v, keyacc, par, r, ss, len, end;
};

__host__ __device__ inline TileLayout tile_layout(bool f64, int cpb, int cap)
{
    TileLayout L;
    size_t o = 0;
    L.cs = o; o += align16(sizeof(int) * (size_t)(cpb + 1));
    // member indices and velocities are staged for the FP64 canonical sums only
    L.idx = o; o += align16(f64 ? sizeof(int) * (size_t)cap : 0);
    L.cl = o; o += align16(sizeof(uint16_t) * (size_t)cap);
    L.v = o; o += align16(f64 ? 8 * 3 * (size_t)cap : 0);
    L.keyacc = o; o += align16(f64 ? sizeof(uint64_t) * (size_t)cap : sizeof(long long) * 5 * (size_t)cpb);
    L.par = o; o += align16(f64 ? sizeof(double) * 13 * (size_t)cpb : sizeof(float) * 12 * (size_t)cpb);
    L.r = o; o += align16(sizeof(int) * (size_t)cpb);
    L.ss = o; o += align16(sizeof(int) * (size_t)cpb);
    L.len = o; o += align16((f64 ? 8 : 4) * 3 * (size_t)cpb);  // box edges of each cell's system
    L.end = o;
    return L;
}


template <typename Real, int ITEMS, int INL, bool BIN>
__device__ __forceinline__ void collide_tile(const CollideArgs &A, const TileCfg &T, Real *v, Real *vs, Real *xstream,
                                             const SolvOut<Real> &O)
{
    constexpr bool F64 = sizeof(Real) == 8;
    extern __shared__ __align__(16) unsigned char smem[];
    if (A.advance_step && blockIdx.x == 0 && threadIdx.x == 0) *A.advance_step = *A.advance_step + 1;
    if (A.step_next && blockIdx.x == 0 && threadIdx.x == 0) *A.step_next = *A.d_step + 1;
    const int tile = tile_of_block(T.ntiles);
    if (tile >= T.ntiles) return;
    const SysDev &s = A.s;
    const int t = threadIdx.x;
    const int64_t c0 = (int64_t)tile * T.cpb;
    const int nc = (int)((s.C - c0) < T.cpb ? (s.C - c0) : T.cpb);
    const int m0 = A.cell_start[c0], nm = A.cell_start[c0 + nc] - m0;
    uint32_t st = 0;
    if (nm > T.cap) {
        for (int c = t; c < nc; c += TILE_T) {
            if constexpr (F64) collide_cell_f64_global<INL>(A, c0 + c, v, vs, xstream, O, st);
            else collide_cell_f32_global<INL>(A, c0 + c, v, vs, xstream, O, st);
        }
        if constexpr (BIN) {
            // the tile's new solvent is the contiguous range [q0, q1) of the
            // output; bin it with one device atomic per particle (crowded
            // tiles are rare)
            __syncthreads();  // the block's stores of the new solvent are visible to it
            const int64_t q0 = (int64_t)A.cell_start[c0] - A.site_start[c0];
            const int64_t q1 = (int64_t)A.cell_start[c0 + nc] - A.site_start[c0 + nc];
            const uint64_t step1 = *A.d_step + 1;
            for (int64_t q = q0 + t; q < q1; q += TILE_T) {
                if (q < 0 || q >= s.N) {
                    st |= ST_BINERR;
                    continue;
                }
                const int r = find_sys(s.solv_off, s.nsys, q);
                double sh[3];
                shift_of(s, A.seed, step1, r, sh);
                const int32_t gc = cell_of_pos<Real>(s, r, O.x[q], O.x[s.N + q], O.x[2 * s.N + q], sh, st);
                const unsigned long long old = atomicAdd(&A.bin_counts[gc], 1ull);
                A.bin_slot[q] = (int32_t)(old & 0xffffffffull);
                A.bin_cellid[q] = gc;
            }
        }
        flag(A.status, st);
        return;
    }
    const int cap = T.cap;
    const TileLayout Lo = tile_layout(F64, T.cpb, cap);
    int *s_cs = (int *)(smem + Lo.cs);
    int *s_idx = (int *)(smem + Lo.idx);
    uint16_t *s_cl = (uint16_t *)(smem + Lo.cl);
    Real *s_v = (Real *)(smem + Lo.v);
    uint64_t *s_key = (uint64_t *)(smem + Lo.keyacc);
    int *s_r = (int *)(smem + Lo.r);
    int *s_ss = (int *)(smem + Lo.ss);
    Real *s_len = (Real *)(smem + Lo.len);
    double *s_shift = (double *)(smem + Lo.end);  // BIN: next-step shifts of systems tr0..tr1
    const int64_t N = s.N, S = s.S;
    const bool out = O.v != nullptr;

    // the tile's member gathers (v, and x for the streaming) go out first: they
    // need only the tile's member range, and they are in flight through phase 0
    int kk[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int i = t + j * TILE_T;
        kk[j] = (i < nm) ? A.perm[m0 + i] : -1;
    }
    Real va[ITEMS][3], xo[ITEMS][3];
    int32_t tg[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int32_t k = kk[j];
        if (k >= 0) {
            if (k < N) {
                va[j][0] = v[k]; va[j][1] = v[N + k]; va[j][2] = v[2 * N + k];
                if (xstream) {
                    xo[j][0] = xstream[k]; xo[j][1] = xstream[N + k]; xo[j][2] = xstream[2 * N + k];
                }
                if (out) tg[j] = A.tag ? A.tag[k] : k;
            } else {
                const int64_t q = k - N;
                va[j][0] = vs[q]; va[j][1] = vs[S + q]; va[j][2] = vs[2 * S + q];
            }
        }
    }
    // systems of the tile's first and last cells, found by each wave for
    // itself (every lane is here); a cell's own search is bounded by them
    const int tr0 = find_sys_wave(s.cell_off, s.nsys, c0);
    const int tr1 = find_sys_wave(s.cell_off, s.nsys, c0 + nc - 1);
    // phase 0: the tile's cell ranges and slot -> cell map; this lane's cell
    // system and draws; FP32: clear the cell's fixed-point accumulators
    unsigned long long *s_acc = (unsigned long long *)(smem + Lo.keyacc);
    for (int c = t; c <= nc; c += TILE_T) s_cs[c] = A.cell_start[c0 + c] - m0;
    double nax[3] = {0.0, 0.0, 1.0}, gvar = 0.0;
    if (t < nc) {
        const int64_t gc = c0 + t;
        const int r = tr0 == tr1 ? tr0 : find_sys_in(s.cell_off, tr0, tr1, gc);
        const int cb0 = A.cell_start[gc] - m0, ce0 = A.cell_start[gc + 1] - m0;
        for (int i = cb0; i < ce0; ++i) s_cl[i] = (uint16_t)t;
        cell_axis_gamma<INL>(A, gc, r, ce0 - cb0, nax, gvar, st);
        if constexpr (!F64) {
#pragma unroll
            for (int z = 0; z < 5; ++z) s_acc[5 * t + z] = 0ull;
        }
        s_r[t] = r;
        if (out) s_ss[t] = A.site_start[gc];
#pragma unroll
        for (int d = 0; d < 3; ++d) s_len[3 * t + d] = (Real)((double)s.ncell[3 * r + d] * s.a);
    }
    if constexpr (BIN) {  // next-step shift of system tr0 + l by lane TILE_T - 1 - l (a tile has
                          // at least one cell per system, so at most TILE_T systems)
        const int l = TILE_T - 1 - t;
        if (l <= tr1 - tr0 && l < T.cpb) shift_of(s, A.seed, *A.d_step + 1, tr0 + l, s_shift + 3 * l);
    }
    __syncthreads();

    // phase 1: fixed-point sums (FP32) or LDS staging (FP64); slot -> cell map
    const int cb = (t < nc) ? s_cs[t] : 0, ce = (t < nc) ? s_cs[t + 1] : 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int i = t + j * TILE_T;
        if (i < nm) {
            const int32_t k = kk[j];
            if constexpr (F64) {
                s_idx[i] = k;
                s_v[i] = va[j][0]; s_v[cap + i] = va[j][1]; s_v[2 * cap + i] = va[j][2];
                s_key[i] = ((uint64_t)ident(A, k) << 32) | (uint32_t)i;
            } else {
                // exact int64 fixed-point terms, summed per cell with LDS
                // atomics (integer sums: the order does not matter)
                long long w[5];
                fixed_terms(k < N ? s.m : A.site_m[k - N], (float)va[j][0], (float)va[j][1], (float)va[j][2], w,
                            st);
                unsigned long long *acc = s_acc + 5 * (int)s_cl[i];
#pragma unroll
                for (int z = 0; z < 5; ++z) atomicAdd(acc + z, (unsigned long long)w[z]);
            }
        }
    }
    __syncthreads();

    // phase 2: one lane per cell
    if (t < nc) {
        const int b = cb, e = ce, n = e - b;
        if (n >= 2) {
            const Rot R = rotation(nax, A.cos_a, A.sin_a);
            if constexpr (F64) {
                double *par = (double *)(smem + Lo.par) + 13 * t;
                // ascending identity: insertion into the (nearly ordered) segment
                for (int i = b + 1; i < e; ++i) {
                    const uint64_t key = s_key[i];
                    int pos = i;
                    while (pos > b && s_key[pos - 1] > key) {
                        s_key[pos] = s_key[pos - 1];
                        --pos;
                    }
                    s_key[pos] = key;
                }
                double M = 0.0, P0 = 0.0, P1 = 0.0, P2 = 0.0;
                for (int i = b; i < e; ++i) {
                    const int li = (int)(uint32_t)(s_key[i] & 0xffffffffu);
                    const int32_t k = s_idx[li];
                    const double mk = k < N ? s.m : A.site_m[k - N];
                    M = M + mk;
                    P0 = P0 + mk * (double)s_v[li];
                    P1 = P1 + mk * (double)s_v[cap + li];
                    P2 = P2 + mk * (double)s_v[2 * cap + li];
                }
                const double u0 = P0 / M, u1 = P1 / M, u2 = P2 / M;
                double lam = 1.0;
                if (A.kT_cell > 0.0) {
                    double Es = 0.0;
                    for (int i = b; i < e; ++i) {
                        const int li = (int)(uint32_t)(s_key[i] & 0xffffffffu);
                        const int32_t k = s_idx[li];
                        const double d0 = (double)s_v[li] - u0, d1 = (double)s_v[cap + li] - u1,
                                     d2 = (double)s_v[2 * cap + li] - u2;
                        Es = Es + (k < N ? s.m : A.site_m[k - N]) * ((d0 * d0 + d1 * d1) + d2 * d2);
                    }
                    const double E = 0.5 * Es;
                    if (E > 0.0) lam = sqrt((A.kT_cell * gvar) / E);
                }
                par[0] = u0; par[1] = u1; par[2] = u2; par[3] = lam;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) par[4 + 3 * i + j] = R.R[i][j];
            } else {
                long long q[5];
#pragma unroll
                for (int z = 0; z < 5; ++z) q[z] = (long long)s_acc[5 * t + z];
                float *par = (float *)(smem + Lo.par) + 12 * t;
                const double Md = (double)q[0];
                const double u0 = (double)q[1] / Md, u1 = (double)q[2] / Md, u2 = (double)q[3] / Md;
                double lam = 1.0;
                if (A.kT_cell > 0.0) {
                    const double E = fixed_energy(q);
                    if (E > 0.0) lam = sqrt((A.kT_cell * gvar) / E);
                }
                par[0] = (float)u0; par[1] = (float)u1; par[2] = (float)u2;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) par[3 + 3 * i + j] = (float)(lam * R.R[i][j]);
            }
        }
    }
    __syncthreads();

    // phase 3: rotate, stream, write back (solvent out of place: to its
    // cell-order slot, every member whether or not its cell collided).  The
    // out-of-place and in-place forms are separate loops, so each keeps only
    // its own pointers live.
    const Real dtr = (Real)A.dt;
    const bool fon = A.F.on != 0;
    Real fh[3], fg[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        fh[d] = (Real)A.F.h[d];
        fg[d] = (Real)A.F.gdt[d];
    }
    // collided velocity of item j (its cell c); writes a site's back
    auto rotate = [&](int j, int c, Real vn[3]) {
        vn[0] = va[j][0]; vn[1] = va[j][1]; vn[2] = va[j][2];
        if ((s_cs[c + 1] - s_cs[c]) < 2) return;
        if constexpr (F64) {
            const double *par = (const double *)(smem + Lo.par) + 13 * c;
            const double dl[3] = {vn[0] - par[0], vn[1] - par[1], vn[2] - par[2]};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double rr = (par[4 + 3 * d] * dl[0] + par[5 + 3 * d] * dl[1]) + par[6 + 3 * d] * dl[2];
                vn[d] = par[d] + par[3] * rr;
                if (!(vn[d] - vn[d] == 0.0)) st |= ST_NONFINITE;
            }
        } else {
            const float *par = (const float *)(smem + Lo.par) + 12 * c;
            const float dl[3] = {vn[0] - par[0], vn[1] - par[1], vn[2] - par[2]};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                vn[d] = par[d] + ((par[3 + 3 * d] * dl[0] + par[4 + 3 * d] * dl[1]) + par[5 + 3 * d] * dl[2]);
                if (!(vn[d] - vn[d] == 0.0f)) st |= ST_NONFINITE;
            }
        }
        if (kk[j] >= N) {
            const int64_t q = kk[j] - N;
            vs[q] = vn[0]; vs[S + q] = vn[1]; vs[2 * S + q] = vn[2];
        }
    };
    // BIN: the next-step cell of each new solvent particle and its output index
    int32_t gcs[BIN ? ITEMS : 1], dsts[BIN ? ITEMS : 1];
#pragma unroll
    for (int j = 0; j < (BIN ? ITEMS : 1); ++j) gcs[j] = dsts[j] = -1;
    if (out) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int i = t + j * TILE_T;
            if (i >= nm) continue;
            const int c = s_cl[i];
            Real vn[3];
            rotate(j, c, vn);
            if (kk[j] >= N) continue;
            const int64_t dst = (int64_t)(m0 + i) - s_ss[c];
            if (dst < 0 || dst >= N) {  // only with a corrupted permutation
                st |= ST_BINERR;
                continue;
            }
            Real yw[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const Real L = s_len[3 * c + d];
                Real y = xo[j][d] + vn[d] * dtr;
                Real vo = vn[d];
                if (fon) {
                    y = y + fh[d];
                    vo = vo + fg[d];
                }
                yw[d] = RealOps<Real>::wrap(y, L, st);
                O.x[d * N + dst] = yw[d];
                O.v[d * N + dst] = vo;
            }
            O.tag[dst] = tg[j];
            if constexpr (BIN) {
                const int r = s_r[c];
                if (r - tr0 >= T.cpb) {  // only with systems of no cells
                    st |= ST_BINERR;
                    continue;
                }
                const double *sh = s_shift + 3 * (r - tr0);
                const double shv[3] = {sh[0], sh[1], sh[2]};
                gcs[j] = cell_of_pos<Real>(s, r, yw[0], yw[1], yw[2], shv, st);
                dsts[j] = (int32_t)dst;
            }
        }
        if constexpr (BIN) {
            // phase 4: count the new solvent per next-step cell in an LDS hash
            // table (over the tile's LDS, free now), one device atomic per
            // distinct cell for its base slot; slot = base + rank in the block
            constexpr int HT = TILE_T * ITEMS, HT_BITS = ITEMS == 1 ? 8 : ITEMS == 2 ? 9 : ITEMS == 4 ? 10 : 11;
            static_assert((1 << HT_BITS) == HT, "hash size");
            uint32_t *hkey = (uint32_t *)smem;
            int32_t *hcnt = (int32_t *)(smem + sizeof(uint32_t) * HT);
            __syncthreads();  // phase 3's LDS reads are done
#pragma unroll
            for (int it = 0; it < ITEMS; ++it) {
                hkey[t + it * TILE_T] = BIN_EMPTY;
                hcnt[t + it * TILE_T] = 0;
            }
            __syncthreads();
            int hs[ITEMS], rk[ITEMS];
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                hs[j] = rk[j] = 0;
                if (gcs[j] < 0) continue;
                const uint32_t key = (uint32_t)gcs[j];
                uint32_t h = (key * 2654435761u) >> (32 - HT_BITS);
                while (true) {  // ends: at most HT members, so fewer distinct keys than slots
                    const uint32_t old = atomicCAS(&hkey[h], BIN_EMPTY, key);
                    if (old == BIN_EMPTY || old == key) break;
                    h = (h + 1) & (HT - 1);
                }
                hs[j] = (int)h;
                rk[j] = atomicAdd(&hcnt[h], 1);
            }
            __syncthreads();
            unsigned long long base[ITEMS];
            uint32_t keys[ITEMS];
#pragma unroll
            for (int it = 0; it < ITEMS; ++it) {
                const int i = t + it * TILE_T;
                keys[it] = hkey[i];
                base[it] = 0ull;
                if (keys[it] != BIN_EMPTY) base[it] = atomicAdd(&A.bin_counts[keys[it]], (unsigned long long)hcnt[i]);
            }
#pragma unroll
            for (int it = 0; it < ITEMS; ++it)
                if (keys[it] != BIN_EMPTY) hcnt[t + it * TILE_T] = (int32_t)(base[it] & 0xffffffffull);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                if (gcs[j] < 0) continue;
                A.bin_slot[dsts[j]] = hcnt[hs[j]] + rk[j];
                A.bin_cellid[dsts[j]] = gcs[j];
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int i = t + j * TILE_T;
            if (i >= nm) continue;
            const int c = s_cl[i];
            const int32_t k = kk[j];
            Real vn[3];
            rotate(j, c, vn);
            if (k >= N) continue;
            const bool moved = (s_cs[c + 1] - s_cs[c]) >= 2;
            if (xstream) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const Real L = s_len[3 * c + d];
                    Real y = xo[j][d] + vn[d] * dtr;
                    if (fon) y = y + fh[d];
                    xstream[d * N + k] = RealOps<Real>::wrap(y, L, st);
                    if (moved || fon) v[d * N + k] = fon ? vn[d] + fg[d] : vn[d];
                }
            } else if (moved) {
                v[k] = vn[0]; v[N + k] = vn[1]; v[2 * N + k] = vn[2];
            }
        }
    }
    flag(A.status, st);
}

// One kernel per items-per-thread choice, each with the draws read from the
// draws pass or made inside (suffix _d), and each of those with the binning of
// the new solvent for the next step (suffix _b).  The FP32 4-item form without
// draws is held to 80 VGPRs (six waves per SIMD to hide the gather latency;
// measured faster than five), the 2-item form to 72 (seven waves) and the
// 8-item form with draws to 128 (four waves; the compiler's own choice, 129,
// drops it to three); the other forms keep the compiler's allocation (a tighter
// cap spills).
#define MPCD_COLLIDE_KERNEL(NAME, ATTR, REAL, ITEMS, INL, BIN)                                                 \
    __global__ __launch_bounds__(TILE_T) ATTR void NAME(CollideArgs A, TileCfg T, REAL *v, REAL *vs,           \
                                                        REAL *xstream, SolvOut<REAL> O)                       \
    {                                                                                                          \
        collide_tile<REAL, ITEMS, INL, BIN>(A, T, v, vs, xstream, O);                                         \
    }
#define MPCD_COLLIDE_PAIR(NAME, ATTR, REAL, ITEMS, INL)                                                        \
    MPCD_COLLIDE_KERNEL(NAME, ATTR, REAL, ITEMS, INL, false)                                                   \
    MPCD_COLLIDE_KERNEL(NAME##_b, ATTR, REAL, ITEMS, INL, true)
MPCD_COLLIDE_PAIR(k_collide_tiled_f32_i2, __attribute__((amdgpu_waves_per_eu(7))), float, 2, 0)
MPCD_COLLIDE_PAIR(k_collide_tiled_f32, __attribute__((amdgpu_waves_per_eu(6))), float, 4, 0)
MPCD_COLLIDE_PAIR(k_collide_tiled_f32_i8, , float, 8, 0)
MPCD_COLLIDE_PAIR(k_collide_tiled_f32_i2_d, , float, 2, 1)
MPCD_COLLIDE_PAIR(k_collide_tiled_f32_d, , float, 4, 1)
MPCD_COLLIDE_PAIR(k_collide_tiled_f32_i8_d, __attribute__((amdgpu_waves_per_eu(4))), float, 8, 1)
MPCD_COLLIDE_PAIR(k_collide_tiled_f64_i1, , double, 1, 0)
MPCD_COLLIDE_PAIR(k_collide_tiled_f64, , double, 2, 0)
MPCD_COLLIDE_PAIR(k_collide_tiled_f64_i4, , double, 4, 0)
MPCD_COLLIDE_PAIR(k_collide_tiled_f64_i1_d, , double, 1, 1)
MPCD_COLLIDE_PAIR(k_collide_tiled_f64_d, , double, 2, 1)
MPCD_COLLIDE_PAIR(k_collide_tiled_f64_i4_d, , double, 4, 1)
#undef MPCD_COLLIDE_PAIR
#undef MPCD_COLLIDE_KERNEL

// ---------------------------------------------------------------------------
// (a1) site thermalization, Eqs. (5) and (7): one block per body.
//
// Each lane takes one site of a chunk: space-frame offset d_j = A dhat_j, site
// position, random velocity vt_j, and the terms m_j vt_j, d_j x m_j vt_j into
// LDS.  Lanes 0..5 then each add one of the six components over the chunk in
// site order (the order of a sequential host loop), carrying their partial
// sums across chunks.  Lane 0 forms Vt, omega_t and the body's V, omega; all
// lanes then write v_j = (V - Vt) + (omega - omega_t) x d_j + vt_j.
// Block 0 also draws the step's grid shifts.

// ---------------------------------------------------------------------------
// Binned solvent layout: definitions shared by the site binning (inside the
// thermalization) and the brick kernels further below.
//
// Each system's cells are grouped into bricks of BX x BY x BZ cells (powers of
// two, chosen per system from its density; narrower at the far faces).  The
// solvent arrays hold one region per brick, and a step's solvent lies in the
// region of the brick of its cell on that step's shifted grid.  A region is
// split into NCLS sub-regions, one per brick that can write into it: the
// brick itself and its neighbours one brick away along each axis (periodic),
// the "class" of the writer.  Each sub-region therefore has one writer per
// step, which stores its fill with a plain store (no device atomics).  A
// particle that moves farther than a neighbouring brick, or finds its
// sub-region full, spills into a shared overflow list.  Fills are kept per
// step parity: the step with index t reads the fills of parity t & 1 and
// writes parity (t + 1) & 1.  The surface sites of each brick are listed in
// the brick's site slots by the thermalization of the same step.
struct BrickInfo {
    int64_t off;      // first slot of the brick's region (its NCLS sub-regions follow)
    int32_t cap;      // region capacity
    int32_t sys;      // system of the brick
    int32_t soff;     // first site slot
    int16_t scap;     // site slot capacity
    int16_t org[3];   // first cell of the brick within its system
    uint8_t dim[3];   // cells along each axis
    uint8_t pad;
};
static_assert(sizeof(BrickInfo) == 32, "brick table entry");

constexpr int NCLS = 27;           // writer classes of a region
constexpr int BIN_OVF_CAP = 8192;  // solvent overflow entries per parity
// control words of the binned workspace
enum { BC_OVF0 = 1, BC_OVF1 = 2, BC_SOVF = 3, BC_WORDS = 16 };

struct BinnedDev {
    const BrickInfo *brick;  // [nbricks]
    const int32_t *subpre;   // [nbricks][NCLS + 1] first slot of each sub-region within the region
    const int4 *wtab;        // [nbricks][NCLS] the sub-region a brick writes with each class: first
                             // slot, capacity, destination brick (-1: none), unused
    const int32_t *sys_bb;   // [nsys + 1] first brick of each system
    const int32_t *sys_bg;   // [6 nsys] log2 of the brick extent (3), bricks per axis (3)
    int32_t *cnt;            // [2][nbricks][NCLS] sub-region fills, by step parity
    int32_t *scnt;           // [nbricks] sites per brick
    int32_t *sslot;          // site slots: site index
    int32_t *ctrl;           // [BC_WORDS]
    int32_t *ovf_dest;       // [2 BIN_OVF_CAP] overflow entries: destination brick,
    int32_t *ovf_tag;        // [2 BIN_OVF_CAP] identity,
    void *ovf_xv;            // [2][6][BIN_OVF_CAP] position and velocity (prec)
    int32_t *sovf;           // [2 sovf_cap]: (brick, site) pairs
    int32_t *oflag;          // [2][nbricks] nonzero: the overflow list may hold entries for the brick
    double *shtab;           // [2][1 + 6 nsys] step index, then each system's shifts for it and the next step
    int64_t nbricks, cap;    // bricks; slots of one set of solvent arrays
    int32_t sovf_cap;
};

// Writer class of a region along one axis of nb (periodic) bricks: 0 when the
// writing brick bs is the region's brick bd, 1 when bs = bd + 1, 2 when
// bs = bd - 1 (distinct from 1 only for nb >= 3), -1 otherwise.  The class of
// a region is cx + 3 cy + 9 cz.
__host__ __device__ __forceinline__ int class_code(int bs, int bd, int nb)
{
    int d = bs - bd;
    if (d < 0) d += nb;
    if (d == 0) return 0;
    if (d == 1) return 1;
    if (d == nb - 1) return 2;
    return -1;
}

__host__ __device__ __forceinline__ bool code_valid(int c, int nb) { return c == 0 || (c == 1 && nb >= 2) || (c == 2 && nb >= 3); }

// The region a writing brick at coordinate bs fills with code c (the inverse of class_code).
__host__ __device__ __forceinline__ int code_dst(int bs, int c, int nb)
{
    return c == 0 ? bs : c == 1 ? (bs + nb - 1) % nb : (bs + 1) % nb;
}

// Cell coordinates of a position on a shifted grid (as the binning computes
// them) and the brick of that cell; returns the brick index.
template <typename Real>
__device__ __forceinline__ int32_t brick_of_pos(const SysDev &s, const BinnedDev &bn, int r, Real p0, Real p1, Real p2,
                                                const double sh[3], int j[3], uint32_t &st)
{
    const int nx = s.ncell[3 * r], ny = s.ncell[3 * r + 1], nz = s.ncell[3 * r + 2];
    j[0] = axis_cell(p0, sh[0], s.a, s.inv_a, nx, st);
    j[1] = axis_cell(p1, sh[1], s.a, s.inv_a, ny, st);
    j[2] = axis_cell(p2, sh[2], s.a, s.inv_a, nz, st);
    const int32_t *g = bn.sys_bg + 6 * r;
    return bn.sys_bb[r] + ((j[2] >> g[2]) * g[4] + (j[1] >> g[1])) * g[3] + (j[0] >> g[0]);
}

// Site binning of the binned layout inside the thermalization: the site's
// brick on the step's grid, one device atomic per run of equal bricks within
// a wave, a slot in the brick's site list or, when that is full, an entry of
// the site overflow list.
struct BrickSiteBin {
    BinnedDev bn;
};

template <typename Real>
__device__ __forceinline__ void brick_bin_site(const SysDev &s, const BrickSiteBin &bb, int r, bool valid, int64_t j,
                                               const Real xr[3], const double *bsh, uint32_t &st)
{
    const BinnedDev &bn = bb.bn;
    int jc[3];
    const double sh[3] = {bsh[0], bsh[1], bsh[2]};
    const int32_t b = valid ? brick_of_pos<Real>(s, bn, r, xr[0], xr[1], xr[2], sh, jc, st) : -1;
    // the brick's site list, loaded before the counter's round trip
    int32_t soff = 0, scap = 0;
    if (b >= 0) {
        soff = bn.brick[b].soff;
        scap = bn.brick[b].scap;
    }
    const int lane = threadIdx.x & 63;
    const unsigned long long le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const int32_t prev = __shfl_up(b, 1, 64);
    const bool head = (lane == 0) || (prev != b);
    const unsigned long long heads = __ballot(head);
    const int hl = 63 - __clzll(heads & le);
    const unsigned long long above = heads & ~le;
    const int nh = above ? (__ffsll((long long)above) - 1) : 64;
    int base = 0;
    if (head && b >= 0) base = atomicAdd(&bn.scnt[b], nh - hl);
    base = __shfl(base, hl, 64);
    if (b < 0) return;
    const int rank = base + (lane - hl);
    if (rank < scap) {
        bn.sslot[soff + rank] = (int32_t)j;
    } else {
        const int e = atomicAdd(&bn.ctrl[BC_SOVF], 1);
        if (e < bn.sovf_cap) {
            bn.sovf[2 * e] = b;
            bn.sovf[2 * e + 1] = (int32_t)j;
        } else {
            st |= ST_BINERR;
        }
    }
}

constexpr int WAVE = 64;
constexpr int BODY_T = 256;
static_assert(BODY_T == BIN_T, "k_prep bins solvent with BODY_T-thread blocks");
constexpr int SH_PAD = BODY_T + 1;  // row padding against LDS bank conflicts

__device__ __forceinline__ void draw_shifts(const SysDev &s, uint64_t seed, uint64_t step, double *shift)
{
    for (int r = threadIdx.x; r < s.nsys; r += blockDim.x) {
        const Words w = rng_draw(seed, RNG_SHIFT, step, 0, s.replica0 + (uint64_t)r, 0);
#pragma unroll
        for (int k = 0; k < 3; ++k) shift[3 * r + k] = shift_component(w.w[k], s.a);
    }
}

// Lanes 0..5 add column t of sh over [0, cnt) in order into acc.
__device__ __forceinline__ void ordered_add(const double *sh, int cnt, double &acc)
{
    const int t = threadIdx.x;
    if (t < 6) {
        const double *row = sh + t * SH_PAD;
        for (int i = 0; i < cnt; ++i) acc = acc + row[i];
    }
}

// Thermalization of body b by one BODY_T block.  With `counts` set, the
// block also bins its sites (cell from the stored site position and the grid
// shift `bsh` of the body's system, which must be visible after the first
// barrier).
struct ThermLds {
    double sh[6 * SH_PAD];
    double sacc[6];
    double dvw[6];
    double bv[11];  // the body's angular momentum (4), mass, inertia (3) and momentum (3)
};

template <typename Real>
__device__ void thermalize_body(const SysDev &s, const BodyDev &bd, int64_t b, double kT, int thermalize,
                                uint64_t seed, uint64_t step, Real *xs, Real *vs, double *site_d, double *vpre,
                                const double *bsh, unsigned long long *counts, int32_t *cellid, int32_t *slot,
                                const BrickSiteBin *bbin, ThermLds &lds, uint32_t &st)
{
    double *sh = lds.sh, *sacc = lds.sacc, *dvw = lds.dvw;
    const int t = threadIdx.x;
    const int64_t B = s.B, S = s.S;
    const int r = find_sys_wave(s.body_off, s.nsys, b);  // called by whole blocks
    double q[4], A[3][3], R[3], Lbox[3];
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = bd.quat[i * B + b];
    quat_matrix(q, A);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        R[k] = bd.pos[k * B + b];
        Lbox[k] = (double)s.ncell[3 * r + k] * s.a;
    }
    const int64_t j0 = bd.site_off[b], j1 = bd.site_off[b + 1];
    const int64_t sbase = bd.site_off[s.body_off[r]];
    const uint64_t rep = s.replica0 + (uint64_t)r;
    // the body quantities of the closing update, loaded by 11 lanes now and
    // put in LDS after the sites (their latency hides behind the draws)
    double bvt = 0.0;
    if (t < 11) {
        const double *src = t < 4 ? bd.angmom + t * B
                            : t == 4 ? bd.mass
                            : t < 8  ? bd.inertia + (t - 5) * B
                                     : bd.mom + (t - 8) * B;
        bvt = src[b];
    }
    // a body of at most BODY_T sites is one chunk: each lane keeps its site's
    // thermal velocity for the closing pass instead of storing and reloading it
    const bool one = j1 - j0 <= BODY_T;
    double vkeep[3] = {0.0, 0.0, 0.0};
    double acc = 0.0;
    for (int64_t c0 = j0; c0 < j1; c0 += BODY_T) {
        const int64_t j = c0 + t;
        Real xr[3] = {(Real)0, (Real)0, (Real)0};
        if (j < j1) {
            const double dh[3] = {bd.site_d[j], bd.site_d[S + j], bd.site_d[2 * S + j]};
            double d[3], vt[3] = {0.0, 0.0, 0.0}, pv[3], c[3];
            matvec(A, dh, d);
            if (thermalize) {
                double z[3];
                st |= site_normals(seed, step, (uint64_t)(j - sbase), rep, z);
                const double sig = sqrt(kT / bd.site_m[j]);
#pragma unroll
                for (int k = 0; k < 3; ++k) vt[k] = sig * z[k];
            }
            const double mj = bd.site_m[j];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                site_d[k * S + j] = d[k];
                xr[k] = (Real)wrap_d(R[k] + d[k], Lbox[k], st);
                xs[k * S + j] = xr[k];
                if (one) vkeep[k] = vt[k];
                else vpre[k * S + j] = vt[k];
                pv[k] = mj * vt[k];
            }
            cross3(d, pv, c);
#pragma unroll
            for (int k = 0; k < 3; ++k) { sh[k * SH_PAD + t] = pv[k]; sh[(3 + k) * SH_PAD + t] = c[k]; }
        }
        __syncthreads();
        if (counts) {
            // bin this chunk's sites (all lanes take part in the run detection)
            const int32_t gc = (j < j1) ? cell_of_pos<Real>(s, r, xr[0], xr[1], xr[2], bsh, st) : -1;
            int hl, base;
            run_slots(gc, true, counts, hl, base);
            const int bb = __shfl(base, hl, 64);
            if (j < j1) {
                slot[s.N + j] = bb + ((threadIdx.x & 63) - hl);
                cellid[s.N + j] = gc;
            }
        } else if (bbin) {  // binned layout: the brick's site list (all lanes take part)
            brick_bin_site<Real>(s, *bbin, r, j < j1, j, xr, bsh, st);
        }
        ordered_add(sh, (int)((j1 - c0) < BODY_T ? (j1 - c0) : BODY_T), acc);
        __syncthreads();
    }
    if (t < 6) sacc[t] = acc;
    if (t < 11) lds.bv[t] = bvt;
    __syncthreads();
    if (t == 0) {
        double p[4], I[3], V[3], w[3];
#pragma unroll
        for (int i = 0; i < 4; ++i) p[i] = lds.bv[i];
        const double Mb = lds.bv[4];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            I[k] = lds.bv[5 + k];
            V[k] = lds.bv[8 + k] / Mb;
        }
        body_omega(q, p, A, I, w);
        double Vt[3], Lt[3], Lth[3], wth[3], wt[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) { Vt[k] = sacc[k] / Mb; Lt[k] = sacc[3 + k]; }
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
            const double vj = (dV[k] + c[k]) + (one ? vkeep[k] : vpre[k * S + j]);
            const Real vr = (Real)vj;
            if (!(vj - vj == 0.0)) st |= ST_NONFINITE;
            vs[k * S + j] = vr;
            vpre[k * S + j] = (double)vr;
        }
    }
}

template <typename Real>
__global__ __launch_bounds__(BODY_T) void k_thermalize(SysDev s, BodyDev bd, double kT, int thermalize, uint64_t seed,
                                                       const uint64_t *d_step, Real *xs, Real *vs, double *site_d,
                                                       double *vpre, uint32_t *status)
{
    __shared__ ThermLds lds;
    const int64_t b = blockIdx.x;
    if (b >= s.B) return;
    uint32_t st = 0;
    thermalize_body<Real>(s, bd, b, kT, thermalize, seed, *d_step, xs, vs, site_d, vpre, nullptr, nullptr, nullptr,
                          nullptr, nullptr, lds, st);
    flag(status, st);
}

// Body role of the first kernel (a whole BODY_T block): body b's grid shift
// into bsh, then its sites thermalized and binned for step `step`.
template <typename Real>
__device__ __forceinline__ void prep_body_block(const SysDev &s, const BodyDev &bd, int64_t b, double kT,
                                                int thermalize, uint64_t seed, uint64_t step, Real *xs, Real *vs,
                                                double *site_d, double *vpre, unsigned long long *counts,
                                                int32_t *cellid, int32_t *slot, double *bsh, ThermLds &th,
                                                uint32_t &st)
{
    const int rb = find_sys_wave(s.body_off, s.nsys, b);  // every lane of the block is here
    if (threadIdx.x == 64 || (BODY_T <= 64 && threadIdx.x == 0)) shift_of(s, seed, step, rb, bsh);
    thermalize_body<Real>(s, bd, b, kT, thermalize, seed, step, xs, vs, site_d, vpre, bsh, counts, cellid, slot, nullptr,
                          th, st);
}

// Solvent role of the first kernel (a whole BODY_T block): bin the PREP_CHUNK
// solvent particles from kbase for step `step`.  After the block's position
// loads are issued, wave 0 finds the system and draws the shift of the
// chunk's first particle and wave 1 (in parallel) those of its last.
template <typename Real>
__device__ __forceinline__ void prep_solvent_block(const SysDev &s, uint64_t seed, uint64_t step, const Real *x,
                                                   unsigned long long *counts, int32_t *cellid, int32_t *slot,
                                                   int64_t kbase, double *bsh, int *bsr, BinLds &bin, uint32_t &st)
{
    const int64_t k1 = s.N;
    const int64_t kl = ((kbase + PREP_CHUNK < k1) ? kbase + PREP_CHUNK : k1) - 1;
    BlockShift bs;
    bs.arr = nullptr; bs.lds = bsh; bs.sys = bsr; bs.seed = seed; bs.step = step;
    bin_chunk<Real, false>(s, x, nullptr, nullptr, bs, counts, cellid, slot, kbase, k1, bin, st, [&] {
        if (threadIdx.x < 128) {  // whole waves 0 and 1
            const int e = threadIdx.x >> 6;
            const int r = find_sys_wave(s.solv_off, s.nsys, e ? kl : kbase);
            if ((threadIdx.x & 63) == 0) {
                bsr[e] = r;
                shift_of(s, seed, step, r, bsh + 3 * e);
            }
        }
    });
}

// First kernel of a step: blocks [0, B) thermalize one body each and bin its
// sites; the remaining blocks bin PREP_CHUNK solvent particles each.  Every
// block draws the grid shifts it needs; block 0 also stores them.  PART 0 is
// that whole kernel; PART 1 its body blocks (with the shift store and the
// grid clearing) and PART 2 its solvent blocks, compiled without the body
// code, for a schedule that bins the solvent on another stream.
template <typename Real, int PART>
__global__ __launch_bounds__(BODY_T) void k_prep(SysDev s, BodyDev bd, double kT, int thermalize, uint64_t seed,
                                                 const uint64_t *d_step, const Real *x, Real *xs, Real *vs,
                                                 double *site_d, double *vpre, unsigned long long *counts,
                                                 int32_t *grid_count, int64_t grid_n, int32_t *cellid,
                                                 int32_t *slot, double *shift_out, uint32_t *status)
{
    __shared__ double bsh[6];
    __shared__ int bsr[2];
    __shared__ union {  // a block either thermalizes a body or bins solvent
        ThermLds th;
        BinLds bin;
    } lds;
    const uint64_t step = *d_step;
    uint32_t st = 0;
    if constexpr (PART != 2) {
        if (blockIdx.x == 0) draw_shifts(s, seed, step, shift_out);
        // clear the body-centre grid for this step's insertions (after the drift)
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; grid_count && q < grid_n;
             q += (int64_t)gridDim.x * blockDim.x)
            grid_count[q] = 0;
    }
    if (PART == 1 || (PART == 0 && (int64_t)blockIdx.x < s.B)) {
        if constexpr (PART != 2)
            prep_body_block<Real>(s, bd, blockIdx.x, kT, thermalize, seed, step, xs, vs, site_d, vpre, counts, cellid,
                                  slot, bsh, lds.th, st);
    } else {
        const int64_t kbase = ((int64_t)blockIdx.x - (PART == 0 ? s.B : 0)) * PREP_CHUNK;
        prep_solvent_block<Real>(s, seed, step, x, counts, cellid, slot, kbase, bsh, bsr, lds.bin, st);
    }
    flag(status, st);
}

// (a4) J_b = sum m (v - v_pre), K_b = sum d x m (v - v_pre) in site order;
// the result is valid in lanes 0..5 (component = lane) of a BODY_T block.
template <typename Real>
__device__ __forceinline__ double transfer_sums(const BodyDev &bd, int64_t S, int64_t b, const Real *vs,
                                                const double *site_d, const double *vpre, double *sh)
{
    const int t = threadIdx.x;
    const int64_t j0 = bd.site_off[b], j1 = bd.site_off[b + 1];
    double acc = 0.0;
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
            for (int k = 0; k < 3; ++k) { sh[k * SH_PAD + t] = mdv[k]; sh[(3 + k) * SH_PAD + t] = c[k]; }
        }
        __syncthreads();
        ordered_add(sh, (int)((j1 - c0) < BODY_T ? (j1 - c0) : BODY_T), acc);
        __syncthreads();
    }
    return acc;
}

template <typename Real>
__global__ __launch_bounds__(BODY_T) void k_sites_to_body(SysDev s, BodyDev bd, const Real *vs, const double *site_d,
                                                          const double *vpre, double *J, double *K)
{
    __shared__ double sh[6 * SH_PAD];
    const int64_t b = blockIdx.x;
    if (b >= s.B) return;
    const double acc = transfer_sums<Real>(bd, s.S, b, vs, site_d, vpre, sh);
    const int t = threadIdx.x;
    if (t < 3) J[t * s.B + b] = acc;
    else if (t < 6) K[(t - 3) * s.B + b] = acc;
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

// Impulse (J, K), half kick with the stored F, T, drift, NO_SQUISH rotation.
// ---- hashed grid of body centres (WCA neighbour search) -------------------
//
// Per system, ng = floor(0.999 L / rc) cells per axis (at least 1), so a cell
// is wider than the cutoff rc and every partner within rc of a body lies in one
// of the 27 cells around it (cells repeat when ng < 3).  Cells hash into a
// power-of-two table of GRID_K-slot buckets.  A bucket can also hold bodies of
// other cells or systems; the lookup filters by system and distance and visits
// each bucket once, so it finds exactly the partners of the all-pairs loop.

struct BodyGrid {
    int32_t *count;  // nullptr: no grid
    int32_t *body;
    uint32_t mask;
    double rc;
};

__device__ __forceinline__ void grid_geometry(const SysDev &s, int r, double rc, int ng[3], double cw[3])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double L = (double)s.ncell[3 * r + k] * s.a;
        int n = (int)floor((0.999 * L) / rc);
        n = n < 1 ? 1 : n;
        ng[k] = n;
        cw[k] = L / (double)n;
    }
}

__device__ __forceinline__ int grid_axis(double x, double w, int n)
{
    int c = (int)floor(x / w);
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

__device__ __forceinline__ uint32_t grid_hash(int r, int cx, int cy, int cz, uint32_t mask)
{
    return (((uint32_t)r * 73856093u) ^ ((uint32_t)cx * 19349663u) ^ ((uint32_t)cy * 83492791u) ^
            ((uint32_t)cz * 2654435761u)) & mask;
}

__device__ void grid_insert(const SysDev &s, const BodyDev &bd, const BodyGrid &g, int64_t b)
{
    const int r = find_sys(s.body_off, s.nsys, b);
    int ng[3];
    double cw[3];
    grid_geometry(s, r, g.rc, ng, cw);
    const int64_t B = s.B;
    const uint32_t h = grid_hash(r, grid_axis(bd.pos[b], cw[0], ng[0]), grid_axis(bd.pos[B + b], cw[1], ng[1]),
                                 grid_axis(bd.pos[2 * B + b], cw[2], ng[2]), g.mask);
    const int slot = atomicAdd(&g.count[h], 1);
    if (slot < GRID_K) g.body[(size_t)h * GRID_K + slot] = (int32_t)b;
}

__global__ void k_grid_insert(SysDev s, BodyDev bd, BodyGrid g)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < s.B) grid_insert(s, bd, g, b);
}

// ---- site-site WCA (mode 2) ----------------------------------------------
//
// Space-frame offsets d_j = A(q) dhat_j and unwrapped positions R + d_j of a
// body's sites at the force evaluation, written by the whole block.  A site
// farther than `reach` from its centre is flagged (the neighbour search
// relies on the bound).
struct SiteFrames {
    double *pos, *off;  // [3S] each; nullptr: not mode 2
    double reach;
};

__device__ void site_frames_body(const SysDev &s, const BodyDev &bd, int64_t b, const double pose[7],
                                 const SiteFrames &fr, uint32_t &st)
{
    const int64_t S = s.S;
    double A[3][3];
    quat_matrix(pose, A);
    const double lim = fr.reach * fr.reach;
    for (int64_t j = bd.site_off[b] + threadIdx.x; j < bd.site_off[b + 1]; j += blockDim.x) {
        const double dh[3] = {bd.site_d[j], bd.site_d[S + j], bd.site_d[2 * S + j]};
        double d[3];
        matvec(A, dh, d);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            fr.off[k * S + j] = d[k];
            fr.pos[k * S + j] = pose[4 + k] + d[k];
        }
        if (!((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2] <= lim)) st |= ST_REACH;
    }
}

__global__ __launch_bounds__(BODY_T) void k_site_frames(SysDev s, BodyDev bd, SiteFrames fr, uint32_t *status)
{
    const int64_t b = blockIdx.x;
    if (b >= s.B) return;
    const int64_t B = s.B;
    double pose[7];
#pragma unroll
    for (int i = 0; i < 4; ++i) pose[i] = bd.quat[i * B + b];
#pragma unroll
    for (int k = 0; k < 3; ++k) pose[4 + k] = bd.pos[k * B + b];
    uint32_t st = 0;
    site_frames_body(s, bd, b, pose, fr, st);
    flag(status, st);
}

__device__ void body_first_update(const SysDev &s, const BodyDev &bd, int64_t b, const double *Jb,
                                  const double *Kb, double dt, uint32_t &st, double *pose_out = nullptr)
{
    const int64_t B = s.B;
    const int r = find_sys(s.body_off, s.nsys, b);
    const double hdt = 0.5 * dt;
    double q[4], p[4], A[3][3], P[3], v3[3], h3[3], dq[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) { q[i] = bd.quat[i * B + b]; p[i] = bd.angmom[i * B + b]; }
    quat_matrix(q, A);
#pragma unroll
    for (int k = 0; k < 3; ++k) P[k] = bd.mom[k * B + b];
    if (Jb) {
#pragma unroll
        for (int k = 0; k < 3; ++k) P[k] = P[k] + Jb[k];
    }
    if (Kb) {
#pragma unroll
        for (int k = 0; k < 3; ++k) v3[k] = Kb[k];
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
    if (pose_out) {  // new q (4) and R (3) for the rest of the block
#pragma unroll
        for (int i = 0; i < 4; ++i) pose_out[i] = q[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) pose_out[4 + k] = bd.pos[k * B + b];
    }
}

__global__ void k_body_first(SysDev s, BodyDev bd, const double *J, const double *K, double dt,
                             uint32_t *status)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= s.B) return;
    uint32_t st = 0;
    double Jb[3], Kb[3];
    if (J)
        for (int k = 0; k < 3; ++k) Jb[k] = J[k * s.B + b];
    if (K)
        for (int k = 0; k < 3; ++k) Kb[k] = K[k * s.B + b];
    body_first_update(s, bd, b, J ? Jb : nullptr, K ? Kb : nullptr, dt, st);
    flag(status, st);
}

// Momentum transfer fused with the first half of the body update (one block
// per body); J and K are also written out.
// After the brick collision of step t (the step index is still t): clear the
// site counts and the overflow flags and counters that step read, ready for step t+1's
// site binning and for step t+1's writers (which count into this parity's
// overflow list).  The sub-region fills need no clearing: every valid
// sub-region is stored by its writer every step.  The brick kernel only reads
// these, so it can be launched again on the same input.
__device__ __forceinline__ void binned_finish(const BinnedDev &bn, uint64_t step)
{
    const int par = (int)(step & 1);
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    int32_t *flags = bn.oflag + (int64_t)par * bn.nbricks;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < bn.nbricks; q += nt) {
        bn.scnt[q] = 0;
        flags[q] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        bn.ctrl[BC_OVF0 + par] = 0;
        bn.ctrl[BC_SOVF] = 0;
    }
}

template <typename Real>
__global__ __launch_bounds__(BODY_T) void k_transfer_first(SysDev s, BodyDev bd, const Real *vs, const double *site_d,
                                                           const double *vpre, double *J, double *K, double dt,
                                                           BodyGrid grid, SiteFrames fr, uint32_t *status,
                                                           BinnedDev bn, const uint64_t *d_step)
{
    if (d_step) binned_finish(bn, *d_step);  // binned layout: the brick collision's fills are spent
    __shared__ double sh[6 * SH_PAD];
    __shared__ double jk[6];
    __shared__ double pose[7];
    const int64_t b = blockIdx.x;
    if (b >= s.B) return;
    const double acc = transfer_sums<Real>(bd, s.S, b, vs, site_d, vpre, sh);
    const int t = threadIdx.x;
    if (t < 6) jk[t] = acc;
    __syncthreads();
    if (t == 0) {
        uint32_t st = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) { J[k * s.B + b] = jk[k]; K[k * s.B + b] = jk[3 + k]; }
        body_first_update(s, bd, b, jk, jk + 3, dt, st, pose);
        if (grid.count) grid_insert(s, bd, grid, b);
        flag(status, st);
    }
    if (fr.pos) {
        __syncthreads();
        uint32_t st = 0;
        site_frames_body(s, bd, b, pose, fr, st);
        flag(status, st);
    }
}

// Core-shifted WCA between body centres, Eq. (1).  One wave per body.  With
// the body-centre grid, lanes evaluate the bodies of the 27 surrounding
// buckets and lane 0 adds the interacting partners' contributions in ascending
// partner index; without it (or when a bucket overflowed) lanes sweep all
// bodies of the system and lanes 0..2 add the x, y, z components in ascending
// partner index.  Either way the sums follow a sequential host loop over
// partners.  With kick != 0 the second half kick follows in the same lane
// (it needs only this body's new force); with advance_step != NULL block 0
// then advances the step counter (last kernel of a step).
constexpr int FRC_T = 64;

// LDS of the body forces for a block of NT threads.  The grid path keeps at
// most FRC_HCAP partners within the cutoff (a body with more takes the
// all-pairs path, with the same sums), so that the LDS stays small and many
// one-wave blocks share a CU.
constexpr int FRC_NCAND = 27 * GRID_K;
constexpr int FRC_HCAP = 96;
template <int NT> struct ForceLds {
    union {
        double sf[3][NT + 1];     // all-pairs path: each lane's contribution
        double hc[3][FRC_HCAP];  // grid path: the contributions of the hits
    };
    int shit[NT];
    double fsh[3];
    uint32_t s_h[27];
    int s_n[27], s_pre[28];
    int s_ovf, s_nhit;
    int hj[FRC_HCAP];
};

// The forces (and kick) of body i = blockIdx.x < B by a block of NT threads.
template <int NT>
__device__ void body_forces_block(const SysDev &s, const BodyDev &bd, const mpcd_wca &wca, const BodyGrid &grid,
                                  const ExtForce &E, double dt, int kick, uint64_t *advance_step, uint32_t *status,
                                  ForceLds<NT> &Lf)
{
    constexpr int NCAND = FRC_NCAND;
    auto &sf = Lf.sf;
    auto &shit = Lf.shit;
    auto &fsh = Lf.fsh;
    auto &s_h = Lf.s_h;
    auto &s_n = Lf.s_n;
    auto &s_pre = Lf.s_pre;
    int &s_ovf = Lf.s_ovf;
    int &s_nhit = Lf.s_nhit;
    auto &hj = Lf.hj;
    auto &hc = Lf.hc;
    (void)NCAND;
    const int64_t i = blockIdx.x;
    if (advance_step && i == 0 && threadIdx.x == 0) *advance_step = *advance_step + 1;
    const int t = threadIdx.x;
    const int64_t B = s.B;
    uint32_t st = 0;
    double f = 0.0;  // component t (lanes 0..2)
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
        const int64_t jb = s.body_off[r], je = s.body_off[r + 1];
        // grid path: the 27 buckets around this body, each once
        bool use_grid = grid.count != nullptr;
        if (use_grid) {
            int ng[3];
            double cw[3];
            grid_geometry(s, r, grid.rc, ng, cw);
            if (t == 0) {
                s_ovf = 0;
                s_nhit = 0;
            }
            if (t < 27) {
                const int d[3] = {t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1};
                int nc[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    int c = grid_axis(Ri[k], cw[k], ng[k]) + d[k];
                    c = c < 0 ? c + ng[k] : (c >= ng[k] ? c - ng[k] : c);
                    nc[k] = c;
                }
                s_h[t] = grid_hash(r, nc[0], nc[1], nc[2], grid.mask);
            }
            __syncthreads();
            if (t < 27) {
                const uint32_t h = s_h[t];
                bool dup = false;
                for (int u = 0; u < t; ++u) dup = dup || (s_h[u] == h);
                const int n = dup ? 0 : grid.count[h];
                if (n > GRID_K) s_ovf = 1;
                s_n[t] = n;
            }
            __syncthreads();
            if (t == 0) {
                int acc_n = 0;
                for (int u = 0; u < 27; ++u) {
                    s_pre[u] = acc_n;
                    acc_n += s_n[u] < GRID_K ? s_n[u] : GRID_K;
                }
                s_pre[27] = acc_n;
            }
            __syncthreads();
            use_grid = s_ovf == 0;  // a full bucket: fall back to all pairs
        }
        if (use_grid) {
            const int total = s_pre[27];
            for (int idx = t; idx < total; idx += NT) {
                int u = 0;
                while (u < 26 && s_pre[u + 1] <= idx) ++u;
                const int64_t j = grid.body[(size_t)s_h[u] * GRID_K + (idx - s_pre[u])];
                if (j == i || j < jb || j >= je) continue;
                double dr[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    double d = Ri[k] - bd.pos[k * B + j];
                    if (d > 0.5 * Lb[k]) d = d - Lb[k];
                    else if (d < -0.5 * Lb[k]) d = d + Lb[k];
                    dr[k] = d;
                }
                const double r2 = (dr[0] * dr[0] + dr[1] * dr[1]) + dr[2] * dr[2];
                if (!(r2 <= rc2)) continue;
                const double rr = sqrt(r2);
                const double sh = rr - wca.delta;
                if (!(sh > 0.0)) {
                    st |= ST_NONFINITE;
                    continue;
                }
                const double is = wca.sigma / sh;
                const double is2 = is * is;
                const double is6 = (is2 * is2) * is2;
                const double is12 = is6 * is6;
                const double fr = ((24.0 * wca.eps) * (2.0 * is12 - is6)) / sh;
                const double fo = fr / rr;
                const int pos = atomicAdd(&s_nhit, 1);
                if (pos < FRC_HCAP) {
                    hj[pos] = (int)j;
#pragma unroll
                    for (int k = 0; k < 3; ++k) hc[k][pos] = fo * dr[k];
                }
            }
            __syncthreads();
            use_grid = s_nhit <= FRC_HCAP;  // more partners than the list holds: all pairs
        }
        if (use_grid) {
            if (t == 0) {
                // partners in ascending index, then the sequential sums
                const int nh = s_nhit;
                for (int a = 1; a < nh; ++a) {
                    const int jk = hj[a];
                    const double c0 = hc[0][a], c1 = hc[1][a], c2 = hc[2][a];
                    int q = a;
                    while (q > 0 && hj[q - 1] > jk) {
                        hj[q] = hj[q - 1];
                        hc[0][q] = hc[0][q - 1]; hc[1][q] = hc[1][q - 1]; hc[2][q] = hc[2][q - 1];
                        --q;
                    }
                    hj[q] = jk;
                    hc[0][q] = c0; hc[1][q] = c1; hc[2][q] = c2;
                }
                double f0 = 0.0, f1 = 0.0, f2 = 0.0;
                for (int a = 0; a < nh; ++a) {
                    f0 = f0 + hc[0][a];
                    f1 = f1 + hc[1][a];
                    f2 = f2 + hc[2][a];
                }
                fsh[0] = f0; fsh[1] = f1; fsh[2] = f2;
            }
            __syncthreads();
            if (t < 3) f = fsh[t];
        }
        for (int64_t j0 = jb; !use_grid && j0 < je; j0 += NT) {
            const int64_t j = j0 + t;
            int hit = 0;
            double c[3] = {0.0, 0.0, 0.0};
            if (j < je && j != i) {
                double dr[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    double d = Ri[k] - bd.pos[k * B + j];
                    if (d > 0.5 * Lb[k]) d = d - Lb[k];
                    else if (d < -0.5 * Lb[k]) d = d + Lb[k];
                    dr[k] = d;
                }
                const double r2 = (dr[0] * dr[0] + dr[1] * dr[1]) + dr[2] * dr[2];
                if (r2 <= rc2) {
                    const double rr = sqrt(r2);
                    const double sh = rr - wca.delta;
                    if (sh > 0.0) {
                        const double is = wca.sigma / sh;
                        const double is2 = is * is;
                        const double is6 = (is2 * is2) * is2;
                        const double is12 = is6 * is6;
                        const double fr = ((24.0 * wca.eps) * (2.0 * is12 - is6)) / sh;
                        const double fo = fr / rr;
#pragma unroll
                        for (int k = 0; k < 3; ++k) c[k] = fo * dr[k];
                        hit = 1;
                    } else {
                        st |= ST_NONFINITE;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) sf[k][t] = c[k];
            shit[t] = hit;
            __syncthreads();
            if (t < 3) {
                const int cnt = (int)((je - j0) < NT ? (je - j0) : NT);
                for (int q = 0; q < cnt; ++q)
                    if (shit[q]) f = f + sf[t][q];
            }
            __syncthreads();
        }
    }
    if (t < 3) {
        if (E.on) f = f + E.f[t];  // external force at the centre
        fsh[t] = f;
        bd.force[t * B + i] = f;
        bd.torque[t * B + i] = 0.0;
    }
    __syncthreads();
    if (kick && t == 0) {
        // second half kick: P += dt/2 F; p += dt S(q)(0, A^T T)
        const double hdt = 0.5 * dt;
        double q[4], A[3][3], v3[3], h3[3], dq[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) q[k] = bd.quat[k * B + i];
        quat_matrix(q, A);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double Pk = bd.mom[k * B + i] + hdt * fsh[k];
            if (!(Pk - Pk == 0.0)) st |= ST_NONFINITE;
            bd.mom[k * B + i] = Pk;
            v3[k] = 0.0;
        }
        matTvec(A, v3, h3);
        qmul_pure(q, h3, dq);
#pragma unroll
        for (int k = 0; k < 4; ++k) bd.angmom[k * B + i] = bd.angmom[k * B + i] + dt * dq[k];
    }
    flag(status, st);
}

__global__ __launch_bounds__(FRC_T) void k_body_forces(SysDev s, BodyDev bd, mpcd_wca wca, BodyGrid grid, ExtForce E,
                                                       double dt, int kick, uint64_t *advance_step, uint32_t *status)
{
    __shared__ ForceLds<FRC_T> Lf;
    if ((int64_t)blockIdx.x >= s.B) {
        if (advance_step && blockIdx.x == 0 && threadIdx.x == 0) *advance_step = *advance_step + 1;
        return;
    }
    body_forces_block<FRC_T>(s, bd, wca, grid, E, dt, kick, advance_step, status, Lf);
}

// Last kernel of step t fused with the first kernel of step t+1 (a schedule
// of captured steps): blocks [0, B) compute body b's centre forces and second
// half kick (block 0 also advances the step counter), then thermalize body
// b's sites for step t+1 and bin them; the other blocks bin PREP_CHUNK
// particles each of the solvent step t wrote, for step t+1.  The index t+1
// comes from step_next, stored by step t's collision (the counter advances in
// this launch).  The body-centre grid is read here, so step t+1's scatter
// clears it.  One LDS union serves the three roles.
template <typename Real>
__global__ __launch_bounds__(BODY_T) void k_forces_prep(SysDev s, BodyDev bd, mpcd_wca wca, BodyGrid grid,
                                                        ExtForce E, double dt, uint64_t *advance_step, double kT,
                                                        int thermalize, uint64_t seed, const uint64_t *step_next,
                                                        const Real *x, Real *xs, Real *vs, double *site_d,
                                                        double *vpre, unsigned long long *counts, int32_t *cellid,
                                                        int32_t *slot, double *shift_out, uint32_t *status)
{
    __shared__ double bsh[6];
    __shared__ int bsr[2];
    __shared__ union {
        ForceLds<BODY_T> f;
        ThermLds th;
        BinLds bin;
    } lds;
    uint32_t st = 0;
    if ((int64_t)blockIdx.x < s.B) {
        body_forces_block<BODY_T>(s, bd, wca, grid, E, dt, 1, advance_step, status, lds.f);
        __syncthreads();  // the kick is stored (by thread 0, which reads it back); the LDS is free
        const uint64_t step = *step_next;
        if (blockIdx.x == 0) draw_shifts(s, seed, step, shift_out);
        prep_body_block<Real>(s, bd, blockIdx.x, kT, thermalize, seed, step, xs, vs, site_d, vpre, counts, cellid,
                              slot, bsh, lds.th, st);
    } else {
        prep_solvent_block<Real>(s, seed, *step_next, x, counts, cellid, slot, ((int64_t)blockIdx.x - s.B) * PREP_CHUNK,
                                 bsh, bsr, lds.bin, st);
    }
    flag(status, st);
}


// Site-site WCA (mode 2), one block per body.  The neighbour bodies (centres
// within 2 reach + rc, from the 27 surrounding buckets of a grid whose cells
// are at least that wide) are listed in ascending index; without the grid, or
// when a bucket overflowed, every body of the system is a candidate in
// ascending index.  Lane t takes site j of the chunk: f_j sums the pair forces
// of the candidates' sites within the cutoff, in ascending body and site index
// (a candidate whose centre is farther than reach + rc from the site cannot
// contribute and is skipped).  Lanes 0..5 then add f_j and d_j x f_j in site
// order.  With kick != 0 the second half kick follows; with advance_step set,
// block 0 advances the step counter.
// Minimum image t - L rint(t / L).  Within half a box the quotient rounds to
// a zero (ties to even at exactly one half) and the result is t itself (a
// negative zero becomes +0, as t - L rint(t / L) gives), so that case skips
// the division.
__device__ __forceinline__ double min_image(double t, double L)
{
    if (fabs(t) < 0.5 * L) return t + 0.0;
    return t - L * rint(t / L);
}

__global__ __launch_bounds__(BODY_T) void k_site_forces(SysDev s, BodyDev bd, mpcd_wca wca, BodyGrid grid,
                                                        SiteFrames fr, ExtForce E, double dt, int kick,
                                                        uint64_t *advance_step, uint32_t *status)
{
    constexpr int NCAND = 27 * GRID_K;
    __shared__ uint32_t s_h[27];
    __shared__ int s_n[27], s_pre[28];
    __shared__ int s_ovf, s_nnb;
    __shared__ int nb[NCAND];
    __shared__ double sh[6 * SH_PAD];
    __shared__ double sp[3][BODY_T];  // a chunk of one candidate body's site positions
    __shared__ float spf[3][BODY_T];  // and the same rounded to FP32, for a conservative pair filter
    __shared__ float sof[3][BODY_T];  // their offsets from that body's centre (minimum image), in FP32
    __shared__ double fT[6];
    const int64_t i = blockIdx.x;
    if (advance_step && i == 0 && threadIdx.x == 0) *advance_step = *advance_step + 1;
    if (i >= s.B) return;
    const int t = threadIdx.x;
    const int64_t B = s.B, S = s.S;
    uint32_t st = 0;
    const int r = find_sys(s.body_off, s.nsys, i);
    const double rc = wca.delta + 0x1.1f59ac3c7d6c0p+0 * wca.sigma;
    const double rc2 = rc * rc;
    double Lb[3], Ri[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        Lb[k] = (double)s.ncell[3 * r + k] * s.a;
        Ri[k] = bd.pos[k * B + i];
    }
    const int64_t jb = s.body_off[r], je = s.body_off[r + 1];
    // centre-distance bounds with a margin far above rounding
    const double reach_b = 2.0 * wca.reach + rc, cut_b = (reach_b * reach_b) * (1.0 + 1e-9) + 1e-12;
    const double reach_s = wca.reach + rc, cut_s = (reach_s * reach_s) * (1.0 + 1e-9) + 1e-12;
    // Wave cull of a candidate's sites.  Take a site j of this body within
    // reach_s of candidate centre C (offset e_j), and a site u of the
    // candidate (offset o_u, |o_u| <= reach), both as minimum images.  On an
    // axis longer than 2 reach + 2 rc, e_j - o_u is the pair's own minimum
    // image whenever the pair lies within rc (another image would put them at
    // least L - rc apart on that axis), so then |e_j - o_u| <= rc on every
    // axis.  A site u outside the box of the wave's e_j, grown by rc + 0.01
    // (far above the FP32 rounding of offsets this small), adds nothing to any
    // lane of the wave and is skipped.  On shorter boxes every site is kept.
    const bool cull = Lb[0] > 2.0 * (wca.reach + rc) + 0.1 && Lb[1] > 2.0 * (wca.reach + rc) + 0.1 &&
                      Lb[2] > 2.0 * (wca.reach + rc) + 0.1;
    const float grow = (float)(rc + 0.01);
    bool use_grid = grid.count != nullptr;
    if (use_grid) {
        int ng[3];
        double cw[3];
        grid_geometry(s, r, grid.rc, ng, cw);
        if (t == 0) {
            s_ovf = 0;
            s_nnb = 0;
        }
        if (t < 27) {
            const int d[3] = {t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1};
            int nc[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                int c = grid_axis(Ri[k], cw[k], ng[k]) + d[k];
                c = c < 0 ? c + ng[k] : (c >= ng[k] ? c - ng[k] : c);
                nc[k] = c;
            }
            s_h[t] = grid_hash(r, nc[0], nc[1], nc[2], grid.mask);
        }
        __syncthreads();
        if (t < 27) {
            const uint32_t h = s_h[t];
            bool dup = false;
            for (int u = 0; u < t; ++u) dup = dup || (s_h[u] == h);
            const int n = dup ? 0 : grid.count[h];
            if (n > GRID_K) s_ovf = 1;
            s_n[t] = n;
        }
        __syncthreads();
        if (t == 0) {
            int acc_n = 0;
            for (int u = 0; u < 27; ++u) {
                s_pre[u] = acc_n;
                acc_n += s_n[u] < GRID_K ? s_n[u] : GRID_K;
            }
            s_pre[27] = acc_n;
        }
        __syncthreads();
        use_grid = s_ovf == 0;
        if (use_grid) {
            for (int idx = t; idx < s_pre[27]; idx += BODY_T) {
                int u = 0;
                while (u < 26 && s_pre[u + 1] <= idx) ++u;
                const int64_t j = grid.body[(size_t)s_h[u] * GRID_K + (idx - s_pre[u])];
                if (j == i || j < jb || j >= je) continue;
                double d2 = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double d = min_image(Ri[k] - bd.pos[k * B + j], Lb[k]);
                    d2 = d2 + d * d;
                }
                if (d2 <= cut_b) nb[atomicAdd(&s_nnb, 1)] = (int)j;
            }
            __syncthreads();
            if (t == 0) {
                const int n = s_nnb;
                for (int a = 1; a < n; ++a) {
                    const int v = nb[a];
                    int q = a;
                    while (q > 0 && nb[q - 1] > v) {
                        nb[q] = nb[q - 1];
                        --q;
                    }
                    nb[q] = v;
                }
            }
            __syncthreads();
        }
    }
    const int ncand = use_grid ? s_nnb : (int)(je - jb);
    const int64_t j0 = bd.site_off[i], j1 = bd.site_off[i + 1];
    double acc = 0.0;
    for (int64_t c0 = j0; c0 < j1; c0 += BODY_T) {
        // one site of body i per thread; the candidate bodies in ascending
        // order, each one's sites staged through LDS in chunks and taken in
        // ascending order (the same pairs and sums as one site at a time)
        const int64_t j = c0 + t;
        const bool active = j < j1;
        double pj[3] = {0.0, 0.0, 0.0};
        if (active) {
            pj[0] = fr.pos[j];
            pj[1] = fr.pos[S + j];
            pj[2] = fr.pos[2 * S + j];
        }
        // FP32 filter: a pair whose FP32 minimum-image distance exceeds rc +
        // 0.01 is farther than rc in FP64 (the FP32 rounding of coordinates up
        // to 2^15 cell edges moves a separation by far less than 0.01), so it
        // adds nothing; every other pair takes the exact FP64 path
        const float pjf[3] = {(float)pj[0], (float)pj[1], (float)pj[2]};
        const float Lf[3] = {(float)Lb[0], (float)Lb[1], (float)Lb[2]};
        const float iLf[3] = {1.0f / Lf[0], 1.0f / Lf[1], 1.0f / Lf[2]};
        const float limf = (float)((rc + 0.01) * (rc + 0.01));
        double f[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < ncand; ++q) {
            const int64_t b2 = use_grid ? (int64_t)nb[q] : jb + q;
            if (b2 == i) continue;  // (uniform)
            bool near = false;
            float ef[3] = {0.0f, 0.0f, 0.0f};
            if (active) {
                double d2 = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double d = min_image(pj[k] - bd.pos[k * B + b2], Lb[k]);
                    ef[k] = (float)d;
                    d2 = d2 + d * d;
                }
                near = d2 <= cut_s;
            }
            if (!__syncthreads_or(near)) continue;  // no site of this chunk within reach of b2
            // the box of this wave's near sites (offsets from b2's centre)
            float lo[3], hi[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                lo[k] = near ? ef[k] : INFINITY;
                hi[k] = near ? ef[k] : -INFINITY;
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    lo[k] = fminf(lo[k], __shfl_xor(lo[k], o, 64));
                    hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], o, 64));
                }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                lo[k] -= grow;
                hi[k] += grow;
            }
            const bool wnear = __ballot(near) != 0;
            const int64_t k0 = bd.site_off[b2], k1 = bd.site_off[b2 + 1];
            for (int64_t kc = k0; kc < k1; kc += BODY_T) {
                const int nk = (int)((k1 - kc) < BODY_T ? (k1 - kc) : BODY_T);
                if (t < nk) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const double x = fr.pos[k * S + kc + t];
                        sp[k][t] = x;
                        spf[k][t] = (float)x;
                        sof[k][t] = (float)min_image(x - bd.pos[k * B + b2], Lb[k]);
                    }
                }
                __syncthreads();
                // 64 candidate sites at a time: the wave keeps those inside
                // its box and takes them in ascending order
                for (int u0 = 0; wnear && u0 < nk; u0 += 64) {
                    const int uq = u0 + (t & 63);
                    bool keep = uq < nk;
                    if (keep && cull) {
#pragma unroll
                        for (int k = 0; k < 3; ++k) keep = keep && sof[k][uq] >= lo[k] && sof[k][uq] <= hi[k];
                    }
                    for (unsigned long long m = __ballot(keep); m != 0; m &= m - 1) {
                        const int u = u0 + __builtin_ctzll(m);
                        if (!near) continue;
                        float r2f = 0.0f;
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            float d = pjf[k] - spf[k][u];
                            d = d - Lf[k] * rintf(d * iLf[k]);
                            r2f = r2f + d * d;
                        }
                        if (!(r2f <= limf)) continue;
                        double dr[3];
#pragma unroll
                        for (int k = 0; k < 3; ++k) dr[k] = min_image(pj[k] - sp[k][u], Lb[k]);
                        const double r2 = (dr[0] * dr[0] + dr[1] * dr[1]) + dr[2] * dr[2];
                        if (!(r2 <= rc2)) continue;
                        const double rr = sqrt(r2);
                        const double shf = rr - wca.delta;
                        if (!(shf > 0.0)) {
                            st |= ST_NONFINITE;
                            continue;
                        }
                        const double is = wca.sigma / shf;
                        const double is2 = is * is;
                        const double is6 = (is2 * is2) * is2;
                        const double is12 = is6 * is6;
                        const double frr = ((24.0 * wca.eps) * (2.0 * is12 - is6)) / shf;
                        const double fo = frr / rr;
#pragma unroll
                        for (int k = 0; k < 3; ++k) f[k] = f[k] + fo * dr[k];
                    }
                }
                __syncthreads();  // the chunk is consumed
            }
        }
        if (active) {
            const double d[3] = {fr.off[j], fr.off[S + j], fr.off[2 * S + j]};
            double c[3];
            cross3(d, f, c);
#pragma unroll
            for (int k = 0; k < 3; ++k) { sh[k * SH_PAD + t] = f[k]; sh[(3 + k) * SH_PAD + t] = c[k]; }
        }
        __syncthreads();
        ordered_add(sh, (int)((j1 - c0) < BODY_T ? (j1 - c0) : BODY_T), acc);
        __syncthreads();
    }
    if (t < 6) fT[t] = (E.on && t < 3) ? acc + E.f[t] : acc;  // external force at the centre
    __syncthreads();
    if (t == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            bd.force[k * B + i] = fT[k];
            bd.torque[k * B + i] = fT[3 + k];
        }
        if (kick) {
            const double hdt = 0.5 * dt;
            double q[4], A[3][3], v3[3], h3[3], dq[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) q[k] = bd.quat[k * B + i];
            quat_matrix(q, A);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double Pk = bd.mom[k * B + i] + hdt * fT[k];
                if (!(Pk - Pk == 0.0)) st |= ST_NONFINITE;
                bd.mom[k * B + i] = Pk;
                v3[k] = fT[3 + k];
            }
            matTvec(A, v3, h3);
            qmul_pure(q, h3, dq);
#pragma unroll
            for (int k = 0; k < 4; ++k) bd.angmom[k * B + i] = bd.angmom[k * B + i] + dt * dq[k];
        }
    }
    flag(status, st);
}

// ---------------------------------------------------------------------------
// Harmonic-bond comparator (Sec. II.B.1): bonded surface and centre sites
// moved by velocity Verlet.  One launch per Verlet step; blocks [0, nsb) take
// one surface site per thread, the next B blocks one centre each.  Positions
// are read from one buffer and written to the other, so every force of a step
// sees the positions of that step.  Phase 0: first half kick and drift (forces
// from the previous step); phase 1: new forces, second half kick of the
// previous step, first half kick and drift of the next; phase 2: new forces
// and the last second half kick; phase 3: forces only.

struct HarmDev {
    int64_t B, S;
    const int64_t *site_off;
    const int32_t *site_body;
    const int64_t *adj_off;
    const int32_t *adj;
    const double *adj_r0, *rc0, *site_m;
    double *vc, *fs, *fc;
    int32_t *imgs, *imgc;
    double mc, kb;
};

__device__ __forceinline__ void harm_bond(double kb, double r0, const double d[3], double f[3])
{
    const double r = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    const double fo = (-kb * (r - r0)) / r;
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] = f[k] + fo * d[k];
}

__device__ __forceinline__ void harm_drift(double &x, double v, double dt, double L, int32_t &img, uint32_t &st)
{
    double y = x + v * dt;
    if (y >= L) { y = y - L; img += 1; }
    else if (y < 0.0) { y = y + L; img -= 1; }
    if (!(y >= 0.0 && y <= L)) st |= (y != y) ? ST_NONFINITE : ST_ESCAPE;
    x = y;
}

__global__ __launch_bounds__(BODY_T) void k_harm_substep(SysDev s, HarmDev h, mpcd_wca wca, const double *xs_in,
                                                         double *xs_out, double *vs, const double *xc_in,
                                                         double *xc_out, double dt, int phase, int nsb,
                                                         uint32_t *status)
{
    __shared__ double sh[3 * SH_PAD];
    __shared__ double fsum[3];
    __shared__ int s_nhit;
    const int t = threadIdx.x;
    const int64_t S = h.S, B = h.B;
    const double hdt = 0.5 * dt;
    uint32_t st = 0;
    if ((int)blockIdx.x < nsb) {
        const int64_t j = (int64_t)blockIdx.x * BODY_T + t;
        if (j >= S) return;
        const int64_t b = h.site_body[j];
        const int r = find_sys(s.body_off, s.nsys, b);
        double Lb[3], xj[3], f[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Lb[k] = (double)s.ncell[3 * r + k] * s.a;
            xj[k] = xs_in[k * S + j];
        }
        if (phase == 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) f[k] = h.fs[k * S + j];
        } else {  // phases 1, 2, 3: forces at the input positions
            double d[3];
            for (int64_t e = h.adj_off[j]; e < h.adj_off[j + 1]; ++e) {
                const int64_t k2 = h.adj[e];
#pragma unroll
                for (int k = 0; k < 3; ++k) d[k] = min_image(xj[k] - xs_in[k * S + k2], Lb[k]);
                harm_bond(h.kb, h.adj_r0[e], d, f);
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) d[k] = min_image(xj[k] - xc_in[k * B + b], Lb[k]);
            harm_bond(h.kb, h.rc0[j], d, f);
#pragma unroll
            for (int k = 0; k < 3; ++k) h.fs[k * S + j] = f[k];
        }
        if (phase == 3) return;
        const double m = h.site_m[j];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double v = vs[k * S + j];
            if (phase >= 1) v = v + hdt * (f[k] / m);
            if (phase <= 1) {
                v = v + hdt * (f[k] / m);
                double x = xj[k];
                harm_drift(x, v, dt, Lb[k], h.imgs[k * S + j], st);
                xs_out[k * S + j] = x;
            }
            vs[k * S + j] = v;
        }
        flag(status, st);
        return;
    }
    const int64_t b = (int64_t)blockIdx.x - nsb;
    if (b >= B) return;
    const int r = find_sys(s.body_off, s.nsys, b);
    double Lb[3], xb[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        Lb[k] = (double)s.ncell[3 * r + k] * s.a;
        xb[k] = xc_in[k * B + b];
    }
    double f = 0.0;  // component t (lanes 0..2)
    if (phase >= 1) {
        // bonds to the centre, in site order
        const int64_t j0 = h.site_off[b], j1 = h.site_off[b + 1];
        for (int64_t c0 = j0; c0 < j1; c0 += BODY_T) {
            const int64_t j = c0 + t;
            if (j < j1) {
                double d[3], fj[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int k = 0; k < 3; ++k) d[k] = min_image(xb[k] - xs_in[k * S + j], Lb[k]);
                harm_bond(h.kb, h.rc0[j], d, fj);
#pragma unroll
                for (int k = 0; k < 3; ++k) sh[k * SH_PAD + t] = fj[k];
            }
            __syncthreads();
            if (t < 3) {
                const int cnt = (int)((j1 - c0) < BODY_T ? (j1 - c0) : BODY_T);
                for (int i = 0; i < cnt; ++i) f = f + sh[t * SH_PAD + i];
            }
            __syncthreads();
        }
        // WCA of Eq. (1) with the other centres, ascending index
        if (wca.mode == 1) {
            const double rc = wca.delta + 0x1.1f59ac3c7d6c0p+0 * wca.sigma;
            const double rc2 = rc * rc;
            const int64_t jb = s.body_off[r], je = s.body_off[r + 1];
            for (int64_t c0 = jb; c0 < je; c0 += BODY_T) {
                const int64_t b2 = c0 + t;
                int hit = 0;
                double c[3] = {0.0, 0.0, 0.0};
                if (b2 < je && b2 != b) {
                    double dr[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        double d = xb[k] - xc_in[k * B + b2];
                        if (d > 0.5 * Lb[k]) d = d - Lb[k];
                        else if (d < -0.5 * Lb[k]) d = d + Lb[k];
                        dr[k] = d;
                    }
                    const double r2 = (dr[0] * dr[0] + dr[1] * dr[1]) + dr[2] * dr[2];
                    if (r2 <= rc2) {
                        const double rr = sqrt(r2);
                        const double shf = rr - wca.delta;
                        if (shf > 0.0) {
                            const double is = wca.sigma / shf;
                            const double is2 = is * is;
                            const double is6 = (is2 * is2) * is2;
                            const double is12 = is6 * is6;
                            const double fr = ((24.0 * wca.eps) * (2.0 * is12 - is6)) / shf;
                            const double fo = fr / rr;
#pragma unroll
                            for (int k = 0; k < 3; ++k) c[k] = fo * dr[k];
                            hit = 1;
                        } else {
                            st |= ST_NONFINITE;
                        }
                    }
                }
                // compact the interacting partners, keeping ascending order
                const int pos = block_exclusive_scan<BODY_T>(hit, &s_nhit);
                const int nhit = s_nhit;
                if (hit) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) sh[k * SH_PAD + pos] = c[k];
                }
                __syncthreads();
                if (t < 3)
                    for (int i = 0; i < nhit; ++i) f = f + sh[t * SH_PAD + i];
                __syncthreads();
            }
        }
        if (t < 3) h.fc[t * B + b] = f;
    } else if (t < 3) {
        f = h.fc[t * B + b];
    }
    if (t < 3) fsum[t] = f;
    __syncthreads();
    if (t < 3 && phase != 3) {
        const int k = t;
        double v = h.vc[k * B + b];
        const double fk = fsum[k];
        if (phase >= 1) v = v + hdt * (fk / h.mc);
        if (phase <= 1) {
            v = v + hdt * (fk / h.mc);
            double x = xb[k];
            harm_drift(x, v, dt, Lb[k], h.imgc[k * B + b], st);
            xc_out[k * B + b] = x;
        }
        h.vc[k * B + b] = v;
    }
    flag(status, st);
}

// ---------------------------------------------------------------------------
// Reverse nonequilibrium shear (Sec. III.B, viscosity).  Solvent in the lower
// slab y0 <= y < y0 + dy is ranked by |v_x - target|, in the upper slab
// y1 <= y < y1 + dy by |v_x + target| (ties: lower identity first); the first
// np = min(npairs, n_lower, n_upper) of each exchange v_x pairwise.
//  1. k_rn_hist: per slab, member count (each block stores its own) and a
//     histogram of key bins; the last bin holds every key >= RN_KMAX and is
//     not counted, since a threshold never needs to look past it.
//  2. k_rn_thresh (one block): per slab, the smallest bin by which np members
//     have accumulated (a block prefix sum over the bins), else the last bin;
//     every member of the top np lies in a bin <= it.
//  3. k_rn_collect: the members in those bins (a superset of the top np).
//  4. k_rn_swap (one block): rank of each candidate in the (key, identity)
//     order, pairwise exchange of the first np (2 np distinct particles, one
//     thread per pair), the moved momentum m (v_lower - v_upper) added in rank
//     order, counters cleared.
// ctl words: [2..3] threshold bins, [4..5] candidates, [6] np (others unused).

struct RnArgs {
    double y0, y1, dy, target, m;
    int npairs;
    int32_t *hist, *bcnt, *ctl, *id, *kk;
    double *key;
};

template <typename Real>
__device__ __forceinline__ int rn_slab(const RnArgs &R, const Real *x, const Real *v, int64_t N, int64_t k,
                                       double &key)
{
    const double y = (double)x[N + k];
    const double vx = (double)v[k];
    if (y >= R.y0 && y < R.y0 + R.dy) {
        key = fabs(vx - R.target);
        return 0;
    }
    if (y >= R.y1 && y < R.y1 + R.dy) {
        key = fabs(vx + R.target);
        return 1;
    }
    return -1;
}

__device__ __forceinline__ int rn_bin(double key)
{
    const double b = key * ((double)RN_BINS / RN_KMAX);
    return b < (double)(RN_BINS - 1) ? (int)b : RN_BINS - 1;
}

template <typename Real>
__global__ __launch_bounds__(256) void k_rn_hist(RnArgs R, const Real *x, const Real *v, int64_t N)
{
    __shared__ int s_n[2];
    if (threadIdx.x < 2) s_n[threadIdx.x] = 0;
    __syncthreads();
    int n0 = 0, n1 = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (int64_t)gridDim.x * blockDim.x) {
        double key;
        const int sl = rn_slab(R, x, v, N, k, key);
        if (sl < 0) continue;
        const int b = rn_bin(key);
        if (b < RN_BINS - 1) atomicAdd(&R.hist[sl * RN_BINS + b], 1);
        n0 += sl == 0;
        n1 += sl == 1;
    }
    // slab counts: each block stores its own (a slab in brick order touches
    // most blocks; one address per slab would serialize them)
    if (n0) atomicAdd(&s_n[0], n0);
    if (n1) atomicAdd(&s_n[1], n1);
    __syncthreads();
    if (threadIdx.x < 2) R.bcnt[threadIdx.x * RN_HBLOCKS + blockIdx.x] = s_n[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_rn_thresh(RnArgs R)
{
    constexpr int PER = RN_BINS / 256;
    static_assert(RN_BINS % 256 == 0, "bins per thread");
    __shared__ int s_b[2], s_tot, s_n[2];
    const int t = threadIdx.x;
    if (t < 2) s_b[t] = RN_BINS - 1;
    // both slabs' bins and the histogram blocks' member counts, in flight together
    static_assert(RN_HBLOCKS % 256 == 0, "counts per thread");
    int hv[2][PER], sum[2] = {0, 0}, c0 = 0, c1 = 0;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl)
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            hv[sl][i] = R.hist[sl * RN_BINS + t * PER + i];
            sum[sl] += hv[sl][i];
        }
#pragma unroll
    for (int b = t; b < RN_HBLOCKS; b += 256) {
        c0 += R.bcnt[b];
        c1 += R.bcnt[RN_HBLOCKS + b];
    }
    (void)block_exclusive_scan<256, int>(c0, &s_n[0]);  // slab member counts
    (void)block_exclusive_scan<256, int>(c1, &s_n[1]);
    const int n0 = s_n[0], n1 = s_n[1];
    int np = R.npairs;
    if (n0 < np) np = n0;
    if (n1 < np) np = n1;
    if (np < 0) np = 0;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
        const int excl = block_exclusive_scan<256, int>(sum[sl], &s_tot);
        // the one thread whose bins carry the prefix across np: its first bin
        // by which np members have accumulated (else its last)
        if (np > 0 && excl < np && excl + sum[sl] >= np) {
            int cum = excl, b = PER - 1;
            bool found = false;
#pragma unroll
            for (int i = 0; i < PER - 1; ++i) {
                if (!found && cum + hv[sl][i] >= np) {
                    b = i;
                    found = true;
                }
                cum += hv[sl][i];
            }
            s_b[sl] = t * PER + b;
        }
    }
    __syncthreads();
    if (t < 2) R.ctl[2 + t] = (np == 0) ? -1 : s_b[t];
    if (t == 0) R.ctl[6] = np;
    for (int i = t; i < 2 * RN_BINS; i += blockDim.x) R.hist[i] = 0;  // ready for the next exchange
}

template <typename Real>
__global__ __launch_bounds__(256) void k_rn_collect(RnArgs R, const Real *x, const Real *v, const int32_t *tag,
                                                    int64_t N, uint32_t *status)
{
    uint32_t st = 0;
    const int th0 = R.ctl[2], th1 = R.ctl[3];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (int64_t)gridDim.x * blockDim.x) {
        double key;
        const int sl = rn_slab(R, x, v, N, k, key);
        if (sl < 0 || rn_bin(key) > (sl ? th1 : th0)) continue;
        const int pos = atomicAdd(&R.ctl[4 + sl], 1);
        if (pos >= 0 && pos < RN_CAP) {
            R.key[sl * RN_CAP + pos] = key;
            R.id[sl * RN_CAP + pos] = tag ? tag[k] : (int32_t)k;
            R.kk[sl * RN_CAP + pos] = (int32_t)k;
        } else {
            st |= ST_BINERR;
        }
    }
    flag(status, st);
}

template <typename Real>
__global__ __launch_bounds__(1024) void k_rn_swap(RnArgs R, Real *v, int64_t N, double *dp, uint32_t *status)
{
    __shared__ double sk[2][RN_CAP];
    __shared__ int32_t sid[2][RN_CAP], skk[2][RN_CAP];
    __shared__ int32_t sel[2][RN_MAXPAIRS];  // particle of rank r in each slab
    __shared__ double s_dm[RN_MAXPAIRS];
    const int t = threadIdx.x;
    // pairs to swap: never more than either slab's stored candidates
    int nc[2];
    for (int sl = 0; sl < 2; ++sl) {
        const int n = R.ctl[4 + sl];
        nc[sl] = n < 0 ? 0 : (n > RN_CAP ? RN_CAP : n);
    }
    int np = R.ctl[6];
    const bool short_list = np > nc[0] || np > nc[1];
    if (np > nc[0]) np = nc[0];
    if (np > nc[1]) np = nc[1];
    if (np > RN_MAXPAIRS) np = RN_MAXPAIRS;
    if (np < 0) np = 0;
    for (int i = t; i < 2 * RN_MAXPAIRS; i += blockDim.x) sel[i / RN_MAXPAIRS][i % RN_MAXPAIRS] = -1;
    // both candidate lists in one round trip, not waiting for the counts
    // (entries past a list's count are never read)
    for (int i = t; i < 2 * RN_CAP; i += blockDim.x) {
        const int sl = i / RN_CAP, j = i % RN_CAP;
        sk[sl][j] = R.key[i];
        sid[sl][j] = R.id[i];
        skk[sl][j] = R.kk[i];
    }
    __syncthreads();
    // rank in the (key, identity) order = number of candidates before it, both
    // slabs at once; the threads of a wave read the same entry j together (an
    // LDS broadcast)
    for (int q = t; q < nc[0] + nc[1]; q += blockDim.x) {
        const int sl = q < nc[0] ? 0 : 1;
        const int i = sl ? q - nc[0] : q;
        const int n = nc[sl];
        const double *sks = sk[sl];
        const int32_t *sis = sid[sl];
        {
            const double ki = sks[i];
            const int32_t ii = sis[i];
            int r = 0, j = 0;
            for (; j + 8 <= n; j += 8) {  // eight reads in flight per wait
                double kj[8];
                int32_t ij[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    kj[u] = sks[j + u];
                    ij[u] = sis[j + u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) r += (int)((kj[u] < ki) | ((kj[u] == ki) & (ij[u] < ii)));
            }
            for (; j < n; ++j) r += (int)((sks[j] < ki) | ((sks[j] == ki) & (sis[j] < ii)));
            if (r < np) sel[sl][r] = skk[sl][i];
        }
    }
    __syncthreads();
    // the 2 np particles are distinct (a particle is in one slab at most, and
    // once in its slab's list): one thread per pair
    uint32_t st = (t == 0 && short_list) ? ST_BINERR : 0u;
    for (int i = t; i < np; i += blockDim.x) {
        const int32_t kl = sel[0][i], ku = sel[1][i];
        if (kl < 0 || kl >= N || ku < 0 || ku >= N) {
            st |= ST_BINERR;
            s_dm[i] = 0.0;
            continue;
        }
        const Real vl = v[kl], vu = v[ku];
        v[kl] = vu;
        v[ku] = vl;
        s_dm[i] = R.m * ((double)vl - (double)vu);
    }
    flag(status, st);
    __syncthreads();
    if (t == 0) {
        double acc = *dp;
        int i = 0;
        for (; i + 8 <= np; i += 8) {  // rank order; the reads batched
            double d[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) d[u] = s_dm[i + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = acc + d[u];
        }
        for (; i < np; ++i) acc = acc + s_dm[i];
        *dp = acc;
    }
    if (t < 16) R.ctl[t] = 0;
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

// ---------------------------------------------------------------------------
// Binned step: one block per brick.
//
// The block loads its brick's members in one sweep: the solvent of the
// region's sub-regions (position, velocity, identity), the sites listed for
// the brick and any overflow entries addressed to it, kept in registers
// (ITEMS per thread).  While those loads are in flight, one lane per cell
// takes the cell's first random call (axis, Box-Muller pair, test uniforms).
// Each member's cell on this step's grid is local to the brick, so the cell
// sums are complete in LDS (FP32: exact int64 fixed-point sums with LDS
// atomics).  One lane per cell then finishes the thermostat variate from its
// member count and forms u and lambda R; every member is rotated, the sites'
// velocities are written back to the site arrays, and the solvent is
// streamed and written straight into the region of its brick on the NEXT
// step's grid, in the sub-region of this brick's class there, at the rank
// an LDS counter gives it.  The block stores the fill of each sub-region it
// writes.  The solvent therefore crosses HBM once per step (read and written
// once), with no cell lists, scan, scatter, permutation or device atomics.
// A brick with more members than the block holds in registers takes a
// two-pass path (sums, then a second load to rotate and write); so does a
// four-wave block with a cell whose thermostat variate needs more than the
// first random call (about one cell in ten thousand), whose further calls
// then run with no members held in registers.
// A brick block holds its members in registers, in one of two shapes.  Four
// waves of seven members per lane (1792; under 128 VGPRs, four waves per
// SIMD) with 35 KB of LDS leave four blocks resident per CU, against two for
// eight waves of four members per lane (2048), so more of the solvent is in
// flight; the eight-wave shape is faster when there are too few bricks to
// fill the CUs over several rounds.  Bricks are planned for 2048 members
// either way (their expected members and sites, with margins); the rare
// brick of a four-wave layout with more than 1792 takes the two-pass path.
constexpr int BRICK_PLAN_MEMBERS = 2048;    // members a planned brick may expect, margins included
constexpr int BRICK_MEMBERS_WIDE = 1792;    // members a four-wave block holds in registers
constexpr int BRICK_MEMBERS_NARROW = 2048;  // and an eight-wave block
constexpr int BRICK_MAXC = 256;      // cells per brick at most (one lane per cell)
constexpr int BRICK_OVL = 512;       // overflow entries per brick and kind a block takes
constexpr int BRICK_T_WIDE = 256;    // threads of a block of the many-brick shape (seven members per lane)
constexpr int BRICK_T_NARROW = 512;  // and of the few-brick shape (four per lane)
constexpr int64_t BRICK_WIDE_MIN = 4096;  // bricks from which the four-wave shape is used

// A binned solvent slot is one record: in FP32 seven values, 28 bytes
// (position, identity as the int32 bits of the fourth value, velocity), read
// and written as a 16-byte and a 12-byte access (4-byte aligned), so that a
// run of slots fills whole cache lines; in FP64 eight values, 64 bytes
// (position, identity as the bits of the fourth, velocity, one unused).
// The FP32 record accesses are nontemporal: each record is read once and
// written once per step, and the next step reads it only after the whole
// array has streamed through the caches.
constexpr int REC_F32 = 7, REC_F64 = 8;
typedef float f4u_t __attribute__((ext_vector_type(4), aligned(4)));  // a record's first 16 bytes
typedef float f3u_t __attribute__((ext_vector_type(3), aligned(4)));  // and its last 12

__device__ __forceinline__ void rec_load(const float *rec, int64_t q, float p[3], float w[3], int32_t &id)
{
    const float *r = rec + REC_F32 * q;
    const f4u_t a = __builtin_nontemporal_load((const f4u_t *)r);
    const f3u_t c = __builtin_nontemporal_load((const f3u_t *)(r + 4));
    p[0] = a.x; p[1] = a.y; p[2] = a.z;
    id = __float_as_int(a.w);
    w[0] = c.x; w[1] = c.y; w[2] = c.z;
}

__device__ __forceinline__ void rec_store(float *rec, int64_t q, const float p[3], const float w[3], int32_t id)
{
    float *r = rec + REC_F32 * q;
    f4u_t a;
    a.x = p[0]; a.y = p[1]; a.z = p[2]; a.w = __int_as_float(id);
    f3u_t c;
    c.x = w[0]; c.y = w[1]; c.z = w[2];
    __builtin_nontemporal_store(a, (f4u_t *)r);
    __builtin_nontemporal_store(c, (f3u_t *)(r + 4));
}

__device__ __forceinline__ void rec_load(const double *rec, int64_t q, double p[3], double w[3], int32_t &id)
{
    const double2 *r = (const double2 *)rec + 4 * q;
    const double2 a = r[0], c = r[1], e = r[2], f = r[3];
    p[0] = a.x; p[1] = a.y; p[2] = c.x;
    id = (int32_t)__double_as_longlong(c.y);
    w[0] = e.x; w[1] = e.y; w[2] = f.x;
}

__device__ __forceinline__ void rec_store(double *rec, int64_t q, const double p[3], const double w[3], int32_t id)
{
    double2 *r = (double2 *)rec + 4 * q;
    r[0] = make_double2(p[0], p[1]);
    r[1] = make_double2(p[2], __longlong_as_double((long long)id));
    r[2] = make_double2(w[0], w[1]);
    r[3] = make_double2(w[2], 0.0);
}

template <typename Real> struct BrickArgs {
    SysDev s;
    BinnedDev bn;
    const Real *rec;  // binned solvent records of this step: [cap] records
    Real *reco;       // and of the next step
    Real *xs, *vs;      // sites [3][S]
    const double *site_m;
    double cos_a, sin_a, kT_cell, dt;
    uint64_t seed;
    const uint64_t *d_step;
    double *shift_out;    // when set, block 0 stores the step's grid shifts there
    int32_t *grid_clear;  // body-centre grid cleared for this step's insertions
    int64_t grid_n;
    Forcing F;
    uint32_t *status;
};

struct BrickLds32 {
    unsigned long long acc[5 * BRICK_MAXC];
    int cnt[BRICK_MAXC];
    // per cell: the values of its first random call until its FP32 collision
    // parameters (u, lambda R) replace them; one lane forms both
    union {
        CellDrawPre pre;
        float par[12];
        double pad[9];  // a stride of 18 banks: the cells' parameters spread over the LDS banks
    } cell[BRICK_MAXC];
    unsigned char more[BRICK_MAXC];  // the cell's Gamma variate needs further calls
    int cpre[NCLS + 1];             // exclusive prefix of the input sub-region fills
    int32_t csub[NCLS + 1];         // this brick's sub-region offsets
    int wcnt[NCLS];                 // members written per class of this brick
    int32_t wdst[NCLS], wcap[NCLS]; // the region written with each class, its sub-region capacity
    int32_t woff[NCLS];             // and its first slot
    int32_t lovf[BRICK_OVL], lsovf[BRICK_OVL];
    double sh[3], sh1[3];
    int hdr[8];  // region members, sites, overflow solvent, overflow sites, the two list lengths,
                 // site overflow, solvent overflow flag
};

// The shift table of the parity of step u: u, then each system's grid shifts
// for steps u and u + 1 (threads of one block, strided over the systems).
__device__ __forceinline__ void binned_store_shifts(const SysDev &s, const BinnedDev &bn, uint64_t seed, uint64_t u)
{
    double *tab = bn.shtab + (int64_t)(u & 1) * (1 + 6 * (int64_t)s.nsys);
    for (int r = threadIdx.x; r < s.nsys; r += blockDim.x) {
        shift_of(s, seed, u, r, tab + 1 + 6 * r);
        shift_of(s, seed, u + 1, r, tab + 4 + 6 * r);
    }
    if (threadIdx.x == 0) tab[0] = (double)u;
}

// Member i of the brick: region solvent (sub-region by sub-region), listed
// sites, then overflow solvent and overflow sites; id is the solvent identity,
// or -(site + 1).
template <typename Real>
__device__ __forceinline__ bool brick_member(const BrickArgs<Real> &A, const BrickInfo &bi, int par_in, int i,
                                             const BrickLds32 &L, Real p[3], Real w[3], int32_t &id, uint32_t &st)
{
    const int64_t S = A.s.S;
    // the member counts and the own sub-region's bounds are uniform: scalar registers
    const int nreg = __builtin_amdgcn_readfirstlane(L.hdr[0]), nsite = __builtin_amdgcn_readfirstlane(L.hdr[1]);
    const int novf = __builtin_amdgcn_readfirstlane(L.hdr[2]), own = __builtin_amdgcn_readfirstlane(L.cpre[1]);
    int64_t j = -1;
    if (i < own) {  // most members are the brick's own (class 0), at its sub-region's start
        rec_load(A.rec, bi.off + __builtin_amdgcn_readfirstlane(L.csub[0]) + i, p, w, id);
        return true;
    }
    if (i < nreg) {
        int lo = 1, hi = NCLS - 1;  // the last sub-region c with cpre[c] <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L.cpre[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        rec_load(A.rec, bi.off + L.csub[lo] + (i - L.cpre[lo]), p, w, id);
        return true;
    }
    if (i < nreg + nsite) {
        j = A.bn.sslot[bi.soff + (i - nreg)];
    } else if (i < nreg + nsite + novf) {
        const int64_t k = L.lovf[i - nreg - nsite];
        const Real *o = (const Real *)A.bn.ovf_xv + (int64_t)par_in * 6 * BIN_OVF_CAP;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            p[d] = o[d * BIN_OVF_CAP + k];
            w[d] = o[(3 + d) * BIN_OVF_CAP + k];
        }
        id = A.bn.ovf_tag[(int64_t)par_in * BIN_OVF_CAP + k];
        return true;
    } else {
        j = A.bn.sovf[2 * L.lsovf[i - nreg - nsite - novf] + 1];
    }
    if (j < 0 || j >= S) {
        st |= ST_BINERR;
        return false;
    }
    p[0] = A.xs[j]; p[1] = A.xs[S + j]; p[2] = A.xs[2 * S + j];
    w[0] = A.vs[j]; w[1] = A.vs[S + j]; w[2] = A.vs[2 * S + j];
    id = -(int32_t)j - 1;
    return true;
}

// The FP32 grid of a brick's system, converted once per block: the shifts of
// this step and the next rounded to float, the cell edge or its inverse, the
// cells per axis (as int and float) and the brick geometry.  brick_axis_cell
// performs exactly the operations of axis_cell(float, ...), so cells agree
// bit for bit with every other binning.
struct BrickGrid {
    float sh[3], sh1[3];
    float mul, a;  // mul != 0: a is a power of two and cells use g * mul
    float nf[3];
    int n[3], lg[3], nb[3], bb0;
};

__device__ __forceinline__ BrickGrid brick_grid_of(const SysDev &s, const BinnedDev &bn, int r, const double *sh,
                                                   const double *sh1)
{
    // every value is uniform over the block: held in scalar registers
    auto uf = [](float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); };
    auto ui = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
    BrickGrid G;
    const int32_t *g = bn.sys_bg + 6 * r;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        G.sh[d] = uf((float)sh[d]);
        G.sh1[d] = uf((float)sh1[d]);
        G.n[d] = ui(s.ncell[3 * r + d]);
        G.nf[d] = uf((float)G.n[d]);
        G.lg[d] = ui(g[d]);
        G.nb[d] = ui(g[3 + d]);
    }
    G.mul = uf(s.inv_a != 0.0 ? (float)s.inv_a : 0.0f);
    G.a = uf((float)s.a);
    G.bb0 = ui(bn.sys_bb[r]);
    return G;
}

// Status conditions of a lane's members, gathered as lane masks and turned
// into status bits once (per member they would cost a few vector operations
// per test).
struct LaneFlags {
    bool nonfinite = false, escape = false, binerr = false;
    __device__ __forceinline__ uint32_t bits() const
    {
        return (nonfinite ? ST_NONFINITE : 0u) | (escape ? ST_ESCAPE : 0u) | (binerr ? ST_BINERR : 0u);
    }
};

// UNIT: the cell edge is 1, where g * mul is g itself (the same value, without
// the multiplier or the division path in the block's registers).
template <bool UNIT>
__device__ __forceinline__ int brick_axis_cell(float x, float sf, const BrickGrid &G, int d, LaneFlags &lf)
{
    // selects rather than branches: the per-member code stays one basic block
    const float g = x - sf;
    const float jf = floorf(UNIT ? g : (G.mul != 0.0f ? g * G.mul : g / G.a));
    const bool ok = jf >= -1.0f && jf <= G.nf[d];  // cells -1 .. n: at most one box edge off
    const bool nan = g != g;
    lf.nonfinite = lf.nonfinite || nan;
    lf.escape = lf.escape || (!ok && !nan);
    // exact in range; out of range the value is never selected
    const unsigned j = (unsigned)(int)jf;
    const unsigned n = (unsigned)G.n[d];
    // the periodic wrap: -1 -> n - 1, n -> 0, else unchanged (the least of
    // j, j + n and j - n as unsigned)
    const unsigned r = min(min(j, j + n), j - n);
    return ok ? (int)r : 0;
}

// Local cell of a member on this step's grid from the block's FP32 grid (-1
// and BINERR when the member is not in this brick: only with a corrupted state).
template <bool UNIT>
__device__ __forceinline__ int brick_local_cell_g(const BrickGrid &G, const BrickInfo &bi, const float p[3],
                                                  LaneFlags &lf)
{
    int lc[3];
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lc[d] = brick_axis_cell<UNIT>(p[d], G.sh[d], G, d, lf) - bi.org[d];
        in = in && (unsigned)lc[d] < (unsigned)bi.dim[d];
    }
    lf.binerr = lf.binerr || !in;
    return in ? (lc[2] * bi.dim[1] + lc[1]) * bi.dim[0] + lc[0] : -1;
}

// Local cell of a member on this step's grid (-1 and BINERR when the member is
// not in this brick: only with a corrupted state).
template <typename Real>
__device__ __forceinline__ int brick_local_cell(const SysDev &s, const BinnedDev &bn, const BrickInfo &bi, int64_t b,
                                                const Real p[3], const double *sh, uint32_t &st)
{
    const int r = bi.sys;
    int lc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lc[d] = axis_cell(p[d], sh[d], s.a, s.inv_a, s.ncell[3 * r + d], st) - bi.org[d];
        if ((unsigned)lc[d] >= (unsigned)bi.dim[d]) {  // the brick is cells org .. org + dim - 1
            st |= ST_BINERR;
            return -1;
        }
    }
    (void)bn;
    (void)b;
    return (lc[2] * bi.dim[1] + lc[1]) * bi.dim[0] + lc[0];
}

// The canonical index (within its system) of cell c of a brick.
__device__ __forceinline__ uint64_t brick_cell_canonical(const SysDev &s, const BrickInfo &bi, int c)
{
    const int r = bi.sys;
    const int cx = c % bi.dim[0], cy = (c / bi.dim[0]) % bi.dim[1], cz = c / (bi.dim[0] * bi.dim[1]);
    const int nx = s.ncell[3 * r], ny = s.ncell[3 * r + 1];
    return (uint64_t)(((int64_t)(bi.org[2] + cz) * ny + (bi.org[1] + cy)) * nx + (bi.org[0] + cx));
}

// A cell's count word: members in the low 16 bits, members whose mass term
// is in the mass sum (sites, and solvent whose terms overflowed and add
// nothing) in the high 16 bits.  The other solvent members' mass terms all
// equal the solvent's, so they are added per cell from the count rather
// than one LDS atomic each.
__device__ __forceinline__ int brick_cnt_members(int cw) { return cw & 0xffff; }

__device__ __forceinline__ void brick_sum_member(unsigned long long *acc, int *cnt, bool solvent, const long long q[5])
{
    const bool counted = solvent && q[0] != 0;  // q[0] is 0 when the terms overflowed
#pragma unroll
    for (int z = 0; z < 5; ++z)
        if (z > 0 || !solvent) atomicAdd(acc + z, (unsigned long long)q[z]);
    atomicAdd(cnt, counted ? 1 : 1 + (1 << 16));
}

// Per-cell FP32 parameters from the exact fixed-point sums (u and lambda R
// rounded to float), the draws finished from the cell's first call.
//
// FIRST: only call 0's two Gamma tests; false (and par untouched) when both
// reject, and the cell is then finished by the full form, which repeats
// those tests and continues the stream exactly as cell_draw_post does.  The
// brick block holding its members in registers takes this form, so that
// the further generator calls, which are rare, do not add to its registers.
template <bool FIRST>
__device__ __forceinline__ bool brick_cell_params_f32(const SysDev &s, const BrickInfo &bi, int c, int cw,
                                                      long long q0_solvent, const unsigned long long *acc,
                                                      const CellDrawPre &P, double ca, double sa, double kT_cell,
                                                      uint64_t seed, uint64_t step, float *par, uint32_t &st)
{
    const int n = brick_cnt_members(cw);
    CellDraw D;
    if (FIRST) {
        if (!cell_draw_first(P, kT_cell > 0.0, 0.5 * (double)(3 * (n - 1)), D)) return false;
    } else {
        st |= cell_draw_post(seed, step, brick_cell_canonical(s, bi, c), s.replica0 + (uint64_t)bi.sys, P,
                             kT_cell > 0.0, 0.5 * (double)(3 * (n - 1)), D);
    }
    long long q[5];
#pragma unroll
    for (int z = 0; z < 5; ++z) q[z] = (long long)acc[5 * c + z];
    // the solvent's mass terms, all equal, from their count (exact: the same
    // int64 sum as adding each one)
    q[0] += (long long)(n - (cw >> 16)) * q0_solvent;
    const Rot R = rotation(D.n, ca, sa);
    const double Md = (double)q[0];
    const double u0 = (double)q[1] / Md, u1 = (double)q[2] / Md, u2 = (double)q[3] / Md;
    double lam = 1.0;
    if (kT_cell > 0.0) {
        const double E = fixed_energy(q);
        if (E > 0.0) lam = sqrt((kT_cell * D.g) / E);
    }
    par[0] = (float)u0; par[1] = (float)u1; par[2] = (float)u2;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) par[3 + 3 * i + j] = (float)(lam * R.R[i][j]);
    return true;
}

// Rotation of one FP32 member about its cell's mean velocity (cells of fewer
// than two members are left alone).
__device__ __forceinline__ void brick_rotate_f32(const float *par, float w[3], uint32_t &st)
{
    const float dl[3] = {w[0] - par[0], w[1] - par[1], w[2] - par[2]};
    bool fin = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        w[d] = par[d] + ((par[3 + 3 * d] * dl[0] + par[4 + 3 * d] * dl[1]) + par[5 + 3 * d] * dl[2]);
        fin = fin && (w[d] - w[d] == 0.0f);
    }
    st |= fin ? 0u : ST_NONFINITE;
}

// Streaming of a solvent member (position and velocity in place) and the
// class of this brick in the region of its brick on the next step's grid (-1
// beyond the neighbouring bricks; *dst receives that brick).
template <typename Real>
__device__ __forceinline__ int brick_stream(const BrickArgs<Real> &A, const BrickInfo &bi, const Real L[3], Real p[3],
                                            Real w[3], const double *sh1, int32_t *dst, uint32_t &st)
{
    const Real dtr = (Real)A.dt;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        Real y = p[d] + w[d] * dtr;
        if (A.F.on) {
            y = y + (Real)A.F.h[d];
            w[d] = w[d] + (Real)A.F.gdt[d];
        }
        p[d] = Prec<Real>::wrap(y, L[d], st);
    }
    int jc[3];
    const double shv[3] = {sh1[0], sh1[1], sh1[2]};
    *dst = brick_of_pos<Real>(A.s, A.bn, bi.sys, p[0], p[1], p[2], shv, jc, st);
    const int32_t *g = A.bn.sys_bg + 6 * bi.sys;
    int cls = 0, mul = 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int c = class_code(bi.org[d] >> g[d], jc[d] >> g[d], g[3 + d]);
        if (c < 0) return -1;
        cls += c * mul;
        mul *= 3;
    }
    return cls;
}

// Streaming of a solvent member with the block's FP32 grid (the same
// operations as brick_stream): its writer class in the region of its brick on
// the next step's grid, or -1 beyond the neighbouring bricks with *dst that
// brick.
template <bool UNIT>
__device__ __forceinline__ int brick_stream_g(const BrickArgs<float> &A, const BrickGrid &G, const BrickInfo &bi,
                                              const float L[3], float p[3], float w[3], int32_t *dst, LaneFlags &lf)
{
    const float dtr = (float)A.dt;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float y = p[d] + w[d] * dtr;
        if (A.F.on) {
            y = y + (float)A.F.h[d];
            w[d] = w[d] + (float)A.F.gdt[d];
        }
        // the periodic wrap of wrap_f, as selects
        y = y >= L[d] ? y - L[d] : (y < 0.0f ? y + L[d] : y);
        const bool nan = y != y;
        lf.nonfinite = lf.nonfinite || nan;
        lf.escape = lf.escape || (!(y >= 0.0f && y <= L[d]) && !nan);
        p[d] = y;
    }
    int jc[3], cls = 0, mul = 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        jc[d] = brick_axis_cell<UNIT>(p[d], G.sh1[d], G, d, lf);
        // class_code as selects
        int e = (bi.org[d] >> G.lg[d]) - (jc[d] >> G.lg[d]);
        e = e < 0 ? e + G.nb[d] : e;
        const int c = e == 0 ? 0 : e == 1 ? 1 : e == G.nb[d] - 1 ? 2 : -1;
        cls = (c < 0 || cls < 0) ? -1 : cls + c * mul;
        mul *= 3;
    }
    if (cls < 0)
        *dst = G.bb0 + ((jc[2] >> G.lg[2]) * G.nb[1] + (jc[1] >> G.lg[1])) * G.nb[0] + (jc[0] >> G.lg[0]);
    return cls;
}

// Write one new solvent member into slot `slot` of the sub-region at `off` (of
// capacity `cap`) of the output, or into the overflow list for brick b.
template <typename Real>
__device__ __forceinline__ void brick_put(const BrickArgs<Real> &A, int par_out, int32_t b, int64_t off, int32_t cap,
                                          int32_t slot, const Real p[3], const Real w[3], int32_t id, uint32_t &st)
{
    if (slot < cap) {
        rec_store(A.reco, off + slot, p, w, id);
        return;
    }
    const int e = atomicAdd(&A.bn.ctrl[BC_OVF0 + par_out], 1);
    if (e >= BIN_OVF_CAP) {
        st |= ST_BINERR;
        return;
    }
    Real *o = (Real *)A.bn.ovf_xv + (int64_t)par_out * 6 * BIN_OVF_CAP;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        o[d * BIN_OVF_CAP + e] = p[d];
        o[(3 + d) * BIN_OVF_CAP + e] = w[d];
    }
    A.bn.ovf_tag[(int64_t)par_out * BIN_OVF_CAP + e] = id;
    A.bn.ovf_dest[(int64_t)par_out * BIN_OVF_CAP + e] = b;
    A.bn.oflag[(int64_t)par_out * A.bn.nbricks + b] = 1;  // any writer may store it: no atomic needed
}

// A streamed solvent member into its class's sub-region of the next step's
// region (rank from the block's LDS counter), or the overflow list.
template <typename Real>
__device__ __forceinline__ void brick_emit(const BrickArgs<Real> &A, BrickLds32 &L, int par_out, int cls, int32_t dst,
                                           const Real p[3], const Real w[3], int32_t id, uint32_t &st)
{
    if (cls < 0) {
        brick_put<Real>(A, par_out, dst, 0, 0, 0, p, w, id, st);  // beyond the neighbouring bricks
        return;
    }
    const int rank = atomicAdd(&L.wcnt[cls], 1);
    brick_put<Real>(A, par_out, dst, L.woff[cls], L.wcap[cls], rank, p, w, id, st);
}

template <int BRICK_T, bool UNIT>
__global__ __launch_bounds__(BRICK_T) __attribute__((amdgpu_waves_per_eu(4))) void
k_brick_collide_f32(BrickArgs<float> A)
{
    constexpr int ITEMS = (BRICK_T == BRICK_T_WIDE ? BRICK_MEMBERS_WIDE : BRICK_MEMBERS_NARROW) / BRICK_T;
    __shared__ BrickLds32 L;
    const int t = threadIdx.x;
    const SysDev &s = A.s;
    const BinnedDev &bn = A.bn;
    const uint64_t step = *A.d_step;
    const int par_in = (int)(step & 1), par_out = par_in ^ 1;
    uint32_t st = 0;
    LaneFlags lf;  // status conditions of the fast path's members
    const int64_t b = tile_of_block((int)bn.nbricks);
    if (b < bn.nbricks) {
        const BrickInfo bi = bn.brick[b];
        const int r = bi.sys;
        const int ncb = bi.dim[0] * bi.dim[1] * bi.dim[2];
        // The brick's own sub-region starts its region, and at 2 or more
        // solvent per cell its first 2 ncb slots are as good as always filled:
        // each lane loads its first members (512 per block at most) from there
        // before the header arrives.  One beyond the fill is discarded and
        // loaded again from its place; the slots read stay within the region.
        constexpr int KSPEC = 512 / BRICK_T;
        const int spec = min(min(512, 2 * ncb), bi.cap);
        float p[ITEMS][3], w[ITEMS][3];
        int32_t id[ITEMS];
#pragma unroll
        for (int k = 0; k < KSPEC; ++k) {
            const int i = t + k * BRICK_T;
            id[k] = 0;
            if (i < spec) rec_load(A.rec, bi.off + i, p[k], w[k], id[k]);
        }
        // wave 0 reads the brick's header in one round: the input fills (a
        // sub-region without a writer has capacity 0) and their exclusive
        // prefix, the sub-regions this brick writes, the site count, the
        // overflow flag and list lengths, and the grid shifts of this step and
        // the next from the table the previous launch (or the packing) stored,
        // drawn here if it is stale.
        int v = 0, s0 = 0, s1 = 0, nsc = 0, ofl = 0, ovl = 0, sovl = 0;
        int4 wt = make_int4(0, 0, 0, 0);
        double tab0 = 0.0, tabw = 0.0;
        if (t < NCLS) {
            const int32_t *sp = bn.subpre + b * (NCLS + 1);
            s0 = sp[t];
            s1 = sp[t + 1];
            v = bn.cnt[((int64_t)par_in * bn.nbricks + b) * NCLS + t];
            wt = bn.wtab[b * NCLS + t];  // the sub-region this brick writes with class t
        }
        if (t == 32) nsc = bn.scnt[b];
        if (t == 33) ofl = bn.oflag[(int64_t)par_in * bn.nbricks + b];
        if (t == 34) ovl = bn.ctrl[BC_OVF0 + par_in];
        if (t == 35) sovl = bn.ctrl[BC_SOVF];
        if (t >= 40 && t < 46) {
            const double *tab = bn.shtab + (int64_t)par_in * (1 + 6 * (int64_t)s.nsys);
            tab0 = tab[0];
            tabw = tab[1 + 6 * r + (t - 40)];
        }
        if (t < 64) {
            if (t < NCLS) {
                L.csub[t] = s0;
                if (t == NCLS - 1) L.csub[NCLS] = s1;
                v = min(v, s1 - s0);
                L.wcnt[t] = 0;
                L.woff[t] = wt.x;
                L.wcap[t] = wt.y;
                L.wdst[t] = wt.z;
            }
            if (t == 32) {
                L.hdr[1] = min(nsc, (int)bi.scap);
                L.hdr[6] = nsc > (int)bi.scap;  // sites of this brick in the site overflow list
            }
            if (t == 33) L.hdr[7] = ofl;
            if (t == 34) L.hdr[4] = min(ovl, BIN_OVF_CAP);
            if (t == 35) L.hdr[5] = min(sovl, bn.sovf_cap);
            if (t == 36) {
                L.hdr[2] = 0;
                L.hdr[3] = 0;
            }
            if (t >= 40 && t < 46) {
                const int k = t - 40;
                if (tab0 == (double)step) {
                    if (k < 3) L.sh[k] = tabw;
                    else L.sh1[k - 3] = tabw;
                } else if (k == 0) {
                    shift_of(s, A.seed, step, r, L.sh);
                } else if (k == 1) {
                    shift_of(s, A.seed, step + 1, r, L.sh1);
                }
            }
            int a = v;
#pragma unroll
            for (int o = 1; o < 32; o <<= 1) {
                const int u = __shfl_up(a, o, 64);
                if ((t & 63) >= o) a += u;
            }
            if (t <= NCLS) L.cpre[t] = a - v;
            if (t == NCLS - 1) L.hdr[0] = a;
        }
        for (int c = t; c < ncb; c += BRICK_T) {
            L.cnt[c] = 0;
#pragma unroll
            for (int z = 0; z < 5; ++z) L.acc[5 * c + z] = 0ull;
        }
        __syncthreads();
        if (L.hdr[6] || L.hdr[7]) {  // (uniform) overflow entries may be addressed to this brick
            if (L.hdr[7])
                for (int e = t; e < L.hdr[4]; e += BRICK_T)
                    if (bn.ovf_dest[(int64_t)par_in * BIN_OVF_CAP + e] == (int32_t)b) {
                        const int k = atomicAdd(&L.hdr[2], 1);
                        if (k < BRICK_OVL) L.lovf[k] = e;
                    }
            if (L.hdr[6])
                for (int e = t; e < L.hdr[5]; e += BRICK_T)
                    if (bn.sovf[2 * e] == (int32_t)b) {
                        const int k = atomicAdd(&L.hdr[3], 1);
                        if (k < BRICK_OVL) L.lsovf[k] = e;
                    }
            __syncthreads();
            if (L.hdr[2] > BRICK_OVL || L.hdr[3] > BRICK_OVL) {
                st |= ST_BINERR;
                __syncthreads();
                if (t == 0) {
                    L.hdr[2] = min(L.hdr[2], BRICK_OVL);
                    L.hdr[3] = min(L.hdr[3], BRICK_OVL);
                }
                __syncthreads();
            }
        }
        const int nmem = L.hdr[0] + L.hdr[1] + L.hdr[2] + L.hdr[3];
        const BrickGrid G = brick_grid_of(s, bn, r, L.sh, L.sh1);
        const double mS_solvent = s.m * FIX_SCALE;  // the solvent's fixed-point mass, once
        const long long q0_solvent = fix_round_any(mS_solvent);
        const float Lb[3] = {(float)((double)s.ncell[3 * r] * s.a), (float)((double)s.ncell[3 * r + 1] * s.a),
                             (float)((double)s.ncell[3 * r + 2] * s.a)};
        bool more = false;  // a cell of the register path needs further Gamma calls
        if (nmem <= ITEMS * BRICK_T) {
            int lc[ITEMS];
            const int own = __builtin_amdgcn_readfirstlane(L.cpre[1]);
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int i = t + k * BRICK_T;
                lc[k] = -1;
                if (k < KSPEC && i < spec && i < own) {
                    lc[k] = 0;  // loaded before the header
                } else {
                    id[k] = 0;
                    if (i < nmem && brick_member<float>(A, bi, par_in, i, L, p[k], w[k], id[k], st)) lc[k] = 0;
                }
            }
            // the cells' first random calls while the member loads are in flight
            for (int c = t; c < ncb; c += BRICK_T)
                cell_draw_pre(A.seed, step, brick_cell_canonical(s, bi, c), s.replica0 + (uint64_t)r, L.cell[c].pre);
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                if (lc[k] < 0) continue;
                lc[k] = brick_local_cell_g<UNIT>(G, bi, p[k], lf);
                if (lc[k] < 0) continue;
                long long q[5];
                if (id[k] >= 0) {
                    fixed_terms_scaled(mS_solvent, q0_solvent, w[k][0], w[k][1], w[k][2], q, st);
                } else {
                    fixed_terms(A.site_m[-(int64_t)id[k] - 1], w[k][0], w[k][1], w[k][2], q, st);
                }
                brick_sum_member(L.acc + 5 * lc[k], &L.cnt[lc[k]], id[k] >= 0, q);
            }
            __syncthreads();
            // the four-wave block takes only call 0's Gamma tests here; a cell
            // whose variate needs further calls (about one in ten thousand)
            // makes the block finish from a second load of its members.  The
            // eight-wave block, whose occupancy the registers of the further
            // calls do not lower, draws in full.
            constexpr bool SPLIT = BRICK_T == BRICK_T_WIDE;
            bool pend = false;
            for (int c = t; c < ncb; c += BRICK_T)
                if (brick_cnt_members(L.cnt[c]) >= 2) {
                    const bool done =
                        brick_cell_params_f32<SPLIT>(s, bi, c, L.cnt[c], q0_solvent, L.acc, L.cell[c].pre, A.cos_a,
                                                     A.sin_a, A.kT_cell, A.seed, step, L.cell[c].par, st);
                    L.more[c] = !done;
                    pend = pend || !done;
                }
            more = SPLIT ? __syncthreads_or(pend) : (__syncthreads(), false);
          if (!more) {
            // rotate and stream every member and take its rank in its class
            // from the LDS counters; the stores wait until the counts are final
            // (a barrier after global stores would wait for their completion)
            int rank[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                if (lc[k] < 0) continue;
                if (brick_cnt_members(L.cnt[lc[k]]) >= 2) brick_rotate_f32(L.cell[lc[k]].par, w[k], st);
                if (id[k] < 0) continue;  // a site: written back below
                int32_t dst = 0;
                const int cls = brick_stream_g<UNIT>(A, G, bi, Lb, p[k], w[k], &dst, lf);
                lc[k] = cls >= 0 ? cls : NCLS;  // NCLS: beyond the neighbouring bricks
                rank[k] = cls > 0 ? atomicAdd(&L.wcnt[cls], 1) : dst;  // the own class: below
            }
            {
                // the brick's own class (most members): one LDS atomic per wave
                // for all of its lanes' items, then each member's rank from the
                // ballots, item by item
                const int lane = threadIdx.x & 63;
                const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
                int tot = 0;
#pragma unroll
                for (int k = 0; k < ITEMS; ++k) tot += __popcll(__ballot(lc[k] == 0 && id[k] >= 0));
                int base = 0;
                if (lane == 0 && tot > 0) base = atomicAdd(&L.wcnt[0], tot);
                base = __shfl(base, 0, 64);
#pragma unroll
                for (int k = 0; k < ITEMS; ++k) {
                    const bool own = lc[k] == 0 && id[k] >= 0;
                    const unsigned long long m = __ballot(own);
                    if (own) rank[k] = base + __popcll(m & below);
                    base += __popcll(m);
                }
            }
            __syncthreads();
            if (t < NCLS && L.wdst[t] >= 0)  // the fill of every sub-region this brick writes (zero included)
                bn.cnt[((int64_t)par_out * bn.nbricks + L.wdst[t]) * NCLS + t] = L.wcnt[t];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                if (lc[k] < 0) continue;
                if (id[k] < 0) {  // a site: its new velocity back to the site arrays
                    const int64_t j = -(int64_t)id[k] - 1, S = s.S;
                    A.vs[j] = w[k][0]; A.vs[S + j] = w[k][1]; A.vs[2 * S + j] = w[k][2];
                } else if (lc[k] == NCLS) {
                    brick_put<float>(A, par_out, rank[k], 0, 0, 0, p[k], w[k], id[k], st);
                } else {
                    const int c = lc[k];
                    brick_put<float>(A, par_out, L.wdst[c], L.woff[c], L.wcap[c], rank[k], p[k], w[k], id[k], st);
                }
            }
          }
        } else {
            // more members than the block holds: sums over chunks of the
            // member list, then a second load of each member to rotate it
            for (int c = t; c < ncb; c += BRICK_T)
                cell_draw_pre(A.seed, step, brick_cell_canonical(s, bi, c), s.replica0 + (uint64_t)r, L.cell[c].pre);
            for (int i = t; i < nmem; i += BRICK_T) {
                float p[3], w[3];
                int32_t id;
                if (!brick_member<float>(A, bi, par_in, i, L, p, w, id, st)) continue;
                const int c = brick_local_cell<float>(s, bn, bi, b, p, L.sh, st);
                if (c < 0) continue;
                long long q[5];
                if (id >= 0) {
                    fixed_terms_scaled(mS_solvent, q0_solvent, w[0], w[1], w[2], q, st);
                } else {
                    fixed_terms(A.site_m[-(int64_t)id - 1], w[0], w[1], w[2], q, st);
                }
                brick_sum_member(L.acc + 5 * c, &L.cnt[c], id >= 0, q);
            }
            __syncthreads();
            for (int c = t; c < ncb; c += BRICK_T)
                if (brick_cnt_members(L.cnt[c]) >= 2)
                    brick_cell_params_f32<false>(s, bi, c, L.cnt[c], q0_solvent, L.acc, L.cell[c].pre, A.cos_a,
                                                 A.sin_a, A.kT_cell, A.seed, step, L.cell[c].par, st);
            __syncthreads();
        }
        if (nmem > ITEMS * BRICK_T || more) {
            if (more) {  // the cells whose Gamma variate needs further calls
                for (int c = t; c < ncb; c += BRICK_T)
                    if (brick_cnt_members(L.cnt[c]) >= 2 && L.more[c])
                        brick_cell_params_f32<false>(s, bi, c, L.cnt[c], q0_solvent, L.acc, L.cell[c].pre, A.cos_a,
                                                     A.sin_a, A.kT_cell, A.seed, step, L.cell[c].par, st);
                __syncthreads();
            }
            // second load: each member is read again before its own write (a
            // site appears once in a brick's list, and nothing has been
            // written yet)
            for (int i = t; i < nmem; i += BRICK_T) {
                float p[3], w[3];
                int32_t id;
                if (!brick_member<float>(A, bi, par_in, i, L, p, w, id, st)) continue;
                const int c = brick_local_cell<float>(s, bn, bi, b, p, L.sh, st);
                if (c < 0) continue;
                if (brick_cnt_members(L.cnt[c]) >= 2) brick_rotate_f32(L.cell[c].par, w, st);
                if (id < 0) {
                    const int64_t j = -(int64_t)id - 1, S = s.S;
                    A.vs[j] = w[0]; A.vs[S + j] = w[1]; A.vs[2 * S + j] = w[2];
                    continue;
                }
                int32_t dst;
                const int cls = brick_stream<float>(A, bi, Lb, p, w, L.sh1, &dst, st);
                brick_emit<float>(A, L, par_out, cls, dst, p, w, id, st);
            }
            __syncthreads();
            if (t < NCLS && L.wdst[t] >= 0)
                bn.cnt[((int64_t)par_out * bn.nbricks + L.wdst[t]) * NCLS + t] = L.wcnt[t];
        }
    }
    // after the brick's barriers, so that their waits do not include these
    // stores: block 0 stores the step's grid shifts and the next step's shift
    // table (the other parity), and every block clears its share of the
    // body-centre grid for this step's insertions
    if (blockIdx.x == 0) {
        if (A.shift_out) draw_shifts(s, A.seed, step, A.shift_out);
        binned_store_shifts(s, bn, A.seed, step + 1);
    }
    for (int64_t q = (int64_t)blockIdx.x * BRICK_T + t; A.grid_clear && q < A.grid_n; q += (int64_t)gridDim.x * BRICK_T)
        A.grid_clear[q] = 0;
    flag(A.status, st | lf.bits());
}

__global__ void k_binned_finish(BinnedDev bn, const uint64_t *d_step) { binned_finish(bn, *d_step); }

// The shift table of the step *d_step (one block), for the first brick
// collision after a packing.
__global__ void k_binned_shtab(SysDev s, BinnedDev bn, uint64_t seed, const uint64_t *d_step)
{
    binned_store_shifts(s, bn, seed, *d_step);
}

// The site lists cleared, for a site listing launched on its own.
__global__ void k_binned_clear_sites(BinnedDev bn)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < bn.nbricks; q += (int64_t)gridDim.x * blockDim.x)
        bn.scnt[q] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) bn.ctrl[BC_SOVF] = 0;
}

// The output overflow counter cleared, for a brick collision launched on its
// own (in the step sequence it is clear already).
__global__ void k_binned_clear_out(BinnedDev bn, const uint64_t *d_step)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) bn.ctrl[BC_OVF0 + (int)((*d_step + 1) & 1)] = 0;
}

// Thermalization of each body's sites for the step and their binning into the
// bricks' site lists (binned layout); one block per body.
template <typename Real>
__global__ __launch_bounds__(BODY_T) void k_therm_bin(SysDev s, BodyDev bd, BrickSiteBin bb, double kT, int thermalize,
                                                      uint64_t seed, const uint64_t *d_step, Real *xs, Real *vs,
                                                      double *site_d, double *vpre, uint32_t *status)
{
    __shared__ double bsh[3];
    __shared__ ThermLds lds;
    const int64_t b = blockIdx.x;
    if (b >= s.B) return;
    uint32_t st = 0;
    const uint64_t step = *d_step;
    const int r = find_sys_wave(s.body_off, s.nsys, b);  // every lane of the block is here
    if (threadIdx.x == 64 || (BODY_T <= 64 && threadIdx.x == 0)) shift_of(s, seed, step, r, bsh);
    thermalize_body<Real>(s, bd, b, kT, thermalize, seed, step, xs, vs, site_d, vpre, bsh, nullptr, nullptr, nullptr,
                          &bb, lds, st);
    flag(status, st);
}

// Dense solvent (x[3][N], v[3][N], identities) into the regions of the bricks
// of its cells on the grid of the step *d_step.
template <typename Real>
__global__ void k_binned_pack(SysDev s, BinnedDev bn, uint64_t seed, const uint64_t *d_step, const Real *x,
                              const Real *v, const int32_t *tag, Real *rec, uint32_t *status)
{
    uint32_t st = 0;
    const uint64_t step = *d_step;
    const int par = (int)(step & 1);
    BrickArgs<Real> A;
    A.bn = bn;
    A.reco = rec;
    const int64_t N = s.N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = find_sys(s.solv_off, s.nsys, i);
        double sh[3];
        shift_of(s, seed, step, r, sh);
        const Real p[3] = {x[i], x[N + i], x[2 * N + i]}, w[3] = {v[i], v[N + i], v[2 * N + i]};
        int jc[3];
        const int32_t b = brick_of_pos<Real>(s, bn, r, p[0], p[1], p[2], sh, jc, st);
        const BrickInfo bi = bn.brick[b];
        const int32_t *sp = bn.subpre + (int64_t)b * (NCLS + 1);  // class 0: the brick's own sub-region
        const int slot = atomicAdd(&bn.cnt[((int64_t)par * bn.nbricks + b) * NCLS], 1);
        brick_put<Real>(A, par, b, bi.off + sp[0], sp[1] - sp[0], slot, p, w, tag ? tag[i] : (int32_t)i, st);
    }
    flag(status, st);
}

// Binned solvent of the step *d_step back to dense arrays in identity order
// (x[:, id] = the member's position, tag[id] = id).
template <typename Real>
__global__ void k_binned_unpack(SysDev s, BinnedDev bn, const uint64_t *d_step, const Real *rec, Real *x, Real *v,
                                int32_t *tag, uint32_t *status)
{
    uint32_t st = 0;
    const int par = (int)(*d_step & 1);
    const int64_t N = s.N;
    auto put = [&](int32_t id, const Real p[3], const Real w[3]) {
        if (id < 0 || id >= N) {
            st |= ST_BINERR;
            return;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[d * N + id] = p[d];
            v[d * N + id] = w[d];
        }
        tag[id] = id;
    };
    for (int64_t b = blockIdx.x; b < bn.nbricks; b += gridDim.x) {
        const BrickInfo bi = bn.brick[b];
        const int32_t *sp = bn.subpre + b * (NCLS + 1);
        for (int c = 0; c < NCLS; ++c) {  // fills of sub-regions without a writer stay zero
            const int n = min(bn.cnt[((int64_t)par * bn.nbricks + b) * NCLS + c], sp[c + 1] - sp[c]);
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                Real p[3], w[3];
                int32_t id;
                rec_load(rec, bi.off + sp[c] + i, p, w, id);
                put(id, p, w);
            }
        }
    }
    const int novf = min(bn.ctrl[BC_OVF0 + par], BIN_OVF_CAP);
    const Real *o = (const Real *)bn.ovf_xv + (int64_t)par * 6 * BIN_OVF_CAP;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < novf; e += (int64_t)gridDim.x * blockDim.x) {
        const Real p[3] = {o[e], o[BIN_OVF_CAP + e], o[2 * BIN_OVF_CAP + e]};
        const Real w[3] = {o[3 * BIN_OVF_CAP + e], o[4 * BIN_OVF_CAP + e], o[5 * BIN_OVF_CAP + e]};
        put(bn.ovf_tag[(int64_t)par * BIN_OVF_CAP + e], p, w);
    }
    flag(status, st);
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

// ---------------------------------------------------------------------------
// Binned layout: host-side plan of the bricks, regions and site lists

// Brick shapes, log2 of the extent along x, y, z, largest first (256 .. 8 cells).
constexpr int BRICK_SHAPES[6][3] = {{3, 3, 2}, {3, 2, 2}, {2, 2, 2}, {2, 2, 1}, {2, 1, 1}, {1, 1, 1}};

// Sub-region capacity for mu expected members: mu + 6 sqrt(mu) + 16 (a
// Poisson count exceeds it with probability below 1e-9); site list capacity:
// the brick's cells + 64, at most the system's sites.  The brick's own class
// expects the whole brick; a neighbour's class the solvent of a layer of
// depth SUBREGION_DEPTH cells along each axis where the two bricks differ (a
// step's shift change moves cell boundaries by less than one cell, and
// streaming moves a particle by |v| dt, about 0.1 cells at kT = 1).
constexpr double SUBREGION_DEPTH = 1.25;
int64_t region_cap(double mu) { return (int64_t)ceil(mu + 6.0 * sqrt(mu)) + 16; }
int64_t site_cap(int64_t ncb, int64_t S_r) { return ncb + 64 < S_r ? ncb + 64 : S_r; }

// Members a brick block holds in registers (FP32) or LDS (FP64).
int brick_block_members(int prec) { return prec == MPCD_F64 ? 1024 : BRICK_PLAN_MEMBERS; }

int32_t sovf_cap_of(const mpcd_sys *sys)
{
    const int64_t sc = sys->n_sites / 4 > 1024 ? sys->n_sites / 4 : 1024;
    return (int32_t)(sc < ((int64_t)1 << 22) ? sc : ((int64_t)1 << 22));
}

struct BinnedPlan {
    int64_t nbricks = 0, cap = 0, sslots = 0;
    int32_t sovf_cap = 0;
    std::vector<BrickInfo> brick;
    std::vector<int32_t> subpre, sys_bb, sys_bg;
    std::vector<int4> wtab;
};

// tables == false: sizes only.
int binned_plan(const mpcd_sys *sys, const int32_t *ncell, const int64_t *solv_off, const int64_t *site_off_sys,
                bool tables, BinnedPlan &P)
{
    if (check_sizes(sys) != MPCD_OK || !ncell || !solv_off || !site_off_sys) return MPCD_EINVAL;
    const int nsys = sys->nsys;
    if (solv_off[0] != 0 || solv_off[nsys] != sys->n_solvent || site_off_sys[0] != 0 ||
        site_off_sys[nsys] != sys->n_sites)
        return MPCD_EINVAL;
    const int target = brick_block_members(sys->prec) - 64;  // room for overflow entries
    int64_t C = 0;
    if (tables) {
        P.sys_bb.assign(nsys + 1, 0);
        P.sys_bg.assign(6 * (size_t)nsys, 0);
        P.brick.clear();
        P.subpre.clear();
    }
    for (int r = 0; r < nsys; ++r) {
        const int n[3] = {ncell[3 * r], ncell[3 * r + 1], ncell[3 * r + 2]};
        if (n[0] < 1 || n[1] < 1 || n[2] < 1 || n[0] > 32767 || n[1] > 32767 || n[2] > 32767) return MPCD_EINVAL;
        const int64_t Cr = (int64_t)n[0] * n[1] * n[2];
        const int64_t Nr = solv_off[r + 1] - solv_off[r], Sr = site_off_sys[r + 1] - site_off_sys[r];
        if (Nr < 0 || Sr < 0) return MPCD_EINVAL;
        C += Cr;
        const double rho = (double)Nr / (double)Cr;
        int k = 0;
        for (; k < 6; ++k) {
            const int64_t ncb = (int64_t)1 << (BRICK_SHAPES[k][0] + BRICK_SHAPES[k][1] + BRICK_SHAPES[k][2]);
            if (region_cap(rho * (double)ncb) + site_cap(ncb, Sr) <= target) break;
        }
        if (k == 6) return MPCD_EINVAL;  // denser than a brick block can hold
        const int lg[3] = {BRICK_SHAPES[k][0], BRICK_SHAPES[k][1], BRICK_SHAPES[k][2]};
        int nb[3];
        for (int d = 0; d < 3; ++d) nb[d] = (n[d] + (1 << lg[d]) - 1) >> lg[d];
        if (tables) {
            P.sys_bb[r] = (int32_t)P.nbricks;
            for (int d = 0; d < 3; ++d) {
                P.sys_bg[6 * r + d] = lg[d];
                P.sys_bg[6 * r + 3 + d] = nb[d];
            }
        }
        for (int bz = 0; bz < nb[2]; ++bz)
            for (int by = 0; by < nb[1]; ++by)
                for (int bx = 0; bx < nb[0]; ++bx) {
                    const int o[3] = {bx << lg[0], by << lg[1], bz << lg[2]};
                    int dim[3];
                    for (int d = 0; d < 3; ++d) dim[d] = std::min(1 << lg[d], n[d] - o[d]);
                    const int64_t ncb = (int64_t)dim[0] * dim[1] * dim[2];
                    // sub-regions: one per writer class with a distinct writer
                    int64_t cs = 0;
                    int32_t pre[NCLS + 1];
                    for (int c = 0; c < NCLS; ++c) {
                        const int c3[3] = {c % 3, (c / 3) % 3, c / 9};
                        double vol = 1.0;
                        bool valid = true;
                        for (int d = 0; d < 3; ++d) {
                            valid = valid && code_valid(c3[d], nb[d]);
                            vol *= c3[d] == 0 ? (double)dim[d] : SUBREGION_DEPTH;
                        }
                        pre[c] = (int32_t)cs;
                        if (valid) cs += region_cap(rho * vol);
                    }
                    pre[NCLS] = (int32_t)cs;
                    const int64_t ct = site_cap(ncb, Sr);
                    if (tables) {
                        P.subpre.insert(P.subpre.end(), pre, pre + NCLS + 1);
                        BrickInfo bi;
                        bi.off = P.cap;
                        bi.cap = (int32_t)cs;
                        bi.sys = r;
                        bi.soff = (int32_t)P.sslots;
                        bi.scap = (int16_t)ct;
                        bi.pad = 0;
                        for (int d = 0; d < 3; ++d) {
                            bi.org[d] = (int16_t)o[d];
                            bi.dim[d] = (uint8_t)dim[d];
                        }
                        P.brick.push_back(bi);
                    }
                    P.nbricks += 1;
                    P.cap += cs;
                    P.sslots += ct;
                }
        if (tables) P.sys_bb[r + 1] = (int32_t)P.nbricks;
    }
    if (C != sys->n_cells) return MPCD_EINVAL;
    if (P.cap >= ((int64_t)1 << 31) || P.sslots >= ((int64_t)1 << 31) || P.nbricks >= ((int64_t)1 << 30))
        return MPCD_EINVAL;
    P.sovf_cap = sovf_cap_of(sys);
    if (tables) {  // the sub-region each brick writes with each class (the inverse of the class code)
        P.wtab.assign((size_t)P.nbricks * NCLS, make_int4(0, 0, -1, 0));
        for (int64_t b = 0; b < P.nbricks; ++b) {
            const BrickInfo &bi = P.brick[b];
            const int32_t *g = &P.sys_bg[6 * bi.sys];
            for (int c = 0; c < NCLS; ++c) {
                const int c3[3] = {c % 3, (c / 3) % 3, c / 9};
                if (!(code_valid(c3[0], g[3]) && code_valid(c3[1], g[4]) && code_valid(c3[2], g[5]))) continue;
                int bc[3];
                for (int d = 0; d < 3; ++d) bc[d] = code_dst(bi.org[d] >> g[d], c3[d], g[3 + d]);
                const int32_t db = P.sys_bb[bi.sys] + (bc[2] * g[4] + bc[1]) * g[3] + bc[0];
                const int32_t *dp = &P.subpre[(size_t)db * (NCLS + 1)];
                P.wtab[(size_t)b * NCLS + c] = make_int4((int)(P.brick[db].off + dp[c]), dp[c + 1] - dp[c], db, 0);
            }
        }
    }
    return MPCD_OK;
}

struct BinnedLayout {
    size_t ctrl, brick, subpre, sys_bb, sys_bg, cnt, scnt, sslot, ovf_dest, ovf_tag, ovf_xv, sovf, oflag, shtab, wtab,
        total;
};

BinnedLayout binned_layout(const mpcd_sys *sys, int64_t nbricks, int64_t sslots, int32_t sovf_cap)
{
    BinnedLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    L.ctrl = take(sizeof(int32_t) * BC_WORDS);
    L.brick = take(sizeof(BrickInfo) * (size_t)nbricks);
    L.subpre = take(sizeof(int32_t) * (NCLS + 1) * (size_t)nbricks);
    L.sys_bb = take(sizeof(int32_t) * (size_t)(sys->nsys + 1));
    L.sys_bg = take(sizeof(int32_t) * 6 * (size_t)sys->nsys);
    L.cnt = take(sizeof(int32_t) * 2 * NCLS * (size_t)nbricks);
    L.scnt = take(sizeof(int32_t) * (size_t)nbricks);
    L.sslot = take(sizeof(int32_t) * (size_t)(sslots > 0 ? sslots : 1));
    L.ovf_dest = take(sizeof(int32_t) * 2 * BIN_OVF_CAP);
    L.ovf_tag = take(sizeof(int32_t) * 2 * BIN_OVF_CAP);
    L.ovf_xv = take(esize(sys) * 12 * BIN_OVF_CAP);
    L.sovf = take(sizeof(int32_t) * 2 * (size_t)sovf_cap);
    L.oflag = take(sizeof(int32_t) * 2 * (size_t)nbricks);
    L.shtab = take(sizeof(double) * 2 * (1 + 6 * (size_t)sys->nsys));
    L.wtab = take(sizeof(int4) * NCLS * (size_t)nbricks);
    L.total = off;
    return L;
}

int check_binned(const mpcd_sys *sys, const mpcd_binned *b)
{
    if (!b || !b->ws || !aligned(b->ws, 256) || b->nbricks < 1 || b->capacity < 0 || b->site_slots < 0)
        return MPCD_EINVAL;
    if (b->ws_bytes < binned_layout(sys, b->nbricks, b->site_slots, sovf_cap_of(sys)).total) return MPCD_EWORKSPACE;
    return MPCD_OK;
}

BinnedDev binned_dev(const mpcd_sys *sys, const mpcd_binned *b)
{
    const BinnedLayout L = binned_layout(sys, b->nbricks, b->site_slots, sovf_cap_of(sys));
    BinnedDev d;
    char *w = (char *)b->ws;
    d.ctrl = (int32_t *)(w + L.ctrl);
    d.brick = (const BrickInfo *)(w + L.brick);
    d.subpre = (const int32_t *)(w + L.subpre);
    d.wtab = (const int4 *)(w + L.wtab);
    d.sys_bb = (const int32_t *)(w + L.sys_bb);
    d.sys_bg = (const int32_t *)(w + L.sys_bg);
    d.cnt = (int32_t *)(w + L.cnt);
    d.scnt = (int32_t *)(w + L.scnt);
    d.sslot = (int32_t *)(w + L.sslot);
    d.ovf_dest = (int32_t *)(w + L.ovf_dest);
    d.ovf_tag = (int32_t *)(w + L.ovf_tag);
    d.ovf_xv = (void *)(w + L.ovf_xv);
    d.sovf = (int32_t *)(w + L.sovf);
    d.oflag = (int32_t *)(w + L.oflag);
    d.shtab = (double *)(w + L.shtab);
    d.nbricks = b->nbricks;
    d.cap = b->capacity;
    d.sovf_cap = sovf_cap_of(sys);
    return d;
}


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

int mpcd_cell_order(int32_t nsys, const int32_t *ncell, int64_t *pos)
{
    if (nsys < 1 || !ncell || !pos) return MPCD_EINVAL;
    int64_t off = 0;
    for (int32_t r = 0; r < nsys; ++r) {
        const int nx = ncell[3 * r], ny = ncell[3 * r + 1], nz = ncell[3 * r + 2];
        if (nx < 1 || ny < 1 || nz < 1 || (int64_t)nx * ny * nz >= ((int64_t)1 << 31)) return MPCD_EINVAL;
        for (int jz = 0; jz < nz; ++jz)
            for (int jy = 0; jy < ny; ++jy)
                for (int jx = 0; jx < nx; ++jx)
                    pos[off + ((int64_t)jz * ny + jy) * nx + jx] = off + brick_index(nx, ny, nz, jx, jy, jz);
        off += (int64_t)nx * ny * nz;
    }
    return MPCD_OK;
}

int mpcd_tile_shape(const mpcd_sys *sys, const mpcd_tune *tune, int32_t out[4])
{
    TRY(check_sizes(sys));
    const mpcd_tune tu = tune ? *tune : mpcd_tune{0, 0, 0, 0, 0};
    if (!out || !tune_ok(tu, sys->prec == MPCD_F64)) return MPCD_EINVAL;
    const TileCfg T = tile_config(sys, tu);
    out[0] = T.items;
    out[1] = T.cpb;
    out[2] = T.cap;
    out[3] = T.ntiles;
    return MPCD_OK;
}

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
    const int64_t NT = sys->n_solvent + sys->n_sites;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(2 * sys->n_cells, 256)), dim3(256), 0, st,
                       at<int32_t>(ws, L.counts), 2 * sys->n_cells, 0);
    if (NT > 0)  // the permutation holds valid particle indices from the start
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(NT, 256)), dim3(256), 0, st, at<int32_t>(ws, L.perm), NT, 0);
    // the scan's ticket counter and tile descriptors (state 0: not published)
    const int64_t ntiles = (sys->n_cells + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, at<int32_t>(ws, L.scan_ctl), (int64_t)2, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(2 * ntiles, 256)), dim3(256), 0, st, at<int32_t>(ws, L.scan_d0),
                       2 * ntiles, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(2 * ntiles, 256)), dim3(256), 0, st, at<int32_t>(ws, L.scan_d1),
                       2 * ntiles, 0);
    // the exchange's histograms and control words start at zero; each exchange
    // leaves them at zero for the next
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(2 * RN_BINS, 256)), dim3(256), 0, st, at<int32_t>(ws, L.rn_hist),
                       (int64_t)(2 * RN_BINS), 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, at<int32_t>(ws, L.rn_ctl), (int64_t)16, 0);
    return launch_check();
}

int mpcd_stream(void *stream, const mpcd_sys *sys, void *x, void *v, double dt, const double *g, void *ws,
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
    const unsigned gr = grid_for(sys->n_solvent, 256);
    const Forcing F = make_forcing(g, dt);
    if (sys->prec == MPCD_F64)
        hipLaunchKernelGGL(k_stream<double>, dim3(gr), dim3(256), 0, st, sd, (double *)x, (double *)v, dt, F,
                           at<uint32_t>(ws, L.status));
    else
        hipLaunchKernelGGL(k_stream<float>, dim3(gr), dim3(256), 0, st, sd, (float *)x, (float *)v, dt, F,
                           at<uint32_t>(ws, L.status));
    return launch_check();
}

// ---------------------------------------------------------------------------
// Launch helpers (arguments validated by the callers)

struct Ctx {
    const mpcd_sys *sys;
    SysDev sd;
    Layout L;
    void *ws;
    uint32_t *status;
    mpcd_tune tune;
};

static Ctx make_ctx(const mpcd_sys *sys, void *ws, const mpcd_tune *tune = nullptr)
{
    Ctx c;
    c.sys = sys;
    c.tune = tune ? *tune : mpcd_tune{0, 0, 0, 0, 0};
    c.sd = make_sysdev(sys);
    c.L = layout_of(sys);
    c.ws = ws;
    c.status = at<uint32_t>(ws, c.L.status);
    return c;
}

static void launch_shift(const Ctx &c, hipStream_t st, uint64_t seed, const uint64_t *d_step)
{
    hipLaunchKernelGGL(k_shift, dim3(grid_for(c.sys->nsys, 64)), dim3(64), 0, st, c.sd, seed, d_step,
                       at<double>(c.ws, c.L.shift));
}

static void launch_bin_count(const Ctx &c, hipStream_t st, const void *x, const void *xs, const int32_t *site_body,
                             int64_t k0, int64_t k1)
{
    if (k1 <= k0) return;
    const unsigned g = (unsigned)((k1 - k0 + PREP_CHUNK - 1) / PREP_CHUNK);
    double *shift = at<double>(c.ws, c.L.shift);
    u64 *counts = at<u64>(c.ws, c.L.counts);
    int32_t *cellid = at<int32_t>(c.ws, c.L.cellid);
    int32_t *slot = at<int32_t>(c.ws, c.L.slot);
    if (c.sys->prec == MPCD_F64)
        hipLaunchKernelGGL(k_bin_count<double>, dim3(g), dim3(BIN_T), 0, st, c.sd, (const double *)x,
                           (const double *)xs, site_body, shift, counts, cellid, slot, c.status, k0, k1);
    else
        hipLaunchKernelGGL(k_bin_count<float>, dim3(g), dim3(BIN_T), 0, st, c.sd, (const float *)x,
                           (const float *)xs, site_body, shift, counts, cellid, slot, c.status, k0, k1);
}

static void launch_scan(const Ctx &c, hipStream_t st)
{
    const int64_t NT = c.sys->n_solvent + c.sys->n_sites, C = c.sys->n_cells;
    const int V = scan_v(C);
    const int64_t nb = (C + (int64_t)SCAN_T * V - 1) / ((int64_t)SCAN_T * V);
    u64 *counts = at<u64>(c.ws, c.L.counts);
    int32_t *cs = at<int32_t>(c.ws, c.L.cell_start), *ss = at<int32_t>(c.ws, c.L.site_start);
    const ScanWs W{at<u64>(c.ws, c.L.scan_ctl), at<u64>(c.ws, c.L.scan_d0), at<u64>(c.ws, c.L.scan_d1)};
    hipLaunchKernelGGL(V == 16 ? k_scan<16> : k_scan<4>, dim3((unsigned)nb), dim3(SCAN_T), 0, st, counts, C, nb, W,
                       cs, ss, (int32_t)NT, (int32_t)c.sys->n_sites, c.status);
}

// clear_grid: also clear the body-centre grid (a step whose first kernel ran
// fused into the previous step's last).
static void launch_scatter(const Ctx &c, hipStream_t st, int32_t *clear_grid = nullptr, int64_t grid_n = 0)
{
    const int64_t NT = c.sys->n_solvent + c.sys->n_sites;
    if (NT == 0) return;
    hipLaunchKernelGGL(k_bin_scatter, dim3((unsigned)((NT + BIN_CHUNK - 1) / BIN_CHUNK)), dim3(BIN_T), 0, st, NT,
                       c.sys->n_solvent, at<int32_t>(c.ws, c.L.cellid), at<int32_t>(c.ws, c.L.slot),
                       at<int32_t>(c.ws, c.L.cell_start), at<int32_t>(c.ws, c.L.site_start),
                       at<int32_t>(c.ws, c.L.perm), clear_grid, grid_n, c.status);
}

static CollideArgs collide_args(const Ctx &c, const int32_t *tag, const mpcd_bodies *bodies, double cos_a,
                                double sin_a, double kT_cell, uint64_t seed, const uint64_t *d_step, double dt,
                                uint64_t *advance)
{
    CollideArgs A;
    A.s = c.sd;
    A.site_m = bodies ? bodies->site_m : nullptr;
    A.tag = tag;
    A.cell_start = at<int32_t>(c.ws, c.L.cell_start);
    A.site_start = at<int32_t>(c.ws, c.L.site_start);
    A.perm = at<int32_t>(c.ws, c.L.perm);
    A.draws = at<double>(c.ws, c.L.draws);
    A.cos_a = cos_a;
    A.sin_a = sin_a;
    A.kT_cell = kT_cell;
    A.dt = dt;
    A.seed = seed;
    A.d_step = d_step;
    A.status = c.status;
    A.advance_step = advance;
    A.step_next = nullptr;
    A.F = make_forcing(nullptr, dt);
    A.inline_draws = 0;
    A.bin_counts = nullptr;
    A.bin_cellid = nullptr;
    A.bin_slot = nullptr;
    return A;
}

static unsigned draw_blocks(int64_t C, const mpcd_tune &tu)
{
    const int per = tu.draw_cells ? tu.draw_cells : DRAW_CELLS_PER_LANE;
    const int64_t lanes = (C + per - 1) / per;
    return grid_for(lanes > 0 ? lanes : 1, BIN_T);
}

static void launch_draws(const Ctx &c, hipStream_t st, const CollideArgs &A)
{
    hipLaunchKernelGGL(k_cell_draws, dim3(draw_blocks(c.sys->n_cells, c.tune)), dim3(BIN_T), 0, st, A,
                       at<double>(c.ws, c.L.draws));
}

// x_stream: positions streamed in place, or (out of place) read and streamed
// into x_out.  v_out == nullptr: in place.
// A.bin_counts set (out of place only): the kernel also bins the new solvent
// for the next step; its LDS then also holds the tile's hash table.
static void launch_collide(const Ctx &c, hipStream_t st, const CollideArgs &A, void *v, void *vs, void *x_stream,
                           void *x_out = nullptr, void *v_out = nullptr, int32_t *tag_out = nullptr)
{
    const bool f64 = c.sys->prec == MPCD_F64;
    const TileCfg T = tile_config(c.sys, c.tune);
    const dim3 grid(xcd_grid(T.ntiles));
    const bool b = A.bin_counts != nullptr && v_out != nullptr;
    size_t lds = tile_layout(f64, T.cpb, T.cap).end;
    if (b) {  // + the next-step shifts of the tile's systems; the hash table overlays the tile
        lds += sizeof(double) * 3 * (size_t)T.cpb;
        if (lds < 8 * (size_t)T.cap) lds = 8 * (size_t)T.cap;
    }
    const bool d = A.inline_draws != 0;
    if (f64) {
        const SolvOut<double> O{(double *)x_out, (double *)v_out, tag_out};
        auto kern = T.items == 1 ? (b ? (d ? k_collide_tiled_f64_i1_d_b : k_collide_tiled_f64_i1_b)
                                      : (d ? k_collide_tiled_f64_i1_d : k_collide_tiled_f64_i1))
                  : T.items == 4 ? (b ? (d ? k_collide_tiled_f64_i4_d_b : k_collide_tiled_f64_i4_b)
                                      : (d ? k_collide_tiled_f64_i4_d : k_collide_tiled_f64_i4))
                                 : (b ? (d ? k_collide_tiled_f64_d_b : k_collide_tiled_f64_b)
                                      : (d ? k_collide_tiled_f64_d : k_collide_tiled_f64));
        hipLaunchKernelGGL(kern, grid, dim3(TILE_T), lds, st, A, T, (double *)v, (double *)vs, (double *)x_stream, O);
    } else {
        const SolvOut<float> O{(float *)x_out, (float *)v_out, tag_out};
        auto kern = T.items == 2 ? (b ? (d ? k_collide_tiled_f32_i2_d_b : k_collide_tiled_f32_i2_b)
                                      : (d ? k_collide_tiled_f32_i2_d : k_collide_tiled_f32_i2))
                  : T.items == 8 ? (b ? (d ? k_collide_tiled_f32_i8_d_b : k_collide_tiled_f32_i8_b)
                                      : (d ? k_collide_tiled_f32_i8_d : k_collide_tiled_f32_i8))
                                 : (b ? (d ? k_collide_tiled_f32_d_b : k_collide_tiled_f32_b)
                                      : (d ? k_collide_tiled_f32_d : k_collide_tiled_f32));
        hipLaunchKernelGGL(kern, grid, dim3(TILE_T), lds, st, A, T, (float *)v, (float *)vs, (float *)x_stream, O);
    }
}

static void launch_thermalize(const Ctx &c, hipStream_t st, const mpcd_bodies *bodies, double kT, int thermalize,
                              uint64_t seed, const uint64_t *d_step, void *xs, void *vs)
{
    if (c.sys->n_bodies == 0 || c.sys->n_sites == 0) return;
    const BodyDev bd = make_bodydev(bodies);
    double *site_d = at<double>(c.ws, c.L.site_d), *vpre = at<double>(c.ws, c.L.vpre);
    const dim3 gb((unsigned)c.sys->n_bodies);
    if (c.sys->prec == MPCD_F64)
        hipLaunchKernelGGL(k_thermalize<double>, gb, dim3(BODY_T), 0, st, c.sd, bd, kT, thermalize, seed, d_step,
                           (double *)xs, (double *)vs, site_d, vpre, c.status);
    else
        hipLaunchKernelGGL(k_thermalize<float>, gb, dim3(BODY_T), 0, st, c.sd, bd, kT, thermalize, seed, d_step,
                           (float *)xs, (float *)vs, site_d, vpre, c.status);
}

// Thermalization + site binning + solvent binning in one launch.
static BodyGrid body_grid(const Ctx &c, const mpcd_wca &wca)
{
    BodyGrid g;
    const bool on = (wca.mode == 1 || wca.mode == 2) && c.sys->n_bodies > 0;
    g.count = on ? at<int32_t>(c.ws, c.L.grid_count) : nullptr;
    g.body = on ? at<int32_t>(c.ws, c.L.grid_body) : nullptr;
    g.mask = c.L.grid_mask;
    const double rc = wca.delta + 0x1.1f59ac3c7d6c0p+0 * wca.sigma;
    g.rc = wca.mode == 2 ? 2.0 * wca.reach + rc : rc;  // centre distance within which bodies interact
    return g;
}

static SiteFrames site_frames(const Ctx &c, const mpcd_wca &wca)
{
    SiteFrames f;
    const bool on = wca.mode == 2 && c.sys->n_sites > 0;
    f.pos = on ? at<double>(c.ws, c.L.wpos) : nullptr;
    f.off = on ? at<double>(c.ws, c.L.woff) : nullptr;
    f.reach = wca.reach;
    return f;
}

// Standalone entry points: rebuild the body-centre grid from the current
// positions (the fused step clears it in k_prep and fills it after the drift).
static void launch_body_grid(const Ctx &c, hipStream_t st, const mpcd_bodies *bodies, const mpcd_wca &wca)
{
    const SiteFrames fr = site_frames(c, wca);
    if (fr.pos)
        hipLaunchKernelGGL(k_site_frames, dim3((unsigned)c.sys->n_bodies), dim3(BODY_T), 0, st, c.sd,
                           make_bodydev(bodies), fr, c.status);
    const BodyGrid g = body_grid(c, wca);
    if (!g.count) return;
    const int64_t G = (int64_t)c.L.grid_mask + 1;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(G, 256)), dim3(256), 0, st, g.count, G, 0);
    hipLaunchKernelGGL(k_grid_insert, dim3(grid_for(c.sys->n_bodies, 64)), dim3(64), 0, st, c.sd,
                       make_bodydev(bodies), g);
}

static void launch_prep(const Ctx &c, hipStream_t st, const mpcd_bodies *bodies, double kT, int thermalize,
                        uint64_t seed, const uint64_t *d_step, const void *x, void *xs, void *vs,
                        const mpcd_wca &wca, int part = 0)
{
    const BodyGrid grid = body_grid(c, wca);
    const int64_t grid_n = grid.count ? (int64_t)c.L.grid_mask + 1 : 0;
    const int64_t N = c.sys->n_solvent;
    const int64_t nb = (c.sys->n_sites > 0) ? c.sys->n_bodies : 0;
    const int64_t nchunks = (N + PREP_CHUNK - 1) / PREP_CHUNK;
    const BodyDev bd = make_bodydev(bodies);
    SysDev sd = c.sd;
    if (nb == 0) sd.B = 0;  // no site work: every block bins solvent
    double *site_d = at<double>(c.ws, c.L.site_d), *vpre = at<double>(c.ws, c.L.vpre);
    u64 *counts = at<u64>(c.ws, c.L.counts);
    int32_t *cellid = at<int32_t>(c.ws, c.L.cellid);
    int32_t *slot = at<int32_t>(c.ws, c.L.slot);
    double *shift = at<double>(c.ws, c.L.shift);
    // part 1: the body blocks alone; part 2: the solvent blocks alone (both
    // only with sites); otherwise the whole kernel
    const int pk = (nb > 0 && (part == 1 || part == 2)) ? part : 0;
    const int64_t nblocks = pk == 1 ? nb : pk == 2 ? nchunks : nb + nchunks;
    if (nblocks <= 0 && pk != 0) return;
    const dim3 g((unsigned)(nblocks > 0 ? nblocks : 1));
    if (c.sys->prec == MPCD_F64) {
        auto k = pk == 1 ? k_prep<double, 1> : pk == 2 ? k_prep<double, 2> : k_prep<double, 0>;
        hipLaunchKernelGGL(k, g, dim3(BODY_T), 0, st, sd, bd, kT, thermalize, seed, d_step, (const double *)x,
                           (double *)xs, (double *)vs, site_d, vpre, counts, grid.count, grid_n, cellid, slot, shift,
                           c.status);
    } else {
        auto k = pk == 1 ? k_prep<float, 1> : pk == 2 ? k_prep<float, 2> : k_prep<float, 0>;
        hipLaunchKernelGGL(k, g, dim3(BODY_T), 0, st, sd, bd, kT, thermalize, seed, d_step, (const float *)x,
                           (float *)xs, (float *)vs, site_d, vpre, counts, grid.count, grid_n, cellid, slot, shift,
                           c.status);
    }
}

// Scatter fused with the per-cell draws in one launch.
static void launch_scatter_draws(const Ctx &c, hipStream_t st, const CollideArgs &A, int32_t *clear_grid = nullptr,
                                 int64_t grid_n = 0)
{
    const int64_t NT = c.sys->n_solvent + c.sys->n_sites;
    const int nsc = (int)((NT + BIN_CHUNK - 1) / BIN_CHUNK);
    const int ndr = (int)draw_blocks(c.sys->n_cells, c.tune);
    hipLaunchKernelGGL(k_scatter_draws, dim3((unsigned)(nsc + ndr)), dim3(BIN_T), 0, st, NT,
                       at<int32_t>(c.ws, c.L.cellid), at<int32_t>(c.ws, c.L.slot), at<int32_t>(c.ws, c.L.perm), ndr,
                       A, at<double>(c.ws, c.L.draws), clear_grid, grid_n);
}

// Step t's forces and kick fused with step t+1's first kernel (k_forces_prep):
// x is the solvent step t wrote, step_next the index t+1 stored by step t's
// collision.
static void launch_forces_prep(const Ctx &c, hipStream_t st, const mpcd_bodies *bodies, const mpcd_wca &wca,
                               const double *f_ext, double dt, uint64_t *advance, double kT, int thermalize,
                               uint64_t seed, const uint64_t *step_next, const void *x, void *xs, void *vs,
                               bool solvent = true)
{
    // solvent == false: the collision has binned the new solvent already
    const int64_t nchunks = solvent ? (c.sys->n_solvent + PREP_CHUNK - 1) / PREP_CHUNK : 0;
    const dim3 g((unsigned)(c.sys->n_bodies + nchunks));
    const BodyDev bd = make_bodydev(bodies);
    const BodyGrid grid = body_grid(c, wca);
    const ExtForce E = make_ext(f_ext);
    double *site_d = at<double>(c.ws, c.L.site_d), *vpre = at<double>(c.ws, c.L.vpre);
    u64 *counts = at<u64>(c.ws, c.L.counts);
    int32_t *cellid = at<int32_t>(c.ws, c.L.cellid), *slot = at<int32_t>(c.ws, c.L.slot);
    double *shift = at<double>(c.ws, c.L.shift);
    if (c.sys->prec == MPCD_F64)
        hipLaunchKernelGGL(k_forces_prep<double>, g, dim3(BODY_T), 0, st, c.sd, bd, wca, grid, E, dt, advance, kT,
                           thermalize, seed, step_next, (const double *)x, (double *)xs, (double *)vs, site_d, vpre,
                           counts, cellid, slot, shift, c.status);
    else
        hipLaunchKernelGGL(k_forces_prep<float>, g, dim3(BODY_T), 0, st, c.sd, bd, wca, grid, E, dt, advance, kT,
                           thermalize, seed, step_next, (const float *)x, (float *)xs, (float *)vs, site_d, vpre,
                           counts, cellid, slot, shift, c.status);
}

// binned, d_step: also clear the binned layout's spent fills (binned_finish).
static void launch_transfer_first(const Ctx &c, hipStream_t st, const mpcd_bodies *bodies, const void *vs, double *J,
                                  double *K, double dt, const mpcd_wca &wca, const mpcd_binned *binned = nullptr,
                                  const uint64_t *d_step = nullptr)
{
    const BodyGrid grid = body_grid(c, wca);
    const SiteFrames fr = site_frames(c, wca);
    if (c.sys->n_bodies == 0) return;
    const BodyDev bd = make_bodydev(bodies);
    BinnedDev bn;
    memset(&bn, 0, sizeof bn);
    if (binned) bn = binned_dev(c.sys, binned);
    const uint64_t *ds = binned ? d_step : nullptr;
    const dim3 gb((unsigned)c.sys->n_bodies);
    if (c.sys->prec == MPCD_F64)
        hipLaunchKernelGGL(k_transfer_first<double>, gb, dim3(BODY_T), 0, st, c.sd, bd, (const double *)vs,
                           at<double>(c.ws, c.L.site_d), at<double>(c.ws, c.L.vpre), J, K, dt, grid, fr, c.status, bn,
                           ds);
    else
        hipLaunchKernelGGL(k_transfer_first<float>, gb, dim3(BODY_T), 0, st, c.sd, bd, (const float *)vs,
                           at<double>(c.ws, c.L.site_d), at<double>(c.ws, c.L.vpre), J, K, dt, grid, fr, c.status, bn,
                           ds);
}

static void launch_forces(const Ctx &c, hipStream_t st, const mpcd_bodies *bodies, const mpcd_wca &wca,
                          const double *f_ext, double dt, int kick, uint64_t *advance)
{
    const ExtForce E = make_ext(f_ext);
    if (c.sys->n_bodies == 0) return;
    if (wca.mode == 2)
        hipLaunchKernelGGL(k_site_forces, dim3((unsigned)c.sys->n_bodies), dim3(BODY_T), 0, st, c.sd,
                           make_bodydev(bodies), wca, body_grid(c, wca), site_frames(c, wca), E, dt, kick, advance,
                           c.status);
    else
        hipLaunchKernelGGL(k_body_forces, dim3((unsigned)c.sys->n_bodies), dim3(FRC_T), 0, st, c.sd,
                           make_bodydev(bodies), wca, body_grid(c, wca), E, dt, kick, advance, c.status);
}

static void launch_reorder(const Ctx &c, hipStream_t st, void *x, void *v, int32_t *tag)
{
    const int64_t N = c.sys->n_solvent, NT = c.sys->n_solvent + c.sys->n_sites;
    if (N == 0) return;
    const int64_t nb = (NT + BIN_CHUNK - 1) / BIN_CHUNK;
    const int32_t *perm = at<int32_t>(c.ws, c.L.perm);
    int32_t *partial = at<int32_t>(c.ws, c.L.partial);
    char *tmp = at<char>(c.ws, c.L.rtmp);
    const size_t es = esize(c.sys);
    int32_t *ttag = (int32_t *)(tmp + 6 * es * (size_t)N);
    const unsigned gcp = grid_for(N, 256);
    hipLaunchKernelGGL(k_reorder_count, dim3((unsigned)nb), dim3(BIN_T), 0, st, perm, NT, N, partial);
    hipLaunchKernelGGL(k_partials_scan, dim3(1), dim3(SCAN_T), 0, st, partial, nb);
    if (c.sys->prec == MPCD_F64) {
        double *tx = (double *)tmp, *tv = tx + 3 * N;
        hipLaunchKernelGGL(k_reorder_gather<double>, dim3((unsigned)nb), dim3(BIN_T), 0, st, perm, NT, N, partial,
                           (const double *)x, (const double *)v, (const int32_t *)tag, tx, tv, ttag);
        hipLaunchKernelGGL(k_reorder_copy<double>, dim3(gcp), dim3(256), 0, st, N, (double *)x, (double *)v, tag,
                           (const double *)tx, (const double *)tv, (const int32_t *)ttag);
    } else {
        float *tx = (float *)tmp, *tv = tx + 3 * N;
        hipLaunchKernelGGL(k_reorder_gather<float>, dim3((unsigned)nb), dim3(BIN_T), 0, st, perm, NT, N, partial,
                           (const float *)x, (const float *)v, (const int32_t *)tag, tx, tv, ttag);
        hipLaunchKernelGGL(k_reorder_copy<float>, dim3(gcp), dim3(256), 0, st, N, (float *)x, (float *)v, tag,
                           (const float *)tx, (const float *)tv, (const int32_t *)ttag);
    }
}

// ---------------------------------------------------------------------------
// Entry points

// ---- binned layout launches ----

static BrickSiteBin brick_site_bin(const Ctx &c, const mpcd_binned *b)
{
    BrickSiteBin bb;
    bb.bn = binned_dev(c.sys, b);
    return bb;
}

static void launch_therm_bin(const Ctx &c, hipStream_t st, const mpcd_bodies *bodies, double kT, int thermalize,
                             uint64_t seed, const uint64_t *d_step, void *xs, void *vs, const mpcd_binned *b)
{
    if (c.sys->n_bodies == 0 || c.sys->n_sites == 0) return;
    const BodyDev bd = make_bodydev(bodies);
    double *site_d = at<double>(c.ws, c.L.site_d), *vpre = at<double>(c.ws, c.L.vpre);
    const dim3 g((unsigned)c.sys->n_bodies);
    if (c.sys->prec == MPCD_F64)
        hipLaunchKernelGGL(k_therm_bin<double>, g, dim3(BODY_T), 0, st, c.sd, bd, brick_site_bin(c, b), kT,
                           thermalize, seed, d_step, (double *)xs, (double *)vs, site_d, vpre, c.status);
    else
        hipLaunchKernelGGL(k_therm_bin<float>, g, dim3(BODY_T), 0, st, c.sd, bd, brick_site_bin(c, b), kT, thermalize,
                           seed, d_step, (float *)xs, (float *)vs, site_d, vpre, c.status);
}

// The brick collision of the binned layout (FP32).
static void launch_brick_collide(const Ctx &c, hipStream_t st, const mpcd_step_args *a)
{
    const mpcd_params &p = a->par;
    BrickArgs<float> A;
    A.s = c.sd;
    A.bn = binned_dev(c.sys, a->binned);
    A.rec = (const float *)a->x;
    A.reco = (float *)a->x_out;
    A.xs = (float *)a->xs;
    A.vs = (float *)a->vs;
    A.site_m = a->bodies.site_m;
    A.cos_a = p.cos_a;
    A.sin_a = p.sin_a;
    A.kT_cell = p.kT_cell;
    A.dt = p.dt;
    A.seed = p.seed;
    A.d_step = a->d_step;
    A.shift_out = at<double>(c.ws, c.L.shift);
    const BodyGrid grid = body_grid(c, p.wca);
    A.grid_clear = grid.count;
    A.grid_n = grid.count ? (int64_t)c.L.grid_mask + 1 : 0;
    A.F = make_forcing(p.g, p.dt);
    A.status = c.status;
    const dim3 nblk(xcd_grid(a->binned->nbricks));
    const bool wide = a->binned->nbricks >= BRICK_WIDE_MIN, unit = a->sys->a == 1.0;
    if (wide && unit)
        hipLaunchKernelGGL((k_brick_collide_f32<BRICK_T_WIDE, true>), nblk, dim3(BRICK_T_WIDE), 0, st, A);
    else if (wide)
        hipLaunchKernelGGL((k_brick_collide_f32<BRICK_T_WIDE, false>), nblk, dim3(BRICK_T_WIDE), 0, st, A);
    else if (unit)
        hipLaunchKernelGGL((k_brick_collide_f32<BRICK_T_NARROW, true>), nblk, dim3(BRICK_T_NARROW), 0, st, A);
    else
        hipLaunchKernelGGL((k_brick_collide_f32<BRICK_T_NARROW, false>), nblk, dim3(BRICK_T_NARROW), 0, st, A);
}

static int bin_checks(const mpcd_sys *sys, const void *x, const void *xs, const mpcd_bodies *bodies,
                      const uint64_t *d_step, void *ws, size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    if (!ok_arr(x, sys->n_solvent, esize(sys)) || !ok_arr(xs, sys->n_sites, esize(sys)) || !d_step)
        return MPCD_EINVAL;
    if (sys->n_sites > 0 && (!bodies || !bodies->site_body)) return MPCD_EINVAL;
    return MPCD_OK;
}

int mpcd_bin(void *stream, const mpcd_sys *sys, const void *x, const void *xs, const mpcd_bodies *bodies,
             uint64_t seed, const uint64_t *d_step, void *ws, size_t ws_bytes)
{
    TRY(bin_checks(sys, x, xs, bodies, d_step, ws, ws_bytes));
    const Ctx c = make_ctx(sys, ws);
    hipStream_t st = (hipStream_t)stream;
    launch_shift(c, st, seed, d_step);
    launch_bin_count(c, st, x, xs, bodies ? bodies->site_body : nullptr, 0, sys->n_solvent + sys->n_sites);
    launch_scan(c, st);
    launch_scatter(c, st);
    return launch_check();
}

int mpcd_reorder(void *stream, const mpcd_sys *sys, void *x, void *v, int32_t *tag, void *ws, size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    const int64_t N = sys->n_solvent;
    if (!ok_arr(x, N, esize(sys)) || !ok_arr(v, N, esize(sys)) || !ok_arr(tag, N, 4)) return MPCD_EINVAL;
    launch_reorder(make_ctx(sys, ws), (hipStream_t)stream, x, v, tag);
    return launch_check();
}

static int collide_checks(const mpcd_sys *sys, const void *v, const int32_t *tag, const void *vs,
                          const mpcd_bodies *bodies, const uint64_t *d_step, void *ws, size_t ws_bytes,
                          const void *x_stream, double dt)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    if (!ok_arr(v, sys->n_solvent, esize(sys)) || !ok_arr(vs, sys->n_sites, esize(sys)) || !d_step)
        return MPCD_EINVAL;
    if (tag && !aligned(tag, 4)) return MPCD_EINVAL;
    if (sys->n_sites > 0 && (!bodies || !bodies->site_m)) return MPCD_EINVAL;
    if (x_stream && (!aligned(x_stream, esize(sys)) || !(dt > 0.0))) return MPCD_EINVAL;
    return MPCD_OK;
}

// Out-of-place solvent output: all three arrays or none; it needs the input
// positions (the solvent is streamed into x_out) and may not alias the inputs.
static int out_checks(const mpcd_sys *sys, const void *v, const int32_t *tag, const void *x, const void *x_out,
                      const void *v_out, const int32_t *tag_out)
{
    if (!x_out && !v_out && !tag_out) return MPCD_OK;
    const int64_t N = sys->n_solvent;
    if (N == 0) return MPCD_OK;
    if (!x_out || !v_out || !tag_out || !x) return MPCD_EINVAL;
    if (!ok_arr(x_out, N, esize(sys)) || !ok_arr(v_out, N, esize(sys)) || !ok_arr(tag_out, N, 4)) return MPCD_EINVAL;
    if (x_out == x || x_out == v || v_out == x || v_out == v || (tag && (const void *)tag_out == (const void *)tag))
        return MPCD_EINVAL;
    return MPCD_OK;
}

int mpcd_collide(void *stream, const mpcd_sys *sys, void *v, const int32_t *tag, void *vs,
                 const mpcd_bodies *bodies, double cos_a, double sin_a, double kT_cell, uint64_t seed,
                 const uint64_t *d_step, void *ws, size_t ws_bytes, void *x_stream, double dt)
{
    TRY(collide_checks(sys, v, tag, vs, bodies, d_step, ws, ws_bytes, x_stream, dt));
    const Ctx c = make_ctx(sys, ws);
    hipStream_t st = (hipStream_t)stream;
    const CollideArgs A = collide_args(c, tag, bodies, cos_a, sin_a, kT_cell, seed, d_step, dt, nullptr);
    launch_draws(c, st, A);
    launch_collide(c, st, A, v, vs, x_stream);
    return launch_check();
}

int mpcd_cell_draws(void *stream, const mpcd_sys *sys, double kT_cell, uint64_t seed, const uint64_t *d_step,
                    void *ws, size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    if (!d_step) return MPCD_EINVAL;
    const Ctx c = make_ctx(sys, ws);
    const CollideArgs A = collide_args(c, nullptr, nullptr, 1.0, 0.0, kT_cell, seed, d_step, 1.0, nullptr);
    launch_draws(c, (hipStream_t)stream, A);
    return launch_check();
}

int mpcd_collide_drawn(void *stream, const mpcd_sys *sys, void *v, const int32_t *tag, void *vs,
                       const mpcd_bodies *bodies, double cos_a, double sin_a, double kT_cell,
                       const uint64_t *d_step, void *ws, size_t ws_bytes, void *x_stream, double dt,
                       void *x_out, void *v_out, int32_t *tag_out, uint64_t seed, const mpcd_tune *tune)
{
    TRY(collide_checks(sys, v, tag, vs, bodies, d_step, ws, ws_bytes, x_stream, dt));
    TRY(out_checks(sys, v, tag, x_stream, x_out, v_out, tag_out));
    if (tune && !tune_ok(*tune, sys->prec == MPCD_F64)) return MPCD_EINVAL;
    const Ctx c = make_ctx(sys, ws, tune);
    CollideArgs A = collide_args(c, tag, bodies, cos_a, sin_a, kT_cell, c.tune.draws_inline ? seed : 0, d_step, dt,
                                 nullptr);
    A.inline_draws = c.tune.draws_inline;
    launch_collide(c, (hipStream_t)stream, A, v, vs, x_stream, x_out, v_out, tag_out);
    return launch_check();
}

static int thermalize_checks(const mpcd_sys *sys, const mpcd_bodies *bodies, double kT, int32_t thermalize,
                             const uint64_t *d_step, const void *xs, const void *vs, void *ws, size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    TRY(check_bodies(sys, bodies));
    if (!ok_arr(xs, sys->n_sites, esize(sys)) || !ok_arr(vs, sys->n_sites, esize(sys)) || !d_step)
        return MPCD_EINVAL;
    if (thermalize && !(kT > 0.0)) return MPCD_EINVAL;
    return MPCD_OK;
}

int sites_thermalize(void *stream, const mpcd_sys *sys, const mpcd_bodies *bodies, double kT,
                     int32_t thermalize, uint64_t seed, const uint64_t *d_step, void *xs, void *vs, void *ws,
                     size_t ws_bytes)
{
    TRY(thermalize_checks(sys, bodies, kT, thermalize, d_step, xs, vs, ws, ws_bytes));
    launch_thermalize(make_ctx(sys, ws), (hipStream_t)stream, bodies, kT, thermalize, seed, d_step, xs, vs);
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
    const Ctx c = make_ctx(sys, ws);
    const BodyDev bd = make_bodydev(bodies);
    hipStream_t st = (hipStream_t)stream;
    const dim3 g((unsigned)sys->n_bodies);
    if (sys->prec == MPCD_F64)
        hipLaunchKernelGGL(k_sites_to_body<double>, g, dim3(BODY_T), 0, st, c.sd, bd, (const double *)vs,
                           at<double>(ws, c.L.site_d), at<double>(ws, c.L.vpre), J, K);
    else
        hipLaunchKernelGGL(k_sites_to_body<float>, g, dim3(BODY_T), 0, st, c.sd, bd, (const float *)vs,
                           at<double>(ws, c.L.site_d), at<double>(ws, c.L.vpre), J, K);
    return launch_check();
}

static int wca_check(const mpcd_wca *wca)
{
    if (!wca || wca->mode < 0 || wca->mode > 2) return MPCD_EINVAL;
    if (wca->mode != 0 && !(wca->sigma > 0.0 && wca->eps >= 0.0 && wca->delta >= 0.0)) return MPCD_EINVAL;
    if (wca->mode == 2 && !(wca->reach >= 0.0 && wca->reach < 1e300)) return MPCD_EINVAL;
    return MPCD_OK;
}

int body_forces(void *stream, const mpcd_sys *sys, const mpcd_bodies *bodies, const mpcd_wca *wca,
                const double *f_ext, void *ws, size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    TRY(check_bodies(sys, bodies));
    TRY(wca_check(wca));
    const Ctx c = make_ctx(sys, ws);
    launch_body_grid(c, (hipStream_t)stream, bodies, *wca);
    launch_forces(c, (hipStream_t)stream, bodies, *wca, f_ext, 0.0, 0, nullptr);
    return launch_check();
}

int body_integrate(void *stream, const mpcd_sys *sys, const mpcd_bodies *bodies, const double *J,
                   const double *K, const mpcd_wca *wca, const double *f_ext, double dt, void *ws,
                   size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    TRY(check_bodies(sys, bodies));
    TRY(wca_check(wca));
    if (!(dt > 0.0)) return MPCD_EINVAL;
    if ((J && !aligned(J, 8)) || (K && !aligned(K, 8))) return MPCD_EINVAL;
    if (sys->n_bodies == 0) return MPCD_OK;
    const Ctx c = make_ctx(sys, ws);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_body_first, dim3(grid_for(sys->n_bodies, 64)), dim3(64), 0, st, c.sd, make_bodydev(bodies),
                       J, K, dt, c.status);
    launch_body_grid(c, st, bodies, *wca);
    launch_forces(c, st, bodies, *wca, f_ext, dt, 1, nullptr);
    return launch_check();
}

int mpcd_advance_step(void *stream, uint64_t *d_step)
{
    if (!d_step || !aligned(d_step, 8)) return MPCD_EINVAL;
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, (hipStream_t)stream, d_step);
    return launch_check();
}

// ---- reverse nonequilibrium exchange ----

static int rnemd_checks(const mpcd_sys *sys, const void *x, const void *v, const int32_t *tag, const mpcd_rnemd *r,
                        const double *dp, void *ws, size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    if (!r || !dp || !aligned(dp, 8)) return MPCD_EINVAL;
    if (sys->nsys != 1) return MPCD_ENOTSUP;
    if (!ok_arr(x, sys->n_solvent, esize(sys)) || !ok_arr(v, sys->n_solvent, esize(sys))) return MPCD_EINVAL;
    if (tag && !aligned(tag, 4)) return MPCD_EINVAL;
    if (!(r->dy > 0.0) || r->npairs < 0 || r->npairs > RN_MAXPAIRS) return MPCD_EINVAL;
    return MPCD_OK;
}

// The exchange's four kernels on the buffers in R (histogram and control
// words zero on entry; both are left zero), flags ORed into *status.
static void launch_rnemd_on(RnArgs R, hipStream_t st, const mpcd_sys *sys, const void *x, void *v,
                            const int32_t *tag, const mpcd_rnemd *r, double *dp, uint32_t *status)
{
    const int64_t N = sys->n_solvent;
    if (N == 0 || r->npairs == 0) return;
    R.y0 = r->y0; R.y1 = r->y1; R.dy = r->dy; R.target = r->target; R.m = sys->m_solvent;
    R.npairs = r->npairs;
    const unsigned g = grid_for(N, 256, 8192);
    if (sys->prec == MPCD_F64) {
        hipLaunchKernelGGL(k_rn_hist<double>, dim3(RN_HBLOCKS), dim3(256), 0, st, R, (const double *)x,
                           (const double *)v, N);
        hipLaunchKernelGGL(k_rn_thresh, dim3(1), dim3(256), 0, st, R);
        hipLaunchKernelGGL(k_rn_collect<double>, dim3(g), dim3(256), 0, st, R, (const double *)x, (const double *)v,
                           tag, N, status);
        hipLaunchKernelGGL(k_rn_swap<double>, dim3(1), dim3(1024), 0, st, R, (double *)v, N, dp, status);
    } else {
        hipLaunchKernelGGL(k_rn_hist<float>, dim3(RN_HBLOCKS), dim3(256), 0, st, R, (const float *)x,
                           (const float *)v, N);
        hipLaunchKernelGGL(k_rn_thresh, dim3(1), dim3(256), 0, st, R);
        hipLaunchKernelGGL(k_rn_collect<float>, dim3(g), dim3(256), 0, st, R, (const float *)x, (const float *)v,
                           tag, N, status);
        hipLaunchKernelGGL(k_rn_swap<float>, dim3(1), dim3(1024), 0, st, R, (float *)v, N, dp, status);
    }
}

static void launch_rnemd(const Ctx &c, hipStream_t st, const void *x, void *v, const int32_t *tag,
                         const mpcd_rnemd *r, double *dp)
{
    RnArgs R;
    R.hist = at<int32_t>(c.ws, c.L.rn_hist);
    R.bcnt = at<int32_t>(c.ws, c.L.rn_bcnt);
    R.ctl = at<int32_t>(c.ws, c.L.rn_ctl);
    R.key = at<double>(c.ws, c.L.rn_key);
    R.id = at<int32_t>(c.ws, c.L.rn_id);
    R.kk = at<int32_t>(c.ws, c.L.rn_k);
    launch_rnemd_on(R, st, c.sys, x, v, tag, r, dp, c.status);
}

// ---------------------------------------------------------------------------
// The exchange without allocation: its buffers live in one static device
// array per GPU (the control words and histogram first, cleared by every
// call, then the block counts and the candidate lists, which every call
// writes before it reads them).  Each device's copy of the array sits at its
// own address, looked up once per device with that device current; host code
// uses only that address, never the array's name.
constexpr size_t RNS_CTL = 0, RNS_HIST = 256, RNS_BCNT = RNS_HIST + sizeof(int32_t) * 2 * RN_BINS,
                 RNS_KEY = RNS_BCNT + sizeof(int32_t) * 2 * RN_HBLOCKS, RNS_ID = RNS_KEY + sizeof(double) * 2 * RN_CAP,
                 RNS_K = RNS_ID + sizeof(int32_t) * 2 * RN_CAP, RNS_BYTES = RNS_K + sizeof(int32_t) * 2 * RN_CAP;
static_assert(RNS_BYTES == MPCD_RNEMD_SCRATCH_BYTES, "the exchange's static scratch size");
static_assert(RNS_HIST % 256 == 0 && RNS_BCNT % 256 == 0 && RNS_KEY % 256 == 0 && RNS_ID % 256 == 0 &&
                  RNS_K % 256 == 0, "256-byte aligned parts");

static __device__ __align__(256) unsigned char scratch[RNS_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[SCRATCH_MAX_DEVICES];

// The device address of this device's scratch array (looked up on the first
// call per device, with the device current).
static int scratch_on_device(int dev, void **out)
{
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return MPCD_ENOTSUP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        TRY(hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))));
        if (!ptr) return MPCD_EHIP;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return MPCD_OK;
}

int mpcd_rnemd_exchange(void *stream, const mpcd_sys *sys, const void *x, void *v, const int32_t *tag,
                        const mpcd_rnemd *r, double *dp, void *ws, size_t ws_bytes)
{
    TRY(rnemd_checks(sys, x, v, tag, r, dp, ws, ws_bytes));
    launch_rnemd(make_ctx(sys, ws), (hipStream_t)stream, x, v, tag, r, dp);
    return launch_check();
}

int mpcd_rnemd_exchange_noalloc(void *stream, const mpcd_sys *sys, const void *x, void *v, const int32_t *tag,
                                const mpcd_rnemd *r, double *dp, uint32_t *status)
{
    TRY(check_sys(sys));
    if (!r || !dp || !aligned(dp, 8) || !status || !aligned(status, 4)) return MPCD_EINVAL;
    if (sys->nsys != 1) return MPCD_ENOTSUP;
    if (!ok_arr(x, sys->n_solvent, esize(sys)) || !ok_arr(v, sys->n_solvent, esize(sys))) return MPCD_EINVAL;
    if (tag && !aligned(tag, 4)) return MPCD_EINVAL;
    // the scratch holds the lists of npairs <= RN_MAXPAIRS ranked members
    if (!(r->dy > 0.0) || r->npairs < 0 || r->npairs > RN_MAXPAIRS) return MPCD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    TRY(hip_check(hipGetDevice(&dev)));
    if (st) {  // the stream must belong to the current device (the array is per device)
        int sdev = -1;
        TRY(hip_check(hipStreamGetDevice(st, &sdev)));
        if (sdev != dev) return MPCD_EINVAL;
    }
    void *ptr = nullptr;
    TRY(scratch_on_device(dev, &ptr));
    char *w = (char *)ptr;
    if (sys->n_solvent == 0 || r->npairs == 0) return MPCD_OK;
    // control words and histogram start at zero (a fill kernel, not a memset node)
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for((int64_t)(RNS_BCNT / 4), 256)), dim3(256), 0, st, (int32_t *)w,
                       (int64_t)(RNS_BCNT / 4), 0);
    RnArgs R;
    R.ctl = (int32_t *)(w + RNS_CTL);
    R.hist = (int32_t *)(w + RNS_HIST);
    R.bcnt = (int32_t *)(w + RNS_BCNT);
    R.key = (double *)(w + RNS_KEY);
    R.id = (int32_t *)(w + RNS_ID);
    R.kk = (int32_t *)(w + RNS_K);
    launch_rnemd_on(R, st, sys, x, v, tag, r, dp, status);
    return launch_check();
}

static int step_checks(const mpcd_step_args *a)
{
    if (!a || !a->sys) return MPCD_EINVAL;
    const mpcd_sys *s = a->sys;
    const mpcd_params &p = a->par;
    TRY(thermalize_checks(s, &a->bodies, p.kT, p.thermalize, a->d_step, a->xs, a->vs, a->ws, a->ws_bytes));
    TRY(wca_check(&p.wca));
    if (!tune_ok(p.tune, s->prec == MPCD_F64)) return MPCD_EINVAL;
    if (!(p.dt > 0.0)) return MPCD_EINVAL;
    if (!ok_arr(a->J, s->n_bodies, 8) || !ok_arr(a->K, s->n_bodies, 8)) return MPCD_EINVAL;
    if (a->binned) {  // x and x_out: the solvent records of this step and the next
        TRY(check_binned(s, a->binned));
        if (s->prec != MPCD_F32 || a->rnemd || !p.fuse_stream) return MPCD_ENOTSUP;
        if (!a->x || !a->x_out || !aligned(a->x, 16) || !aligned(a->x_out, 16) || a->x == a->x_out) return MPCD_EINVAL;
        if (a->v || a->tag || a->v_out || a->tag_out || a->reorder_every != 0) return MPCD_EINVAL;
        if (s->n_sites > 0 && !a->bodies.site_m) return MPCD_EINVAL;
        return MPCD_OK;
    }
    TRY(bin_checks(s, a->x, a->xs, &a->bodies, a->d_step, a->ws, a->ws_bytes));
    TRY(collide_checks(s, a->v, a->tag, a->vs, &a->bodies, a->d_step, a->ws, a->ws_bytes, a->x, p.dt));
    if (a->reorder_every < 0 || (a->reorder_every > 0 && !ok_arr(a->tag, s->n_solvent, 4))) return MPCD_EINVAL;
    TRY(out_checks(s, a->v, a->tag, a->x, a->x_out, a->v_out, a->tag_out));
    if (a->v_out && !p.fuse_stream) return MPCD_ENOTSUP;
    if (a->rnemd)
        TRY(rnemd_checks(s, a->v_out ? a->x_out : a->x, a->v_out ? a->v_out : a->v, a->tag, a->rnemd, a->rnemd_dp,
                         a->ws, a->ws_bytes));
    return MPCD_OK;
}

// Reverse nonequilibrium exchange at the end of a step, on the new solvent.
static void step_rnemd(const Ctx &c, hipStream_t st, const mpcd_step_args *a)
{
    if (!a->rnemd) return;
    if (a->v_out)
        launch_rnemd(c, st, a->x_out, a->v_out, a->tag_out, a->rnemd, a->rnemd_dp);
    else
        launch_rnemd(c, st, a->x, a->v, a->tag, a->rnemd, a->rnemd_dp);
}

// Overlap schedule of a captured run of out-of-place steps: the solvent of
// step t+1 is binned on a second stream right after step t's collision
// (it needs only the new solvent positions), beside step t's body update;
// step t+1 then thermalizes and bins its sites alone and joins that binning
// before its scan.  The early binning reads the step index t+1 that the
// collision stored, not the counter that step t's force kernel advances.
//
// Schedule 2 (fused): step t's force kernel also runs step t+1's first kernel
// (k_forces_prep: each body block computes its forces and kick, then
// thermalizes and bins its sites for t+1; extra blocks bin the new solvent),
// so step t+1 starts at its scan and its scatter clears the body-centre grid.
// Centre-centre WCA only (site-site WCA has a force kernel of its own).
//
// Schedule 3: as schedule 2, but step t's collision bins the new solvent for
// t+1 itself (it holds the new positions in registers), so the fused force
// kernel runs its body blocks only.
struct Overlap {
    int mode;         // 1: side stream; 2: fused into the force kernel; 3: 2 with the solvent binned by the collision
    hipStream_t side;
    hipEvent_t fork, join;
    bool pre_binned;  // this step's first kernel has run already (mode 1: its solvent part, joined by `join`)
    bool bin_next;    // run the next step's first kernel (its solvent part with mode 1) during this step
};

static int overlap_mode(const mpcd_step_args *a)
{
    const int m = a->par.tune.overlap;
    if (!m || !a->v_out || a->reorder_every != 0 || a->sys->n_bodies == 0 || a->sys->n_sites == 0 ||
        a->sys->n_solvent == 0)
        return 0;
    if (m >= 2 && a->par.wca.mode == 2) return 0;
    return m;
}

// One step: [thermalize + site binning | solvent binning] (one launch), scan,
// [scatter | per-cell draws] (one launch), collide + stream, transfer fused
// with the first body half-step, forces fused with the second half kick and
// the step-counter advance.  The same operations in the same order, per
// particle, cell and body, as calling the entry points in sequence.
// One step of the binned layout: thermalize + site binning, the brick
// collision (collide, stream, bin the new solvent for the next step),
// transfer fused with the first body half-step, forces fused with the second
// half kick and the step-counter advance.  (Fusing the forces with the next
// step's thermalization into one launch was slower: one-wave force blocks,
// and thermalization blocks without the force code's LDS and registers, each
// fill the CUs better.)
static int step_binned(void *stream, const mpcd_step_args *a)
{
    const mpcd_sys *s = a->sys;
    const mpcd_params &p = a->par;
    const Ctx c = make_ctx(s, a->ws, &p.tune);
    hipStream_t st = (hipStream_t)stream;
    launch_therm_bin(c, st, &a->bodies, p.kT, p.thermalize, p.seed, a->d_step, a->xs, a->vs, a->binned);
    launch_brick_collide(c, st, a);
    if (s->n_bodies == 0) {
        const BinnedDev bn = binned_dev(s, a->binned);
        hipLaunchKernelGGL(k_binned_finish, dim3(grid_for(bn.nbricks, 256)), dim3(256), 0, st, bn, a->d_step);
        hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, a->d_step);
        return launch_check();
    }
    launch_transfer_first(c, st, &a->bodies, a->vs, a->J, a->K, p.dt, p.wca, a->binned, a->d_step);
    launch_forces(c, st, &a->bodies, p.wca, p.f_ext, p.dt, 1, a->d_step);
    return launch_check();
}

static int step_impl(void *stream, const mpcd_step_args *a, const Overlap *ov)
{
    TRY(step_checks(a));
    if (a->binned) return step_binned(stream, a);
    const mpcd_sys *s = a->sys;
    const mpcd_params &p = a->par;
    const Ctx c = make_ctx(s, a->ws, &p.tune);
    hipStream_t st = (hipStream_t)stream;
    const bool fused_in = ov && ov->mode >= 2 && ov->pre_binned;  // first kernel ran in the last step's
    if (ov && ov->pre_binned) {
        if (ov->mode == 1) {
            launch_prep(c, st, &a->bodies, p.kT, p.thermalize, p.seed, a->d_step, a->x, a->xs, a->vs, p.wca, 1);
            TRY(hip_check(hipStreamWaitEvent(st, ov->join, 0)));
        }
    } else {
        launch_prep(c, st, &a->bodies, p.kT, p.thermalize, p.seed, a->d_step, a->x, a->xs, a->vs, p.wca);
    }
    launch_scan(c, st);
    CollideArgs A = collide_args(c, a->tag, &a->bodies, p.cos_a, p.sin_a, p.kT_cell, p.seed, a->d_step, p.dt,
                                 nullptr);
    uint64_t *step_next = at<uint64_t>(c.ws, c.L.step_next);
    if (ov && ov->bin_next) A.step_next = step_next;
    if (ov && ov->bin_next && ov->mode == 3) {  // the collision bins the new solvent for the next step
        A.bin_counts = at<u64>(c.ws, c.L.counts);
        A.bin_cellid = at<int32_t>(c.ws, c.L.cellid);
        A.bin_slot = at<int32_t>(c.ws, c.L.slot);
    }
    if (p.fuse_stream) A.F = make_forcing(p.g, p.dt);
    const BodyGrid grid = body_grid(c, p.wca);
    int32_t *clear_grid = fused_in ? grid.count : nullptr;
    const int64_t grid_n = clear_grid ? (int64_t)c.L.grid_mask + 1 : 0;
    if (p.tune.draws_inline) {  // the collision draws; the scatter runs alone
        A.inline_draws = 1;
        launch_scatter(c, st, clear_grid, grid_n);
    } else {
        launch_scatter_draws(c, st, A, clear_grid, grid_n);
    }
    if (a->v_out)
        launch_collide(c, st, A, a->v, a->vs, a->x, a->x_out, a->v_out, a->tag_out);
    else
        launch_collide(c, st, A, a->v, a->vs, p.fuse_stream ? a->x : nullptr);
    if (ov && ov->bin_next && ov->mode == 1) {  // next step's solvent binning beside this step's body update
        TRY(hip_check(hipEventRecord(ov->fork, st)));
        TRY(hip_check(hipStreamWaitEvent(ov->side, ov->fork, 0)));
        launch_prep(c, ov->side, &a->bodies, p.kT, p.thermalize, p.seed, step_next, a->x_out, a->xs, a->vs, p.wca,
                    2);
        TRY(hip_check(hipEventRecord(ov->join, ov->side)));
    }
    if (!p.fuse_stream) TRY(mpcd_stream(stream, s, a->x, a->v, p.dt, p.g, a->ws, a->ws_bytes));
    if (s->n_bodies == 0) {
        hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, a->d_step);
        step_rnemd(c, st, a);
        return launch_check();
    }
    launch_transfer_first(c, st, &a->bodies, a->vs, a->J, a->K, p.dt, p.wca);
    if (ov && ov->bin_next && ov->mode >= 2)  // forces, kick and the next step's first kernel in one launch
        launch_forces_prep(c, st, &a->bodies, p.wca, p.f_ext, p.dt, a->d_step, p.kT, p.thermalize, p.seed, step_next,
                           a->x_out, a->xs, a->vs, ov->mode == 2);
    else
        launch_forces(c, st, &a->bodies, p.wca, p.f_ext, p.dt, 1, a->d_step);
    step_rnemd(c, st, a);
    return launch_check();
}

int mpcd_step(void *stream, const mpcd_step_args *a) { return step_impl(stream, a, nullptr); }

int mpcd_forces_prep(void *stream, const mpcd_step_args *a, const uint64_t *step_next)
{
    TRY(step_checks(a));
    if (!ok_arr(step_next, 1, 8)) return MPCD_EINVAL;
    const mpcd_sys *s = a->sys;
    const mpcd_params &p = a->par;
    if (s->n_bodies == 0 || s->n_sites == 0 || p.wca.mode == 2) return MPCD_ENOTSUP;
    const Ctx c = make_ctx(s, a->ws, &p.tune);
    launch_forces_prep(c, (hipStream_t)stream, &a->bodies, p.wca, p.f_ext, p.dt, a->d_step, p.kT, p.thermalize,
                       p.seed, step_next, a->x, a->xs, a->vs);
    return launch_check();
}

int mpcd_graph_create(void *stream, const mpcd_step_args *args, int32_t nsteps, void **graph_exec)
{
    if (!stream || !args || nsteps < 1 || !graph_exec) return MPCD_EINVAL;
    TRY(step_checks(args));
    // out of place (the dense form's three output arrays, or the binned records)
    const bool oop = args->x_out != nullptr;
    if (oop && ((nsteps & 1) || (!args->binned && !args->tag))) return MPCD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    // (the binned layout's steps are captured as they run eagerly)
    const int omode = (nsteps < 2 || args->binned) ? 0 : overlap_mode(args);
    Overlap ov{omode, nullptr, nullptr, nullptr, false, false};
    const bool overlap = omode != 0;
    if (omode == 1) {  // default-priority side stream and the two events, for the capture only
        int rc0 = hip_check(hipStreamCreateWithFlags(&ov.side, hipStreamNonBlocking));
        if (rc0 == MPCD_OK) rc0 = hip_check(hipEventCreateWithFlags(&ov.fork, hipEventDisableTiming));
        if (rc0 == MPCD_OK) rc0 = hip_check(hipEventCreateWithFlags(&ov.join, hipEventDisableTiming));
        if (rc0 != MPCD_OK) {
            if (ov.join) (void)hipEventDestroy(ov.join);
            if (ov.fork) (void)hipEventDestroy(ov.fork);
            if (ov.side) (void)hipStreamDestroy(ov.side);
            return rc0;
        }
    }
    auto release = [&]() {
        if (omode != 1) return;
        (void)hipEventDestroy(ov.join);
        (void)hipEventDestroy(ov.fork);
        (void)hipStreamDestroy(ov.side);
    };
    int rc = hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    if (rc != MPCD_OK) {
        release();
        return rc;
    }
    mpcd_step_args swapped = *args;  // odd steps of the out-of-place form: outputs become inputs
    if (oop) {
        swapped.x = args->x_out;
        swapped.v = args->v_out;
        swapped.tag = args->tag_out;
        swapped.x_out = args->x;
        swapped.v_out = args->v;
        swapped.tag_out = (int32_t *)args->tag;
    }
    for (int i = 0; i < nsteps && rc == MPCD_OK; ++i) {
        ov.pre_binned = overlap && i > 0;
        ov.bin_next = overlap && i + 1 < nsteps;
        rc = step_impl(stream, (oop && (i & 1)) ? &swapped : args, overlap ? &ov : nullptr);
        if (rc == MPCD_OK && !oop && args->reorder_every > 0 && (i + 1) % args->reorder_every == 0)
            rc = mpcd_reorder(stream, args->sys, args->x, args->v, (int32_t *)args->tag, args->ws, args->ws_bytes);
    }
    hipGraph_t graph = nullptr;
    const int rc_end = hip_check(hipStreamEndCapture(st, &graph));
    if (rc == MPCD_OK) rc = rc_end;
    hipGraphExec_t exec = nullptr;
    if (rc == MPCD_OK) rc = hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    if (graph) (void)hipGraphDestroy(graph);
    release();
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

// ---- harmonic-bond comparator ----

static HarmDev make_harmdev(const mpcd_sys *sys, const mpcd_harm *h)
{
    HarmDev d;
    d.B = sys->n_bodies;
    d.S = sys->n_sites;
    d.site_off = h->site_off;
    d.site_body = h->site_body;
    d.adj_off = h->adj_off;
    d.adj = h->adj;
    d.adj_r0 = h->adj_r0;
    d.rc0 = h->rc0;
    d.site_m = h->site_m;
    d.vc = h->vc;
    d.fs = h->fs;
    d.fc = h->fc;
    d.imgs = h->imgs;
    d.imgc = h->imgc;
    d.mc = h->mc;
    d.kb = h->kb;
    return d;
}

static int harm_checks(const mpcd_sys *sys, const mpcd_harm *h, const double *xs, const mpcd_wca *wca, void *ws,
                       size_t ws_bytes)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    TRY(wca_check(wca));
    if (!h || sys->prec != MPCD_F64) return h ? MPCD_ENOTSUP : MPCD_EINVAL;
    if (wca->mode == 2) return MPCD_ENOTSUP;
    const int64_t S = sys->n_sites, B = sys->n_bodies;
    if (!ok_arr(xs, S, 8) || !ok_arr(h->xs_alt, S, 8) || !ok_arr(h->xc, B, 8) || !ok_arr(h->xc_alt, B, 8) ||
        !ok_arr(h->vc, B, 8) || !ok_arr(h->fs, S, 8) || !ok_arr(h->fc, B, 8) || !ok_arr(h->imgs, S, 4) ||
        !ok_arr(h->imgc, B, 4) || !ok_arr(h->site_off, B + 1, 8) || !ok_arr(h->site_body, S, 4) ||
        !ok_arr(h->adj_off, S + 1, 8) || !ok_arr(h->rc0, S, 8) || !ok_arr(h->site_m, S, 8))
        return MPCD_EINVAL;
    if (!(h->mc > 0.0) || !(h->kb >= 0.0)) return MPCD_EINVAL;
    return MPCD_OK;
}

static void launch_harm(const Ctx &c, hipStream_t st, const mpcd_harm *h, const mpcd_wca &wca, const double *xs_in,
                        double *xs_out, double *vs, const double *xc_in, double *xc_out, double dt, int phase)
{
    const int64_t S = c.sys->n_sites, B = c.sys->n_bodies;
    const int nsb = (int)((S + BODY_T - 1) / BODY_T);
    if (nsb + B == 0) return;
    hipLaunchKernelGGL(k_harm_substep, dim3((unsigned)(nsb + B)), dim3(BODY_T), 0, st, c.sd, make_harmdev(c.sys, h),
                       wca, xs_in, xs_out, vs, xc_in, xc_out, dt, phase, nsb, c.status);
}

int harm_forces(void *stream, const mpcd_sys *sys, const mpcd_harm *h, const double *xs, const mpcd_wca *wca,
                void *ws, size_t ws_bytes)
{
    TRY(harm_checks(sys, h, xs, wca, ws, ws_bytes));
    launch_harm(make_ctx(sys, ws), (hipStream_t)stream, h, *wca, xs, nullptr, nullptr, h->xc, nullptr, 1.0, 3);
    return launch_check();
}

int harm_md(void *stream, const mpcd_sys *sys, const mpcd_harm *h, double *xs, double *vs, const mpcd_wca *wca,
            double dt, int32_t nsub, void *ws, size_t ws_bytes)
{
    TRY(harm_checks(sys, h, xs, wca, ws, ws_bytes));
    if (!ok_arr(vs, sys->n_sites, 8) || !(dt > 0.0) || nsub < 2 || (nsub & 1)) return MPCD_EINVAL;
    const Ctx c = make_ctx(sys, ws);
    hipStream_t st = (hipStream_t)stream;
    double *xsb[2] = {xs, h->xs_alt}, *xcb[2] = {h->xc, h->xc_alt};
    launch_harm(c, st, h, *wca, xsb[0], xsb[1], vs, xcb[0], xcb[1], dt, 0);
    for (int i = 1; i < nsub; ++i)
        launch_harm(c, st, h, *wca, xsb[i & 1], xsb[(i + 1) & 1], vs, xcb[i & 1], xcb[(i + 1) & 1], dt, 1);
    launch_harm(c, st, h, *wca, xsb[0], nullptr, vs, xcb[0], nullptr, dt, 2);
    return launch_check();
}

// One collision period of the harmonic model: bin solvent and surface sites,
// per-cell draws, collision (the surface sites as heavy solvent) fused with the
// solvent streaming, nsub Verlet steps of dt_md for the sites, step counter.
int harm_step(void *stream, const mpcd_step_args *a, const mpcd_harm *h, double dt_md, int32_t nsub)
{
    if (!a || !a->sys) return MPCD_EINVAL;
    const mpcd_sys *s = a->sys;
    const mpcd_params &p = a->par;
    TRY(harm_checks(s, h, (const double *)a->xs, &p.wca, a->ws, a->ws_bytes));
    if (!p.fuse_stream || p.thermalize) return MPCD_ENOTSUP;
    TRY(out_checks(s, a->v, a->tag, a->x, a->x_out, a->v_out, a->tag_out));
    TRY(mpcd_bin(stream, s, a->x, a->xs, &a->bodies, p.seed, a->d_step, a->ws, a->ws_bytes));
    TRY(mpcd_cell_draws(stream, s, p.kT_cell, p.seed, a->d_step, a->ws, a->ws_bytes));
    TRY(mpcd_collide_drawn(stream, s, a->v, a->tag, a->vs, &a->bodies, p.cos_a, p.sin_a, p.kT_cell, a->d_step,
                           a->ws, a->ws_bytes, a->x, p.dt, a->x_out, a->v_out, a->tag_out, p.seed, nullptr));
    TRY(harm_md(stream, s, h, (double *)a->xs, (double *)a->vs, &p.wca, dt_md, nsub, a->ws, a->ws_bytes));
    return mpcd_advance_step(stream, a->d_step);
}

int harm_graph_create(void *stream, const mpcd_step_args *args, const mpcd_harm *h, double dt_md, int32_t nsub,
                      int32_t nperiods, void **graph_exec)
{
    if (!stream || !args || !h || nperiods < 1 || !graph_exec) return MPCD_EINVAL;
    if (args->v_out && ((nperiods & 1) || !args->tag)) return MPCD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    mpcd_step_args swapped = *args;
    if (args->v_out) {
        swapped.x = args->x_out;
        swapped.v = args->v_out;
        swapped.tag = args->tag_out;
        swapped.x_out = args->x;
        swapped.v_out = args->v;
        swapped.tag_out = (int32_t *)args->tag;
    }
    TRY(hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)));
    int rc = MPCD_OK;
    for (int i = 0; i < nperiods && rc == MPCD_OK; ++i)
        rc = harm_step(stream, (args->v_out && (i & 1)) ? &swapped : args, h, dt_md, nsub);
    hipGraph_t graph = nullptr;
    const int rc_end = hip_check(hipStreamEndCapture(st, &graph));
    if (rc == MPCD_OK) rc = rc_end;
    hipGraphExec_t exec = nullptr;
    if (rc == MPCD_OK) rc = hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    if (graph) (void)hipGraphDestroy(graph);
    TRY(rc);
    *graph_exec = (void *)exec;
    return MPCD_OK;
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

int mpcd_binned_sites(void *stream, const mpcd_step_args *a)
{
    TRY(step_checks(a));
    if (!a->binned) return MPCD_EINVAL;
    const mpcd_params &p = a->par;
    const Ctx c = make_ctx(a->sys, a->ws, &p.tune);
    hipStream_t st = (hipStream_t)stream;
    const BinnedDev bn = binned_dev(a->sys, a->binned);
    hipLaunchKernelGGL(k_binned_clear_sites, dim3(grid_for(bn.nbricks, 256)), dim3(256), 0, st, bn);
    launch_therm_bin(c, st, &a->bodies, p.kT, p.thermalize, p.seed, a->d_step, a->xs, a->vs, a->binned);
    return launch_check();
}

int mpcd_binned_collide(void *stream, const mpcd_step_args *a)
{
    TRY(step_checks(a));
    if (!a->binned) return MPCD_EINVAL;
    const Ctx c = make_ctx(a->sys, a->ws, &a->par.tune);
    hipStream_t st = (hipStream_t)stream;
    const BinnedDev bn = binned_dev(a->sys, a->binned);
    hipLaunchKernelGGL(k_binned_clear_out, dim3(grid_for(bn.nbricks, 256)), dim3(256), 0, st, bn, a->d_step);
    launch_brick_collide(c, st, a);
    return launch_check();
}

int mpcd_binned_layout(const mpcd_sys *sys, const int32_t *ncell, const int64_t *solv_off, const int64_t *site_off_sys,
                       mpcd_binned *out)
{
    if (!out) return MPCD_EINVAL;
    BinnedPlan P;
    TRY(binned_plan(sys, ncell, solv_off, site_off_sys, false, P));
    out->nbricks = P.nbricks;
    out->capacity = P.cap;
    out->site_slots = P.sslots;
    out->items = sys->prec == MPCD_F64 ? 0
                 : P.nbricks >= BRICK_WIDE_MIN ? BRICK_MEMBERS_WIDE / BRICK_T_WIDE : BRICK_MEMBERS_NARROW / BRICK_T_NARROW;
    out->ws_bytes = binned_layout(sys, P.nbricks, P.sslots, P.sovf_cap).total;
    return MPCD_OK;
}

int mpcd_binned_init(void *stream, const mpcd_sys *sys, const int32_t *ncell, const int64_t *solv_off,
                     const int64_t *site_off_sys, const mpcd_binned *b)
{
    BinnedPlan P;
    TRY(binned_plan(sys, ncell, solv_off, site_off_sys, true, P));
    TRY(check_binned(sys, b));
    if (P.nbricks != b->nbricks || P.cap != b->capacity || P.sslots != b->site_slots) return MPCD_EINVAL;
    const BinnedLayout L = binned_layout(sys, P.nbricks, P.sslots, P.sovf_cap);
    char *w = (char *)b->ws;
    hipStream_t st = (hipStream_t)stream;
    // every launch before this copy has finished; the copy blocks until done
    TRY(hip_check(hipStreamSynchronize(st)));
    TRY(hip_check(hipMemcpy(w + L.brick, P.brick.data(), sizeof(BrickInfo) * P.brick.size(), hipMemcpyHostToDevice)));
    TRY(hip_check(hipMemcpy(w + L.subpre, P.subpre.data(), sizeof(int32_t) * P.subpre.size(), hipMemcpyHostToDevice)));
    TRY(hip_check(hipMemcpy(w + L.sys_bb, P.sys_bb.data(), sizeof(int32_t) * P.sys_bb.size(), hipMemcpyHostToDevice)));
    TRY(hip_check(hipMemcpy(w + L.sys_bg, P.sys_bg.data(), sizeof(int32_t) * P.sys_bg.size(), hipMemcpyHostToDevice)));
    TRY(hip_check(hipMemcpy(w + L.wtab, P.wtab.data(), sizeof(int4) * P.wtab.size(), hipMemcpyHostToDevice)));
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, (int32_t *)(w + L.ctrl), (int64_t)BC_WORDS, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(2 * NCLS * P.nbricks, 256)), dim3(256), 0, st,
                       (int32_t *)(w + L.cnt), 2 * NCLS * P.nbricks, 0);  // both parities' fills
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(P.nbricks, 256)), dim3(256), 0, st, (int32_t *)(w + L.scnt),
                       P.nbricks, 0);  // the site counts
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(2 * P.nbricks, 256)), dim3(256), 0, st, (int32_t *)(w + L.oflag),
                       2 * P.nbricks, 0);  // the overflow flags
    const int64_t tab_words = 4 * (1 + 6 * (int64_t)sys->nsys);  // both shift tables: NaN, matching no step
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(tab_words, 256)), dim3(256), 0, st, (int32_t *)(w + L.shtab),
                       tab_words, -1);
    return launch_check();
}

int mpcd_binned_pack(void *stream, const mpcd_sys *sys, const void *x, const void *v, const int32_t *tag, void *rec,
                     uint64_t seed, const uint64_t *d_step, void *ws, size_t ws_bytes, const mpcd_binned *b)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    TRY(check_binned(sys, b));
    const size_t es = esize(sys);
    const int64_t N = sys->n_solvent;
    if (!ok_arr(x, N, es) || !ok_arr(v, N, es) || !ok_arr(tag, 0, 4) || !rec || !aligned(rec, 16) || !d_step)
        return MPCD_EINVAL;
    const BinnedDev bn = binned_dev(sys, b);
    const SysDev sd = make_sysdev(sys);
    hipStream_t st = (hipStream_t)stream;
    uint32_t *status = at<uint32_t>(ws, layout_of(sys).status);
    // clear both parities' fills and overflow counters: the step parity is read on the device
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(2 * NCLS * bn.nbricks, 256)), dim3(256), 0, st, bn.cnt,
                       2 * NCLS * bn.nbricks, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, bn.ctrl + BC_OVF0, (int64_t)2, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(2 * bn.nbricks, 256)), dim3(256), 0, st, bn.oflag, 2 * bn.nbricks, 0);
    hipLaunchKernelGGL(k_binned_shtab, dim3(1), dim3(256), 0, st, sd, bn, seed, d_step);
    if (N > 0) {
        const unsigned g = grid_for(N, 256, 1 << 16);
        if (sys->prec == MPCD_F64)
            hipLaunchKernelGGL(k_binned_pack<double>, dim3(g), dim3(256), 0, st, sd, bn, seed, d_step,
                               (const double *)x, (const double *)v, tag, (double *)rec, status);
        else
            hipLaunchKernelGGL(k_binned_pack<float>, dim3(g), dim3(256), 0, st, sd, bn, seed, d_step,
                               (const float *)x, (const float *)v, tag, (float *)rec, status);
    }
    return launch_check();
}

int mpcd_binned_unpack(void *stream, const mpcd_sys *sys, const void *rec, void *x, void *v, int32_t *tag,
                       const uint64_t *d_step, void *ws, size_t ws_bytes, const mpcd_binned *b)
{
    TRY(check_sys(sys));
    TRY(check_ws(sys, ws, ws_bytes));
    TRY(check_binned(sys, b));
    const size_t es = esize(sys);
    const int64_t N = sys->n_solvent;
    if (!ok_arr(x, N, es) || !ok_arr(v, N, es) || !ok_arr(tag, N, 4) || !rec || !aligned(rec, 16) || !d_step)
        return MPCD_EINVAL;
    if (N == 0) return MPCD_OK;
    const BinnedDev bn = binned_dev(sys, b);
    const SysDev sd = make_sysdev(sys);
    hipStream_t st = (hipStream_t)stream;
    uint32_t *status = at<uint32_t>(ws, layout_of(sys).status);
    const unsigned g = (unsigned)std::min<int64_t>(bn.nbricks, 1 << 16);
    if (sys->prec == MPCD_F64)
        hipLaunchKernelGGL(k_binned_unpack<double>, dim3(g), dim3(256), 0, st, sd, bn, d_step, (const double *)rec,
                           (double *)x, (double *)v, tag, status);
    else
        hipLaunchKernelGGL(k_binned_unpack<float>, dim3(g), dim3(256), 0, st, sd, bn, d_step, (const float *)rec,
                           (float *)x, (float *)v, tag, status);
    return launch_check();
}

}  // extern "C"
