/*
 * mpcd.h -- C ABI of libmpcd.so: one step of multiparticle collision dynamics
 * (MPCD, stochastic rotation dynamics) with colloids represented as rigid
 * bodies of discrete surface sites, as hand-written HIP kernels for gfx950.
 *
 * Method: Bush, Palmer, Howard, "Simulating hydrodynamic interactions in
 * colloidal suspensions using multiparticle collision dynamics with rigid-body
 * constraints", arXiv 2604.14307.  Section/equation numbers below refer to it.
 *
 * One step, in this order (the paper does not fix the order; the collision is
 * taken at the start of the step and the collision period equals the step):
 *   sites_thermalize  Eq. (5) site positions/velocities, then Eq. (7)
 *   mpcd_bin          random grid shift + counting sort of solvent and sites
 *   mpcd_collide      per-cell SRD rotation (+ optional cell thermostat),
 *                     optionally fused with the solvent streaming
 *   sites_to_body     net momentum J and angular momentum K of each body's sites
 *   body_integrate    impulse (J, K) + quaternion velocity-Verlet (Miller et al.)
 *   mpcd_stream       ballistic solvent streaming (when not fused)
 *   mpcd_advance_step step counter += 1 (on the device)
 * mpcd_step runs the whole sequence.
 *
 * Conventions (all entry points):
 *  - Every array argument is a DEVICE pointer unless marked "host".  The caller
 *    owns and allocates every buffer, including the workspace of
 *    mpcd_workspace_bytes() bytes.  The library keeps no pointer after a call.
 *  - Arrays are component-major ("SoA"): x[0..n) are the x components,
 *    x[n..2n) the y components, x[2n..3n) the z components.  Per-system arrays
 *    (ncell, offsets) are system-major.  Quaternions are (w, x, y, z).
 *  - Solvent and site positions/velocities are double when prec == MPCD_F64,
 *    float when prec == MPCD_F32.  Body arrays are always double.
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as
 *    void*), allocate nothing, never synchronize (except mpcd_status) and are
 *    graph-capturable.  The step index is read from a device uint64_t so a
 *    captured graph replays correctly.
 *  - Several independent periodic boxes ("systems", e.g. replicas) may be
 *    advanced together: nsys > 1 with per-system offsets.  A system's results
 *    do not depend on the other systems.
 *  - Random numbers: Philox4x64-10, key (seed, purpose), counter
 *    (step, entity, replica0 + system, call); purpose 0 grid shift (entity 0),
 *    1 a cell's collision axis and thermostat Gamma variate (entity = cell
 *    index within its system; a call's four words read as eight 32-bit
 *    halves, high half first.  The axis comes from call 0 without rejection:
 *    half 0 gives z uniform in (-1, 1), half 1 the azimuth phi (Archimedes),
 *    n = (sqrt(1-z^2) cos phi, sqrt(1-z^2) sin phi, z).  While the variate is
 *    pending, each call's halves 2 and 3 give a Box-Muller normal pair and
 *    halves 4 and 5 the uniforms of two Marsaglia-Tsang tests, the cosine
 *    normal first; calls continue until one test accepts, at most 64),
 *    3 site velocities (entity = site index within its system; one call,
 *    Box-Muller pairs from words (0, 1) and (2, 3), the second pair's sine
 *    dropped).
 *  - Limits: total solvent + sites < 2^31; total cells < 2^31.
 *
 * Errors: 0 on success, else a negative code below; nothing is launched then.
 * Device-side anomalies set sticky bits in the workspace, read by mpcd_status.
 */
#ifndef MPCD_H
#define MPCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { MPCD_F64 = 0, MPCD_F32 = 1 };

enum {
    MPCD_OK = 0,
    MPCD_EINVAL = -1,     /* null/misaligned pointer, bad size or parameter */
    MPCD_EWORKSPACE = -2, /* workspace too small */
    MPCD_EHIP = -3,       /* a HIP call failed: see mpcd_last_hip_error() */
    MPCD_ENOTSUP = -4     /* unsupported precision/feature combination */
};

/* Sticky status bits. */
#define MPCD_FLAG_NONFINITE 1u /* a NaN/Inf velocity, position or momentum    */
#define MPCD_FLAG_ESCAPE 2u    /* a particle moved more than one box length    */
#define MPCD_FLAG_FIXOVF 4u    /* FP32 path: fixed-point cell sum overflow     */
#define MPCD_FLAG_RNGLOOP 8u   /* a rejection sampler used all 64 Philox calls */
#define MPCD_FLAG_BINERR 16u   /* inconsistent binning counts (particles dropped) */
#define MPCD_FLAG_REACH 32u    /* WCA mode 2: a site lies beyond mpcd_wca.reach  */
#define MPCD_FLAG_CROWD 64u    /* FP64: a cell above 16384 members was not collided
                                  (its canonical ordering is quadratic)          */

/* Geometry and sizes of nsys independent periodic boxes of cubic cells. */
typedef struct {
    int32_t nsys;         /* number of systems (>= 1)                          */
    int32_t prec;         /* MPCD_F64 or MPCD_F32 solvent/site storage          */
    double a;             /* cell edge (> 0); box edge of system r = ncell * a  */
    double m_solvent;     /* solvent particle mass (> 0)                        */
    int64_t n_solvent;    /* host: total solvent particles over all systems     */
    int64_t n_sites;      /* host: total surface sites                          */
    int64_t n_bodies;     /* host: total rigid bodies                           */
    int64_t n_cells;      /* host: total cells = sum over r of nx*ny*nz         */
    uint64_t replica0;    /* host: Philox replica id of system 0                */
    const int32_t *ncell;    /* [3*nsys] cells per axis (nx,ny,nz) of system r  */
    const int64_t *solv_off; /* [nsys+1] solvent of system r: [off[r], off[r+1]) */
    const int64_t *cell_off; /* [nsys+1] global cell index of system r's cell 0  */
    const int64_t *body_off; /* [nsys+1] bodies of system r                      */
} mpcd_sys;

/* Rigid bodies (always double).  Body b owns sites [site_off[b], site_off[b+1]). */
typedef struct {
    double *pos;            /* [3B] centre of mass R, wrapped into [0, L)      */
    int32_t *image;         /* [3B] periodic image counters of R                */
    double *quat;           /* [4B] orientation q (w,x,y,z), body -> space      */
    double *mom;            /* [3B] linear momentum P                           */
    double *angmom;         /* [4B] conjugate quaternion momentum p (Miller)    */
    double *force;          /* [3B] force from the last evaluation              */
    double *torque;         /* [3B] torque (space frame) from the last evaluation */
    const double *mass;     /* [B] total mass M = sum of site masses            */
    const double *inertia;  /* [3B] principal moments (body frame is principal) */
    const int64_t *site_off;  /* [B+1]                                          */
    const int32_t *site_body; /* [S] body of each site                          */
    const double *site_d;     /* [3S] body-frame site offsets from R            */
    const double *site_m;     /* [S] site masses                                */
} mpcd_bodies;

/* Colloid repulsion, Eq. (1): core-shifted WCA u(r; eps, sigma, delta), cut
 * at delta + 2^(1/6) sigma.  Mode 1: between body centres (forces only).
 * Mode 2: between surface sites of different bodies; the force on body b is
 * the sum of its sites' forces and its torque the sum of d_j x f_j (f_j summed
 * over the other bodies in ascending index and their sites in ascending
 * index; F and T in site order).  `reach` (mode 2) bounds |d_j| over all
 * sites; a site found farther from its body centre sets MPCD_FLAG_REACH. */
typedef struct {
    int32_t mode;        /* 0 off, 1 body centres, 2 sites of different bodies */
    double eps, sigma, delta;
    double reach;        /* mode 2: max distance of a site from its body centre */
} mpcd_wca;

/* Launch shapes of the step (all zero: defaults).  They change how work is
 * split over blocks, never the results: every choice gives the same bits.
 * A collision tile is a block of 256 threads that owns consecutive cells and
 * stages up to 256 * tile_items members in LDS; tile_items is 2, 4 or 8 for
 * FP32 (default 4) and 1, 2 or 4 for FP64 (default 2).  tile_fill (10..100,
 * default 70) is the percentage of that capacity an average tile may fill;
 * it sets the cells per tile (a power of two, 8..256).  draw_cells (1..16,
 * default 1) is the number of cells each lane of the per-cell draws takes.
 * draws_inline (0 or 1): 1 makes the collision draw each cell's random axis
 * and gamma variate itself, in place of a separate draws pass (the same
 * values).  overlap (0..3), for mpcd_graph_create (out-of-place steps
 * with sites and no reorder; elsewhere ignored): 1 bins the solvent of each
 * next step on a second stream beside the current step's body update; 2 runs
 * each next step's first kernel inside the current step's force kernel
 * (centre-centre WCA only); 3 is 2 with the next step's solvent binned by the
 * current step's collision (the force kernel then thermalizes and bins the
 * sites only).
 * Out-of-range values: MPCD_EINVAL. */
typedef struct {
    int32_t tile_items;
    int32_t tile_fill;
    int32_t draw_cells;
    int32_t draws_inline;
    int32_t overlap;
} mpcd_tune;

/* Scalars of one step. */
typedef struct {
    double dt;           /* step = collision period (0.1 tau in the paper)     */
    double cos_a, sin_a; /* SRD rotation angle (130 degrees in the paper)      */
    double kT;           /* site thermalization temperature, Eq. (7)           */
    double kT_cell;      /* cell thermostat temperature; <= 0 turns it off     */
    uint64_t seed;       /* Philox key word 0                                  */
    int32_t thermalize;  /* 1: Eq. (7) thermalization; 0: rigid velocities only */
    int32_t fuse_stream; /* 1: stream the solvent inside mpcd_collide          */
    mpcd_wca wca;
    /* Forced flow (sedimentation, Sec. III.B): every body feels the constant
     * force f_ext at its centre, and every solvent particle the constant
     * acceleration g, streamed as x + v dt + h with h = (dt/2)(g dt), then
     * v + g dt.  Choosing g = -B f_ext / (N m) makes the system force free.
     * All zero: no forcing. */
    double g[3];
    double f_ext[3];
    mpcd_tune tune;      /* launch shapes; zero: defaults                    */
} mpcd_params;

/* All buffers of one step (for mpcd_step and graph capture). */
typedef struct {
    const mpcd_sys *sys;   /* host pointer to the geometry                      */
    mpcd_bodies bodies;
    void *x, *v;           /* [3N] solvent positions, velocities (prec)         */
    const int32_t *tag;    /* [N] solvent identities, or NULL (= index)         */
    void *xs, *vs;         /* [3S] site positions, velocities (prec)            */
    double *J, *K;         /* [3B] collision impulse and angular impulse        */
    uint64_t *d_step;      /* device step counter                               */
    void *ws;              /* workspace                                         */
    size_t ws_bytes;
    mpcd_params par;
    int32_t reorder_every; /* graphs: mpcd_reorder after every this many steps (0: never;
                              ignored out of place)                             */
    /* Out-of-place solvent (all three set, or all NULL): the step reads x, v,
     * tag and writes the new solvent state to x_out, v_out, tag_out in cell
     * order (the storage order that makes the next step's gathers and
     * binning atomics local; it replaces mpcd_reorder).  Requires
     * fuse_stream = 1; the output arrays may not alias the inputs; the
     * inputs are left unchanged.  The caller swaps the two sets after each
     * step.  mpcd_graph_create then captures an even number of steps that
     * alternate between the two sets, so a replay leaves the state in x, v,
     * tag (tag must then be non-NULL). */
    void *x_out, *v_out;   /* [3N] (prec)                                        */
    int32_t *tag_out;      /* [N]                                                */
    /* Optional reverse nonequilibrium exchange after the step (NULL: none):
     * see mpcd_rnemd_exchange; rnemd_dp is its device accumulator. */
    const struct mpcd_rnemd_s *rnemd;
    double *rnemd_dp;
    /* Binned solvent layout (NULL: the dense layout above).  When set, x and
     * x_out are the solvent record arrays of this step and the next
     * (binned->capacity records each, 16-byte aligned, see
     * mpcd_binned_layout), and v, tag, v_out, tag_out must be NULL. */
    const struct mpcd_binned_s *binned;
} mpcd_step_args;

/* Binned solvent layout, a storage form of the solvent in which one step of
 * the collision (Sec. II.A) reads and writes each solvent particle once.
 *
 * Each system's cells are grouped into bricks of up to 8 x 8 x 4 cells
 * (smaller bricks for denser systems; narrower at the far faces of the box).
 * A solvent particle is one record: in FP32 seven floats, 28 bytes (position
 * x, y, z; its identity as the int32 bits of the fourth value; velocity x, y,
 * z), in FP64 eight doubles (the same with one unused value).  The record array
 * holds one region per brick: on a step with index t, a particle is stored in
 * the region of the brick of its cell on step t's shifted grid.  A region is
 * split into 27 sub-regions, one per brick that can write into it (the brick
 * itself and its neighbours along each axis), each of fixed capacity (mean
 * occupancy + 6 standard deviations + 16; none for a neighbour that does not
 * exist), in no particular order within a sub-region.  The step collides each
 * brick's particles and sites in one block and writes each new solvent
 * particle straight into its writer's sub-region of the region of its brick
 * on step t+1's grid, so every sub-region has one writer, which also stores
 * its fill: no device atomics.  The record arrays are double-buffered (x ->
 * x_out, swapped by the caller after every step, as in the out-of-place
 * dense form).  Sub-region fills are kept in the binned workspace per step
 * parity (the parity of *d_step), which is why the caller's swap must follow
 * every step.  A particle beyond its sub-region's capacity, or beyond the
 * neighbouring bricks, goes to a shared overflow list of 8192 entries per
 * parity (the brick is flagged for its reader); beyond that list
 * MPCD_FLAG_BINERR is set and the state is invalid.  The surface sites are
 * listed per brick by the thermalization of the same step (sites beyond a
 * brick's list go to a second shared list).  Results are identical to the
 * dense form's in identity order (the same per-cell sums, draws and
 * rounding).  FP32 only: other precisions return MPCD_ENOTSUP from the step;
 * no reverse nonequilibrium exchange.
 *
 * Host fields are filled by mpcd_binned_layout; ws and ws_bytes are the
 * caller's device buffer for the brick tables, fills, site lists and
 * overflow lists (allocated by the caller, >= 256-byte aligned). */
typedef struct mpcd_binned_s {
    void *ws;            /* device: binned workspace                          */
    size_t ws_bytes;     /* bytes of ws (>= the ws_bytes the layout reports)  */
    int64_t nbricks;     /* host: bricks over all systems                     */
    int64_t capacity;    /* host: records of one solvent record array         */
    int64_t site_slots;  /* host: site list entries over all bricks           */
    int32_t items;       /* host: members per thread of a brick block: 7 in   */
                         /* four-wave blocks (layouts of 4096 bricks or more), */
                         /* else 4 in eight-wave blocks                        */
} mpcd_binned;

/* Plan of the binned layout (host only; no device work).  ncell: host
 * [3*nsys] cells per axis of each system; solv_off, site_off_sys: host
 * [nsys+1] offsets of each system's solvent and sites.  Fills every field of
 * *out except ws (out->ws_bytes: the bytes the binned workspace needs).
 * MPCD_EINVAL for inconsistent sizes or a system too dense for a brick. */
int mpcd_binned_layout(const mpcd_sys *sys, const int32_t *ncell, const int64_t *solv_off,
                       const int64_t *site_off_sys, mpcd_binned *out);

/* Write the brick tables of the layout into b->ws and clear its fills and
 * overflow counters.  The host arrays are those given to mpcd_binned_layout.
 * Synchronous (a blocking copy of the tables); call once before the first
 * pack. */
int mpcd_binned_init(void *stream, const mpcd_sys *sys, const int32_t *ncell, const int64_t *solv_off,
                     const int64_t *site_off_sys, const mpcd_binned *b);

/* Dense solvent (x, v: [3N] prec, tag: [N] identities or NULL = index) into
 * the record array rec (b->capacity records, 16-byte aligned) for the step
 * *d_step (its grid shift, Sec. II.A).  Clears both parities' fills and
 * overflow lists first, and stores that step's shift table. */
int mpcd_binned_pack(void *stream, const mpcd_sys *sys, const void *x, const void *v, const int32_t *tag, void *rec,
                     uint64_t seed, const uint64_t *d_step, void *ws, size_t ws_bytes, const mpcd_binned *b);

/* The solvent records of the step *d_step back to dense arrays in identity
 * order: x[:, id], v[:, id] of the particle with identity id, tag[id] = id.
 * The records and fills are left unchanged. */
int mpcd_binned_unpack(void *stream, const mpcd_sys *sys, const void *rec, void *x, void *v, int32_t *tag,
                       const uint64_t *d_step, void *ws, size_t ws_bytes, const mpcd_binned *b);

/* The first kernel of a step of the binned layout on its own: the sites of
 * step *d_step placed and thermalized (Eqs. (5) and (7), as sites_thermalize)
 * and listed in the bricks of their cells on that step's grid (Sec. II.A),
 * after clearing the site lists.  Followed by mpcd_binned_collide it gives
 * the step's collision; mpcd_step runs both itself (with clear lists), so do
 * not call it before mpcd_step.  args as for mpcd_step, with args->binned
 * set; MPCD_EINVAL without it. */
int mpcd_binned_sites(void *stream, const mpcd_step_args *args);

/* The collision of one step of the binned layout alone (Sec. II.A, with the
 * sites as heavy solvent, Sec. II.B.2): collide, stream and bin the solvent
 * records of step *d_step from x into x_out (the next step's regions, whose
 * fills it stores), and write the sites' new velocities
 * in place.  It needs that step's sites thermalized and listed (as mpcd_step
 * does first) and leaves the input fills, the site lists and the step counter
 * unchanged, so it can be launched again on the same input (the sites then
 * enter with the velocities it wrote).  args as for mpcd_step, with
 * args->binned set; MPCD_EINVAL without it. */
int mpcd_binned_collide(void *stream, const mpcd_step_args *args);

/* Workspace bytes for sys (host-side sizes only).  The workspace holds the cell
 * counts and starts, the per-particle cell/slot/permutation, the per-step grid
 * shifts, per-site scratch and the status word.  Initialise once with
 * mpcd_ws_init before the first step. */
size_t mpcd_workspace_bytes(const mpcd_sys *sys);

/* Cell storage order.  The cell lists (cell_start, the permutation) and the
 * out-of-place solvent hold a system's cells in brick order: bricks of
 * 8 x 8 x 4 cells (narrower at the far faces), bricks x-fastest, the cells of
 * a brick x-fastest; systems follow each other.  pos (host, [sum of the
 * systems' cell counts]) receives, for every cell in canonical order (system,
 * then (j_z n_y + j_y) n_x + j_x), its global storage position.  ncell: host
 * [3*nsys].  Host only; no device work. */
int mpcd_cell_order(int32_t nsys, const int32_t *ncell, int64_t *pos);

/* The collision tiles a tuning gives for sys (host only): out[0] items per
 * thread, out[1] cells per tile, out[2] member capacity, out[3] tiles.
 * tune may be NULL (defaults). */
int mpcd_tile_shape(const mpcd_sys *sys, const mpcd_tune *tune, int32_t out[4]);

/* Byte offsets inside the workspace (for inspection by tests and tools):
 * out[0] status word (uint32), out[1] grid shifts [3*nsys] (double),
 * out[2] cell_start [n_cells+1] (int32, cells in storage order, see
 * mpcd_cell_order), out[3] permutation [N+S] (int32, particles grouped by
 * cell, solvent before sites within a cell), out[4] storage position of
 * each particle's cell (int32),
 * out[5] slot within the cell (int32), out[6] site offsets d_j [3S] (double),
 * out[7] site velocities entering the collision [3S] (double). */
int mpcd_workspace_offsets(const mpcd_sys *sys, int64_t out[8]);

/* Zero the cell counters, the reverse nonequilibrium exchange's histograms
 * and control words and the status word of a fresh workspace (any prior
 * contents); every other region is written before it is read. */
int mpcd_ws_init(void *stream, const mpcd_sys *sys, void *ws, size_t ws_bytes);

/* Streaming, Sec. II.A: x <- wrap(x + v dt) per component, one periodic
 * correction.  g (host, 3 doubles, or NULL): a constant acceleration (forced
 * flow, Sec. III.B), x <- wrap((x + v dt) + (dt/2)(g dt)), v <- v + g dt.
 * x, v: [3N] (prec); v is written only when g is non-zero. */
int mpcd_stream(void *stream, const mpcd_sys *sys, void *x, void *v, double dt, const double *g,
                void *ws, size_t ws_bytes);

/* Random grid shift and cell binning, Sec. II.A.  Shift s in [-a/2, a/2)^3 per
 * system and step on a 2^-24 a grid; particle k (solvent 0..N-1, then sites
 * N..N+S-1) goes to cell floor((x - s)/a) mod n of its system; counting sort
 * (count, exclusive scan, scatter) into the workspace.  x: [3N], xs: [3S]
 * (prec); bodies supplies site_body/site_off (may be NULL when S == 0). */
int mpcd_bin(void *stream, const mpcd_sys *sys, const void *x, const void *xs,
             const mpcd_bodies *bodies, uint64_t seed, const uint64_t *d_step, void *ws,
             size_t ws_bytes);

/* SRD collision, Sec. II.A; sites take part like heavy solvent, Sec. II.B.2.
 * For every cell with >= 2 particles: M, P summed over its members (FP64: in
 * ascending identity -- solvent tag, then N_total + site index; FP32: exact
 * int64 fixed-point sums at 2^-32), u = P/M, random axis n, rotation R(n, a);
 * with kT_cell > 0 the relative kinetic energy E is rescaled to
 * kT_cell * Gamma(3(n_c - 1)/2) (Eq. (6) with 3(n_c-1) degrees of freedom);
 * v <- u + lambda R (v - u).  When x_stream != NULL the solvent is then streamed
 * by dt in the same pass.  Requires mpcd_bin for the same step.
 * v: [3N], vs: [3S] (prec, in place); tag: [N] or NULL. */
int mpcd_collide(void *stream, const mpcd_sys *sys, void *v, const int32_t *tag, void *vs,
                 const mpcd_bodies *bodies, double cos_a, double sin_a, double kT_cell,
                 uint64_t seed, const uint64_t *d_step, void *ws, size_t ws_bytes,
                 void *x_stream, double dt);

/* mpcd_collide in two parts.  mpcd_cell_draws draws every cell's random axis
 * (Sec. II.A) and, when kT_cell > 0, its Gamma(3(n_c - 1)/2) variate (Eq. (6))
 * into the workspace, from the cell occupancies of the last mpcd_bin.
 * mpcd_collide_drawn then performs the collision of mpcd_collide with those
 * draws; kT_cell must be the value given to mpcd_cell_draws.  The pair gives
 * the same results as mpcd_collide.  With x_out, v_out, tag_out non-NULL
 * (all three) the solvent is collided and streamed out of place, as in
 * mpcd_step: x_stream (required) and v, tag are read and left unchanged, and
 * the new state goes to the outputs in cell order.  tune (host, may be NULL
 * for the defaults) sets the collision tile shape, as in mpcd_params; with
 * tune->draws_inline the collision draws each cell's axis and gamma variate
 * itself (from seed and *d_step) and mpcd_cell_draws is not needed. */
int mpcd_cell_draws(void *stream, const mpcd_sys *sys, double kT_cell, uint64_t seed,
                    const uint64_t *d_step, void *ws, size_t ws_bytes);
int mpcd_collide_drawn(void *stream, const mpcd_sys *sys, void *v, const int32_t *tag, void *vs,
                       const mpcd_bodies *bodies, double cos_a, double sin_a, double kT_cell,
                       const uint64_t *d_step, void *ws, size_t ws_bytes, void *x_stream,
                       double dt, void *x_out, void *v_out, int32_t *tag_out, uint64_t seed,
                       const mpcd_tune *tune);

/* Site positions and thermalized velocities, Eqs. (5) and (7).  Per body:
 * V = P/M, omega = A (Lhat / I) with Lhat_k = p . P_k q / 2; site offset
 * d_j = A dhat_j, position wrap(R + d_j); random velocities vt_j ~ N(0, kT/m_j);
 * Vt = sum m_j vt_j / M, Lt = sum d_j x m_j vt_j, wt = A((A^T Lt) / I) (site
 * order); v_j = (V - Vt) + (omega - wt) x d_j + vt_j.  thermalize == 0 gives the
 * rigid velocities of Eq. (5).  Writes xs, vs: [3S] (prec) and keeps d_j and
 * the velocities entering the collision in the workspace. */
int sites_thermalize(void *stream, const mpcd_sys *sys, const mpcd_bodies *bodies, double kT,
                     int32_t thermalize, uint64_t seed, const uint64_t *d_step, void *xs,
                     void *vs, void *ws, size_t ws_bytes);

/* Momentum transfer, Sec. II.B.2: J_b = sum_j m_j (v_j - v_j^pre),
 * K_b = sum_j d_j x m_j (v_j - v_j^pre) in site order, double.  J, K: [3B]. */
int sites_to_body(void *stream, const mpcd_sys *sys, const mpcd_bodies *bodies, const void *vs,
                  void *ws, size_t ws_bytes, double *J, double *K);

/* Body update: P += J, p += 2 S(q)(0, A^T K); then one quaternion velocity-
 * Verlet step (Miller et al., cited in Sec. II.B.2): half kick with the stored
 * F, T; drift R += dt P/M (wrap, image); NO_SQUISH free rotation about body
 * axes 3,2,1,2,3 for dt/2, dt/2, dt, dt/2, dt/2; new F, T from Eq. (1); half
 * kick.  J, K may be NULL (no impulse). */
int body_integrate(void *stream, const mpcd_sys *sys, const mpcd_bodies *bodies, const double *J,
                   const double *K, const mpcd_wca *wca, const double *f_ext, double dt, void *ws,
                   size_t ws_bytes);

/* Evaluate F, T at the current positions (Eq. (1)); call once before the first
 * step so the first half kick uses the right force.  f_ext (host, 3 doubles,
 * or NULL): a constant force added at every body centre (Sec. III.B). */
int body_forces(void *stream, const mpcd_sys *sys, const mpcd_bodies *bodies, const mpcd_wca *wca,
                const double *f_ext, void *ws, size_t ws_bytes);

/* Reverse nonequilibrium shear, Sec. III.B (viscosity): the solvent in the
 * lower slab y0 <= y < y0 + dy is ranked by |v_x - target| and in the upper slab
 * y1 <= y < y1 + dy by |v_x + target| (ties: lower identity first); the first
 * min(npairs, n_lower, n_upper) of each exchange v_x pairwise, and *dp (device
 * double) accumulates the moved momentum m (v_lower - v_upper), in rank order.
 * One system (nsys == 1); npairs <= 1024.  The ranking reads the members
 * whose key lies in the key bins (width 1e-4 below 0.4096, then one bin for
 * all larger keys) up to the bin of the last ranked member: at most 2048 per
 * slab (more set MPCD_FLAG_BINERR, as in a slab whose ranked members reach the
 * last bin when that bin is crowded).  x, v: [3N] (prec); tag: [N] distinct
 * identities or NULL (index). */
typedef struct mpcd_rnemd_s {
    double y0, y1, dy;     /* slab lower edges and width                         */
    double target;         /* |target velocity| (0.5 in the paper)               */
    int32_t npairs;        /* pairs per exchange (100 in the paper)              */
} mpcd_rnemd;

int mpcd_rnemd_exchange(void *stream, const mpcd_sys *sys, const void *x, void *v, const int32_t *tag,
                        const mpcd_rnemd *r, double *dp, void *ws, size_t ws_bytes);

/* The same exchange with no allocation and no workspace, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Its buffers (histogram, control
 * words, candidate lists) are one static device array of
 * MPCD_RNEMD_SCRATCH_BYTES per GPU, held from the first call on that GPU
 * until the process ends; the call allocates nothing and calls no allocating
 * library routine.  Arguments, limits (nsys == 1, npairs <= 1024) and results
 * are those of mpcd_rnemd_exchange, bit for bit; status (device, 4-byte
 * aligned) receives the flags ORed in (MPCD_FLAG_BINERR as above), where
 * mpcd_rnemd_exchange uses the workspace's status word.  The stream must
 * belong to the current device (else MPCD_EINVAL).  Every call on a GPU uses
 * that GPU's one array: calls that overlap on one GPU (other streams, other
 * host threads) race and must be serialised by the caller.  Each call clears
 * what must start at zero itself; the array keeps the last call's lists. */
#define MPCD_RNEMD_SCRATCH_BYTES 106752
int mpcd_rnemd_exchange_noalloc(void *stream, const mpcd_sys *sys, const void *x, void *v, const int32_t *tag,
                                const mpcd_rnemd *r, double *dp, uint32_t *status);

/* Harmonic-bond comparator, Sec. II.B.1: a colloid is a centre site plus
 * surface sites; each surface site is bonded to its nearest surface neighbours
 * and to the centre by u_b = (k_b / 2)(r - r_b)^2, Eq. (2).  All sites move by
 * velocity Verlet with a small step dt_md; the surface sites collide like
 * heavy solvent (they are the "sites" of mpcd_sys, FP64 only), the centres
 * carry the WCA of Eq. (1) (mode 1) and do not collide.  Forces: a surface
 * site sums its surface bonds in stored (ascending partner) order, then its
 * centre bond; a centre sums its bonds in site order, then the WCA partners in
 * ascending index.  Bond vectors use the minimum image t - L rint(t / L).
 * Positions ping-pong between the caller's arrays and the _alt arrays inside
 * harm_md; after an (even) number of Verlet steps they are back in xs, xc. */
typedef struct {
    double *xs_alt;             /* [3S] second buffer of surface positions      */
    double *xc, *xc_alt, *vc;   /* [3B] centre positions (two buffers), velocities */
    double *fs, *fc;            /* [3S], [3B] forces at the current positions   */
    int32_t *imgs, *imgc;       /* [3S], [3B] periodic image counters           */
    double mc, kb;              /* centre mass, spring constant                 */
    const int64_t *site_off;    /* [B+1] surface sites of each colloid          */
    const int32_t *site_body;   /* [S] colloid of each surface site             */
    const int64_t *adj_off;     /* [S+1] bonds of each surface site             */
    const int32_t *adj;         /* bonded surface partner, ascending per site   */
    const double *adj_r0;       /* rest length of each listed bond              */
    const double *rc0;          /* [S] rest length of each centre bond          */
    const double *site_m;       /* [S] surface site masses                      */
} mpcd_harm;

/* Forces on all sites at the positions xs (surface) and h->xc (centres). */
int harm_forces(void *stream, const mpcd_sys *sys, const mpcd_harm *h, const double *xs,
                const mpcd_wca *wca, void *ws, size_t ws_bytes);
/* nsub (even, >= 2) velocity-Verlet steps of dt: v += (dt/2)(f/m), x += v dt
 * (wrapped, images counted), new forces, v += (dt/2)(f/m).  Requires the
 * forces of the current positions in h->fs, h->fc (harm_forces, or the last
 * harm_md). */
int harm_md(void *stream, const mpcd_sys *sys, const mpcd_harm *h, double *xs, double *vs,
            const mpcd_wca *wca, double dt, int32_t nsub, void *ws, size_t ws_bytes);
/* One collision period: grid shift and binning of solvent and surface sites,
 * collision (surface sites as heavy solvent) fused with solvent streaming over
 * par.dt (out of place when x_out.. are set), nsub Verlet steps of dt_md
 * (nsub dt_md = par.dt in the paper's protocol), step counter + 1.  a->xs,
 * a->vs are the surface sites (double); a->bodies supplies site_body and
 * site_m; par.thermalize must be 0 and par.fuse_stream 1. */
int harm_step(void *stream, const mpcd_step_args *a, const mpcd_harm *h, double dt_md, int32_t nsub);
/* A HIP graph of nperiods harm_step calls (even when out of place). */
int harm_graph_create(void *stream, const mpcd_step_args *a, const mpcd_harm *h, double dt_md,
                      int32_t nsub, int32_t nperiods, void **graph_exec);

/* Storage reorder: permute the solvent (x, v and identity tags, [3N], [3N],
 * [N]) into the order of the last mpcd_bin (grouped by cell), so that the
 * gathers of the next steps stay local as the solvent diffuses.  Changes only
 * where particles are stored: with tags, every result is the same as without
 * the reorder.  tag must be non-NULL (initially 0..N-1 in system order).
 * Uses the workspace's staging area; costs two passes over the solvent. */
int mpcd_reorder(void *stream, const mpcd_sys *sys, void *x, void *v, int32_t *tag, void *ws, size_t ws_bytes);

/* *d_step += 1 on the device. */
int mpcd_advance_step(void *stream, uint64_t *d_step);

/* One whole step (the sequence above), then mpcd_advance_step. */
int mpcd_step(void *stream, const mpcd_step_args *args);

/* The last kernel of step t fused with the first kernel of step t+1, as the
 * fused graph schedule (tune.overlap = 2) runs it, for callers that schedule
 * steps themselves: the body forces of Eq. (1) and the second half kick
 * (Sec. II.B.2) with the step-counter advance, then each body's sites
 * thermalized (Eq. 7) and binned, and the solvent x of args (the positions
 * step t wrote: after an out-of-place step, the caller's current arrays)
 * binned, for step t+1.  step_next: device uint64 holding t+1
 * (read on the device; *d_step still holds t).  Step t+1 then continues from
 * its scan, and its scatter must clear the body-centre grid (the fused graph
 * schedule does both).  Needs bodies with sites and centre-centre or no WCA:
 * otherwise MPCD_ENOTSUP. */
int mpcd_forces_prep(void *stream, const mpcd_step_args *args, const uint64_t *step_next);

/* Capture nsteps calls of mpcd_step into a HIP graph (stream must not be the
 * null stream); replay with mpcd_graph_launch; free with mpcd_graph_destroy. */
int mpcd_graph_create(void *stream, const mpcd_step_args *args, int32_t nsteps, void **graph_exec);
int mpcd_graph_launch(void *stream, void *graph_exec);
int mpcd_graph_destroy(void *graph_exec);

/* Synchronize the stream and copy the sticky status bits to *flags (host). */
int mpcd_status(void *stream, const void *ws, size_t ws_bytes, uint32_t *flags);

/* The HIP error code of the last MPCD_EHIP return (per thread). */
int mpcd_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MPCD_H */
