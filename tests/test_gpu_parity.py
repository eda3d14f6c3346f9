"""GPU parity: the HIP path through the C ABI against the CPU oracle.

FP64: bit-exact, per stage and per step (both sides evaluate the same
operations in the same order with contraction off and draw the same Philox
numbers).  FP32: from an identical (FP32-representable) state, one step is
within 1e-5 relative velocity error of the FP64 oracle, excluding cells whose
membership differs because FP32 rounding of x - s moved a particle across a
cell boundary (counted and bounded).
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2604_14307_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def gpu_system(*a, **k):
    from paper_2604_14307_amd.sim import GPUSystem
    return GPUSystem(*a, **k)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


STATE_KEYS = ("x", "v", "R", "img", "q", "P", "p", "F", "T", "xs", "vs")


def assert_same(o, gd, keys=STATE_KEYS, where=""):
    for k in keys:
        a = getattr(o, k)
        b = gd[k]
        assert a.shape == b.shape, (k, a.shape, b.shape)
        if not np.array_equal(a, b):
            diff = np.argwhere(a != b)
            i = tuple(diff[0])
            raise AssertionError("%s: %s differs at %s (%d elements): oracle %r gpu %r"
                                 % (where, k, i, len(diff), a[i], b[i]))


def run_parity(wl, par, nsteps, fuse=True, check_every=1, step0=0, reorder_every=0, out_of_place=True,
               after_step=None):
    o = oracle.OracleSystem(wl, par)
    g = gpu_system(wl, par, prec="f64", fuse_stream=fuse, out_of_place=out_of_place)
    o.body_forces()
    g.body_forces()
    g.set_step(step0)
    assert_same(o, g.download()[0], ("F", "T"), "initial forces")
    for n in range(nsteps):
        assert o.step(step0 + n) == 0
        g.step(1)
        if after_step:
            after_step(o, n)
        if reorder_every and (n + 1) % reorder_every == 0:
            g.reorder()
        if (n + 1) % check_every == 0 or n == nsteps - 1:
            assert_same(o, g.download()[0], where="step %d" % (step0 + n))
    assert g.status() == 0
    return o, g


# ---------------------------------------------------------------------------

def test_device_double_sqrt_and_division_are_correctly_rounded():
    """The FP64 bit-exactness relies on IEEE correctly rounded / and sqrt."""
    rng = np.random.default_rng(0)
    n = 1 << 24
    for _ in range(4):
        a = np.exp(rng.uniform(-50, 50, n)) * rng.choice([-1.0, 1.0], n)
        b = np.exp(rng.uniform(-50, 50, n))
        ta, tb = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
        assert np.array_equal((ta / tb).cpu().numpy(), a / b)
        assert np.array_equal(torch.sqrt(tb).cpu().numpy(), np.sqrt(b))


def test_stages_bit_exact_single_sphere():
    wl, par, _ = W.config(0, kT_cell=1.0)
    o = oracle.OracleSystem(wl, par)
    g = gpu_system(wl, par, prec="f64")
    step = 7
    g.set_step(step)
    say("thermalize")
    o.sites_thermalize(step)
    g.sites_thermalize()
    gd = g.download()[0]
    assert_same(o, gd, ("xs", "vs"), "thermalize")
    d, vpre = g.site_state()
    assert np.array_equal(d, o.d) and np.array_equal(vpre, o.vpre)
    say("bin")
    sh = o.shift(step)
    cell, cs, mem, _ = o.bin(sh)
    g.bin()
    gcs, gperm, gshift = g.bins()
    assert np.array_equal(gshift[0], sh)
    assert np.array_equal(gcs, cs)
    for c in range(o.C):
        assert np.array_equal(np.sort(gperm[gcs[c]:gcs[c + 1]]), mem[cs[c]:cs[c + 1]])
    say("collide")
    o.collide(step, cs, mem)
    g.collide(stream_x=False)
    assert_same(o, g.download()[0], ("v", "vs"), "collide")
    say("transfer")
    J, K = o.sites_to_body()
    g.sites_to_body()
    gd = g.download()[0]
    assert np.array_equal(J, gd["J"]) and np.array_equal(K, gd["K"])
    say("stream")
    o.stream()
    g.stream_solvent()
    assert_same(o, g.download()[0], ("x",), "stream")
    say("bodies")
    o.body_integrate(J, K)
    g.body_integrate()
    assert_same(o, g.download()[0], ("R", "img", "q", "P", "p", "F", "T"), "body_integrate")
    assert g.status() == 0


@pytest.mark.parametrize("kT_cell", [1.0, 0.0])
def test_split_draws_then_collide_bit_exact(kT_cell):
    """mpcd_cell_draws + mpcd_collide_drawn equals the oracle's collision."""
    wl, par, _ = W.config(0, kT_cell=kT_cell)
    o = oracle.OracleSystem(wl, par)
    g = gpu_system(wl, par, prec="f64")
    step = 3
    g.set_step(step)
    o.sites_thermalize(step)
    g.sites_thermalize()
    cell, cs, mem, _ = o.bin(o.shift(step))
    g.bin()
    o.collide(step, cs, mem)
    say("split collide kT_cell=%g" % kT_cell)
    g.cell_draws()
    g.collide_drawn(stream_x=False)
    assert_same(o, g.download()[0], ("v", "vs"), "split collide")
    assert g.status() == 0


@pytest.mark.parametrize("kT_cell", [1.0, 0.0])
def test_single_sphere_100_steps_bit_exact(kT_cell):
    wl, par, meta = W.config(0, kT_cell=kT_cell)
    say("single sphere kT_cell=%g" % kT_cell)
    run_parity(wl, par, meta["steps"])


def test_in_place_form_bit_exact():
    """The in-place form (solvent storage order kept) over 100 steps."""
    wl, par, meta = W.config(0, kT_cell=1.0)
    say("in place")
    run_parity(wl, par, meta["steps"], check_every=10, out_of_place=False)


def test_binning_of_many_cells_matches_the_oracle():
    """Above 2^19 cells the scan takes 16 counters per thread (fewer, larger
    tiles); two binnings in a row (the second scan reads the first one's tile
    descriptors as stale) still give the oracle's cell lists."""
    wl = W.make_system((96, 96, 64), 2, [], [], np.zeros((0, 4)), np.random.default_rng(93))
    par = W.srd_params(93, kT_cell=1.0)
    o = oracle.OracleSystem(wl, par)
    g = gpu_system(wl, par, prec="f64")
    assert g.C > 2 ** 19
    for step in (5, 6):
        say("many-cell binning, step %d" % step)
        g.set_step(step)
        cell, cs, mem, _ = o.bin(o.shift(step))
        g.bin()
        gcs, gperm, _ = g.bins()
        assert np.array_equal(gcs, cs)
        owner = np.repeat(np.arange(o.C), np.diff(cs))
        a = np.lexsort((gperm, owner))
        b = np.lexsort((mem, owner))
        assert np.array_equal(gperm[a], mem[b])
    assert g.status() == 0


def test_out_of_place_step_writes_solvent_in_cell_order():
    """After an out-of-place step the solvent storage holds the previous
    storage's particles in the order of the step's cell lists (solvent before
    sites in each cell)."""
    wl, par, _ = W.config(0)
    g = gpu_system(wl, par, prec="f64")
    g.body_forces()
    g.step(2)
    tag_before = g.tag.cpu().numpy().copy()
    g.step(1)
    cs, perm, _ = g.bins(storage=True)
    sol = perm[perm < g.N]
    assert np.array_equal(g.tag.cpu().numpy(), tag_before[sol])
    for c in range(g.C):  # solvent first within each cell
        seg = perm[cs[c]:cs[c + 1]]
        kinds = seg >= g.N
        assert np.all(kinds[:-1] <= kinds[1:])
    # repeating the last collide + stream pass from its inputs gives the same bits
    before = g.download()[0]
    g.recollide_last()
    assert_same(oracle_like(before), g.download()[0], ("x", "v"), "recollide")


class oracle_like:
    def __init__(self, d):
        self.__dict__.update(d)


def test_storage_reorder_keeps_results_bit_exact():
    """Reordering the solvent storage (with identity tags) changes nothing."""
    wl, par, _ = W.config(0)
    say("reorder every 3 steps")
    o, g = run_parity(wl, par, 30, reorder_every=3, out_of_place=False)
    tag = g.tag.cpu().numpy()
    assert not np.array_equal(tag, np.arange(len(tag)))  # storage really was permuted
    assert np.array_equal(np.sort(tag), np.arange(len(tag)))


def test_unfused_stream_matches_fused():
    wl, par, _ = W.config(0)
    say("unfused")
    run_parity(wl, par, 20, fuse=False)


def test_naive_scheme_bit_exact():
    wl, par, _ = W.config(0)
    par = dict(par, thermalize=0)
    run_parity(wl, par, 20)


def test_suspension_with_wca_bit_exact():
    wl = W.suspension((12, 12, 12), 5, 6, 2.0, 60, 5.0, seed=31)
    par = W.srd_params(31, kT_cell=1.0, wca=W.wca_spheres(sigma=4.0))
    say("suspension 12^3, 6 bodies")
    run_parity(wl, par, 40, check_every=5)


def test_ragged_box_and_density_bit_exact():
    rng = np.random.default_rng(5)
    tpl = W.sphere_template(1.5, 40, 5.0)
    wl = W.make_system((7, 9, 11), 3.7, [tpl, tpl], [(2.0, 3.0, 4.0), (5.0, 6.5, 8.0)],
                       W.random_quaternions(rng, 2), rng)
    par = W.srd_params(77, kT_cell=1.0, wca=W.wca_spheres(sigma=3.0))
    say("ragged 7x9x11")
    run_parity(wl, par, 30, check_every=3)


def test_pure_solvent_and_sites_only():
    rng = np.random.default_rng(6)
    wl = W.make_system((6, 6, 6), 5, [], [], np.zeros((0, 4)), rng)
    say("pure solvent")
    run_parity(wl, W.srd_params(6), 10)
    tpl = W.sphere_template(2.0, 80, 5.0)
    wl = W.make_system((6, 6, 6), 0, [tpl], [(3.0, 3.0, 3.0)], np.array([[1.0, 0, 0, 0]]), rng)
    say("sites only")
    run_parity(wl, W.srd_params(7), 10)


def test_empty_cells_and_crowded_cells():
    """Density 0.5 leaves most cells empty or single; a dense clump makes cells
    with more members than the LDS-ordered fast path holds (slow path)."""
    rng = np.random.default_rng(8)
    wl = W.make_system((8, 8, 8), 0.5, [], [], np.zeros((0, 4)), rng)
    clump = np.array([[2.1], [2.2], [2.3]]) + 0.05 * rng.random((3, 60))
    wl["x"] = np.concatenate([wl["x"], clump], axis=1)
    wl["v"] = np.concatenate([wl["v"], 0.01 * rng.normal(size=(3, 60))], axis=1)
    say("empty + crowded")
    run_parity(wl, W.srd_params(8, kT_cell=1.0), 5)


def test_batched_replicas_match_each_replica_alone():
    systems, par, _ = W.batched_replicas(nrep=4, seed=9, lo=6, hi=10)
    say("batched 4 replicas")
    g = gpu_system(systems, par, prec="f64")
    g.body_forces()
    os_ = [oracle.OracleSystem(s, par, replica=r) for r, s in enumerate(systems)]
    for o in os_:
        o.body_forces()
    for n in range(15):
        for o in os_:
            assert o.step(n) == 0
        g.step(1)
    gd = g.download()
    for r, o in enumerate(os_):
        assert_same(o, gd[r], where="replica %d" % r)
    # replica 2 alone on the GPU with replica id 2 gives the same bits
    g2 = gpu_system(systems[2], par, prec="f64", replica0=2)
    g2.body_forces()
    g2.step(15)
    assert_same(os_[2], g2.download()[0], where="replica 2 alone")


@pytest.mark.parametrize("out_of_place", [True, False])
def test_graph_replay_matches_eager(out_of_place):
    wl, par, _ = W.config(0)
    say("graph out_of_place=%s" % out_of_place)
    ge = gpu_system(wl, par, prec="f64", out_of_place=out_of_place)
    gg = gpu_system(wl, par, prec="f64", out_of_place=out_of_place)
    for g in (ge, gg):
        g.body_forces()
    nsteps, every = (6, 0) if out_of_place else (5, 2)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        gg.graph(nsteps, reorder_every=every)
        for rep in range(4):
            gg.graph_launch()
            torch.cuda.synchronize()
            for i in range(nsteps):
                ge.step(1)
                if every and (i + 1) % every == 0:
                    ge.reorder()
            torch.cuda.synchronize()
            a, b = ge.download()[0], gg.download()[0]
            for k in STATE_KEYS:
                assert np.array_equal(a[k], b[k]), (rep, k)
            # storage order within a cell follows atomic arrival order, so only
            # the state in identity order is unique; the tags stay a permutation
            assert np.array_equal(np.sort(gg.tag.cpu().numpy()), np.arange(gg.N))
        gg.release_graph()


@pytest.mark.parametrize("mode,items,fill", [(1, 0, 0), (2, 0, 0), (3, 0, 0), (3, 1, 100)])
@pytest.mark.parametrize("prec,exchange", [("f64", False), ("f32", False), ("f32", True)])
def test_overlapped_graph_matches_eager(prec, exchange, mode, items, fill):
    """Graphs that run each next step's first kernel during the current step
    (mode 1: its solvent binning on a second stream beside the body update;
    mode 2: inside the force kernel; mode 3: the solvent binned by the
    collision, the sites in the force kernel) give the state of the same steps
    run one by one (bodies with sites, WCA, out of place; with the exchange
    appended).  The full-capacity tiles (fill 100) overflow often, so the
    collision's per-cell fallback bins its tiles too."""
    # density 8: the full-capacity tiles hold 8 cells' worth on average
    wl = W.suspension((14, 18, 11), 8 if fill else 5, 4, 2.0, 60, 5.0, seed=91)
    par = W.srd_params(91, kT_cell=1.0, wca=W.wca_spheres(sigma=4.0))
    say("overlapped graph %s exchange=%s mode %d items %d fill %d" % (prec, exchange, mode, items, fill))
    ge, gg = gpu_system(wl, par, prec=prec), gpu_system(wl, par, prec=prec)
    # both scatter kernels clear the body-centre grid in modes 2 and 3: the one
    # fused with the draws pass (FP32 here) and the one without it
    inl = 0 if (mode >= 2 and prec == "f32") else 1
    it = (2 if prec == "f32" else 1) if items else 0
    ge.set_tuning(it, fill, 0, inl, 0)
    gg.set_tuning(it, fill, 0, inl, mode)
    for g in (ge, gg):
        g.body_forces()
        if exchange:
            g.set_rnemd(0.0, 9.0, 1.0, 0.5, 20)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        gg.graph(6)
        for rep in range(3):
            gg.graph_launch()
            ge.step(6)
            torch.cuda.synchronize()
            a, b = ge.download()[0], gg.download()[0]
            for k in STATE_KEYS:
                assert np.array_equal(a[k], b[k]), (rep, k)
            assert float(ge.rnemd_dp.cpu()[0]) == float(gg.rnemd_dp.cpu()[0])
            assert int(ge.d_step.cpu()[0]) == int(gg.d_step.cpu()[0]) == 6 * (rep + 1)
        gg.release_graph()
    assert ge.status() == 0 and gg.status() == 0


def test_forces_prep_entry_point():
    """mpcd_forces_prep after step t: the counter advances to t+1, and its
    binning for t+1 (site positions and every particle's cell) equals that of
    the separate entry points (sites_thermalize, mpcd_bin) at step t+1.
    Bodies without sites, or with site-site WCA, are not supported."""
    wl = W.suspension((14, 18, 11), 5, 4, 2.0, 60, 5.0, seed=92)
    par = W.srd_params(92, kT_cell=1.0, wca=W.wca_spheres(sigma=4.0))
    ga, gb = gpu_system(wl, par, prec="f64"), gpu_system(wl, par, prec="f64")
    for g in (ga, gb):
        g.body_forces()
        g.step(3)
    t = int(ga.d_step.cpu()[0])
    nxt = torch.tensor([t + 1], dtype=torch.int64, device="cuda")
    ga.forces_prep(nxt)
    assert int(ga.d_step.cpu()[0]) == t + 1
    gb.set_step(t + 1)
    gb.sites_thermalize()
    gb.bin()
    ca = ga.ws_view("cellid", torch.int32, ga.N + ga.S).cpu().numpy()
    cb = gb.ws_view("cellid", torch.int32, gb.N + gb.S).cpu().numpy()
    # the solvent's storage order within a cell follows atomic arrival, so the
    # cells are compared by identity (tag); sites are stored in body order
    ida, idb = np.empty(ga.N, np.int32), np.empty(gb.N, np.int32)
    ida[ga.tag.cpu().numpy()] = ca[:ga.N]
    idb[gb.tag.cpu().numpy()] = cb[:gb.N]
    assert np.array_equal(ida, idb)
    assert np.array_equal(ca[ga.N:], cb[gb.N:])
    assert np.array_equal(ga.download()[0]["xs"], gb.download()[0]["xs"])
    assert ga.status() == 0 and gb.status() == 0
    # unsupported: pure solvent (no sites)
    ws = W.make_system((8, 8, 8), 5, [], [], np.zeros((0, 4)), np.random.default_rng(93))
    g0 = gpu_system(ws, W.srd_params(93, kT_cell=1.0), prec="f64")
    import ctypes
    a = g0.step_args()
    enotsup = -4  # MPCD_ENOTSUP
    assert g0.lib.mpcd_forces_prep(g0.stream, ctypes.byref(a), ctypes.c_void_p(nxt.data_ptr())) == enotsup


def point_bodies(ncell, centres, seed):
    """Bodies of one unit-mass site each at the given centres (no solvent)."""
    rng = np.random.default_rng(seed)
    tpl = W.rigid_template(np.zeros((1, 3)), 1.0)
    q = np.tile([1.0, 0.0, 0.0, 0.0], (len(centres), 1))
    return W.make_system(ncell, 0, [tpl] * len(centres), centres, q, rng)


# slots per bucket of the kernels' body-centre grid
GRID_SLOTS = 32


def fullest_grid_cell(centres, ncell, rc):
    """Bodies in the fullest cell of the body-centre grid (cells of edge
    L / floor(0.999 L / rc) per axis, as the kernels build it)."""
    L = np.asarray(ncell, dtype=np.float64)
    ng = np.maximum(np.floor(0.999 * L / rc), 1.0)
    cell = np.floor(np.asarray(centres) / (L / ng)).astype(np.int64)
    _, counts = np.unique(cell, axis=0, return_counts=True)
    return int(counts.max())


def ball_cluster(rng, n, centre, radius):
    """n points uniform in a ball."""
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    return np.asarray(centre) + d * (radius * rng.random(n) ** (1.0 / 3.0))[:, None]


@pytest.mark.parametrize("case", ["many", "crowded", "hits"])
def test_wca_forces_neighbour_grid_bit_exact(case):
    """Body-centre WCA forces through the hashed neighbour grid equal the
    oracle's all-pairs loop: 2000 random point bodies (many partners per
    body); 45 bodies crowded into one grid cell (a bucket of 32 slots
    overflows and the kernel falls back to all pairs); and a ball of 120
    bodies around one body at a grid corner, spread over eight cells, so
    that bodies have more partners within the cutoff than the kernel's hit
    list holds (96) while no bucket overflows (again all pairs)."""
    rng = np.random.default_rng(12)
    if case == "many":
        ncell, centres = (20, 20, 20), rng.random((2000, 3)) * 20.0
    elif case == "hits":
        ncell = (20, 20, 20)
        corner = np.full(3, 8 * 20.0 / 17.0)  # a corner of the grid's cells (17 per axis)
        centres = np.concatenate([corner[None, :], ball_cluster(rng, 120, corner, 1.0), rng.random((400, 3)) * 20.0])
        rc = 2.0 ** (1.0 / 6.0)
        assert fullest_grid_cell(centres, ncell, rc) <= GRID_SLOTS
        d = centres[:, None, :] - centres[None, :, :]
        d -= 20.0 * np.rint(d / 20.0)
        partners = ((d ** 2).sum(-1) <= rc * rc).sum(1) - 1
        assert partners.max() > 96
    else:
        ncell = (3, 3, 3)
        centres = np.concatenate([0.2 + 1.1 * rng.random((45, 3)), 1.6 + 1.3 * rng.random((10, 3))])
    wl = point_bodies(ncell, centres, 13)
    par = W.srd_params(13, wca=W.wca_spheres(sigma=1.0))
    if case == "crowded":
        assert fullest_grid_cell(centres, ncell, 2.0 ** (1.0 / 6.0)) > GRID_SLOTS
    o = oracle.OracleSystem(wl, par)
    g = gpu_system(wl, par, prec="f64")
    o.body_forces()
    g.body_forces()
    say("wca grid %s: %d bodies" % (case, g.B))
    assert_same(o, g.download()[0], ("F", "T"), "forces")
    assert np.count_nonzero(o.F) > 0
    assert g.status() == 0


def small_shapes(ncell, density, centres, seed):
    """Dumbbells (2 x 6 sites), 8-site cubes and 4-site rods, unit site mass."""
    rng = np.random.default_rng(seed)
    cube = np.array([[x, y, z] for x in (-0.7, 0.7) for y in (-0.7, 0.7) for z in (-0.7, 0.7)])
    rod = np.array([[0.0, 0.0, z] for z in (-1.5, -0.5, 0.5, 1.5)])
    dumb = np.concatenate([W.fibonacci_sphere(6, 0.6) + [0, 0, 1.2], W.fibonacci_sphere(6, 0.6) - [0, 0, 1.2]])
    kinds = [W.rigid_template(x, 1.0) for x in (dumb, cube, rod)]
    tpls = [kinds[b % 3] for b in range(len(centres))]
    return W.make_system(ncell, density, tpls, centres, W.random_quaternions(rng, len(centres)), rng)


def test_site_wca_mixed_shapes_bit_exact():
    """Cubes, rods and dumbbells in contact, WCA between sites of different
    bodies (forces and torques), full steps against the oracle.  The layout
    (random sequential addition of radius-1.3 spheres, seed 74) starts bodies
    in contact without violent overlaps; contacts come and go during the run,
    and the state compared after them carries their forces."""
    rng = np.random.default_rng(74)
    centres = W.rsa_positions_radii(rng, np.array([10.0, 10.0, 10.0]), np.full(10, 1.3))
    wl = small_shapes((10, 10, 10), 3, centres, 74)
    par = W.srd_params(74, kT_cell=1.0, wca=W.wca_sites(sigma=0.8))
    o0 = oracle.OracleSystem(wl, par)
    o0.body_forces()
    assert np.count_nonzero(o0.T) >= 6  # the bodies interact from the start
    say("site WCA shapes 10^3")
    contact = []
    o, g = run_parity(wl, par, 12, check_every=3, after_step=lambda o, n: contact.append(np.count_nonzero(o.T)))
    assert sum(c > 0 for c in contact[:-1]) >= 1, contact  # bodies touch again before the last comparison


@pytest.mark.parametrize("ncell", [(6, 6, 6), (6, 6, 4)])
def test_site_wca_small_box_bit_exact(ncell):
    """Two cubes in contact in a small box: site-site forces and torques, then
    full steps, against the oracle.  With 6 cells on every axis the kernel
    culls candidate sites by each wave's box; with 4 cells on one axis (no
    longer than twice the cubes' reach plus the cutoff) it keeps them all."""
    rng = np.random.default_rng(75)
    cube = np.array([[x, y, z] for x in (-0.7, 0.7) for y in (-0.7, 0.7) for z in (-0.7, 0.7)])
    tpl = W.rigid_template(cube, 1.0)
    # two unrotated cubes whose facing sites are 0.85 apart, inside the cutoff
    # 0.8 * 2^(1/6) but clear of the repulsive core
    centres = np.array([[1.5, 3.0, 3.0], [3.75, 3.0, 3.0]])
    quats = np.array([[1.0, 0.0, 0.0, 0.0]] * 2)
    if ncell[2] == 4:
        centres[:, 2] = 2.0
    wl = W.make_system(ncell, 3, [tpl] * 2, centres, quats, rng)
    par = W.srd_params(75, kT_cell=1.0, wca=W.wca_sites(sigma=0.8))
    o0 = oracle.OracleSystem(wl, par)
    o0.body_forces()
    assert np.count_nonzero(o0.F) >= 2  # the cubes interact from the start
    say("site WCA cubes %s" % (ncell,))
    run_parity(wl, par, 8, check_every=4)


def edge_system(a, ncell=(10, 10, 10), density=5, seed=77):
    """One sphere of 100 sites (radius 2a) at the centre of a box of cell edge a."""
    rng = np.random.default_rng(seed)
    tpl = W.sphere_template(2.0 * a, 100, 5.0)
    centre = 0.5 * a * np.asarray(ncell, dtype=np.float64)[None, :]
    return W.make_system(ncell, density, [tpl], centre, W.random_quaternions(rng, 1), rng, a=a)


@pytest.mark.parametrize("a", [0.5, 1.5])
def test_non_unit_cell_edge_bit_exact(a):
    """A cell edge other than 1: a power of two (the kernels multiply by its
    exact reciprocal) and 1.5 (they divide), full steps against the oracle."""
    wl = edge_system(a)
    par = W.srd_params(77, kT_cell=1.0)
    say("cell edge %g" % a)
    run_parity(wl, par, 6, check_every=3)


def test_bodies_of_more_sites_than_a_block_bit_exact():
    """Two spheres of 600 sites, three chunks of a 256-thread body block: the
    site thermalization stores and reloads the thermal velocities between
    its passes, and the transfer's ordered sums run over chunks.  Full steps
    against the oracle."""
    wl = W.suspension((12, 12, 12), 5, 2, 2.0, 600, 5.0, seed=36)
    par = W.srd_params(36, kT_cell=1.0, wca=W.wca_spheres(sigma=4.0))
    say("600-site spheres")
    run_parity(wl, par, 6, check_every=3)


def test_site_wca_bodies_of_more_sites_than_a_block_bit_exact():
    """Two spheres of 300 sites in contact through site-site WCA: each body's
    sites take two chunks of the block, and so do each candidate's staged
    sites, which the waves cull by their boxes.  Forces, torques and full
    steps against the oracle."""
    rng = np.random.default_rng(76)
    tpl = W.sphere_template(1.5, 300, 5.0)
    centres = np.array([[4.0, 5.0, 5.0], [7.25, 5.0, 5.0]])
    wl = W.make_system((10, 10, 10), 3, [tpl] * 2, centres, W.random_quaternions(rng, 2), rng)
    par = W.srd_params(76, kT_cell=1.0, wca=W.wca_sites(sigma=0.3))
    o0 = oracle.OracleSystem(wl, par)
    o0.body_forces()
    assert np.count_nonzero(o0.T) > 0  # the spheres interact from the start
    say("site WCA 300-site spheres")
    run_parity(wl, par, 6, check_every=3)


def test_site_wca_crowded_bodies_fall_back_to_all_pairs():
    """Small shapes packed so a grid bucket overflows: every body of the
    system becomes a candidate, with the same sums."""
    rng = np.random.default_rng(52)
    cube = np.array([[x, y, z] for x in (-0.5, 0.5) for y in (-0.5, 0.5) for z in (-0.5, 0.5)])
    tpl = W.rigid_template(cube, 1.0)
    centres = np.concatenate([0.5 + 2.5 * rng.random((45, 3)), 6.0 + 3.0 * rng.random((10, 3))])
    wl = W.make_system((10, 10, 10), 0, [tpl] * 55, centres, W.random_quaternions(rng, 55), rng)
    par = W.srd_params(52, wca=W.wca_sites(sigma=0.7))
    # the grid's cutoff for site-site WCA: twice the sites' reach plus the pair cutoff
    assert fullest_grid_cell(centres, (10, 10, 10), 2.0 * np.sqrt(0.75) + 0.7 * 2.0 ** (1.0 / 6.0)) > GRID_SLOTS
    o = oracle.OracleSystem(wl, par)
    g = gpu_system(wl, par, prec="f64")
    o.body_forces()
    g.body_forces()
    say("site WCA crowded")
    assert_same(o, g.download()[0], ("F", "T"), "forces")
    assert np.count_nonzero(o.T) > 0
    assert g.status() == 0


def test_site_wca_full_size_shapes_sampled():
    """128^3 cells, 21M solvent, 2000 cubes, rods and dumbbells (326,670 sites,
    placed without overlap): after 40 FP32 steps the FP64 site-site forces and
    torques of sampled bodies (some in contact) equal the oracle's at the same
    body poses."""
    wl, par, _ = W.config(4)
    say("complex shapes full size")
    g = gpu_system(wl, par, prec="f32")
    del wl["x"], wl["v"]
    g.body_forces()
    g.step(40)
    assert g.status() == 0
    gd = g.download()[0]
    touching = np.flatnonzero(np.abs(gd["F"]).sum(0) > 0)
    say("%d bodies in contact" % len(touching))
    assert len(touching) >= 4
    idx = np.unique(np.concatenate([[0, 1999], touching[:: max(1, len(touching) // 6)][:6]]))
    wl2 = dict(wl, x=np.zeros((3, 0)), v=np.zeros((3, 0)), R=gd["R"], q=gd["q"])
    o = oracle.OracleSystem(wl2, par)
    F, T, fl = o.site_wca_bodies(idx)
    assert fl == 0
    assert np.array_equal(F, gd["F"][:, idx]) and np.array_equal(T, gd["T"][:, idx])


@pytest.mark.parametrize("form", ["out_of_place", "in_place", "unfused"])
def test_forced_flow_bit_exact(form):
    """Sedimentation forcing (Sec. III.B): a constant force on every body and
    the balancing solvent acceleration, in every streaming form."""
    wl = W.suspension((12, 12, 12), 5, 4, 2.0, 60, 5.0, seed=63)
    par = W.sedimentation(W.srd_params(63, kT_cell=1.0, wca=W.wca_spheres(sigma=4.0)), wl, (0.5, 0.1, -0.2))
    say("forced flow %s" % form)
    run_parity(wl, par, 20, fuse=(form != "unfused"), out_of_place=(form == "out_of_place"), check_every=5)


def test_forced_flow_with_site_wca_bit_exact():
    rng = np.random.default_rng(74)
    centres = W.rsa_positions_radii(rng, np.array([10.0, 10.0, 10.0]), np.full(10, 1.3))
    wl = small_shapes((10, 10, 10), 3, centres, 74)
    par = W.sedimentation(W.srd_params(74, kT_cell=1.0, wca=W.wca_sites(sigma=0.8)), wl, (0.0, 0.0, 0.3))
    say("forced flow, site WCA")
    run_parity(wl, par, 8, check_every=4)


def test_full_size_suspension_bit_exact_few_steps():
    """60^3 cells, 1.08M solvent, 191 spheres x 200 sites, WCA: the benchmark
    workload, checked bit for bit over 3 steps."""
    wl, par, _ = W.config(1)
    say("full size 60^3")
    run_parity(wl, par, 3)


@pytest.mark.parametrize("ci,prec", [(1, "f64"), (1, "f32"), (3, "f32")])
def test_full_size_in_the_bench_launch_configuration(ci, prec):
    """The benchmark workloads (the 60^3 suspension; the 512 batched
    replicas, 17.4M solvent) run the way the bench times them: the committed
    tuned launch shape and schedule for the workload, steps as replays of a
    captured HIP graph on a side stream.  FP64: bit for bit against the oracle
    after 4 steps.  FP32: bit for bit against 4 eager steps of the same shape
    (the schedules change the order of launches, never the arithmetic)."""
    import os
    from paper_2604_14307_amd import tune
    wl, par = W.config(ci)[:2]
    cache = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2604_14307_amd",
                         "tuning_gfx950.json")
    g = gpu_system(wl, par, prec=prec)
    g.body_forces()
    e = tune.autotune(g, cache_path=cache, write=False)
    assert e["cached"]
    say("full size workload %d %s, tuned shape %s" % (ci, prec, list(e["tune"])))
    torch.cuda.synchronize()  # the set-up work ran on the default stream
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g.graph(2)
        g.graph_launch()
        g.graph_launch()
        torch.cuda.synchronize()
        g.release_graph()
    assert g.status() == 0
    if prec == "f64":
        o = oracle.OracleSystem(wl, par)
        o.body_forces()
        for n in range(4):
            assert o.step(n) == 0
        assert_same(o, g.download()[0], where="graph of the tuned shape")
    else:
        ge = gpu_system(wl, par, prec=prec)
        ge.set_tuning(*(list(e["tune"][:4]) + [0]))
        ge.body_forces()
        ge.step(4)
        a, b = ge.download()[0], g.download()[0]
        for k in STATE_KEYS:
            assert np.array_equal(a[k], b[k]), k
        assert ge.status() == 0


# ---------------------------------------------------------------------------
# FP32 form

def cells_of(cs, perm, nt):
    cell = np.empty(nt, dtype=np.int64)
    for c in range(len(cs) - 1):
        cell[perm[cs[c]:cs[c + 1]]] = c
    return cell


def fp32_one_step(wl, par, warm=3):
    g = gpu_system(wl, par, prec="f32")
    g.body_forces()
    g.step(warm)
    s0 = g.download()[0]
    step = warm
    # oracle state = the FP32 state upcast (exactly representable)
    wl2 = dict(wl)
    for k in ("x", "v", "R", "img", "q", "P", "p", "F", "T"):
        wl2[k] = s0[k]
    o = oracle.OracleSystem(wl2, par)
    o.sites_thermalize(step)
    cell64, cs64, mem64, _ = o.bin(o.shift(step))
    o.collide(step, cs64, mem64)
    J, K = o.sites_to_body()
    o.stream()
    o.body_integrate(J, K)
    g.sites_thermalize()
    g.bin()
    gcs, gperm, _ = g.bins()
    g.collide(stream_x=True)
    g.sites_to_body()
    g.body_integrate()
    g.advance()
    s1 = g.download()[0]
    nt = o.N + o.S
    # perm holds storage indices; solvent storage k holds identity tag[k]
    cell_st = cells_of(gcs, gperm, nt)
    tag = g.tag.cpu().numpy().astype(np.int64)
    cell32 = cell_st.copy()
    cell32[tag] = cell_st[:o.N]
    bad_cells = np.unique(np.concatenate([cell64[cell32 != cell64], cell32[cell32 != cell64]]))
    bad = np.isin(cell64, bad_cells) | np.isin(cell32, bad_cells)
    v64 = np.concatenate([o.v, o.vs], axis=1)[:, ~bad]
    v32 = np.concatenate([s1["v"], s1["vs"]], axis=1)[:, ~bad]
    rel = np.linalg.norm(v32 - v64) / np.linalg.norm(v64)
    return rel, int(bad.sum()), nt, g, o, s1


def test_fp32_one_step_within_1e5_of_fp64_oracle():
    wl, par, _ = W.config(0)
    rel, nbad, nt, g, o, s1 = fp32_one_step(wl, par)
    say("fp32 rel err %.3e, excluded %d of %d" % (rel, nbad, nt))
    assert rel <= 1e-5
    assert nbad <= 0.01 * nt
    assert g.status() == 0
    # the body update is FP64 from (almost) identical impulses
    assert np.allclose(s1["P"], o.P, rtol=1e-4, atol=1e-6)


def test_fp32_full_size_within_1e5():
    wl, par, _ = W.config(1)
    rel, nbad, nt, g, o, s1 = fp32_one_step(wl, par, warm=2)
    say("fp32 full size rel err %.3e, excluded %d of %d" % (rel, nbad, nt))
    assert rel <= 1e-5
    assert nbad <= 0.001 * nt


# ---------------------------------------------------------------------------
# Harmonic-bond comparator (Sec. II.B.1)

def harmonic_gpu(*a, **k):
    from paper_2604_14307_amd.sim import HarmonicGPU
    return HarmonicGPU(*a, **k)


HARM_KEYS = ("x", "v", "xs", "vs", "xc", "vc", "fs", "fc", "imgs", "imgc")


def harmonic_parity(hw, par, nper, nsub=50, dt_md=0.002):
    o = oracle.HarmonicOracle(hw, par)
    g = harmonic_gpu(hw, par)
    assert o.forces() == 0
    g.forces()
    assert_same(o, g.download(), ("fs", "fc"), "harmonic forces")
    for n in range(nper):
        assert o.step(n, dt_md, nsub) == 0
        g.step(dt_md, nsub)
        assert_same(o, g.download(), HARM_KEYS, "harmonic period %d" % n)
    assert g.status() == 0
    return o, g


def test_harmonic_single_sphere_bit_exact():
    wl, par, _ = W.config(0, kT_cell=1.0)
    say("harmonic single sphere")
    harmonic_parity(W.harmonic_from_rigid(wl), dict(par, thermalize=0), 6)


def test_harmonic_spheres_in_contact_bit_exact():
    wl = W.suspension((12, 12, 12), 3, 2, 1.5, 40, 5.0, seed=75)
    wl["R"][:, 0] = (4.0, 6.0, 6.0)
    wl["R"][:, 1] = (7.9, 6.3, 6.1)
    par = dict(W.srd_params(75, kT_cell=1.0, wca=W.wca_spheres(sigma=4.0)), thermalize=0)
    say("harmonic spheres in contact")
    o, g = harmonic_parity(W.harmonic_from_rigid(wl), par, 4)
    assert np.abs(o.fc).max() > 0


def test_harmonic_graph_matches_eager():
    wl, par, _ = W.config(0, kT_cell=1.0)
    hw, par = W.harmonic_from_rigid(wl), dict(par, thermalize=0)
    ge, gg = harmonic_gpu(hw, par), harmonic_gpu(hw, par)
    ge.forces()
    gg.forces()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        gg.graph(0.002, 50, 2)
        for rep in range(3):
            gg.graph_launch()
            ge.step(0.002, 50, 2)
            a, b = ge.download(), gg.download()
            for k in HARM_KEYS:
                assert np.array_equal(a[k], b[k]), (rep, k)
        gg.release_graph()


def test_harmonic_full_size_one_period_bit_exact():
    wl, par, _ = W.config(1, kT_cell=1.0)
    say("harmonic 60^3")
    harmonic_parity(W.harmonic_from_rigid(wl), dict(par, thermalize=0), 1)


# ---------------------------------------------------------------------------
# Reverse nonequilibrium shear (Sec. III.B)

@pytest.mark.parametrize("bodies", [False, True])
def test_rnemd_exchange_bit_exact(bodies):
    if bodies:
        wl = W.suspension((8, 16, 8), 5, 2, 1.5, 40, 5.0, seed=82)
        par = W.srd_params(82, kT_cell=1.0, wca=W.wca_spheres(sigma=3.0))
    else:
        wl = W.make_system((8, 16, 8), 5, [], [], np.zeros((0, 4)), np.random.default_rng(83))
        par = W.srd_params(83, kT_cell=1.0)
    o = oracle.OracleSystem(wl, par)
    g = gpu_system(wl, par, prec="f64")
    o.body_forces()
    g.body_forces()
    g.set_rnemd(0.0, 8.0, 1.0, 0.5, 12)
    dp = 0.0
    say("rnemd bodies=%s" % bodies)
    for n in range(30):
        assert o.step(n) == 0
        dp, ns = o.rnemd(0.0, 8.0, 1.0, 0.5, 12, dp)
        assert ns == 12
        g.step(1)
        if n % 5 == 4:
            assert_same(o, g.download()[0], ("x", "v", "P", "p"), "rnemd step %d" % n)
            assert float(g.rnemd_dp.cpu()[0]) == dp
    assert g.status() == 0


# The exchange's state occupies the end of the workspace: key-bin histograms
# (2 x 4096 int32), per-block member counts (2 x 1024 int32, rewritten by every
# exchange), 16 control words (padded to 256 bytes), then the candidate keys,
# identities and indices (2 x 2048 each).
RN_HIST, RN_BCNT, RN_CTL = 2 * 4096 * 4, 2 * 1024 * 4, 256
RN_TAIL = RN_HIST + RN_BCNT + RN_CTL + 2 * 2048 * 8 + 2 * 2048 * 4 + 2 * 2048 * 4


def test_rnemd_from_dirty_workspace():
    """A workspace with arbitrary prior contents: initialisation must leave the
    exchange's histograms and counters at zero, and the exchange then matches
    the oracle bit for bit."""
    wl = W.make_system((8, 16, 8), 5, [], [], np.zeros((0, 4)), np.random.default_rng(85))
    par = W.srd_params(85, kT_cell=1.0)
    o = oracle.OracleSystem(wl, par)
    g = gpu_system(wl, par, prec="f64")
    assert g.ws_bytes == g.ws.numel() and g.ws_bytes > RN_TAIL
    g.ws[g.ws_bytes - RN_TAIL:].fill_(0xFF)
    g.ws_init()
    tail = g.ws[g.ws_bytes - RN_TAIL:].cpu().numpy()
    hist = tail[:RN_HIST].view(np.int32)
    ctl = tail[RN_HIST + RN_BCNT:RN_HIST + RN_BCNT + 64].view(np.int32)
    assert not hist.any() and not ctl.any(), "exchange state not cleared by initialisation"
    g.set_rnemd(0.0, 8.0, 1.0, 0.5, 16)
    dp = 0.0
    for n in range(8):
        assert o.step(n) == 0
        dp, ns = o.rnemd(0.0, 8.0, 1.0, 0.5, 16, dp)
        g.step(1)
    assert_same(o, g.download()[0], ("x", "v"), "dirty workspace")
    assert float(g.rnemd_dp.cpu()[0]) == dp
    assert g.status() == 0


@pytest.mark.parametrize("exchange", [False, True])
def test_solvent_graph_matches_eager(exchange):
    wl = W.make_system((8, 16, 8), 5, [], [], np.zeros((0, 4)), np.random.default_rng(84))
    par = W.srd_params(84, kT_cell=1.0)
    say("solvent graph exchange=%s" % exchange)
    ge, gg = gpu_system(wl, par, prec="f64"), gpu_system(wl, par, prec="f64")
    for g in (ge, gg):
        if exchange:
            g.set_rnemd(0.0, 8.0, 1.0, 0.5, 20)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        gg.graph(6)
        for rep in range(3):
            gg.graph_launch()
            ge.step(6)
            a, b = ge.download()[0], gg.download()[0]
            assert np.array_equal(a["v"], b["v"]) and np.array_equal(a["x"], b["x"])
            assert float(ge.rnemd_dp.cpu()[0]) == float(gg.rnemd_dp.cpu()[0])
        gg.release_graph()
    assert ge.status() == 0 and gg.status() == 0


# ---------------------------------------------------------------------------
# Launch shapes change the split of work, never the results

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_every_launch_shape_gives_the_same_bits(prec):
    wl = W.suspension((14, 18, 11), 5, 4, 2.0, 60, 5.0, seed=88)
    par = W.srd_params(88, kT_cell=1.0, wca=W.wca_spheres(sigma=4.0))
    items = (1, 2, 4) if prec == "f64" else (2, 4, 8)
    shapes = [(0, 0, 0, 0)] + [(it, fill, dc, inl) for it in items
                               for fill, dc, inl in ((10, 3, 0), (55, 1, 1), (100, 16, 0), (100, 1, 1))]
    ref = None
    for sh in shapes:
        g = gpu_system(wl, par, prec=prec)
        g.set_tuning(*sh)
        say("shape %s %s -> tile %s" % (prec, sh, g.tile_shape()))
        g.body_forces()
        g.step(6)
        st = g.download()[0]
        assert g.status() == 0
        if ref is None:
            ref = st
            continue
        for k in ("x", "v", "xs", "vs", "R", "q", "P", "p", "F", "T"):
            assert np.array_equal(ref[k], st[k]), (sh, k)


def test_autotune_keeps_the_state_and_reuses_its_cache(tmp_path):
    from paper_2604_14307_amd import tune
    wl = W.suspension((16, 16, 16), 5, 4, 2.0, 60, 5.0, seed=89)
    par = W.srd_params(89, kT_cell=1.0, wca=W.wca_spheres(sigma=4.0))
    g = gpu_system(wl, par, prec="f32")
    g.body_forces()
    g.step(2)
    before = {k: v.cpu().clone() for k, v in g.snapshot().items()}
    cache = str(tmp_path / "tune.json")
    e = tune.autotune(g, steps=4, repeats=2, cache_path=cache)
    after = g.snapshot()
    for k in before:
        assert torch.equal(before[k], after[k].cpu()), k
    assert not e["cached"] and e["shapes_tried"] >= 6 and e["ms_per_step"] <= e["default_ms_per_step"]
    assert tuple(g.tile_shape()) == tuple(e["tile"])
    g2 = gpu_system(wl, par, prec="f32")
    e2 = tune.autotune(g2, steps=4, cache_path=cache)
    assert e2["cached"] and list(e2["tune"]) == list(e["tune"])
    assert g.status() == 0


def test_snapshot_waits_for_steps_on_another_stream():
    """Steps queued on a side stream must be complete in a snapshot taken from
    the default stream (the tuner snapshots after such warmup steps)."""
    wl = W.make_system((12, 12, 12), 5, [], [], np.zeros((0, 4)), np.random.default_rng(90))
    par = W.srd_params(90, kT_cell=1.0)
    g = gpu_system(wl, par, prec="f32")
    ref = gpu_system(wl, par, prec="f32")
    torch.cuda.synchronize()  # the set-up work ran on the default stream
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g.step(40)
    snap = g.snapshot()
    ref.step(40)
    torch.cuda.synchronize()
    # storage order within a cell follows atomic arrival: compare by identity
    a, b = torch.argsort(snap["tag"].long()), torch.argsort(ref.tag.long())
    assert torch.equal(snap["tag"][a], ref.tag[b])
    assert torch.equal(snap["v"][:, a], ref.v[:, b]) and torch.equal(snap["x"][:, a], ref.x[:, b])
