"""GPU parity of the binned solvent layout.

The binned layout stores the solvent in per-brick regions of each step's grid
and collides a brick per block; it performs the same per-cell sums (exact
int64 fixed point in FP32), draws and roundings as the dense layout, so every
result, in identity order, must equal the dense FP32 path's bit for bit.  The
dense FP32 path, in the graph form the bench times, is itself held to the FP64
oracle (1e-5 relative L2 and max-abs per step, test_gpu_bench_form.py), so the
binned form meets the same bounds.  Covered here: pack/unpack round trips, eager steps and
graph replays, bodies with centre WCA, site-site WCA, forced flow, pure
solvent, batched replicas, a brick whose region overflows into the shared
overflow list, a brick with more members than a block holds in registers, and a
brick with more sites than its site list holds, in both block shapes.
"""
import sys

import numpy as np
import pytest

from paper_2604_14307_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

STATE_KEYS = ("x", "v", "R", "img", "q", "P", "p", "F", "T", "xs", "vs")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_system(*a, **k):
    from paper_2604_14307_amd.sim import GPUSystem
    return GPUSystem(*a, **k)


def assert_same_states(a, b, where=""):
    for r, (sa, sb) in enumerate(zip(a, b)):
        for k in STATE_KEYS:
            if not np.array_equal(sa[k], sb[k]):
                i = tuple(np.argwhere(sa[k] != sb[k])[0])
                raise AssertionError("%s system %d: %s differs at %s: %r vs %r" % (where, r, k, i, sa[k][i], sb[k][i]))


def dense_and_binned(systems, par, nsteps, graph=False, check_every=1):
    gd = gpu_system(systems, par, prec="f32")
    gb = gpu_system(systems, par, prec="f32", layout="binned")
    for g in (gd, gb):
        g.body_forces()
    assert_same_states(gd.download(), gb.download(), "initial")
    if graph:
        torch.cuda.synchronize()  # the set-up work ran on the default stream
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            gb.graph(2)
            for n in range(nsteps // 2):
                gb.graph_launch()
                torch.cuda.synchronize()
                gd.step(2)
                torch.cuda.synchronize()
                assert_same_states(gd.download(), gb.download(), "graph replay %d" % n)
            gb.release_graph()
    else:
        for n in range(nsteps):
            gd.step(1)
            gb.step(1)
            if (n + 1) % check_every == 0 or n == nsteps - 1:
                assert gb.status() == 0, "step %d" % n
                assert_same_states(gd.download(), gb.download(), "step %d" % n)
    assert gd.status() == 0 and gb.status() == 0
    return gd, gb


def test_pack_unpack_round_trip():
    wl, par, _ = W.config(0)
    g = gpu_system(wl, par, prec="f32", layout="binned")
    xd, vd, td = g.dense_solvent()
    assert np.array_equal(td.cpu().numpy(), np.arange(g.N))
    assert np.array_equal(xd.cpu().numpy(), np.asarray(wl["x"], dtype=np.float32))
    assert np.array_equal(vd.cpu().numpy(), np.asarray(wl["v"], dtype=np.float32))
    g.set_step(7)  # repacks on the grid of step 7
    xd2, vd2, _ = g.dense_solvent()
    assert torch.equal(xd, xd2) and torch.equal(vd, vd2)
    assert g.status() == 0


@pytest.mark.parametrize("kT_cell", [1.0, 0.0])
def test_single_sphere_binned_equals_dense(kT_cell):
    wl, par, _ = W.config(0, kT_cell=kT_cell)
    dense_and_binned(wl, par, 30, check_every=5)


def test_single_sphere_binned_graph_equals_dense():
    wl, par, _ = W.config(0)
    _, gb = dense_and_binned(wl, par, 8, graph=True)
    assert gb.status() == 0


def test_batched_replicas_binned_equals_dense():
    systems, par, _ = W.batched_replicas(nrep=6, seed=9, lo=6, hi=13)
    dense_and_binned(systems, par, 12, check_every=4)
    dense_and_binned(systems, par, 6, graph=True)


def test_pure_solvent_and_forced_flow_binned():
    wl = W.make_system((12, 9, 7), 4, [], np.zeros((0, 3)), np.zeros((0, 4)), np.random.default_rng(3))
    par = W.srd_params(5, kT_cell=1.0)
    dense_and_binned(wl, par, 10, check_every=5)
    wl, par, _ = W.config(0)
    dense_and_binned(wl, W.sedimentation(par, [wl], force=(0.5, -0.2, 0.1)), 10, check_every=5)


def test_site_site_wca_binned():
    wl = W.shapes((16, 16, 16), 3, 1, 1, 1, seed=31)
    par = W.srd_params(31, kT_cell=1.0, wca=W.wca_sites())
    dense_and_binned(wl, par, 8, check_every=4)


def test_crowded_brick_overflow_and_two_pass_path():
    """Extra solvent crowded into one cell beside the sphere: that brick's
    region overflows into the shared overflow list, and with the sphere's
    sites the brick then has more members than a block holds in registers
    (the two-pass path).  The crowd disperses over the steps."""
    base, par, _ = W.config(0)
    rng = np.random.default_rng(5)
    # the crowded brick (8 x 8 x 4 cells) then holds about 1280 + 900 solvent
    # against a region capacity of 1759 (density 5.9 per cell): about 420
    # overflow entries, and more than the 2048 members a block holds
    extra = 900
    xe = np.array([[5.5], [5.5], [6.5]]) + 0.4 * (rng.random((3, extra)) - 0.5)
    ve = rng.normal(0.0, 1.0, (3, extra))
    wl = dict(base)
    wl["x"] = np.concatenate([base["x"], xe], axis=1)
    wl["v"] = np.concatenate([base["v"], ve], axis=1)
    gd, gb = dense_and_binned(wl, par, 6)
    assert gb.status() == 0


@pytest.mark.parametrize("a,ncell,density", [(0.5, (10, 10, 10), 5), (1.5, (10, 10, 10), 5),
                                             (0.5, (128, 128, 64), 1)])
def test_non_unit_cell_edge(a, ncell, density):
    """A cell edge other than 1 (the brick collision's general cell form, by
    the exact reciprocal for 0.5 and by division for 1.5), in the eight-wave
    block and, in a box of 4096 bricks, the four-wave block: the binned step
    against the dense FP32 form."""
    rng = np.random.default_rng(78)
    tpl = W.sphere_template(2.0 * a, 100, 5.0)
    centre = 0.5 * a * np.asarray(ncell, dtype=np.float64)[None, :]
    wl = W.make_system(ncell, density, [tpl], centre, W.random_quaternions(rng, 1), rng, a=a)
    par = W.srd_params(78, kT_cell=1.0)
    gd, gb = dense_and_binned(wl, par, 4, check_every=2)
    assert gb.binned.items == (7 if ncell[0] == 128 else 4)


def test_bodies_of_more_sites_than_a_block():
    """Two spheres of 600 sites (three chunks of the thermalization's block,
    more sites than a brick's list holds): the binned step against the dense
    FP32 form."""
    wl = W.suspension((12, 12, 12), 5, 2, 2.0, 600, 5.0, seed=36)
    par = W.srd_params(36, kT_cell=1.0, wca=W.wca_spheres(sigma=4.0))
    dense_and_binned(wl, par, 6, check_every=3)


def test_site_list_overflow():
    """Six spheres of 100 sites packed into one brick of 8 x 8 x 4 cells: the
    brick's site list (its 256 cells + 64 slots) overflows into the shared
    site list, which the brick then scans.  No WCA, so the spheres may
    overlap; the thermostat is on."""
    rng = np.random.default_rng(41)
    tpl = W.sphere_template(1.5, 100, 5.0)
    centres = np.array([[2.0 + 1.3 * (b % 3), 2.5 + 2.5 * (b // 3), 2.0] for b in range(6)])
    wl = W.make_system((16, 16, 16), 5, [tpl] * 6, centres, W.random_quaternions(rng, 6), rng)
    par = W.srd_params(41, kT_cell=1.0)
    dense_and_binned(wl, par, 8, check_every=2)


def test_four_wave_blocks_crowded_brick_with_site_overflow():
    """A box of 4096 bricks, which takes the four-wave brick block (seven
    members per lane; the smaller systems above take the eight-wave block).
    In its first brick six overlapping spheres of 100 sites overflow the
    brick's site list, and 600 extra solvent crowded among them overflow its
    region into the shared overflow list, so the brick has more members than
    a block holds in registers (the two-pass path)."""
    rng = np.random.default_rng(43)
    tpl = W.sphere_template(1.5, 100, 5.0)
    centres = np.array([[2.0 + 1.3 * (b % 3), 2.5 + 2.5 * (b // 3), 2.0] for b in range(6)])
    wl = W.make_system((128, 128, 64), 5, [tpl] * 6, centres, W.random_quaternions(rng, 6), rng)
    extra = 600
    xe = np.array([[3.5], [4.0], [2.0]]) + 0.4 * (rng.random((3, extra)) - 0.5)
    ve = rng.normal(0.0, 1.0, (3, extra))
    wl["x"] = np.concatenate([wl["x"], xe], axis=1)
    wl["v"] = np.concatenate([wl["v"], ve], axis=1)
    par = W.srd_params(43, kT_cell=1.0)
    say("binned four-wave blocks, crowded brick")
    gd, gb = dense_and_binned(wl, par, 4, check_every=2)
    assert gb.binned.nbricks >= 4096 and gb.binned.items == 7


@pytest.mark.parametrize("ncell,density", [((16, 16, 16), 1), ((128, 128, 64), 1.5)])
def test_low_density_binned(ncell, density):
    """Few solvent per cell (the eight-wave block at 16^3, the four-wave block
    on 4096 bricks): a brick's own sub-region then holds fewer members than
    its lanes load before the header, and those lanes load again."""
    rng = np.random.default_rng(47)
    tpl = W.sphere_template(2.0, 100, 5.0)
    wl = W.make_system(ncell, density, [tpl], np.array([[5.0, 5.0, 5.0]]), W.random_quaternions(rng, 1), rng)
    par = W.srd_params(47, kT_cell=1.0)
    say("binned low density %r" % (ncell,))
    dense_and_binned(wl, par, 4, check_every=2)


def test_full_size_suspension_binned_equals_dense():
    wl, par, _ = W.config(1)
    say("binned 60^3")
    dense_and_binned(wl, par, 4, check_every=2)


def test_full_size_batched_binned_graph_equals_dense():
    systems, par, _ = W.config(3)
    say("binned batched 512")
    dense_and_binned(systems, par, 4, graph=True)


def collided(g):
    """The solvent the last standalone collision wrote (the other set of
    arrays, on the next step's grid), dense in identity order."""
    g._swap()
    g.d_step.add_(1)
    xd, vd, _ = g.dense_solvent()
    out = (xd.cpu().numpy(), vd.cpu().numpy())
    g.d_step.sub_(1)
    g._swap()
    return out


def test_binned_collide_is_repeatable():
    """The standalone collision (as the bench times it) leaves its inputs
    unchanged: launched twice on the same step it writes the same solvent, and
    that solvent is the step's own."""
    wl, par, _ = W.config(0)
    g = gpu_system(wl, par, prec="f32", layout="binned")
    g.body_forces()
    g.step(3)
    ref = gpu_system(wl, par, prec="f32", layout="binned")
    ref.body_forces()
    ref.step(4)
    g.binned_sites()
    vs0 = g.vs.clone()
    g.binned_collide()
    torch.cuda.synchronize()
    first = collided(g)
    g.vs.copy_(vs0)
    g.binned_collide()
    torch.cuda.synchronize()
    second = collided(g)
    for a, b in zip(first, second):
        assert np.array_equal(a, b)
    r = ref.download()[0]
    assert np.array_equal(first[0], r["x"].astype(np.float32))
    assert np.array_equal(first[1], r["v"].astype(np.float32))
    assert g.status() == 0
