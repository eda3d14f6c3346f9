"""GPU parity of the step in the form the bench times it, against the oracle.

The bench replays captured HIP graphs of out-of-place steps with the committed
tuned launch shape and graph schedule of each workload (the fused force and
binning kernel, or the binning inside the collision).  Here that same form is
compared with the CPU oracle:

* FP32, one step at a time.  From the GPU's FP32 state, upcast (exactly) into
  the oracle, one oracle step is compared with the GPU's step.  Both steps of
  a two-step graph are covered: its first step equals one eager out-of-place
  step of the same kernels, its second step runs on the cell lists that the
  first step's fused binning produced, and the graph's result must equal two
  eager steps bit for bit.  Velocities must stay within 1e-5 relative L2
  error (solvent and sites together, Sec. II.A), and within stated max-abs
  bounds per observable; particles in cells whose membership differs because
  FP32 rounding of x - s moved a member across a cell boundary are excluded
  and counted, and so are bodies with a site in such a cell.
* FP64, the 512 batched replicas: bit for bit against each replica's oracle
  after four steps of graph replays.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2604_14307_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CACHE = os.path.join(ROOT, "paper_2604_14307_amd", "tuning_gfx950.json")
STATE_KEYS = ("x", "v", "R", "img", "q", "P", "p", "F", "T", "xs", "vs")
BODY_KEYS = ("x", "v", "R", "img", "q", "P", "p", "F", "T")

# max-abs error bounds of one FP32 step against the FP64 oracle (good cells):
# velocities in units of sqrt(kT/m) of the particle, positions in cell edges
# (a float position of at most 64 carries 2^-18 = 3.8e-6 of rounding)
MAXABS = {"v_solvent": 1e-5, "v_site": 1e-5, "x_solvent": 1e-5}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def tuned_system(systems, par, prec):
    from paper_2604_14307_amd import tune
    from paper_2604_14307_amd.sim import GPUSystem
    g = GPUSystem(systems, par, prec=prec)
    g.body_forces()
    e = tune.autotune(g, cache_path=CACHE, write=False)
    assert e["cached"], "the bench workloads have committed launch shapes"
    return g, e


def gpu_cells(g, tag_in):
    """Cell (canonical global index) of every particle in the last binning, by
    identity: solvent by the tag it carried into the step, then sites N + j."""
    cc, members, _ = g.bins()
    cnt = np.diff(cc)
    owner = np.repeat(np.arange(len(cnt), dtype=np.int64), cnt)
    ident = members.copy()
    sol = members < g.N
    ident[sol] = tag_in[members[sol]]
    cell = np.full(g.N + g.S, -1, dtype=np.int64)
    cell[ident] = owner
    assert np.all(cell >= 0)
    return cell


def oracle_step(wl, state, par, r, step):
    """One oracle step, stage by stage, from a GPU state upcast to FP64;
    returns the oracle and the cell of each particle (solvent, then sites)."""
    wl2 = dict(wl)
    for k in BODY_KEYS:
        wl2[k] = state[k]
    o = oracle.OracleSystem(wl2, par, replica=r)
    assert o.sites_thermalize(step) == 0
    cell, cs, mem, fl = o.bin(o.shift(step))
    assert fl == 0
    assert o.collide(step, cs, mem) == 0
    J, K = o.sites_to_body()
    assert o.stream() == 0
    assert o.body_integrate(J, K) == 0
    return o, cell.astype(np.int64)


def lhat(q, p):
    """Body-frame angular momentum Lhat_k = p . P_k q / 2 (Miller et al.)."""
    P1 = np.stack([-q[1], q[0], q[3], -q[2]])
    P2 = np.stack([-q[2], -q[3], q[0], q[1]])
    P3 = np.stack([-q[3], q[2], -q[1], q[0]])
    return 0.5 * np.stack([(p * P1).sum(0), (p * P2).sum(0), (p * P3).sum(0)])


class ErrorTally:
    """Accumulates the error of one FP32 step over systems."""

    def __init__(self, par):
        self.num = self.den = 0.0
        self.excluded = self.total = 0
        self.maxabs = dict.fromkeys(MAXABS, 0.0)
        self.body_rel = self.body_L = 0.0
        self.bodies_excluded = self.bodies_total = 0
        self.kT = par["kT"]

    def add(self, o, cell64, s1, cell32, m_solvent):
        flip = cell32 != cell64
        bad_cells = np.unique(np.concatenate([cell64[flip], cell32[flip]]))
        bad = np.isin(cell64, bad_cells) | np.isin(cell32, bad_cells)
        good = ~bad
        v64 = np.concatenate([o.v, o.vs], axis=1)
        v32 = np.concatenate([s1["v"], s1["vs"]], axis=1)
        d = (v32 - v64)[:, good]
        self.num += float((d * d).sum())
        self.den += float((v64[:, good] ** 2).sum())
        self.excluded += int(bad.sum())
        self.total += len(bad)
        N = o.N
        gs, gt = good[:N], good[N:]
        if gs.any():
            self.maxabs["v_solvent"] = max(self.maxabs["v_solvent"], float(
                np.abs(s1["v"] - o.v)[:, gs].max() / math.sqrt(self.kT / m_solvent)))
            # positions: minimum image (a wrap can put the two sides a box apart)
            L = np.array(o.ncell, dtype=np.float64)[:, None] * o.a
            dx = s1["x"] - o.x
            dx -= L * np.rint(dx / L)
            self.maxabs["x_solvent"] = max(self.maxabs["x_solvent"], float(np.abs(dx)[:, gs].max() / o.a))
        if gt.any():
            sig = np.sqrt(self.kT / o.sm)[None, :]
            self.maxabs["v_site"] = max(self.maxabs["v_site"], float((np.abs(s1["vs"] - o.vs) / sig)[:, gt].max()))
        if o.B:
            # bodies whose sites all collided in good cells (a flipped cell
            # changes a site's impulse at order one)
            ok = np.array([gt[o.site_off[b]:o.site_off[b + 1]].all() for b in range(o.B)])
            self.bodies_excluded += int((~ok).sum())
            self.bodies_total += o.B
            if ok.any():
                scale = np.sqrt(self.kT * o.M)[None, :]
                self.body_rel = max(self.body_rel, float((np.abs(s1["P"] - o.P) / scale)[:, ok].max()))
                Lg = lhat(s1["q"], s1["p"])
                sL = np.sqrt(self.kT * np.where(o.I > 0.0, o.I, 1.0))
                self.body_L = max(self.body_L, float((np.abs(Lg - o.body_angmom_bodyframe()) / sL)[:, ok].max()))

    def report(self, label):
        rel = math.sqrt(self.num / self.den)
        say("%s: rel L2 %.3e, excluded %d of %d, max-abs %s; bodies (%d of %d excluded): P %.2e sqrt(kT M), "
            "Lhat %.2e sqrt(kT I)" % (label, rel, self.excluded, self.total,
                                      ", ".join("%s %.2e" % kv for kv in sorted(self.maxabs.items())),
                                      self.bodies_excluded, self.bodies_total, self.body_rel, self.body_L))
        return rel


def split(g, states, cells):
    """Per-system views of the state and the cells (local cell indices)."""
    out = []
    for r, s in enumerate(states):
        n0, n1 = g.solv_off_h[r], g.solv_off_h[r + 1]
        s0, s1 = g.N + g.site_sys_off_h[r], g.N + g.site_sys_off_h[r + 1]
        c = np.concatenate([cells[n0:n1], cells[s0:s1]]) - g.cell_off_h[r]
        out.append((s, c))
    return out


@pytest.mark.parametrize("ci", [1, 3])
def test_fp32_bench_form_within_1e5_of_fp64_oracle(ci):
    wls, par, meta = W.config(ci)
    systems = wls if isinstance(wls, list) else [wls]
    g, e = tuned_system(systems, par, "f32")
    say("FP32 bench form, workload %d (%s), tuned shape %s" % (ci, meta["name"], list(e["tune"])))
    torch.cuda.synchronize()  # the set-up work ran on the default stream
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g.graph(2)
        g.graph_launch()  # two steps in the bench's form before the compared ones
        torch.cuda.synchronize()
        snap = g.snapshot()
        step0 = int(g.d_step.item())
        s0 = g.download()
        tag0 = g.tag.cpu().numpy().astype(np.int64)
        g.step(1)  # the graph's first step: one out-of-place step of the same kernels
        torch.cuda.synchronize()
        s1 = g.download()
        cells1 = gpu_cells(g, tag0)
        tag1 = g.tag.cpu().numpy().astype(np.int64)
        g.step(1)
        torch.cuda.synchronize()
        s2e = g.download()
        cells2 = gpu_cells(g, tag1)
        g.restore(snap)
        g.graph_launch()  # both steps as the bench replays them
        torch.cuda.synchronize()
        s2g = g.download()
        g.release_graph()
    assert g.status() == 0
    for r in range(len(systems)):
        for k in STATE_KEYS:
            assert np.array_equal(s2g[r][k], s2e[r][k]), (r, k)
    for label, (sin, sout, cells, step) in (("first step", (s0, s1, cells1, step0)),
                                           ("second step", (s1, s2g, cells2, step0 + 1))):
        tally = ErrorTally(par)
        for r, (so, c32) in enumerate(split(g, sout, cells)):
            o, c64 = oracle_step(systems[r], sin[r], par, r, step)
            tally.add(o, c64, so, c32, float(systems[r]["m"]))
        rel = tally.report("workload %d, %s" % (ci, label))
        assert rel <= 1e-5
        assert tally.excluded <= 1e-3 * tally.total
        for k, bound in MAXABS.items():
            assert tally.maxabs[k] <= bound, (label, k, tally.maxabs[k])
        assert tally.bodies_excluded <= 0.05 * tally.bodies_total
        assert tally.body_rel <= 1e-5, (label, tally.body_rel)
        assert tally.body_L <= 1e-5, (label, tally.body_L)


def test_fp64_batched_bench_form_bit_exact():
    """The 512 batched replicas (17.4M solvent) in FP64, as the bench runs
    them (tuned shape and schedule, graph replays on a side stream): every
    replica bit for bit against its oracle after four steps."""
    systems, par, meta = W.config(3)
    g, e = tuned_system(systems, par, "f64")
    say("FP64 batched bench form, tuned shape %s" % list(e["tune"]))
    torch.cuda.synchronize()  # the set-up work ran on the default stream
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g.graph(2)
        g.graph_launch()
        g.graph_launch()
        torch.cuda.synchronize()
        g.release_graph()
    assert g.status() == 0
    gd = g.download()
    for r, wl in enumerate(systems):
        o = oracle.OracleSystem(wl, par, replica=r)
        assert o.body_forces() == 0
        for n in range(4):
            assert o.step(n) == 0
        for k in STATE_KEYS:
            a, b = getattr(o, k), gd[r][k]
            if not np.array_equal(a, b):
                i = tuple(np.argwhere(a != b)[0])
                raise AssertionError("replica %d: %s differs at %s: oracle %r gpu %r" % (r, k, i, a[i], b[i]))
