"""Batched flow-curve sweep (several boxes behind one handle) against the FP64 oracle run box
by box, on an MI355X.

Each box has its own volume fraction, size, shear rate and hence its own Lees-Edwards
offset; one counting sort and one pair launch cover all of them.  Per box and per step:
positions bit-identical, pair set bit-identical (and no pair across boxes), cell_start of the
box equal to the oracle's counting sort shifted by the box's first slot, forces / torques /
stress / history within the FP64 tolerances of the single-box tests (1e-10)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2108_01013_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_inf(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def box_history(hp, hx, lo, hi):
    m = (hp[:, 0] >= lo) & (hp[:, 0] < hi)
    assert np.all((hp[m, 1] >= lo) & (hp[m, 1] < hi)), "history pair across boxes"
    return (hp[m] - lo).astype(np.int32), hx[m]


def check_box(sim, b, ws, s1, uh, wh, pairs, cs, perm, hist, nstep, use_cells):
    w = ws[b]
    p = sim.params_list[b]
    sl = sim.box_slice(b)
    lo, hi = sl.start, sl.stop
    x = s1["x"][sl]
    delta = oracle.le_offset(p, nstep)
    m = (pairs[:, 0] >= lo) & (pairs[:, 0] < hi)
    assert np.all((pairs[m, 1] >= lo) & (pairs[m, 1] < hi)), "pair across boxes"
    pg = pairs[m] - lo
    po = oracle.pairs_cells(p, x, w.rad, delta) if use_cells else oracle.pairs_brute(p, x, w.rad, delta)
    assert np.array_equal(pg, po), f"box {b}: pair sets differ"
    bi = sim.box_info(b)
    dims = np.array(bi["cells"], np.int32)
    assert tuple(dims) == tuple(oracle.cell_dims(p, np.max(w.rad)))
    c0, nc = bi["first_cell"], int(np.prod(dims))
    cs_o, order_o = oracle.cell_sort(p, x, dims)
    assert np.array_equal(cs[c0:c0 + nc + 1] - lo, cs_o), f"box {b}: cell_start"
    F, T, S, H, npairs = oracle.forces(p, x, uh[sl], wh[sl], w.rad, nstep, hist, use_cells=use_cells)
    assert rel_inf(s1["F"][sl], F) < TOL, f"box {b}: F"
    assert rel_inf(s1["T"][sl], T) < TOL, f"box {b}: T"
    return S, H, npairs


def run_lockstep(ws, gds, steps, step0=0, use_cells=False, check=None, tiled=True):
    from paper_2108_01013_amd.dss import Batch
    params = [dict(w.params, shear_rate=g) for w, g in zip(ws, gds)]
    sim = Batch(params, record_pairs=True)
    sim.set_tuning(tiled=tiled)
    sim.set_particles([w.x for w in ws], [w.rad for w in ws])
    B = len(ws)
    if step0:
        sim.set_step(step0)
        sim.compute_forces()
    nstep = step0
    check = list(range(B)) if check is None else check
    hp, hx = sim.history()
    contacts = 0
    for k in range(steps):
        s0 = sim.state()
        hists, starts = {}, {}
        for b in check:
            sl = sim.box_slice(b)
            p = params[b]
            a, aw = oracle.accelerations(p, ws[b].rad, s0["F"][sl], s0["T"][sl])
            bp, bx = box_history(hp, hx, sl.start, sl.stop)
            st = oracle.State(s0["x"][sl], s0["u"][sl], s0["w"][sl], a, aw, ws[b].rad.copy(), nstep,
                              oracle.History(bp, bx))
            hists[b] = st
            starts[b] = oracle.kick_drift(p, st)
        sim.step(1)
        nstep += 1
        s1 = sim.state()
        uh, wh = sim.eval_velocities()
        pairs = sim.pairs()
        _, cs, perm = sim.cells()
        last, _, _ = sim.read_stress()
        hp, hx = sim.history()
        for b in check:
            sl = sim.box_slice(b)
            assert np.array_equal(s1["x"][sl], starts[b][0]), f"step {k} box {b}: positions"
            S, H, npairs = check_box(sim, b, ws, s1, uh, wh, pairs, cs, perm, hists[b].history, nstep, use_cells)
            assert rel_inf(last[b], S) < TOL, f"step {k} box {b}: Sigma"
            assert sim.box_info(b)["n_pairs"] == npairs
            bp, bx = box_history(hp, hx, sl.start, sl.stop)
            assert np.array_equal(bp, H.pairs), f"step {k} box {b}: history"
            if len(bp):
                assert np.max(np.abs(bx - H.xi)) <= 1e-10 * np.max(np.abs(H.xi))
            contacts += len(bp)
    return sim, contacts


def small_boxes():
    sizes = [700, 1000, 1300, 900, 1600]
    phis = [0.40, 0.45, 0.50, 0.55, 0.58]
    return [synth.bidisperse_box(n, f, seed=50 + b) for b, (n, f) in enumerate(zip(sizes, phis))]


@pytest.mark.parametrize("step0", [0, 123_457])
def test_batch_lockstep_small(step0):
    ws = small_boxes()
    gds = [0.01, 0.1, 1.0, 3.0, 10.0]
    say(f"case: batch lockstep 5 boxes step0={step0}")
    sim, contacts = run_lockstep(ws, gds, steps=6, step0=step0)
    assert contacts > 0
    # every box's Lees-Edwards offset follows its own shear rate and box
    for b in range(5):
        bi = sim.box_info(b)
        p = sim.params_list[b]
        assert bi["le_offset"] == oracle.le_offset(p, step0 + 6)
    sim.close()


def test_batch_lockstep_per_particle_rows():
    """Every cell row of every box on the per-particle path (tiling off): each row finds its
    box in the table."""
    ws = small_boxes()
    gds = [0.01, 0.1, 1.0, 3.0, 10.0]
    say("case: batch lockstep 5 boxes, every row on the per-particle path")
    sim, contacts = run_lockstep(ws, gds, steps=3, tiled=False)
    assert contacts > 0
    sim.close()


def test_batch_multi_workgroup_scan():
    """More than 65535 cells over all boxes: the cell-count scan runs over several workgroups."""
    ws = [synth.bidisperse_box(10_000, 0.30, seed=70 + b) for b in range(10)]
    gds = [10.0 ** (-2 + 3 * b / 9) for b in range(10)]
    say("case: batch multi-workgroup scan 10 x 10000")
    sim, _ = run_lockstep(ws, gds, steps=2, use_cells=True, check=[0, 4, 9])
    last = sim.box_info(9)
    assert last["first_cell"] + np.prod(last["cells"]) > 65535
    sim.close()


def test_batch_stress_sampling_per_box():
    """Per-box samples: box b's mean over a dss_step call equals the mean of its own stress
    read after each sampled step."""
    ws = small_boxes()[:3]
    from paper_2108_01013_amd.dss import Batch
    params = [dict(w.params, shear_rate=g) for w, g in zip(ws, [0.5, 1.0, 2.0])]
    say("case: batch stress sampling")
    sim = Batch(params)
    sim.set_particles([w.x for w in ws], [w.rad for w in ws])
    sim.step(20)
    state = sim.state()
    ref = []
    for k in range(4):
        sim.step(5, stress_every=5)
        last, mean, ns = sim.read_stress()
        assert ns == 1
        assert np.array_equal(mean, last)
        ref.append(last)
    sim.close()
    sim = Batch(params)
    sim.set_particles([w.x for w in ws], [w.rad for w in ws])
    sim.step(20)
    s2 = sim.state()
    # the two runs differ only by the summation order of the force atomics
    assert rel_inf(s2["x"], state["x"]) < 1e-12
    sim.step(20, stress_every=5)
    last, mean, ns = sim.read_stress()
    assert ns == 4
    assert rel_inf(mean, np.mean(ref, axis=0)) < 1e-7
    sim.close()


def test_batch_full_sweep_sampled():
    """The full 64-box sweep of the benchmark (sum N = 1.54M, phi 0.40-0.58, shear rates 1e-2 to
    1e1, several-workgroup scan) in its launch configuration: two lockstep steps, with six
    boxes spread over the volume fractions and shear rates checked against the oracle."""
    say("case: full 64-box sweep, sampled boxes")
    ws, gds = synth.config_sweep(B=64, workers=16, start_method="spawn")
    check = [0, 13, 26, 39, 52, 63]
    sim, contacts = run_lockstep(ws, gds, steps=2, use_cells=True, check=check)
    assert sim.N == sum(len(w.rad) for w in ws) > 1_000_000
    assert contacts > 0
    sim.close()


def test_batch_ec_ranges_lockstep():
    """Electro-chemical ranges with attraction on a batch of two boxes: batches keep the whole
    pair set on their lattice (no far-pair pass), so every cell row is taken on the per-particle
    path.  Three lockstep steps per box against the oracle: positions and pair sets
    bit-identical, F, T, Sigma and history within 1e-10."""
    ws = []
    for n, phi, seed in ((3000, 0.45, 61), (4000, 0.5, 62)):
        w = synth.bidisperse_box(n, phi, seed=seed)
        p = dict(w.params, hamaker=1e-3, F_ER=1.0, ec_ranges=True)
        ws.append(synth.Workload(f"bidisperse N={n} phi={phi}, attraction", w.x, w.rad, w.L, p))
    say("case: batch of 2 boxes with electro-chemical ranges")
    sim, contacts = run_lockstep(ws, [0.5, 2.0], steps=3, use_cells=True)
    for b in range(2):
        assert sim.box_info(b)["ec_far_rows"] == (0, 0)
    sim.close()
