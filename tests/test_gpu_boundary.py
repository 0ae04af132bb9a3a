"""Entry points of the C ABI beyond the time step, through the binding, against the FP64 oracle:
dss_build_neighbours (the counting sort of the current positions with the committed history
carried to the new slots) and the order independence of the read-back calls."""
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


def check_cells(sim, p, x):
    """Per-cell id sets and cell_start of the last counting sort against the oracle's sort of x
    on the GPU's lattice."""
    dims, cs, perm = sim.cells()
    cs_o, order_o = oracle.cell_sort(p, x, dims)
    assert np.array_equal(cs, cs_o)
    for c in range(len(cs) - 1):
        if cs[c + 1] > cs[c]:
            assert np.array_equal(np.sort(perm[cs[c]:cs[c + 1]]), order_o[cs_o[c]:cs_o[c + 1]]), c
    return dims


def test_history_then_pairs():
    """Reading the history must not disturb the listed pairs of the same evaluation."""
    from paper_2108_01013_amd.dss import Simulation
    w = synth.config_small()
    p = w.params
    say("case: history then pairs N=1000")
    sim = Simulation(p, record_pairs=True)
    sim.set_particles(w.x, w.rad)
    sim.step(40)
    hp, hx = sim.history()
    assert len(hp) > 0
    x = sim.state()["x"]
    po = oracle.pairs_brute(p, x, w.rad, oracle.le_offset(p, 40))
    assert np.array_equal(sim.pairs(), po)
    hp2, hx2 = sim.history()
    assert np.array_equal(hp, hp2) and np.array_equal(hx, hx2)
    assert sim.info()["n_pairs"] == len(po)
    sim.close()


@pytest.mark.parametrize("N,cell_scale", [(4000, 1.0), (4000, 1.3), (100_000, 1.1)])
def test_build_neighbours(N, cell_scale):
    """After a run, dss_build_neighbours sorts the current positions (on a new lattice when one is
    pending), keeps the committed history and evaluates the forces at the current state; the run
    continues in lockstep with the oracle."""
    from paper_2108_01013_amd.dss import Simulation
    w = synth.config_single_box() if N == 100_000 else synth.bidisperse_box(N, 0.55, seed=13)
    p = w.params
    say(f"case: build_neighbours N={N} cell_scale={cell_scale}")
    sim = Simulation(p, record_pairs=True)
    sim.set_particles(w.x, w.rad)
    nstep = 12
    sim.step(nstep)
    hp, hx = sim.history()
    dims0, _, _ = sim.cells()
    if cell_scale != 1.0:
        sim.set_tuning(cell_scale=cell_scale)
    sim.build_neighbours()
    s = sim.state()
    dims = check_cells(sim, p, s["x"])
    if cell_scale != 1.0:
        assert tuple(dims) != tuple(dims0)
    hp1, hx1 = sim.history()
    assert np.array_equal(hp1, hp) and np.array_equal(hx1, hx)
    po = oracle.pairs_cells(p, s["x"], w.rad, oracle.le_offset(p, nstep))
    assert np.array_equal(sim.pairs(), po)
    hist = oracle.History(hp.astype(np.int32), hx)
    F, T, S, H, npairs = oracle.forces(p, s["x"], s["u"], s["w"], w.rad, nstep, hist, use_cells=True)
    assert rel_inf(s["F"], F) < TOL and rel_inf(s["T"], T) < TOL
    last, _, _ = sim.read_stress()
    assert rel_inf(last, S) < TOL
    # two more steps in lockstep: the moved rows are found at their new slots
    for k in range(2):
        s0 = sim.state()
        a, aw = oracle.accelerations(p, w.rad, s0["F"], s0["T"])
        st = oracle.State(s0["x"], s0["u"], s0["w"], a, aw, w.rad.copy(), nstep, hist)
        x_o = oracle.kick_drift(p, st)[0]
        sim.step(1)
        nstep += 1
        s1 = sim.state()
        uh, wh = sim.eval_velocities()
        assert np.array_equal(s1["x"], x_o)
        F, T, S, H, npairs = oracle.forces(p, s1["x"], uh, wh, w.rad, nstep, hist, use_cells=True)
        assert rel_inf(s1["F"], F) < TOL and rel_inf(s1["T"], T) < TOL, k
        hp, hx = sim.history()
        assert np.array_equal(hp, H.pairs)
        assert rel_inf(hx, H.xi) < TOL
        hist = oracle.History(hp.astype(np.int32), hx)
    assert sim.info()["error_flags"] == 0
    sim.close()
