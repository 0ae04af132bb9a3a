"""Electro-chemical forces over their own ranges (DSS_FLAG_EC_RANGES; Fig. elch: repulsion
while the surface distance is below 20 lambda_D, attraction below 4 a0) against the FP64
oracle's reading R18, on an MI355X: pair sets bit-identical, forces / torques / stress /
history within 1e-10 (FP64) or 1e-5 (mixed), in lockstep.  On one box the lattice is that of
the lubrication list and the pairs beyond it take k_pairs_ec; the size-class stencils and
batches of boxes keep the whole pair set on their lattice."""
import sys

import numpy as np
import pytest

import oracle
from paper_2108_01013_amd import synth

pytestmark = pytest.mark.gpu

TOL_F = 1e-10
TOL_MIXED = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_inf(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def ec_box():
    w = synth.bidisperse_box(4000, 0.45, seed=11)
    p = dict(w.params, hamaker=1e-3, F_ER=1.0, ec_ranges=True)
    return synth.Workload("bidisperse N=4000 phi=0.45, attraction", w.x, w.rad, w.L, p)


@pytest.mark.parametrize("precision,tiled", [(0, True), (1, True), (0, False)])
def test_ec_ranges_lockstep(ec_box, precision, tiled):
    """tiled False: every row of the lubrication list on the per-particle path, whose partner
    sides add to the atomic record after the far pass stored into it."""
    from paper_2108_01013_amd.dss import Simulation
    w = ec_box
    p = w.params
    tol = TOL_F if precision == 0 else TOL_MIXED
    say(f"case: electro-chemical ranges N=4000 precision={precision} tiled={tiled}")
    sim = Simulation(p, record_pairs=True, precision=precision)
    sim.set_tuning(tiled=tiled)
    sim.set_particles(w.x, w.rad)
    dims = sim.cells()[0]
    # one box: the lattice of the lubrication list, the pairs beyond it on their own pass
    far = sim.box_info(0)["ec_far_rows"]
    assert far[0] > 0 and far[1] > 0
    assert np.array_equal(dims, oracle.cell_dims(dict(p, ec_ranges=False), w.rad.max()))
    # the pair set reaches 4 a0 beyond contact: far more pairs than the lubrication list
    n_lub = len(oracle.pairs_brute(dict(p, ec_ranges=False), w.x, w.rad, 0.0))
    assert sim.info()["n_pairs"] > 10 * n_lub
    sim.step(2)
    hp, hx = sim.history()
    for k in range(3):
        s = sim.state()
        a, aw = oracle.accelerations(p, w.rad, s["F"], s["T"])
        st = oracle.State(s["x"], s["u"], s["w"], a, aw, w.rad.copy(), 2 + k,
                          oracle.History(hp.astype(np.int32), hx))
        x_o = oracle.kick_drift(p, st)[0]
        sim.step(1)
        s1 = sim.state()
        uh, wh = sim.eval_velocities()
        assert np.array_equal(s1["x"], x_o)
        delta = oracle.le_offset(p, 3 + k)
        assert np.array_equal(sim.pairs(), oracle.pairs_brute(p, s1["x"], w.rad, delta)), f"step {k}: pairs"
        F, T, S, H, npairs = oracle.forces(p, s1["x"], uh, wh, w.rad, 3 + k, st.history)
        assert rel_inf(s1["F"], F) < tol, f"step {k}: F {rel_inf(s1['F'], F)}"
        assert rel_inf(s1["T"], T) < tol, f"step {k}: T {rel_inf(s1['T'], T)}"
        last, _, _ = sim.read_stress()
        assert rel_inf(last, S) < tol, f"step {k}: Sigma"
        hp, hx = sim.history()
        assert np.array_equal(hp, H.pairs)
    sim.close()


@pytest.fixture(scope="module")
def ec_poly_box():
    rad = synth.lognormal_radii(4000, hi=5.0, seed=13)
    L = synth.box_for_fraction(rad, 0.45)
    x = synth.relax_positions(rad, L, seed=14)
    p = synth.default_params([L, L, L], hamaker=1e-3, F_ER=1.0, ec_ranges=True)
    return synth.Workload("lognormal N=4000 on [1, 5], phi=0.45, attraction", x, rad, L, p)


@pytest.mark.parametrize("wave_class,precision", [(0, 0), (1, 0), (0, 1)])
def test_ec_ranges_size_class_stencils(ec_poly_box, wave_class, precision):
    """The electro-chemical ranges on the size-class stencils: a particle's class follows its
    reach 2 max(c, 1) a + 4 a0, which bounds every pair cutoff max(c (a_i + a_j), a_i + a_j +
    4 a0) of a partner no larger than itself.  Lognormal radii on [1, 5] (three classes, 5x the
    lubrication list); wave_class 0 (default split) and 1 (classes 1 and up on wavefronts).
    Pair sets bit-identical to the oracle's brute force, F, T, Sigma and history within 1e-10
    (FP64) or 1e-5 (mixed), three steps in lockstep."""
    from paper_2108_01013_amd.dss import Simulation
    w = ec_poly_box
    p = w.params
    say(f"case: electro-chemical ranges on size-class stencils N=4000 wave_class={wave_class} "
        f"precision={precision}")
    tol = TOL_F if precision == 0 else TOL_MIXED
    sim = Simulation(p, record_pairs=True, precision=precision)
    sim.set_tuning(sized=True, wave_class=wave_class)
    sim.set_particles(w.x, w.rad)
    assert sim.box_info(0)["size_classes"] >= 3
    n_lub = len(oracle.pairs_brute(dict(p, ec_ranges=False), w.x, w.rad, 0.0))
    assert sim.info()["n_pairs"] > 4 * n_lub
    assert np.array_equal(sim.pairs(), oracle.pairs_brute(p, w.x, w.rad, 0.0))
    sim.step(2)
    hp, hx = sim.history()
    for k in range(3):
        s = sim.state()
        a, aw = oracle.accelerations(p, w.rad, s["F"], s["T"])
        st = oracle.State(s["x"], s["u"], s["w"], a, aw, w.rad.copy(), 2 + k,
                          oracle.History(hp.astype(np.int32), hx))
        x_o = oracle.kick_drift(p, st)[0]
        sim.step(1)
        s1 = sim.state()
        uh, wh = sim.eval_velocities()
        assert np.array_equal(s1["x"], x_o)
        delta = oracle.le_offset(p, 3 + k)
        assert np.array_equal(sim.pairs(), oracle.pairs_brute(p, s1["x"], w.rad, delta)), f"step {k}: pairs"
        F, T, S, H, npairs = oracle.forces(p, s1["x"], uh, wh, w.rad, 3 + k, st.history)
        assert rel_inf(s1["F"], F) < tol, f"step {k}: F {rel_inf(s1['F'], F)}"
        assert rel_inf(s1["T"], T) < tol, f"step {k}: T {rel_inf(s1['T'], T)}"
        last, _, _ = sim.read_stress()
        assert rel_inf(last, S) < tol, f"step {k}: Sigma"
        hp, hx = sim.history()
        assert np.array_equal(hp, H.pairs)
        if len(hp):
            assert np.max(np.abs(hx - H.xi)) <= tol * np.max(np.abs(H.xi))
    sim.close()


@pytest.fixture(scope="module")
def ec_big_box():
    w = synth.bidisperse_box(20000, 0.5, seed=21)
    p = dict(w.params, hamaker=1e-3, F_ER=1.0, ec_ranges=True)
    return synth.Workload("bidisperse N=20000 phi=0.5, attraction", w.x, w.rad, w.L, p)


@pytest.mark.parametrize("precision", [0, 1])
def test_ec_far_pass_lockstep_20k(ec_big_box, precision):
    """N = 20000 (a lattice of 17+ rows each way, row tiles in use): pair sets bit-identical to
    the oracle's cell search, F, T, Sigma and history within 1e-10 (FP64) / 1e-5 (mixed) over
    two steps; every row on the tiles (the far pairs no longer overflow them); the pair count
    of the stress records equals the recorded set."""
    from paper_2108_01013_amd.dss import Simulation
    w = ec_big_box
    p = w.params
    tol = TOL_F if precision == 0 else TOL_MIXED
    say(f"case: electro-chemical far pass N=20000 precision={precision}")
    sim = Simulation(p, record_pairs=True, precision=precision)
    sim.set_particles(w.x, w.rad)
    bi = sim.box_info(0)
    assert bi["ec_far_rows"][0] > 0
    assert np.array_equal(sim.cells()[0], oracle.cell_dims(dict(p, ec_ranges=False), w.rad.max()))
    assert np.array_equal(sim.pairs(), oracle.pairs_cells(p, w.x, w.rad, 0.0))
    sim.set_timing(True, ["k_pairs", "k_pairs_ec"])
    sim.step(2)
    hp, hx = sim.history()
    for k in range(2):
        s = sim.state()
        a, aw = oracle.accelerations(p, w.rad, s["F"], s["T"])
        st = oracle.State(s["x"], s["u"], s["w"], a, aw, w.rad.copy(), 2 + k,
                          oracle.History(hp.astype(np.int32), hx))
        x_o = oracle.kick_drift(p, st)[0]
        sim.step(1)
        s1 = sim.state()
        uh, wh = sim.eval_velocities()
        assert np.array_equal(s1["x"], x_o)
        delta = oracle.le_offset(p, 3 + k)
        pairs = sim.pairs()
        assert np.array_equal(pairs, oracle.pairs_cells(p, s1["x"], w.rad, delta)), f"step {k}: pairs"
        assert sim.info()["n_pairs"] == len(pairs)
        F, T, S, H, npairs = oracle.forces(p, s1["x"], uh, wh, w.rad, 3 + k, st.history)
        assert rel_inf(s1["F"], F) < tol, f"step {k}: F {rel_inf(s1['F'], F)}"
        assert rel_inf(s1["T"], T) < tol, f"step {k}: T {rel_inf(s1['T'], T)}"
        last, _, _ = sim.read_stress()
        assert rel_inf(last, S) < tol, f"step {k}: Sigma"
        hp, hx = sim.history()
        assert np.array_equal(hp, H.pairs)
    t = sim.timing()
    assert t["k_pairs_ec"][1] > 0
    say(f"k_pairs {t['k_pairs']}, far pass {t['k_pairs_ec']}")
    sim.close()
