"""Size-class stencils (cells fitted to the smallest particles, the search stencil widened for
the larger ones, Section 2.2) against the FP64 oracle, on an MI355X.

Same bars as the row-tile path: pair sets and the class-major counting sort bit-identical,
forces / torques / stress / contact history within 1e-10 (FP64) or 1e-5 (mixed) of the
oracle, in lockstep (the oracle starts every checked step from the GPU's state)."""
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


def _sim(p, **kw):
    from paper_2108_01013_amd.dss import Simulation
    return Simulation(p, **kw)


@pytest.fixture(scope="module")
def poly_box():
    rad = synth.lognormal_radii(3000, seed=7)
    L = synth.box_for_fraction(rad, 0.55)
    x = synth.relax_positions(rad, L, seed=8)
    return synth.Workload("lognormal N=3000 phi=0.55", x, rad, L, synth.default_params([L, L, L]))


def class_major_cells(p, x, rad, dims):
    """Counting sort of the size-class stencils written out on the host: key = class n_cells
    + cell, class = floor(a cls_mul) with cls_mul = 2 c (1 + 1e-9) / min cell width."""
    L = np.asarray(p["L"], np.float64)
    dims = np.asarray(dims)
    cw = L / dims
    cls_mul = p["cutoff_factor"] * 2.0 * (1.0 + 1e-9) / np.min(cw)
    ncls = int(np.floor(np.max(rad) * cls_mul)) + 1
    cls = np.minimum(np.floor(rad * cls_mul).astype(np.int64), ncls - 1)
    c = np.minimum((x / cw).astype(np.int64), dims - 1)
    ncb = int(np.prod(dims))
    key = cls * ncb + (c[:, 2] * dims[1] + c[:, 1]) * dims[0] + c[:, 0]
    counts = np.bincount(key, minlength=ncls * ncb)
    cs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    return ncls, cs, key


def lockstep(sim, p, w, n0, nsteps, tol):
    """nsteps steps, each checked against one oracle step from the GPU state."""
    hp, hx = sim.history()
    contacts = 0
    for k in range(nsteps):
        s = sim.state()
        a, aw = oracle.accelerations(p, w.rad, s["F"], s["T"])
        st = oracle.State(s["x"], s["u"], s["w"], a, aw, w.rad.copy(), n0 + k,
                          oracle.History(hp.astype(np.int32), hx))
        x_o = oracle.kick_drift(p, st)[0]
        sim.step(1)
        s1 = sim.state()
        uh, wh = sim.eval_velocities()
        assert np.array_equal(s1["x"], x_o), f"step {k}: positions"
        delta = oracle.le_offset(p, n0 + k + 1)
        assert np.array_equal(sim.pairs(), oracle.pairs_brute(p, s1["x"], w.rad, delta)), f"step {k}: pairs"
        F, T, S, H, npairs = oracle.forces(p, s1["x"], uh, wh, w.rad, n0 + k + 1, st.history)
        assert rel_inf(s1["F"], F) < tol, f"step {k}: F {rel_inf(s1['F'], F)}"
        assert rel_inf(s1["T"], T) < tol, f"step {k}: T {rel_inf(s1['T'], T)}"
        last, _, _ = sim.read_stress()
        assert rel_inf(last, S) < tol, f"step {k}: Sigma"
        hp, hx = sim.history()
        assert np.array_equal(hp, H.pairs), f"step {k}: history pairs"
        if len(hp):
            assert np.max(np.abs(hx - H.xi)) <= max(tol, 1e-10) * np.max(np.abs(H.xi)) + 1e-300
        contacts = max(contacts, len(hp))
    return contacts


@pytest.mark.parametrize("wave_class", [0, 1, 64])
def test_sized_lockstep_fp64(poly_box, wave_class):
    """Lognormal radii on [1, 10]; wave_class 0 (default split), 1 (almost every particle on a
    wavefront) and 64 (every particle on one lane)."""
    w = poly_box
    p = w.params
    say(f"case: sized N=3000 wave_class={wave_class}")
    sim = _sim(p, record_pairs=True)
    sim.set_tuning(sized=True, wave_class=wave_class)
    sim.set_particles(w.x, w.rad)
    assert sim.info()["capacity"] == oracle.history_capacity(w.rad.max(), w.rad.min())
    dims, cs, perm = sim.cells()
    ncls, cs_o, key = class_major_cells(p, w.x, w.rad, dims)
    assert ncls >= 5
    assert np.array_equal(cs, cs_o)
    for c in np.flatnonzero(np.diff(cs_o)):
        assert np.array_equal(np.sort(perm[cs[c]:cs[c + 1]]), np.flatnonzero(key == c))
    sim.step(3)
    contacts = lockstep(sim, p, w, 3, 3, TOL_F)
    assert contacts > 0
    sim.close()


def test_sized_mixed(poly_box):
    w = poly_box
    p = w.params
    say("case: sized N=3000 mixed")
    sim = _sim(p, record_pairs=True, precision=1)
    sim.set_tuning(sized=True)
    sim.set_particles(w.x, w.rad)
    sim.step(3)
    lockstep(sim, p, w, 3, 2, TOL_MIXED)
    sim.close()


def test_sized_le_offsets(poly_box):
    """Stencil rows across the sheared y faces at offsets spanning the cell alignments."""
    w = poly_box
    p = dict(w.params)
    say("case: sized LE offsets N=3000")
    sim = _sim(p, record_pairs=True)
    sim.set_tuning(sized=True)
    sim.set_particles(w.x, w.rad)
    dims = sim.cells()[0]
    dcell = p["L"][0] / dims[0]
    for frac in (0.0, 0.5, 0.999, 1.0, 2.5, 7.3, dims[0] - 0.5):
        n = int(round(frac * dcell / (p["shear_rate"] * p["L"][1] * p["dt"])))
        sim.set_step(n)
        sim.compute_forces()
        delta = oracle.le_offset(p, n)
        assert np.array_equal(sim.pairs(), oracle.pairs_brute(p, w.x, w.rad, delta)), f"delta={delta}"
        s = sim.state()
        F, T, S, H, npairs = oracle.forces(p, w.x, oracle.ambient_velocity(p, w.x),
                                           oracle.ambient_rotation(p, len(w.rad)), w.rad, n)
        assert rel_inf(s["F"], F) < TOL_F and rel_inf(s["T"], T) < TOL_F
    sim.close()


def test_sized_bidisperse_ties():
    """1 : 1.4 bidisperse (equal radii in one class: ownership by slot order), 5 lockstep steps."""
    w = synth.config_small()
    p = w.params
    say("case: sized bidisperse N=1000")
    sim = _sim(p, record_pairs=True)
    sim.set_tuning(sized=True)
    sim.set_particles(w.x, w.rad)
    lockstep(sim, p, w, 0, 5, TOL_F)
    sim.close()


@pytest.mark.parametrize("queue_cap", [1, 7, 64])
def test_sized_queue_stop_and_resume(poly_box, queue_cap):
    """Pair queues of queue_cap entries, so every stencil scan stops on a full queue and resumes
    after the queue is evaluated, many times per evaluation (at the full queue length this box
    never fills them): lane and wavefront paths, lockstep against the oracle as above."""
    w = poly_box
    p = w.params
    say(f"case: sized N=3000 queue_cap={queue_cap}")
    sim = _sim(p, record_pairs=True)
    sim.set_tuning(sized=True, wave_class=2, queue_cap=queue_cap)
    assert sim.tuning()["queue_cap"] == queue_cap
    sim.set_particles(w.x, w.rad)
    sim.step(2)
    contacts = lockstep(sim, p, w, 2, 2, TOL_F)
    assert contacts > 0
    sim.close()


def test_sized_needs_one_box():
    from paper_2108_01013_amd.dss import Batch, DssError
    w = synth.config_small()
    b = Batch([w.params, w.params])
    with pytest.raises(DssError):
        b.set_tuning(sized=True)
    b.close()


def test_full_size_high_ratio_initial_evaluation():
    """Size ratio 10 at its full size (N = 500k, lognormal radii on [1, 10], phi = 0.55) on the
    size-class stencils in the benchmark's configuration (spacing 1.5, wavefronts from stencil
    radius 3), FP64: the pair set bit-identical to the oracle's cell search and every force,
    torque and the stress within 1e-10.  The centres are uniform at random without relaxation
    (a relaxed packing of this size takes many minutes to generate; one evaluation does not
    need it), so the set holds deep overlaps as well as near misses."""
    from paper_2108_01013_amd.dss import Simulation
    N = 500_000
    rad = synth.lognormal_radii(N, seed=3)
    L = synth.box_for_fraction(rad, 0.55)
    x = np.random.default_rng(1003).uniform(0.0, L, size=(N, 3))
    p = synth.default_params([L, L, L])
    say("case: full-size size ratio 10, N=500k, initial evaluation")
    sim = Simulation(p, record_pairs=True)
    sim.set_tuning(sized=True, cell_scale=1.5, wave_class=2)
    sim.set_particles(x, rad)
    assert sim.box_info(0)["size_classes"] >= 6
    pg = sim.pairs()
    po = oracle.pairs_cells(p, x, rad, 0.0)
    assert len(po) > N and np.array_equal(pg, po)
    s = sim.state()
    F, T, S, H, npairs = oracle.forces(p, x, s["u"], s["w"], rad, 0, use_cells=True)
    assert rel_inf(s["F"], F) < TOL_F and rel_inf(s["T"], T) < TOL_F
    last, _, _ = sim.read_stress()
    assert rel_inf(last, S) < TOL_F
    sim.close()


def test_full_size_high_ratio_mixed_lockstep():
    """Size ratio 10 at its full size in its benchmark's configuration: mixed precision on the
    size-class stencils (spacing 1.5, wavefronts from stencil radius 3), N = 500k lognormal radii
    on [1, 10] at phi = 0.55.  Two time steps in lockstep with the FP64 oracle: pair sets
    bit-identical, F, T, Sigma and the committed stretches within 1e-5, the second step reading
    the history rows that the first committed (the rows of the large particles, sorted by partner
    id, hold tens of entries).  The centres are uniform at random, as in the initial-evaluation
    test (relaxing this size takes many minutes), so most particles start in contact."""
    from paper_2108_01013_amd.dss import DSS_MIXED, Simulation
    N = 500_000
    rad = synth.lognormal_radii(N, seed=3)
    L = synth.box_for_fraction(rad, 0.55)
    x = np.random.default_rng(1003).uniform(0.0, L, size=(N, 3))
    p = synth.default_params([L, L, L])
    say("case: full-size size ratio 10, N=500k, mixed, two lockstep steps")
    sim = Simulation(p, record_pairs=True, precision=DSS_MIXED)
    sim.set_tuning(sized=True, cell_scale=1.5, wave_class=2)
    sim.set_particles(x, rad)
    hp = np.zeros((0, 2), np.int32)
    hx = np.zeros((0, 3))
    for k in range(2):
        s0 = sim.state()
        a, aw = oracle.accelerations(p, rad, s0["F"], s0["T"])
        st = oracle.State(s0["x"], s0["u"], s0["w"], a, aw, rad.copy(), k, oracle.History(hp.astype(np.int32), hx))
        x_o = oracle.kick_drift(p, st)[0]
        sim.step(1)
        s1 = sim.state()
        uh, wh = sim.eval_velocities()
        assert np.array_equal(s1["x"], x_o), f"step {k}: positions"
        assert np.array_equal(sim.pairs(), oracle.pairs_cells(p, s1["x"], rad, oracle.le_offset(p, k + 1))), k
        F, T, S, H, npairs = oracle.forces(p, s1["x"], uh, wh, rad, k + 1, st.history, use_cells=True)
        say(f"step {k}: F {rel_inf(s1['F'], F):.2e} T {rel_inf(s1['T'], T):.2e}")
        assert rel_inf(s1["F"], F) < TOL_MIXED and rel_inf(s1["T"], T) < TOL_MIXED
        last, _, _ = sim.read_stress()
        assert rel_inf(last, S) < TOL_MIXED
        hp, hx = sim.history()
        assert len(hp) > N and np.array_equal(hp, H.pairs)
        assert np.max(np.abs(hx - H.xi)) <= TOL_MIXED * np.max(np.abs(H.xi))
    info = sim.info()
    say(f"contacts {info['n_contacts']}, largest history row {info['max_row_fill']} of {info['capacity']}")
    assert info["error_flags"] == 0 and info["max_row_fill"] > 32
    sim.close()
