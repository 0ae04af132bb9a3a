"""Long contact-history rows (Sec. 2.1, memory paragraph: each particle's row of stored
stretches, sorted by partner id and searched over) against the FP64 oracle, on an MI355X.

Workload: N = 3000 lognormal radii on [1, 10] with the four largest set to 10 (N = 20 000 with
eight for the row tiles, which need four cells of the largest cutoff along x), relaxed at
phi = 0.55, then every radius inflated by 2 % (a compressed box): the largest particles touch
more than 40 others, so rows are filled beyond the eight entries that are read at once and
sorted in registers, and beyond 32 on the size-class stencils (where a pair belongs to its
larger member; on the row tiles a pair belongs to the half-shell owner).  Lockstep (the oracle starts every checked step from the GPU's state): pair
sets bit-identical, F, T, Sigma and the committed stretches within 1e-10 (FP64) / 1e-5 (mixed)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2108_01013_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_inf(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def crowded(N, n_big):
    rad = synth.lognormal_radii(N, seed=3)
    rad[np.argsort(-rad)[:n_big]] = 10.0
    L = synth.box_for_fraction(rad, 0.55)
    x = synth.relax_positions(rad, L, seed=1003)
    return synth.Workload(f"lognormal N={N} phi=0.55, radii x1.02", x, rad * 1.02, L, synth.default_params([L, L, L]))


@pytest.fixture(scope="module")
def crowded_box():
    return crowded(3000, 4)


@pytest.fixture(scope="module")
def crowded_box_wide():
    """N = 20 000 with eight radii of 10: the row tiles need cells wider than the largest pair
    cutoff, four of them along x (at N = 3000 the box holds three)."""
    return crowded(20_000, 8)


def lockstep(sim, p, w, n0, nsteps, tol):
    hp, hx = sim.history()
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
        assert np.array_equal(sim.pairs(), oracle.pairs_cells(p, s1["x"], w.rad, delta)), f"step {k}: pairs"
        F, T, S, H, npairs = oracle.forces(p, s1["x"], uh, wh, w.rad, n0 + k + 1, st.history, use_cells=True)
        assert rel_inf(s1["F"], F) < tol, f"step {k}: F {rel_inf(s1['F'], F)}"
        assert rel_inf(s1["T"], T) < tol, f"step {k}: T {rel_inf(s1['T'], T)}"
        last, _, _ = sim.read_stress()
        assert rel_inf(last, S) < tol, f"step {k}: Sigma"
        hp, hx = sim.history()
        assert np.array_equal(hp, H.pairs), f"step {k}: history pairs"
        assert np.max(np.abs(hx - H.xi)) <= tol * np.max(np.abs(H.xi)), f"step {k}: stretches"
    return sim.info()


@pytest.mark.parametrize("path,precision", [("sized", 0), ("sized_lanes", 0), ("tiles", 0), ("rows", 0),
                                            ("sized", 1)])
def test_long_history_rows(crowded_box, crowded_box_wide, path, precision):
    from paper_2108_01013_amd.dss import Simulation
    w = crowded_box if path.startswith("sized") else crowded_box_wide
    p = w.params
    say(f"case: long history rows, path {path}, precision {precision}")
    sim = Simulation(p, record_pairs=True, precision=precision)
    if path == "sized":
        sim.set_tuning(sized=True)
    elif path == "sized_lanes":
        sim.set_tuning(sized=True, wave_class=64)     # every row sorted by its own lane
    elif path == "rows":
        sim.set_tuning(tiled=False)                   # every row on the per-particle path
    sim.set_particles(w.x, w.rad)
    sim.step(2)
    info = lockstep(sim, p, w, 2, 3, 1e-10 if precision == 0 else 1e-5)
    say(f"max row fill {info['max_row_fill']}, contacts {info['n_contacts']}, capacity {info['capacity']}")
    assert info["error_flags"] == 0
    assert info["max_row_fill"] > (32 if path.startswith("sized") else 8)
    sim.close()
