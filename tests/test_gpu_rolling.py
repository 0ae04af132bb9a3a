"""Rolling resistance (Appendix roll; reading R19) against the FP64 oracle, on an MI355X:
lockstep steps with both springs per contact, on the row tiles and the size-class stencils,
FP64 within 1e-10 and mixed within 1e-5; rolling stretches carried in the history and in
state snapshots."""
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


def rolling(p):
    return dict(p, kr=0.05 * p["kn"], mu_r=0.1)


def lockstep(sim, p, rad, n0, nsteps, tol):
    hp, hx = sim.history()
    _, hr = sim.history(rolling=True)
    worst_xr = 0.0
    for k in range(nsteps):
        s = sim.state()
        a, aw = oracle.accelerations(p, rad, s["F"], s["T"])
        st = oracle.State(s["x"], s["u"], s["w"], a, aw, rad.copy(), n0 + k,
                          oracle.History(hp.astype(np.int32), hx, hr))
        x_o = oracle.kick_drift(p, st)[0]
        sim.step(1)
        s1 = sim.state()
        uh, wh = sim.eval_velocities()
        assert np.array_equal(s1["x"], x_o)
        delta = oracle.le_offset(p, n0 + k + 1)
        assert np.array_equal(sim.pairs(), oracle.pairs_brute(p, s1["x"], rad, delta)), f"step {k}: pairs"
        F, T, S, H, npairs = oracle.forces(p, s1["x"], uh, wh, rad, n0 + k + 1, st.history)
        assert rel_inf(s1["F"], F) < tol, f"step {k}: F {rel_inf(s1['F'], F)}"
        assert rel_inf(s1["T"], T) < tol, f"step {k}: T {rel_inf(s1['T'], T)}"
        last, _, _ = sim.read_stress()
        assert rel_inf(last, S) < tol, f"step {k}: Sigma"
        hp, hx = sim.history()
        hp2, hr = sim.history(rolling=True)
        assert np.array_equal(hp, H.pairs) and np.array_equal(hp2, H.pairs)
        if len(hp):
            assert np.max(np.abs(hx - H.xi)) <= max(tol, 1e-10) * np.max(np.abs(H.xi))
            assert np.max(np.abs(hr - H.xr)) <= max(tol, 1e-10) * np.max(np.abs(H.xr))
            worst_xr = max(worst_xr, float(np.max(np.abs(H.xr))))
    return worst_xr


@pytest.mark.parametrize("precision,tiled", [(0, True), (1, True), (0, False), (1, False)])
def test_rolling_lockstep(precision, tiled):
    """Row tiles, or (tiled False) every row on the per-particle path of the deferred rows."""
    from paper_2108_01013_amd.dss import Simulation
    w = synth.config_small()
    p = rolling(w.params)
    say(f"case: rolling N=1000 precision={precision} tiled={tiled}")
    sim = Simulation(p, record_pairs=True, precision=precision)
    sim.set_tuning(tiled=tiled)
    sim.set_particles(w.x, w.rad)
    sim.step(5)
    xr = lockstep(sim, p, w.rad, 5, 5, TOL_F if precision == 0 else TOL_MIXED)
    assert xr > 0.0          # the rolling springs are loaded
    sim.close()


def test_rolling_size_class_stencils():
    from paper_2108_01013_amd.dss import Simulation
    rad = synth.lognormal_radii(3000, seed=7)
    L = synth.box_for_fraction(rad, 0.55)
    x = synth.relax_positions(rad, L, seed=8)
    p = rolling(synth.default_params([L, L, L]))
    say("case: rolling, size-class stencils, lognormal N=3000")
    sim = Simulation(p, record_pairs=True)
    sim.set_tuning(sized=True, wave_class=2)
    sim.set_particles(x, rad)
    sim.step(3)
    lockstep(sim, p, rad, 3, 2, TOL_F)
    sim.close()


def test_rolling_snapshot_and_refusals():
    from paper_2108_01013_amd.dss import DssError, Simulation
    w = synth.config_small()
    p = rolling(w.params)
    say("case: rolling snapshot N=1000")
    a = Simulation(p)
    a.set_particles(w.x, w.rad)
    a.step(6)
    blob = a.save_state()
    a.step(4)
    b = Simulation(p)
    b.set_particles(w.x, w.rad)
    b.load_state(blob)
    b.step(4)
    sa, sb = a.state(), b.state()
    for k in ("x", "u", "w", "F", "T"):                      # atomic sums reorder: 1e-11
        assert rel_inf(sb[k], sa[k]) < 1e-11, k
    ha, hb = a.history(rolling=True), b.history(rolling=True)
    assert np.array_equal(ha[0], hb[0]) and len(ha[0]) > 0
    assert rel_inf(hb[1], ha[1]) < 1e-9
    c = Simulation(w.params)
    c.set_particles(w.x, w.rad)
    with pytest.raises(DssError):
        c.history(rolling=True)
    with pytest.raises(DssError):
        c.load_state(blob)            # a snapshot with rolling rows does not fit
    for s in (a, b, c):
        s.close()
