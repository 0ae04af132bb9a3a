"""Wavy shear of eq. (uinf) (reading R20: local rotation and strain, Faxen terms, R'(E) columns at
their own particles) on an MI355X: a free sphere against the discrete closed form, and lockstep
parity with the FP64 oracle on the row tiles (FP64 1e-10, mixed 1e-5) and the size-class
stencils."""
import math
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


def wavy(p, amp=20.0, n=1):
    """The paper's wavy case: W / (gdot a0) = 20, one period along L_y."""
    return dict(p, wave_amp=amp * p["shear_rate"] * p["a0"], wave_n=float(n))


@pytest.mark.parametrize("a,y", [(1.0, 3.3), (1.4, 14.1)])
def test_free_sphere_in_wavy_shear(a, y):
    from paper_2108_01013_amd.dss import Simulation
    L = 20.0
    p = synth.default_params([L, L, L], shear_rate=0.7, dt=2e-3)
    p = dict(p, wave_amp=4.0, wave_n=2.0)
    k = 2 * math.pi * 2.0 / L
    say(f"case: free sphere in the wavy shear a={a}")
    sim = Simulation(p)
    sim.set_particles(np.array([[7.0, y, 9.0]]), np.array([a]), u=np.zeros((1, 3)), omega=np.zeros((1, 3)))
    zr = p["dt"] * 15.0 * p["eta0"] / (p["rho"] * a * a)
    zt = p["dt"] * 9.0 * p["eta0"] / (2.0 * p["rho"] * a * a)
    ux_star = 0.7 * y + 4.0 * math.sin(k * y) * (1.0 - a * a * k * k / 6.0)
    wz_star = -0.5 * (0.7 + 4.0 * k * math.cos(k * y))
    for n in (1, 2, 5, 40, 150):
        sim.step(n - sim.info()["step"])
        s = sim.state()
        fz = 1.0 - (1.0 - zr / 2) ** 2 * (1.0 - zr) ** (n - 1)
        ft = 1.0 - (1.0 - zt / 2) ** 2 * (1.0 - zt) ** (n - 1)
        assert abs(s["w"][0, 2] - wz_star * fz) <= 1e-12 * abs(wz_star)
        assert abs(s["u"][0, 0] - ux_star * ft) <= 1e-12 * abs(ux_star)
    sim.close()


def lockstep(sim, p, rad, n0, nsteps, tol):
    hp, hx = sim.history()
    for k in range(nsteps):
        s = sim.state()
        a, aw = oracle.accelerations(p, rad, s["F"], s["T"])
        st = oracle.State(s["x"], s["u"], s["w"], a, aw, rad.copy(), n0 + k, oracle.History(hp.astype(np.int32), hx))
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
        assert rel_inf(last, S) < tol, f"step {k}: Sigma {rel_inf(last, S)}"
        hp, hx = sim.history()
        assert np.array_equal(hp, H.pairs)
        if len(hp):
            assert np.max(np.abs(hx - H.xi)) <= max(tol, 1e-10) * np.max(np.abs(H.xi))


@pytest.mark.parametrize("precision,tiled", [(0, True), (1, True), (0, False), (1, False)])
def test_wavy_lockstep(precision, tiled):
    """Row tiles, or (tiled False) every row on the per-particle path of the deferred rows."""
    from paper_2108_01013_amd.dss import DssError, Simulation
    w = synth.config_small()
    p = wavy(w.params)
    say(f"case: wavy shear N=1000 precision={precision} tiled={tiled}")
    sim = Simulation(p, record_pairs=True, precision=precision)
    sim.set_tuning(tiled=tiled)
    sim.set_particles(w.x, w.rad)
    s0 = sim.state()
    assert rel_inf(s0["u"], oracle.ambient_velocity(p, w.x)) < 1e-15
    assert rel_inf(s0["w"], oracle.ambient_rotation(p, len(w.rad), w.x)) < 1e-15
    sim.step(3)
    lockstep(sim, p, w.rad, 3, 4, TOL_F if precision == 0 else TOL_MIXED)
    if precision == 0:
        sim.compute_forces()
        with pytest.raises(DssError):
            sim.adjoint(4, 2, 2)
    sim.close()


def test_wavy_size_class_stencils():
    from paper_2108_01013_amd.dss import Simulation
    rad = synth.lognormal_radii(3000, seed=7)
    L = synth.box_for_fraction(rad, 0.55)
    x = synth.relax_positions(rad, L, seed=8)
    p = wavy(synth.default_params([L, L, L]), amp=5.0, n=2)
    say("case: wavy shear, size-class stencils, lognormal N=3000")
    sim = Simulation(p, record_pairs=True)
    sim.set_tuning(sized=True, wave_class=2)
    sim.set_particles(x, rad)
    sim.step(2)
    lockstep(sim, p, rad, 2, 2, TOL_F)
    sim.close()
