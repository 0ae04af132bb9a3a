"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on an MI355X.

Tolerances (FP64 mode):
  - pair sets, per-cell id sets, cell_start: bit-identical;
  - positions after the drift and wrap: bit-identical (same IEEE expression, no contraction);
  - forces / torques: max |F_gpu - F_oracle| <= 1e-10 max |F_oracle| (atomics reorder sums);
  - stress: per component <= 1e-10 max |Sigma_oracle|;
  - contact history: same pair set, xi within 1e-10 of the largest |xi|.
Lockstep: at every checked step the oracle starts from the GPU's state, so the comparison is
of one step, not of two chaotic trajectories.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2108_01013_amd import synth

pytestmark = pytest.mark.gpu

TOL_F = 1e-10
TOL_S = 1e-10


def _sim(p, **kw):
    from paper_2108_01013_amd.dss import Simulation
    return Simulation(p, **kw)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_inf(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def oracle_state_from_gpu(p, sim, rad, hist_pairs, hist_xi, step):
    s = sim.state()
    a, aw = oracle.accelerations(p, rad, s["F"], s["T"])
    return oracle.State(s["x"], s["u"], s["w"], a, aw, rad.copy(), step,
                        oracle.History(hist_pairs.astype(np.int32), hist_xi)), s


def check_cells(p, sim, x, rad):
    dims, cs, perm = sim.cells()
    dims_o = oracle.cell_dims(p, np.max(rad))
    assert tuple(dims) == tuple(dims_o)
    cs_o, order_o = oracle.cell_sort(p, x, dims)
    assert np.array_equal(cs, cs_o)
    for c in range(len(cs) - 1):
        a = np.sort(perm[cs[c]:cs[c + 1]])
        b = order_o[cs_o[c]:cs_o[c + 1]]
        assert np.array_equal(a, b)


def test_initial_evaluation_small():
    w = synth.config_small()
    p = w.params
    say("case: initial evaluation N=1000")
    sim = _sim(p, record_pairs=True)
    sim.set_particles(w.x, w.rad)
    st, F, T, S = oracle.init_state(p, w.x, w.rad)
    pg = sim.pairs()
    po = oracle.pairs_brute(p, w.x, w.rad, 0.0)
    assert len(pg) == len(po) and np.array_equal(pg, po)
    check_cells(p, sim, w.x, w.rad)
    s = sim.state()
    assert np.array_equal(s["x"], w.x)
    assert rel_inf(s["F"], F) < TOL_F
    assert rel_inf(s["T"], T) < TOL_F
    last, mean, ns = sim.read_stress()
    assert rel_inf(last, S) < TOL_S
    inf = sim.info()
    assert inf["n_pairs"] == len(po)
    assert inf["step"] == 0
    sim.close()


@pytest.mark.parametrize("step0", [0, 777_777])
def test_lockstep_small(step0):
    """N = 1000 (4 tiles of 256 with a ragged tail), 30 lockstep steps, contacts, LE offsets."""
    w = synth.config_small()
    p = dict(w.params)
    if step0:
        p["shear_rate"] = 1.0
    say(f"case: lockstep N=1000 step0={step0}")
    sim = _sim(p, record_pairs=True)
    sim.set_particles(w.x, w.rad)
    if step0:
        sim.set_step(step0)
        sim.compute_forces()
    hp, hx = sim.history()
    assert len(hp) == 0
    nstep = step0
    contacts_seen = 0
    for k in range(30):
        st, s0 = oracle_state_from_gpu(p, sim, w.rad, hp, hx, nstep)
        x_o, u_sh, w_sh, uh_o, wh_o = oracle.kick_drift(p, st)
        sim.step(1)
        nstep += 1
        s1 = sim.state()
        uh_g, wh_g = sim.eval_velocities()
        # positions, half-step velocities: same IEEE expressions
        assert np.array_equal(s1["x"], x_o), f"step {k}: positions differ"
        assert np.array_equal(uh_g, uh_o) and np.array_equal(wh_g, wh_o)
        # pair set on the GPU's positions at the GPU's Lees-Edwards offset
        delta = oracle.le_offset(p, nstep)
        pg = sim.pairs()
        po = oracle.pairs_brute(p, s1["x"], w.rad, delta)
        assert np.array_equal(pg, po), f"step {k}: pair sets differ"
        check_cells(p, sim, s1["x"], w.rad)
        # forces, torques, stress, new history from the same state
        F, T, S, H, npairs = oracle.forces(p, s1["x"], uh_g, wh_g, w.rad, nstep, st.history)
        assert rel_inf(s1["F"], F) < TOL_F, f"step {k}: F"
        assert rel_inf(s1["T"], T) < TOL_F, f"step {k}: T"
        last, mean, ns = sim.read_stress()
        assert rel_inf(last, S) < TOL_S, f"step {k}: Sigma"
        hp, hx = sim.history()
        assert np.array_equal(hp, H.pairs), f"step {k}: history pairs"
        if len(hp):
            assert np.max(np.abs(hx - H.xi)) <= 1e-10 * np.max(np.abs(H.xi)) + 1e-300
        contacts_seen = max(contacts_seen, len(hp))
        # finishing kick
        u_o, w_o, a_o, aw_o = oracle.finish(p, w.rad, F, T, u_sh, w_sh, st.alpha, st.alpha_w)
        assert rel_inf(s1["u"], u_o) < 1e-12
        assert rel_inf(s1["w"], w_o) < 1e-12
    assert contacts_seen >= 10
    sim.close()


def test_le_crossing_windows_all_offsets():
    """Pair sets across the sheared y faces at offsets spanning every cell alignment."""
    w = synth.config_small()
    p = dict(w.params)
    say("case: LE windows N=1000")
    sim = _sim(p, record_pairs=True)
    sim.set_particles(w.x, w.rad)
    L = p["L"][0]
    dims = oracle.cell_dims(p, w.rad.max())
    dcell = L / dims[0]
    for frac in (0.0, 0.25, 0.5, 0.999, 1.0, 1.5, 3.3, dims[0] - 0.5):
        target = frac * dcell
        n = int(round(target / (p["shear_rate"] * p["L"][1] * p["dt"])))
        sim.set_step(n)
        sim.compute_forces()
        delta = oracle.le_offset(p, n)
        pg = sim.pairs()
        po = oracle.pairs_brute(p, w.x, w.rad, delta)
        assert np.array_equal(pg, po), f"delta={delta}"
        s = sim.state()
        F, T, S, H, npairs = oracle.forces(p, w.x, oracle.ambient_velocity(p, w.x),
                                           oracle.ambient_rotation(p, len(w.rad)), w.rad, n)
        assert rel_inf(s["F"], F) < TOL_F
    sim.close()


@pytest.mark.parametrize("N,phi", [(4000, 0.45), (20000, 0.55)])
def test_multi_tile_forces(N, phi):
    w = synth.bidisperse_box(N, phi, seed=N)
    p = w.params
    say(f"case: multi-tile N={N} phi={phi}")
    sim = _sim(p, record_pairs=True)
    sim.set_particles(w.x, w.rad)
    hp, hx = sim.history()
    nstep = 0
    for k in range(5):
        st, s0 = oracle_state_from_gpu(p, sim, w.rad, hp, hx, nstep)
        sim.step(1)
        nstep += 1
        s1 = sim.state()
        uh, wh = sim.eval_velocities()
        po = oracle.pairs_cells(p, s1["x"], w.rad, oracle.le_offset(p, nstep))
        assert np.array_equal(sim.pairs(), po)
        F, T, S, H, npairs = oracle.forces(p, s1["x"], uh, wh, w.rad, nstep, st.history, use_cells=True)
        assert rel_inf(s1["F"], F) < TOL_F and rel_inf(s1["T"], T) < TOL_F
        last, _, _ = sim.read_stress()
        assert rel_inf(last, S) < TOL_S
        hp, hx = sim.history()
        assert np.array_equal(hp, H.pairs)
    sim.close()


def test_full_size_100k():
    """The benchmark workload (N = 100k, phi = 0.55) in the benchmark's launch configuration:
    10 steps, then the whole state checked against the oracle's evaluation of the same state."""
    w = synth.config_single_box()
    p = w.params
    say("case: full size N=100000")
    sim = _sim(p, record_pairs=True)
    sim.set_particles(w.x, w.rad)
    sim.step(9, stress_every=0)
    hp, hx = sim.history()
    st, s0 = oracle_state_from_gpu(p, sim, w.rad, hp, hx, 9)
    x_o, u_sh, w_sh, uh_o, wh_o = oracle.kick_drift(p, st)
    sim.step(1)
    s1 = sim.state()
    uh, wh = sim.eval_velocities()
    assert np.array_equal(s1["x"], x_o)
    po = oracle.pairs_cells(p, s1["x"], w.rad, oracle.le_offset(p, 10))
    assert np.array_equal(sim.pairs(), po)
    F, T, S, H, npairs = oracle.forces(p, s1["x"], uh, wh, w.rad, 10, st.history, use_cells=True)
    assert rel_inf(s1["F"], F) < TOL_F and rel_inf(s1["T"], T) < TOL_F
    last, _, _ = sim.read_stress()
    assert rel_inf(last, S) < TOL_S
    hp, hx = sim.history()
    assert np.array_equal(hp, H.pairs)
    inf = sim.info()
    assert inf["error_flags"] == 0 and inf["max_row_fill"] <= inf["capacity"]
    sim.close()


# ---------------------------------------------------------------------------------------------
# closed forms on the GPU path (the same pins as the oracle's, through the C ABI)
# ---------------------------------------------------------------------------------------------
def test_gpu_free_sphere_in_shear():
    gd = 1.0
    a = 1.4
    p = synth.default_params([20.0, 20.0, 20.0], shear_rate=gd, dt=2e-3)
    x = np.array([[7.0, 8.0, 9.0]])
    say("case: free sphere")
    sim = _sim(p)
    sim.set_particles(x, np.array([a]), u=np.zeros((1, 3)), omega=np.zeros((1, 3)))
    zr = p["dt"] * 15.0 / (p["rho"] * a * a)
    zt = p["dt"] * 9.0 / (2.0 * p["rho"] * a * a)
    for n in range(1, 60):
        sim.step(1)
        s = sim.state()
        wz = -(gd / 2) * (1.0 - (1.0 - zr / 2) ** 2 * (1.0 - zr) ** (n - 1))
        ux = gd * 8.0 * (1.0 - (1.0 - zt / 2) ** 2 * (1.0 - zt) ** (n - 1))
        assert abs(s["w"][0, 2] - wz) <= 1e-12
        assert abs(s["u"][0, 0] - ux) <= 1e-12 * 8.0
    sim.close()


def test_gpu_einstein_and_stress_sampling():
    L = 40.0
    p = synth.default_params([L, L, L], shear_rate=0.7, eta0=1.3)
    g = np.arange(4) * 10.0 + 3.0
    x = np.array([[a, b, c] for a in g for b in g for c in g])
    rad = np.where(np.arange(len(x)) % 3 == 0, 1.4, 1.0)
    say("case: einstein")
    sim = _sim(p)
    sim.set_particles(x, rad)
    phi = (4.0 / 3.0) * math.pi * np.sum(rad ** 3) / L ** 3
    last, mean, ns = sim.read_stress()
    assert abs(last[0, 1] - 1.3 * 0.7 * (1 + 2.5 * phi)) < 1e-14
    sim.step(20, stress_every=5)
    last, mean, ns = sim.read_stress()
    assert ns == 4
    assert abs(mean[0, 1] - 1.3 * 0.7 * (1 + 2.5 * phi)) < 1e-14
    sim.close()


def test_gpu_hooke():
    L = 20.0
    p = synth.default_params([L, L, L], shear_rate=0.0, F_ER=0.0)
    ai, aj, delta = 1.0, 1.4, 3e-3
    n = np.array([1.0, 2.0, -0.5]) / np.linalg.norm([1.0, 2.0, -0.5])
    xi = np.array([8.0, 9.0, 10.0])
    r = (ai + aj - delta) * n
    say("case: hooke")
    sim = _sim(p)
    sim.set_particles(np.array([xi, xi + r]), np.array([ai, aj]), u=np.zeros((2, 3)), omega=np.zeros((2, 3)))
    s = sim.state()
    assert rel_inf(s["F"][0], -p["kn"] * delta * n) < 1e-9
    last, _, _ = sim.read_stress()
    expect = -(np.linalg.norm(r) * p["kn"] * delta / L ** 3) * np.outer(n, n)
    assert rel_inf(last, expect) < 1e-9
    sim.close()


# ---------------------------------------------------------------------------------------------
# error paths of the C ABI
# ---------------------------------------------------------------------------------------------
def test_abi_errors():
    from paper_2108_01013_amd.dss import DssError
    w = synth.config_small()
    p = w.params
    say("case: abi errors")
    sim = _sim(p)
    with pytest.raises(DssError) as e:
        sim.step(1)
    assert e.value.status == 6
    bad = w.x.copy()
    bad[3, 1] = p["L"][1] + 0.1
    with pytest.raises(DssError) as e:
        sim.set_particles(bad, w.rad)
    assert e.value.status == 1
    with pytest.raises(DssError) as e:
        sim.set_particles(w.x, -w.rad)
    assert e.value.status == 1
    sim.close()
    tiny = synth.default_params([8.0, 8.0, 8.0])
    sim = _sim(tiny)
    with pytest.raises(DssError) as e:
        sim.set_particles(np.array([[1.0, 1.0, 1.0]]), np.array([1.0]))
    assert e.value.status == 4
    sim.close()
    # a row capacity of 1 overflows on a box compressed by 3 % (every particle overlaps its
    # neighbours): reported as DSS_ERR_CAPACITY, rows never written past their capacity
    pc = dict(p, L=[0.97 * v for v in p["L"]])
    sim = _sim(pc, capacity=1)
    with pytest.raises(DssError) as e:
        sim.set_particles(w.x * 0.97, w.rad)
        sim.step(1)
    assert e.value.status == 3
    sim.close()
    sim = _sim(pc)
    sim.set_particles(w.x * 0.97, w.rad)
    sim.step(1)
    assert sim.info()["max_row_fill"] >= 2
    sim.close()


# ---------------------------------------------------------------------------------------------
# Mixed precision (FP32 pair arithmetic, FP64 gap / lubrication argument / accumulation):
# pair sets and positions still bit-identical; forces, torques, stress and history within
# 1e-5 of the FP64 oracle.  The measured errors are printed per result.
# ---------------------------------------------------------------------------------------------
TOL_MIXED = 1e-5


def _mixed_errors(p, sim, rad, hp, hx, nstep):
    st, s0 = oracle_state_from_gpu(p, sim, rad, hp, hx, nstep)
    x_o = oracle.kick_drift(p, st)[0]
    sim.step(1)
    s1 = sim.state()
    uh, wh = sim.eval_velocities()
    assert np.array_equal(s1["x"], x_o)
    po = oracle.pairs_cells(p, s1["x"], rad, oracle.le_offset(p, nstep + 1))
    assert np.array_equal(sim.pairs(), po)
    F, T, S, H, npairs = oracle.forces(p, s1["x"], uh, wh, rad, nstep + 1, st.history, use_cells=True)
    last, _, _ = sim.read_stress()
    hp2, hx2 = sim.history()
    assert np.array_equal(hp2, H.pairs)
    err = {"F": rel_inf(s1["F"], F), "T": rel_inf(s1["T"], T), "Sigma": rel_inf(last, S),
           "eta_r": abs(last[0, 1] - S[0, 1]) / abs(S[0, 1]),
           "xi": float(np.max(np.abs(hx2 - H.xi)) / max(np.max(np.abs(H.xi)), 1e-300)) if len(hx2) else 0.0}
    return err, hp2, hx2


@pytest.mark.parametrize("which", ["small", "100k"])
def test_mixed_precision_parity(which):
    from paper_2108_01013_amd.dss import DSS_MIXED
    w = synth.config_small() if which == "small" else synth.config_single_box()
    p = w.params
    say(f"case: mixed precision {which}")
    sim = _sim(p, precision=DSS_MIXED, record_pairs=True)
    sim.set_particles(w.x, w.rad)
    sim.step(5)
    hp, hx = sim.history()
    worst = {}
    nstep = 5
    for k in range(3):
        err, hp, hx = _mixed_errors(p, sim, w.rad, hp, hx, nstep)
        nstep += 1
        for key, v in err.items():
            worst[key] = max(worst.get(key, 0.0), v)
    say(f"mixed precision max relative errors ({which}, N={len(w.rad)}): " +
        ", ".join(f"{k}={v:.2e}" for k, v in worst.items()))
    for key in ("F", "T", "Sigma", "eta_r", "xi"):
        assert worst[key] < TOL_MIXED, (key, worst[key])
    sim.close()


# ---------------------------------------------------------------------------------------------
# High size ratio: lognormal radii truncated to [1, 10] (the history capacity is the paper's
# estimate for the largest particle), on the row tiles and with every row on the per-particle
# path; FP64 within 1e-10 and mixed within 1e-5 of the oracle.
# ---------------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def poly_box():
    rad = synth.lognormal_radii(3000, seed=7)
    L = synth.box_for_fraction(rad, 0.55)
    x = synth.relax_positions(rad, L, seed=8)
    return synth.Workload("lognormal N=3000 phi=0.55", x, rad, L, synth.default_params([L, L, L]))


@pytest.mark.parametrize("tiled,precision", [(True, 0), (False, 0), (True, 1)])
def test_high_size_ratio(poly_box, tiled, precision):
    w = poly_box
    p = w.params
    say(f"case: size ratio {w.rad.max() / w.rad.min():.1f} N=3000 tiled={tiled} precision={precision}")
    sim = _sim(p, record_pairs=True, precision=precision)
    sim.set_tuning(tiled=tiled)
    sim.set_particles(w.x, w.rad)
    assert sim.info()["capacity"] == oracle.history_capacity(w.rad.max(), w.rad.min())
    sim.step(3)
    hp, hx = sim.history()
    tol = TOL_F if precision == 0 else TOL_MIXED
    for k in range(2):
        st, s0 = oracle_state_from_gpu(p, sim, w.rad, hp, hx, 3 + k)
        x_o = oracle.kick_drift(p, st)[0]
        sim.step(1)
        s1 = sim.state()
        uh, wh = sim.eval_velocities()
        assert np.array_equal(s1["x"], x_o)
        assert np.array_equal(sim.pairs(), oracle.pairs_brute(p, s1["x"], w.rad, oracle.le_offset(p, 4 + k)))
        F, T, S, H, npairs = oracle.forces(p, s1["x"], uh, wh, w.rad, 4 + k, st.history)
        assert rel_inf(s1["F"], F) < tol and rel_inf(s1["T"], T) < tol
        last, _, _ = sim.read_stress()
        assert rel_inf(last, S) < tol
        hp, hx = sim.history()
        assert np.array_equal(hp, H.pairs)
    sim.close()


@pytest.mark.parametrize("case", ["fp64", "mixed", "sized"])
def test_free_trajectory_100_steps(case):
    """100 steps run freely on the GPU and on the oracle from the same initial state, with no
    state passed between them: positions (nearest image), velocities, rotations and the mean of
    the ten stress samples.  fp64 and mixed: the small workload (N = 1000); sized: lognormal
    radii on [1, 10] (N = 3000) on the size-class stencils.  Not a bitwise contract: the force
    atomics sum in another order at every evaluation and the contacts amplify the difference.
    Measured (fp64): 3.6e-15 in position, 8.5e-15 / 9.3e-15 in u / w, 3.9e-16 in the mean
    stress.  Bounds: 1e-10 of the largest value in FP64, 1e-5 in mixed precision."""
    if case == "sized":
        rad = synth.lognormal_radii(3000, seed=7)
        L = synth.box_for_fraction(rad, 0.55)
        x = synth.relax_positions(rad, L, seed=8)
        p = synth.default_params([L, L, L])
    else:
        w = synth.config_small()
        x, rad, p = w.x, w.rad, w.params
    tol = 1e-5 if case == "mixed" else 1e-10
    say(f"case: free trajectory, 100 steps, {case} N={len(rad)}")
    sim = _sim(p, precision=1 if case == "mixed" else 0)
    if case == "sized":
        sim.set_tuning(sized=True, wave_class=2)
    sim.set_particles(x, rad)
    sim.step(100, stress_every=10)
    s = sim.state()
    _, mean_g, ns = sim.read_stress()
    sim.close()
    assert ns == 10
    st, F, T, S = oracle.init_state(p, x, rad)
    samples = []
    for n in range(1, 101):
        st, F, T, S, npairs, _ = oracle.step(p, st, use_cells=True)
        if n % 10 == 0:
            samples.append(S)
    mean_o = np.mean(samples, axis=0)
    delta = oracle.le_offset(p, 100)
    dx = np.array([oracle.min_image(p, delta, a, b) for a, b in zip(st.x, s["x"])])
    ex = float(np.max(np.abs(dx)))
    eu, ew, es = rel_inf(s["u"], st.u), rel_inf(s["w"], st.w), rel_inf(mean_g, mean_o)
    say(f"100-step deviations ({case}): |dx|max {ex:.2e}, u {eu:.2e}, w {ew:.2e}, mean Sigma {es:.2e}")
    assert ex <= tol * p["a0"] and eu < tol and ew < tol and es < tol
