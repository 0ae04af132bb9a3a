"""Discrete adjoint of the time step (dss_adjoint) on an MI355X against central finite
differences of the FP64 oracle's stress objective J = mean_samples(Sigma_xy).

The derivative is that of the run with its pair set, contact states and Coulomb-cap states
held fixed, so every finite difference is checked to stay on the unperturbed run's branch
(same listed-pair counts, contact sets and stick/slip states of every contact at every step,
from the oracle's branch record).  Window: N = 400 bidisperse
spheres at phi = 0.52, mu = 0.1 (sliding contacts, so dJ/dmu != 0), 20 steps, stress every 5,
checkpoints every 7 steps (segments of 7, 7, 6: the segment boundaries and a ragged last
segment are crossed)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2108_01013_amd import synth

pytestmark = pytest.mark.gpu

# finite-difference steps: small enough to stay on the run's branch, large enough that the
# rounding noise of J (~1e-13 absolute) stays below the tolerances
EPS = {"mu": 1e-6, "F_ER": 1e-5, "x": 1e-7, "u": 1e-6, "w": 1e-6}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def window():
    w = synth.bidisperse_box(400, 0.52, seed=21)
    p = dict(w.params, mu=0.1)
    u0 = oracle.ambient_velocity(p, w.x)
    w0 = oracle.ambient_rotation(p, len(w.rad))
    W = np.zeros((3, 3))
    W[0, 1] = 1.0
    return w, p, u0, w0, W


def gpu_adjoint(p, w, u0, w0, W, K=20, se=5, C=7):
    from paper_2108_01013_amd.dss import Simulation
    sim = Simulation(p)
    sim.set_particles(w.x, w.rad, u0, w0)
    r = sim.adjoint(K, se, C, W)
    info = sim.info()
    last, mean, ns = sim.read_stress()
    sim.close()
    return r, info, mean, ns


def fd(p, w, u0, w0, W, br0, perturb, eps, K=20, se=5):
    """Central difference of the oracle's J, or None if a perturbed run left the branch."""
    vals = []
    for sgn in (1.0, -1.0):
        pp, x, u, ww = perturb(sgn * eps)
        J, br = oracle.stress_objective(pp, x, w.rad, u, ww, K, se, W)
        if br != br0:
            return None
        vals.append(J)
    return (vals[0] - vals[1]) / (2 * eps)


def test_adjoint_objective_and_end_state(window):
    w, p, u0, w0, W = window
    say("case: adjoint J and end state N=400")
    r, info, mean, ns = gpu_adjoint(p, w, u0, w0, W)
    J0, _ = oracle.stress_objective(p, w.x, w.rad, u0, w0, 20, 5, W)
    assert abs(r["J"] - J0) <= 1e-10 * abs(J0)
    assert ns == 4 and abs(mean[0, 1] - J0) <= 1e-10 * abs(J0)
    assert info["step"] == 20 and info["error_flags"] == 0


def test_adjoint_parameters_vs_oracle_fd(window):
    w, p, u0, w0, W = window
    say("case: adjoint dJ/dmu, dJ/dF_ER N=400")
    r, *_ = gpu_adjoint(p, w, u0, w0, W)
    _, br0 = oracle.stress_objective(p, w.x, w.rad, u0, w0, 20, 5, W)
    for name, key, tol in (("mu", "dmu", 1e-5), ("F_ER", "dF_ER", 1e-3)):
        g = fd(p, w, u0, w0, W, br0, lambda e: (dict(p, **{name: p[name] + e}), w.x, u0, w0), EPS[name])
        assert g is not None, "finite difference left the branch of the run"
        say(f"d J / d {name}: adjoint {r[key]:.10e}  oracle FD {g:.10e}")
        assert abs(r[key] - g) <= tol * abs(g) + 1e-8, (name, r[key], g)
    assert abs(r["dmu"]) > 1e-3    # sliding contacts: the Coulomb cap is active


@pytest.mark.parametrize("which", ["x", "u", "w"])
def test_adjoint_state_vs_oracle_fd(window, which):
    w, p, u0, w0, W = window
    say(f"case: adjoint dJ/d{which}0 N=400")
    r, *_ = gpu_adjoint(p, w, u0, w0, W)
    _, br0 = oracle.stress_objective(p, w.x, w.rad, u0, w0, 20, 5, W)
    rng = np.random.default_rng({"x": 1, "u": 2, "w": 3}[which])
    checked = 0
    for d in range(8):
        if checked == 3:
            break
        v = rng.normal(size=w.x.shape)
        if which == "x":
            L = np.array(p["L"])
            v[np.any((w.x < 1e-4) | (w.x > L - 1e-4), axis=1)] = 0.0   # stay inside the box
            pert = lambda e: (p, w.x + e * v, u0, w0)  # noqa: E731
        elif which == "u":
            pert = lambda e: (p, w.x, u0 + e * v, w0)  # noqa: E731
        else:
            pert = lambda e: (p, w.x, u0, w0 + e * v)  # noqa: E731
        g = fd(p, w, u0, w0, W, br0, pert, EPS[which])
        if g is None:
            say(f"direction {d}: a listed pair crosses the cutoff within the step; skipped")
            continue
        ad = float(np.sum(r["d" + which] * v))
        say(f"direction {d}: adjoint {ad:.10e}  oracle FD {g:.10e}")
        assert abs(ad - g) <= 1e-5 * abs(g) + 1e-6, (which, d, ad, g)
        checked += 1
    assert checked == 3


def gate_counts(p, x, rad, step):
    """Listed pairs inside the lubrication range, |r| < c (a_i + a_j), and inside the ranges of
    repulsion (h < 20 lambda_D) and attraction (h < 4 a0) at time index step (reading R18)."""
    delta = oracle.le_offset(p, step)
    pr = oracle.pairs_cells(p, x, rad, delta)
    a, b = pr[:, 0], pr[:, 1]
    L = np.asarray(p["L"], np.float64)
    d = x[b] - x[a]
    up, dn = d[:, 1] > L[1] / 2, d[:, 1] < -L[1] / 2
    d[up, 1] -= L[1]
    d[up, 0] -= delta
    d[dn, 1] += L[1]
    d[dn, 0] += delta
    d[:, 0] -= L[0] * np.rint(d[:, 0] / L[0])
    d[:, 2] -= L[2] * np.rint(d[:, 2] / L[2])
    dist = np.sqrt(np.sum(d * d, axis=1))
    s = rad[a] + rad[b]
    h = dist - s
    return (int(np.sum(dist < p["cutoff_factor"] * s)), int(np.sum(h < 20.0 * p["lambda_D"])),
            int(np.sum(h < 4.0 * p["a0"])))


def ec_objective(p, x0, rad, u0, w0, W, K=20, se=5):
    """The oracle's J of the run, with a branch record that also holds the gate counts of every
    evaluation: a finite difference that moves a pair across the edge of a range (where its
    force jumps) leaves the branch."""
    st, F, T, S = oracle.init_state(p, x0, rad, u0, w0, use_cells=True)
    samples, br = [], [gate_counts(p, st.x, rad, 0)]
    for n in range(1, K + 1):
        st, F, T, S, npairs, _ = oracle.step(p, st, use_cells=True)
        br.append((npairs, st.history.pairs.tobytes(), st.history.capped.tobytes(), gate_counts(p, st.x, rad, n)))
        if n % se == 0:
            samples.append(np.asarray(S).reshape(3, 3))
    return float(np.sum(W * np.mean(samples, axis=0))), br


def test_adjoint_ec_ranges_vs_oracle_fd(window):
    """Electro-chemical forces over their own ranges (reading R18: attraction A = 2e-3 out to
    4 a0, repulsion to 20 lambda_D, lubrication only inside 1.1 (a_i + a_j)): J, dJ/dF_ER and
    two directions of dJ/dx0 (40 particles moved each) against central differences of the
    oracle's objective.  N = 4000 at phi = 0.45, so that the lattice of the longer cutoff still
    has 4 x 3 x 3 cells; mu = 1 (the sliding contacts are the window's concern).  The
    forces jump at the edges of the ranges, so the branch record of the finite differences
    also holds the number of pairs inside each range at every evaluation, beside the contact
    sets and the stick/slip state of every contact."""
    _, _, _, _, W = window
    w = synth.bidisperse_box(4000, 0.45, seed=23)
    p = dict(w.params, mu=1.0, ec_ranges=1, hamaker=2e-3)
    u0 = oracle.ambient_velocity(p, w.x)
    w0 = oracle.ambient_rotation(p, len(w.rad))
    say("case: adjoint with the electro-chemical ranges N=4000")
    r, info, mean, ns = gpu_adjoint(p, w, u0, w0, W)
    J0, br0 = ec_objective(p, w.x, w.rad, u0, w0, W)
    assert abs(r["J"] - J0) <= 1e-10 * abs(J0)

    def central(perturb, eps):
        vals = []
        for sgn in (1.0, -1.0):
            pp, x, u, ww = perturb(sgn * eps)
            J, br = ec_objective(pp, x, w.rad, u, ww, W)
            if br != br0:
                return None
            vals.append(J)
        return (vals[0] - vals[1]) / (2 * eps)

    g = central(lambda e: (dict(p, F_ER=p["F_ER"] + e), w.x, u0, w0), EPS["F_ER"])
    assert g is not None, "finite difference left the branch of the run"
    say(f"d J / d F_ER: adjoint {r['dF_ER']:.10e}  oracle FD {g:.10e}")
    assert abs(r["dF_ER"] - g) <= 1e-3 * abs(g) + 1e-8
    rng = np.random.default_rng(11)
    L = np.array(p["L"])
    checked = 0
    for d in range(12):
        if checked == 2:
            break
        # 40 particles moved per direction: few contacts change, so few kinks are met
        v = np.zeros_like(w.x)
        moved = rng.choice(len(w.rad), 40, replace=False)
        v[moved] = rng.normal(size=(40, 3))
        v[np.any((w.x < 1e-4) | (w.x > L - 1e-4), axis=1)] = 0.0
        gx = central(lambda e: (p, w.x + e * v, u0, w0), EPS["x"])
        if gx is None:
            say(f"direction {d}: a pair crosses a cutoff, a range edge or a Coulomb cap; skipped")
            continue
        ad = float(np.sum(r["dx"] * v))
        say(f"direction {d}: adjoint {ad:.10e}  oracle FD {gx:.10e}")
        assert abs(ad - gx) <= 1e-5 * abs(gx) + 1e-6, (d, ad, gx)
        checked += 1
    assert checked == 2


def test_adjoint_rolling_resistance_vs_oracle_fd(window):
    """Rolling resistance (reading R19: k_r = 0.5 k_n, mu_r = 0.1) on the N = 400 window: J,
    dJ/dmu and two directions each of dJ/dx0 and dJ/dw0 against central differences of the
    oracle's objective.  The rolling stretch is carried from step to step like the tangential
    one, so its adjoint crosses every step and every checkpoint segment; on this window rolling
    moves dJ/dw0 by about 2 %, far above the tolerance.  The branch record holds whether each
    rolling spring is at its Coulomb limit, beside the tangential stick/slip state."""
    w, p0, u0, w0, W = window
    p = dict(p0, kr=0.5 * p0["kn"], mu_r=0.1)
    say("case: adjoint with rolling resistance N=400")
    r, info, mean, ns = gpu_adjoint(p, w, u0, w0, W)
    J0, br0 = oracle.stress_objective(p, w.x, w.rad, u0, w0, 20, 5, W)
    Jn, _ = oracle.stress_objective(p0, w.x, w.rad, u0, w0, 20, 5, W)
    assert abs(r["J"] - J0) <= 1e-10 * abs(J0)
    assert abs(J0 - Jn) > 1e-6 * abs(Jn)     # the rolling torques change the run

    def central(perturb, eps):
        vals = []
        for sgn in (1.0, -1.0):
            pp, x, u, ww = perturb(sgn * eps)
            J, br = oracle.stress_objective(pp, x, w.rad, u, ww, 20, 5, W)
            if br != br0:
                return None
            vals.append(J)
        return (vals[0] - vals[1]) / (2 * eps)

    g = central(lambda e: (dict(p, mu=p["mu"] + e), w.x, u0, w0), EPS["mu"])
    assert g is not None, "finite difference left the branch of the run"
    say(f"d J / d mu: adjoint {r['dmu']:.10e}  oracle FD {g:.10e}")
    assert abs(r["dmu"] - g) <= 1e-5 * abs(g) + 1e-8
    L = np.array(p["L"])
    for which, seed in (("x", 31), ("w", 32)):
        rng = np.random.default_rng(seed)
        checked = 0
        for d in range(10):
            if checked == 2:
                break
            v = rng.normal(size=w.x.shape)
            if which == "x":
                v[np.any((w.x < 1e-4) | (w.x > L - 1e-4), axis=1)] = 0.0
                pert = lambda e: (p, w.x + e * v, u0, w0)  # noqa: E731
            else:
                pert = lambda e: (p, w.x, u0, w0 + e * v)  # noqa: E731
            # dJ/dw0 along a direction is ~1e-2 against J ~ 12: a step of 1e-5 keeps the rounding
            # noise of J (~1e-13) far below the tolerance
            gv = central(pert, EPS[which] if which == "x" else 1e-5)
            if gv is None:
                say(f"d{which} direction {d}: a pair crosses a cutoff or a Coulomb limit; skipped")
                continue
            ad = float(np.sum(r["d" + which] * v))
            say(f"d{which} direction {d}: adjoint {ad:.10e}  oracle FD {gv:.10e}")
            assert abs(ad - gv) <= 1e-5 * abs(gv) + 1e-6, (which, d, ad, gv)
            checked += 1
        assert checked == 2, which


def test_adjoint_checkpoint_spacing_invariance(window):
    """The gradient does not depend on the checkpoint spacing (1 segment vs segments of 3)."""
    w, p, u0, w0, W = window
    say("case: adjoint checkpoint spacing N=400")
    a, *_ = gpu_adjoint(p, w, u0, w0, W, C=20)
    b, *_ = gpu_adjoint(p, w, u0, w0, W, C=3)
    for k in ("dx", "du", "dw"):
        assert np.max(np.abs(a[k] - b[k])) <= 1e-8 * np.max(np.abs(a[k])), k
    assert abs(a["dmu"] - b["dmu"]) <= 1e-8 * abs(a["dmu"])


def test_adjoint_workspace_reuse(window):
    """Calls on one handle reuse the adjoint's device workspace (checkpoints, tape, reverse
    buffers): repeated calls from the same state, and a call with more checkpoints and a
    shorter segment in between, give the gradients of a fresh handle."""
    from paper_2108_01013_amd.dss import Simulation
    w, p, u0, w0, W = window
    say("case: adjoint workspace reuse N=400")
    sim = Simulation(p)
    sim.set_particles(w.x, w.rad, u0, w0)
    blob = sim.save_state()
    runs = []
    for K, se, C in ((20, 5, 7), (20, 5, 7), (12, 4, 3), (20, 5, 7)):
        sim.load_state(blob)
        runs.append(sim.adjoint(K, se, C, W))
    sim.close()
    ref20, *_ = gpu_adjoint(p, w, u0, w0, W)
    ref12, *_ = gpu_adjoint(p, w, u0, w0, W, K=12, se=4, C=3)
    for r, ref in zip(runs, (ref20, ref20, ref12, ref20)):
        assert abs(r["J"] - ref["J"]) <= 1e-12 * abs(ref["J"])
        for k in ("dx", "du", "dw"):
            assert np.max(np.abs(r[k] - ref[k])) <= 1e-12 * np.max(np.abs(ref[k])), k
        for k in ("dmu", "dF_ER"):
            assert abs(r[k] - ref[k]) <= 1e-12 * abs(ref[k]), k


def test_adjoint_rows_on_per_particle_path(window):
    """Every cell row on the per-particle path (tiling off), in the forward run and in the
    recomputed segments, whose pair records then come from that path: the gradients of the row
    tiles.  Only the order of the FP64 force sums differs (the partner sides are added
    atomically), about 1e-16 relative per evaluation, grown over the 20 steps of the window."""
    from paper_2108_01013_amd.dss import Simulation
    w, p, u0, w0, W = window
    say("case: adjoint with every row on the per-particle path N=400")
    sim = Simulation(p)
    sim.set_tuning(tiled=False)
    sim.set_particles(w.x, w.rad, u0, w0)
    r = sim.adjoint(20, 5, 7, W)
    sim.close()
    ref, *_ = gpu_adjoint(p, w, u0, w0, W)
    rel = {k: float(np.max(np.abs(r[k] - ref[k])) / np.max(np.abs(ref[k]))) for k in ("J", "dx", "du", "dw", "dmu", "dF_ER")}
    say(f"relative differences to the row tiles: {rel}")
    tol = 1e-12                # measured: at most 4e-16
    assert abs(r["J"] - ref["J"]) <= tol * abs(ref["J"])
    for k in ("dx", "du", "dw"):
        assert np.max(np.abs(r[k] - ref[k])) <= tol * np.max(np.abs(ref[k])), k
    for k in ("dmu", "dF_ER"):
        assert abs(r[k] - ref[k]) <= tol * abs(ref[k]), k


@pytest.mark.parametrize("cap", [1, 3])
def test_adjoint_pair_list_overflow(window, cap):
    """Per-particle lists of recorded pairs cut to cap entries (tuning adj_cap), so that most
    particles' pairs go through the overflow list: the gradients equal the default's."""
    from paper_2108_01013_amd.dss import DssError, Simulation
    w, p, u0, w0, W = window
    say(f"case: adjoint pair lists of {cap} N=400")
    sim = Simulation(p)
    with pytest.raises(DssError):
        sim.set_tuning(adj_cap=5000)
    sim.set_tuning(adj_cap=cap)
    assert sim.tuning()["adj_cap"] == cap
    sim.set_particles(w.x, w.rad, u0, w0)
    r = sim.adjoint(20, 5, 7, W)
    sim.close()
    ref, *_ = gpu_adjoint(p, w, u0, w0, W)
    assert abs(r["J"] - ref["J"]) <= 1e-12 * abs(ref["J"])
    for k in ("dx", "du", "dw"):
        assert np.max(np.abs(r[k] - ref[k])) <= 1e-12 * np.max(np.abs(ref[k])), k
    for k in ("dmu", "dF_ER"):
        assert abs(r[k] - ref[k]) <= 1e-12 * abs(ref[k]), k


def test_adjoint_torch_function(window):
    """torch.autograd through StressObjective equals the direct adjoint."""
    import torch

    from paper_2108_01013_amd.adjoint import stress_objective
    w, p, u0, w0, W = window
    say("case: adjoint torch.autograd N=400")
    dev = torch.device("cuda", 0)
    x = torch.tensor(w.x, device=dev, requires_grad=True)
    u = torch.tensor(u0, device=dev, requires_grad=True)
    om = torch.tensor(w0, device=dev, requires_grad=True)
    mu = torch.tensor(p["mu"], dtype=torch.float64, requires_grad=True)
    fer = torch.tensor(p["F_ER"], dtype=torch.float64, requires_grad=True)
    J = stress_objective(x, u, om, mu, fer, torch.tensor(w.rad, device=dev), p, 20, 5, 7)
    (2.0 * J).backward()
    r, *_ = gpu_adjoint(p, w, u0, w0, W)
    assert abs(J.item() - r["J"]) <= 1e-10 * abs(r["J"])
    assert np.max(np.abs(x.grad.cpu().numpy() - 2 * r["dx"])) <= 1e-8 * np.max(np.abs(r["dx"]))
    assert abs(mu.grad.item() - 2 * r["dmu"]) <= 1e-8 * abs(r["dmu"])


def test_adjoint_full_size_50k():
    """The adjoint workload (N = 50k, phi = 0.56, 200 steps, checkpoints every 20): J equals
    the forward run's, the gradient is finite, and a directional derivative in F_ER matches
    a GPU finite difference over a 10-step window."""
    from paper_2108_01013_amd.dss import Simulation
    w = synth.bidisperse_box(50_000, 0.56, seed=5)
    p = w.params
    W = np.zeros((3, 3))
    W[0, 1] = 1.0
    say("case: adjoint N=50000 200 steps")
    sim = Simulation(p)
    sim.set_particles(w.x, w.rad)
    r = sim.adjoint(200, 10, 20, W)
    sim.close()
    for k in ("dx", "du", "dw"):
        assert np.all(np.isfinite(r[k]))
    sim = Simulation(p)
    sim.set_particles(w.x, w.rad)
    sim.step(200, stress_every=10)
    _, mean, ns = sim.read_stress()
    sim.close()
    assert ns == 20 and abs(mean[0, 1] - r["J"]) <= 1e-8 * abs(r["J"])
    # short window: FD in F_ER on the GPU forward
    sim = Simulation(p)
    sim.set_particles(w.x, w.rad)
    r10 = sim.adjoint(10, 5, 5, W)
    sim.close()
    vals = []
    for sgn in (1.0, -1.0):
        s2 = Simulation(dict(p, F_ER=p["F_ER"] + sgn * 1e-5))
        s2.set_particles(w.x, w.rad)
        s2.step(10, stress_every=5)
        _, m2, _ = s2.read_stress()
        s2.close()
        vals.append(m2[0, 1])
    g = (vals[0] - vals[1]) / 2e-5
    say(f"N=50000 d J / d F_ER over 10 steps: adjoint {r10['dF_ER']:.8e}  GPU FD {g:.8e}")
    assert abs(r10["dF_ER"] - g) <= 1e-3 * abs(g) + 1e-9


def test_adjoint_mixed_forward(window):
    """Forward in mixed precision (FP32 pair arithmetic), reverse in FP64: the gradient agrees
    with the FP64 oracle's finite differences to the mixed mode's accuracy."""
    from paper_2108_01013_amd.dss import DSS_MIXED, Simulation
    w, p, u0, w0, W = window
    say("case: adjoint with a mixed-precision forward N=400")
    sim = Simulation(p, precision=DSS_MIXED)
    sim.set_particles(w.x, w.rad, u0, w0)
    r = sim.adjoint(20, 5, 7, W)
    sim.close()
    J0, br0 = oracle.stress_objective(p, w.x, w.rad, u0, w0, 20, 5, W)
    assert abs(r["J"] - J0) <= 1e-5 * abs(J0)
    g = fd(p, w, u0, w0, W, br0, lambda e: (dict(p, mu=p["mu"] + e), w.x, u0, w0), EPS["mu"])
    assert g is not None and abs(r["dmu"] - g) <= 1e-4 * abs(g)
    rng = np.random.default_rng(9)
    L = np.array(p["L"])
    checked = 0
    for d in range(8):
        v = rng.normal(size=w.x.shape)
        v[np.any((w.x < 1e-4) | (w.x > L - 1e-4), axis=1)] = 0.0
        g = fd(p, w, u0, w0, W, br0, lambda e: (p, w.x + e * v, u0, w0), EPS["x"])
        if g is None:
            say(f"mixed forward: direction {d} leaves the branch; skipped")
            continue
        ad = float(np.sum(r["dx"] * v))
        say(f"mixed forward: d J / d x0 . v adjoint {ad:.8e} oracle FD {g:.8e}")
        assert abs(ad - g) <= 1e-4 * abs(g)
        checked += 1
        break
    assert checked == 1


def test_adjoint_config5_vs_oracle_fd():
    """The adjoint workload at its full size: N = 50k bidisperse spheres at phi = 0.56, a 20-step
    window from the relaxed packing (stress every 10, checkpoints every 10, so a segment boundary
    is crossed).  J, dJ/dmu, dJ/dF_ER and one localized direction of dJ/dx0 (40 particles moved)
    against central finite differences of the FP64 oracle at eps = 1e-6, each kept only when
    both perturbed runs stay on the unperturbed run's branch (pair sets, contact sets and the
    stick/slip state of every contact at every step; a smaller eps is tried when one does not).
    Both forward precisions: FP64 (tolerance 1e-5) and mixed (FP32 pair arithmetic, tolerance
    1e-4; the gradient is that of the mixed run's own trajectory).  A central difference cannot
    resolve a derivative below the rounding of J itself: each bound adds 4 ulp(J) / (2 eps)
    (J ~ 17 and eps = 1e-6 give 7e-9, about 3e-5 of dJ/dF_ER ~ 2.6e-4), and dJ/dF_ER is also
    checked at eps = 1e-4 (resolution 7e-11), where the 1e-5 bound is far above the noise."""
    from paper_2108_01013_amd.dss import DSS_FP64, DSS_MIXED, Simulation
    w = synth.bidisperse_box(50_000, 0.56, seed=5)
    p = w.params
    u0 = oracle.ambient_velocity(p, w.x)
    w0 = oracle.ambient_rotation(p, len(w.rad))
    W = np.zeros((3, 3))
    W[0, 1] = 1.0
    K, se, C = 20, 10, 10
    say("case: adjoint N=50000 phi=0.56, 20-step window, FP64 and mixed forward")
    res = {}
    for prec in (DSS_FP64, DSS_MIXED):
        sim = Simulation(p, precision=prec)
        sim.set_particles(w.x, w.rad, u0, w0)
        res[prec] = sim.adjoint(K, se, C, W)
        sim.close()
    J0, br0 = oracle.stress_objective(p, w.x, w.rad, u0, w0, K, se, W, use_cells=True)
    say(f"J: oracle {J0:.12e}  FP64 {res[DSS_FP64]['J']:.12e}  mixed {res[DSS_MIXED]['J']:.12e}")
    assert abs(res[DSS_FP64]["J"] - J0) <= 1e-10 * abs(J0)
    assert abs(res[DSS_MIXED]["J"] - J0) <= 1e-5 * abs(J0)
    n_slip = sum(int(np.count_nonzero(np.frombuffer(b[2], np.int32) & 1)) for b in br0)
    say(f"sliding contact-steps in the window: {n_slip}")
    assert n_slip > 0          # else dJ/dmu would vanish identically

    def central(perturb, steps=(1e-6, 2.5e-7, 6.25e-8)):
        for eps in steps:
            vals = []
            for sgn in (1.0, -1.0):
                pp, x = perturb(sgn * eps)
                J, br = oracle.stress_objective(pp, x, w.rad, u0, w0, K, se, W, use_cells=True)
                if br != br0:
                    break
                vals.append(J)
            if len(vals) == 2:
                return (vals[0] - vals[1]) / (2 * eps), eps
            say(f"eps {eps:g}: a perturbed run leaves the branch")
        return None, None

    def check(name, ad, g, eps):
        noise = 4.0 * float(np.spacing(abs(J0))) / (2.0 * eps)
        e64 = abs(ad[DSS_FP64] - g)
        emx = abs(ad[DSS_MIXED] - g)
        say(f"{name}: oracle FD {g:.10e} (eps {eps:g}, resolution {noise:.1e})  FP64 {ad[DSS_FP64]:.10e} "
            f"(rel {e64 / abs(g):.2e})  mixed {ad[DSS_MIXED]:.10e} (rel {emx / abs(g):.2e})")
        assert e64 <= 1e-5 * abs(g) + noise, (name, e64)
        assert emx <= 1e-4 * abs(g) + noise, (name, emx)

    for name, key in (("mu", "dmu"), ("F_ER", "dF_ER")):
        g, eps = central(lambda e: (dict(p, **{name: p[name] + e}), w.x))
        assert g is not None, name
        check("dJ/d" + name, {k: v[key] for k, v in res.items()}, g, eps)
    g, eps = central(lambda e: (dict(p, F_ER=p["F_ER"] + e), w.x), steps=(1e-4, 2.5e-5))
    assert g is not None
    check("dJ/dF_ER", {k: v["dF_ER"] for k, v in res.items()}, g, eps)
    rng = np.random.default_rng(41)
    L = np.array(p["L"])
    checked = 0
    for d in range(8):
        v = np.zeros_like(w.x)
        moved = rng.choice(len(w.rad), 40, replace=False)
        v[moved] = rng.normal(size=(40, 3))
        v[np.any((w.x < 1e-4) | (w.x > L - 1e-4), axis=1)] = 0.0
        g, eps = central(lambda e: (p, w.x + e * v))
        if g is None:
            say(f"x0 direction {d}: leaves the branch; another 40 particles")
            continue
        check(f"dJ/dx0 . v (direction {d})", {k: float(np.sum(r["dx"] * v)) for k, r in res.items()}, g, eps)
        checked += 1
        break
    assert checked == 1
