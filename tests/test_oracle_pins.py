"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: a textbook closed form,
an exact invariant of the paper's formulas, a discrete closed form of the time scheme,
brute force, or a value derived by hand from the paper's definitions.  A dropped term, a
wrong sign, index or transposed operand anywhere in the pair physics breaks at least one.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2108_01013_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def params(L=30.0, **over):
    return synth.default_params([L, L, L], **over)


def rel(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


# ---------------------------------------------------------------------------------------------
# P14: history capacity (Sec. 2.1 memory paragraph), hand-evaluated values
# ---------------------------------------------------------------------------------------------
def test_history_capacity_golden():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "history_capacity.txt")) if l.strip()
            and not l.startswith("#")]
    assert rows
    for a_max, a_min, M in rows:
        assert oracle.history_capacity(float(a_max), float(a_min)) == int(M)


# ---------------------------------------------------------------------------------------------
# P3: Reynolds squeeze flow between two spheres (textbook lubrication limit), reading R1
#   F = 6 pi eta0 (a_i a_j / (a_i + a_j))^2 v / h, with h regularised to h + eps (a_i + a_j) / 2
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("ai,aj", [(1.0, 1.0), (1.0, 1.4), (1.4, 1.0), (1.0, 3.0), (2.5, 1.0)])
@pytest.mark.parametrize("h", [0.0, 0.01, 0.07])
def test_reynolds_squeeze(ai, aj, h):
    p = params(shear_rate=0.0, eta0=1.7)
    n = unit([0.3, -0.5, 0.8])
    r = (ai + aj + h) * n
    v = 0.37
    out = oracle.pair_eval(p, ai, aj, r, np.zeros(3), -v * n, np.zeros(3), np.zeros(3))
    astar = ai * aj / (ai + aj)
    heff = h + p["eps_lub"] * (ai + aj) / 2.0
    expect = -6.0 * math.pi * p["eta0"] * astar ** 2 * v / heff * n   # pushes i away from j
    assert rel(out["FL_i"], expect) < 1e-12
    assert rel(out["FL_j"], -expect) < 1e-12
    assert np.max(np.abs(out["TL_i"])) < 1e-12 * np.linalg.norm(expect)
    assert np.max(np.abs(out["TL_j"])) < 1e-12 * np.linalg.norm(expect)


# ---------------------------------------------------------------------------------------------
# P4: action-reaction of every pair force (each row of the resistance matrices is evaluated
# independently, so F_j = -F_i is a property of the printed coefficient table)
# ---------------------------------------------------------------------------------------------
def test_pair_action_reaction_random():
    rng = np.random.default_rng(11)
    p = params(shear_rate=0.8, hamaker=0.3)
    for _ in range(200):
        ai, aj = rng.uniform(1.0, 3.0, 2)
        n = unit(rng.normal(size=3))
        h = rng.uniform(-0.02, 0.2) * (ai + aj)
        r = (ai + aj + h) * n
        out = oracle.pair_eval(p, ai, aj, r, rng.normal(size=3), rng.normal(size=3), rng.normal(size=3),
                               rng.normal(size=3), rng.normal(size=3) * 1e-4)
        for key in ("FL", "FC", "FE"):
            scale = np.linalg.norm(out[key + "_i"]) + 1e-300
            assert np.max(np.abs(out[key + "_i"] + out[key + "_j"])) <= 1e-12 * scale


def test_total_pair_force_vanishes():
    w = synth.config_small()
    p = w.params
    st, F, T, S = oracle.init_state(p, w.x, w.rad)
    # remove the Stokes drag: what remains is a sum of equal and opposite pair forces
    U = oracle.ambient_velocity(p, st.x)
    stokes = -6.0 * math.pi * p["eta0"] * w.rad[:, None] * (st.u - U)
    pair_total = (F - stokes).sum(axis=0)
    assert np.max(np.abs(pair_total)) <= 1e-12 * np.abs(F - stokes).sum()


# ---------------------------------------------------------------------------------------------
# Angular momentum of a touching pair: T_i + T_j + r x F_j = 0 for any motion (lubrication).
# Holds at |r| = a_i + a_j for the printed Y^A, Y^B, Y^C, Y^G, Y^H with readings R2-R6.
# ---------------------------------------------------------------------------------------------
def test_lubrication_angular_momentum_at_contact():
    rng = np.random.default_rng(5)
    p = params(shear_rate=1.3)
    for _ in range(100):
        ai, aj = rng.uniform(1.0, 4.0, 2)
        n = unit(rng.normal(size=3))
        r = (ai + aj) * n
        out = oracle.pair_eval(p, ai, aj, r, rng.normal(size=3), rng.normal(size=3), rng.normal(size=3),
                               rng.normal(size=3))
        L = out["TL_i"] + out["TL_j"] + np.cross(r, out["FL_j"])
        scale = np.linalg.norm(out["TL_i"]) + np.linalg.norm(out["TL_j"]) + np.linalg.norm(r) * np.linalg.norm(
            out["FL_j"])
        assert np.max(np.abs(L)) <= 1e-12 * scale


# ---------------------------------------------------------------------------------------------
# P5: rigid rotation of a touching pair produces no lubrication force or torque (reading R2:
# the Y^C blocks act through the tangential projector; with "n x" this fails).
# ---------------------------------------------------------------------------------------------
def test_rigid_rotation_invariance():
    rng = np.random.default_rng(7)
    p = params(shear_rate=0.0)
    for _ in range(100):
        ai, aj = rng.uniform(1.0, 4.0, 2)
        n = unit(rng.normal(size=3))
        r = (ai + aj) * n
        Om = rng.normal(size=3)
        ui = rng.normal(size=3)
        out = oracle.pair_eval(p, ai, aj, r, ui, ui + np.cross(Om, r), Om, Om)
        ref = oracle.pair_eval(p, ai, aj, r, np.zeros(3), np.cross(Om, r), np.zeros(3), np.zeros(3))
        scale = np.linalg.norm(ref["FL_i"]) + np.linalg.norm(ref["TL_i"])
        assert scale > 1e-3
        for key in ("FL_i", "FL_j", "TL_i", "TL_j"):
            assert np.max(np.abs(out[key])) <= 1e-12 * scale, key


# ---------------------------------------------------------------------------------------------
# P6: affine-strain equivalence.  Particles carried by the ambient straining flow (u' = 0,
# w' = 0, E != 0) feel the same lubrication as a pair in quiescent fluid whose relative velocity
# is E r (u'_j - u'_i = E r, w = 0, E = 0).  Pins the R'(E) assembly, readings R3-R5.
# ---------------------------------------------------------------------------------------------
def test_affine_strain_equivalence():
    rng = np.random.default_rng(9)
    gd = 0.9
    pA = params(shear_rate=gd)
    pB = params(shear_rate=0.0)
    E = np.zeros((3, 3))
    E[0, 1] = E[1, 0] = gd / 2
    W = np.array([0.0, 0.0, -gd / 2])
    for _ in range(100):
        ai, aj = rng.uniform(1.0, 4.0, 2)
        n = unit(rng.normal(size=3))
        r = (ai + aj) * n
        A = oracle.pair_eval(pA, ai, aj, r, np.zeros(3), np.zeros(3), W, W)
        B = oracle.pair_eval(pB, ai, aj, r, np.zeros(3), E @ r, np.zeros(3), np.zeros(3))
        scale = np.linalg.norm(B["FL_i"]) + np.linalg.norm(B["TL_i"]) + np.linalg.norm(B["TL_j"])
        for key in ("FL_i", "FL_j", "TL_i", "TL_j"):
            assert np.max(np.abs(A[key] - B[key])) <= 1e-12 * scale, key


def test_lubrication_matrix_symmetric_and_dissipative():
    """The printed upper triangle completed by symmetry; the dissipation V.R.V of the assembled
    matrix is non-negative at every gap (a resistance matrix cannot feed energy into the flow)."""
    rng = np.random.default_rng(3)
    p = params()
    for _ in range(50):
        ai, aj = rng.uniform(1.0, 5.0, 2)
        n = unit(rng.normal(size=3))
        h = rng.uniform(0.0, 0.1) * (ai + aj)
        R = oracle.lub_matrix(p, ai, aj, h, n)
        assert np.array_equal(R, R.T)
        ev = np.linalg.eigvalsh(R)
        assert ev.min() >= -1e-10 * ev.max()


# ---------------------------------------------------------------------------------------------
# P7: a free sphere in simple shear.  For this scheme the discrete solution from u = w = 0 is
#   w_z^n = -(gdot/2) [1 - (1 - z/2)^2 (1 - z)^(n-1)],  z = dt / tau_r,  tau_r = rho a^2 / (15 eta0)
#   u_x^n = gdot y [1 - (1 - z/2)^2 (1 - z)^(n-1)],     z = dt / tau_t,  tau_t = 2 rho a^2 / (9 eta0)
# and w_z -> -gdot/2: the sphere turns at half the shear rate.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("a", [1.0, 1.4])
def test_free_sphere_in_shear(a):
    gd = 1.0
    p = params(L=20.0, shear_rate=gd, dt=2e-3)
    x = np.array([[7.0, 8.0, 9.0]])
    rad = np.array([a])
    st, F, T, S = oracle.init_state(p, x, rad, u=np.zeros((1, 3)), w=np.zeros((1, 3)))
    zr = p["dt"] * 15.0 * p["eta0"] / (p["rho"] * a * a)
    zt = p["dt"] * 9.0 * p["eta0"] / (2.0 * p["rho"] * a * a)
    y = x[0, 1]
    for n in range(1, 400):
        st, F, T, S, npairs, _ = oracle.step(p, st)
        assert npairs == 0
        wz = -(gd / 2) * (1.0 - (1.0 - zr / 2) ** 2 * (1.0 - zr) ** (n - 1))
        ux = gd * y * (1.0 - (1.0 - zt / 2) ** 2 * (1.0 - zt) ** (n - 1))
        assert abs(st.w[0, 2] - wz) <= 1e-12 * gd
        assert abs(st.u[0, 0] - ux) <= 1e-12 * gd * y
        assert abs(st.x[0, 1] - y) == 0.0
    assert abs(st.w[0, 2] + gd / 2) < 1e-9


# ---------------------------------------------------------------------------------------------
# P8: Einstein viscosity.  No listed pairs: Sigma_xy = eta0 gdot (1 + 5 phi / 2) exactly and the
# normal stress differences and pressure vanish (eqs. stress, stresslet with S^S only).
# ---------------------------------------------------------------------------------------------
def test_einstein_limit():
    L = 40.0
    p = params(L=L, shear_rate=0.7, eta0=1.3)
    g = np.arange(4) * 10.0 + 3.0
    x = np.array([[a, b, c] for a in g for b in g for c in g])
    rad = np.where(np.arange(len(x)) % 3 == 0, 1.4, 1.0)
    st, F, T, S = oracle.init_state(p, x, rad)
    assert len(oracle.pairs_brute(p, x, rad, 0.0)) == 0
    phi = (4.0 / 3.0) * math.pi * np.sum(rad ** 3) / L ** 3
    rh = oracle.rheology(S, p)
    assert abs(S[0, 1] - p["eta0"] * p["shear_rate"] * (1 + 2.5 * phi)) < 1e-14
    assert abs(rh["N1"]) < 1e-15 and abs(rh["N2"]) < 1e-15 and abs(rh["Pi"]) < 1e-15
    assert np.max(np.abs(F)) < 1e-12 and np.max(np.abs(T)) < 1e-12


# ---------------------------------------------------------------------------------------------
# P9: Hooke contact.  Two spheres at rest pressed by delta: F = k_n delta along the line of
# centres and the virial stress Sigma = -(|r| k_n delta / V) n n (eq. stress, reading R8/R9).
# ---------------------------------------------------------------------------------------------
def test_hooke_two_spheres():
    L = 20.0
    p = params(L=L, shear_rate=0.0, F_ER=0.0)
    ai, aj, delta = 1.0, 1.4, 3e-3
    n = unit([1.0, 2.0, -0.5])
    xi = np.array([8.0, 9.0, 10.0])
    r = (ai + aj - delta) * n
    x = np.array([xi, xi + r])
    rad = np.array([ai, aj])
    F, T, S, H, npairs = oracle.forces(p, x, np.zeros((2, 3)), np.zeros((2, 3)), rad, 0)
    assert npairs == 1 and len(H.pairs) == 1
    assert list(H.capped) == [0]                       # a spring at rest sticks
    assert rel(F[0], -p["kn"] * delta * n) < 1e-9
    assert rel(F[1], p["kn"] * delta * n) < 1e-9
    expect = -(np.linalg.norm(r) * p["kn"] * delta / L ** 3) * np.outer(n, n)
    assert rel(S, expect) < 1e-9
    assert oracle.rheology(S, p)["Pi"] > 0.0


# ---------------------------------------------------------------------------------------------
# P10: Coulomb sliding (eq. csi, reading R11).  Fixed overlap, constant tangential slip v:
# xi_k = min(k v dt, mu k_n delta / k_t) along the slip; F_tan = k_t xi; T_i = a_i n x F_tan,
# T_j = (a_j / a_i) T_i.  Rolling without slip leaves xi = 0.
# ---------------------------------------------------------------------------------------------
def test_coulomb_sliding_sequence():
    p = params(shear_rate=0.0, F_ER=0.0, dt=1e-4, mu=0.5)
    ai, aj, delta = 1.0, 1.4, 2e-3
    n = np.array([1.0, 0.0, 0.0])
    r = (ai + aj - delta) * n
    v = 3.0
    xi = np.zeros(3)
    cap = p["mu"] * p["kn"] * delta / p["kt"]
    capped_seen = False
    for k in range(1, 40):
        out = oracle.pair_eval(p, ai, aj, r, np.zeros(3), np.array([0.0, v, 0.0]), np.zeros(3), np.zeros(3), xi)
        xi = out["xi"]
        expect = min(k * v * p["dt"], cap)
        capped_seen |= k * v * p["dt"] > cap
        assert out["contact"]
        assert out["capped"] == (k * v * p["dt"] >= cap) and not out["rcapped"]   # the slip flag
        assert abs(xi[1] - expect) <= 1e-12 * cap and xi[0] == 0.0 and xi[2] == 0.0
        Ft = p["kt"] * xi
        assert rel(out["FC_i"], -p["kn"] * delta * n + Ft) < 1e-12
        assert rel(out["TC_i"], ai * np.cross(n, Ft)) < 1e-12
        assert rel(out["TC_j"], aj * np.cross(n, Ft)) < 1e-12
    assert capped_seen
    # rolling without slip: contact points move together, the spring does not stretch
    om = v / (ai + aj)
    out = oracle.pair_eval(p, ai, aj, r, np.zeros(3), np.array([0.0, v, 0.0]), np.array([0.0, 0.0, om]),
                           np.array([0.0, 0.0, om]))
    assert np.max(np.abs(out["xi"])) < 1e-15


# ---------------------------------------------------------------------------------------------
# Electro-chemical forces (eqs. rep, att): the two branches meet at d = 0, the repulsion decays
# by exp(-d / lambda_D), and both are central.
# ---------------------------------------------------------------------------------------------
def test_electrochemical_continuity_and_decay():
    p = params(shear_rate=0.0, eta0=0.0, hamaker=0.0, F_ER=2.0, lambda_D=0.05, a0=1.0)
    ai, aj = 1.0, 1.4
    n = unit([0.2, 0.1, 1.0])

    def FE(h, pp):
        return oracle.pair_eval(pp, ai, aj, (ai + aj + h) * n, np.zeros(3), np.zeros(3), np.zeros(3),
                                np.zeros(3))["FE_i"]

    pn = dict(p, kn=0.0, kt=0.0, gamma_n=0.0)   # isolate the electro-chemical part under overlap
    abar = 2 * ai * aj / (ai + aj)
    assert rel(FE(0.0, p), -p["F_ER"] * abar / p["a0"] * n) < 1e-15
    assert rel(FE(-1e-9, pn), FE(0.0, p)) < 1e-15
    assert abs(np.linalg.norm(FE(0.03, p)) / np.linalg.norm(FE(0.13, p)) - math.exp(0.1 / 0.05)) < 1e-12
    pa = dict(p, F_ER=0.0, hamaker=0.5, eps_vdw=0.01)
    pan = dict(pa, kn=0.0, kt=0.0, gamma_n=0.0)
    eps = 0.01 * abar
    assert rel(FE(0.0, pa), 0.5 * abar / (12 * eps ** 2) * n) < 1e-14
    assert rel(FE(-1e-9, pan), FE(0.0, pa)) < 1e-14


# ---------------------------------------------------------------------------------------------
# P11: Lees-Edwards invariance (eq. le, reading R10).  A pair that straddles the y faces feels
# the same forces, torques and stress as the same relative configuration inside the box.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("step", [0, 1234, 98765])
def test_lees_edwards_invariance(step):
    L = 25.0
    p = params(L=L, shear_rate=1.0, dt=1e-3, hamaker=0.2)
    delta = oracle.le_offset(p, step)
    rng = np.random.default_rng(step)
    ai, aj = 1.0, 1.4
    r = unit([0.3, 1.0, 0.2]) * (ai + aj - 1e-3)
    upa, upb = rng.normal(size=3), rng.normal(size=3)
    wa, wb = rng.normal(size=3), rng.normal(size=3)
    xa_in = np.array([5.0, 0.5 * L, 5.0])
    xb_in = xa_in + r
    xa_x = np.array([5.0, L - 0.4, 5.0])
    xb_img = xa_x + r                                # above the top face
    xb_x = np.array([(xb_img[0] - delta) % L, xb_img[1] - L, xb_img[2]])
    res = []
    for xa, xb in ((xa_in, xb_in), (xa_x, xb_x)):
        x = np.array([xa, xb])
        rad = np.array([ai, aj])
        u = oracle.ambient_velocity(p, x) + np.array([upa, upb])
        w = np.array([wa, wb])
        H = oracle.History(np.array([[0, 1]], np.int32), np.array([[0.0, 1e-5, 2e-5]]))
        res.append(oracle.forces(p, x, u, w, rad, step, H))
    (F1, T1, S1, H1, n1), (F2, T2, S2, H2, n2) = res
    assert n1 == n2 == 1
    assert rel(F2, F1) < 1e-9 and rel(T2, T1) < 1e-9 and rel(S2, S1) < 1e-9
    assert rel(H2.xi, H1.xi) < 1e-9


# ---------------------------------------------------------------------------------------------
# P12: contact lifecycle through the integrator: approach -> contact (xi starts from 0) ->
# separation (entry dropped) -> re-contact (starts from 0 again).
# ---------------------------------------------------------------------------------------------
def test_contact_lifecycle():
    L = 20.0
    p = params(L=L, shear_rate=0.0, eta0=0.0, F_ER=0.0, dt=1e-4, mu=0.3)
    ai, aj = 1.0, 1.0
    x = np.array([[8.0, 10.0, 10.0], [10.05, 10.3, 10.0]])
    u = np.array([[0.5, 0.0, 0.0], [-0.5, 0.0, 0.0]])
    st, F, T, S = oracle.init_state(p, x, np.array([ai, aj]), u=u, w=np.zeros((2, 3)))
    phases = []
    first_xi = []
    for k in range(3000):
        prev = len(st.history.pairs)
        x_before, u_before, w_before, a_before = st.x.copy(), st.u.copy(), st.w.copy(), st.alpha.copy()
        aw_before = st.alpha_w.copy()
        st, F, T, S, npairs, (uh, wh) = oracle.step(p, st)
        now = len(st.history.pairs)
        if prev == 0 and now == 1:
            phases.append("contact")
            # first contact: xi = T(u_t) dt with the half-step velocities
            r = oracle.min_image(p, 0.0, st.x[0], st.x[1])
            n = r / np.linalg.norm(r)
            du = uh[1] - uh[0]
            vt = du - np.cross(ai * wh[0] + aj * wh[1], n)
            ut = vt - np.dot(vt, n) * n
            xi = ut * p["dt"]
            xi -= np.dot(xi, n) * n
            first_xi.append((st.history.xi[0].copy(), xi))
        if prev == 1 and now == 0:
            phases.append("separate")
            if phases.count("separate") == 1:
                st.u = -st.u                            # send them back towards each other
        if phases.count("separate") == 2:
            break
    assert phases == ["contact", "separate", "contact", "separate"]
    for got, expect in first_xi:
        assert rel(got, expect) < 1e-12


# ---------------------------------------------------------------------------------------------
# P13: two spheres on a linear spring (no damping, no fluid): the relative coordinate follows
# the velocity-Verlet recursion exactly, h^n = h^0 cos(n theta), cos theta = 1 - (w0 dt)^2 / 2,
# w0^2 = k_n (1/m_i + 1/m_j), while the spheres overlap.
# ---------------------------------------------------------------------------------------------
def test_harmonic_contact_verlet_dispersion():
    L = 20.0
    p = params(L=L, shear_rate=0.0, eta0=0.0, F_ER=0.0, gamma_n=0.0, dt=2e-5)
    ai, aj, h0 = 1.0, 1.4, -4e-3
    n = unit([1.0, 0.5, 0.25])
    x = np.array([[6.0, 7.0, 8.0], [6.0, 7.0, 8.0] + (ai + aj + h0) * n])
    rad = np.array([ai, aj])
    st, F, T, S = oracle.init_state(p, x, rad, u=np.zeros((2, 3)), w=np.zeros((2, 3)))
    mi, mj = oracle.particle_mass(p, ai), oracle.particle_mass(p, aj)
    w0 = math.sqrt(p["kn"] * (1 / mi + 1 / mj))
    theta = math.acos(1.0 - (w0 * p["dt"]) ** 2 / 2.0)
    nsteps = int((math.pi / 2) / theta) - 1
    assert nsteps > 20
    for k in range(1, nsteps + 1):
        st, F, T, S, npairs, _ = oracle.step(p, st)
        h = np.linalg.norm(oracle.min_image(p, 0.0, st.x[0], st.x[1])) - ai - aj
        assert abs(h - h0 * math.cos(k * theta)) <= 1e-9 * abs(h0)


# ---------------------------------------------------------------------------------------------
# P1: brute force = cell-list search, across Lees-Edwards offsets and on minimal lattices
# ---------------------------------------------------------------------------------------------
def test_cell_search_equals_brute_force():
    w = synth.config_small()
    p = w.params
    dims = oracle.cell_dims(p, w.rad.max())
    dcell = p["L"][0] / dims[0]
    for delta in (0.0, 0.5 * dcell, dcell, (dims[0] - 0.5) * dcell, 1.2345):
        b = oracle.pairs_brute(p, w.x, w.rad, delta)
        c = oracle.pairs_cells(p, w.x, w.rad, delta)
        assert len(b) > 0
        assert np.array_equal(b, c)
        assert len(np.unique(b[:, 0].astype(np.int64) * 10 ** 6 + b[:, 1])) == len(b)


def test_cell_search_minimal_lattice():
    rng = np.random.default_rng(21)
    rad = np.where(rng.random(90) < 0.3, 1.4, 1.0)
    Lx, Ly, Lz = 4.01 * 3.08, 3.01 * 3.08, 3.05 * 3.08
    p = synth.default_params([Lx, Ly, Lz])
    x = rng.uniform(0, 1, size=(90, 3)) * np.array([Lx, Ly, Lz])
    dims = oracle.cell_dims(p, rad.max())
    assert tuple(dims) == (4, 3, 3)
    for delta in (0.0, 1.0, 3.5, 7.9, 11.9):
        b = oracle.pairs_brute(p, x, rad, delta)
        c = oracle.pairs_cells(p, x, rad, delta)
        assert len(b) > 10
        assert np.array_equal(b, c)


def test_min_image_le_offset():
    L = 10.0
    p = params(L=L)
    # b just above the bottom face sees a (near the top face) through the sheared image
    delta = 2.5
    xa = np.array([1.0, 9.5, 5.0])
    xb = np.array([1.0 - delta + 0.2, 0.3, 5.1])
    r = oracle.min_image(p, delta, xa, xb)
    assert np.allclose(r, [0.2, 0.8, 0.1], atol=1e-13)
    assert oracle.le_offset(params(L=L, shear_rate=0.5, dt=1e-2), 3000) == math.fmod(0.5 * L * 30.0, L)


# ---------------------------------------------------------------------------------------------
# P2: counting sort = stable placement of ids by cell (exclusive scan of the per-cell counts)
# ---------------------------------------------------------------------------------------------
def test_counting_sort():
    w = synth.config_small()
    p = w.params
    dims = oracle.cell_dims(p, w.rad.max())
    cs, order = oracle.cell_sort(p, w.x, dims)
    cell = np.minimum((w.x / (np.array(p["L"]) / dims)).astype(np.int64), dims - 1)
    cid = (cell[:, 2] * dims[1] + cell[:, 1]) * dims[0] + cell[:, 0]
    counts = np.bincount(cid, minlength=int(np.prod(dims)))
    assert np.array_equal(cs, np.concatenate([[0], np.cumsum(counts)]))
    assert np.array_equal(order, np.argsort(cid, kind="stable"))


# ---------------------------------------------------------------------------------------------
# Integrator consistency on the full suspension: the state stays finite and the pair set,
# forces and stress are the same whether the pairs come from the cell list or brute force.
# ---------------------------------------------------------------------------------------------
def test_cells_and_brute_give_same_step():
    w = synth.config_small()
    p = w.params
    st, F, T, S = oracle.init_state(p, w.x, w.rad)
    a, *_ = oracle.step(p, st, use_cells=False)
    b, *_ = oracle.step(p, st, use_cells=True)
    assert np.array_equal(a.x, b.x)
    assert rel(b.u, a.u) < 1e-14 and np.array_equal(a.history.pairs, b.history.pairs)


# ---------------------------------------------------------------------------------------------
# The tangential spring lives in the tangent plane (eq. csi: xi = T int u_t): after a rotation of
# the line of centres the stored stretch is projected again, xi_new . n = 0.
# ---------------------------------------------------------------------------------------------
def test_tangential_spring_stays_tangent():
    rng = np.random.default_rng(17)
    p = params(shear_rate=0.5)
    for _ in range(50):
        ai, aj = rng.uniform(1.0, 2.0, 2)
        n = unit(rng.normal(size=3))
        r = (ai + aj - 1e-3) * n
        xi_old = rng.normal(size=3) * 1e-4            # has a normal component w.r.t. the new n
        out = oracle.pair_eval(p, ai, aj, r, rng.normal(size=3), rng.normal(size=3), rng.normal(size=3),
                               rng.normal(size=3), xi_old)
        assert out["contact"]
        assert abs(np.dot(out["xi"], n)) <= 1e-14 * np.linalg.norm(out["xi"])


# ---------------------------------------------------------------------------------------------
# Coulomb's law at saturation (eqs. contact0, csi): once sliding, the tangential contact force
# equals mu times the normal contact force, dashpot included; the normal part is read back from
# the returned contact force itself.
# ---------------------------------------------------------------------------------------------
def test_coulomb_law_at_saturation_with_dashpot():
    p = params(shear_rate=0.0, F_ER=0.0, gamma_n=300.0, mu=0.4)
    ai, aj, delta = 1.0, 1.4, 1e-3
    n = unit([0.5, 0.3, -0.2])
    r = (ai + aj - delta) * n
    t1 = unit(np.cross(n, [0.0, 0.0, 1.0]))
    for vn in (-2.0, 0.7):                              # approaching and separating
        du = 5.0 * t1 + vn * n
        xi_old = 1.0 * t1                               # far beyond the cap
        out = oracle.pair_eval(p, ai, aj, r, np.zeros(3), du, np.zeros(3), np.zeros(3), xi_old)
        Fc = out["FC_i"]
        Fn = np.dot(Fc, n) * n
        Ft = Fc - Fn
        assert abs(np.linalg.norm(Ft) - p["mu"] * np.linalg.norm(Fn)) <= 1e-12 * np.linalg.norm(Fn)
        assert np.dot(Ft, t1) > 0.0


# ---------------------------------------------------------------------------------------------
# Restitution of a linear spring-dashpot (eq. contact0): a head-on collision without fluid
# rebounds with e = exp(-pi zeta / sqrt(1 - zeta^2)), zeta = gamma_n / (2 sqrt(k_n m_red)).
# The scheme's O(dt) error is far below the tolerance at w0 dt = 2e-3.
# ---------------------------------------------------------------------------------------------
def test_restitution_coefficient():
    L = 20.0
    p = params(L=L, shear_rate=0.0, eta0=0.0, F_ER=0.0, gamma_n=50.0, dt=2e-6)
    ai = aj = 1.0
    v = 1.0
    x = np.array([[8.0, 10.0, 10.0], [10.0 + 2e-4, 10.0, 10.0]])
    u = np.array([[0.5 * v, 0.0, 0.0], [-0.5 * v, 0.0, 0.0]])
    st, F, T, S = oracle.init_state(p, x, np.array([ai, aj]), u=u, w=np.zeros((2, 3)))
    m = oracle.particle_mass(p, ai)
    mred = m / 2
    zeta = p["gamma_n"] / (2 * math.sqrt(p["kn"] * mred))
    e = math.exp(-math.pi * zeta / math.sqrt(1 - zeta ** 2))
    touched = False
    for _ in range(20000):
        st, *_ = oracle.step(p, st)
        if len(st.history.pairs):
            touched = True
        elif touched:
            break
    assert touched and not len(st.history.pairs)
    vrel = st.u[1, 0] - st.u[0, 0]
    assert abs(vrel / v - e) < 5e-3


# ---------------------------------------------------------------------------------------------
# Both Lees-Edwards branches of the nearest image: b above the top face and b below the bottom
# face of the box as seen from a.
# ---------------------------------------------------------------------------------------------
def test_min_image_both_faces():
    L = 10.0
    p = params(L=L)
    delta = 2.5
    xa = np.array([1.0, 0.3, 5.0])                    # a near the bottom, b near the top
    xb = np.array([(1.0 + delta - 0.2) % L, 9.5, 5.1])
    assert np.allclose(oracle.min_image(p, delta, xa, xb), [-0.2, -0.8, 0.1], atol=1e-13)
    assert np.allclose(oracle.min_image(p, delta, xb, xa), [0.2, 0.8, -0.1], atol=1e-13)


@pytest.mark.parametrize("face", ["top", "bottom"])
def test_lees_edwards_invariance_both_faces(face):
    L = 25.0
    step = 4321
    p = params(L=L, shear_rate=1.0, dt=1e-3)
    delta = oracle.le_offset(p, step)
    ai, aj = 1.0, 1.4
    sgn = 1.0 if face == "top" else -1.0
    r = unit([0.3, sgn * 1.0, 0.2]) * (ai + aj - 1e-3)
    rng = np.random.default_rng(1)
    upa, upb = rng.normal(size=3), rng.normal(size=3)
    xa_in = np.array([5.0, 0.5 * L, 5.0])
    xa_x = np.array([5.0, L - 0.4 if face == "top" else 0.4, 5.0])
    xb_img = xa_x + r
    shift = -delta if face == "top" else delta
    xb_x = np.array([(xb_img[0] + shift) % L, xb_img[1] - sgn * L, xb_img[2]])
    res = []
    for xa, xb in ((xa_in, xa_in + r), (xa_x, xb_x)):
        x = np.array([xa, xb])
        u = oracle.ambient_velocity(p, x) + np.array([upa, upb])
        res.append(oracle.forces(p, x, u, np.zeros((2, 3)), np.array([ai, aj]), step))
    assert res[0][4] == res[1][4] == 1
    for k in range(3):
        assert rel(res[1][k], res[0][k]) < 1e-9


# ---------------------------------------------------------------------------------------------
# R18: electro-chemical forces over their own ranges (Fig. elch: repulsion while the surface
# distance is below 20 lambda_D, attraction while it is below 4 a0), lubrication kept on
# |r| < c (a_i + a_j).  Closed forms of eqs. (rep) and (att) beyond the lubrication range,
# the switch-offs at the range ends, the pair set by brute force against the plain distance
# definition, and the cell search on the longer cutoff.
# ---------------------------------------------------------------------------------------------
def test_ec_ranges_closed_forms():
    ai, aj = 1.0, 1.4
    abar = 2 * ai * aj / (ai + aj)
    n = unit([0.3, -0.2, 0.9])
    up_i, up_j = np.array([0.1, -0.3, 0.2]), np.array([-0.2, 0.05, 0.4])
    wi, wj = np.array([0.3, 0.1, -0.2]), np.array([-0.1, 0.2, 0.5])

    def ev(pp, h):
        return oracle.pair_eval(pp, ai, aj, (ai + aj + h) * n, up_i, up_j, wi, wj)

    # repulsion only, beyond the lubrication range (d* = 2 h / (a_i + a_j) > 0.2)
    p = params(F_ER=2.0, lambda_D=0.05, a0=1.0, hamaker=0.0, ec_ranges=1.0)
    for h in (0.3, 0.7, 0.99):
        e = ev(p, h)
        assert np.all(e["FL_i"] == 0.0) and np.all(e["TL_i"] == 0.0) and np.all(e["TL_j"] == 0.0)
        assert np.all(e["SL"] == 0.0) and not e["contact"]
        assert rel(e["FE_i"], -2.0 * abar * math.exp(-h / 0.05) * n) < 1e-12   # h from |r| - s
        assert rel(e["SE"], np.outer((ai + aj + h) * n, e["FE_i"])) < 1e-14
    assert np.all(ev(p, 1.0 + 1e-12)["FE_i"] == 0.0)           # 20 lambda_D = 1.0
    # inside the lubrication range nothing changes against the default reading (R12)
    p0 = params(F_ER=2.0, lambda_D=0.05, a0=1.0)
    for h in (0.01, 0.2):
        e1, e0 = ev(p, h), ev(p0, h)
        for k in ("FL_i", "TL_i", "TL_j", "FE_i", "SL", "SE"):
            assert np.array_equal(e1[k], e0[k])
    # attraction only (F_ER = 0), eq. (att), up to 4 a0
    pa = params(F_ER=0.0, hamaker=0.5, eps_vdw=0.01, a0=1.0, ec_ranges=1.0)
    eps = 0.01 * abar
    for h in (0.5, 2.0, 3.9):
        e = ev(pa, h)
        assert np.all(e["FL_i"] == 0.0)
        assert rel(e["FE_i"], 0.5 * abar / (12 * (h * h + eps * eps)) * n) < 1e-14
    assert np.all(ev(pa, 4.0 + 1e-12)["FE_i"] == 0.0)


def test_ec_ranges_pair_set_and_cells():
    w = synth.config_small()
    p = dict(w.params, hamaker=0.02, ec_ranges=1.0)
    # longest range 4 a0 = 4: a pair is listed iff |r| < max(1.1 s, s + 4), s = a_i + a_j
    N = 300
    x, rad = w.x[:N], w.rad[:N]
    delta = 3.21
    b = oracle.pairs_brute(p, x, rad, delta)
    ref = []
    for i in range(N):
        for j in range(i + 1, N):
            r = oracle.min_image(p, delta, x[i], x[j])
            s = rad[i] + rad[j]
            if np.dot(r, r) < max(1.1 * s, s + 4.0) ** 2:
                ref.append((i, j))
    assert len(ref) > 10 * len(oracle.pairs_brute(w.params, x, rad, delta))
    assert np.array_equal(b, np.asarray(ref, np.int32).reshape(-1, 2))
    dims = oracle.cell_dims(p, rad.max())
    assert np.all(dims == np.floor(np.asarray(p["L"]) / ((2 * rad.max() + 4.0) * (1 + 1e-9))).astype(int))
    assert np.array_equal(oracle.pairs_cells(p, w.x, w.rad, delta), oracle.pairs_brute(p, w.x, w.rad, delta))


# ---------------------------------------------------------------------------------------------
# R19: rolling resistance (Appendix roll).  With a_i w_i + a_j w_j = 0 the contact does not
# slide, and a constant rolling velocity u_r = a_ij n x (w_i - w_j) loads the rolling spring
# linearly until the Coulomb limit mu_r |F_nor| / k_r; the torques are a_ij n x k_r xi^r on i
# and its opposite on j; no force, no stress.
# ---------------------------------------------------------------------------------------------
def test_rolling_spring_sequence():
    ai, aj = 1.0, 1.4
    aij = 2 * ai * aj / (ai + aj)
    p = params(shear_rate=0.0, eta0=0.0, F_ER=0.0, kr=0.05 * 4e5, mu_r=0.1, gamma_n=0.0)
    n = unit([0.1, 0.3, 0.95])
    h = -0.01
    r = (ai + aj + h) * n
    Om = np.cross(n, unit([1.0, -0.4, 0.2]))          # perpendicular to n
    wi, wj = Om, -(ai / aj) * Om                       # a_i w_i + a_j w_j = 0: no sliding
    ur = aij * np.cross(n, wi - wj)
    cap = p["mu_r"] * p["kn"] * abs(h) / p["kr"]
    xr = np.zeros(3)
    xi = np.zeros(3)
    saturated = False
    for k in range(1, 400):
        e = oracle.pair_eval(p, ai, aj, r, np.zeros(3), np.zeros(3), wi, wj, xi, xr)
        assert e["contact"]
        xi, xr = e["xi"], e["xr"]
        assert np.linalg.norm(xi) < 1e-13                                     # no sliding
        want = min(k * np.linalg.norm(ur) * p["dt"], cap)
        assert abs(np.linalg.norm(xr) - want) <= 1e-12 * want
        assert rel(xr, want * unit(ur)) < 1e-12
        assert rel(e["TR_i"], aij * np.cross(n, p["kr"] * xr)) < 1e-13
        assert rel(e["TC_j"], -e["TC_i"]) < 1e-12                # only the rolling torque acts
        assert rel(e["TC_i"], e["TR_i"]) < 1e-12
        assert rel(e["FC_i"], p["kn"] * h * n) < 1e-11           # no rolling force (h from |r|)
        assert e["rcapped"] == (k * np.linalg.norm(ur) * p["dt"] >= cap) and not e["capped"]
        saturated = saturated or want == cap
    assert saturated


def test_rolling_symmetry_and_switch_off():
    rng = np.random.default_rng(5)
    ai, aj = 1.0, 1.4
    pr = params(kr=0.1 * 4e5, mu_r=0.3)
    p0 = params()
    for _ in range(20):
        n = unit(rng.normal(size=3))
        r = (ai + aj - 0.02 * rng.random()) * n
        upi, upj = rng.normal(size=3), rng.normal(size=3)
        wi, wj = rng.normal(size=3), rng.normal(size=3)
        xi0 = np.cross(n, rng.normal(size=3)) * 1e-6
        xr0 = np.cross(n, rng.normal(size=3)) * 1e-6
        a = oracle.pair_eval(pr, ai, aj, r, upi, upj, wi, wj, xi0, xr0)
        b = oracle.pair_eval(pr, aj, ai, -r, upj, upi, wj, wi, -xi0, xr0)   # the same pair seen from j
        assert rel(a["xr"], b["xr"]) < 1e-12                     # the rolling stretch has no orientation
        assert rel(a["TR_i"], -b["TR_i"]) < 1e-12
        assert rel(a["TC_i"], b["TC_j"]) < 1e-12 and rel(a["TC_j"], b["TC_i"]) < 1e-12
        z = oracle.pair_eval(p0, ai, aj, r, upi, upj, wi, wj, xi0, xr0)   # k_r = 0: no rolling
        assert np.all(z["xr"] == 0.0) and np.all(z["TR_i"] == 0.0)
        for k in ("FC_i", "FC_j", "SC", "SL", "SE", "FL_i", "xi"):
            assert np.array_equal(a[k], z[k])
        assert rel(a["TC_i"] - a["TR_i"], z["TC_i"]) < 1e-12
        assert rel(a["TC_j"] + a["TR_i"], z["TC_j"]) < 1e-12


# ---------------------------------------------------------------------------------------------
# Observables (Sec. 3): the slab volumes against the spherical-cap formula V = pi h^2 (3a - h)/3
# and the sphere volume, the clusters against scipy's connected components and hand graphs,
# the diffusivity's unwrapping and the autocorrelation on hand values.
# ---------------------------------------------------------------------------------------------
def test_phi_profile_slab_volumes():
    L = 20.0
    p = params(L=L)
    nb = 10
    slab = L * L * (L / nb)
    a = 0.7
    # inside one slab: the whole sphere
    prof = oracle.phi_profile(p, [5.0], [a], nb, 1.0)
    assert abs(prof[0, 2] * slab - 4 / 3 * math.pi * a ** 3) < 1e-12 and np.count_nonzero(prof) == 1
    # a cap of height h above the face y = 4: pi h^2 (3a - h) / 3
    for h in (0.1, 0.35, 0.7, 1.1):
        yc = 4.0 - a + h
        prof = oracle.phi_profile(p, [yc], [a], nb, 1.0)
        cap = math.pi * h * h * (3 * a - h) / 3
        assert abs(prof[0, 2] * slab - cap) < 1e-12 * max(cap, 1.0)
    # across the periodic face: the two bins at the ends, summing to the sphere
    prof = oracle.phi_profile(p, [0.2], [1.4], nb, 1.0)
    assert prof[1, 9] > 0 and prof[1, 0] > 0 and np.all(prof[0] == 0)
    assert abs(prof.sum() * slab - 4 / 3 * math.pi * 1.4 ** 3) < 1e-11
    # many spheres: total over bins = total volume (global volume fraction)
    rng = np.random.default_rng(3)
    y = rng.uniform(0, L, 200)
    r = rng.uniform(1.0, 1.4, 200)
    prof = oracle.phi_profile(p, y, r, 7, 1.2)
    assert abs(prof.sum() * L ** 3 / 7 - 4 / 3 * math.pi * np.sum(r ** 3)) < 1e-9
    assert abs(prof[1].sum() * L ** 3 / 7 - 4 / 3 * math.pi * np.sum(r[r > 1.2] ** 3)) < 1e-9


def test_contact_clusters_against_library():
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    assert list(oracle.contact_clusters(5, [(0, 1), (1, 2)])) == [2, 0, 1, 0, 0]        # chain + 2 isolated
    assert list(oracle.contact_clusters(4, [(0, 1), (1, 2), (0, 2)], cap=2)) == [1, 1]  # triangle in the cap bin
    rng = np.random.default_rng(9)
    for N, E in ((50, 30), (400, 380), (1000, 200)):
        pairs = np.unique(np.sort(rng.integers(0, N, size=(E, 2)), axis=1), axis=0)
        pairs = pairs[pairs[:, 0] != pairs[:, 1]]
        g = coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(N, N))
        n, lab = connected_components(g, directed=False)
        sizes = np.bincount(np.bincount(lab), minlength=N + 1)[1:]
        assert np.array_equal(oracle.contact_clusters(N, pairs), sizes)
        assert oracle.contact_clusters(N, pairs).sum() == n


def test_diffusivity_and_autocorrelation_hand_values():
    p = params(L=10.0, shear_rate=2.0, a0=1.0)
    # particle 0 crossed the top face once (y = 9.9 -> 0.05 + L), particle 1 moved down by 0.3
    y0 = np.array([9.9, 5.0])
    y1 = np.array([0.05 + 10.0, 4.7])
    D = oracle.shear_diffusivity(p, y0, y1, 0.5)
    assert abs(D - ((0.15 ** 2 + 0.3 ** 2) / 2) / (2 * 0.5 * 2.0)) < 1e-15
    assert oracle.velocity_autocorrelation([1.0, -2.0], [0.5, -1.0]) == (0.5 + 2.0) / (0.25 + 1.0)


# ---------------------------------------------------------------------------------------------
# R20: wavy shear, eq. (uinf).  A free sphere at height y relaxes, with the discrete solution of
# P7, to the Faxen velocity u_x* = gdot y + W sin(k y) (1 - a^2 k^2 / 6) and to the local
# rotation -(gdot + W k cos(k y)) / 2; the stress of free spheres is the Faxen stresslet sum;
# each column of R'(E) takes its own particle's strain (linearity), and each column is
# force-free (action-reaction); W = 0 leaves every result unchanged.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("a,y", [(1.0, 3.3), (1.4, 14.1)])
def test_free_sphere_in_wavy_shear(a, y):
    L = 20.0
    gd, Wa, nw = 0.7, 4.0, 2.0
    p = params(L=L, shear_rate=gd, dt=2e-3, wave_amp=Wa, wave_n=nw)
    k = 2 * math.pi * nw / L
    x = np.array([[7.0, y, 9.0]])
    rad = np.array([a])
    st, F, T, S = oracle.init_state(p, x, rad, u=np.zeros((1, 3)), w=np.zeros((1, 3)))
    zr = p["dt"] * 15.0 * p["eta0"] / (p["rho"] * a * a)
    zt = p["dt"] * 9.0 * p["eta0"] / (2.0 * p["rho"] * a * a)
    ux_star = gd * y + Wa * math.sin(k * y) * (1.0 - a * a * k * k / 6.0)
    wz_star = -0.5 * (gd + Wa * k * math.cos(k * y))
    for n in range(1, 300):
        st, F, T, S, npairs, _ = oracle.step(p, st)
        assert npairs == 0
        fz = 1.0 - (1.0 - zr / 2) ** 2 * (1.0 - zr) ** (n - 1)
        ft = 1.0 - (1.0 - zt / 2) ** 2 * (1.0 - zt) ** (n - 1)
        assert abs(st.w[0, 2] - wz_star * fz) <= 1e-12 * abs(wz_star)
        assert abs(st.u[0, 0] - ux_star * ft) <= 1e-12 * abs(ux_star)
    # stress of the free sphere: eta0 gdot + (20/3 pi eta0 a^3 (E_xy(y) + a^2/10 lap E_xy)) / V
    Exy = 0.5 * (gd + Wa * k * math.cos(k * y))
    lapE = -0.5 * Wa * k ** 3 * math.cos(k * y)
    want = p["eta0"] * gd + 20.0 / 3.0 * math.pi * p["eta0"] * a ** 3 * (Exy + a * a / 10.0 * lapE) / L ** 3
    assert abs(S[0, 1] - want) < 1e-14 and abs(S[1, 0] - want) < 1e-14 and abs(S[0, 0]) < 1e-15


def test_wavy_strain_columns():
    p = params(L=20.0, shear_rate=0.5, wave_amp=3.0, wave_n=1.0)
    p0 = params(L=20.0, shear_rate=0.5)
    rng = np.random.default_rng(4)
    for _ in range(10):
        n = unit(rng.normal(size=3))
        ai, aj, h = 1.0, 1.4, 0.03 * rng.random()
        yi, yj = rng.uniform(0, 20, 2)
        sij = oracle.lub_strain_terms(p, ai, aj, h, n, yi, yj)
        sji = oracle.lub_strain_terms(p, ai, aj, h, n, yj, yi)
        sii = oracle.lub_strain_terms(p, ai, aj, h, n, yi, yi)
        sjj = oracle.lub_strain_terms(p, ai, aj, h, n, yj, yj)
        assert np.max(np.abs(sij + sji - sii - sjj)) <= 1e-12 * np.max(np.abs(sii) + np.abs(sjj))
        assert np.max(np.abs(sij[0:3] + sij[3:6])) <= 1e-12 * np.max(np.abs(sij))       # force-free
        assert not np.allclose(sij, sii)                                                  # E_j matters
        assert np.array_equal(oracle.lub_strain_terms(p0, ai, aj, h, n, yi, yj),
                              oracle.lub_strain_terms(p0, ai, aj, h, n))                 # W = 0: uniform


# ---------------------------------------------------------------------------------------------
# Magnitude of the log-singular Y coefficients (Appendix A: Y = g^Y log(1 / (d* + eps))).  A pair
# sliding past another in quiescent fluid feels only the tangential block: F_i = 6 pi eta0
# g^{Y^A_ii} ln(1/(d* + eps)) v t, F_j = -F_i.  Hand-evaluated values over sizes, size ratios and
# gaps (tests/golden/lubrication_tangential.txt); for equal spheres g = a/6, Jeffrey and Onishi's
# equal-sphere coefficient.  A base-10 logarithm, eps outside the logarithm or a wrong a_i power
# fails.  The rigid-rotation pin then ties Y^B and Y^C to this magnitude.
# ---------------------------------------------------------------------------------------------
def _rows(name):
    return [l.split() for l in open(os.path.join(GOLDEN, name)) if l.strip() and not l.startswith("#")]


def test_tangential_lubrication_golden():
    rows = _rows("lubrication_tangential.txt")
    assert len(rows) >= 6
    for ai, aj, h, eps, val in rows:
        ai, aj, h, eps, val = map(float, (ai, aj, h, eps, val))
        p = params(shear_rate=0.0, eta0=1.3, eps_lub=eps)
        n = unit([0.3, -0.5, 0.8])
        t = unit(np.cross(n, [1.0, 0.0, 0.0]))
        v = 0.29
        out = oracle.pair_eval(p, ai, aj, (ai + aj + h) * n, np.zeros(3), v * t, np.zeros(3), np.zeros(3))
        expect = 6.0 * math.pi * p["eta0"] * val * v * t
        assert rel(out["FL_i"], expect) < 1e-12, (ai, aj, h)
        assert rel(out["FL_j"], -expect) < 1e-12, (ai, aj, h)


# ---------------------------------------------------------------------------------------------
# Lubrication stresslet S^L = 1/2 [r (x) F^L_i + (r (x) F^L_i)^T] (eq. stresslet).
#  - Squeeze: with the Reynolds closed form F^L_i = -6 pi eta0 (a_i a_j/(a_i+a_j))^2 v / h_eff n,
#    S^L = |r| F n (x) n.
#  - Sliding: with the golden tangential force, S^L = |r|/2 (n (x) F_t + F_t (x) n) (symmetric).
#  - In a box: a lubricated pair carried by the ambient shear (u' = 0, w' = 0, no contact, no
#    repulsion) raises Sigma_xy above the Einstein value by exactly F_i.(E r) / (gdot V) (the
#    stress power of the pair equals the work rate of its force on the affine relative motion),
#    and that excess is positive and Sigma stays symmetric.  Dropping S^L, flipping its sign or
#    leaving it unsymmetrised fails.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("ai,aj,h", [(1.0, 1.4, 0.01), (2.5, 1.0, 0.0), (1.0, 1.0, 0.07)])
def test_lubrication_stresslet_squeeze(ai, aj, h):
    p = params(shear_rate=0.0, eta0=1.7)
    n = unit([0.3, -0.5, 0.8])
    r = (ai + aj + h) * n
    v = 0.37
    out = oracle.pair_eval(p, ai, aj, r, np.zeros(3), -v * n, np.zeros(3), np.zeros(3))
    astar = ai * aj / (ai + aj)
    heff = h + p["eps_lub"] * (ai + aj) / 2.0
    F = -6.0 * math.pi * p["eta0"] * astar ** 2 * v / heff
    assert rel(out["SL"], np.linalg.norm(r) * F * np.outer(n, n)) < 1e-12


def test_lubrication_stresslet_sliding():
    ai, aj, h, eps, val = map(float, _rows("lubrication_tangential.txt")[3])
    p = params(shear_rate=0.0, eta0=1.3, eps_lub=eps)
    n = unit([0.3, -0.5, 0.8])
    t = unit(np.cross(n, [1.0, 0.0, 0.0]))
    v = 0.29
    r = (ai + aj + h) * n
    out = oracle.pair_eval(p, ai, aj, r, np.zeros(3), v * t, np.zeros(3), np.zeros(3))
    Ft = 6.0 * math.pi * p["eta0"] * val * v * t
    expect = 0.5 * np.linalg.norm(r) * (np.outer(n, Ft) + np.outer(Ft, n))
    assert rel(out["SL"], expect) < 1e-12
    assert np.array_equal(out["SL"], out["SL"].T)


@pytest.mark.parametrize("nvec", [[1.0, 1.0, 0.0], [1.0, -1.0, 0.0], [0.3, 0.8, -0.5], [-0.7, 0.2, 0.6]])
def test_sheared_pair_stress_above_einstein(nvec):
    L = 30.0
    gd = 0.8
    p = params(L=L, shear_rate=gd, F_ER=0.0, eta0=1.1)
    ai, aj, h = 1.0, 1.4, 0.02
    n = unit(nvec)
    r = (ai + aj + h) * n
    x0 = np.array([12.0, 14.0, 15.0])
    x = np.array([x0, x0 + r])
    rad = np.array([ai, aj])
    u = oracle.ambient_velocity(p, x)
    w = oracle.ambient_rotation(p, 2, x)
    F, T, S, H, npairs = oracle.forces(p, x, u, w, rad, 0)
    assert npairs == 1 and len(H.pairs) == 0
    V = L ** 3
    phi = (4.0 / 3.0) * math.pi * np.sum(rad ** 3) / V
    einstein = p["eta0"] * gd * (1.0 + 2.5 * phi)
    E = np.zeros((3, 3))
    E[0, 1] = E[1, 0] = gd / 2.0
    excess = S[0, 1] - einstein
    power = float(F[0] @ (E @ r)) / (gd * V)
    assert excess > 0.0
    assert abs(excess - power) <= 1e-12 * abs(power)
    assert abs(S[0, 1] - S[1, 0]) <= 1e-14 * abs(S[0, 1])


# ---------------------------------------------------------------------------------------------
# Columns of R'(E) (eq. rlu1): column i takes the ambient strain at particle i, column j the
# strain at j.  In the wavy shear with no mean shear, the local strain vanishes at k y = pi/2
# (cos = 0) and is W k at y = 0, so one column at a time is switched on; each must give the
# printed coefficients of its own column (golden values of the Appendix A table,
# tests/golden/lubrication_g.txt).  A swap of the columns (F_i taking g^{X^G_ji} with the strain
# at i) fails for any alpha != 1.
# ---------------------------------------------------------------------------------------------
def _golden_g():
    from fractions import Fraction
    g = {}
    for ai, aj, name, val in _rows("lubrication_g.txt"):
        g[(float(Fraction(ai)), float(Fraction(aj)), name)] = float(Fraction(val))
    return g


@pytest.mark.parametrize("ai,aj", [(1.0, 1.4), (2.5, 3.5)])
@pytest.mark.parametrize("h", [0.0, 0.04])
@pytest.mark.parametrize("col", ["i", "j"])
def test_strain_columns_golden(ai, aj, h, col):
    L, Wa = 20.0, 3.0
    p = params(L=L, shear_rate=0.0, wave_amp=Wa, wave_n=1.0)
    k = 2.0 * math.pi / L
    g = _golden_g()
    n = unit([0.6, 0.7, -0.4])
    s = Wa * k                        # local shear rate at y = 0; zero at y = L/4
    E = np.zeros((3, 3))
    E[0, 1] = E[1, 0] = s / 2.0
    P = float(n @ E @ n)              # E : N - Tr E / 3 (traceless E)
    Qn = 2.0 * E @ n - 2.0 * P * n
    nperp = 2.0 * np.cross(n, E @ n)
    eps = p["eps_lub"]
    d = 2.0 * h / (ai + aj)
    X = 1.0 / (d + eps)
    Y = math.log(1.0 / (d + eps))
    K = 6.0 * math.pi * p["eta0"]
    if col == "i":
        yi, yj = 0.0, L / 4.0
        names = ("XG_ii", "YG_ii", "XG_ij", "YG_ij", "YH_ii", "YH_ij")
    else:
        yi, yj = L / 4.0, 0.0
        names = ("XG_ji", "YG_ji", "XG_jj", "YG_jj", "YH_ji", "YH_jj")
    c = [g[(ai, aj, nm)] for nm in names]
    want = np.concatenate([K * (c[0] * X * P * n + c[1] * Y * Qn), K * (c[2] * X * P * n + c[3] * Y * Qn),
                           K * c[4] * Y * nperp, K * c[5] * Y * nperp])
    got = oracle.lub_strain_terms(p, ai, aj, h, n, yi, yj)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
