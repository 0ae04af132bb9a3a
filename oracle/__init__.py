"""FP64 CPU oracle for the dense-suspension time step (arXiv 2108.01013).

TEST INFRASTRUCTURE ONLY: this package may be imported by ``tests/``, by the
smoke check in ``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``;
nothing in the product package imports it.  It shares no code with the HIP
library.  The arithmetic lives in ``dss_oracle.c`` (plain C, FP64, compiled with
gcc, no FMA contraction); this module only marshals numpy arrays and composes the
step in the order of the paper's modified velocity-Verlet scheme (Sec. 2.1):

    drift + half kick  ->  Lees-Edwards wrap (eq. le)  ->  pair set  ->
    forces/torques/stress at (x^{n+1}, u^{n+1/2})  ->  finishing kick.

Every function cites the passage it follows in the C source.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dss_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libdss_oracle.so")

PAIR_OUT = 69

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int32_p = ctypes.POINTER(ctypes.c_int32)
_c_int64_p = ctypes.POINTER(ctypes.c_int64)


def build() -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3)] + [(n, ctypes.c_double) for n in (
        "shear_rate", "eta0", "rho", "kn", "kt", "gamma_n", "mu", "F_ER", "lambda_D", "a0",
        "hamaker", "eps_vdw", "eps_lub", "cutoff_factor", "dt", "ec_ranges", "kr", "mu_r", "wave_amp",
        "wave_n")]


# optional parameters and their defaults (R18: electro-chemical forces over their own ranges;
# R19: rolling resistance, off at k_r = 0; R20: wavy shear, off at wave_amp = 0)
_OPTIONAL = {"ec_ranges": 0.0, "kr": 0.0, "mu_r": 0.0, "wave_amp": 0.0, "wave_n": 0.0}


PARAM_NAMES = [f[0] for f in _Params._fields_]

_lib = None


def lib():
    """Load the compiled oracle, building it first if it is missing or stale."""
    global _lib
    if _lib is not None:
        return _lib
    if (not os.path.exists(_LIB_PATH)) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    L = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER(_Params)
    sig = {
        "orc_particle_mass": (ctypes.c_double, [P, ctypes.c_double]),
        "orc_particle_inertia": (ctypes.c_double, [P, ctypes.c_double]),
        "orc_history_capacity": (ctypes.c_int, [ctypes.c_double, ctypes.c_double]),
        "orc_le_offset": (ctypes.c_double, [P, ctypes.c_int64]),
        "orc_min_image": (None, [P, ctypes.c_double, _c_double_p, _c_double_p, _c_double_p]),
        "orc_pairs_brute": (ctypes.c_int64, [P, ctypes.c_int64, _c_double_p, _c_double_p, ctypes.c_double,
                                             ctypes.c_int64, _c_int32_p]),
        "orc_pairs_cells": (ctypes.c_int64, [P, ctypes.c_int64, _c_double_p, _c_double_p, ctypes.c_double,
                                             ctypes.c_int64, _c_int32_p]),
        "orc_cell_dims": (None, [P, ctypes.c_double, _c_int32_p]),
        "orc_cell_of": (ctypes.c_int32, [P, _c_int32_p, _c_double_p]),
        "orc_cell_sort": (None, [P, ctypes.c_int64, _c_double_p, _c_int32_p, _c_int32_p, _c_int32_p]),
        "orc_lub_matrix": (None, [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _c_double_p,
                                  _c_double_p]),
        "orc_lub_strain_terms": (None, [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _c_double_p,
                                        ctypes.c_double, ctypes.c_double, _c_double_p]),
        "orc_pair_eval": (None, [P, ctypes.c_double, ctypes.c_double, _c_double_p, ctypes.c_double, ctypes.c_double,
                                 _c_double_p, _c_double_p, _c_double_p, _c_double_p, _c_double_p, _c_double_p,
                                 _c_double_p]),
        "orc_forces_ex": (ctypes.c_int64, [P, ctypes.c_int64, _c_double_p, _c_double_p, _c_double_p, _c_double_p,
                                           ctypes.c_int64, ctypes.c_int, ctypes.c_int64, _c_int32_p, _c_double_p,
                                           _c_double_p, ctypes.c_int64, _c_int32_p, _c_double_p, _c_double_p,
                                           _c_int32_p, _c_int64_p, _c_double_p, _c_double_p, _c_double_p]),
        "orc_kick_drift": (None, [P, ctypes.c_int64, ctypes.c_int64, _c_double_p, _c_double_p, _c_double_p,
                                  _c_double_p, _c_double_p, _c_double_p, _c_double_p]),
        "orc_finish": (None, [P, ctypes.c_int64, _c_double_p, _c_double_p, _c_double_p, _c_double_p,
                              _c_double_p, _c_double_p, _c_double_p]),
        "orc_accelerations": (None, [P, ctypes.c_int64, _c_double_p, _c_double_p, _c_double_p, _c_double_p,
                                     _c_double_p]),
        "orc_num_threads": (ctypes.c_int, []),
        "orc_set_num_threads": (None, [ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _params(p: dict) -> _Params:
    s = _Params()
    L = p["L"]
    s.L[0], s.L[1], s.L[2] = float(L[0]), float(L[1]), float(L[2])
    for n in PARAM_NAMES[1:]:
        setattr(s, n, float(p[n]) if n in p else _OPTIONAL[n])
    return s


def _d(a):
    return a.ctypes.data_as(_c_double_p)


def _i32(a):
    return a.ctypes.data_as(_c_int32_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ----------------------------------------------------------------------------------------------
# elementary pieces
# ----------------------------------------------------------------------------------------------
def particle_mass(p, a):
    return lib().orc_particle_mass(ctypes.byref(_params(p)), float(a))


def particle_inertia(p, a):
    return lib().orc_particle_inertia(ctypes.byref(_params(p)), float(a))


def history_capacity(a: float, a_min: float) -> int:
    """Row capacity M of the reduced history matrix (Sec. 2.1, memory paragraph)."""
    return int(lib().orc_history_capacity(float(a), float(a_min)))


def le_offset(p, step: int) -> float:
    """Lees-Edwards offset delta = fmod(gdot L_y t, L_x) at t = step * dt (eq. le)."""
    return lib().orc_le_offset(ctypes.byref(_params(p)), int(step))


def min_image(p, delta, xa, xb):
    r = np.zeros(3)
    lib().orc_min_image(ctypes.byref(_params(p)), float(delta), _d(_f64(xa)), _d(_f64(xb)), _d(r))
    return r


def pairs_brute(p, x, rad, delta) -> np.ndarray:
    """All listed pairs (a < b, |r| < c (a_a + a_b)) by the O(N^2) check; sorted (N_p, 2) int32."""
    x = _f64(x, (-1, 3))
    rad = _f64(rad)
    N = len(rad)
    cap = 16 * N + 16
    while True:
        out = np.zeros((cap, 2), np.int32)
        n = lib().orc_pairs_brute(ctypes.byref(_params(p)), N, _d(x), _d(rad), float(delta), cap, _i32(out))
        if n <= cap:
            return out[:n].copy()
        cap = int(n)


def pairs_cells(p, x, rad, delta) -> np.ndarray:
    """Listed pairs through the cell list (OpenMP); same output as pairs_brute."""
    x = _f64(x, (-1, 3))
    rad = _f64(rad)
    N = len(rad)
    cap = 16 * N + 16
    while True:
        out = np.zeros((cap, 2), np.int32)
        n = lib().orc_pairs_cells(ctypes.byref(_params(p)), N, _d(x), _d(rad), float(delta), cap, _i32(out))
        if n <= cap:
            return out[:n].copy()
        cap = int(n)


def cell_dims(p, a_max) -> np.ndarray:
    n = np.zeros(3, np.int32)
    lib().orc_cell_dims(ctypes.byref(_params(p)), float(a_max), _i32(n))
    return n


def cell_sort(p, x, dims):
    """Counting sort into the cell lattice: (cell_start[n_cells+1], order[N]) with ids ascending per cell."""
    x = _f64(x, (-1, 3))
    dims = np.ascontiguousarray(dims, np.int32)
    N = x.shape[0]
    ncell = int(dims[0]) * int(dims[1]) * int(dims[2])
    cs = np.zeros(ncell + 1, np.int32)
    order = np.zeros(N, np.int32)
    lib().orc_cell_sort(ctypes.byref(_params(p)), N, _d(x), _i32(dims), _i32(cs), _i32(order))
    return cs, order


def cell_of(p, dims, x) -> np.ndarray:
    x = _f64(x, (-1, 3))
    dims = np.ascontiguousarray(dims, np.int32)
    P = _params(p)
    return np.array([lib().orc_cell_of(ctypes.byref(P), _i32(dims), _d(np.ascontiguousarray(xi)))
                     for xi in x], np.int32)


def lub_matrix(p, ai, aj, h, n) -> np.ndarray:
    """The 12x12 lubrication resistance of eq. (rlu) (prefactor 6 pi eta0 included)."""
    R = np.zeros((12, 12))
    lib().orc_lub_matrix(ctypes.byref(_params(p)), float(ai), float(aj), float(h), _d(_f64(n)), _d(R))
    return R


def lub_strain_terms(p, ai, aj, h, n, yi=0.0, yj=0.0) -> np.ndarray:
    """The 12-vector (F_i, F_j, T_i, T_j) of eq. (rlu1) applied to (n, n, n_perp_i, n_perp_j),
    with the ambient strain of each column taken at that particle's height."""
    out = np.zeros(12)
    lib().orc_lub_strain_terms(ctypes.byref(_params(p)), float(ai), float(aj), float(h), _d(_f64(n)), float(yi),
                               float(yj), _d(out))
    return out


def pair_eval(p, ai, aj, r, upi, upj, wi, wj, xi_old=(0.0, 0.0, 0.0), xr_old=(0.0, 0.0, 0.0), yi=0.0,
              yj=0.0) -> dict:
    """One listed pair; velocities u' are fluctuations u - U_inf(x), w raw angular velocities;
    xi_old, xr_old: stored tangential and rolling stretches; yi, yj: the wrapped heights of the
    two particles (the ambient rotation and strain depend on them in the wavy shear)."""
    out = np.zeros(PAIR_OUT)
    lib().orc_pair_eval(ctypes.byref(_params(p)), float(ai), float(aj), _d(_f64(r)), float(yi), float(yj),
                        _d(_f64(upi)), _d(_f64(upj)), _d(_f64(wi)), _d(_f64(wj)), _d(_f64(xi_old)),
                        _d(_f64(xr_old)), _d(out))
    return {
        "FL_i": out[0:3], "FL_j": out[3:6], "TL_i": out[6:9], "TL_j": out[9:12],
        "FC_i": out[12:15], "FC_j": out[15:18], "TC_i": out[18:21], "TC_j": out[21:24],
        "FE_i": out[24:27], "FE_j": out[27:30],
        "SL": out[30:39].reshape(3, 3), "SC": out[39:48].reshape(3, 3), "SE": out[48:57].reshape(3, 3),
        "xi": out[57:60], "contact": bool(out[60] != 0.0), "xr": out[61:64], "TR_i": out[64:67],
        "capped": bool(out[67] != 0.0), "rcapped": bool(out[68] != 0.0),
    }


# ----------------------------------------------------------------------------------------------
# forces and the time step
# ----------------------------------------------------------------------------------------------
@dataclass
class History:
    """Map {(a, b), a < b} -> xi (tangential stretch oriented for (a, b)) and xr (rolling
    stretch, the same from either side; zeros without rolling resistance), sorted by (a, b).
    capped: per entry, bit 0 set when the Coulomb cap of eq. (csi) limited xi at the evaluation
    that wrote it (the contact slides), bit 1 when the rolling limit limited xr (None when not
    recorded, e.g. a history built from the GPU's export)."""
    pairs: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    xi: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    xr: np.ndarray | None = None
    capped: np.ndarray | None = None

    def rolling(self):
        return np.zeros_like(self.xi) if self.xr is None else self.xr

    def as_dict(self):
        return {(int(a), int(b)): self.xi[k] for k, (a, b) in enumerate(self.pairs)}


def forces(p, x, u, w, rad, step, history: History | None = None, use_cells=False):
    """Forces, torques, bulk stress and the new contact history at one state (eqs. NErhs, stress).

    Returns (F, T, Sigma(3x3), History_new, n_pairs)."""
    x = _f64(x, (-1, 3))
    u = _f64(u, (-1, 3))
    w = _f64(w, (-1, 3))
    rad = _f64(rad)
    N = len(rad)
    history = history or History()
    hp = np.ascontiguousarray(history.pairs, np.int32).reshape(-1, 2)
    hx = _f64(history.xi, (-1, 3))
    hr = _f64(history.rolling(), (-1, 3))
    hcap = max(16, 8 * N)
    F = np.zeros((N, 3))
    T = np.zeros((N, 3))
    S = np.zeros(9)
    while True:
        hp_new = np.zeros((hcap, 2), np.int32)
        hx_new = np.zeros((hcap, 3))
        hr_new = np.zeros((hcap, 3))
        hc_new = np.zeros(hcap, np.int32)
        nh = ctypes.c_int64(0)
        np_ = lib().orc_forces_ex(ctypes.byref(_params(p)), N, _d(x), _d(u), _d(w), _d(rad), int(step),
                                  int(bool(use_cells)), len(hp), _i32(hp), _d(hx), _d(hr), hcap, _i32(hp_new),
                                  _d(hx_new), _d(hr_new), _i32(hc_new), ctypes.byref(nh), _d(F), _d(T), _d(S))
        if np_ >= 0:
            break
        hcap = int(nh.value)
    k = int(nh.value)
    return F, T, S.reshape(3, 3), History(hp_new[:k].copy(), hx_new[:k].copy(), hr_new[:k].copy(),
                                          hc_new[:k].copy()), int(np_)


@dataclass
class State:
    """Oracle state at time index ``step``: x^n, u^n, w^n, alpha^n, alpha_w^n and the history H^n."""
    x: np.ndarray
    u: np.ndarray
    w: np.ndarray
    alpha: np.ndarray
    alpha_w: np.ndarray
    rad: np.ndarray
    step: int
    history: History

    def copy(self):
        return State(self.x.copy(), self.u.copy(), self.w.copy(), self.alpha.copy(), self.alpha_w.copy(),
                     self.rad.copy(), self.step, History(self.history.pairs.copy(), self.history.xi.copy(),
                                                         self.history.rolling().copy(),
                                                         None if self.history.capped is None
                                                         else self.history.capped.copy()))


def _wave(p):
    """(W, k) of the wavy shear, eq. (uinf), k = 2 pi n / L_y; W = 0 for the simple shear."""
    return float(p.get("wave_amp", 0.0)), 2.0 * math.pi * float(p.get("wave_n", 0.0)) / p["L"][1]


def ambient_velocity(p, x):
    """U_inf(x) = (gdot y + W sin(k y), 0, 0): the simple shear of Sec. 2 with the wave of eq. (uinf)."""
    x = _f64(x, (-1, 3))
    U = np.zeros_like(x)
    U[:, 0] = p["shear_rate"] * x[:, 1]
    W, k = _wave(p)
    if W != 0.0:
        U[:, 0] += W * np.sin(k * x[:, 1])
    return U


def ambient_rotation(p, N, x=None):
    """Omega_inf = (0, 0, -(gdot + W k cos(k y)) / 2) at each particle (x needed for the wave)."""
    W = np.zeros((N, 3))
    Wa, k = _wave(p)
    if Wa != 0.0:
        W[:, 2] = -0.5 * (p["shear_rate"] + Wa * k * np.cos(k * _f64(x, (-1, 3))[:, 1]))
    else:
        W[:, 2] = -0.5 * p["shear_rate"]
    return W


def accelerations(p, rad, F, T):
    rad = _f64(rad)
    N = len(rad)
    a = np.zeros((N, 3))
    aw = np.zeros((N, 3))
    lib().orc_accelerations(ctypes.byref(_params(p)), N, _d(rad), _d(_f64(F, (-1, 3))), _d(_f64(T, (-1, 3))),
                            _d(a), _d(aw))
    return a, aw


def init_state(p, x, rad, u=None, w=None, use_cells=False):
    """Initial state: u^0 = U_inf(x^0), w^0 = Omega_inf unless given, alpha^0 = F(x^0, u^0)/m.

    The evaluation at t = 0 only defines alpha^0; the contact history H^0 is empty, so every
    tangential spring starts from xi(t0) = 0 at the first step (eq. csi)."""
    x = _f64(x, (-1, 3)).copy()
    rad = _f64(rad).copy()
    u = ambient_velocity(p, x) if u is None else _f64(u, (-1, 3)).copy()
    w = ambient_rotation(p, len(rad), x) if w is None else _f64(w, (-1, 3)).copy()
    F, T, S, H, npairs = forces(p, x, u, w, rad, 0, None, use_cells)
    a, aw = accelerations(p, rad, F, T)
    return State(x, u, w, a, aw, rad, 0, History()), F, T, S


def kick_drift(p, st: State):
    """Drift + half kick + Lees-Edwards wrap at t_{n+1}; returns (x^{n+1}, u^n shifted, w^n, u^{n+1/2}, w^{n+1/2})."""
    x = st.x.copy()
    u = st.u.copy()
    w = st.w.copy()
    uh = np.zeros_like(u)
    wh = np.zeros_like(w)
    lib().orc_kick_drift(ctypes.byref(_params(p)), len(st.rad), st.step + 1, _d(x), _d(u), _d(w), _d(st.alpha),
                         _d(st.alpha_w), _d(uh), _d(wh))
    return x, u, w, uh, wh


def finish(p, rad, F, T, u, w, alpha, alpha_w):
    """u^{n+1} = u^n + dt/2 (alpha^n + alpha^{n+1}); returns (u, w, alpha, alpha_w) at n+1."""
    u = _f64(u, (-1, 3)).copy()
    w = _f64(w, (-1, 3)).copy()
    a = _f64(alpha, (-1, 3)).copy()
    aw = _f64(alpha_w, (-1, 3)).copy()
    lib().orc_finish(ctypes.byref(_params(p)), len(rad), _d(_f64(rad)), _d(_f64(F, (-1, 3))), _d(_f64(T, (-1, 3))),
                     _d(u), _d(w), _d(a), _d(aw))
    return u, w, a, aw


def step(p, st: State, use_cells=False):
    """One modified velocity-Verlet step (Sec. 2.1).  Returns (State^{n+1}, F, T, Sigma, n_pairs, (uh, wh))."""
    x, u, w, uh, wh = kick_drift(p, st)
    F, T, S, H, npairs = forces(p, x, uh, wh, st.rad, st.step + 1, st.history, use_cells)
    u, w, a, aw = finish(p, st.rad, F, T, u, w, st.alpha, st.alpha_w)
    return State(x, u, w, a, aw, st.rad.copy(), st.step + 1, H), F, T, S, npairs, (uh, wh)


def rheology(Sigma, p):
    """sigma = S_12, N1 = S_11 - S_22, N2 = S_22 - S_33, Pi = -Tr S / 3, eta_r = sigma/(eta0 gdot) (Sec. 2)."""
    S = np.asarray(Sigma).reshape(3, 3)
    sig = S[0, 1]
    out = {"sigma": sig, "N1": S[0, 0] - S[1, 1], "N2": S[1, 1] - S[2, 2], "Pi": -np.trace(S) / 3.0}
    g = p["shear_rate"] * p["eta0"]
    out["eta_r"] = sig / g if g != 0 else float("nan")
    return out


def stress_objective(p, x0, rad, u0, w0, n_steps: int, stress_every: int, weight, use_cells=False):
    """J = sum_ab weight_ab mean_samples(Sigma_ab) over a run of n_steps steps from (x0, u0, w0)
    with an empty initial history, Sigma sampled at the time indices that are multiples of
    stress_every (eq. stress).  Also returns the run's branch record per step (the number of
    listed pairs, the contact pairs, and each contact's stick/slip state: whether the Coulomb
    cap, and with rolling resistance the rolling limit, bound at that step), so that a finite
    difference of J can be checked to stay on one branch: J is smooth in the inputs while none
    of these changes.  The adjoint's reference is the central finite difference of this
    function."""
    st, F, T, S = init_state(p, x0, rad, u0, w0, use_cells)
    W = np.asarray(weight, dtype=np.float64).reshape(3, 3)
    samples, branch = [], []
    for n in range(1, n_steps + 1):
        st, F, T, S, npairs, _ = step(p, st, use_cells)
        branch.append((npairs, st.history.pairs.tobytes(), st.history.capped.tobytes()))
        if n % stress_every == 0:
            samples.append(np.asarray(S).reshape(3, 3))
    return float(np.sum(W * np.mean(samples, axis=0))), branch


# ----------------------------------------------------------------------------------------------
# Observables of Sec. 3, written out from their definitions (plain numpy / Python)
# ----------------------------------------------------------------------------------------------
def shear_diffusivity(p, y0_unwrapped, y_unwrapped, elapsed):
    """Eq. (diffY): D_y = <[y(t) - y(t0)]^2> / (2 (t - t0) a0^2 gdot), average over particles;
    y unwrapped across the sheared y faces (gdot taken as 1 when it is 0)."""
    dy = np.asarray(y_unwrapped, np.float64) - np.asarray(y0_unwrapped, np.float64)
    gd = p["shear_rate"] if p["shear_rate"] != 0.0 else 1.0
    return float(np.mean(dy * dy) / (2.0 * elapsed * p["a0"] ** 2 * gd)) if elapsed > 0 else 0.0


def velocity_autocorrelation(v0, v):
    """Eq. (corrV): C_v = <v'(t) v'(t0)> / <v'(t)^2>, v' the shear-wise velocity fluctuation."""
    v0 = np.asarray(v0, np.float64)
    v = np.asarray(v, np.float64)
    return float(np.sum(v * v0) / np.sum(v * v))


def phi_profile(p, y, rad, nbins, a_split):
    """Local volume fraction along y (Fig. localPhi): for every slab [k, k+1) L_y/nbins of the
    periodic y axis, the volume of each sphere inside it, pi [a^2 z - z^3/3] between the slab
    faces clipped to [-a, a] (z measured from the centre), over the slab volume; row 0 for
    radii <= a_split, row 1 for larger ones."""
    L = p["L"]
    dy = L[1] / nbins
    out = np.zeros((2, nbins))
    for yc, a in zip(np.asarray(y, np.float64), np.asarray(rad, np.float64)):
        g = 1 if a > a_split else 0
        for b in range(int(math.floor((yc - a) / dy)), int(math.floor((yc + a) / dy)) + 1):
            lo = max(b * dy - yc, -a)
            hi = min((b + 1) * dy - yc, a)
            if hi > lo:
                out[g, b % nbins] += math.pi * ((a * a * hi - hi ** 3 / 3.0) - (a * a * lo - lo ** 3 / 3.0))
    return out / (L[0] * L[2] * dy)


def contact_clusters(N, pairs, cap=None):
    """Clusters of contacting particles (Fig. histo): connected components of the graph whose
    edges are the contact pairs, by breadth-first search; returns the histogram h[s - 1] =
    number of clusters of s particles (sizes >= cap in the last entry)."""
    cap = cap or N
    adj = [[] for _ in range(N)]
    for a, b in np.asarray(pairs, np.int64).reshape(-1, 2):
        adj[a].append(b)
        adj[b].append(a)
    seen = np.zeros(N, bool)
    hist = np.zeros(cap, np.int64)
    for s in range(N):
        if seen[s]:
            continue
        seen[s] = True
        queue, size = [s], 0
        while queue:
            v = queue.pop()
            size += 1
            for w in adj[v]:
                if not seen[w]:
                    seen[w] = True
                    queue.append(w)
        hist[min(size, cap) - 1] += 1
    return hist
