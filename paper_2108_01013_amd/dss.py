"""Python binding of libdss (the HIP library behind include/dss.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
Arrays may be numpy arrays (host memory) or torch CUDA tensors (device memory, passed by
pointer, on the current torch stream).  There is no CPU fallback: if libdss.so is missing
or fails to load, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdss.so")

DSS_FP64 = 0
DSS_MIXED = 1
DSS_ERR_CAPACITY = 3
DSS_FLAG_RECORD_PAIRS = 1
DSS_FLAG_EC_RANGES = 2

STATUS = {0: "DSS_OK", 1: "DSS_ERR_ARG", 2: "DSS_ERR_HIP", 3: "DSS_ERR_CAPACITY", 4: "DSS_ERR_BOX",
          5: "DSS_ERR_UNSTABLE", 6: "DSS_ERR_STATE"}

EXPORTS = ["dss_create", "dss_create_batch", "dss_set_particles", "dss_set_particles_batch", "dss_set_step", "dss_build_neighbours", "dss_compute_forces", "dss_step", "dss_prepare_steps",
           "dss_read_stress", "dss_read_stress_batch", "dss_get_box_info", "dss_get_state", "dss_get_eval_velocities", "dss_get_pairs", "dss_get_cells", "dss_get_rolling_history",
           "dss_observe_start", "dss_observe", "dss_phi_profile", "dss_phi_profile_noalloc", "dss_contact_clusters",
           "dss_get_history", "dss_get_info", "dss_save_state", "dss_load_state", "dss_set_timing",
           "dss_get_timing", "dss_set_tuning", "dss_get_tuning", "dss_adjoint", "dss_last_error",
           "dss_status_string", "dss_destroy"]


class DssError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = ([("L", ctypes.c_double * 3)]
                + [(n, ctypes.c_double) for n in ("shear_rate", "eta0", "rho", "kn", "kt", "gamma_n", "mu", "F_ER",
                                                  "lambda_D", "a0", "hamaker", "eps_vdw", "eps_lub", "cutoff_factor",
                                                  "dt")]
                + [("precision", ctypes.c_int32), ("capacity", ctypes.c_int32), ("flags", ctypes.c_int32),
                   ("reserved", ctypes.c_int32), ("k_roll", ctypes.c_double), ("mu_roll", ctypes.c_double),
                   ("wave_amp", ctypes.c_double), ("wave_n", ctypes.c_double)])


class Info(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_int64), ("step", ctypes.c_int64), ("cells", ctypes.c_int32 * 3),
                ("capacity", ctypes.c_int32), ("n_pairs", ctypes.c_int64), ("n_contacts", ctypes.c_int64),
                ("max_row_fill", ctypes.c_int32), ("error_flags", ctypes.c_int32), ("le_offset", ctypes.c_double)]


class BoxInfo(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_int64), ("first_id", ctypes.c_int64), ("cells", ctypes.c_int32 * 3),
                ("first_cell", ctypes.c_int32), ("n_pairs", ctypes.c_int64), ("n_contacts", ctypes.c_int64),
                ("max_row_fill", ctypes.c_int32), ("size_classes", ctypes.c_int32), ("L", ctypes.c_double * 3),
                ("shear_rate", ctypes.c_double), ("le_offset", ctypes.c_double), ("ec_far_rows", ctypes.c_int32 * 2)]


class Tuning(ctypes.Structure):
    _fields_ = [("cell_scale", ctypes.c_double), ("tile_scale", ctypes.c_double), ("tiled", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("sized", ctypes.c_int32), ("wave_class", ctypes.c_int32),
                ("queue_cap", ctypes.c_int32), ("adj_cap", ctypes.c_int32)]


_lib = None


def load_library():
    """Load libdss.so (built in-tree by paper_2108_01013_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libdss.so not built at {LIB_PATH}; run __graft_entry__.build()")
    # torch ships its own HIP runtime under the same soname; loading torch first makes libdss
    # bind to that one, so a process that also uses torch on the GPU holds a single runtime
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    H = ctypes.c_void_p
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    st = ctypes.c_int
    sig = {
        "dss_create": (st, [ctypes.POINTER(Params), vp, ctypes.POINTER(H)]),
        "dss_create_batch": (st, [ctypes.POINTER(Params), ctypes.c_int32, vp, ctypes.POINTER(H)]),
        "dss_set_particles": (st, [H, i64, vp, vp, vp, vp, ctypes.c_int]),
        "dss_set_particles_batch": (st, [H, vp, vp, vp, vp, vp, ctypes.c_int]),
        "dss_read_stress_batch": (st, [H, vp, vp, ctypes.POINTER(i64)]),
        "dss_get_box_info": (st, [H, ctypes.c_int32, ctypes.POINTER(BoxInfo)]),
        "dss_set_step": (st, [H, i64]),
        "dss_build_neighbours": (st, [H]),
        "dss_compute_forces": (st, [H]),
        "dss_step": (st, [H, i64, i64, ctypes.c_int]),
        "dss_prepare_steps": (st, [H, i64, i64]),
        "dss_read_stress": (st, [H, vp, vp, ctypes.POINTER(i64)]),
        "dss_get_state": (st, [H, vp, vp, vp, vp, vp, ctypes.c_int]),
        "dss_get_eval_velocities": (st, [H, vp, vp, ctypes.c_int]),
        "dss_get_pairs": (st, [H, i64, vp, ctypes.POINTER(i64)]),
        "dss_get_cells": (st, [H, vp, i64, vp, vp]),
        "dss_get_history": (st, [H, i64, vp, vp, ctypes.POINTER(i64)]),
        "dss_get_rolling_history": (st, [H, i64, vp, vp, ctypes.POINTER(i64)]),
        "dss_observe_start": (st, [H]),
        "dss_observe": (st, [H, vp]),
        "dss_phi_profile": (st, [H, ctypes.c_int32, ctypes.c_double, vp]),
        "dss_phi_profile_noalloc": (st, [H, ctypes.c_int32, ctypes.c_double, vp]),
        "dss_contact_clusters": (st, [H, i64, vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "dss_get_info": (st, [H, ctypes.POINTER(Info)]),
        "dss_save_state": (st, [H, vp, ctypes.POINTER(ctypes.c_size_t)]),
        "dss_load_state": (st, [H, vp, ctypes.c_size_t]),
        "dss_set_timing": (st, [H, ctypes.c_int]),
        "dss_get_timing": (st, [H, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
        "dss_set_tuning": (st, [H, ctypes.POINTER(Tuning)]),
        "dss_get_tuning": (st, [H, ctypes.POINTER(Tuning)]),
        "dss_adjoint": (st, [H, i64, i64, i64, vp, ctypes.POINTER(ctypes.c_double), vp, vp, vp, vp,
                             ctypes.c_int]),
        "dss_last_error": (ctypes.c_char_p, [H]),
        "dss_status_string": (ctypes.c_char_p, [st]),
        "dss_destroy": (None, [H]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def make_params(p: dict, precision: int = DSS_FP64, capacity: int = 0, flags: int = 0) -> Params:
    s = Params()
    for d in range(3):
        s.L[d] = float(p["L"][d])
    for n, _ in Params._fields_[1:16]:
        setattr(s, n, float(p[n]))
    s.precision = int(precision)
    s.capacity = int(capacity)
    s.flags = int(flags) | (DSS_FLAG_EC_RANGES if p.get("ec_ranges") else 0)
    s.reserved = 0
    s.k_roll = float(p.get("kr", 0.0))      # rolling resistance (Appendix roll), off at 0
    s.mu_roll = float(p.get("mu_r", 0.0))
    s.wave_amp = float(p.get("wave_amp", 0.0))   # wavy shear (eq. uinf), off at 0
    s.wave_n = float(p.get("wave_n", 0.0))
    return s


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a):
    """(pointer, keep-alive, on_device) for a numpy array or a torch tensor."""
    if a is None:
        return None, None, None
    if _is_torch(a):
        if not a.is_contiguous() or a.dtype.__repr__() != "torch.float64":
            raise ValueError("torch tensors must be contiguous float64")
        return ctypes.c_void_p(a.data_ptr()), a, bool(a.is_cuda)
    arr = np.ascontiguousarray(a, dtype=np.float64)
    return ctypes.c_void_p(arr.ctypes.data), arr, False


class Simulation:
    """One box of N spheres behind a dss_handle."""

    def __init__(self, params: dict, precision: int = DSS_FP64, capacity: int = 0, record_pairs: bool = False,
                 stream=None):
        self.lib = load_library()
        self.params = dict(params)
        flags = DSS_FLAG_RECORD_PAIRS if record_pairs else 0
        self._p = make_params(params, precision, capacity, flags)
        self.h = ctypes.c_void_p()
        # stream: a hipStream_t handle (e.g. torch.cuda.current_stream().cuda_stream), or None for a
        # stream owned by the library handle
        s = self.lib.dss_create(ctypes.byref(self._p), ctypes.c_void_p(stream) if stream else None,
                                ctypes.byref(self.h))
        if s != 0:
            raise DssError(s, "dss_create failed")
        self.N = 0
        self.precision = int(precision)

    def _check(self, s, allow=()):
        if s != 0 and s not in allow:
            msg = self.lib.dss_last_error(self.h)
            raise DssError(s, msg.decode() if msg else "")

    def close(self):
        if self.h:
            self.lib.dss_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------------------------------
    def set_particles(self, x, radius, u=None, omega=None):
        px, kx, dev = _ptr(x)
        pr, kr, dev_r = _ptr(radius)
        pu, ku, dev_u = _ptr(u)
        pw, kw, dev_w = _ptr(omega)
        devs = {d for d in (dev, dev_r, dev_u, dev_w) if d is not None}
        if len(devs) != 1:
            raise ValueError("all arrays must live on the same side (host or device)")
        N = (kr.numel() if _is_torch(kr) else kr.size)
        self._check(self.lib.dss_set_particles(self.h, int(N), px, pr, pu, pw, int(dev)))
        self.N = int(N)
        rad = (kr.detach().cpu().numpy() if _is_torch(kr) else kr)
        self._set_class([rad], [self.params])

    def _set_class(self, radii, params):
        """Volume fraction and size ratio of the loaded boxes (the autotuner's workload class)."""
        phis = [float(np.sum(r ** 3)) * 4.0 * np.pi / 3.0 / float(np.prod(p["L"])) for r, p in zip(radii, params)]
        self.phi_mean = float(np.mean(phis))
        self.size_ratio = float(max(np.max(r) for r in radii) / min(np.min(r) for r in radii))

    def set_step(self, n):
        self._check(self.lib.dss_set_step(self.h, int(n)))

    def build_neighbours(self):
        self._check(self.lib.dss_build_neighbours(self.h))

    def compute_forces(self):
        self._check(self.lib.dss_compute_forces(self.h))

    def step(self, n=1, stress_every=0, sync=True):
        self._check(self.lib.dss_step(self.h, int(n), int(stress_every), int(bool(sync))))

    def prepare_steps(self, n, stress_every=0):
        """Capture the graphs that step(n, stress_every) from the current state will replay,
        without running anything."""
        self._check(self.lib.dss_prepare_steps(self.h, int(n), int(stress_every)))

    def read_stress(self):
        last = np.zeros(9)
        mean = np.zeros(9)
        ns = ctypes.c_int64(0)
        self._check(self.lib.dss_read_stress(self.h, last.ctypes.data_as(ctypes.c_void_p),
                                             mean.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ns)))
        return last.reshape(3, 3), mean.reshape(3, 3), int(ns.value)

    def state(self):
        out = {k: np.zeros((self.N, 3)) for k in ("x", "u", "w", "F", "T")}
        self._check(self.lib.dss_get_state(self.h, *[ctypes.c_void_p(out[k].ctypes.data) for k in
                                                     ("x", "u", "w", "F", "T")], 0))
        return out

    def state_into(self, x=None, u=None, w=None, F=None, T=None):
        """Write the state into caller tensors/arrays (all on the same side)."""
        ptrs = [_ptr(a) for a in (x, u, w, F, T)]
        devs = {p[2] for p in ptrs if p[2] is not None}
        if len(devs) > 1:
            raise ValueError("mixed host/device outputs")
        self._check(self.lib.dss_get_state(self.h, *[p[0] for p in ptrs], int(devs.pop() if devs else 0)))

    def eval_velocities(self):
        u = np.zeros((self.N, 3))
        w = np.zeros((self.N, 3))
        self._check(self.lib.dss_get_eval_velocities(self.h, ctypes.c_void_p(u.ctypes.data),
                                                     ctypes.c_void_p(w.ctypes.data), 0))
        return u, w

    def pairs(self):
        n = ctypes.c_int64(0)
        self._check(self.lib.dss_get_pairs(self.h, 0, None, ctypes.byref(n)), allow=(DSS_ERR_CAPACITY,))
        buf = np.zeros((max(n.value, 1), 2), np.int32)
        self._check(self.lib.dss_get_pairs(self.h, len(buf), ctypes.c_void_p(buf.ctypes.data), ctypes.byref(n)))
        p = buf[: n.value]
        return p[np.lexsort((p[:, 1], p[:, 0]))]

    def _ncell_total(self, dims):
        inf = BoxInfo()
        self._check(self.lib.dss_get_box_info(self.h, 0, ctypes.byref(inf)))
        return int(np.prod(dims)) * int(inf.size_classes)

    def box_info(self, b):
        inf = BoxInfo()
        self._check(self.lib.dss_get_box_info(self.h, int(b), ctypes.byref(inf)))
        return {"n_particles": inf.n_particles, "first_id": inf.first_id, "cells": tuple(inf.cells),
                "first_cell": inf.first_cell, "n_pairs": inf.n_pairs, "n_contacts": inf.n_contacts,
                "max_row_fill": inf.max_row_fill, "size_classes": inf.size_classes, "L": tuple(inf.L),
                "shear_rate": inf.shear_rate, "le_offset": inf.le_offset, "ec_far_rows": tuple(inf.ec_far_rows)}

    def cells(self):
        dims = np.zeros(3, np.int32)
        self._check(self.lib.dss_get_cells(self.h, ctypes.c_void_p(dims.ctypes.data), 0, None, None))
        ncell = self._ncell_total(dims)
        cs = np.zeros(ncell + 1, np.int32)
        perm = np.zeros(self.N, np.int32)
        self._check(self.lib.dss_get_cells(self.h, ctypes.c_void_p(dims.ctypes.data), ncell + 1,
                                           ctypes.c_void_p(cs.ctypes.data), ctypes.c_void_p(perm.ctypes.data)))
        return dims, cs, perm

    def history(self, rolling=False):
        """Committed contact history: (pairs (id_min, id_max) sorted, tangential stretches), or
        with rolling=True the rolling stretches of the same contacts."""
        n = ctypes.c_int64(0)
        cap = max(64, 8 * self.N)
        fn = self.lib.dss_get_rolling_history if rolling else self.lib.dss_get_history
        while True:
            pr = np.zeros((cap, 2), np.int32)
            xi = np.zeros((cap, 3))
            s = fn(self.h, cap, ctypes.c_void_p(pr.ctypes.data), ctypes.c_void_p(xi.ctypes.data), ctypes.byref(n))
            if s == 3 and n.value > cap:
                cap = int(n.value)
                continue
            self._check(s)
            break
        pr, xi = pr[: n.value], xi[: n.value]
        order = np.lexsort((pr[:, 1], pr[:, 0]))
        return pr[order], xi[order]

    KERNELS = ("k_predict", "k_scan", "k_scatter", "k_pairs", "k_finish", "k_pairs_vjp", "k_integrate_vjp",
               "k_pairs_ec")

    def set_tuning(self, cell_scale=None, tile_scale=None, tiled=None, graph=None, sized=None, wave_class=None,
                   queue_cap=None, adj_cap=None):
        """Change launch tuning (results do not depend on it); unspecified fields keep their value.
        sized: size-class stencils (one box); wave_class: first size class on one wavefront per
        particle (0 = default); queue_cap: length of the size-class pair queues (0 = full; a
        small value exercises the scans' stop and resume); adj_cap: capacity of the adjoint's
        per-particle pair lists (0 = default; a small value exercises the overflow list)."""
        t = Tuning()
        self._check(self.lib.dss_get_tuning(self.h, ctypes.byref(t)))
        if queue_cap is not None:
            t.queue_cap = int(queue_cap)
        if adj_cap is not None:
            t.adj_cap = int(adj_cap)
        if sized is not None:
            t.sized = int(bool(sized))
        if wave_class is not None:
            t.wave_class = int(wave_class)
        if cell_scale is not None:
            t.cell_scale = float(cell_scale)
        if tile_scale is not None:
            t.tile_scale = float(tile_scale)
        if tiled is not None:
            t.tiled = int(bool(tiled))
        if graph is not None:
            t.graph = int(bool(graph))
        self._check(self.lib.dss_set_tuning(self.h, ctypes.byref(t)))

    def adjoint(self, n_steps, stress_every, ckpt_every=20, weight=None):
        """Run n_steps steps and return J = sum weight * mean Sigma and its gradient by the
        discrete adjoint: {"J", "dmu", "dF_ER", "dx", "du", "dw"} (by id, host arrays).
        weight: 3 x 3 (default: the shear stress Sigma_xy)."""
        if weight is None:
            weight = np.zeros((3, 3))
            weight[0, 1] = 1.0
        wt = np.ascontiguousarray(np.asarray(weight, np.float64).reshape(9))
        J = ctypes.c_double(0.0)
        th = np.zeros(2)
        dx = np.zeros((self.N, 3))
        du = np.zeros((self.N, 3))
        dw = np.zeros((self.N, 3))
        vp = ctypes.c_void_p
        self._check(self.lib.dss_adjoint(self.h, int(n_steps), int(stress_every), int(ckpt_every),
                                         vp(wt.ctypes.data), ctypes.byref(J), vp(th.ctypes.data),
                                         vp(dx.ctypes.data), vp(du.ctypes.data), vp(dw.ctypes.data), 0))
        return {"J": J.value, "dmu": th[0], "dF_ER": th[1], "dx": dx, "du": du, "dw": dw}

    def adjoint_into(self, n_steps, stress_every, ckpt_every, weight, dx, du, dw):
        """As adjoint(), writing the state gradients into device tensors; returns (J, dmu, dF_ER)."""
        wt = np.ascontiguousarray(np.asarray(weight, np.float64).reshape(9))
        J = ctypes.c_double(0.0)
        th = np.zeros(2)
        ptrs = [_ptr(a) for a in (dx, du, dw)]
        devs = {q[2] for q in ptrs if q[2] is not None}
        if devs != {True}:
            raise ValueError("adjoint_into takes device tensors")
        self._check(self.lib.dss_adjoint(self.h, int(n_steps), int(stress_every), int(ckpt_every),
                                         ctypes.c_void_p(wt.ctypes.data), ctypes.byref(J),
                                         ctypes.c_void_p(th.ctypes.data), *[q[0] for q in ptrs], 1))
        return J.value, th[0], th[1]

    def observe_start(self):
        """The current state becomes the reference time of observe()."""
        self._check(self.lib.dss_observe_start(self.h))

    def observe(self) -> dict:
        """Shear-wise diffusivity D_y (eq. diffY) and velocity autocorrelation C_v (eq. corrV)
        since observe_start, with the mean squared shear-wise displacement and t - t0."""
        out = np.zeros(4)
        self._check(self.lib.dss_observe(self.h, ctypes.c_void_p(out.ctypes.data)))
        return {"D_y": out[0], "C_v": out[1], "msd_y": out[2], "elapsed": out[3]}

    def phi_profile(self, nbins: int, a_split: float) -> np.ndarray:
        """Local volume fraction along y: (2, nbins), row 0 radius <= a_split, row 1 larger."""
        phi = np.zeros(2 * nbins)
        self._check(self.lib.dss_phi_profile(self.h, int(nbins), float(a_split), ctypes.c_void_p(phi.ctypes.data)))
        return phi.reshape(2, nbins)

    def phi_profile_noalloc(self, nbins: int, a_split: float) -> np.ndarray:
        """phi_profile through the entry point that allocates no device memory."""
        phi = np.zeros(2 * int(nbins))
        self._check(self.lib.dss_phi_profile_noalloc(self.h, int(nbins), float(a_split),
                                                     ctypes.c_void_p(phi.ctypes.data)))
        return phi.reshape(2, int(nbins))

    def contact_clusters(self, cap: int | None = None) -> np.ndarray:
        """Histogram of the sizes of clusters of contacting particles: h[s - 1] clusters of s."""
        cap = int(cap or self.N)
        hist = np.zeros(cap, np.int64)
        nc, big = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(self.lib.dss_contact_clusters(self.h, cap, ctypes.c_void_p(hist.ctypes.data), ctypes.byref(nc),
                                                  ctypes.byref(big)))
        return hist

    def save_state(self) -> bytes:
        """Snapshot of the whole time-stepping state (host bytes)."""
        n = ctypes.c_size_t(0)
        self._check(self.lib.dss_save_state(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self.lib.dss_save_state(self.h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def load_state(self, blob: bytes):
        """Restore a snapshot taken with save_state on a handle of the same configuration."""
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self.lib.dss_load_state(self.h, buf, ctypes.c_size_t(len(blob))))

    def tuning(self):
        t = Tuning()
        self._check(self.lib.dss_get_tuning(self.h, ctypes.byref(t)))
        return {"cell_scale": t.cell_scale, "tile_scale": t.tile_scale, "tiled": bool(t.tiled),
                "graph": bool(t.graph), "sized": bool(t.sized), "wave_class": int(t.wave_class),
                "queue_cap": int(t.queue_cap), "adj_cap": int(t.adj_cap)}

    def set_timing(self, enable=True, kernels=None):
        """Time the named kernels (all if None) with HIP events; enable=False stops."""
        if not enable:
            mask = 0
        elif kernels is None:
            mask = -1
        else:
            mask = sum(1 << self.KERNELS.index(k) for k in kernels)
        self._check(self.lib.dss_set_timing(self.h, int(mask)))

    def timing(self):
        """{kernel name: (total ms, launches)} since set_timing(True)."""
        out = {}
        for k, name in enumerate(self.KERNELS):
            ms = ctypes.c_double(0.0)
            n = ctypes.c_int64(0)
            self._check(self.lib.dss_get_timing(self.h, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def info(self):
        inf = Info()
        self._check(self.lib.dss_get_info(self.h, ctypes.byref(inf)))
        return {"n_particles": inf.n_particles, "step": inf.step, "cells": tuple(inf.cells),
                "capacity": inf.capacity, "n_pairs": inf.n_pairs, "n_contacts": inf.n_contacts,
                "max_row_fill": inf.max_row_fill, "error_flags": inf.error_flags, "le_offset": inf.le_offset}


class Batch(Simulation):
    """B independent boxes (flow-curve sweep) behind one dss_handle: per-box L and shear rate,
    one counting sort and one pair launch per step over all boxes, one stress tensor per box.
    Particle ids run over the boxes in order (box b: ids first_id .. first_id + N_b - 1)."""

    def __init__(self, params_list, precision: int = DSS_FP64, capacity: int = 0, record_pairs: bool = False,
                 stream=None):
        self.lib = load_library()
        self.params_list = [dict(p) for p in params_list]
        self.params = self.params_list[0]
        self.B = len(self.params_list)
        flags = DSS_FLAG_RECORD_PAIRS if record_pairs else 0
        arr = (Params * self.B)(*[make_params(p, precision, capacity, flags) for p in self.params_list])
        self._p = arr
        self.h = ctypes.c_void_p()
        s = self.lib.dss_create_batch(arr, self.B, ctypes.c_void_p(stream) if stream else None,
                                      ctypes.byref(self.h))
        if s != 0:
            raise DssError(s, "dss_create_batch failed")
        self.N = 0
        self.sizes = None
        self.precision = int(precision)

    def set_particles(self, xs, radii, us=None, omegas=None):
        """xs, radii (, us, omegas): one host array per box."""
        sizes = np.array([len(r) for r in radii], np.int64)
        x = np.ascontiguousarray(np.concatenate(xs), np.float64)
        r = np.ascontiguousarray(np.concatenate(radii), np.float64)
        u = None if us is None else np.ascontiguousarray(np.concatenate(us), np.float64)
        w = None if omegas is None else np.ascontiguousarray(np.concatenate(omegas), np.float64)
        vp = ctypes.c_void_p
        self._check(self.lib.dss_set_particles_batch(
            self.h, vp(sizes.ctypes.data), vp(x.ctypes.data), vp(r.ctypes.data),
            vp(u.ctypes.data) if u is not None else None, vp(w.ctypes.data) if w is not None else None, 0))
        self.sizes = sizes
        self.offsets = np.concatenate([[0], np.cumsum(sizes)])
        self.N = int(sizes.sum())
        self._set_class([np.asarray(a, np.float64) for a in radii], self.params_list)

    def read_stress(self):
        """(last, mean, n_samples): last and mean are B x 3 x 3."""
        last = np.zeros(9 * self.B)
        mean = np.zeros(9 * self.B)
        ns = ctypes.c_int64(0)
        self._check(self.lib.dss_read_stress_batch(self.h, last.ctypes.data_as(ctypes.c_void_p),
                                                   mean.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ns)))
        return last.reshape(self.B, 3, 3), mean.reshape(self.B, 3, 3), int(ns.value)

    def _ncell_total(self, dims):
        last = self.box_info(self.B - 1)
        return int(last["first_cell"] + np.prod(last["cells"]))

    def box_slice(self, b):
        return slice(int(self.offsets[b]), int(self.offsets[b + 1]))
