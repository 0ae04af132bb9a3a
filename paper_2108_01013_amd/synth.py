"""Seeded synthetic inputs: particle radii, box size and overlap-free positions.

This module holds none of the method's arithmetic.  It only draws radii with the
size distributions used in the paper's workloads (bidisperse 1:1.4 at equal
volume, Sec. 3.1 tables; 3:1 at V2/V1 = 0.25, Sec. 2.1 scaling test; a truncated
lognormal for the size-ratio-10 case), sizes a cubic box for a target volume
fraction, places centres uniformly at random and removes overlaps with a generic
soft-sphere push (nearest neighbours from ``scipy.spatial.cKDTree``).  The paper's
own initial conditions come from a sphere-packing program that is not available;
these stand in for them.  Both the HIP path and the oracle receive the arrays
produced here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.spatial import cKDTree


def default_params(L, **over) -> dict:
    """Physical parameters in units eta0 = a_min = gdot_ref = 1.

    St = rho a0^2 gdot / eta0 = 0.1, k_hat = 4e5, k_t/k_n = 2/7, gamma_n gdot/k_n = 1e-7,
    mu = 1, F_ER = 1 (gdot_0 = 1), lambda_D = 0.05, no attraction, eps_lub = 0.02,
    pair cutoff 1.1 (a_i + a_j), dt = 1e-4."""
    kn = 4.0e5
    p = dict(L=[float(L[0]), float(L[1]), float(L[2])], shear_rate=1.0, eta0=1.0, rho=0.1, kn=kn,
             kt=kn * 2.0 / 7.0, gamma_n=1.0e-7 * kn, mu=1.0, F_ER=1.0, lambda_D=0.05, a0=1.0, hamaker=0.0,
             eps_vdw=0.01, eps_lub=0.02, cutoff_factor=1.1, dt=1.0e-4)
    p.update(over)
    return p


def bidisperse_radii(N: int, ratio: float = 1.4, vol_ratio: float = 1.0, seed: int = 0) -> np.ndarray:
    """N radii, a1 = 1 and a2 = ratio, with total volume ratio V2/V1 = vol_ratio, in shuffled order."""
    n_large = int(round(N * vol_ratio / (vol_ratio + ratio ** 3)))
    rad = np.ones(N)
    rad[:n_large] = ratio
    rng = np.random.default_rng(seed)
    rng.shuffle(rad)
    return rad


def lognormal_radii(N: int, median: float = 1.5, sigma: float = 0.5, lo: float = 1.0, hi: float = 10.0,
                    seed: int = 0) -> np.ndarray:
    """N radii with ln a ~ Normal(ln median, sigma), truncated to [lo, hi] by rejection."""
    rng = np.random.default_rng(seed)
    out = np.empty(0)
    while out.size < N:
        draw = np.exp(rng.normal(math.log(median), sigma, size=2 * N))
        out = np.concatenate([out, draw[(draw >= lo) & (draw <= hi)]])
    return out[:N].copy()


def box_for_fraction(rad: np.ndarray, phi: float) -> float:
    """Side of the cubic box holding the spheres at volume fraction phi."""
    vol = (4.0 / 3.0) * math.pi * float(np.sum(rad ** 3))
    return (vol / phi) ** (1.0 / 3.0)


def _min_image(d, L):
    return d - L * np.round(d / L)


def _near_pairs(x: np.ndarray, r: np.ndarray, L: float, skin: float, wide: bool):
    """Candidate pairs (i, j) with |x_i - x_j| < r_i + r_j + skin, each once.  For a narrow
    size distribution one fixed-radius query (2 r_max + skin); for a wide one every particle
    queries 2 r_i + skin and keeps the partners that are smaller (ties: lower index), so the
    work follows the particle sizes instead of the largest one."""
    tree = cKDTree(x, boxsize=L)
    if not wide:
        return tree.query_pairs(2.0 * float(r.max()) + skin, output_type="ndarray")
    nb = tree.query_ball_point(x, 2.0 * r + skin, return_sorted=True)
    cnt = np.fromiter((len(q) for q in nb), np.int64, len(nb))
    pi = np.repeat(np.arange(len(r)), cnt)
    pj = np.concatenate([np.asarray(q, np.int64) for q in nb]) if cnt.sum() else np.zeros(0, np.int64)
    own = (r[pj] < r[pi]) | ((r[pj] == r[pi]) & (pj < pi))
    return np.stack([pi[own], pj[own]], axis=1)


def relax_positions(rad: np.ndarray, L: float, seed: int = 0, tol: float = 1e-3, max_sweeps: int = 20000,
                    x0: np.ndarray | None = None) -> np.ndarray:
    """Uniform random centres in [0, L)^3, then overlap removal by a soft-sphere push.

    Radii are inflated from 0.8x to 1x in stages; at each stage every overlapping pair is pushed
    apart along its centre line (heavy-ball momentum 0.9 on the displacements).  Stops when the
    largest overlap is below tol * min(a_i, a_j).  Size ratios above 2 use size-aware
    neighbour queries."""
    rng = np.random.default_rng(seed)
    N = len(rad)
    x = rng.uniform(0.0, L, size=(N, 3)) if x0 is None else np.array(x0, dtype=np.float64)
    a_max = float(rad.max())
    wide = a_max > 2.0 * float(rad.min())
    skin = 0.3 * float(rad.min())
    stages = list(np.linspace(0.8, 1.0, 9))
    sweeps = 0
    for si, scale in enumerate(stages):
        r = rad * scale
        final = si == len(stages) - 1
        goal = tol if final else 0.05
        x_ref = None
        vel = np.zeros((N, 3))
        while sweeps < max_sweeps:
            if x_ref is None or np.max(np.abs(_min_image(x - x_ref, L))) > 0.5 * skin:
                x %= L
                x[x >= L] = 0.0
                prs = _near_pairs(x, r, L, skin, wide)
                d = _min_image(x[prs[:, 1]] - x[prs[:, 0]], L)
                keep = np.sqrt(np.einsum("ij,ij->i", d, d)) < r[prs[:, 0]] + r[prs[:, 1]] + skin
                pi, pj = prs[keep, 0], prs[keep, 1]
                ri, rj = r[pi], r[pj]
                rmin = np.minimum(ri, rj)
                wi = rj ** 3 / (ri ** 3 + rj ** 3)   # the lighter particle moves more
                wj = 1.0 - wi
                x_ref = x.copy()
            d = _min_image(x[pj] - x[pi], L)
            dist = np.sqrt(np.einsum("ij,ij->i", d, d))
            ov = (ri + rj) - dist
            hit = ov > 0.0
            sweeps += 1
            worst = float(np.max(ov[hit] / rmin[hit])) if hit.any() else 0.0
            if worst < goal:
                break
            push = np.where(hit, (0.5 * ov + 0.2 * tol * rmin) / np.maximum(dist, 1e-12), 0.0)
            disp = np.empty((N, 3))
            for c in range(3):
                disp[:, c] = (np.bincount(pj, weights=push * wj * d[:, c], minlength=N)
                              - np.bincount(pi, weights=push * wi * d[:, c], minlength=N))
            vel = 0.9 * vel + disp
            x += vel
    x %= L
    x[x >= L] = 0.0
    return x


@dataclass
class Workload:
    name: str
    x: np.ndarray
    rad: np.ndarray
    L: float
    params: dict


def bidisperse_box(N: int, phi: float, seed: int, ratio: float = 1.4, vol_ratio: float = 1.0,
                   tol: float = 1e-3, **param_over) -> Workload:
    rad = bidisperse_radii(N, ratio, vol_ratio, seed)
    L = box_for_fraction(rad, phi)
    x = relax_positions(rad, L, seed=seed + 1000, tol=tol)
    p = default_params([L, L, L], **param_over)
    return Workload(f"bidisperse N={N} phi={phi} ratio={ratio}", x, rad, L, p)


def config_small(seed: int = 1) -> Workload:
    """N = 1000 bidisperse (1 : 1.4, equal volumes), phi = 0.50, mu = 1, gdot = 1, dt = 1e-4."""
    return bidisperse_box(1000, 0.50, seed)


def config_single_box(seed: int = 2, N: int = 100_000) -> Workload:
    """N = 100k bidisperse (1 : 1.4, equal volumes), phi = 0.55, mu = 1, gdot = 1, dt = 1e-4."""
    return bidisperse_box(N, 0.55, seed)


def config_high_ratio(seed: int = 3, N: int = 500_000) -> Workload:
    """N = 500k, ln a ~ Normal(ln 1.5, 0.5) truncated to [1, 10] (size ratio 10), phi = 0.55,
    mu = 1, gdot = 1, dt = 1e-4."""
    rad = lognormal_radii(N, seed=seed)
    L = box_for_fraction(rad, 0.55)
    x = relax_positions(rad, L, seed=seed + 1000)
    return Workload(f"lognormal N={N} phi=0.55 a in [1, 10]", x, rad, L, default_params([L, L, L]))


SWEEP_PHI = (0.40, 0.45, 0.50, 0.55, 0.58)


def _sweep_box(args):
    b, n, phi, seed = args
    return bidisperse_box(int(n), phi, seed=seed + 17 * b)


def config_sweep(B: int = 64, seed: int = 3, n_lo: int = 2000, n_hi: int = 50_000, workers: int = 0,
                 start_method: str = "fork"):
    """Flow-curve sweep: B bidisperse boxes (1 : 1.4, equal volumes), N_b uniform on
    {n_lo .. n_hi}, phi_b = SWEEP_PHI[b mod 5], shear rate 10^(-2 + 3 b / (B - 1)) spanning
    three decades.  Returns (workloads, shear rates).  workers > 1 relaxes the boxes in that
    many processes: forked before any GPU work, or started afresh ("spawn") in a process that
    already uses the GPU (the workers only run numpy and scipy)."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=B)
    jobs = [(b, sizes[b], SWEEP_PHI[b % len(SWEEP_PHI)], seed) for b in range(B)]
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context(start_method).Pool(workers) as pool:
            ws = pool.map(_sweep_box, jobs, chunksize=1)
    else:
        ws = [_sweep_box(j) for j in jobs]
    gds = [10.0 ** (-2.0 + 3.0 * b / max(B - 1, 1)) for b in range(B)]
    return ws, gds
