"""The allocation-free entry point dss_phi_profile_noalloc, through the C ABI, against
dss_phi_profile (the entry point whose kernels it shares): two calls in a row on one GPU, the
second with a smaller input (fewer bins, then a handle with fewer particles), and a case whose
grid is capped by the size of the device array (the sums then run in another order).
Tolerance 1e-12 of the largest bin: sums of at most a few thousand positive terms of one sign
in FP64."""
import numpy as np
import pytest

from paper_2108_01013_amd import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_phi_profile_noalloc_matches_phi_profile():
    from paper_2108_01013_amd.dss import DssError, Simulation
    w = synth.bidisperse_box(20_000, 0.50, seed=17)
    sim = Simulation(w.params)
    sim.set_particles(w.x, w.rad)
    sim.step(5)
    a = sim.phi_profile(333, 1.2)
    b = sim.phi_profile_noalloc(333, 1.2)
    assert rel(b, a) <= 1e-12
    # second call, smaller input
    c = sim.phi_profile_noalloc(16, 1.2)
    assert rel(c, sim.phi_profile(16, 1.2)) <= 1e-12
    # the profile integrates to the volume fraction of each group
    phi = (4.0 / 3.0) * np.pi * np.array([np.sum(w.rad[w.rad <= 1.2] ** 3), np.sum(w.rad[w.rad > 1.2] ** 3)]) / w.L ** 3
    assert np.max(np.abs(c.mean(axis=1) - phi)) <= 1e-12
    with pytest.raises(DssError):
        sim.phi_profile_noalloc(2049, 1.2)
    with pytest.raises(DssError):
        sim.phi_profile_noalloc(0, 1.2)
    sim.close()
    # a handle with fewer particles on the same GPU (the device array keeps the last call's contents)
    s = synth.bidisperse_box(2000, 0.45, seed=18)
    sim2 = Simulation(s.params)
    sim2.set_particles(s.x, s.rad)
    assert rel(sim2.phi_profile_noalloc(7, 1.0), sim2.phi_profile(7, 1.0)) <= 1e-12
    sim2.close()


def test_phi_profile_noalloc_capped_grid():
    """N = 80 000 and 2048 bins: the partial profiles of one workgroup per 256 particles (313)
    would exceed the device array, so fewer workgroups stride over the particles."""
    from paper_2108_01013_amd.dss import Simulation
    rng = np.random.default_rng(19)
    N, L = 80_000, 200.0
    x = rng.uniform(0.0, L, size=(N, 3))
    rad = np.where(rng.random(N) < 0.5, 1.0, 1.4)
    p = synth.default_params([L, L, L])
    sim = Simulation(p)
    sim.set_particles(x, rad)
    for nb in (2048, 64):
        assert rel(sim.phi_profile_noalloc(nb, 1.2), sim.phi_profile(nb, 1.2)) <= 1e-12, nb
    sim.close()
