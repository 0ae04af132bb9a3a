"""Observables of Sec. 3 on the GPU (dss_observe, dss_phi_profile, dss_contact_clusters)
against the oracle's definitions evaluated on the GPU's states, on an MI355X.

The shear-wise positions are unwrapped on the host from consecutive states (a jump of more
than L_y / 2 in one step is a crossing of the sheared y faces), independently of the
library's crossing counters."""
import sys

import numpy as np
import pytest

import oracle
from paper_2108_01013_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_diffusivity_and_autocorrelation():
    from paper_2108_01013_amd.dss import DssError, Simulation
    w = synth.config_small()
    p = w.params
    L = p["L"][1]
    say("case: observables D_y, C_v N=1000")
    # particles near both y faces are launched across them
    u = oracle.ambient_velocity(p, w.x)
    near_top = np.argsort(L - w.x[:, 1])[:6]
    near_bot = np.argsort(w.x[:, 1])[:6]
    u[near_top, 1] = 400.0
    u[near_bot, 1] = -400.0
    sim = Simulation(p)
    sim.set_particles(w.x, w.rad, u=u)
    with pytest.raises(DssError):
        sim.observe()
    sim.observe_start()
    s = sim.state()
    y0 = s["x"][:, 1].copy()
    v0 = s["u"][:, 1].copy()
    y_prev, img = y0.copy(), np.zeros(len(y0))
    for k in range(40):
        sim.step(1)
        y = sim.state()["x"][:, 1]
        img += (y - y_prev < -L / 2).astype(float) - (y - y_prev > L / 2).astype(float)
        y_prev = y.copy()
    assert np.count_nonzero(img > 0) >= 1 and np.count_nonzero(img < 0) >= 1   # both faces crossed
    s = sim.state()
    ob = sim.observe()
    elapsed = 40 * p["dt"]
    assert abs(ob["elapsed"] - elapsed) < 1e-15
    D = oracle.shear_diffusivity(p, y0, s["x"][:, 1] + img * L, elapsed)
    C = oracle.velocity_autocorrelation(v0, s["u"][:, 1])
    assert abs(ob["D_y"] - D) <= 1e-12 * abs(D)
    assert abs(ob["C_v"] - C) <= 1e-12 * abs(C)
    sim.close()


def test_phi_profile():
    from paper_2108_01013_amd.dss import Simulation
    w = synth.bidisperse_box(4000, 0.55, seed=14)
    p = w.params
    say("case: phi profile N=4000")
    sim = Simulation(p)
    sim.set_particles(w.x, w.rad)
    sim.step(20)
    x = sim.state()["x"]
    for nb in (1, 16, 333):
        g = sim.phi_profile(nb, 1.2)
        o = oracle.phi_profile(p, x[:, 1], w.rad, nb, 1.2)
        assert np.max(np.abs(g - o)) <= 1e-12 * np.max(o)
    assert abs(sim.phi_profile(1, 1.2).sum() - 0.55) < 1e-3      # the box's volume fraction
    sim.close()


@pytest.mark.parametrize("mu,hamaker", [(1.0, 0.0), (1.0, 2e-3)])
def test_contact_clusters(mu, hamaker):
    from paper_2108_01013_amd.dss import Simulation
    w = synth.bidisperse_box(4000, 0.55, seed=14)
    p = dict(w.params, mu=mu, hamaker=hamaker)
    say(f"case: contact clusters N=4000 hamaker={hamaker}")
    sim = Simulation(p)
    sim.set_particles(w.x, w.rad)
    sim.step(30)
    pairs, _ = sim.history()
    assert len(pairs) > 100
    for cap in (4000, 8):
        g = sim.contact_clusters(cap)
        o = oracle.contact_clusters(4000, pairs, cap)
        assert np.array_equal(g, o), (cap, np.flatnonzero(g != o)[:10])
    # the observables share the handle's work buffers: other requests in between
    x = sim.state()["x"]
    assert np.max(np.abs(sim.phi_profile(64, 1.2) - oracle.phi_profile(p, x[:, 1], w.rad, 64, 1.2))) <= 1e-12
    assert np.array_equal(sim.contact_clusters(4000), oracle.contact_clusters(4000, pairs, 4000))
    sim.close()
