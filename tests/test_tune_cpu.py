"""Host logic of the autotuner with a stand-in simulation (no GPU): it times every legal
candidate, applies and caches the fastest, and reuses the cache for the same workload class."""
import time

import pytest

from paper_2108_01013_amd import tune


class FakeSim:
    """Step time depends on the tuning; cell_scale 1.3 is refused like an illegal lattice."""

    def __init__(self, N=20000, phi=0.55, B=1):
        self.N, self.phi_mean, self.size_ratio, self.precision = N, phi, 1.4, 0
        if B > 1:
            self.B = B
        self.t = {"cell_scale": 1.0, "tile_scale": 1.0, "tiled": True, "graph": True}
        self.calls = []

    def set_tuning(self, **kw):
        from paper_2108_01013_amd.dss import DssError
        if kw.get("cell_scale") == 1.3:
            raise DssError(4, "lattice too small")
        self.t.update(kw)
        self.calls.append(dict(kw))

    def step(self, n, sync=True):
        # milliseconds per step, so that the ranking survives the host's scheduling jitter
        cost = 2e-3 * (1.0 + abs(self.t["tile_scale"] - 1.5) + (0.0 if self.t["tiled"] else 2.0))
        time.sleep(cost * n)


def test_autotune_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "t.json")
    sim = FakeSim()
    rec = tune.autotune(sim, trial_steps=3, cache_path=path)
    assert not rec["cached"]
    assert rec["tuning"]["tile_scale"] == 1.5 and rec["tuning"]["tiled"]
    assert all(t["tuning"]["cell_scale"] != 1.3 for t in rec["trials"])
    assert len(rec["trials"]) == len(tune.CANDIDATES) - 1
    assert sim.t["tile_scale"] == 1.5
    sim2 = FakeSim()
    rec2 = tune.autotune(sim2, trial_steps=3, cache_path=path)
    assert rec2["cached"] and sim2.calls == [dict(rec["tuning"], graph=True)]
    # another workload class is tuned afresh
    sim3 = FakeSim(N=2000, phi=0.40, B=8)
    assert tune.workload_key(sim3) != tune.workload_key(sim)
    assert not tune.autotune(sim3, trial_steps=1, cache_path=path)["cached"]


@pytest.mark.parametrize("N,phi,key", [(100_000, 0.55, "B1:N2^17:phi0.55:ratio1.40:prec0"),
                                       (1000, 0.51, "B1:N2^10:phi0.50:ratio1.40:prec0")])
def test_workload_key(N, phi, key):
    assert tune.workload_key(FakeSim(N, phi)) == key


def test_size_class_candidates_only_for_one_wide_box():
    wide = FakeSim(N=500_000)
    wide.size_ratio = 9.98
    assert any(c.get("sized") for c in tune.candidates_for(wide))
    assert all(c["sized"] is False for c in tune.CANDIDATES)
    narrow = FakeSim(N=100_000)
    assert tune.candidates_for(narrow) == tune.CANDIDATES
    batch = FakeSim(N=20_000, B=8)
    batch.size_ratio = 9.98
    assert tune.candidates_for(batch) == tune.CANDIDATES
