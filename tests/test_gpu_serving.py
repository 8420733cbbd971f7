"""Continuous-batching MD serving on the GPU: every request's trajectory is
bit-identical alone and in the mix (packed with whatever else was running)."""
import numpy as np
import pytest

import synth
from paper_2605_22698_amd.serving import GpuExecutor, Request, Server
from tests.gpu_util import model, say

pytestmark = pytest.mark.gpu


class StepClock:
    """Virtual time: 1 ms per engine step, so arrivals interleave with steps
    deterministically."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def _requests(n):
    rng = np.random.default_rng(71)
    out, t = [], 0.0
    for k in range(n):
        t += rng.exponential(0.004)
        m = int(rng.integers(30, 160))
        b = synth.jittered_lattice(m, 0.1, 0.3, 4, np.random.default_rng(100 + k))
        v = synth.maxwell_boltzmann(b, 300.0, np.random.default_rng(200 + k))
        out.append(Request(k, t, b.pos, v, b.species, b.cell[0], b.pbc[0], int(rng.integers(10, 30))))
    return out


def _serve(m, reqs, budget, max_active=64, friction=0.0, pressure=None):
    clock = StepClock()
    ex = GpuExecutor(m, synth.SPECIES_MASS[:4], 5.0, skin=1.0, rebuild_every=7, temperature_K=300.0,
                     friction_per_fs=friction, pressure_bar=pressure, barostat_interval=3, volume_fraction=0.01)
    step = ex.step

    def timed_step():
        ms = step()
        clock.t += 1e-3
        return ms
    ex.step = timed_step
    srv = Server(ex, budget, max_active=max_active, clock=clock)
    for r in reqs:
        srv.submit(r)

    def idle(dt):
        clock.t += max(dt, 1e-6)
    stats = srv.run(idle_wait=idle)
    return srv, stats


def test_alone_equals_in_mix():
    m = model(synth.serving_model(), 4)
    reqs = _requests(6)
    srv, stats = _serve(m, reqs, budget=1 << 40)
    say(f"serving: {stats.summary()}")
    assert stats.repacks >= 3
    mixed = {r.rid: r for r in srv.done}
    for r in _requests(6):
        alone, _ = _serve(m, [Request(r.rid, 0.0, r.pos, r.vel, r.species, r.cell, r.pbc, r.n_steps)], 1 << 40)
        a = alone.done[0]
        assert np.array_equal(a.final_pos, mixed[r.rid].final_pos), r.rid
        assert np.array_equal(a.final_vel, mixed[r.rid].final_vel), r.rid


def test_budget_forces_queueing_on_gpu():
    m = model(synth.serving_model(), 4)
    reqs = _requests(5)
    one = GpuExecutor(m, synth.SPECIES_MASS[:4], 5.0).footprint(max(r.n_atoms for r in reqs))
    srv, stats = _serve(m, reqs, budget=int(one * 1.2))
    assert all(r.steps_done == r.n_steps for r in srv.done)
    assert any(r.admitted_at > r.arrival for r in srv.done)


def test_langevin_requests_alone_equal_in_mix():
    # NVT requests keep their own seed and step counter across repacks
    m = model(synth.serving_model(), 4)
    reqs = _requests(5)
    for k, r in enumerate(reqs):
        r.seed = 1000 + k
    srv, stats = _serve(m, reqs, budget=1 << 40, friction=0.05)
    assert stats.repacks >= 3
    mixed = {r.rid: r for r in srv.done}
    for k, r in enumerate(_requests(5)):
        alone, _ = _serve(m, [Request(r.rid, 0.0, r.pos, r.vel, r.species, r.cell, r.pbc, r.n_steps, seed=1000 + k)],
                          1 << 40, friction=0.05)
        a = alone.done[0]
        assert np.array_equal(a.final_pos, mixed[r.rid].final_pos), r.rid
        assert np.array_equal(a.final_vel, mixed[r.rid].final_vel), r.rid


def test_npt_requests_alone_equal_in_mix():
    # NPT requests: own seeds, own proposal schedule, volume step fixed from
    # their initial volume; cells change and continue across repacks
    m = model(synth.serving_model(), 4)
    reqs = _requests(5)
    for k, r in enumerate(reqs):
        r.seed = 2000 + k
    srv, stats = _serve(m, reqs, budget=1 << 40, friction=0.05, pressure=1000.0)
    assert stats.repacks >= 3
    mixed = {r.rid: r for r in srv.done}
    moved = 0
    for k, r in enumerate(_requests(5)):
        alone, _ = _serve(m, [Request(r.rid, 0.0, r.pos, r.vel, r.species, r.cell, r.pbc, r.n_steps, seed=2000 + k)],
                          1 << 40, friction=0.05, pressure=1000.0)
        a = alone.done[0]
        assert np.array_equal(a.final_pos, mixed[r.rid].final_pos), r.rid
        assert np.array_equal(a.final_vel, mixed[r.rid].final_vel), r.rid
        assert np.array_equal(a.final_cell, mixed[r.rid].final_cell), r.rid
        moved += int(not np.array_equal(a.final_cell, r.cell))
    assert moved > 0  # some volume moves were accepted
