"""Scheduler logic of the serving loop on a CPU fake executor (no GPU)."""
import numpy as np

from paper_2605_22698_amd.serving import Request, Server


class FakeExecutor:
    """Free particles (x += dt v); 100 bytes of 'device memory' per atom; every
    packed step takes 1 ms of virtual time plus 1 us per atom."""

    def __init__(self, clock):
        self.clock = clock
        self.md = None
        self.max_footprint = 0
        self.launches = 0

    def footprint(self, n_atoms):
        return 100 * n_atoms

    def upload(self, r):
        return {"pos": r.pos.copy(), "vel": r.vel.copy(), "species": r.species}

    def launch(self, parts):
        self.launches += 1
        self.md = [dict(p) for p in parts] if parts else None
        n = sum(len(p["species"]) for p in parts)
        self.max_footprint = max(self.max_footprint, self.footprint(n))

    def step(self):
        n = 0
        for p in self.md:
            p["pos"] = p["pos"] + 0.5 * p["vel"]
            n += len(p["species"])
        ms = 1.0 + 1e-3 * n
        self.clock.t += ms / 1e3
        return ms

    def states(self):
        return [{"pos": _Arr(p["pos"]), "vel": _Arr(p["vel"])} for p in self.md]

    def close(self):
        self.md = None


class _Arr(np.ndarray):
    def __new__(cls, a):
        return np.asarray(a).copy().view(cls)

    def cpu(self):
        return self

    def numpy(self):
        return np.asarray(self)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def wait(self, dt):
        self.t += max(dt, 1e-6)


def _requests(n, seed=0, lo=5, hi=60):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for k in range(n):
        t += rng.exponential(0.01)
        m = int(rng.integers(lo, hi))
        out.append(Request(k, t, rng.standard_normal((m, 3)), rng.standard_normal((m, 3)), np.zeros(m, np.int32),
                           np.eye(3) * 10, np.ones(3, np.uint8), int(rng.integers(3, 40))))
    return out


def _serve(reqs, budget, max_active=64):
    clock = Clock()
    ex = FakeExecutor(clock)
    srv = Server(ex, budget, max_active=max_active, clock=clock)
    for r in reqs:
        srv.submit(r)
    stats = srv.run(idle_wait=clock.wait)
    return srv, ex, stats


def test_every_request_finishes_with_its_own_trajectory():
    reqs = _requests(20)
    srv, ex, stats = _serve(reqs, budget=10 ** 9)
    assert len(srv.done) == 20 and not srv.pending and not srv.active
    for r in srv.done:
        assert r.steps_done == r.n_steps
        np.testing.assert_allclose(r.final_pos, r.pos + 0.5 * r.n_steps * r.vel, atol=1e-12)
    assert stats.summary()["atom_steps"] == sum(r.n_atoms * r.n_steps for r in reqs)


def test_small_budget_queues_but_never_overcommits():
    reqs = _requests(25, seed=1)
    budget = 100 * 120
    srv, ex, stats = _serve(reqs, budget)
    assert ex.max_footprint <= budget
    assert all(r.steps_done == r.n_steps for r in srv.done)
    # first come first served: admission order follows arrival order
    adm = sorted(srv.done, key=lambda r: (r.admitted_at, r.rid))
    assert [r.rid for r in adm] == sorted(r.rid for r in srv.done)
    # some request had to wait for memory
    assert any(r.admitted_at > r.arrival + 1e-9 for r in srv.done)


def test_admits_while_others_run():
    reqs = _requests(10, seed=2, lo=5, hi=10)
    for r in reqs:
        r.n_steps = 200
    srv, ex, stats = _serve(reqs, budget=10 ** 9)
    first = min(srv.done, key=lambda r: r.rid)
    later = [r for r in srv.done if r.rid > first.rid]
    assert any(first.admitted_at < r.admitted_at < first.finished_at for r in later)
    assert stats.repacks >= 2


def test_rejects_request_that_can_never_fit_and_respects_slots():
    reqs = _requests(8, seed=3)
    big = Request(99, 0.0, np.zeros((500, 3)), np.zeros((500, 3)), np.zeros(500, np.int32), np.eye(3) * 30,
                  np.ones(3, np.uint8), 5)
    srv, ex, stats = _serve(reqs + [big], budget=100 * 200, max_active=2)
    assert big.rejected and stats.rejected == 1
    assert all(r.steps_done == r.n_steps for r in srv.done if not r.rejected)


def test_iteration_latency_includes_repacks():
    # a repack (new packed state) costs 5 ms of virtual time here: the
    # per-iteration wall times include it, the device step times do not
    reqs = _requests(12, seed=4)
    clock = Clock()
    ex = FakeExecutor(clock)
    plain_launch = ex.launch

    def slow_launch(parts):
        clock.t += 5e-3
        plain_launch(parts)
    ex.launch = slow_launch
    srv = Server(ex, 10 ** 9, clock=clock)
    for r in reqs:
        srv.submit(r)
    stats = srv.run(idle_wait=clock.wait)
    s = stats.summary()
    assert len(stats.iter_ms) == len(stats.step_ms) == s["steps"]
    assert all(it >= st - 1e-9 for it, st in zip(stats.iter_ms, stats.step_ms))
    # every repack but the last (which empties the pack) precedes a step
    assert sum(it - st > 4.9 for it, st in zip(stats.iter_ms, stats.step_ms)) == stats.repacks - 1
    assert s["p99_iter_ms"] > s["p99_ms"]


def test_pressure_without_thermostat_is_rejected():
    import pytest
    from paper_2605_22698_amd.serving import GpuExecutor
    with pytest.raises(ValueError, match="Langevin"):
        GpuExecutor(None, [1.0], 5.0, pressure_bar=1.0)
