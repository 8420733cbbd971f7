"""GPU velocity-Verlet MD vs the oracle integrator, plus NVE conservation and
packing invariance of trajectories."""
import numpy as np
import pytest

import synth
from oracle import md as omd
from oracle import model as om
from tests.gpu_util import device, model, say

pytestmark = pytest.mark.gpu


def _run_gpu(m, b, vel, n_steps, dt, rebuild_every=20, skin=1.0):
    import torch
    import paper_2605_22698_amd as e3
    d = device()
    cfg = synth.ModelConfig.from_json(m.config_json)
    md = e3.MD(m, b.offsets, torch.tensor(b.pos, dtype=torch.float64, device=d),
               torch.tensor(vel, dtype=torch.float64, device=d), torch.tensor(b.species, dtype=torch.int32, device=d),
               synth.SPECIES_MASS[:cfg.n_species], b.cell, b.pbc, cfg.cutoff, skin, rebuild_every)
    E = torch.empty(b.n_structures, dtype=torch.float64, device=d)
    md.step(n_steps, dt, E)
    x, v, F = md.state()
    torch.cuda.synchronize()
    return x.cpu().numpy(), v.cpu().numpy(), E.cpu().numpy(), md


def _min_image(d, b):
    owner = np.repeat(np.arange(b.n_structures), np.diff(b.offsets))
    L = b.cell[owner][:, [0, 1, 2], [0, 1, 2]]
    per = b.pbc[owner].astype(bool)
    return np.where(per, d - np.round(d / np.where(per, L, 1.0)) * L, d)


@pytest.mark.parametrize("rebuild_every", [3, 20])
def test_trajectory_matches_oracle(rebuild_every):
    cfg = synth.ModelConfig(lmax=2, channels=32, layers=2, n_species=4, cutoff=5.0, avg_neighbors=10.0)
    b = synth.jittered_lattice(40, 0.1, 0.3, 4, np.random.default_rng(51))
    vel = synth.maxwell_boltzmann(b, 300.0, np.random.default_rng(52))
    m = model(cfg, 7)
    say(f"md parity rebuild_every={rebuild_every}")
    x, v, E, _ = _run_gpu(m, b, vel, 12, 0.5, rebuild_every=rebuild_every)
    om_m = om.Model(cfg, synth.model_weights(cfg, 7))

    def force(xx):
        Es, F, _ = om.energy_forces(om_m, synth.Batch(xx, b.species, b.cell, b.pbc, b.offsets))
        return Es, F
    xr, vr, Er = omd.velocity_verlet(force, b.pos, vel, synth.SPECIES_MASS[b.species], 0.5, 12)
    assert np.abs(_min_image(x - xr, b)).max() < 1e-9
    assert np.abs(v - vr).max() < 1e-9
    assert abs(E[0] - Er[-1][0]) <= 1e-5 * abs(Er[-1][0])


def test_nve_energy_conservation():
    import torch
    cfg, b = synth.single_config(n=600)
    vel = synth.maxwell_boltzmann(b, 300.0, np.random.default_rng(53))
    m = model(cfg, 2)
    mass = synth.SPECIES_MASS[b.species]
    x0, v0, E0, md = _run_gpu(m, b, vel, 0, 0.5)
    tot0 = E0[0] + omd.kinetic_energy(v0, mass)
    d = device()
    E = torch.empty(1, dtype=torch.float64, device=d)
    totals = []
    for _ in range(10):
        md.step(40, 0.5, E)
        _, v, _ = md.state()
        torch.cuda.synchronize()
        totals.append(E.item() + omd.kinetic_energy(v.cpu().numpy(), mass))
    ke = omd.kinetic_energy(v0, mass)
    drift = max(abs(t - tot0) for t in totals)
    say(f"NVE 400 steps: max |dE_total| {drift:.3e} eV (KE {ke:.3f} eV)")
    assert drift < 1e-4 * ke
    steps, rebuilds, violations = md.stats()
    # at least every 20 steps; earlier when the forecast displacement reaches
    # skin/2, or after a step that overran it
    assert steps == 400 and rebuilds >= 20 and rebuilds >= violations


@pytest.mark.parametrize("skin", [0.0, 0.1])
def test_skin_overrun_rebuilds_within_the_step(skin):
    # No scheduled rebuild within the run: every rebuild is an early one. With
    # skin 0 every drift overruns skin/2, and each step is redone on new lists
    # after its force evaluation was queued (46 pairs enter the cutoff over
    # these 12 steps, so a step left on stale lists would leave the oracle's
    # trajectory, which finds its neighbours anew every step). With skin 0.1
    # the drift's forecast mostly brings the rebuild forward instead.
    cfg = synth.ModelConfig(lmax=2, channels=32, layers=2, n_species=4, cutoff=5.0, avg_neighbors=10.0)
    b = synth.jittered_lattice(40, 0.1, 0.3, 4, np.random.default_rng(51))
    vel = synth.maxwell_boltzmann(b, 600.0, np.random.default_rng(55))
    m = model(cfg, 7)
    say(f"skin guard skin={skin}")
    x, v, E, md = _run_gpu(m, b, vel, 12, 0.5, rebuild_every=1000, skin=skin)
    steps, rebuilds, violations = md.stats()
    say(f"  steps {steps}, rebuilds {rebuilds}, overruns {violations}")
    assert steps == 12
    if skin == 0.0:
        assert violations == 12 and rebuilds == 12
    else:
        assert 2 <= rebuilds <= 12 and violations <= rebuilds
    om_m = om.Model(cfg, synth.model_weights(cfg, 7))

    def force(xx):
        Es, F, _ = om.energy_forces(om_m, synth.Batch(xx, b.species, b.cell, b.pbc, b.offsets))
        return Es, F
    xr, vr, Er = omd.velocity_verlet(force, b.pos, vel, synth.SPECIES_MASS[b.species], 0.5, 12)
    assert np.abs(_min_image(x - xr, b)).max() < 1e-9
    assert np.abs(v - vr).max() < 1e-9
    assert abs(E[0] - Er[-1][0]) <= 1e-5 * abs(Er[-1][0])


def test_packed_trajectories_equal_single():
    cfg, b, _, _ = synth.differentiation_config(4, 30, 80)
    vel = synth.maxwell_boltzmann(b, 300.0, np.random.default_rng(54))
    m = model(cfg, 3)
    x, v, E, _ = _run_gpu(m, b, vel, 25, 0.5, rebuild_every=10, skin=0.8)
    for s in (1, 2):
        a, z = b.offsets[s], b.offsets[s + 1]
        xs, vs, Es, _ = _run_gpu(m, b.structure(s), vel[a:z], 25, 0.5, rebuild_every=10, skin=0.8)
        assert np.array_equal(xs, x[a:z]) and np.array_equal(vs, v[a:z]) and Es[0] == E[s]


def _two_structures():
    b1 = synth.jittered_lattice(30, 0.1, 0.3, 4, np.random.default_rng(61))
    b2 = synth.jittered_lattice(40, 0.1, 0.3, 4, np.random.default_rng(62))
    return synth.concat([b1, b2])


@pytest.mark.parametrize("rebuild_every", [4, 20])
def test_langevin_trajectory_matches_oracle(rebuild_every):
    import torch
    import paper_2605_22698_amd as e3
    cfg = synth.ModelConfig(lmax=2, channels=32, layers=2, n_species=4, cutoff=5.0, avg_neighbors=10.0)
    b = _two_structures()
    vel = synth.maxwell_boltzmann(b, 300.0, np.random.default_rng(63))
    m = model(cfg, 7)
    seeds, step0 = [7, 9], [3, 11]
    T, gamma, dt, n = 300.0, 0.05, 0.5, 12
    say(f"langevin parity rebuild_every={rebuild_every}")
    d = device()
    md = e3.MD(m, b.offsets, torch.tensor(b.pos, dtype=torch.float64, device=d),
               torch.tensor(vel, dtype=torch.float64, device=d), torch.tensor(b.species, dtype=torch.int32, device=d),
               synth.SPECIES_MASS[:cfg.n_species], b.cell, b.pbc, cfg.cutoff, 1.0, rebuild_every)
    md.set_langevin(T, gamma, seeds, step0)
    E = torch.empty(b.n_structures, dtype=torch.float64, device=d)
    md.step(n, dt, E)
    x, v, _ = md.state()
    torch.cuda.synchronize()
    x, v, E = x.cpu().numpy(), v.cpu().numpy(), E.cpu().numpy()
    om_m = om.Model(cfg, synth.model_weights(cfg, 7))

    def force(xx):
        Es, F, _ = om.energy_forces(om_m, synth.Batch(xx, b.species, b.cell, b.pbc, b.offsets))
        return Es, F
    xr, vr, Er = omd.langevin_baoab(force, b.pos, vel, synth.SPECIES_MASS[b.species], dt, n, T, gamma, b.offsets,
                                    seeds, step0)
    assert np.abs(_min_image(x - xr, b)).max() < 1e-9
    assert np.abs(v - vr).max() < 1e-9
    assert np.all(np.abs(E - Er[-1]) <= 1e-5 * np.abs(Er[-1]))
    # the thermostat acted: the trajectory is not the velocity-Verlet one
    xv, _, _ = omd.velocity_verlet(force, b.pos, vel, synth.SPECIES_MASS[b.species], dt, n)
    assert np.abs(_min_image(xv - xr, b)).max() > 1e-6


def test_langevin_packed_equals_alone():
    import torch
    import paper_2605_22698_amd as e3
    cfg, b, _, _ = synth.differentiation_config(3, 30, 80)
    vel = synth.maxwell_boltzmann(b, 300.0, np.random.default_rng(64))
    m = model(cfg, 3)
    d = device()
    seeds = [101, 202, 303]
    step0 = [0, 5, 17]

    def run(bb, vv, sd, s0):
        md = e3.MD(m, bb.offsets, torch.tensor(bb.pos, dtype=torch.float64, device=d),
                   torch.tensor(vv, dtype=torch.float64, device=d),
                   torch.tensor(bb.species, dtype=torch.int32, device=d), synth.SPECIES_MASS[:cfg.n_species],
                   bb.cell, bb.pbc, cfg.cutoff, 0.8, 10)
        md.set_langevin(300.0, 0.02, sd, s0)
        md.step(25, 0.5)
        x, v, _ = md.state()
        torch.cuda.synchronize()
        return x.cpu().numpy(), v.cpu().numpy()
    x, v = run(b, vel, seeds, step0)
    for s in range(3):
        a, z = b.offsets[s], b.offsets[s + 1]
        xs, vs = run(b.structure(s), vel[a:z], [seeds[s]], [step0[s]])
        assert np.array_equal(xs, x[a:z]) and np.array_equal(vs, v[a:z])


def test_langevin_equilibrates_to_target_temperature():
    import torch
    import paper_2605_22698_amd as e3
    cfg, b = synth.single_config(n=300)
    m = model(cfg, 2)
    d = device()
    mass = synth.SPECIES_MASS[b.species]
    md = e3.MD(m, b.offsets, torch.tensor(b.pos, dtype=torch.float64, device=d),
               torch.zeros((b.n_atoms, 3), dtype=torch.float64, device=d),
               torch.tensor(b.species, dtype=torch.int32, device=d), synth.SPECIES_MASS[:cfg.n_species],
               b.cell, b.pbc, cfg.cutoff, 1.0, 20)
    T = 300.0
    md.set_langevin(T, 0.1, [2026])
    md.step(600, 0.5)
    temps = []
    for _ in range(100):
        md.step(10, 0.5)
        _, v, _ = md.state()
        torch.cuda.synchronize()
        ke = omd.kinetic_energy(v.cpu().numpy(), mass)
        temps.append(2.0 * ke / (3.0 * b.n_atoms * omd.KB_EV))
    t_mean = float(np.mean(temps))
    say(f"Langevin NVT: mean T {t_mean:.1f} K (target {T} K)")
    assert abs(t_mean / T - 1.0) < 0.05


def test_npt_trajectory_matches_oracle():
    # Langevin + Monte Carlo barostat: positions, velocities, cells and the
    # accept/reject decisions of 3 proposals per structure agree with the oracle
    import torch
    import paper_2605_22698_amd as e3
    cfg = synth.ModelConfig(lmax=2, channels=32, layers=2, n_species=4, cutoff=5.0, avg_neighbors=10.0)
    b = _two_structures()
    vel = synth.maxwell_boltzmann(b, 300.0, np.random.default_rng(63))
    m = model(cfg, 7)
    T, gamma, dt, n, P, interval, frac = 300.0, 0.05, 0.5, 12, 1000.0, 4, 0.01
    # the two structures are on different proposal schedules (step counts 3 and 10)
    seeds, step0, bseeds, move0 = [7, 9], [3, 10], [21, 22], [0, 5]
    say("npt parity")
    d = device()
    md = e3.MD(m, b.offsets, torch.tensor(b.pos, dtype=torch.float64, device=d),
               torch.tensor(vel, dtype=torch.float64, device=d), torch.tensor(b.species, dtype=torch.int32, device=d),
               synth.SPECIES_MASS[:cfg.n_species], b.cell, b.pbc, cfg.cutoff, 1.0, 20)
    md.set_langevin(T, gamma, seeds, step0)
    md.set_barostat(P, interval, frac, bseeds, move0)
    E = torch.empty(b.n_structures, dtype=torch.float64, device=d)
    md.step(n, dt, E)
    x, v, _ = md.state()
    torch.cuda.synchronize()
    x, v, E = x.cpu().numpy(), v.cpu().numpy(), E.cpu().numpy()
    cells, proposed, accepted = md.cells()
    om_m = om.Model(cfg, synth.model_weights(cfg, 7))

    def force(xx, boxes):
        cell = np.array([np.diag(bb) for bb in boxes])
        Es, F, _ = om.energy_forces(om_m, synth.Batch(xx, b.species, cell, b.pbc, b.offsets))
        return Es, F
    boxes0 = np.array([np.diag(c) for c in b.cell])
    xr, vr, boxes, Er, dec = omd.langevin_npt(force, b.pos, vel, boxes0, synth.SPECIES_MASS[b.species], dt, n, T,
                                              gamma, b.offsets, seeds, step0, P, interval, frac, bseeds, move0)
    dec = np.array([a for _, a in dec])
    assert proposed == dec.size and accepted == int(dec.sum())
    assert 0 < accepted < proposed  # both outcomes exercised
    assert np.abs(np.array([np.diag(c) for c in cells]) - boxes).max() < 1e-12
    assert np.abs(x - xr).max() < 1e-9  # positions are unwrapped on both sides
    assert np.abs(v - vr).max() < 1e-9
    assert np.all(np.abs(E - Er[-1]) <= 1e-5 * np.abs(Er[-1]))
