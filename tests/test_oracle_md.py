"""Pins of the oracle's velocity-Verlet and Langevin integrators."""
import math

import numpy as np

import synth
from oracle import md
from oracle import md as omd
from oracle import model as om


def test_harmonic_oscillator_matches_exact_solution():
    k, mass, x0 = 2.0, 12.0, 0.3
    omega = math.sqrt(k * md.ACCEL_UNIT / mass)

    def force(x):
        return np.zeros(1), -k * x
    dt, n = 0.5, 400
    x, v, _ = md.velocity_verlet(force, np.array([[x0, 0, 0]]), np.zeros((1, 3)), np.array([mass]), dt, n)
    # Velocity Verlet on a harmonic oscillator is a rotation in phase space
    # with the modified frequency 2/dt asin(omega dt / 2).
    om_mod = 2.0 / dt * math.asin(omega * dt / 2.0)
    assert abs(x[0, 0] - x0 * math.cos(om_mod * n * dt)) < 1e-12
    assert abs(x[0, 0] - x0 * math.cos(omega * n * dt)) < 1e-3 * x0


def _model_system():
    cfg = synth.ModelConfig(lmax=2, channels=8, layers=2, n_species=4, cutoff=5.0, avg_neighbors=10.0)
    m = om.Model(cfg, synth.model_weights(cfg, 21))
    b = synth.jittered_lattice(16, 0.1, 0.3, 4, np.random.default_rng(22))
    v = synth.maxwell_boltzmann(b, 300.0, np.random.default_rng(23))

    def force(x):
        E, F, _ = om.energy_forces(m, synth.Batch(x, b.species, b.cell, b.pbc, b.offsets))
        return E, F
    return b, v, force, synth.SPECIES_MASS[b.species]


def test_reversible_and_momentum_conserving():
    b, v, force, mass = _model_system()
    x1, v1, _ = md.velocity_verlet(force, b.pos, v, mass, 0.5, 10)
    p0 = (mass[:, None] * v).sum(0)
    p1 = (mass[:, None] * v1).sum(0)
    np.testing.assert_allclose(p1, p0, atol=1e-13)
    x2, v2, _ = md.velocity_verlet(force, x1, -v1, mass, 0.5, 10)
    np.testing.assert_allclose(x2, b.pos, atol=1e-11)
    np.testing.assert_allclose(-v2, v, atol=1e-12)


def test_energy_conservation():
    b, v, force, mass = _model_system()
    E0, _ = force(b.pos)
    tot0 = E0[0] + md.kinetic_energy(v, mass)
    x, v1, Es = md.velocity_verlet(force, b.pos, v, mass, 0.25, 40)
    tot1 = Es[-1][0] + md.kinetic_energy(v1, mass)
    assert abs(tot1 - tot0) < 1e-3 * max(1e-3, md.kinetic_energy(v, mass))


def test_maxwell_boltzmann_temperature():
    b = synth.jittered_lattice(2000, 0.1, 0.3, 5, np.random.default_rng(1))
    v = synth.maxwell_boltzmann(b, 300.0, np.random.default_rng(2))
    ke = md.kinetic_energy(v, synth.SPECIES_MASS[b.species])
    T = 2 * ke / (3 * b.n_atoms * synth.KB_EV)
    assert abs(T - 300.0) < 15.0
    np.testing.assert_allclose((synth.SPECIES_MASS[b.species][:, None] * v).sum(0), 0, atol=1e-12)


def test_langevin_without_friction_is_velocity_verlet():
    rng_np = np.random.default_rng(3)
    x0 = rng_np.normal(size=(5, 3))
    v0 = rng_np.normal(size=(5, 3)) * 0.01
    m = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    k = 2.5

    def force(x):
        return np.array([0.5 * k * np.sum(x * x)]), -k * x
    xa, va, _ = omd.velocity_verlet(force, x0, v0, m, 0.7, 30)
    xb, vb, _ = omd.langevin_baoab(force, x0, v0, m, 0.7, 30, 300.0, 0.0, [0, 5], [11], [0])
    assert np.abs(xa - xb).max() < 1e-12 and np.abs(va - vb).max() < 1e-12


def test_langevin_samples_boltzmann_temperature_in_harmonic_well():
    # independent atoms in a harmonic well: <m v^2/kappa> = kB T per component and
    # <k x^2> = kB T (BAOAB samples the configurational distribution of a
    # harmonic well with an error of order (dt omega)^2 ~ 1e-3 here)
    n, T, k, gamma, dt = 60, 300.0, 1.0, 0.05, 1.0
    m = np.full(n, 12.0)
    x0 = np.zeros((n, 3))
    v0 = np.zeros((n, 3))

    def force(x):
        return np.array([0.5 * k * np.sum(x * x)]), -k * x
    kT = omd.KB_EV * T
    # warm up, then average over a second stretch
    x, v, _ = omd.langevin_baoab(force, x0, v0, m, dt, 300, T, gamma, [0, n], [5], [0])
    ke, pe, cnt = 0.0, 0.0, 0
    for block in range(8):
        x, v, _ = omd.langevin_baoab(force, x, v, m, dt, 100, T, gamma, [0, n], [5], [300 + 100 * block])
        ke += np.mean(m[:, None] * v * v / omd.ACCEL_UNIT)
        pe += np.mean(k * x * x)
        cnt += 1
    assert abs(ke / cnt / kT - 1.0) < 0.08
    assert abs(pe / cnt / kT - 1.0) < 0.08


def test_mc_barostat_ideal_gas_volume():
    # E = 0: the volume moves alone sample p(V) ~ V^N exp(-P V / kT),
    # so <V> = (N + 1) kT / P (about 174 A^3 here; proposals up to +-60 A^3)
    n, T, P_bar = 20, 300.0, 5000.0
    kT = omd.KB_EV * T
    P = P_bar * omd.BAR_EV_A3
    x = np.random.default_rng(5).uniform(0, 10, size=(n, 3))
    boxes = np.array([[10.0, 10.0, 10.0]])
    E = np.zeros(1)
    vols = []
    for mv in range(6000):
        x, boxes, E, _ = omd.barostat_move(lambda xx, bb: np.zeros(1), x, boxes, E, [0, n], T, P_bar, [60.0],
                                           [17], [mv])
        if mv >= 1000:
            vols.append(np.prod(boxes[0]))
    expect = (n + 1) * kT / P
    assert abs(np.mean(vols) / expect - 1.0) < 0.05
    # and the relative fluctuation of an ideal gas, 1 / sqrt(N + 1)
    assert abs(np.std(vols) / np.mean(vols) * np.sqrt(n + 1) - 1.0) < 0.15


def test_npt_without_moves_is_langevin():
    rng_np = np.random.default_rng(8)
    x0 = rng_np.normal(size=(6, 3))
    v0 = rng_np.normal(size=(6, 3)) * 0.01
    m = np.full(6, 4.0)

    def force(x, boxes=None):
        return np.array([0.5 * np.sum(x * x)]), -x
    xa, va, _ = omd.langevin_baoab(force, x0, v0, m, 0.5, 10, 300.0, 0.1, [0, 6], [3], [0])
    xb, vb, bb, _, dec = omd.langevin_npt(force, x0, v0, np.array([[9.0, 9.0, 9.0]]), m, 0.5, 10, 300.0, 0.1,
                                          [0, 6], [3], [0], 1.0, 100, 0.01, [4], [0])
    assert not dec and np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(bb, [[9.0, 9.0, 9.0]])


def test_npt_schedule_is_per_structure_and_packing_independent():
    # Batched independent simulations (Section 5.5): each structure proposes a
    # volume move after the steps that bring its OWN step count (step0 + steps
    # taken) to a multiple of the interval, and a structure's trajectory is the
    # same alone and packed with another on a different phase.
    rng_np = np.random.default_rng(41)
    n = (5, 4)
    off = [0, n[0], n[0] + n[1]]
    x0 = rng_np.uniform(0.0, 8.0, size=(sum(n), 3))
    v0 = rng_np.normal(size=(sum(n), 3)) * 0.01
    m = np.full(sum(n), 12.0)
    boxes0 = np.array([[8.0, 8.0, 8.0], [7.5, 7.5, 7.5]])
    kspring = 0.05

    def force(x, boxes, offsets=off):
        # each structure in a harmonic well at its box centre (energy changes with the volume)
        E = np.zeros(len(offsets) - 1)
        F = np.zeros_like(x)
        for s in range(len(offsets) - 1):
            a, b = offsets[s], offsets[s + 1]
            d = x[a:b] - 0.5 * boxes[s]
            E[s] = 0.5 * kspring * np.sum(d * d)
            F[a:b] = -kspring * d
        return E, F

    interval, steps = 5, 13
    step0, seeds, bseeds, move0 = [0, 3], [11, 12], [21, 22], [0, 7]
    xp, vp, bp, Ep, dec = omd.langevin_npt(force, x0, v0, boxes0, m, 0.5, steps, 300.0, 0.05, off, seeds, step0,
                                           2000.0, interval, 0.02, bseeds, move0)
    # structure 0 proposes after its steps 5 and 10; structure 1 (3 steps in) after 2, 7 and 12
    assert [s for s, _ in dec] == [1, 0, 1, 0, 1]
    for s in range(2):
        a, b = off[s], off[s + 1]
        lo = [0, b - a]

        def force_s(x, boxes, s=s):
            return force(x, boxes, offsets=lo)
        xs, vs, bs, Es, ds = omd.langevin_npt(force_s, x0[a:b], v0[a:b], boxes0[s:s + 1], m[a:b], 0.5, steps, 300.0,
                                              0.05, lo, [seeds[s]], [step0[s]], 2000.0, interval, 0.02, [bseeds[s]],
                                              [move0[s]])
        assert np.array_equal(xs, xp[a:b]) and np.array_equal(vs, vp[a:b]) and np.array_equal(bs[0], bp[s])
        assert [acc for _, acc in ds] == [acc for q, acc in dec if q == s]
        assert [float(e[0]) for e in Es] == [float(e[s]) for e in Ep]
    assert not np.array_equal(bp, boxes0)  # some move was accepted
