#!/usr/bin/env python3
"""Throughput of the equivariant interaction on one MI355X.

A step is one velocity-Verlet MD step of the whole hot path on a 3,000-atom
periodic box (0.1 atoms/A^3, jittered lattice, 4 species, r_c 5 A, l_max 3,
128 channels, 2 layers, FP32): half kick, drift, edge selection inside the
cutoff from the skin list, radial MLP, tensor product + neighbour sum,
channel mix, gate, readout, FP64 energy sum, the full adjoint to forces, half
kick; the neighbour lists are rebuilt on the device every 20 steps (skin 1 A).
Inputs are synthetic and resident in HBM before timing starts.

Prints one JSON line: atom-steps/s, the roofline position of the dominant
kernel (timed live with HIP events on the launch stream), and the FP64 CPU
oracle timed on a bounded sample on the host cores.
"""
import argparse
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12        # bytes/s
PEAK_FP32_MFMA = 157.3e12
PEAK_FP32_VALU = 157.3e12           # datasheet, counts packed FP32
PEAK_FP32_VALU_NONPACKED = 78.65e12  # 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
# kernels that run a stage in place of the general one: (stage, last layer) -> kernel
KERNEL_OF_STAGE = {("tp_bwd_edge", True): "k_tps_bwd_sender", ("tp_bwd_node", False): "k_tp_msg_node"}
KAPPA = 0.009648533


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cg_nnz():
    """Nonzeros per path of the compiled CG table (for the algorithmic flop model)."""
    text = open(os.path.join(ROOT, "paper_2605_22698_amd", "csrc", "cg_tables.inc")).read()

    def arr(name):
        m = re.search(name + r"\[[^\]]*\] = \{([^}]*)\}", text)
        return [int(x) for x in m.group(1).split(",")]
    b = arr("kNzBegin")
    return arr("kL1"), arr("kL2"), arr("kL3"), [b[i + 1] - b[i] for i in range(len(b) - 1)]


def layer_paths(cfg, t):
    L1, L2, L3, NZ = cg_nnz()
    l1max = 0 if t == 1 else cfg.lmax
    # the last layer evaluates its scalar outputs only, except with the product
    # block (which needs every order of A~)
    l3max = 0 if t == cfg.layers and getattr(cfg, "correlation", 1) != 2 else cfg.lmax
    return [(L1[g], L2[g], L3[g], NZ[g]) for g in range(len(L1))
            if L1[g] <= l1max and L2[g] <= cfg.lmax and L3[g] <= l3max]


def work_model(cfg, t, E, N, pairs=False):
    """Algorithmic (flops, HBM bytes) of one launch of each stage of layer t.
    pairs: the layer's radial MLP runs once per edge pair and R is stored once
    per pair (an unchunked layer in an energy+forces evaluation); every pruned
    edge has its reverse in the list, so there are E / 2 pairs."""
    C = cfg.channels
    P = (E + 1) // 2 if pairs else E   # radial MLP evaluations = R rows
    ps = layer_paths(cfg, t)
    PC = len(ps) * C
    nc_in = 1 if t == 1 else (cfg.lmax + 1) ** 2
    nout = sum(2 * l3 + 1 for (_, _, l3, _) in ps)
    H = cfg.radial_hidden
    mlp_hidden = 2 * (cfg.n_basis * H + H * H)
    tp_flops = 2 * C * sum(nz + 2 * l3 + 1 for (_, _, l3, nz) in ps)
    out = {}
    # species-factorised first layer: the hidden MLP's pre-activation P2 once
    # per edge pair (the first layer is never chunked; stored, 4 H bytes),
    # the outer product per edge, G per atom; the adjoint reads P2 per edge
    # (no hidden-layer recompute)
    nc3 = (cfg.lmax + 1) ** 2 if cfg.layers > 1 else 1
    s64 = cfg.n_species * H
    Ph = (E + 1) // 2
    out["first_fwd"] = (Ph * mlp_hidden + E * 2 * H * nc3, Ph * (16 + 4 * H) + E * (24 + 4 * H) + N * 4 * nc3 * s64)
    out["first_bwd"] = (E * (2 * H * H + 2 * H * cfg.n_basis + 4 * H * nc3),
                        E * (24 + 16 + 4 * H) + N * 4 * nc3 * s64)
    # fused last layer (scalar outputs): hidden MLP, T = sum_e H2 s^T and its
    # W3 contraction forward; R recomputed, dH2 = W3 dR, MLP adjoint, and the
    # contracted-feature terms backward. Bytes: edge vectors, h once per atom,
    # A / dA once per atom, g read and written.
    NL = cfg.lmax + 1
    NY = (cfg.lmax + 1) ** 2
    out["last_fwd"] = (E * (mlp_hidden + 2 * H * NL * C + 2 * C * NY) + N * 2 * H * NL * C,
                       E * 20 + N * 4 * (NY * C + NL * C))
    out["last_bwd"] = (E * (mlp_hidden + 4 * H * NL * C + 2 * H * H + 2 * H * cfg.n_basis + 6 * C * NY),
                       E * (20 + 32) + N * 4 * (3 * NY * C + NL * C))
    # radial MLP: flops on the matrix cores; bytes = edge vectors in, R out
    # (per pair: the owner's edge vector and its owner and reverse indices)
    out["radial_fwd"] = (P * (mlp_hidden + 2 * H * PC), P * (16 + 4 * PC + (8 if pairs else 0)))
    # adjoint: recompute hidden layers, dR W3^T, dH2 W2^T, dH1 W1^T; dR and dY
    # of every edge in (summed per pair), g read+write
    out["radial_bwd"] = (P * (mlp_hidden + 2 * H * PC + 2 * H * H + 2 * H * cfg.n_basis),
                         E * (16 + 4 * PC + 64 + 32) + (P * 8 if pairs else 0))
    # tensor product + neighbour sum: R streamed once (each pair's row, found
    # through the edge's pair index), h read and A written once per atom
    r_in = P * 4 * PC + (E * 4 if pairs else 0)
    out["tp_fwd"] = (E * tp_flops, r_in + E * (16 + 4) + N * 4 * C * (nc_in + nout))
    edge_adj = E * (tp_flops + 2 * C * sum(nz for *_, nz in ps) + 2 * C * nout)
    node_adj = E * 2 * C * sum(nz + 2 * l3 + 1 for (_, _, l3, nz) in ps)
    if t == cfg.layers and C in (64, 128, 256) and getattr(cfg, "correlation", 1) != 2:
        # scalar-output layer: the sender-side adjoint (tps.hip) gives dR, dY
        # and dh in one pass: R read once, dR and dY written, edge vector, sender
        # and reverse index per edge; h, dA and dh (read and written) once per atom
        out["tp_bwd_edge"] = (edge_adj + (node_adj if t > 1 else 0),
                              r_in + E * (4 * PC + 64 + 16 + 4 + 4)
                              + N * 4 * C * (nc_in + nout + (2 * nc_in if t > 1 else 0)))
    elif t > 1:
        # every path: the edge adjoint also writes each edge's sender-gradient
        # message (nc_in x C values); the node pass reads the messages of each
        # sender's edges (and the reverse index) and reads/writes dh once
        out["tp_bwd_edge"] = (edge_adj + 2 * E * C * sum(nz for *_, nz in ps),
                              r_in + E * (4 * PC + 16 + 4 + 64 + 4 * nc_in * C) + N * 4 * C * (nc_in + nout))
        out["tp_bwd_node"] = (E * nc_in * C, E * (4 * nc_in * C + 8) + N * 4 * C * 2 * nc_in)
    else:
        out["tp_bwd_edge"] = (edge_adj, r_in + E * (4 * PC + 16 + 4 + 64) + N * 4 * C * (nc_in + nout))
        out["tp_bwd_node"] = (node_adj, r_in + E * (16 + 4) + N * 4 * C * (nc_in + nout))
    return out


def fp32_row_pattern(cfg, kern, t):
    """The FP32-mode instantiation of a per-edge kernel of layer t, as the
    100,000-atom traffic summary lists it: the radial kernels serve several
    layers (rows split by layer), the tensor-product kernels are per layer
    kind by their template arguments (1: every path, 2: scalar outputs)."""
    kind = 2 if t == cfg.layers else 1
    # chunked layers run the per-edge instantiations (radial mode 0 / no
    # pairs, R rows without the pair index)
    if kern.startswith("k_radial"):
        return re.escape(kern) + r"<8, (\d+, )?false, float, (0|false)> \[layer %d\]" % t
    if kern in ("k_tp_fwd", "k_tp_bwd_edge", "k_tps_bwd_sender"):
        return re.escape(kern) + r"<%d, %d, \d+(, (true|false))?, float(, false)?>" % (cfg.lmax, kind)
    return re.escape(kern) + r"(<.*>)?"


def measured_traffic(kernel, summary="md_step_3000_hbm_traffic.md", pattern=None):
    """HBM bytes per launch of a kernel (FETCH_SIZE + WRITE_SIZE,
    copy-calibrated) from a committed counter summary, or None when the
    kernel's source file has changed since the counters were taken. kernel:
    the name as listed, with its template arguments or without (the first
    listed); pattern (a regular expression), when given, must match the
    listed name whole instead."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    for line in open(path):
        m = re.match(r"\|\s*`([^`]+)`\s*\|\s*\d+\s*\|\s*([\d.]+)\s*\|\s*([\d.]+)\s*\|\s*(\S+)\s*\|\s*(\S+)", line)
        if not m:
            continue
        name = m.group(1)
        hit = re.fullmatch(pattern, name) if pattern else kernel in (name, name.split("<")[0])
        if not hit:
            continue
        src = os.path.join(ROOT, "paper_2605_22698_amd", "csrc", m.group(4))
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != m.group(5):
            return None
        return (float(m.group(2)) + float(m.group(3))) * 1024 * 1024
    return None


def serving_run(e3, synth, torch, dev, n_requests, n_steps, log):
    """Continuous-batching MD: Poisson arrivals, atom counts log-uniform in
    [50, 5000], 0.1 atoms/A^3, 4 species, l_max 3, 128 channels, FP32,
    0.5 fs steps at 300 K, rebuild every 20 steps, n_steps steps per request;
    arrival rate set so the offered load is about 80% of a measured capacity.
    Run twice: with the device's memory as the admission budget, and with a
    budget of about four mean-size requests or the largest one (requests then
    queue)."""
    from paper_2605_22698_amd.serving import GpuExecutor, Request, Server
    cfg = synth.serving_model()
    m = e3.Model(cfg.to_json(), synth.flatten_weights(cfg, synth.model_weights(cfg, 4)), device=dev)
    reqs = synth.serving_requests(n_requests, rate_per_s=1.0)
    mean_atoms = float(np.mean([r[1].n_atoms for r in reqs]))
    # capacity probe: one packed batch of the first requests
    ex = GpuExecutor(m, synth.SPECIES_MASS[:4], cfg.cutoff)
    probe = [ex.upload(Request(k, 0.0, b.pos, v, b.species, b.cell[0], b.pbc[0], 1))
             for k, (_, b, v) in enumerate(reqs[:4])]
    ex.launch(probe)
    ex.step()
    ms = np.median([ex.step() for _ in range(5)])
    ex.close()
    cap = sum(p["pos"].shape[0] for p in probe) / (ms / 1e3)          # atom-steps/s
    rate = 0.8 * cap / (mean_atoms * n_steps)                          # requests/s
    arr = np.cumsum(np.random.default_rng(synth.MASTER_SEED).exponential(1.0 / rate, size=len(reqs)))
    device_bytes = int(torch.cuda.get_device_properties(dev).total_memory)
    # about four mean-size requests, and never less than the largest one (none is refused)
    small = int(ex.footprint(int(max(4 * mean_atoms, 1.1 * max(r[1].n_atoms for r in reqs)))))
    out = {"requests": len(reqs), "steps_per_request": n_steps, "mean_atoms": mean_atoms, "arrival_rate_per_s": rate,
           "note": "step_ms: device time of each packed step; iter_ms: wall time of each engine iteration, "
                   "repacks included"}
    for name, budget in (("device_budget", device_bytes), ("small_budget", small)):
        srv = Server(GpuExecutor(m, synth.SPECIES_MASS[:4], cfg.cutoff), budget_bytes=budget)
        for k, ((_, b, v), t) in enumerate(zip(reqs, arr)):
            srv.submit(Request(k, float(t), b.pos, v, b.species, b.cell[0], b.pbc[0], n_steps))
        stats = srv.run(idle_wait=lambda dt: time.sleep(min(dt, 0.01)))
        summ = stats.summary()
        waits = [r.admitted_at - r.arrival for r in srv.done if r.admitted_at is not None]
        lat = [r.finished_at - r.arrival for r in srv.done if r.finished_at is not None]
        log(f"serving ({name}): {summ}")
        out[name] = {"budget_bytes": budget, "rejected": summ["rejected"],
                     "p50_step_ms": summ["p50_ms"], "p99_step_ms": summ["p99_ms"],
                     "p50_iter_ms": summ["p50_iter_ms"], "p99_iter_ms": summ["p99_iter_ms"],
                     "atom_steps_per_s": summ["atom_steps_per_s"],
                     "atom_steps_per_busy_s": summ["atom_steps_per_busy_s"], "repacks": summ["repacks"],
                     "p50_queue_wait_s": float(np.percentile(waits, 50)) if waits else 0.0,
                     "p99_queue_wait_s": float(np.percentile(waits, 99)) if waits else 0.0,
                     "p50_request_latency_s": float(np.percentile(lat, 50)) if lat else 0.0,
                     "p99_request_latency_s": float(np.percentile(lat, 99)) if lat else 0.0,
                     "wall_s": summ["wall_s"]}
    m.close()
    return out


def product_work(cfg, t, N):
    """Algorithmic (flops, HBM bytes) of one launch of the product block of
    layer t, forward and adjoint, per (atom, channel): forward 3 flops per CG
    nonzero of each coupling (l1 <= l2, L <= Lo), 2 per output component of
    each coupling for its weight, 1 per component of B for the linear term;
    adjoint 5 per nonzero (both factors), 1 per output component of each
    coupling, 1 per component of B. Bytes = A~ in and B out (forward), A~ and
    dB in and dA~ out (adjoint)."""
    L1, L2, L3, NZ = cg_nnz()
    lo = 0 if t == cfg.layers else cfg.lmax
    na, nb = (cfg.lmax + 1) ** 2, (lo + 1) ** 2
    sel = [g for g in range(len(L1)) if L1[g] <= L2[g] <= cfg.lmax and L3[g] <= lo]
    nz = sum(NZ[g] for g in sel)
    nout = sum(2 * L3[g] + 1 for g in sel)
    per_fwd = 3 * nz + 2 * nout + nb
    per_bwd = 5 * nz + nout + nb
    NCn = N * cfg.channels
    return {"product_fwd": (per_fwd * NCn, 4 * NCn * (na + nb)),
            "product_bwd": (per_bwd * NCn, 4 * NCn * (2 * na + nb))}


def product_run(e3, synth, torch, dev, n_atoms, steps, warmup, log):
    """MD of the single-structure box with the product block of body order 2
    (MACE's symmetric contraction, correlation 2) in both layers; the dominant
    product kernel against HBM; one Hessian-vector product and one
    parameter gradient of that model on the box."""
    cfg1, b = synth.single_config(n=n_atoms)
    cfg = synth.ModelConfig(**{**cfg1.__dict__, "correlation": 2})
    vel = synth.maxwell_boltzmann(b, 300.0, synth.seed_for(2, 9))
    pos_d = torch.tensor(b.pos, dtype=torch.float64, device=dev)
    vel_d = torch.tensor(vel, dtype=torch.float64, device=dev)
    sp_d = torch.tensor(b.species, dtype=torch.int32, device=dev)
    energy = torch.empty(1, dtype=torch.float64, device=dev)
    m = e3.Model(cfg.to_json(), synth.flatten_weights(cfg, synth.model_weights(cfg, 2)), device=dev)
    md = e3.MD(m, b.offsets, pos_d, vel_d, sp_d, synth.SPECIES_MASS[:4], b.cell, b.pbc, cfg.cutoff, 1.0, 20)
    md.step(warmup, 0.5, energy)
    torch.cuda.synchronize()
    # the product kernels' times from a few fully timed steps, then the
    # timed region with only the slowest of them bracketed by events
    kp = max(5, steps // 5)
    m.profile(True)
    md.step(kp, 0.5, energy)
    torch.cuda.synchronize()
    m.profile(False)
    best = None
    stage = {}
    for t in range(1, cfg.layers + 1):
        for s, (flops, nbytes) in product_work(cfg, t, b.n_atoms).items():
            tot, n = m.stage_time(f"{s}@{t}")
            stage[f"{s}@{t}"] = tot / kp
            if n and (best is None or tot / n > best[0]):
                best = (tot / n, s, t, flops, nbytes)
    _, s, t, flops, nbytes = best
    m.profile(True, only=f"{s}@{t}")
    t1 = time.perf_counter()
    md.step(steps, 0.5, energy)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    m.profile(False)
    tot, n = m.stage_time(f"{s}@{t}")
    ms = tot / n
    out = {"workload": f"MD step, {b.n_atoms}-atom periodic box, l_max 3, 128 channels, 2 layers, "
                       f"product block of body order 2 in both layers (every layer keeps all orders of A~)",
           "value": b.n_atoms * steps / dt, "ms_per_step": 1e3 * dt / steps, "steps": steps}
    out["stage_ms_per_step"] = stage
    out["roofline"] = {"bound": "hbm", "achieved": nbytes / (ms / 1e3) / 1e9, "peak": PEAK_HBM / 1e9,
                       "unit": "GB/s", "frac": nbytes / (ms / 1e3) / PEAK_HBM,
                       "traffic": measured_traffic(f"k_{s}", "product_hbm_traffic.md"),
                       "kernel": f"{s} (layer {t})", "avg_launch_ms": ms,
                       "algorithmic_per_launch": {"flops": flops, "bytes": nbytes}}
    # the block's second-order pass on the same box: one Hessian-vector
    # product, and the weight gradient of an energy + force loss
    xpos, _, _ = md.state()
    g = m.build_graph(b.offsets, xpos, sp_d, b.cell, b.pbc, cfg.cutoff, 0.0)
    v = torch.randn((b.n_atoms, 3), generator=torch.Generator().manual_seed(11)).to(device=dev, dtype=torch.float32)
    gE = torch.ones(1, dtype=torch.float64, device=dev)
    gF = (0.01 * v).contiguous()

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) / k
    out["ms_hessian_vector_product"] = 1e3 * timed(lambda: m.hessian_vector(g, xpos, v), 5)
    out["ms_param_grad"] = 1e3 * timed(lambda: m.param_grad(g, xpos, gE, gF), 5)
    out["ms_energy_forces"] = 1e3 * timed(lambda: m.energy_forces(g, xpos), 10)
    g.close()
    md.close()
    log(f"product block: {out['value']:.3e} atom-steps/s; {s}@{t} {ms:.4f} ms, "
        f"{out['roofline']['achieved']:.0f} GB/s ({out['roofline']['frac']:.1%}); "
        f"Hessian-vector product {out['ms_hessian_vector_product']:.2f} ms, "
        f"parameter gradient {out['ms_param_grad']:.2f} ms")
    return out


def nve_run(e3, synth, torch, dev, n_atoms, steps, log):
    """Energy conservation of the MD path: NVE from 300 K on the
    single-structure box (0.5 fs, skin 1 A, rebuild every 20 steps) in FP32
    and in BF16 mode; the total energy (potential + kinetic, FP64) sampled
    every 100 steps. Reported: its largest deviation from the start and the
    slope of a least-squares line, per atom."""
    cfg, b = synth.single_config(n=n_atoms)
    vel = synth.maxwell_boltzmann(b, 300.0, synth.seed_for(2, 9))
    w = synth.flatten_weights(cfg, synth.model_weights(cfg, 2))
    mass = synth.SPECIES_MASS[b.species][:, None]
    amu_A2_fs2_to_eV = 1.0 / KAPPA
    out = {"workload": f"NVE from 300 K, {b.n_atoms}-atom periodic box (the benchmark box), 0.5 fs, "
                       f"{steps} steps, skin 1 A, rebuild every 20 steps", "steps": steps}
    for name, prec in (("fp32", e3.FP32), ("bf16", e3.BF16_MIX)):
        m = e3.Model(cfg.to_json(), w, precision=prec, device=dev)
        md = e3.MD(m, b.offsets, torch.tensor(b.pos, dtype=torch.float64, device=dev),
                   torch.tensor(vel, dtype=torch.float64, device=dev),
                   torch.tensor(b.species, dtype=torch.int32, device=dev), synth.SPECIES_MASS[:4], b.cell, b.pbc,
                   cfg.cutoff, 1.0, 20)
        energy = torch.empty(1, dtype=torch.float64, device=dev)
        t_ps, tot = [], []
        md.step(1, 0.5, energy)
        for k in range(0, steps + 1, 100):
            if k:
                md.step(100, 0.5, energy)
            _, v, _ = md.state()
            ke = 0.5 * float(np.sum(mass * v.cpu().numpy() ** 2)) * amu_A2_fs2_to_eV
            t_ps.append(k * 0.5e-3)
            tot.append(energy.item() + ke)
        tot = np.array(tot)
        slope = float(np.polyfit(np.array(t_ps), tot, 1)[0])
        _, rebuilds, violations = md.stats()
        out[name] = {"max_dev_meV_per_atom": 1e3 * float(np.abs(tot - tot[0]).max()) / b.n_atoms,
                     "drift_meV_per_atom_per_ps": 1e3 * slope / b.n_atoms,
                     "rebuilds": rebuilds, "skin_violations": violations}
        md.close()
        m.close()
        log(f"NVE {name}: max |dE| {out[name]['max_dev_meV_per_atom']:.4f} meV/atom, drift "
            f"{out[name]['drift_meV_per_atom_per_ps']:.4f} meV/atom/ps")
    return out


def capture_run(e3, synth, torch, dev, reps, log):
    """Launch-bound small inputs: energy+forces of the 24-atom cluster (l_max
    2, 32 channels) and of a 100-atom periodic box (the benchmark model),
    eager against a HIP graph of the allocation-free entry point replayed on
    the same buffers; microseconds per evaluation."""
    import ctypes
    from paper_2605_22698_amd import _lib
    out = {}
    cases = [("tiny_24_atoms", synth.tiny_config()),
             ("box_100_atoms", (synth.single_config(n=3000)[0],
                                synth.jittered_lattice(100, 0.1, 0.3, 4, np.random.default_rng(7))))]
    for name, (cfg, b) in cases:
        m = e3.Model(cfg.to_json(), synth.flatten_weights(cfg, synth.model_weights(cfg, 1)), device=dev)
        pos = torch.tensor(b.pos, dtype=torch.float64, device=dev)
        sp = torch.tensor(b.species, dtype=torch.int32, device=dev)
        g = m.build_graph(b.offsets, pos, sp, b.cell, b.pbc, cfg.cutoff, 1.0)
        E = torch.empty(b.n_structures, dtype=torch.float64, device=dev)
        F = torch.empty((b.n_atoms, 3), dtype=torch.float32, device=dev)

        def static_call():
            _lib.check(_lib.lib().e3mi_energy_forces_static(
                m.handle, g.handle, _lib.ptr(pos), _lib.ptr(E), _lib.ptr(F), None,
                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        static_call()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            with torch.cuda.graph(graph, stream=st):
                static_call()
        torch.cuda.current_stream().wait_stream(st)
        torch.cuda.synchronize()

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return 1e6 * (time.perf_counter() - t1) / reps
        out[name] = {"atoms": b.n_atoms, "eager_us": timed(lambda: m.energy_forces(g, pos)),
                     "graph_replay_us": timed(graph.replay)}
        g.close()
        m.close()
        log(f"{name}: eager {out[name]['eager_us']:.1f} us, graph replay {out[name]['graph_replay_us']:.1f} us")
    return out


def grad_run(e3, synth, torch, dev, reps, log, cpu_baseline=True):
    """Training step of the differentiation batch (64 periodic boxes of 20-200
    atoms, 5 species, l_max 3, 64 channels, 2 layers, FP32): loss = energy MSE
    + force MSE against seeded targets and its gradient with respect to every
    weight through the autograd Function (forward: energy+forces; backward:
    the library's second-order pass), timed per evaluation; the FP64 oracle's
    loss and gradient timed on a bounded sample of the batch's structures."""
    cfg, b, e_ref, f_ref = synth.differentiation_config()
    wflat = synth.flatten_weights(cfg, synth.model_weights(cfg, 3))
    m = e3.Model(cfg.to_json(), wflat, device=dev)
    pos = torch.tensor(b.pos, dtype=torch.float64, device=dev)
    g = m.build_graph(b.offsets, pos, torch.tensor(b.species, dtype=torch.int32, device=dev), b.cell, b.pbc,
                      cfg.cutoff, 0.5)
    w = torch.tensor(wflat, dtype=torch.float64, device=dev, requires_grad=True)
    et = torch.tensor(e_ref, device=dev)
    ft = torch.tensor(f_ref, device=dev)

    def step():
        w.grad = None
        E, F = e3.energy_forces(w, pos, m, g)
        loss = torch.mean((E - et) ** 2) + torch.sum((F.double() - ft) ** 2) / F.numel()
        loss.backward()
        return loss

    step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / reps
    out = {"workload": f"loss + parameter gradients of {b.n_structures} periodic boxes of 20-200 atoms "
                       f"({b.n_atoms} atoms), 5 species, l_max 3, 64 channels, 2 layers, FP32",
           "ms_per_evaluation": 1e3 * dt, "structures_per_s": b.n_structures / dt, "atoms_per_s": b.n_atoms / dt,
           "weights": int(w.numel()), "evaluations": reps}
    ref_path = os.path.join(ROOT, "tests", "golden", "grad_batch_64.npz")
    if os.path.exists(ref_path):
        ref = np.load(ref_path)
        loss = step()
        gg = w.grad.cpu().numpy()
        out["errors_vs_oracle"] = {"loss_rel": abs(loss.item() - float(ref["loss"])) / abs(float(ref["loss"])),
                                   "grad_rel_l2": float(np.linalg.norm(gg - ref["grad"]) / np.linalg.norm(ref["grad"]))}
    if cpu_baseline:
        import torch as _t
        from oracle import model as om
        _t.set_num_threads(min(os.cpu_count() or 1, 64))
        om_model = om.Model(cfg, synth.model_weights(cfg, 3))
        k = 4
        sub = synth.concat([b.structure(s) for s in range(k)])
        tc = time.perf_counter()
        om.loss_and_grads(om_model, sub, e_ref[:k], f_ref[:int(b.offsets[k])])
        tcpu = time.perf_counter() - tc
        out["cpu_baseline"] = {"value": sub.n_atoms / tcpu, "unit": "atoms/s (loss + gradient)",
                               "cores": _t.get_num_threads(), "kind": "oracle",
                               "sample": f"one FP64 loss + gradient of the batch's first {k} structures "
                                         f"({sub.n_atoms} atoms), {tcpu:.1f} s"}
    log(f"grad: {out['ms_per_evaluation']:.2f} ms per loss+gradient of {b.n_atoms} atoms")
    m.close()
    return out


def hessian_run(e3, synth, torch, dev, n_atoms, reps, log):
    """Hessian-vector products: full Hessians of a batch of small open
    molecules (at most 31 atoms, the sizes of the paper's Hessian study) from
    3 max N_s products, against energy+forces of the same batch; and one
    product on the single-structure box."""
    rng = synth.seed_for(7)
    sizes = rng.integers(10, 32, size=64)
    b = synth.concat([synth.open_box(int(n), 4, rng) for n in sizes])
    cfg1, box = synth.single_config(n=n_atoms)
    cfg = cfg1
    m = e3.Model(cfg.to_json(), synth.flatten_weights(cfg, synth.model_weights(cfg, 2)), device=dev)
    pos = torch.tensor(b.pos, dtype=torch.float64, device=dev)
    g = m.build_graph(b.offsets, pos, torch.tensor(b.species, dtype=torch.int32, device=dev), b.cell, b.pbc,
                      cfg.cutoff, 0.0)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) / k
    t_ef = timed(lambda: m.energy_forces(g, pos), reps)
    t_h = timed(lambda: m.hessian(g, pos), max(1, reps // 10))
    out = {"workload": f"full Hessians of {b.n_structures} open molecules of 10-31 atoms ({b.n_atoms} atoms), "
                       f"l_max 3, 128 channels, 2 layers, r_c 5 A; {3 * int(sizes.max())} products per batch",
           "structures_per_s": b.n_structures / t_h, "ms_per_batch": 1e3 * t_h,
           "ms_energy_forces_per_batch": 1e3 * t_ef, "hessian_over_energy_forces": t_h / t_ef,
           "ms_per_product": 1e3 * t_h / (3 * int(sizes.max()))}
    posb = torch.tensor(box.pos, dtype=torch.float64, device=dev)
    gb = m.build_graph(box.offsets, posb, torch.tensor(box.species, dtype=torch.int32, device=dev), box.cell,
                       box.pbc, cfg.cutoff, 0.0)
    v = torch.tensor(np.random.default_rng(5).normal(size=box.pos.shape), dtype=torch.float32, device=dev)
    out["ms_per_product_box"] = 1e3 * timed(lambda: m.hessian_vector(gb, posb, v), reps)
    out["ms_energy_forces_box"] = 1e3 * timed(lambda: m.energy_forces(gb, posb), reps)
    out["box"] = f"{box.n_atoms}-atom periodic box of the main workload"
    log(f"hessian: {out['structures_per_s']:.1f} full Hessians/s ({out['hessian_over_energy_forces']:.1f}x E+F); "
        f"H v on the box {out['ms_per_product_box']:.2f} ms vs E+F {out['ms_energy_forces_box']:.2f} ms")
    return out


def oracle_errors(E, F, Ei, ref):
    """Errors of one GPU evaluation against a stored oracle result (energy
    relative to |E| and to sum |E_i|, per-atom energies relative to max |E_i|,
    forces max-abs and relative to max |F|)."""
    dE = abs(float(E[0]) - float(ref["energy"][0]))
    sum_ei = float(np.abs(ref["atom_energy"]).sum())
    dF = float(np.abs(F - ref["forces"]).max())
    return {"energy_rel_to_E": dE / abs(float(ref["energy"][0])), "energy_rel_to_sum_abs_Ei": dE / sum_ei,
            "energy_eV_per_atom": dE / len(ref["atom_energy"]),
            "atom_energy_rel_to_max": float(np.abs(Ei - ref["atom_energy"]).max() / np.abs(ref["atom_energy"]).max()),
            "force_max_abs_eV_per_A": dF, "force_rel_to_max": dF / float(np.abs(ref["forces"]).max())}


def gpu_errors(e3, torch, dev, cfg, w, b, ref, prec):
    m = e3.Model(cfg.to_json(), w, precision=prec, device=dev)
    pos = torch.tensor(b.pos, dtype=torch.float64, device=dev)
    g = m.build_graph(b.offsets, pos, torch.tensor(b.species, dtype=torch.int32, device=dev), b.cell, b.pbc,
                      cfg.cutoff, 1.0)
    E, F, Ei = m.energy_forces(g, pos, atom_energy=True)
    torch.cuda.synchronize()
    out = oracle_errors(E.cpu().numpy(), F.double().cpu().numpy(), Ei.cpu().numpy(), ref)
    g.close()
    m.close()
    return out


def scale_run(e3, synth, torch, dev, steps, warmup, log, cpu_baseline=True):
    """The 100,000-atom, 3-layer box (r_c 6 A): MD atom-steps/s in FP32 and in
    BF16 mode over `steps` timed steps (neighbour lists rebuilt every 20 steps
    or earlier, so a rebuild falls inside the timed region once steps >= 20);
    the dominant stage of an FP32 step against its roofline; the errors of
    both precisions against the FP64 oracle on the independent 2,000-atom box;
    the oracle timed on a bounded sample. Its middle layer keeps per-edge R,
    about 106 GB in FP32 for the 9 million edges, so it runs in receiver
    chunks of at most 8 GiB."""
    cfg, b = synth.scale_config()
    w = synth.flatten_weights(cfg, synth.model_weights(cfg, 5))
    vel = synth.maxwell_boltzmann(b, 300.0, synth.seed_for(5, 9))
    pos_d = torch.tensor(b.pos, dtype=torch.float64, device=dev)
    vel_d = torch.tensor(vel, dtype=torch.float64, device=dev)
    sp_d = torch.tensor(b.species, dtype=torch.int32, device=dev)
    energy = torch.empty(1, dtype=torch.float64, device=dev)
    out = {"workload": f"MD step, {b.n_atoms}-atom periodic box, 0.1 atoms/A^3, 4 species, r_c 6 A, l_max 3, "
                       f"128 channels, 3 layers, skin 1 A, rebuild every 20 steps", "steps": steps}
    for name, prec in (("fp32", e3.FP32), ("bf16", e3.BF16_MIX)):
        m = e3.Model(cfg.to_json(), w, precision=prec, device=dev)
        md = e3.MD(m, b.offsets, pos_d, vel_d, sp_d, synth.SPECIES_MASS[:4], b.cell, b.pbc, cfg.cutoff, 1.0, 20)
        md.step(warmup, 0.5, energy)
        torch.cuda.synchronize()
        _, r0, _ = md.stats()
        t1 = time.perf_counter()
        md.step(steps, 0.5, energy)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        _, r1, v1 = md.stats()
        out[f"value_{name}"] = b.n_atoms * steps / dt
        out[f"ms_per_step_{name}"] = 1e3 * dt / steps
        out[f"rebuilds_in_timed_{name}"] = r1 - r0
        out[f"energy_eV_{name}"] = energy.item()
        if name == "fp32":
            # stage split of two fully timed steps; the dominant stage's roofline
            # (per step: a chunked layer launches its stages once per chunk)
            m.profile(True)
            md.step(2, 0.5, energy)
            torch.cuda.synchronize()
            m.profile(False)
            xpos, _, _ = md.state()
            g = m.build_graph(b.offsets, xpos, sp_d, b.cell, b.pbc, cfg.cutoff, 0.0)
            m.energy_forces(g, xpos)
            n_edges = g.last_edge_count()
            g.close()
            best, stage = None, {}
            for t in range(1, cfg.layers + 1):
                for st_name, (flops, nbytes) in work_model(cfg, t, n_edges, b.n_atoms).items():
                    tot, n = m.stage_time(f"{st_name}@{t}")
                    if n == 0:
                        continue
                    stage[f"{st_name}@{t}"] = tot / 2
                    # a layer in receiver chunks recomputes R chunk by chunk in
                    # the adjoint: its radial forward covers every edge twice per step
                    chunks = m.stage_time(f"tp_fwd@{t}")[1] / 2
                    passes = 2 if st_name == "radial_fwd" and chunks > 1 else 1
                    if best is None or tot > best[0]:
                        best = (tot, n, st_name, t, flops * passes, nbytes * passes)
            tot, n, st_name, t, flops, nbytes = best
            step_s = tot / 2 / 1e3
            t_hbm, t_alu = nbytes / PEAK_HBM, flops / PEAK_FP32_VALU
            mfma = st_name.startswith("radial") or st_name.startswith("first")
            if mfma and flops / PEAK_FP32_MFMA > t_hbm:
                roof = {"bound": "mfma", "achieved": flops / step_s / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                        "unit": "TFLOP/s"}
            elif not mfma and t_alu > t_hbm:
                roof = {"bound": "alu", "achieved": flops / step_s / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                        "unit": "TFLOP/s"}
            else:
                roof = {"bound": "hbm", "achieved": nbytes / step_s / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
            roof["frac"] = roof["achieved"] / roof["peak"]
            if not mfma:
                # the VALU peak above counts packed FP32, which this build does not emit
                roof["frac_of_nonpacked_alu"] = flops / step_s / PEAK_FP32_VALU_NONPACKED
            kern = KERNEL_OF_STAGE.get((st_name, t == cfg.layers), "k_" + st_name)
            traffic = measured_traffic(kern, "scale_100k_hbm_traffic.md", fp32_row_pattern(cfg, kern, t))
            roof["traffic"] = None if traffic is None else traffic * n / 2
            roof["kernel"] = f"{st_name} (layer {t}), {kern}"
            roof["launches_per_step"] = n / 2
            roof["ms_per_step"] = tot / 2
            roof["algorithmic_per_step"] = {"flops": flops, "bytes": nbytes, "edges": n_edges}
            out["roofline"] = roof
            out["stage_ms_per_step"] = stage
        md.close()
        m.close()
        torch.cuda.empty_cache()
        log(f"100k box {name}: {out[f'value_{name}']:.3e} atom-steps/s ({out[f'ms_per_step_{name}']:.0f} ms/step)")
    out["bf16_over_fp32"] = out["value_bf16"] / out["value_fp32"]
    # errors against the FP64 oracle on the independent 2,000-atom box
    ref_path = os.path.join(ROOT, "tests", "golden", "scale_sub_2000.npz")
    if os.path.exists(ref_path):
        ref = np.load(ref_path)
        cfg_s, bs = synth.scale_subbox()
        ws = synth.flatten_weights(cfg_s, synth.model_weights(cfg_s, 5))
        out["errors_vs_oracle_2000_atoms"] = {
            "fp32": gpu_errors(e3, torch, dev, cfg_s, ws, bs, ref, e3.FP32),
            "bf16": gpu_errors(e3, torch, dev, cfg_s, ws, bs, ref, e3.BF16_MIX)}
    if cpu_baseline:
        out["cpu_baseline"] = oracle_sample(synth, cfg, 500, 5, 5, 4096,
                                            "box of the same recipe and model (r_c 6 A, 3 layers)")
    return out


def oracle_sample(synth, cfg, n_atoms, seed_key, weight_key, chunk, what):
    """One FP64 oracle energy+forces evaluation of an n-atom periodic box on the
    host cores (neighbour list excluded), as atom-steps/s."""
    import torch as _t
    from oracle import model as om
    _t.set_num_threads(min(os.cpu_count() or 1, 64))
    bs = synth.jittered_lattice(n_atoms, synth.DENSITY, 0.3, cfg.n_species, synth.seed_for(seed_key, 13))
    om_model = om.Model(cfg, synth.model_weights(cfg, weight_key))
    edges = om._edges(bs, cfg.cutoff)
    tc = time.perf_counter()
    om.energy_forces(om_model, bs, edges=edges, edge_chunk=chunk)
    tcpu = time.perf_counter() - tc
    return {"value": bs.n_atoms / tcpu, "unit": "atom-steps/s", "cores": _t.get_num_threads(), "kind": "oracle",
            "sample": f"one FP64 energy+forces evaluation of a {bs.n_atoms}-atom periodic {what} "
                      f"(neighbour list excluded), {tcpu:.1f} s"}


COULOMB_FLOPS_PER_PAIR = 20  # distance 8, rsqrt 1, potential 2, force factor 3, force 6


def coulomb_run(e3, synth, torch, dev, steps, warmup, log):
    """Electrostatics (charge head + soft-core Coulomb over all pairs of each
    open structure): MD atom-steps/s of a batch of charged open clusters with
    and without the term, and the pair kernel against the FP32 vector peak on
    one large cluster."""
    cfg, b = synth.electrostatics_config()
    wd = synth.model_weights(cfg, 8)
    cfg0 = synth.ModelConfig(**{**cfg.__dict__, "coulomb": False})
    out = {"workload": f"{b.n_structures} open clusters, {b.n_atoms} atoms (20-200 each), 0.1 atoms/A^3, "
                       f"total charges in {{-1, 0, 1}}, l_max 3, 128 channels, 2 layers, r_c 5 A, r0 2 A"}
    vel = synth.maxwell_boltzmann(b, 300.0, synth.seed_for(6, 9))
    pos_d = torch.tensor(b.pos, dtype=torch.float64, device=dev)
    vel_d = torch.tensor(vel, dtype=torch.float64, device=dev)
    sp_d = torch.tensor(b.species, dtype=torch.int32, device=dev)
    energy = torch.empty(b.n_structures, dtype=torch.float64, device=dev)
    for key, c, w in (("with", cfg, wd), ("without", cfg0, {k: v for k, v in wd.items() if k not in ("qhead", "qbias")})):
        m = e3.Model(c.to_json(), synth.flatten_weights(c, w), device=dev)
        md = e3.MD(m, b.offsets, pos_d, vel_d, sp_d, synth.SPECIES_MASS[:4], b.cell, b.pbc, c.cutoff, 1.0, 20)
        if c.coulomb:
            md.set_total_charge(b.charge)
        md.step(warmup, 0.5, energy)
        torch.cuda.synchronize()
        if c.coulomb:
            m.profile(True, only="coulomb")
        t1 = time.perf_counter()
        md.step(steps, 0.5, energy)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        m.profile(False)
        out[f"value_{key}"] = b.n_atoms * steps / dt
        out[f"ms_per_step_{key}"] = 1e3 * dt / steps
        if c.coulomb:
            tot, n = m.stage_time("coulomb")
            out["coulomb_kernel_ms_per_step"] = tot / steps
        md.close()
        log(f"coulomb batch ({key} the term): {out[f'value_{key}']:.3e} atom-steps/s")
    out["steps"] = steps
    # pair kernel on one large open cluster
    n_big = 20000
    bb = synth.open_box(n_big, 4, synth.seed_for(6, 11))
    m = e3.Model(cfg.to_json(), synth.flatten_weights(cfg, wd), device=dev)
    pb = torch.tensor(bb.pos, dtype=torch.float64, device=dev)
    g = m.build_graph(bb.offsets, pb, torch.tensor(bb.species, dtype=torch.int32, device=dev), bb.cell, bb.pbc,
                      cfg.cutoff, 0.0)
    g.set_total_charge([0.0])
    m.energy_forces(g, pb)
    torch.cuda.synchronize()
    m.profile(True)
    for _ in range(5):
        m.energy_forces(g, pb)
    torch.cuda.synchronize()
    m.profile(False)
    tot, n = m.stage_time("coulomb")
    avg_s = tot / n / 1e3
    flops = float(n_big) * (n_big - 1) * COULOMB_FLOPS_PER_PAIR
    out["roofline"] = {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                       "unit": "TFLOP/s", "frac": flops / avg_s / PEAK_FP32_VALU,
                       "frac_of_nonpacked_alu": flops / avg_s / PEAK_FP32_VALU_NONPACKED,
                       "traffic": measured_traffic("k_coulomb<16>", "coulomb_hbm_traffic.md"),
                       "kernel": f"k_coulomb, one open cluster of {n_big} atoms", "avg_launch_ms": tot / n,
                       "algorithmic_per_launch": {"flops": flops, "pairs": n_big * (n_big - 1)}}
    log(f"coulomb pair kernel: {tot / n:.3f} ms for {n_big} atoms, "
        f"{out['roofline']['achieved']:.1f} TFLOP/s ({out['roofline']['frac']:.1%})")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--atoms", type=int, default=3000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-atoms", type=int, default=400)
    ap.add_argument("--no-extras", action="store_true", help="skip the BF16 and serving side measurements")
    ap.add_argument("--serving-requests", type=int, default=64)
    ap.add_argument("--serving-steps", type=int, default=200, help="MD steps per serving request")
    ap.add_argument("--scale-steps", type=int, default=20,
                    help="timed steps of the 100,000-atom box (a rebuild falls inside from 20 on)")
    ap.add_argument("--capture-only", action="store_true",
                    help="only run the small-input eager / graph-replay measurement")
    ap.add_argument("--nve-only", action="store_true",
                    help="only run the NVE energy-conservation measurement (--steps steps, FP32 and BF16)")
    ap.add_argument("--grad-only", action="store_true",
                    help="only run the differentiation-batch measurement (loss + parameter gradients)")
    ap.add_argument("--coulomb-only", action="store_true",
                    help="only run the electrostatics measurement (for profiling its kernels)")
    ap.add_argument("--scale-only", action="store_true",
                    help="only run the 100,000-atom FP32 / BF16 measurement")
    ap.add_argument("--hessian-only", action="store_true",
                    help="only run the Hessian-vector-product measurement (for profiling its kernels)")
    ap.add_argument("--product-only", action="store_true",
                    help="only run the product-block measurement (for profiling its kernels)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run plain 256 MiB device-to-device copies (PMC byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(separate structures or requests would go to separate GPUs; one large structure would shard by "
              "spatial domains with a halo exchange of boundary features per layer).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2605_22698_amd as e3
    import synth

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_launch": src.numel() * 4,
                          "bytes_written_per_launch": dst.numel() * 4, "launches": 10}), flush=True)
        return
    if args.scale_only:
        print(json.dumps({"scale": scale_run(e3, synth, torch, dev, args.steps, args.warmup, log,
                                             not args.no_cpu_baseline)}), flush=True)
        return
    if args.capture_only:
        print(json.dumps({"launch_bound": capture_run(e3, synth, torch, dev, 200, log)}), flush=True)
        return
    if args.nve_only:
        print(json.dumps({"nve": nve_run(e3, synth, torch, dev, args.atoms, args.steps, log)}), flush=True)
        return
    if args.grad_only:
        print(json.dumps({"grad": grad_run(e3, synth, torch, dev, args.steps, log, not args.no_cpu_baseline)}),
              flush=True)
        return
    if args.hessian_only:
        print(json.dumps({"hessian": hessian_run(e3, synth, torch, dev, args.atoms, args.steps, log)}), flush=True)
        return
    if args.product_only:
        print(json.dumps({"product": product_run(e3, synth, torch, dev, args.atoms, args.steps, args.warmup, log)}),
              flush=True)
        return
    if args.coulomb_only:
        print(json.dumps({"coulomb": coulomb_run(e3, synth, torch, dev, args.steps, args.warmup, log)}), flush=True)
        return
    cfg, b = synth.single_config(n=args.atoms)
    w = synth.flatten_weights(cfg, synth.model_weights(cfg, 2))
    m = e3.Model(cfg.to_json(), w, device=dev)
    vel = synth.maxwell_boltzmann(b, 300.0, synth.seed_for(2, 9))
    pos_d = torch.tensor(b.pos, dtype=torch.float64, device=dev)
    vel_d = torch.tensor(vel, dtype=torch.float64, device=dev)
    sp_d = torch.tensor(b.species, dtype=torch.int32, device=dev)
    masses = synth.SPECIES_MASS[:cfg.n_species]
    skin, rebuild_every, dt = 1.0, 20, 0.5
    md = e3.MD(m, b.offsets, pos_d, vel_d, sp_d, masses, b.cell, b.pbc, cfg.cutoff, skin, rebuild_every)
    energy = torch.empty(1, dtype=torch.float64, device=dev)
    md.step(args.warmup, dt, energy)
    torch.cuda.synchronize()

    # ---- profiled segment before the timed region: every stage is timed, to
    # split the step and find the dominant kernel (each timed stage adds a
    # few microseconds of device time, so the timed region below brackets
    # only the dominant kernel) ----
    k_prof = max(10, args.steps // 10)
    m.profile(True)
    md.step(k_prof, dt, energy)
    torch.cuda.synchronize()
    m.profile(False)
    stages = ["prune", "embed", "first_fwd", "radial_fwd", "tp_fwd", "mix_fwd", "gate_fwd", "readout", "gate_bwd",
              "mix_bwd", "first_bwd", "tp_bwd_edge", "radial_bwd", "tp_bwd_node", "forces", "md_update",
              "graph_build", "last_fwd", "last_bwd"]
    stage_ms = {}
    for s in stages:
        tot, n = m.stage_time(s)
        stage_ms[s] = (tot, n)
    # exact edge count at this configuration (same graph the steps use)
    g_pos, _, _ = md.state()
    g = m.build_graph(b.offsets, g_pos, sp_d, b.cell, b.pbc, cfg.cutoff, 0.0)
    m.energy_forces(g, g_pos)
    n_edges = g.last_edge_count()
    best = None
    for t in range(1, cfg.layers + 1):
        wm = work_model(cfg, t, n_edges, b.n_atoms, pairs=True)
        for s, (flops, nbytes) in wm.items():
            tot, n = m.stage_time(f"{s}@{t}")
            if n == 0:
                continue
            if best is None or tot > best[0]:
                best = (tot, n, s, t, flops, nbytes)
    _, _, dom_s, dom_t, flops, nbytes = best

    # ---- timed region ----
    m.profile(True, only=f"{dom_s}@{dom_t}")
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(args.steps):
        md.step(1, dt, energy)
        evs[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    gpu_ms = float(step_ms.sum())
    m.profile(False)
    steps_done, rebuilds, violations = md.stats()
    E_now = energy.item()

    value = b.n_atoms * args.steps / (wall)
    ms_per_step = 1e3 * wall / args.steps

    # ---- roofline of the dominant kernel, timed over the timed region ----
    s, t = dom_s, dom_t
    tot, n = m.stage_time(f"{s}@{t}")
    avg_s = tot / n / 1e3
    mfma = s.startswith("radial") or s.startswith("first") or s.startswith("last")
    peak_flop = PEAK_FP32_MFMA if mfma else PEAK_FP32_VALU
    t_hbm, t_flop = nbytes / PEAK_HBM, flops / peak_flop
    if t_flop >= t_hbm:
        bound = "mfma" if mfma else "alu"
        roof = {"bound": bound, "achieved": flops / avg_s / 1e12, "peak": peak_flop / 1e12, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": nbytes / avg_s / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    # the last layer's edge adjoint stage is the sender-side kernel (tps.hip)
    roof["traffic"] = measured_traffic("k_tps_bwd_sender" if (s, t) == ("tp_bwd_edge", cfg.layers) else "k_" + s)
    roof["kernel"] = f"{s} (layer {t})"
    roof["avg_launch_ms"] = tot / n
    roof["algorithmic_per_launch"] = {"flops": flops, "bytes": nbytes, "edges": n_edges,
                                      "edge_pairs": (n_edges + 1) // 2}

    md.close()

    # ---- side measurements: BF16 mode, NPT, continuous-batching serving ----
    extras = {}
    if not args.no_extras:
        m16 = e3.Model(cfg.to_json(), w, precision=e3.BF16_MIX, device=dev)
        md16 = e3.MD(m16, b.offsets, pos_d, vel_d, sp_d, masses, b.cell, b.pbc, cfg.cutoff, skin, rebuild_every)
        md16.step(args.warmup, dt, energy)
        torch.cuda.synchronize()
        k16 = max(20, args.steps // 2)
        t1 = time.perf_counter()
        md16.step(k16, dt, energy)
        torch.cuda.synchronize()
        t16 = time.perf_counter() - t1
        extras["bf16"] = {"value": b.n_atoms * k16 / t16, "ms_per_step": 1e3 * t16 / k16, "steps": k16,
                          "speedup_over_fp32": (b.n_atoms * k16 / t16) / value}
        md16.close()
        ref_path = os.path.join(ROOT, "tests", "golden", "single_3000.npz")
        if args.atoms == 3000 and os.path.exists(ref_path):
            # both precisions against the FP64 oracle on the starting structure
            ref = np.load(ref_path)
            extras["bf16"]["errors_vs_oracle"] = gpu_errors(e3, torch, dev, cfg, w, b, ref, e3.BF16_MIX)
            extras["fp32_errors_vs_oracle"] = gpu_errors(e3, torch, dev, cfg, w, b, ref, e3.FP32)
        # NPT: Langevin (300 K, 0.01/fs) with a Monte Carlo volume move every 25 steps at 1 bar
        mdp = e3.MD(m, b.offsets, pos_d, vel_d, sp_d, masses, b.cell, b.pbc, cfg.cutoff, skin, rebuild_every)
        mdp.set_langevin(300.0, 0.01, [2026])
        mdp.set_barostat(1.0, 25, 0.002, [2027])
        mdp.step(args.warmup, dt, energy)
        torch.cuda.synchronize()
        kp = max(100, args.steps)
        t1 = time.perf_counter()
        mdp.step(kp, dt, energy)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t1
        _, prop, acc = mdp.cells()
        extras["npt"] = {"value": b.n_atoms * kp / tp, "ms_per_step": 1e3 * tp / kp, "steps": kp,
                         "barostat": "Langevin 300 K, friction 0.01/fs, volume move every 25 steps at 1 bar",
                         "proposals": prop, "accepted": acc}
        mdp.close()
        extras["nve"] = nve_run(e3, synth, torch, dev, args.atoms, 2000, log)
        extras["launch_bound"] = capture_run(e3, synth, torch, dev, 200, log)
        extras["serving"] = serving_run(e3, synth, torch, dev, args.serving_requests, args.serving_steps, log)
        extras["coulomb"] = coulomb_run(e3, synth, torch, dev, max(20, args.steps // 2), args.warmup, log)
        extras["product"] = product_run(e3, synth, torch, dev, args.atoms, max(20, args.steps // 4), args.warmup, log)
        extras["grad"] = grad_run(e3, synth, torch, dev, 20, log, not args.no_cpu_baseline)
        extras["hessian"] = hessian_run(e3, synth, torch, dev, args.atoms, 20, log)
        extras["scale"] = scale_run(e3, synth, torch, dev, args.scale_steps, 2, log, not args.no_cpu_baseline)

    # ---- oracle on the host cores (bounded sample) ----
    cpu = None
    if not args.no_cpu_baseline:
        import torch as _t
        from oracle import model as om
        _t.set_num_threads(min(os.cpu_count() or 1, 64))
        cfg_s, bs = synth.single_config(n=args.cpu_sample_atoms, seed_key=12)
        om_model = om.Model(cfg_s, synth.model_weights(cfg_s, 2))
        edges = om._edges(bs, cfg_s.cutoff)
        om.energy_forces(om_model, synth.Batch(bs.pos[:8], bs.species[:8], bs.cell, bs.pbc,
                                               np.array([0, 8])))  # warm caches
        tc = time.perf_counter()
        om.energy_forces(om_model, bs, edges=edges, edge_chunk=8192)
        tcpu = time.perf_counter() - tc
        cpu = {"value": bs.n_atoms / tcpu, "unit": "atom-steps/s", "cores": _t.get_num_threads(), "kind": "oracle",
               "sample": f"one FP64 energy+forces evaluation of a {bs.n_atoms}-atom periodic box of the same "
                         f"recipe and model (neighbour list excluded), {tcpu:.1f} s"}

    out = {
        "metric": "atom-steps/s (energy+forces)",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"MD step, {b.n_atoms}-atom periodic box, 0.1 atoms/A^3, 4 species, r_c 5 A, "
                               f"l_max 3, 128 channels, 2 layers, last layer scalar outputs only",
                   "n_atoms": b.n_atoms, "n_edges": n_edges, "dt_fs": dt, "skin": skin,
                   "rebuild_every": rebuild_every, "precision": "fp32"},
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "gpu_ms_per_step": gpu_ms / args.steps,
        "stage_ms_per_step": {k: v[0] / k_prof for k, v in stage_ms.items()},
        "stage_ms_note": f"from {k_prof} fully timed steps before the timed region",
        "rebuilds": rebuilds,
        "skin_violations": violations,
        "energy_eV": E_now,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
