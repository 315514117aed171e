"""Benchmark of the hybrid symplectic step on one MI355X.

Workload: the 2048-planetesimal disk (masses dN/dm ~ m^-2 on [1e-9, 1e-7],
a ~ U(0.5, 4), e ~ Ray(0.02), i ~ Ray(0.01), dt = 0.01 orbit, n1 = 3,
n2 = 0.4), FP64, with encounters resolved by Bulirsch-Stoer per group.

value = N (N - 1) x steps / wall time of the whole steps (every step runs one
all-pairs kick plus the opening kick, Sun kicks, drift, encounter search,
grouping and BS): whole-step pair-interaction throughput with the state
resident in HBM.  The roofline entry covers the pair-kick kernel, timed live
with HIP events on the stream it runs on.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector peak (256 CU x 2.4 GHz x 128)
HBM_PEAK_GBS = 8000.0
FLOPS_PER_PAIR = 18              # 3 sub, 5 for r^2, sqrt, r^2 r, div, m/r^3, 3 FMA
N_BODIES = 2048


def _kernel_source_hash(files=("device_math.h", "massive.hip", "genga_impl.h")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1404_2324_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TP_SOURCES = ("device_math.h", "bs_device.h", "tp.hip", "genga_impl.h")


def _tp_traffic_per_step():
    """HBM bytes per test-particle step (the particle kernels) and per
    k_tp_main launch from the committed counter summary, or None when their
    source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "tp_step_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != _kernel_source_hash(TP_SOURCES):
        return None
    return d


def _traffic_per_launch():
    """HBM bytes per kick launch from the committed counter summary, or None
    when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "kick_n2048_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != _kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_steps(O, op, s, budget_s, max_steps):
    sim = O.MassiveSim(op, s.m, s.x, s.u, coords="helio")
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and steps < max_steps:
        sim.step(1)
        steps += 1
    return steps, time.perf_counter() - t0


def cpu_baseline(s, gp, budget_s: float = 12.0, budget_1core_s: float = 10.0):
    """The oracle on the same workload, on all host cores and on one core
    (OpenMP threads set in the oracle), timed on a prefix of the run."""
    import oracle as O
    op = O.params(G=gp.G, m0=gp.m0, dt=gp.dt, n1=gp.n1, n2=gp.n2, pf=gp.pf,
                  bs_tol=gp.bs_tol, bs_max_depth=gp.bs_max_depth,
                  kepler_max_iter=gp.kepler_max_iter)
    avail = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    cores = O.set_threads(min(avail, int(omp)) if omp else avail)
    steps, dt = _oracle_steps(O, op, s, budget_s, 400)
    one = O.set_threads(1)
    steps1, dt1 = _oracle_steps(O, op, s, budget_1core_s, 400)
    O.set_threads(cores)
    n = len(s.m)
    return {"value": n * (n - 1) * steps / dt, "unit": "pair interactions/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(),
            "one_core": {"value": n * (n - 1) * steps1 / dt1, "cores": one,
                         "sample": f"first {steps1} steps ({dt1:.1f} s)"},
            "sample": f"first {steps} steps of the same 2048-body workload "
                      f"({dt:.1f} s; the oracle recomputes every pair in both half kicks "
                      f"and Hermite-tests every pair)"}


TP_BYTES = 104  # per particle-step: x, v read and written (96 B) + the 32-bit mask both ways


def tp_measure(G, W, torch, steps: int, ntp: int = 1_000_000):
    """Test-particle mode: 8 planets and 10^6 particles (Sec. 3.3), with
    physical radii (bulk density 2 g/cm^3, particles 10 km): particles that
    hit a planet are removed."""
    planets, xt, ut = W.test_particles(ntp=ntp)
    sim = G.TestParticleSimulation(planets.m, planets.x, planets.u, xt, ut, G.default_params(),
                                   coords="helio", radii=W.tp_radii(planets.m, ntp))
    sim.step(4)
    sim.check()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    sim.check()
    sec = e0.elapsed_time(e1) / 1e3
    st = sim.stats()
    sim.close()
    return {"workload": f"tp_8p_{ntp}", "steps": steps, "ms_per_step": sec * 1e3 / steps,
            "tp_steps_per_s": ntp * steps / sec,
            "algorithmic_GBps": TP_BYTES * ntp * steps / sec / 1e9,
            "hbm_frac": TP_BYTES * ntp * steps / sec / 1e9 / HBM_PEAK_GBS,
            "tp_enc_last_step": st["tp_enc"], "bs_substeps": st["bs_substeps"],
            "removed": st["tp_removed"], "counters": _tp_counter_rates(sec / steps)}


def _tp_counter_rates(step_s: float):
    """HBM traffic of the particle kernels from rocprofv3 FETCH_SIZE and
    WRITE_SIZE (profiles/tp_step_traffic.json), over this run's step time."""
    d = _tp_traffic_per_step()
    if d is None:
        return None
    return {"bytes_per_step": d["bytes_per_step"], "k_tp_main_bytes": d["k_tp_main_bytes"],
            "GBps": d["bytes_per_step"] / step_s / 1e9,
            "hbm_frac": d["bytes_per_step"] / step_s / 1e9 / HBM_PEAK_GBS}


def energy_measure(G, W, torch, steps: int = 1000, every: int = 10):
    """The 16-body system for 1000 steps: relative energy error statistics
    (Sec. 4.1) and angular-momentum drift, energy read every 10 steps."""
    s = W.plain_n16()
    sim = G.Simulation(s.m, s.x, s.u, G.default_params(), coords="helio")
    E0, L0 = sim.energy()
    errs, t = [], []
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    gpu_ms = 0.0
    for k in range(steps // every):
        e0.record(stream)
        sim.step(every)
        e1.record(stream)
        E, L = sim.energy()          # synchronises
        gpu_ms += e0.elapsed_time(e1)
        errs.append(abs((E - E0) / E0))
        t.append((k + 1) * every)
    sim.check()
    st = sim.stats()
    _, L = sim.energy()
    sim.close()
    errs = np.asarray(errs)
    slope = float(np.polyfit(np.asarray(t, dtype=float), errs, 1)[0])
    return {"workload": "plain_n16", "steps": steps, "dE_rel_max": float(errs.max()),
            "dE_rel_median": float(np.median(errs)), "dE_rel_final": float(errs[-1]),
            "dE_rel_slope_per_step": slope,
            "L_rel_drift": float(np.linalg.norm(L - L0) / np.linalg.norm(L0)),
            "enc_total": st["enc_total"], "steps_per_s": steps / (gpu_ms / 1e3)}


def batch_measure(G, W, torch, steps: int, cpu: bool):
    """Batched mode: 4096 independent systems of 2..32 bodies (Sec. 3.4), all
    steps in one captured launch; the tuner's table comes from init."""
    off, m0s, m, x, u = W.batched()
    sim = G.BatchedSimulation(off, m0s, m, x, u, G.default_params())
    times, choice = sim.tune(4)
    sim.step(2)
    sim.check()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    _, done0 = sim.status()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    sim.check()
    sec = e0.elapsed_time(e1) / 1e3
    st = sim.stats()
    status, done = sim.status()
    sim.close()
    nsys = len(off) - 1
    sizes = np.diff(off)
    completed = int((done - done0).sum())  # a stopped system takes no more steps
    out = {"workload": f"batched_{nsys}_systems_2_32", "systems": nsys, "bodies": int(off[-1]),
           "steps": steps, "launches": 1, "ms_per_step": sec * 1e3 / steps,
           "system_steps_per_s": completed / sec,
           "system_steps_timed": completed,
           "pair_interactions_per_s": float((sizes * (sizes - 1)).sum()) * steps / sec,
           "tuner": {"choice": choice, "us_per_variant_4_steps": times},
           "enc_total": st["enc_total"], "bs_substeps": st["bs_substeps"],
           "max_group_last_step": st["max_group"],
           "systems_stopped": int((status != 0).sum()),
           "system_steps_completed": int(done.sum())}
    if cpu:  # CPU baseline leg: the oracle on a sample of the same systems
        import oracle as O
        t0 = time.perf_counter()
        ns, nst = 64, 20
        v = np.concatenate([O.helio_to_dem(O.params(), m[off[k]:off[k + 1]], u[off[k]:off[k + 1]])
                            for k in range(ns)])
        O.batched_run(O.params(), off[:ns + 1], m0s[:ns], m[:off[ns]], x[:off[ns]], v, nst)
        dt = time.perf_counter() - t0
        # systems run one after another; inside a system the oracle's row
        # loops use its OpenMP threads
        out["cpu_oracle"] = {"system_steps_per_s": ns * nst / dt,
                             "sample": f"first {ns} systems x {nst} steps, one system at a time",
                             "cores": O.threads()}
    return out


def adjoint_measure(G, W, torch, steps: int, ckpt: int = 32):
    """Adjoint of the encounter-free map: 1024 systems x 8 planets, a
    checkpoint every 32 steps.  Ratio = backward (segment recompute + VJP)
    over the plain forward of the same packed kernel (one checkpoint)."""
    m, x, u = W.adjoint_systems()
    nsys = m.shape[0]
    off = np.arange(0, 8 * nsys + 1, 8, dtype=np.int32)
    gp = G.default_params(encounter_free=1)
    sim = G.BatchedSimulation(off, np.ones(nsys), m.reshape(-1), x.reshape(-1, 3),
                              u.reshape(-1, 3), gp, coords="helio")
    xd, vd = sim.state("dem")
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
    # loss sum |x_T - x_target|^2, x_target = the map from the initial
    # conditions perturbed by 1e-6 (relative, normal; seed + 1000): its
    # gradient with respect to x_T seeds the backward pass
    rng = np.random.default_rng(W.SEED_BASE + 5 + 1000)
    xp = xd * (1.0 + 1e-6 * torch.tensor(rng.standard_normal(tuple(xd.shape)), device="cuda"))
    vp = vd * (1.0 + 1e-6 * torch.tensor(rng.standard_normal(tuple(vd.shape)), device="cuda"))
    sim.set_state(xp, vp, coords="dem")
    sim.adj_forward(steps, steps)            # warm-up (one checkpoint): the target
    xt, _ = sim.state("dem")
    sim.set_state(xd, vd, coords="dem")
    sim.adj_forward(steps, steps)
    xT, _ = sim.state("dem")
    gx = (2.0 * (xT - xt)).contiguous()
    gv = torch.zeros_like(gx)
    sim.set_state(xd, vd, coords="dem")
    torch.cuda.synchronize()
    ev[0].record(stream)
    sim.adj_forward(steps, steps)            # plain forward (same kernel)
    ev[1].record(stream)
    torch.cuda.synchronize()
    sim.set_state(xd, vd, coords="dem")
    torch.cuda.synchronize()
    ev[2].record(stream)
    sim.adj_forward(steps, ckpt)             # forward keeping checkpoints
    ev[3].record(stream)
    sim.adj_backward(gx, gv)                 # recompute + VJP
    ev[4].record(stream)
    torch.cuda.synchronize()
    sim.check()
    sim.set_state(xd, vd, coords="dem")
    torch.cuda.synchronize()
    ev[5].record(stream)
    sim.step(steps)                          # the general batched kernel, same work
    ev[6].record(stream)
    torch.cuda.synchronize()
    sim.check()
    fwd = ev[0].elapsed_time(ev[1])
    fck = ev[2].elapsed_time(ev[3])
    bwd = ev[3].elapsed_time(ev[4])
    gen = ev[5].elapsed_time(ev[6])
    sim.close()
    return {"workload": f"adjoint_{nsys}x8_encounter_free", "steps": steps, "ckpt_every": ckpt,
            "loss": float(((xT - xt) ** 2).sum()),
            "forward_ms": fwd, "forward_ckpt_ms": fck, "backward_ms": bwd,
            "adjoint_forward_ratio": bwd / fwd, "forward_plus_backward_ratio": (fck + bwd) / fwd,
            "general_batched_kernel_ms": gen,
            "system_steps_per_s_forward": nsys * steps / (fwd / 1e3)}


def hybrid_adjoint_measure(G, W, torch, steps: int, ckpt: int = 16, cpu: bool = True):
    """Adjoint of the hybrid step with encounters (changeover, groups, BS):
    1024 systems x 8 planets packed so that encounters happen every step
    (~140 encounters and ~120 BS substeps per system over 64 steps), a
    checkpoint every 16 steps.  Ratio = backward (segment recompute, BS
    rerun keeping its substeps, VJPs) over the forward without checkpoints;
    beside it the general batched kernel on the same systems and steps."""
    nsys, npl = 1024, 8
    m, x, u = W.encounter_systems(nsys=nsys, nplanets=npl, seed_index=7, da=0.03, dphase=0.3)
    off = np.arange(0, npl * nsys + 1, npl, dtype=np.int32)
    gp = G.default_params()
    sim = G.BatchedSimulation(off, np.ones(nsys), m.reshape(-1), x.reshape(-1, 3),
                              u.reshape(-1, 3), gp, coords="helio")
    xd, vd = sim.state("dem")
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
    # loss sum |x_T - x_target|^2 with x_target from initial conditions
    # perturbed by 1e-6 (relative, normal; seed + 1000)
    rng = np.random.default_rng(W.SEED_BASE + 7 + 1000)
    xp = xd * (1.0 + 1e-6 * torch.tensor(rng.standard_normal(tuple(xd.shape)), device="cuda"))
    vp = vd * (1.0 + 1e-6 * torch.tensor(rng.standard_normal(tuple(vd.shape)), device="cuda"))
    sim.set_state(xp, vp, coords="dem")
    sim.adj_forward(steps, steps)            # warm-up: the target
    xt, _ = sim.state("dem")
    sim.set_state(xd, vd, coords="dem")
    sim.adj_forward(steps, steps)
    xT, _ = sim.state("dem")
    gx = (2.0 * (xT - xt)).contiguous()
    gv = torch.zeros_like(gx)
    sim.set_state(xd, vd, coords="dem")
    torch.cuda.synchronize()
    ev[0].record(stream)
    sim.adj_forward(steps, steps)            # forward (one checkpoint)
    ev[1].record(stream)
    torch.cuda.synchronize()
    sim.set_state(xd, vd, coords="dem")
    torch.cuda.synchronize()
    ev[2].record(stream)
    sim.adj_forward(steps, ckpt)             # forward keeping checkpoints
    ev[3].record(stream)
    sim.adj_backward(gx, gv)
    ev[4].record(stream)
    torch.cuda.synchronize()
    sim.check()
    sim.set_state(xd, vd, coords="dem")
    sim.step(1)                              # the batched kernel's tuner runs here, untimed
    sim.set_state(xd, vd, coords="dem")
    torch.cuda.synchronize()
    ev[5].record(stream)
    sim.step(steps)                          # the general batched kernel, same systems
    ev[6].record(stream)
    torch.cuda.synchronize()
    sim.check()
    fwd = ev[0].elapsed_time(ev[1])
    fck = ev[2].elapsed_time(ev[3])
    bwd = ev[3].elapsed_time(ev[4])
    gen = ev[5].elapsed_time(ev[6])
    sim.close()
    out = {"workload": f"hybrid_adjoint_{nsys}x{npl}_encounters", "steps": steps,
           "ckpt_every": ckpt, "loss": float(((xT - xt) ** 2).sum()),
           "forward_ms": fwd, "forward_ckpt_ms": fck, "backward_ms": bwd,
           "adjoint_forward_ratio": bwd / fwd, "forward_plus_backward_ratio": (fck + bwd) / fwd,
           "general_batched_kernel_ms": gen,
           "system_steps_per_s_forward": nsys * steps / (fwd / 1e3)}
    if cpu:
        # the oracle's complex-step derivative (one direction, every decision
        # fixed) on a sample: the CPU's cost of one directional derivative
        import oracle as O
        p = O.params()
        ns = 16
        t0 = time.perf_counter()
        for k in range(ns):
            vk = O.helio_to_dem(p, m[k], u[k])
            O.cs_massive(p, m[k], x[k], vk, None, np.ones_like(x[k]), None, steps)
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"directional_derivatives_per_s": ns / dt,
                             "sample": f"first {ns} systems x {steps} steps, one direction each",
                             "cores": 1}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--kick-steps", type=int, default=64,
                    help="steps run launch by launch to time the pair kernel")
    ap.add_argument("--big-n", type=int, default=16384,
                    help="bodies of the encounter-free kick capability run (0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tp-steps", type=int, default=100,
                    help="steps of the 10^6-particle run reported under extra (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=10000,
                    help="steps of the 4096-system batched run reported under extra (0: skip)")
    ap.add_argument("--energy-steps", type=int, default=1000,
                    help="steps of the 16-body energy-error run reported under extra (0: skip)")
    ap.add_argument("--adj-steps", type=int, default=1000,
                    help="steps of the 1024 x 8 adjoint run reported under extra (0: skip)")
    ap.add_argument("--hist-steps", type=int, default=100,
                    help="steps of the 2048-body disk after the timing for the candidate, "
                         "encounter and group-size statistics (0: skip)")
    ap.add_argument("--energy-long-steps", type=int, default=10000,
                    help="steps of the 2048-body disk after the timing, |dE/E| every 1000 (0: skip)")
    ap.add_argument("--hadj-steps", type=int, default=64,
                    help="steps of the 1024 x 8 hybrid (encounter) adjoint run under extra (0: skip)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed region run one 256 MiB device copy (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the systems here shard with no exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1404_2324_amd import genga as G
    from paper_1404_2324_amd import workloads as W

    s = W.planetesimals(N_BODIES)
    gp = G.default_params()
    sim = G.Simulation(s.m, s.x, s.u, gp, coords="helio")
    n = sim.n
    stream = torch.cuda.current_stream()
    E_init, L_init = sim.energy()

    sim.step(args.warmup)
    sim.check()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = sim.sync()
    if status != G.OK:
        raise G.GengaError(status, "device status after the timed steps")
    gpu_ms = e0.elapsed_time(e1)
    sec = gpu_ms / 1e3
    st = sim.stats()

    # live timing of the closing-kick pair kernel inside real steps (launched
    # one by one with HIP events around it on the context's stream)
    # every kernel of the step timed on its own dispatch timestamps (HIP
    # events recorded by the dispatches, on the context's stream)
    split = sim.step_kernel_us(min(args.kick_steps, 512))
    tot_us = sum(split.values())
    # candidates, encounters and group sizes over 100 further steps, one at a
    # time (outside the timed region): the per-step counts and the histogram
    # of group sizes (connected components of each step's encounter pairs)
    per_step = None
    if args.hist_steps > 0:
        nc, ne, sizes = [], [], {}
        for _ in range(args.hist_steps):
            sim.step(1)
            ij = sim.encounters()[0]
            nc.append(sim.stats()["n_cand"])
            ne.append(len(ij))
            parent = {}

            def root(a):
                while parent.setdefault(a, a) != a:
                    parent[a] = parent[parent[a]]
                    a = parent[a]
                return a

            for i, j in ij:
                ri, rj = root(int(i)), root(int(j))
                if ri != rj:
                    parent[max(ri, rj)] = min(ri, rj)
            comp = {}
            for b in parent:
                r = root(b)
                comp[r] = comp.get(r, 0) + 1
            for c in comp.values():
                sizes[c] = sizes.get(c, 0) + 1
        sim.check()
        per_step = {"steps": args.hist_steps,
                    "candidates_mean": float(np.mean(nc)), "candidates_max": int(max(nc)),
                    "encounters_mean": float(np.mean(ne)), "encounters_max": int(max(ne)),
                    "group_size_hist": {str(k): sizes[k] for k in sorted(sizes)}}
    # energy and angular momentum of the disk over a longer run (outside the
    # timed region): |dE/E| (Sec. 4.1) every 1000 steps
    energy_long = None
    if args.energy_long_steps > 0:
        done = args.warmup + args.steps + min(args.kick_steps, 512) + max(args.hist_steps, 0)
        errs, failure = [], None
        try:
            for _ in range(args.energy_long_steps // 1000):
                sim.step(1000)
                sim.check()
                E, L = sim.energy()
                done += 1000
                errs.append(abs((E - E_init) / E_init))
        except G.GengaError as err:  # reported, not hidden: the run stops there
            failure = str(err)
        _, L = sim.energy()
        energy_long = {"workload": "planetesimals_n2048", "steps": done,
                       "dE_rel_every_1000": [float(e) for e in errs],
                       "dE_rel_max": float(max(errs)) if errs else None,
                       "L_rel_drift": float(np.linalg.norm(L - L_init) / np.linalg.norm(L_init)),
                       "enc_total": sim.stats()["enc_total"], "failure": failure}
    dominant = max(split, key=split.get)
    kick_us = split["k_pair_part"]
    kick_s = kick_us * 1e-6

    # capability of the same pair kernel at a size that fills the chip
    big = None
    if args.big_n > 0:
        sb = W.planetesimals(args.big_n, seed_index=2)
        simb = G.Simulation(sb.m, sb.x, sb.u, G.default_params(encounter_free=1), coords="helio")
        simb.step(2)
        big_us = simb.step_profiled(8)
        nb = args.big_n
        big = {"n_bodies": nb, "kernel_us": big_us,
               "pair_rate": nb * (nb - 1) / (big_us * 1e-6),
               "tflops": FLOPS_PER_PAIR * nb * (nb - 1) / (big_us * 1e-6) / 1e12}
        simb.close()

    extra = {}
    if per_step is not None:
        extra["encounters_n2048"] = per_step
    if energy_long is not None:
        extra["energy_n2048"] = energy_long
    if args.energy_steps > 0:
        extra["energy"] = energy_measure(G, W, torch, args.energy_steps)
    if args.tp_steps > 0:
        extra["test_particles"] = tp_measure(G, W, torch, args.tp_steps)
    if args.batch_steps > 0:
        extra["batched"] = batch_measure(G, W, torch, args.batch_steps, not args.no_cpu)
    if args.adj_steps > 0:
        extra["adjoint"] = adjoint_measure(G, W, torch, args.adj_steps)
    if args.hadj_steps > 0:
        extra["hybrid_adjoint"] = hybrid_adjoint_measure(G, W, torch, args.hadj_steps,
                                                         cpu=not args.no_cpu)

    if args.calib_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    pairs = n * (n - 1)
    flops = FLOPS_PER_PAIR * pairs
    achieved = flops / kick_s / 1e12
    traffic = _traffic_per_launch()
    out = {
        "metric": "FP64 pair interactions/s",
        "value": pairs * args.steps / sec,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "planetesimals_n2048", "n_bodies": n, "dt": gp.dt,
                   "n1": gp.n1, "n2": gp.n2, "bs_tol": gp.bs_tol,
                   "host_wall_s": wall},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": traffic,
                     "kernel": "k_pair_part<0> (closing-kick pair kernel: every pair, the "
                               "prechecker, partial sums per partner split)",
                     "kernel_us": kick_s * 1e6,
                     "epilogue_kernel_us": split["k_pair_finish"],
                     "flops_per_pair": FLOPS_PER_PAIR,
                     "kick_pair_rate": pairs / kick_s,
                     "large_n": big},
        "step_kernels": {
            "us": split,
            "share": {k: v / tot_us for k, v in split.items()},
            "dominant": dominant,
            "dominant_bound": ("latency: one workgroup per encounter group (its waves try "
                               "several halving depths at once), and the step waits for the "
                               "group with the most sequential BS substeps"
                               if dominant == "k_group_bs" else "see roofline"),
        },
        "stats": {k: st[k] for k in ("n_cand", "n_enc", "n_groups", "max_group",
                                      "kepler_iter_max", "bs_substeps", "enc_total",
                                      "full_kicks")},
    }
    if extra:
        out["extra"] = extra
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(s, gp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
