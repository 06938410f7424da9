"""NEP MD throughput on one MI355X: the 131,072-atom 4-species FCC alloy.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-bf16] [--no-cpu]

A step is one velocity-Verlet NVE step of the whole hot path (cell sort and
neighbour rows, descriptors, network on MFMA, partial forces, Newton-3 force
and virial gather, float64 integration, thermo reduction every 10 steps).
Positions, velocities and species are resident in device memory before the
timed region; the timed region is one nep_md_run_dev call of K steps,
bracketed by device synchronisations.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "fcc131k"
THERMO_EVERY = 10
SKIN = 0.8   # Angstrom: rows at r_c + 0.8 A, rebuilt after a 0.4 A displacement (fastest of 0.6-1.3 A measured)
# MI355X: FP32 vector peak without packed-FP32 instructions (all device code is
# built with packed FP32 disabled): 256 CU x 64 lanes x 2 flop x 2.4 GHz
PEAK_FP32_VALU = 256 * 64 * 2 * 2.4e9 / 1e12
PEAK_FP32_MFMA = 157.3
PEAK_BF16_MFMA = 2500.0
PEAK_HBM = 8000.0  # GB/s


def measured_traffic(kernel):
    """HBM bytes per launch of the named partial-force kernel variant from the
    committed FETCH_SIZE/WRITE_SIZE counter summary, or None when that variant
    was not profiled or any source it is built from has changed since."""
    import hashlib
    import json
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        rec = json.load(open(os.path.join(here, "profiles", "partial_forces_fcc131k_traffic.json")))
        digest = hashlib.sha256()
        for f in rec["sources"]:
            digest.update(open(os.path.join(here, f), "rb").read())
        # the profiled name may carry one more template argument (the basis
        # shape the library specialised the kernel for)
        names = [k for k in rec["variants"] if k == kernel or k.startswith(kernel[:-1] + ", ")]
        if len(names) != 1:
            return None
        v = rec["variants"][names[0]]
    except (OSError, KeyError, ValueError):
        return None
    if digest.hexdigest() != rec["sources_sha256"]:
        return None
    return {"bytes": v["fetch_bytes"] + v["write_bytes"], "fetch_bytes": v["fetch_bytes"],
            "write_bytes": v["write_bytes"], "kernel": names[0], "dispatches": v["dispatches"]}


def algorithmic_flops(h, p_r, p_a):
    """Useful float work per atom of each pass (flop; a multiply-add counts 2).

    p_r, p_a: mean neighbours within r_c^R and r_c^A.  Per bond: the float64
    minimum image and displacement (20), length and direction (8), cutoff
    function and derivative (10); Chebyshev recurrences, basis values and
    derivatives (5-12 per basis function); the radial-function contractions
    (2 n K per value); the angular polynomials and their gradients (2 and 4
    per polynomial) and the n_A x NB contractions with the sums or with
    dU/dS.  The network is 2 GEMMs of 2 N_des N_neu each.
    """
    nR, KR = h["n_max_radial"] + 1, h["basis_radial"] + 1
    nA, KA = h["n_max_angular"] + 1, h["basis_angular"] + 1
    T, L, nd, nn = h["n_types"], h["l_max_3b"], None, h["n_neurons"]
    NB = (L + 1) ** 2 - 1
    nd = nR + nA * (L + (h["l_max_4b"] >= 2) + (h["l_max_5b"] >= 1))
    geom = 20 + 8 + 10
    desc = (p_r * (geom + 5 * KR) + 2 * nR * T * KR
            + p_a * (geom + 5 * KA + 2 * nA * KA + 2 * NB + 2 * nA * NB)
            + nA * (3 * NB + 40))
    mlp = 4 * nd * nn + 6 * nn
    force = (2 * T * KR * nR + p_r * (geom + 12 * KR + 6)
             + p_a * (geom + 12 * KA + 4 * nA * KA + 4 * NB + NB * (4 * nA + 6) + 30)
             + nA * NB * 8)
    gather = (p_r + p_a) * (20 + 6 + 18)
    return dict(descriptor=desc, mlp=mlp, partial_forces=force, gather=gather)


def progress(msg):
    """A progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-2m", action="store_true")
    ap.add_argument("--steps-2m", type=int, default=20)
    ap.add_argument("--skin", type=float, default=SKIN,
                    help="Verlet skin in Angstrom (rows at r_c + skin, rebuilt after skin/2)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-structs", type=int, default=2000)
    ap.add_argument("--batch-sets", type=int, default=50)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-requests-bf16", type=int, default=200)
    ap.add_argument("--serve-budget-gb", type=float, default=2.0)
    return ap.parse_args()


def run_md(handle, pos_d, vel_d, types_d, masses, box, steps, warmup, torch):
    """Time `steps` NVE steps (graph-replayed, no instrumentation); then run the
    same number of steps again with HIP-event timing of every stage on the work
    stream, for the per-kernel averages."""
    th = torch.zeros((max(steps // THERMO_EVERY, 1), 13), dtype=torch.float64,
                     device=pos_d.device)
    if warmup:  # same thermo interval as the timed call: its captured step graph is reused
        handle.md_run_dev(pos_d, vel_d, types_d, masses, box, 1.0, warmup, THERMO_EVERY, th)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    handle.md_run_dev(pos_d, vel_d, types_d, masses, box, 1.0, steps, THERMO_EVERY, th)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rows = th.cpu().numpy()
    handle.set_timing(True)
    handle.md_run_dev(pos_d, vel_d, types_d, masses, box, 1.0, steps, THERMO_EVERY, th)
    torch.cuda.synchronize()
    stages = handle.timing()
    handle.set_timing(False)
    return dt, stages, rows


def serving_leg(nep, synth, params_of, n_req, budget_gb, prec):
    """Poisson stream of eval / 100-step NVE requests (log-uniform 64..100k atoms,
    2 species, FCC or BCC): saturation throughput with every request queued at
    once, then p50/p99 latency at 0.5 and 0.8 of that request rate."""
    h = synth.WORKLOADS["serve2"]
    masses = np.array(synth.MASSES["serve2"])
    reqs = synth.serving_stream(n_requests=n_req, rate_hz=1.0, seed=synth.SEED_STRUCT + 7)
    handle = nep.Handle(h, params_of(h), mlp_precision=prec)
    srv = nep.Server(handle, int(budget_gb * (1 << 30)), max_slots=64)

    def submit(r):
        if r.kind == "eval":
            return srv.submit(r.pos, r.types, r.box)
        return srv.submit(r.pos, r.types, r.box, kind=nep.NEP_REQ_MD, vel=r.vel,
                          masses=masses, n_steps=r.n_steps, dt=1.0)

    # warm-up (autotuner, workspace growth) on a few requests
    for r in reqs[:4]:
        srv.poll(submit(r), wait_ms=-1)
    srv.reset_stats()
    tickets = [submit(r) for r in reqs]
    for t in tickets:
        srv.poll(t, wait_ms=-1)
    sat = srv.stats()
    progress(f"serving saturation: {sat['requests_per_s']:.1f} req/s, p99 {sat['p99_ms']:.0f} ms")
    out = {"requests": n_req, "atoms_mean": float(np.mean([r.pos.shape[1] for r in reqs])),
           "saturation": {"requests_per_s": sat["requests_per_s"],
                          "atom_steps_per_s": sat["atom_steps_per_s"],
                          "p50_ms": sat["p50_ms"], "p99_ms": sat["p99_ms"],
                          "mean_batch_requests": sat["mean_batch_requests"]}}
    base_t = np.array([r.arrival_s for r in reqs])
    for frac in (0.5, 0.8):
        rate = frac * sat["requests_per_s"]
        arrivals = base_t * (1.0 / rate)       # the stream was drawn at 1 Hz
        srv.reset_stats()
        t0 = time.perf_counter()
        tickets = []
        for r, ta in zip(reqs, arrivals):
            dt = ta - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets.append(submit(r))
        for t in tickets:
            srv.poll(t, wait_ms=-1)
        st = srv.stats()
        progress(f"serving at {frac} of saturation: p50 {st['p50_ms']:.0f} ms, p99 {st['p99_ms']:.0f} ms")
        out[f"load_{frac}"] = {"rate_hz": rate, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                               "requests_per_s": st["requests_per_s"],
                               "atom_steps_per_s": st["atom_steps_per_s"],
                               "mean_batch_requests": st["mean_batch_requests"]}
    srv.close()
    handle.close()
    return out


def batch_leg(nep, synth, torch, n_struct, n_sets, reps=3):
    """Training-style population batch: n_struct periodic triclinic cells of
    8-256 atoms, 3 species, evaluated (energy, forces, virial) for n_sets
    parameter vectors z_p = mean + 0.1 eps_p in one nep_compute_batch call
    (rows built once and shared; the per-set passes replayed as one HIP
    graph).  The first call fixes the kernel shapes (autotuner); the next
    `reps` calls are timed whole (rows, graph capture and launch included);
    one more call with HIP-event stage timing gives the graph launch alone."""
    dev = torch.device("cuda:0")
    h = synth.WORKLOADS["train3"]
    structs = synth.random_structures(n_struct)
    pos, types, boxes, offs = synth.concat_structures(structs)
    n, S = pos.shape[1], boxes.shape[0]
    mean = synth.random_params(nep.nep_num_params(h))
    pop = synth.population(mean, n_sets)
    handle = nep.Handle(h, mean)
    pos_d = torch.tensor(pos, device=dev)
    types_d = torch.tensor(types, device=dev)
    e = torch.empty(n_sets, n, dtype=torch.float64, device=dev)
    f = torch.empty(n_sets, 3, n, dtype=torch.float64, device=dev)
    w = torch.empty(n_sets, 9, n, dtype=torch.float64, device=dev)
    t = torch.empty(n_sets, S, 10, dtype=torch.float64, device=dev)
    handle.compute_batch(offs, pos_d, types_d, boxes, pop, e, f, w, t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        handle.compute_batch(offs, pos_d, types_d, boxes, pop, e, f, w, t)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    handle.set_timing(True)
    handle.compute_batch(offs, pos_d, types_d, boxes, pop, e, f, w, t)
    torch.cuda.synchronize()
    stages = handle.timing()
    handle.set_timing(False)
    # the rest of one SNES generation: loss of every set (eq. loss) against
    # synthetic targets, then the SNES update and the next population
    npar = pop.shape[1]
    zeros_e = torch.zeros(S, dtype=torch.float64, device=dev)
    zeros_f = torch.zeros(3, n, dtype=torch.float64, device=dev)
    zeros_w = torch.zeros(S, 6, dtype=torch.float64, device=dev)
    pop_d = torch.tensor(pop, device=dev)
    loss = torch.empty(n_sets, 6, dtype=torch.float64, device=dev)
    mean_d = torch.tensor(mean, device=dev)
    sigma_d = torch.full((npar,), 0.1, dtype=torch.float64, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(synth.SEED_WEIGHTS)
    noise = torch.randn(n_sets, npar, dtype=torch.float64, device=dev, generator=gen)
    lam = (1.0, 1.0, 0.1, 1e-4, 1e-4)
    handle.batch_loss(offs, f, t, zeros_e, zeros_f, lam, loss, virial_target=zeros_w, params=pop_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        handle.batch_loss(offs, f, t, zeros_e, zeros_f, lam, loss, virial_target=zeros_w,
                          params=pop_d)
    torch.cuda.synchronize()
    loss_ms = (time.perf_counter() - t0) / reps * 1e3
    t0 = time.perf_counter()
    for _ in range(reps):
        handle.snes_step(mean_d, sigma_d, noise, loss, 1.0, 0.01, loss_stride=6)
        handle.snes_sample(mean_d, sigma_d, noise, pop_d)
    torch.cuda.synchronize()
    snes_ms = (time.perf_counter() - t0) / reps * 1e3
    # whole device-resident generations: sample -> batch (parameters in device
    # memory, rows reused, cached graph) -> loss -> SNES step, one stream, no
    # host round trip; the first generation builds the rows and the graph
    gens = 5
    handle.compute_batch_dev(offs, pos_d, types_d, boxes, pop_d, None, f, None, t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(gens):
        handle.snes_sample(mean_d, sigma_d, noise, pop_d)
        handle.compute_batch_dev(offs, pos_d, types_d, None, pop_d, None, f, None, t, reuse_rows=True)
        handle.batch_loss(offs, f, t, zeros_e, zeros_f, lam, loss, virial_target=zeros_w,
                          params=pop_d)
        handle.snes_step(mean_d, sigma_d, noise, loss, 1.0, 0.01, loss_stride=6)
    torch.cuda.synchronize()
    gen_dev_ms = (time.perf_counter() - t0) / gens * 1e3
    handle.set_timing(True)
    handle.compute_batch_dev(offs, pos_d, types_d, None, pop_d, None, f, None, t, reuse_rows=True)
    torch.cuda.synchronize()
    st_dev = handle.timing()
    handle.set_timing(False)
    # one parameter set through the same entry point (rows, one set's passes)
    one = [x[:1] for x in (e, f, w, t)]
    handle.compute_batch(offs, pos_d, types_d, boxes, pop[:1], *one)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        handle.compute_batch(offs, pos_d, types_d, boxes, pop[:1], *one)
    torch.cuda.synchronize()
    single_ms = (time.perf_counter() - t0) / reps * 1e3
    handle.close()
    del zeros_e, zeros_f, zeros_w, pop_d, loss, mean_d, sigma_d, noise
    g = stages.get("batch_graph", (float("nan"), 1))
    graph_ms = g[0] / max(g[1], 1)
    gd = st_dev.get("batch_graph", (float("nan"), 1))
    graph_dev_ms = gd[0] / max(gd[1], 1)
    del pos_d, types_d, e, f, w, t
    torch.cuda.empty_cache()
    return {"structures": S, "atoms": n, "param_sets": n_sets,
            "atom_evals_per_s": n * n_sets / dt, "evals_per_s": S * n_sets / dt,
            "ms_per_call": dt * 1e3, "graph_ms": graph_ms,
            "graph_atom_evals_per_s": n * n_sets / (graph_ms * 1e-3),
            "loss_ms": loss_ms, "snes_step_and_sample_ms": snes_ms,
            "generation_ms_host_params": dt * 1e3 + loss_ms + snes_ms,
            "device_generation_ms": gen_dev_ms,
            "device_graph_ms": graph_dev_ms,
            "device_generation_over_graph": gen_dev_ms / graph_dev_ms,
            "single_set_ms_per_call": single_ms,
            "single_set_atom_evals_per_s": n / (single_ms * 1e-3),
            "graph_rate_over_single_set": (n * n_sets / (graph_ms * 1e-3)) / (n / (single_ms * 1e-3)),
            "workload": ("train3: random triclinic cells, 8-256 atoms, density 0.05-0.09 "
                         "atoms/A^3, 3 species; NEP r_c 6/3.5 A, n_max 12/8, N_bas 12/8, "
                         "l_max 4, 100 neurons per species; E, F, W per vector")}


def cpu_baseline(h, params, seconds):
    """The oracle, as it is, on a bounded sample of the same workload: an
    FCC 6x6x6 sub-cell (864 atoms) of the same alloy and model, NVE steps."""
    from oracle import oracle as ora
    from paper_2205_10046_amd import synth
    pos, types, box = synth.lattice("fcc", 6, 4.05, 0.0, 4)
    m = np.array(synth.MASSES[WORKLOAD])
    vel = synth.maxwell_velocities(m[types], 300.0)
    n = pos.shape[1]
    t0 = time.perf_counter()
    ora.md_nve(h, params, pos, vel, types, m, box, 1.0, 1, 0)
    t1 = time.perf_counter() - t0           # one step + the initial evaluation
    steps = max(2, min(200, int(seconds / max(t1 / 2, 1e-3))))
    t0 = time.perf_counter()
    ora.md_nve(h, params, pos, vel, types, m, box, 1.0, steps, 0)
    dt = time.perf_counter() - t0
    # steps + 1 evaluations were done; count steps only
    cores = ora.get_threads()
    # the same sample on one core, fewer steps
    ora.set_threads(1)
    try:
        t0 = time.perf_counter()
        ora.md_nve(h, params, pos, vel, types, m, box, 1.0, 1, 0)
        t1c = time.perf_counter() - t0
        steps1 = max(4, min(50, int(seconds / 3 / max(t1c / 2, 1e-3))))
        t0 = time.perf_counter()
        ora.md_nve(h, params, pos, vel, types, m, box, 1.0, steps1, 0)
        dt1 = time.perf_counter() - t0
    finally:
        ora.set_threads(cores)
    return dict(value=n * steps / dt, unit="atom-step/s", cores=cores,
                kind="oracle",
                sample=(f"FP64 C oracle, {steps} NVE steps of an 864-atom 6x6x6 FCC "
                        f"sub-cell of the same 4-species alloy and model "
                        f"({dt:.1f} s); O(N^2) image pair search as written"),
                single_core={"value": n * steps1 / dt1, "cores": 1, "steps": steps1,
                             "seconds": dt1})


def heat_leg(nep, torch, h, params, pos, vel, types, box, reps=20):
    """Per-atom heat current J_i = W_i . v_i (eq. Ji) of the 131k alloy at
    300 K through nep_heat_current_dev: the whole call (a full evaluation and
    the contraction) and the contraction kernel alone (HIP events), with its
    algorithmic bytes (float32 virial 36 B, float64 velocity 24 B, index 4 B
    read and J_i 24 B written per atom)."""
    dev = torch.device("cuda:0")
    n = pos.shape[1]
    hd = nep.Handle(h, params)
    pos_d, vel_d = torch.tensor(pos, device=dev), torch.tensor(vel, device=dev)
    types_d = torch.tensor(types, device=dev)
    heat = torch.empty(3, n, dtype=torch.float64, device=dev)
    tot = torch.empty(3, dtype=torch.float64, device=dev)
    hd.heat_current_dev(pos_d, vel_d, types_d, box, heat=heat, total=tot)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        hd.heat_current_dev(pos_d, vel_d, types_d, box, heat=heat, total=tot)
    torch.cuda.synchronize()
    call_ms = (time.perf_counter() - t0) / reps * 1e3
    hd.set_timing(True)
    for _ in range(reps):
        hd.heat_current_dev(pos_d, vel_d, types_d, box, heat=heat, total=tot)
    torch.cuda.synchronize()
    st = hd.timing()
    hd.set_timing(False)
    hd.close()
    del pos_d, vel_d, types_d, heat, tot
    torch.cuda.empty_cache()
    k = st.get("heat_current", (float("nan"), 1))
    kernel_ms = k[0] / max(k[1], 1)
    nbytes = 88 * n
    return {"ms_per_call": call_ms, "kernel_ms": kernel_ms, "algorithmic_bytes": nbytes,
            "kernel_GBps": nbytes / (kernel_ms * 1e-3) / 1e9, "atoms": n}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(no multi-GPU path is built).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2205_10046_amd import nep, synth

    dev = torch.device("cuda:0")
    h = synth.WORKLOADS[WORKLOAD]
    # a parameter vector that keeps the lattice solid over the run (see synth)
    params = synth.solid_params(h, nep.nep_num_descriptors(h), nep.nep_num_params(h))
    pos, types, box = synth.fcc131k()
    masses = np.array(synth.MASSES[WORKLOAD])
    vel = synth.maxwell_velocities(masses[types], 300.0)
    n = pos.shape[1]
    p_r, p_a = 54.0, 42.0   # perfect FCC shells within 6 A and 5 A

    results = {}
    for prec in ([nep.NEP_MLP_FP32] + ([] if args.no_bf16 else [nep.NEP_MLP_BF16])):
        handle = nep.Handle(h, params, mlp_precision=prec, skin=args.skin)
        pos_d = torch.tensor(pos, device=dev)
        vel_d = torch.tensor(vel, device=dev)
        types_d = torch.tensor(types, device=dev)
        dt, stages, th = run_md(handle, pos_d, vel_d, types_d, masses, box, args.steps,
                                args.warmup, torch)
        results[prec] = (dt, stages, th)
        progress(f"fcc131k md mlp={'bf16' if prec else 'fp32'}: {dt / args.steps * 1e3:.4f} ms/step")
        if prec == nep.NEP_MLP_FP32:
            tune = handle.tuning()
            sched = handle.md_counters()
        handle.close()
        del pos_d, vel_d, types_d
        torch.cuda.empty_cache()

    try:
        heat = heat_leg(nep, torch, h, params, pos, vel, types, box)
    except nep.NepError as err:  # an auxiliary leg: report it, keep the MD line
        heat = {"error": str(err)}
    dt, stages, th = results[nep.NEP_MLP_FP32]
    value = n * args.steps / dt
    fl = algorithmic_flops(h, p_r, p_a)
    force_kernel = f"k_partial_forces<{tune['ng_force']}, {h['l_max_3b']}, false, {tune['lanes_force']}>"
    tr = measured_traffic(force_kernel)
    avg = {k: v[0] / v[1] for k, v in stages.items()}
    dom = max(("descriptor", "partial_forces"), key=lambda k: avg.get(k, 0.0))
    achieved = fl[dom] * n / (avg[dom] * 1e-3) / 1e12
    mlp_t = fl["mlp"] * n / (avg["mlp"] * 1e-3) / 1e12
    e = th[:, 1] + th[:, 2]
    out = {
        "metric": "NEP MD atom-step/s, 131k atoms, FP32 vs BF16-MLP; served p50/p99 latency",
        "value": value,
        "unit": "atom-step/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded lattice, Maxwell velocities, seeded parameter vector "
                "with a repulsive radial term so the lattice stays solid)",
        "config": {"workload": "fcc131k: 131,072-atom 4-species random FCC alloy "
                               "(32^3 cells, a=4.05 A), NEP r_c 6/5 A, n_max 8/6, "
                               "N_bas 8/6, l_max 4 + 4-body, 50 neurons per species, "
                               "NVE dt=1 fs from 300 K, thermo every 10 steps, "
                               f"rows at r_c + {args.skin:g} A rebuilt after a "
                               f"{args.skin / 2:g} A displacement",
                   "atoms": n, "mlp": "fp32"},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved,
                     "peak": PEAK_FP32_VALU, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU,
                     "traffic": (tr or {}).get("bytes"), "traffic_unit": "bytes per launch",
                     "traffic_detail": tr, "variant": tr["kernel"] if tr else force_kernel, "tuning": tune,
                     "flop_per_atom": fl[dom], "avg_launch_ms": avg[dom]},
        "mlp_roofline": {"bound": "mfma", "achieved": mlp_t, "peak": PEAK_FP32_MFMA,
                         "unit": "TFLOP/s", "frac": mlp_t / PEAK_FP32_MFMA,
                         "avg_launch_ms": avg["mlp"]},
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in stages.items()},
        "nve_drift_eV_per_atom": float(np.abs(e - e[0]).max() / n) if len(e) else None,
        "md_schedule": sched,
        "heat_current": heat,
    }
    if nep.NEP_MLP_BF16 in results:
        dtb, stb, _ = results[nep.NEP_MLP_BF16]
        avgb = {k: v[0] / v[1] for k, v in stb.items()}
        mlpb = fl["mlp"] * n / (avgb["mlp"] * 1e-3) / 1e12
        out["bf16"] = {"value": n * args.steps / dtb, "ms_per_step": dtb / args.steps * 1e3,
                       "mlp_roofline": {"bound": "mfma", "achieved": mlpb,
                                        "peak": PEAK_BF16_MFMA, "unit": "TFLOP/s",
                                        "frac": mlpb / PEAK_BF16_MFMA,
                                        "avg_launch_ms": avgb["mlp"]}}
    out["paper_context"] = {"A100_NEP3_MgAlCu": 1.5e7, "V100_NEP_carbon_4.2A": 3.6e6,
                            "unit": "atom-step/s", "note": "other hardware and models"}
    if not args.no_2m:
        # 2,000,000-atom BCC, l_max = 6 with 4-body and 5-body terms: FP32 vs BF16
        h2 = synth.WORKLOADS["bcc2m"]
        p2 = synth.solid_params(h2, nep.nep_num_descriptors(h2), nep.nep_num_params(h2))
        pos2, types2, box2 = synth.bcc2m()
        m2 = np.array(synth.MASSES["bcc2m"])
        vel2 = synth.maxwell_velocities(m2[types2], 300.0)
        out["bcc2m"] = {"atoms": pos2.shape[1], "steps": args.steps_2m}
        for prec, tag in ((nep.NEP_MLP_FP32, "fp32"), (nep.NEP_MLP_BF16, "bf16")):
            if tag == "bf16" and args.no_bf16:
                continue
            hd = nep.Handle(h2, p2, mlp_precision=prec, skin=args.skin)
            pd_ = torch.tensor(pos2, device=dev)
            vd_ = torch.tensor(vel2, device=dev)
            td_ = torch.tensor(types2, device=dev)
            t2, st2, _ = run_md(hd, pd_, vd_, td_, m2, box2, args.steps_2m, 2, torch)
            out["bcc2m"][tag] = {"value": pos2.shape[1] * args.steps_2m / t2,
                                 "ms_per_step": t2 / args.steps_2m * 1e3,
                                 "stages_ms_per_step": {k: v[0] / args.steps_2m
                                                        for k, v in st2.items()}}
            hd.close()
            del pd_, vd_, td_
            torch.cuda.empty_cache()
            progress(f"bcc2m md {tag}: {t2 / args.steps_2m * 1e3:.3f} ms/step")
    if not args.no_batch:
        out["population_batch"] = batch_leg(nep, synth, torch, args.batch_structs,
                                            args.batch_sets)
        progress(f"population batch: {out['population_batch']['ms_per_call']:.1f} ms per call")
    if not args.no_serve:
        pof = lambda hh: synth.random_params(nep.nep_num_params(hh))  # noqa: E731
        out["serving"] = {"fp32": serving_leg(nep, synth, pof, args.serve_requests,
                                              args.serve_budget_gb, nep.NEP_MLP_FP32)}
        sv = out["serving"]["fp32"]
        progress(f"serving fp32: {sv['saturation']['requests_per_s']:.1f} req/s at saturation, "
                 f"p99 {sv['load_0.5']['p99_ms']:.0f} / {sv['load_0.8']['p99_ms']:.0f} ms at 0.5 / 0.8 load")
        if not args.no_bf16:
            out["serving"]["bf16"] = serving_leg(nep, synth, pof, args.serve_requests_bf16,
                                                 args.serve_budget_gb, nep.NEP_MLP_BF16)
    if not args.no_cpu:
        progress("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(h, params, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
