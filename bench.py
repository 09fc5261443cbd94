#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

One step = one full pass of the hot path over the benchmark inputs:
  * heat: the 512^3 FP64 field (U[0,1] + central Gaussian hot spot, zero
    Dirichlet data), r = 1/6.5, 1000 explicit 7-point steps, Interior
    kernel on the caller's stream and Boundary planes on a second stream,
    two steps per pass over memory (the library's default; bit-identical to
    single steps);
  * CG: the 7-point Laplacian on 256^3 unknowns, b = A x* for a seeded
    x* ~ U[-1,1], x0 = 0, relative residual 1e-10, FP64.
Inputs are resident in HBM before the timed region; each step restarts both
solves from the same inputs.  The headline value is the heat sweep's
GLUP/s (1000 * 510^3 lattice-point updates per step over the heat phase's
time); CG's time-to-1e-10 is reported beside it.

Also reported: the dominant kernel's roofline (algorithmic bytes per launch
over its average HIP-event duration, against 8 TB/s), the HBM traffic that
rocprofv3 counters measured for it (when they were taken on the kernel as it
is now), a copy-probe ceiling, the other heat kernel forms, and the CPU
oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GLUP/s + achieved HBM GB/s (7-pt heat 512³ FP64 vs FP32); CG time-to-1e-10"
PEAK_HBM_GBS = 8000.0
# The Interior kernel of each pass form: its committed rocprofv3 HBM-traffic
# record and the sources it is compiled from.
CSRC = os.path.join(ROOT, "paper_2608_11882_amd", "csrc")
INTERIOR = {
    1: ("heat_interior", os.path.join(ROOT, "profiles", "heat_interior_f64_512_traffic.json"),
        ("heat_kernels.hip", "heat_tile.hpp")),
    2: ("heat2_interior", os.path.join(ROOT, "profiles", "heat2_interior_f64_512_traffic.json"),
        ("heat2_kernels.hip", "heat_tile2.hpp", "heat_tile.hpp")),
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(time_block):
    """Per-launch HBM bytes of the Interior kernel from the committed
    rocprofv3 counter summary, or None when the counters were taken on a
    different kernel source."""
    _, path, files = INTERIOR[time_block]
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != kernel_source_hash(files):
        return None
    return rec.get("hbm_bytes_per_launch")


# Per-point step time k-bar the paper measured on one GPU (tab:used-measurements):
# FP64 heat with a variable coefficient and a source, OpenMP offload,
# N = 512 .. 1280, 500 steps; k-bar = T / (steps (N-2)^3).  Context only:
# another equation (>= 32 B per point) on other hardware.
PAPER_KBAR = (("NVIDIA H100", 6.4042e-11), ("AMD MI250X, one GCD", 13.584e-11),
              ("Intel Data Center GPU Max 1550", 4.6676e-11))


def host_cpu():
    """CPU model, sockets and the physical cores this process may run on."""
    import subprocess
    info = {"nproc": os.cpu_count(), "allowed_cpus": len(os.sched_getaffinity(0))}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        keys = {"Model name": ("model", str), "Socket(s)": ("sockets", int),
                "Core(s) per socket": ("cores_per_socket", int),
                "Thread(s) per core": ("threads_per_core", int)}
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keys and k.strip() not in info:
                name, conv = keys[k.strip()]
                try:
                    info[name] = conv(v.strip())
                except ValueError:
                    info[name] = v.strip()
    except (OSError, subprocess.SubprocessError) as e:
        info["lscpu_error"] = str(e)
    cores = set()
    for c in os.sched_getaffinity(0):
        base = "/sys/devices/system/cpu/cpu%d/topology/" % c
        try:
            with open(base + "physical_package_id") as f1, open(base + "core_id") as f2:
                cores.add((f1.read().strip(), f2.read().strip()))
        except OSError:
            cores.add(("cpu", str(c)))
    info["physical_cores_allowed"] = len(cores)
    return info


def cpu_baseline(gpu_cg_iters, budget_s):
    """The oracle's timing, run in a child process: this one has loaded
    torch, whose OpenMP runtime pins the main thread once OMP_PROC_BIND is
    set, so the child starts a fresh runtime with one thread per physical
    core (OMP_PROC_BIND=close, OMP_PLACES=cores) and no GPU."""
    import subprocess
    env = dict(os.environ)
    env["OMP_PROC_BIND"] = "close"
    env["OMP_PLACES"] = "cores"
    res = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-child",
                          "--cpu-seconds", repr(float(budget_s)),
                          "--cpu-cg-iters", str(int(gpu_cg_iters))],
                         env=env, stdout=subprocess.PIPE, timeout=max(600.0, 20 * budget_s))
    if res.returncode != 0:
        raise RuntimeError("CPU baseline child failed (status %d)" % res.returncode)
    return json.loads(res.stdout.decode().strip().splitlines()[-1])


def cpu_baseline_child(gpu_cg_iters, budget_s):
    """The oracle, as it stands, on a bounded sample of the benchmark
    workload (the same seeded 512^3 field and 256^3 system): at one thread
    and at every physical core this process may use, the median of 3 runs
    each, timing the step (or iteration) loop only, set-up and copies
    excluded.  Runs without torch or a GPU."""
    info = host_cpu()   # before the OpenMP runtime starts and binds threads
    import oracle
    from paper_2608_11882_amd import inputs
    hcfg, ccfg = inputs.HEAT_LARGE, inputs.CG_LARGE
    u0_host = inputs.heat_large_f64(seed=hcfg["seed"], n=hcfg["n"])
    r = hcfg["r"]
    b_host = oracle.lap7_apply(inputs.manufactured_solution(ccfg["n"], seed=ccfg["seed"]))
    ncore = max(1, info["physical_cores_allowed"])
    n = u0_host.shape[0]
    lups_per_step = (n - 2) ** 3

    def heat_runs(threads, steps):
        oracle.set_threads(threads)
        loops = []
        for _ in range(3):
            oracle.heat(u0_host, r, steps)
            loops.append(oracle.last_loop_seconds())
        return loops

    def cg_runs(threads, iters):
        oracle.set_threads(threads)
        loops = []
        for _ in range(3):
            res = oracle.cg(b_host, 1e-30, iters)
            assert res.iters == iters
            loops.append(oracle.last_loop_seconds())
        return loops

    out = {}
    for label, threads, share in (("one_thread", 1, 0.4), ("all_cores", ncore, 0.6)):
        # size each run from one probe step / iteration
        per_step = max(statistics.median(heat_runs(threads, 1)), 1e-4)
        steps = max(1, int(0.5 * share * budget_s / (3 * per_step)))
        log("cpu baseline: heat %d steps x3 on %d thread(s)" % (steps, threads))
        hl = heat_runs(threads, steps)
        per_it = max(statistics.median(cg_runs(threads, 1)), 1e-4)
        iters = max(1, int(0.5 * share * budget_s / (3 * per_it)))
        log("cpu baseline: cg %d iterations x3 on %d thread(s)" % (iters, threads))
        cl = cg_runs(threads, iters)
        hmed, cmed = statistics.median(hl), statistics.median(cl)
        out[label] = {
            "threads": threads,
            "heat_glups": steps * lups_per_step / hmed / 1e9,
            "heat_steps_per_run": steps,
            "heat_loop_s": hl,
            "cg_s_per_iteration": cmed / iters,
            "cg_iterations_per_run": iters,
            "cg_loop_s": cl,
            "cg_time_to_tol_s_extrapolated": cmed / iters * gpu_cg_iters,
        }
    allc = out["all_cores"]
    return {
        "value": allc["heat_glups"],
        "unit": "GLUP/s",
        "cores": ncore,
        "kind": "oracle",
        "sample": ("heat: %d of the workload's 1000 steps on the same 512^3 FP64 field; cg: %d "
                   "iterations on the same 256^3 system (the time to 1e-10 is extrapolated to "
                   "the GPU's %d iterations); median of 3 runs, step / iteration loop timed "
                   "only; all %d physical cores (value) and one thread"
                   % (allc["heat_steps_per_run"], allc["cg_iterations_per_run"], gpu_cg_iters,
                      ncore)),
        "omp": {"OMP_PROC_BIND": os.environ.get("OMP_PROC_BIND"),
                "OMP_PLACES": os.environ.get("OMP_PLACES")},
        "host": info,
        "runs": out,
        "paper_context_glups": {
            hw: {"kbar_s": k, "glups": 1.0 / k / 1e9,
                 "workload": "FP64 variable-coefficient heat with a source, OpenMP offload, "
                             "one device, tab:used-measurements"}
            for hw, k in PAPER_KBAR},
    }


def to_bf16_device(u64_host, dev):
    """bfloat16 copy (torch.bfloat16, same bits) of a float64 host field,
    rounded once per node, converted in chunks of planes."""
    import numpy as np
    import torch
    from paper_2608_11882_amd import inputs
    out = torch.empty(u64_host.shape, dtype=torch.bfloat16, device=dev)
    for k0 in range(0, u64_host.shape[0], 64):
        bits = inputs.to_bf16_bits(u64_host[k0:k0 + 64]).view(np.int16)
        out[k0:k0 + 64].view(torch.int16).copy_(torch.from_numpy(bits))
    return out


def field_errors(got, ref):
    """max |got - ref| and ||got - ref||_2 / ||ref||_2, in float64, by chunks
    of planes (both on the device)."""
    emax, e2, r2 = 0.0, 0.0, 0.0
    for k0 in range(0, got.shape[0], 64):
        g = got[k0:k0 + 64].double()
        rf = ref[k0:k0 + 64].double()
        d = g - rf
        emax = max(emax, d.abs().max().item())
        e2 += (d * d).sum().item()
        r2 += (rf * rf).sum().item()
    return emax, (e2 / r2) ** 0.5 if r2 > 0 else 0.0


SR_SEED = 0x5EED


def timed_sweep(hc, u, un, u0, r, steps, sr=False):
    """Milliseconds of heat_step(u, un, r, steps) started from u0 (with
    sr: the bfloat16 sweep with stochastic rounding)."""
    import torch
    u.copy_(u0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    if sr:
        hc.heat_step_sr(u, un, r, steps, SR_SEED)
    else:
        hc.heat_step(u, un, r, steps, mode="split")
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def precision_section(hc, dev, u_init64, r_large, nsteps_large, with_oracle):
    """Reduced-precision sweeps, outside the timed region:
    * 512^3: the same field and steps as the headline in binary32 (and
      bfloat16 storage), GLUP/s and algorithmic GB/s beside FP64's;
    * 1024^3, r = 0.15, 500 steps, sine mode + U[-1e-3, 1e-3] (seed 3):
      binary32 and bfloat16-storage rates (nearest and stochastic rounding,
      the latter keyed by a fixed seed), and their max and relative-L2
      errors against the FP64 path on the full grid (the FP64 kernels are
      bit-identical to the oracle wherever the tests compare them) and
      against the FP64 oracle itself on a 256^3 instance of the same recipe."""
    import numpy as np
    import torch
    from paper_2608_11882_amd import inputs
    out = {}
    n = u_init64.shape[0]
    lups = nsteps_large * (n - 2) ** 3
    rate = {}
    for name, u0 in (("f64", u_init64), ("f32", u_init64.float()),
                     ("bf16", u_init64.to(torch.float32).to(torch.bfloat16)),
                     ("bf16_sr", u_init64.to(torch.float32).to(torch.bfloat16))):
        # (the bfloat16 rates do not depend on how the field was rounded)
        u, un = torch.empty_like(u0), torch.empty_like(u0)
        sr = name == "bf16_sr"
        timed_sweep(hc, u, un, u0, r_large, 10, sr)
        ms = timed_sweep(hc, u, un, u0, r_large, nsteps_large, sr)
        eb = u0.element_size()
        til = pass_tiling(hc, u, un, sr)
        rate[name] = {"tiling": til,
                      "glups": round(lups / (ms / 1e3) / 1e9, 2),
                      "algo_hbm_gbs": round(n_passes(nsteps_large, til) * eb
                                            * (n ** 3 + (n - 2) ** 3) / (ms / 1e3) / 1e9, 1)}
        del u, un, u0
    out["heat_512_rates"] = rate
    log("precision: 512^3 rates %s" % rate)

    cfg = inputs.HEAT_PRECISION
    N, r, steps, seed = cfg["n"], cfg["r"], cfg["steps"], cfg["seed"]
    log("precision: %d^3 inputs" % N)
    u64h = inputs.sine_field(N, N, N, noise=1e-3, seed=seed)
    lups = steps * (N - 2) ** 3
    res = {}
    ref = None
    for name in ("f64", "f32", "bf16", "bf16_sr"):
        if name == "f64":
            u0 = torch.from_numpy(u64h).to(dev)
        elif name == "f32":
            u0 = torch.from_numpy(u64h).to(dev).float()   # one rounding, to nearest even
        else:
            u0 = to_bf16_device(u64h, dev)
        u, un = torch.empty_like(u0), torch.empty_like(u0)
        sr = name == "bf16_sr"
        timed_sweep(hc, u, un, u0, r, 5, sr)
        ms = timed_sweep(hc, u, un, u0, r, steps, sr)
        eb = u0.element_size()
        til = pass_tiling(hc, u, un, sr)
        rec = {"tiling": til,
               "glups": round(lups / (ms / 1e3) / 1e9, 2),
               "algo_hbm_gbs": round(n_passes(steps, til) * eb * (N ** 3 + (N - 2) ** 3)
                                     / (ms / 1e3) / 1e9, 1),
               "ms": round(ms, 2)}
        del un, u0
        if name == "f64":
            ref = u
        else:
            emax, el2 = field_errors(u, ref)
            rec["max_err_vs_f64_full_grid"] = emax
            rec["rel_l2_err_vs_f64_full_grid"] = el2
            del u
        res[name] = rec
        torch.cuda.empty_cache()
    del ref
    torch.cuda.empty_cache()
    res["grid"] = [N, N, N]
    res["r"] = r
    res["steps"] = steps
    if with_oracle:
        import oracle
        m = 256
        log("precision: FP64 oracle on %d^3, %d steps" % (m, steps))
        s64 = inputs.sine_field(m, m, m, noise=1e-3, seed=seed)
        want = torch.from_numpy(oracle.heat(s64, r, steps)).to(dev)
        sub = {}
        for name in ("f32", "bf16", "bf16_sr"):
            u0 = (torch.from_numpy(s64).to(dev).float() if name == "f32"
                  else to_bf16_device(s64, dev))
            u, un = torch.empty_like(u0), torch.empty_like(u0)
            timed_sweep(hc, u, un, u0, r, steps, name == "bf16_sr")
            emax, el2 = field_errors(u, want)
            sub[name] = {"max_err": emax, "rel_l2_err": el2}
        sub["max_abs_u"] = float(want.abs().max().item())
        res["vs_oracle_256"] = sub
    out["heat_1024_precision"] = res
    return out


def ir_section(hc, b, xs, it64, ms64):
    """CG by binary64 iterative refinement around a binary32 inner CG on the
    same 256^3 system, outside the timed region: time to 1e-10 (median of
    3), inner iterations and outer steps, algorithmic bytes, and the error
    against the manufactured solution beside binary64 CG's."""
    import statistics as st
    import torch
    x = torch.zeros_like(b)
    work = torch.empty(hc.cg_ir_workspace_bytes(*b.shape[::-1]), dtype=torch.uint8, device=b.device)
    hc.cg_solve_ir(b, x, 1e-10, 10000, work=work)
    times = []
    for _ in range(3):
        x.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        status, it, outer, rel = hc.cg_solve_ir(b, x, 1e-10, 10000, work=work)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = st.median(times)
    n = b.numel()
    # inner: 30 B per unknown and iteration on average (d's steps taken two
    # at a time); per outer step: residual (x, b read, s written: 20 B),
    # x += d (20 B), clearing d (4 B), and at most one waiting step of d
    # (12 B, not counted)
    algo = 30.0 * n * it + 44.0 * n * outer
    err = (torch.linalg.norm(x - xs) / torch.linalg.norm(xs)).item()
    return {
        "time_to_tol_s": round(ms / 1e3, 5),
        "run_ms": [round(t, 3) for t in times],
        "status": status,
        "inner_iterations": it,
        "outer_steps": outer,
        "true_relres": rel,
        "us_per_inner_iteration": round(1e3 * ms / max(it, 1), 2),
        "algo_hbm_gbs": round(algo / (ms / 1e3) / 1e9, 1),
        "speedup_vs_f64_cg": round(ms64 / ms, 3),
        "f64_cg_iterations": it64,
        "err_vs_manufactured": err,
        "tiling": hc.get_cg_ir_tiling(),
    }


def batch_section(hc, dev, sequential_solves=True, shape=None):
    """The batched configuration, outside the timed region: 256 FP32
    problems with edges U{32..192} per axis, r ~ U[0.05, 0.16], U[0,1]
    fields, 200 steps.  The batch is autotuned on its own states, then timed
    as one captured graph of 200 persistent launches (median of 3), beside
    the same 200 steps as direct launches and 256 sequential single-problem
    solves (plain one-thread-per-node launches, and the fused z-march).
    With `shape` the batch takes that setting instead of the autotuner's;
    sequential_solves=False leaves out the sequential solves."""
    import numpy as np
    import torch
    from paper_2608_11882_amd import inputs
    cfg = inputs.BATCHED
    dims, rs, rng = inputs.batched_problems(cfg["count"], cfg["lo"], cfg["hi"], cfg["seed"],
                                            cfg["r_lo"], cfg["r_hi"])
    fields = inputs.batched_fields(dims, rng, dtype=np.float32)
    steps = cfg["steps"]
    batch = hc.Batch(dims, rs, "f32")
    u0, u, un = batch.empty(dev), batch.empty(dev), batch.empty(dev)
    for v, f in zip(batch.views(u0), fields):
        v.copy_(torch.from_numpy(f))
    lups = steps * sum((int(d[0]) - 2) * (int(d[1]) - 2) * (int(d[2]) - 2) for d in dims)

    def timed(fn, reps=3):
        out = []
        for _ in range(reps):
            u.copy_(u0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return statistics.median(out)

    if shape is None:
        log("batch: autotune")
        tuned_ms = batch.autotune(u0, trial_steps=20)
    else:
        batch.set_tiling(*shape)
        tuned_ms = float("nan")
    # a pass moves one step's bytes; two steps per pass make steps / 2 passes
    spp = batch.steps_per_pass()
    algo = (steps // spp + steps % spp) * batch.step_bytes
    ms_graph = timed(lambda: batch.step(u, un, steps, graph=True))
    ms_direct = timed(lambda: batch.step(u, un, steps, graph=False))
    res = {
        "problems": len(dims),
        "steps": steps,
        "lups": lups,
        "algo_bytes_per_step": batch.step_bytes,
        "tiling": batch.get_tiling(),
        "steps_per_pass": spp,
        "autotune_ms_per_step": round(tuned_ms, 4) if shape is None else None,
        "autotune_candidates": len(batch.tune_results()) if shape is None else 0,
        "graph": {"ms": round(ms_graph, 3), "glups": round(lups / (ms_graph / 1e3) / 1e9, 2),
                  "algo_hbm_gbs": round(algo / (ms_graph / 1e3) / 1e9, 1),
                  "pct_of_hbm_peak": round(100 * algo / (ms_graph / 1e3) / 1e9 / PEAK_HBM_GBS, 2),
                  "single_step_equivalent_gbs":
                      round(steps * batch.step_bytes / (ms_graph / 1e3) / 1e9, 1)},
        "direct_launches": {"ms": round(ms_direct, 3),
                            "glups": round(lups / (ms_direct / 1e3) / 1e9, 2)},
    }
    if sequential_solves:
        log("batch: sequential single-problem solves")
        # each problem on its own, in a contiguous array of its own (a packed
        # problem's rows are padded, so its view in the batch is strided)
        seq_u = [torch.from_numpy(f).to(dev) for f in fields]
        seq_un = [torch.empty_like(a) for a in seq_u]

        def sequential(mode):
            for p, (a, b) in enumerate(zip(seq_u, seq_un)):
                hc.heat_step(a, b, float(rs[p]), steps, mode=mode)
        ms_plain = timed(lambda: sequential("plain"), reps=1)
        ms_fused = timed(lambda: sequential("fused"), reps=1)
        res["sequential_plain"] = {"ms": round(ms_plain, 3),
                                   "glups": round(lups / (ms_plain / 1e3) / 1e9, 2)}
        res["sequential_fused"] = {"ms": round(ms_fused, 3),
                                   "glups": round(lups / (ms_fused / 1e3) / 1e9, 2)}
        res["speedup_vs_sequential_plain"] = round(ms_plain / ms_graph, 2)
    batch.close()
    return res


PAPER_KBAR_S = 6.4042e-11   # s per interior point and step, FP64 var-kappa, H100, 1 GPU


def n_passes(steps, tiling):
    """Passes over memory a run of `steps` makes (a last odd step is one)."""
    k = tiling["steps_per_pass"]
    return steps // k + steps % k


def pass_tiling(hc, u, un, sr=False):
    """The tile shape (and steps per pass) a sweep of these tensors runs with."""
    if hc.get_time_block() == 2 and not sr:
        return dict(hc.tiling2_for(u, un), steps_per_pass=2)
    return dict(hc.tiling_for(u, un, sr), steps_per_pass=1)


def vk_section(hc, dev):
    """The paper's own equation (variable kappa, source term; Eq. 1-4) on its
    test case (Eq. 2, 3, 5) at 512^3, outside the timed region: 500 steps
    (the paper's runs) in the split, fused and plain forms, FP64 and FP32,
    the Interior kernel's own rate from sampled HIP events, and the FP32
    result's error against FP64."""
    import torch
    from paper_2608_11882_amd import inputs
    cfg = inputs.VARCOEF
    n, steps = cfg["n"], cfg["steps"]
    log("varcoef: paper problem %d^3" % n)
    pb = inputs.paper_problem(n)
    beta = pb["beta"]
    lups = steps * (n - 2) ** 3
    algo_step = 8.0 * 2 * (n ** 3 + (n - 2) ** 3)   # u, kappa over all nodes; rhs, u_new inside
    tb = hc.get_time_block()
    passes = steps // tb + steps % tb              # a pass moves one step's bytes
    kname = "vk2_interior" if tb == 2 else "vk_interior"
    res = {"grid": [n, n, n], "steps": steps, "beta": beta, "dt": pb["dt"],
           "steps_per_pass": tb, "algo_bytes_per_lup_f64_per_pass": 32,
           "paper_kbar_glups_h100": round(1e-9 / PAPER_KBAR_S, 2)}

    def run(u0, kap, rhs, mode, u, un):
        u.copy_(u0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        hc.heat_vk_step(u, un, kap, rhs, beta, steps, mode=mode)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    out64 = None
    for dt, npdt in (("f64", "float64"), ("f32", "float32")):
        tdt = getattr(torch, npdt)
        u0 = torch.from_numpy(pb["u0"]).to(dev, tdt)
        kap = torch.from_numpy(pb["kappa"]).to(dev, tdt)
        rhs = torch.from_numpy(pb["rhs"]).to(dev, tdt)
        u, un = torch.empty_like(u0), torch.empty_like(u0)
        eb = 8 if dt == "f64" else 4
        forms = {}
        for mode in ("split", "fused", "plain"):
            ms = run(u0, kap, rhs, mode, u, un)
            npass = steps if mode == "plain" else passes
            forms[mode] = {"ms": round(ms, 3), "glups": round(lups / (ms / 1e3) / 1e9, 2),
                           "algo_hbm_gbs": round(npass * algo_step * eb / 8 / (ms / 1e3) / 1e9, 1)}
        if tb == 2:
            hc.set_time_block(1)
            for mode in ("split", "fused"):
                ms = run(u0, kap, rhs, mode, u, un)
                forms[mode + "_1_step"] = {"ms": round(ms, 3),
                                           "glups": round(lups / (ms / 1e3) / 1e9, 2)}
            hc.set_time_block(tb)
        hc.prof_enable(True, every=8)
        run(u0, kap, rhs, "split", u, un)
        ims, inb, ibytes = hc.prof_read(kname)
        hc.prof_enable(False)
        ok = bool(torch.isfinite(u).all().item()) and float(u.min()) >= 0.0
        til = (hc.vk2_tiling_for(u, un, kap, rhs) if tb == 2 else hc.vk_tiling_for(u, un, kap, rhs))
        entry = {"tiling": til, "forms_500_steps": forms, "result_ok_nonnegative_finite": ok}
        if inb:
            avg = ims / inb
            entry["interior_kernel"] = {
                "kernel": kname, "steps_per_launch": tb,
                "avg_launch_us": round(avg * 1e3, 2), "timed_launches": inb,
                "algo_bytes_per_launch": ibytes / inb,
                "achieved_gbs": round(ibytes / inb / (avg / 1e3) / 1e9, 1),
                "frac_of_hbm_peak": round(ibytes / inb / (avg / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}
        if dt == "f64":
            out64 = u.clone()
            entry["vs_paper_kbar_h100"] = round(forms["split"]["glups"] * PAPER_KBAR_S * 1e9, 2)
        else:
            d = u.double() - out64
            entry["max_err_vs_f64"] = float(d.abs().max())
            entry["rel_l2_err_vs_f64"] = float(torch.linalg.norm(d) / torch.linalg.norm(out64))
        res[dt] = entry
        del u0, kap, rhs, u, un
    del out64
    torch.cuda.empty_cache()
    return res


def kernels_section(hc, dev):
    """Each hot kernel a few times, for profiler passes (kernel traces and
    counters): the copy probe over two 1 GiB buffers, the two-step heat
    sweep (split form) on the 512^3 FP64 field and on 1024^3 fields in FP64,
    FP32 and bfloat16, the variable-coefficient sweep on the paper's 512^3
    test case (FP64), the batched configuration (FP32, its default shape),
    and 48 iterations of CG on the 256^3 system.  Prints each case's name,
    grid and launches in dispatch order."""
    import numpy as np
    import torch
    from paper_2608_11882_amd import inputs
    out = []

    def case(name, fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        out.append({"case": name, "ms": round(e0.elapsed_time(e1), 3)})
        log("kernels: %s %.3f ms" % (name, out[-1]["ms"]))

    a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        case("copy_probe 2 x 1 GiB", lambda: hc.copy_probe(a, b))
    del a, b
    hcfg = inputs.HEAT_LARGE
    u0 = torch.from_numpy(inputs.heat_large_f64(seed=hcfg["seed"], n=hcfg["n"])).to(dev)
    un = torch.empty_like(u0)
    case("heat f64 512^3 x20", lambda: hc.heat_step(u0, un, hcfg["r"], 20))
    del u0, un
    torch.cuda.empty_cache()
    for dt in ("f64", "f32", "bf16"):
        tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dt]
        n = 1024
        u = torch.rand((n, n, n), dtype=torch.float32, device=dev).to(tdt)
        for sl in (u[0], u[-1], u[:, 0], u[:, -1], u[:, :, 0], u[:, :, -1]):
            sl.zero_()
        un = torch.empty_like(u)
        case("heat %s 1024^3 x8" % dt, lambda: hc.heat_step(u, un, 0.15, 8))
        del u, un
        torch.cuda.empty_cache()
    pb = inputs.paper_problem(inputs.VARCOEF["n"])
    u = torch.from_numpy(pb["u0"]).to(dev)
    kap = torch.from_numpy(pb["kappa"]).to(dev)
    rhs = torch.from_numpy(pb["rhs"]).to(dev)
    un = torch.empty_like(u)
    case("varcoef f64 512^3 x8", lambda: hc.heat_vk_step(u, un, kap, rhs, pb["beta"], 8))
    del u, kap, rhs, un
    torch.cuda.empty_cache()
    cfg = inputs.BATCHED
    dims, rs, rng = inputs.batched_problems(cfg["count"], cfg["lo"], cfg["hi"], cfg["seed"],
                                            cfg["r_lo"], cfg["r_hi"])
    fields = inputs.batched_fields(dims, rng, dtype=np.float32)
    batch = hc.Batch(dims, rs, "f32")
    bu, bn = batch.empty(dev), batch.empty(dev)
    for v, f in zip(batch.views(bu), fields):
        v.copy_(torch.from_numpy(f))
    case("batch f32 256 problems x8 (direct launches)",
         lambda: batch.step(bu, bn, 8, graph=False))
    batch.close()
    del bu, bn
    ccfg = inputs.CG_LARGE
    m = ccfg["n"]
    xs = torch.from_numpy(inputs.manufactured_solution(m, seed=ccfg["seed"])).to(dev)
    bb = torch.empty_like(xs)
    hc.lap7_apply(xs, bb)
    x = torch.zeros_like(bb)
    case("cg f64 256^3 48 iterations", lambda: hc.cg_solve(bb, x, 1e-30, 48))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=24.0,
                    help="CPU time budget of the oracle baseline (0 skips it)")
    ap.add_argument("--heat-steps", type=int, default=1000, help=argparse.SUPPRESS)
    ap.add_argument("--precision", type=int, default=1, help=argparse.SUPPRESS)
    # "batch": only the batched configuration; "batch-kernels": the same
    # without the 256 sequential single-problem solves (for counter passes)
    # "kernels": each hot kernel a few times (kernels_section), for profiler
    # passes
    ap.add_argument("--section", choices=("all", "batch", "batch-kernels", "kernels"),
                    default="all", help=argparse.SUPPRESS)
    # the batch's shape (vec,threads,zdepth,pf,xcd,width_class,grid,item_depth)
    # instead of the autotuner's pick, for those sections
    ap.add_argument("--batch-shape", default=None, help=argparse.SUPPRESS)
    # the CPU baseline's child process (no torch, no GPU)
    ap.add_argument("--cpu-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-cg-iters", type=int, default=0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_child:
        print(json.dumps(cpu_baseline_child(args.cpu_cg_iters, args.cpu_seconds)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    shape = None
    if args.batch_shape:
        try:
            shape = tuple(int(v) for v in args.batch_shape.split(","))
        except ValueError:
            shape = ()
        if len(shape) != 8:
            ap.error("--batch-shape takes 8 comma-separated integers")

    import numpy as np
    import torch

    import paper_2608_11882_amd as hc
    from paper_2608_11882_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    hc.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.section == "kernels":
        print(json.dumps({"kernels": kernels_section(hc, dev)}), flush=True)
        return
    if args.section != "all":
        res = batch_section(hc, dev, sequential_solves=args.section == "batch", shape=shape)
        print(json.dumps({"batch_256_f32": res}), flush=True)
        return

    hcfg, ccfg = inputs.HEAT_LARGE, inputs.CG_LARGE
    n, r, nsteps = hcfg["n"], hcfg["r"], args.heat_steps
    m, tol, maxit = ccfg["n"], ccfg["tol"], ccfg["maxit"]

    log("inputs: heat %d^3, cg %d^3" % (n, m))
    u0_host = inputs.heat_large_f64(seed=hcfg["seed"], n=n)
    u_init = torch.from_numpy(u0_host).to(dev)
    u = torch.empty_like(u_init)
    un = torch.empty_like(u_init)
    xs_host = inputs.manufactured_solution(m, seed=ccfg["seed"])
    xs = torch.from_numpy(xs_host).to(dev)
    b = torch.empty_like(xs)
    hc.lap7_apply(xs, b)
    x = torch.zeros_like(b)
    work = torch.empty(hc.cg_workspace_bytes(m, m, m), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step():
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        u.copy_(u_init)
        x.zero_()
        e0.record()
        hc.heat_step(u, un, r, nsteps, mode="split")
        e1.record()
        st, it, rel = hc.cg_solve(b, x, tol, maxit, work=work)
        e2.record()
        return e0, e1, e2, st, it, rel

    for w in range(args.warmup):
        log("warmup %d/%d" % (w + 1, args.warmup))
        step()
    torch.cuda.synchronize()

    # time every 16th launch of each kernel: the events themselves cost GPU
    # time, so sampling keeps the timed run close to an unmeasured one
    hc.prof_enable(True, every=16)
    records = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        records.append(step())
        log("step %d/%d enqueued" % (k + 1, args.steps))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tb = hc.get_time_block()
    kname = INTERIOR[tb][0]
    int_ms, int_n, int_bytes = hc.prof_read(kname)
    cga_ms, cga_n, cga_b = hc.prof_read("cg_direction")
    cgb_ms, cgb_n, cgb_b = hc.prof_read("cg_update")
    cgx_ms, cgx_n, cgx_b = hc.prof_read("cg_update_x")
    hc.prof_enable(False)

    heat_ms = [e0.elapsed_time(e1) for e0, e1, _, _, _, _ in records]
    cg_ms = [e1.elapsed_time(e2) for _, e1, e2, _, _, _ in records]
    statuses = {rec[3] for rec in records}
    cg_iters = records[-1][4]
    cg_rel = records[-1][5]
    lups = nsteps * (n - 2) ** 3
    heat_s_total = sum(heat_ms) / 1e3
    glups = args.steps * lups / heat_s_total / 1e9
    # the bytes a pass must move: every stored node read once, every updated
    # node written once; with two steps per pass a run of nsteps makes
    # nsteps // 2 + nsteps % 2 passes
    algo_step = 8.0 * (n ** 3 + (n - 2) ** 3)
    passes = nsteps // tb + nsteps % tb
    heat_gbs = args.steps * passes * algo_step / heat_s_total / 1e9
    pass_us = 1e3 * statistics.mean(heat_ms) / passes
    single_step_gbs = args.steps * nsteps * algo_step / heat_s_total / 1e9
    ok_heat = bool(torch.isfinite(u).all().item()) and float(u.min()) >= 0.0

    # dominant kernel: the Interior sweep
    launch_bytes = int_bytes / max(int_n, 1)
    launch_ms = int_ms / max(int_n, 1)
    achieved = launch_bytes / (launch_ms / 1e3) / 1e9
    traffic = measured_traffic(tb)

    # copy-probe ceiling and the other kernel forms (outside the timed region)
    log("copy probe and kernel-form comparison")
    probe = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        hc.copy_probe(u_init, un)
        e1.record()
        torch.cuda.synchronize()
        probe.append(2 * u_init.numel() * 8 / (e0.elapsed_time(e1) / 1e3) / 1e9)
    copy_gbs = statistics.median(probe)
    # every form at one and at two steps per pass (plain: always one)
    variants = {}
    for form_tb in (tb, 3 - tb):
        hc.set_time_block(form_tb)
        for mode in ("split", "fused", "plain"):
            if mode == "plain" and form_tb == 2:
                continue
            u.copy_(u_init)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            hc.heat_step(u, un, r, 100, mode=mode)
            e1.record()
            torch.cuda.synchronize()
            key = mode if mode == "plain" else "%s_%d_step%s" % (mode, form_tb, "s" if form_tb > 1 else "")
            variants[key] = round(100 * (n - 2) ** 3 / (e0.elapsed_time(e1) / 1e3) / 1e9, 2)
    hc.set_time_block(tb)

    prec = varcoef = None
    if args.precision:
        prec = precision_section(hc, dev, u_init, r, nsteps, args.cpu_seconds > 0)
        log("precision: CG with binary32 inner solves")
        prec["cg_ir_256"] = ir_section(hc, b, xs, cg_iters, statistics.median(cg_ms))
        prec["cg_ir_256"]["f64_cg_err_vs_manufactured"] = (
            torch.linalg.norm(x - xs) / torch.linalg.norm(xs)).item()
        log("batched configuration")
        prec["batch_256_f32"] = batch_section(hc, dev)
        varcoef = vk_section(hc, dev)

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(cg_iters, args.cpu_seconds)

    tiling = hc.tiling_for(u, un) if tb == 1 else hc.tiling2_for(u, un)
    out = {
        "metric": METRIC,
        "value": round(glups, 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "heat 7-point FP64 512^3 r=1/6.5 x1000 steps (Interior/Boundary split) "
                        "+ CG 7-point Laplacian FP64 256^3 to relres 1e-10",
            "steps_per_pass": tb,
            "heat_grid": [n, n, n], "heat_steps": nsteps, "heat_r": r,
            "cg_grid": [m, m, m], "cg_tol": tol, "parallelism": "single-gpu",
            "tiling": tiling,
        },
        "heat": {
            "glups": round(glups, 3),
            "steps_per_pass": tb,
            "algo_hbm_gbs": round(heat_gbs, 1),
            "pct_of_hbm_peak": round(100 * heat_gbs / PEAK_HBM_GBS, 2),
            "pct_of_copy_probe": round(100 * heat_gbs / copy_gbs, 2),
            "single_step_equivalent_gbs": round(single_step_gbs, 1),
            "ms_per_time_step": round(sum(heat_ms) / len(heat_ms) / nsteps, 5),
            "run_ms": [round(t, 3) for t in heat_ms],
            "variability": round((max(heat_ms) - min(heat_ms)) / statistics.median(heat_ms), 4),
            "pass_us": round(pass_us, 2),
            "interior_share_of_pass": round(1e3 * launch_ms / pass_us, 4),
            "kernel_forms_glups_100_steps": variants,
            "result_ok": ok_heat,
        },
        "cg": {
            "time_to_tol_s": round(statistics.median(cg_ms) / 1e3, 5),
            "run_ms": [round(t, 3) for t in cg_ms],
            "iterations": cg_iters,
            "true_relres": cg_rel,
            "status": sorted(statuses),
            "us_per_iteration": round(1e3 * statistics.median(cg_ms) / max(cg_iters, 1), 2),
            # 58 B per unknown and iteration on average (x's steps taken four
            # at a time), plus the waiting 24 B steps of x after the last group
            "algo_hbm_gbs": round((58.0 * cg_iters + 24.0 * (cg_iters % 4)) * m ** 3
                                  / (statistics.median(cg_ms) / 1e3) / 1e9, 1),
            "direction_kernel_avg_us": round(1e3 * cga_ms / max(cga_n, 1), 2),
            # the update kernel takes r only (x's step waits) on three
            # iterations of four and r plus x's last four steps on the fourth
            "update_kernel_avg_us": round(1e3 * (3 * cgb_ms / max(cgb_n, 1) + cgx_ms / max(cgx_n, 1)) / 4, 2),
            "update_r_only_avg_us": round(1e3 * cgb_ms / max(cgb_n, 1), 2),
            "update_with_x_avg_us": round(1e3 * cgx_ms / max(cgx_n, 1), 2),
        },
        "precision": prec,
        "varcoef_512": varcoef,
        "copy_probe_gbs": round(copy_gbs, 1),
        "roofline": {
            "kernel": kname + "_f64",
            "steps_per_launch": tb,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "algo_bytes_per_launch": launch_bytes,
            "avg_launch_us": round(launch_ms * 1e3, 3),
            "timed_launches": int_n,
            "launch_sampling": "every 16th launch of each kernel, HIP events on its stream",
            "algo_bytes_rule": "every stored node of the planes the launch reads (its output "
                               "planes and %d on each side) once, every node it writes once"
                               % tb,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
