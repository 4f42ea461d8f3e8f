"""Benchmark: GDOF*iter/s of the spectral-element PCG solve on one MI355X.

One step = one complete solve, from x = 0 to relative residual 1e-10, of
the synthetic workload in the mixed-precision refinement mode (FP32 inner
Jacobi-PCG with FP64 gather-scatter sums and dots, FP64 residuals in the
refinement loop).  value = local dofs x (inner + outer iterations) per
second over the timed steps.  Inputs are resident in HBM before timing.

The default run (box32_N7_deformed, mixed_ir) reports beside it:
  - the same rate over unique nodes; the FP64 solve on the same GPU, the
    refinement with BF16 geometric factors and with the inner direction
    rounded to BF16 every step (an ablation of BF16 operator inputs), and
    the solves to a relative residual of 1e-8 (medians of as many solves as
    timed steps, at most five, after a warm-up);
  - energy-to-solution (the GPU package's energy counter around repeated
    FP64 and mixed solves);
  - the two-level Schwarz / multigrid preconditioner (flexible CG, FP64
    and mixed refinement, medians of five);
  - the roofline of the dominant kernel (the fused operator kernel of the
    inner loop: the first operator launch of every graph chunk records its
    own start and end events on the solve's stream) beside the library's
    streaming copy at the same traffic;
  - the learned-preconditioner leg on box24_N7_lognormal_helmholtz: pairs
    from the FP64 solver, training, scale calibration, then learned flexible
    CG, Jacobi PCG (both inside FP64 refinement) and FP64 Jacobi PCG on a
    held-out right-hand side, to residuals 1e-10 and 1e-8, medians of five;
  - the 64-problem batch (shared graph launches, mixed refinement, median of
    three) against the 64 FP64 solves one after another;
  - the CPU oracle (plain C, FP64, OpenMP over elements) on the host cores:
    its Jacobi-PCG solve of the benchmark workload from x = 0 to 1e-10 is
    timed (cpu_baseline), continued to 1e-13 for the reference solution x*,
    and every GPU solution of both legs is reported with its relative
    c-norm error against the oracle's x* (error_vs_oracle), as are three of
    the batch's problems.
--no-learned, --no-batch and --no-cpu drop those legs; --dot fp32 | dot2 sets the
accumulation of the inner loop's dots.  Other workloads: --workload batch64
(64 uneven problems), --workload box24_N7_lognormal_helmholtz --mode learned
(the learned leg alone, four held-out right-hand sides) and --workload
box20_N7 --mode strategies (the mixed-precision strategy table:
gather-scatter sums, dot accumulation and gather-scatter order).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="box32_N7_deformed",
                    help="box4_N7 | box16_N9_deformed | box32_N7_deformed | "
                         "box24_N7_lognormal_helmholtz | box20_N7 | batch64")
    ap.add_argument("--mode", default="mixed_ir", choices=["mixed_ir", "mixed_ir_bf16g",
                                                           "mixed_ir_bf16p", "fp64", "mixed",
                                                           "learned", "strategies"])
    ap.add_argument("--dot", default="fp64", choices=["fp64", "fp32", "dot2"],
                    help="accumulation of the FP32 loop's dots (mixed / mixed_ir modes)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle (baseline timing and reference solutions)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-preconditioner leg of the default run")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-problem batch leg of the default run")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="short run for hardware-counter collection: a 1 GiB device copy "
                         "(calibration), then 20 inner iterations of the solve; no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharded design is described, not built); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2503_02134_amd import mxsem as mx
    from paper_2503_02134_amd import workloads as W

    mx.lib()
    if args.workload == "batch64":
        return bench_batch(args)
    if args.mode == "learned":
        return bench_learned(args)
    if args.mode == "strategies":
        return bench_strategies(args)
    wl = W.WORKLOADS[args.workload]
    modes = {"mixed_ir": mx.MODE_MIXED_IR, "mixed_ir_bf16g": mx.MODE_MIXED_IR_BF16G,
             "mixed_ir_bf16p": mx.MODE_MIXED_IR_BF16P, "fp64": mx.MODE_FP64,
             "mixed": mx.MODE_MIXED}
    mode = modes[args.mode]
    ctx = mx.Context(0)
    t0 = time.perf_counter()
    xi, _ = mx.mxsem_gll(wl.N)
    bm = W.box_mesh(wl.ne, wl.N, xi, seed=wl.deform_seed)
    kf = W.lognormal_k(bm, wl.k_seed) if wl.k_seed is not None else None
    if wl.rhs == "manufactured":
        f, _ = W.manufactured(bm)
    else:
        f = W.random_smooth_rhs(bm, wl.rhs_seed)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    views = mx.VIEW_F64 | mx.VIEW_F32 | mx.VIEW_BF16
    if wl.name == "box32_N7_deformed" and not args.traffic_probe:
        views |= mx.VIEW_MG  # the multigrid leg below
    mesh = mx.Mesh(ctx, bm.E, wl.N, bm.xyz, bm.glo, bm.bnd, kcoef=kf, helm_h=wl.helm_h,
                   views=views)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    nloc = mesh.nloc
    log(f"workload {wl.name}: E={bm.E} N={wl.N} nloc={nloc} gen {t_gen:.1f}s setup {t_setup:.2f}s")
    b = mesh.mass_rhs(torch.as_tensor(f, device="cuda"))
    x = torch.zeros_like(b)
    opts = dict(mode=mode, tol=wl.tol, max_iter=20000, graph_chunk=16)
    if args.dot != "fp64":
        opts["dot"] = {"fp32": mx.DOT_F32, "dot2": mx.DOT_DOT2}[args.dot]
    if args.traffic_probe:
        return traffic_probe(mesh, b, mode)

    for i in range(args.warmup):
        x.zero_()
        _, st = mesh.solve(b, x, **opts)
        log(f"warmup {i}: it={st.iterations} outer={st.outer} res={st.rel_res:.2e} "
            f"{st.ms:.1f} ms")
    torch.cuda.synchronize()
    iters = 0
    ax_ms = []
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        x.zero_()
        _, st = mesh.solve(b, x, **opts)
        iters += st.iterations + st.outer
        ax_ms.append((st.ax_ms, st.ax_samples))
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for i, st in enumerate(stats):
        log(f"step {i}: it={st.iterations} outer={st.outer} reason={st.reason} "
            f"res={st.rel_res:.2e} {st.ms:.1f} ms ax={st.ax_ms * 1e3:.1f} us")
    value = nloc * iters / elapsed / 1e9
    sols = {args.mode: x.double().cpu().numpy()}  # GPU solutions, checked against the oracle
    copy_gbs = copy_ceiling(ctx, nloc * 20)

    # dominant kernel: fused operator kernel of the inner loop
    tot = sum(s for _, s in ax_ms)
    ax_avg_ms = sum(a * s for a, s in ax_ms) / max(tot, 1)
    vec_bytes = 8 if mode == mx.MODE_FP64 else 4
    # a plain stream of the operator's own split: z, p_old and G read (four
    # times what is written), p and w written
    mix_gbs = mix_ceiling(ctx, 4 * 2 * vec_bytes * nloc, 2 * vec_bytes * nloc)
    g_bytes = 6 * (8 if mode == mx.MODE_FP64 else 2 if mode == mx.MODE_MIXED_IR_BF16G else 4)
    hb = 0 if wl.helm_h == 0 else g_bytes // 6
    bytes_per_dof = 4 * vec_bytes + g_bytes + hb  # z, p_old in; p, w out; G (and h*B) in
    traffic_bytes = nloc * bytes_per_dof
    achieved = traffic_bytes / (ax_avg_ms * 1e-3) / 1e9 if ax_avg_ms > 0 else 0.0

    # FP64 solve and time-to-1e-8: one warm-up solve, then the median of
    # reps solves from x = 0 (reps = the timed steps, at most 5)
    reps = max(1, min(5, args.steps))

    def median_solve(xv, kw, warm=True):
        if warm:
            xv.zero_()
            mesh.solve(b, xv, **kw)
        runs = []
        for _ in range(reps):
            xv.zero_()
            _, st_ = mesh.solve(b, xv, **kw)
            runs.append(st_)
        return sorted(runs, key=lambda r: r.ms)[len(runs) // 2]

    extra = {}
    x64 = torch.zeros_like(b)
    opts64 = dict(mode=mx.MODE_FP64, tol=wl.tol, max_iter=20000, graph_chunk=16)
    s64 = median_solve(x64, opts64)
    extra["fp64"] = {"iterations": s64.iterations, "ms": round(s64.ms, 3),
                     "gdof_iter_s": round(nloc * s64.iterations / (s64.ms * 1e-3) / 1e9, 3),
                     "rel_res": s64.rel_res, "ax_us": round(s64.ax_ms * 1e3, 2),
                     "median_of": reps}
    mstep = sorted(stats, key=lambda r: r.ms)[len(stats) // 2]
    extra["time_to_solution_ms"] = {"fp64": round(s64.ms, 3), args.mode: round(mstep.ms, 3),
                                    "gain": round(s64.ms / mstep.ms, 3),
                                    "median_of": {"fp64": reps, args.mode: len(stats)}}
    sols["fp64"] = x64.cpu().numpy()
    if mode == mx.MODE_MIXED_IR:
        # the same refinement with BF16 geometric factors (FP32 vectors,
        # FP32 accumulation in the operator)
        xb = torch.zeros_like(b)
        _, sb = mesh.solve(b, xb, mode=mx.MODE_MIXED_IR_BF16G, tol=wl.tol, max_iter=20000,
                           graph_chunk=16)
        bb = 4 * 4 + 6 * 2 + (2 if wl.helm_h else 0)
        extra["mixed_ir_bf16g"] = {
            "ms": round(sb.ms, 3), "iterations": sb.iterations, "outer": sb.outer,
            "rel_res": sb.rel_res, "gain_vs_fp64": round(s64.ms / sb.ms, 3),
            "ax_us": round(sb.ax_ms * 1e3, 2),
            "ax_gbs": round(nloc * bb / (sb.ax_ms * 1e-3) / 1e9, 1) if sb.ax_ms > 0 else None}
        sols["mixed_ir_bf16g"] = xb.cpu().numpy()
        # ablation of BF16 operator inputs: the inner direction p rounded to
        # BF16 every step (numerics only; the vectors stay FP32 in memory)
        xp = torch.zeros_like(b)
        _, sp = mesh.solve(b, xp, mode=mx.MODE_MIXED_IR_BF16P, tol=wl.tol, max_iter=20000,
                           graph_chunk=16)
        extra["mixed_ir_bf16p"] = {
            "ms": round(sp.ms, 3), "iterations": sp.iterations, "outer": sp.outer,
            "reason": sp.reason, "fallback_used": sp.fallback_used, "rel_res": sp.rel_res,
            "gain_vs_fp64": round(s64.ms / sp.ms, 3)}
        sols["mixed_ir_bf16p"] = xp.cpu().numpy()
    if views & mx.VIEW_MG:
        # the two-level Schwarz / multigrid preconditioner (the paper's
        # solveM): FP64 and mixed refinement, medians like the FP64 solve
        mgr = {}
        for name, kw in (("fp64", dict(opts64, pc=mx.PC_MG)), (args.mode, dict(opts, pc=mx.PC_MG))):
            xm = torch.zeros_like(b)
            sm = median_solve(xm, kw)
            it = sm.iterations + sm.outer
            mgr[name] = {"ms": round(sm.ms, 3), "iterations": sm.iterations, "outer": sm.outer,
                         "rel_res": sm.rel_res, "median_of": reps,
                         "gdof_iter_s": round(nloc * it / (sm.ms * 1e-3) / 1e9, 3)}
            sols[f"multigrid/{name}"] = xm.cpu().numpy()
            log(f"multigrid {name}: {it} it, {sm.ms:.1f} ms, res {sm.rel_res:.2e}")
        mgr["gain_mixed_over_fp64"] = round(mgr["fp64"]["ms"] / mgr[args.mode]["ms"], 3)
        mgr["gain_over_jacobi"] = {"fp64": round(s64.ms / mgr["fp64"]["ms"], 3),
                                   args.mode: round(mstep.ms / mgr[args.mode]["ms"], 3)}
        extra["multigrid"] = mgr
    tt = {}
    for name, kw in (("fp64", opts64), (args.mode, opts)):
        xt = torch.zeros_like(b)
        st8 = median_solve(xt, dict(kw, tol=1e-8), warm=False)
        tt[name] = {"ms": round(st8.ms, 3), "iterations": st8.iterations, "outer": st8.outer,
                    "rel_res": st8.rel_res, "median_of": reps}
        sols[f"residual_1e-8/{name}"] = xt.cpu().numpy()
    extra["time_to_residual_1e-8"] = tt
    log(f"fp64: {extra['fp64']}; tt1e-8: {tt}")

    # energy to solution: the GPU package's energy counter around repeated solves
    read, why = energy_counter()
    if read is None:
        extra["energy_to_solution"] = {"unavailable": why}
    else:
        # The accumulator and its timestamp advance in steps (about one
        # second apart on this GPU): solves run back to back from one step
        # of the counter to a later one at least 4 s on, so the window holds
        # busy time only; the energy of a solve is the window's average power
        # times the solve's own time.
        en = {}
        for name, kw in (("fp64", opts64), (args.mode, opts)):
            def solve_once():
                x.zero_()
                _, st_ = mesh.solve(b, x, **kw)
                return st_.ms

            _, ts, _ = read()
            for _ in range(20):  # until the counter steps during a solve
                solve_once()
                ja, tsa, _ = read()
                if tsa != ts:
                    break
            times = []
            jb, tsb = ja, tsa
            while tsb - tsa < 4.0 and len(times) < 200:
                times.append(solve_once())
                jb, tsb, _ = read()
            watts = (jb - ja) / (tsb - tsa) if tsb > tsa else float("nan")
            per_ms = sum(times) / len(times)
            en[name] = {"joules_per_solve": round(watts * per_ms * 1e-3, 2),
                        "avg_watts": round(watts, 1), "solve_ms": round(per_ms, 2),
                        "solves": len(times), "counter_window_s": round(tsb - tsa, 3)}
        en["gain"] = round(en["fp64"]["joules_per_solve"] / en[args.mode]["joules_per_solve"], 3)
        en["counter"] = "amdsmi package energy accumulator (whole GPU, idle power included)"
        extra["energy_to_solution"] = en
        log(f"energy: {en}")

    out = {
        "metric": "GDOF*iter/s (local dofs x iterations / s) of the SEM PCG solve",
        "value": round(value, 4),
        "unit": "GDOF*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "ms_per_step_median": round(sorted(st.ms for st in stats)[len(stats) // 2], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f64" if mode == mx.MODE_FP64 else
                  "f32 (f64 gather-scatter sums, dots, refinement residuals)" if args.dot == "fp64"
                  else f"f32 (f64 gather-scatter sums and refinement residuals, {args.dot} dots)"),
        "data": "synthetic",
        "config": {"workload": wl.name, "E": bm.E, "N": wl.N, "nloc": nloc,
                   "mode": args.mode, "pc": "jacobi", "dot": args.dot, "tol": wl.tol,
                   "iterations_per_step": iters / args.steps},
        "roofline": {"bound": "hbm", "kernel": "ax_kernel (fused p-update + local operator)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "copy_ceiling_gbs": copy_gbs,
                     "stream_4to1_ceiling_gbs": mix_gbs,
                     "traffic": ax_traffic_from_profile(mode) if wl.name == "box32_N7_deformed"
                     else None,
                     "bytes_per_launch": traffic_bytes, "avg_launch_us": round(ax_avg_ms * 1e3, 2),
                     "launches_timed": tot},
        "setup_s": round(t_setup, 3),
        # the same rate counted over unique nodes instead of local dofs
        "gdof_iter_s_unique_nodes": round(value * (wl.ne * wl.N + 1) ** 3 / nloc, 4),
        **extra,
    }

    mesh.close()
    learned_sols = None
    if not args.no_learned and args.workload == "box32_N7_deformed":
        out["learned"], learned_sols = learned_leg(ctx, reps, log)
    batch_sols = None
    if not args.no_batch and args.workload == "box32_N7_deformed":
        out["batch"], batch_sols = batch_leg(ctx, 3, 1, keep=batch_oracle_problems())
        log(f"batch: {out['batch']}")
    ctx.close()
    if not args.no_cpu:
        out["cpu_baseline"], errs = oracle_leg(wl, sols)
        out["error_vs_oracle"] = errs
        if learned_sols is not None:
            errs5, cpu5 = oracle_reference_errors(W.WORKLOADS["box24_N7_lognormal_helmholtz"],
                                                  learned_sols["rhs_seed"], learned_sols["x"])
            out["learned"]["error_vs_oracle"] = errs5
            out["learned"]["cpu_oracle"] = cpu5
        if batch_sols is not None:
            out["batch"]["error_vs_oracle"], out["batch"]["cpu_oracle"] = \
                batch_oracle_errors(batch_sols)
    print(json.dumps(out), flush=True)


def energy_counter():
    """The package energy counter of the GPU that torch calls device 0, read
    through amdsmi (matched by PCI bus).  Returns (read, None), read() ->
    (joules, counter timestamp in s, host time in s), or (None, reason) when
    the counter cannot be read."""
    try:
        import amdsmi
        import torch
        amdsmi.amdsmi_init()
        bus = getattr(torch.cuda.get_device_properties(0), "pci_bus_id", None)
        handles = amdsmi.amdsmi_get_processor_handles()
        h = None
        for hh in handles:
            bdf = amdsmi.amdsmi_get_gpu_device_bdf(hh)
            if bus is not None and int(bdf.split(":")[1], 16) == int(bus):
                h = hh
        if h is None and len(handles) == 1:
            h = handles[0]
        if h is None:
            return None, f"no amdsmi device on PCI bus {bus} among {len(handles)}"

        def read():
            d = amdsmi.amdsmi_get_energy_count(h)
            return (d["energy_accumulator"] * d["counter_resolution"] * 1e-6,
                    d["timestamp"] * 1e-9, time.perf_counter())

        d = amdsmi.amdsmi_get_energy_count(h)
        log(f"energy counter: {d}")
        return read, None
    except Exception as e:  # no amdsmi, no permission, no counter
        return None, f"{type(e).__name__}: {e}"


def copy_ceiling(ctx, nbytes):
    """Read + write bandwidth of the library's streaming copy (one pass,
    non-temporal loads and stores) of nbytes: with nbytes = 20 B per local
    dof it moves the same 40 B per dof as one operator launch, so it is the
    measured ceiling set beside the operator kernel's bandwidth.  Median of
    20 launches, each timed by its own events on the context's stream."""
    import torch

    from paper_2503_02134_amd import mxsem as mx
    nbytes = (nbytes // 16) * 16
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        mx.mxsem_stream_copy(ctx.h, src, dst)
    assert torch.equal(src, dst)
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        mx.mxsem_stream_copy(ctx.h, src, dst)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    del src, dst
    sec = sorted(times)[len(times) // 2]
    return round(2 * nbytes / sec / 1e9, 1)


def mix_ceiling(ctx, read_bytes, write_bytes):
    """Bandwidth of the library's streaming mix (mxsem_stream_mix: one pass,
    non-temporal, read_bytes read for write_bytes written) at the operator
    kernel's own split, 32 bytes read and 8 written per local dof: the
    measured ceiling of a plain stream with the operator's bytes.  Median of
    20 launches, each timed by its own events on the context's stream."""
    import torch

    from paper_2503_02134_amd import mxsem as mx
    write_bytes = (write_bytes // 16) * 16
    k = read_bytes // write_bytes
    src = torch.ones(k * write_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty(write_bytes // 4, dtype=torch.float32, device="cuda")
    for _ in range(3):
        mx.mxsem_stream_mix(ctx.h, src, dst)
    assert bool((dst == float(k)).all())
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        mx.mxsem_stream_mix(ctx.h, src, dst)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    del src, dst
    sec = sorted(times)[len(times) // 2]
    return round((k + 1) * write_bytes / sec / 1e9, 1)


def traffic_probe(mesh, b, mode):
    """Kernels whose per-dispatch FETCH_SIZE / WRITE_SIZE counters give the
    operator kernel's HBM traffic: a plain 1 GiB device-to-device copy of
    known size (its counters calibrate the scale), then 20 iterations of the
    inner solve (20 operator-kernel dispatches)."""
    import torch

    from paper_2503_02134_amd import mxsem as mx
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy of {src.numel() * 4} bytes done")
    x = torch.zeros_like(b)
    _, st = mesh.solve(b, x, mode=mx.MODE_MIXED if mode == mx.MODE_MIXED_IR else mode,
                       tol=0.0, max_iter=20, graph_chunk=4)
    torch.cuda.synchronize()
    log(f"probe solve: {st.iterations} iterations")


def ax_traffic_from_profile(mode):
    """HBM bytes per operator-kernel launch measured by the hardware counters,
    read from the committed profile summary; None when the operator kernel's
    source has changed since (its SHA-256 is recorded with the figures)."""
    import hashlib
    import re
    from paper_2503_02134_amd import mxsem as mx
    if mode != mx.MODE_MIXED_IR:
        return None
    prof = os.path.join(ROOT, "profiles", "ax_traffic_box32_N7_deformed.md")
    src = os.path.join(ROOT, "paper_2503_02134_amd", "csrc", "ax.hip")
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m_sha = re.search(r"ax\.hip sha256: ([0-9a-f]{64})", text)
    m_b = re.search(r"traffic_bytes_per_launch: ([0-9]+)", text)
    if not m_sha or not m_b or m_sha.group(1) != sha:
        return None
    return int(m_b.group(1))


def batch_leg(ctx, steps, warmup, keep=()):
    """64 uneven Poisson problems (E in {8^3,12^3,16^3,24^3}, N in {5,7,9},
    seeded smooth RHS) solved together in shared graph launches (mixed
    refinement, medians over `steps` batch solves), against the 64 FP64
    solves one after another on the same GPU.  Returns the result record and
    the solutions of the problems listed in `keep` (for the oracle's errors)."""
    import torch

    from paper_2503_02134_amd import mxsem as mx
    from paper_2503_02134_amd import workloads as W
    draws = W.batch_draws()
    meshes, bs = [], []
    t0 = time.perf_counter()
    for q, (ne, N, seed) in enumerate(draws):
        xi, _ = mx.mxsem_gll(N)
        bm = W.box_mesh(ne, N, xi)
        m = mx.Mesh(ctx, bm.E, N, bm.xyz, bm.glo, bm.bnd)
        f = W.random_smooth_rhs(bm, seed)
        bs.append(m.mass_rhs(torch.as_tensor(f, device="cuda")))
        meshes.append(m)
        del bm
        if q % 16 == 15:
            log(f"batch64: {q + 1} problems set up ({time.perf_counter() - t0:.1f}s)")
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    nloc = [m.nloc for m in meshes]
    log(f"batch64: {len(meshes)} problems, {sum(nloc)} local dofs, setup {t_setup:.1f}s")
    cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), "mxsem_tune.json")
    t0 = time.perf_counter()
    bt = mx.mxsem_batch_create(ctx.h, [m.h for m in meshes], tune_cache=cache)
    t_tune = time.perf_counter() - t0
    xs = [torch.zeros_like(b) for b in bs]
    opts = mx.solve_opts(mode=mx.MODE_MIXED_IR, tol=1e-10, max_iter=20000, graph_chunk=16)
    for _ in range(warmup):
        for x in xs:
            x.zero_()
        mx.mxsem_batch_solve(bt, opts, bs, xs)
    torch.cuda.synchronize()
    times, its = [], 0
    for _ in range(steps):
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = mx.mxsem_batch_solve(bt, opts, bs, xs)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        its = sum(n * (s.iterations + s.outer) for n, s in zip(nloc, sts))
    el = sorted(times)[len(times) // 2]
    conv = sum(s.reason == mx.CONVERGED for s in sts)
    worst = max(s.rel_res for s in sts)
    kept = {p: xs[p].cpu().numpy() for p in keep}
    # the same problems one after another in FP64
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its64 = 0
    for m, b in zip(meshes, bs):
        _, s = m.solve(b, mode=mx.MODE_FP64, tol=1e-10, max_iter=20000)
        its64 += m.nloc * s.iterations
    torch.cuda.synchronize()
    el64 = time.perf_counter() - t0
    rec = {
        "problems": len(meshes), "nloc_total": sum(nloc), "mode": "mixed_ir (batched)",
        "tol": 1e-10, "ms": round(el * 1e3, 3), "median_of": steps,
        "gdof_iter_s": round(its / el / 1e9, 4),
        "converged": conv, "worst_rel_res": worst,
        "sequential_fp64": {"ms": round(el64 * 1e3, 3),
                            "gdof_iter_s": round(its64 / el64 / 1e9, 4)},
        "batch_vs_sequential_fp64_time": round(el64 / el, 3),
        "setup_s": round(t_setup, 2), "tune_s": round(t_tune, 2),
    }
    mx.mxsem_batch_destroy(bt)
    for m in meshes:
        m.close()
    return rec, kept


def bench_batch(args):
    """The batch leg on its own, as the bench line (value: the batched solve's
    GDOF*iter/s)."""
    from paper_2503_02134_amd import mxsem as mx
    ctx = mx.Context(0)
    rec, _ = batch_leg(ctx, max(args.steps, 1), args.warmup)
    out = {
        "metric": "GDOF*iter/s (local dofs x iterations / s) of the SEM PCG solve",
        "value": rec["gdof_iter_s"], "unit": "GDOF*iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": rec["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (f64 gather-scatter sums, dots, refinement residuals)",
        "data": "synthetic",
        "config": {"workload": "batch64", "problems": rec["problems"],
                   "nloc_total": rec["nloc_total"], "mode": rec["mode"], "tol": rec["tol"]},
        **{k: v for k, v in rec.items() if k not in ("problems", "nloc_total", "mode", "tol")},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_learned(args):
    """Log-normal Helmholtz (24^3, N = 7, k = exp(g), h = 1): train the
    learned preconditioner on GPU-generated pairs, calibrate its scale on a
    training right-hand side, then time learned flexible CG (inside FP64
    refinement) on held-out right-hand sides against Jacobi PCG (same
    refinement) and FP64 Jacobi PCG."""
    import numpy as np
    import torch

    from paper_2503_02134_amd import mxsem as mx
    from paper_2503_02134_amd import workloads as W
    from paper_2503_02134_amd.learned import (Network, calibrate_scale, make_pairs, rhs_batch,
                                              train)
    wl = W.WORKLOADS["box24_N7_lognormal_helmholtz"]
    ctx = mx.Context(0)
    xi, _ = mx.mxsem_gll(wl.N)
    bm = W.box_mesh(wl.ne, wl.N, xi)
    kf = W.lognormal_k(bm, wl.k_seed)
    mesh = mx.Mesh(ctx, bm.E, wl.N, bm.xyz, bm.glo, bm.bnd, kcoef=kf, helm_h=wl.helm_h)
    t0 = time.perf_counter()
    train_rhs = rhs_batch(bm, mesh, range(5100, 5116))
    R, E = make_pairs(mesh, train_rhs, samples=8, mesh_np=bm, seed=11)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = Network(mesh, seed=3)
    t0 = time.perf_counter()
    losses = train(net, R, E, steps=300, batch=4, lr=2e-3, seed=1, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del R, E
    lam, cal = calibrate_scale(net, mesh, train_rhs[0], log=log)
    net.attach()
    ev = rhs_batch(bm, mesh, range(5900, 5900 + max(args.steps, 1)))
    nloc = mesh.nloc
    for b in ev[: args.warmup]:
        mesh.solve(b, mode=mx.MODE_MIXED_IR, pc=mx.PC_LEARNED, method=mx.METHOD_FCG, tol=wl.tol)
    torch.cuda.synchronize()
    rows = []
    its = 0
    xl = [torch.zeros_like(b) for b in ev]
    t0 = time.perf_counter()
    for b, x in zip(ev, xl):
        _, st = mesh.solve(b, x, mode=mx.MODE_MIXED_IR, pc=mx.PC_LEARNED, method=mx.METHOD_FCG,
                           tol=wl.tol, max_iter=50000)
        its += st.iterations + st.outer
        rows.append(st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    jac, f64, errs = [], [], []
    for b, x in zip(ev, xl):
        xj = torch.zeros_like(b)
        _, sj = mesh.solve(b, xj, mode=mx.MODE_MIXED_IR, tol=wl.tol, max_iter=50000)
        x6 = torch.zeros_like(b)
        _, s6 = mesh.solve(b, x6, mode=mx.MODE_FP64, tol=wl.tol, max_iter=50000)
        jac.append(sj)
        f64.append(s6)
        errs.append(float(torch.linalg.vector_norm(x - x6) / torch.linalg.vector_norm(x6)))
    # time to a 1e-8 residual on every held-out right-hand side
    tt = {"learned": [], "jacobi_mixed_ir": [], "fp64_jacobi": []}
    for b in ev:
        for name, kw in (("learned", dict(mode=mx.MODE_MIXED_IR, pc=mx.PC_LEARNED,
                                          method=mx.METHOD_FCG)),
                         ("jacobi_mixed_ir", dict(mode=mx.MODE_MIXED_IR)),
                         ("fp64_jacobi", dict(mode=mx.MODE_FP64))):
            xt = torch.zeros_like(b)
            _, s8 = mesh.solve(b, xt, tol=1e-8, max_iter=50000, **kw)
            tt[name].append({"ms": round(s8.ms, 2), "iterations": s8.iterations + s8.outer,
                             "rel_res": s8.rel_res})
    out = {
        "metric": "GDOF*iter/s (local dofs x iterations / s) of the SEM PCG solve",
        "value": round(nloc * its / el / 1e9, 4), "unit": "GDOF*iter/s", "n_gpus": 1,
        "steps": len(ev), "warmup": args.warmup, "ms_per_step": round(el * 1e3 / len(ev), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 loop, bf16-in/f32-accumulate network, f64 sums/dots/refinement",
        "data": "synthetic",
        "config": {"workload": wl.name, "E": bm.E, "N": wl.N, "nloc": nloc,
                   "mode": "mixed_ir + flexible CG, learned preconditioner", "tol": wl.tol},
        "learned": {"iterations": [s.iterations + s.outer for s in rows],
                    "ms": [round(s.ms, 2) for s in rows],
                    "fallback_steps": [s.fallback_used for s in rows],
                    "rel_res": [s.rel_res for s in rows], "rel_diff_vs_fp64": errs,
                    "scale": lam, "calibration_iterations": {str(k): v for k, v in cal.items()},
                    "train_loss_first": losses[0],
                    "train_loss_last20": float(np.mean(losses[-20:])),
                    "train_s": round(t_train, 2), "data_s": round(t_data, 2)},
        "jacobi_mixed_ir": {"iterations": [s.iterations + s.outer for s in jac],
                            "ms": [round(s.ms, 2) for s in jac]},
        "fp64_jacobi": {"iterations": [s.iterations for s in f64],
                        "ms": [round(s.ms, 2) for s in f64]},
        "time_to_1e-8": tt,
    }
    print(json.dumps(out), flush=True)
    net.close()
    mesh.close()
    ctx.close()


def bench_strategies(args):
    """The mixed-precision strategies of Sec. 4.2.1 and Sec. 5.2.1 on one GPU: the
    FP32 CG loop with the gather-scatter sums in FP32 or FP64, the dots in
    FP32, FP64 or compensated FP32 (Dot2), and the gather-scatter in one
    order per node or in the summation order of a pairwise exchange between
    ranks (every element a rank of its own), with the identity and the
    Jacobi preconditioner, to the workload's recursive tolerance; FP64 CG
    beside.  Then the rank-count study: the pairwise order with the elements
    cut into 1 to 64 blocks of ranks, FP32 or FP64 gather-scatter sums.  value: local dofs x iterations / s over every solve of
    the table (the solves differ in cost only by their reductions)."""
    import torch

    from paper_2503_02134_amd import mxsem as mx
    from paper_2503_02134_amd import workloads as W
    wl = W.WORKLOADS[args.workload]
    ctx = mx.Context(0)
    xi, _ = mx.mxsem_gll(wl.N)
    bm = W.box_mesh(wl.ne, wl.N, xi, seed=wl.deform_seed)
    f = W.manufactured(bm)[0] if wl.rhs == "manufactured" else W.random_smooth_rhs(bm, wl.rhs_seed)
    mesh = mx.Mesh(ctx, bm.E, wl.N, bm.xyz, bm.glo, bm.bnd)
    nloc = mesh.nloc
    b = mesh.mass_rhs(torch.as_tensor(f, device="cuda"))
    log(f"strategies on {wl.name}: E={bm.E} N={wl.N} nloc={nloc} tol={wl.tol}")
    pcs = (("identity", mx.PC_IDENTITY), ("jacobi", mx.PC_JACOBI))
    ref = {}
    rows = []
    its = 0
    el = 0.0
    for pname, pc in pcs:
        x64 = torch.zeros_like(b)
        mesh.solve(b, x64, mode=mx.MODE_FP64, pc=pc, tol=wl.tol, max_iter=wl.maxit)  # warm-up
        x64.zero_()
        _, s6 = mesh.solve(b, x64, mode=mx.MODE_FP64, pc=pc, tol=wl.tol, max_iter=wl.maxit)
        ref[pname] = x64
        rows.append({"pc": pname, "loop": "fp64", "gs_sums": "fp64", "dot": "fp64",
                     "order": "one", "reason": s6.reason, "iterations": s6.iterations,
                     "rec_res": s6.rel_res_recursive, "true_res": s6.rel_res,
                     "rel_diff_vs_fp64": 0.0, "ms": round(s6.ms, 2)})
        its += s6.iterations
        el += s6.ms
        for gname, mode in (("fp64", mx.MODE_MIXED), ("fp32", mx.MODE_FP32_ALL)):
            for dname, dot in (("fp64", mx.DOT_F64), ("fp32", mx.DOT_F32), ("dot2", mx.DOT_DOT2)):
                for oname, order in (("one", mx.GS_ORDER_ONE),
                                     ("pairwise_every_element", mx.GS_ORDER_PAIRWISE)):
                    x = torch.zeros_like(b)
                    _, st = mesh.solve(b, x, mode=mode, pc=pc, tol=wl.tol, max_iter=wl.maxit,
                                       dot=dot, gs_order=order)
                    d = float(torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64))
                    log(f"  {pname:8s} gs {gname} dot {dname:4s} {oname:8s}: it={st.iterations:5d} "
                        f"reason={st.reason} rec={st.rel_res_recursive:.2e} true={st.rel_res:.2e} "
                        f"diff={d:.2e} {st.ms:.1f} ms")
                    rows.append({"pc": pname, "loop": "fp32", "gs_sums": gname, "dot": dname,
                                 "order": oname, "reason": st.reason,
                                 "iterations": st.iterations, "rec_res": st.rel_res_recursive,
                                 "true_res": st.rel_res, "rel_diff_vs_fp64": d,
                                 "ms": round(st.ms, 2)})
                    its += st.iterations
                    el += st.ms
    # rank-count study: the pairwise order with the elements cut into
    # px x py x pz blocks of ranks (Jacobi CG, FP64 dots)
    ranks_rows = []
    for layout in ((1, 1, 1), (1, 1, 2), (1, 2, 2), (2, 2, 2), (3, 3, 3), (4, 4, 4), None):
        mesh.set_ranks(None if layout is None else W.block_ranks(wl.ne, *layout))
        nr = bm.E if layout is None else layout[0] * layout[1] * layout[2]
        for gname, mode in (("fp32", mx.MODE_FP32_ALL), ("fp64", mx.MODE_MIXED)):
            x = torch.zeros_like(b)
            _, st = mesh.solve(b, x, mode=mode, pc=mx.PC_JACOBI, tol=wl.tol, max_iter=wl.maxit,
                               dot=mx.DOT_F64, gs_order=mx.GS_ORDER_PAIRWISE)
            log(f"  pairwise ranks {nr:5d} {str(layout):10s} gs {gname}: it={st.iterations:5d} "
                f"reason={st.reason} rec={st.rel_res_recursive:.2e} true={st.rel_res:.2e}")
            ranks_rows.append({"ranks": nr, "layout": "every element" if layout is None else
                               "x".join(str(c) for c in layout), "gs_sums": gname,
                               "reason": st.reason, "iterations": st.iterations,
                               "rec_res": st.rel_res_recursive, "true_res": st.rel_res,
                               "ms": round(st.ms, 2)})
            its += st.iterations
            el += st.ms
    mesh.set_ranks(None)
    reasons = {mx.CONVERGED: "converged", mx.MAX_ITER: "max_iter", mx.STAGNATED: "stagnated",
               mx.BREAKDOWN: "breakdown"}
    for r in rows + ranks_rows:
        r["reason"] = reasons.get(r["reason"], str(r["reason"]))
    out = {
        "metric": "GDOF*iter/s (local dofs x iterations / s) of the SEM PCG solve",
        "value": round(nloc * its / (el / 1e3) / 1e9, 4), "unit": "GDOF*iter/s", "n_gpus": 1,
        "steps": len(rows) + len(ranks_rows), "warmup": 1,
        "ms_per_step": round(el / (len(rows) + len(ranks_rows)), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 loop; gather-scatter sums and dots per row", "data": "synthetic",
        "config": {"workload": wl.name, "E": bm.E, "N": wl.N, "nloc": nloc,
                   "mode": "strategy table", "tol": wl.tol},
        "strategies": rows,
        "pairwise_ranks": ranks_rows,
    }
    print(json.dumps(out), flush=True)
    mesh.close()
    ctx.close()


def learned_leg(ctx, reps, log):
    """The learned preconditioner on box24_N7_lognormal_helmholtz (24^3
    elements, N = 7, log-normal k, h = 1): 128 training pairs from the FP64
    solver on 16 right-hand sides, 300 Adam steps, the correction's scale
    calibrated on a training right-hand side; then, on the held-out
    right-hand side of seed 5900, learned flexible CG and Jacobi PCG (both
    inside FP64 refinement) and FP64 Jacobi PCG, each to relative residuals
    1e-10 and 1e-8, the median of reps solves after a warm-up.  Returns the
    record and the solutions (for the oracle's errors)."""
    import numpy as np
    import torch

    from paper_2503_02134_amd import mxsem as mx
    from paper_2503_02134_amd import workloads as W
    from paper_2503_02134_amd.learned import (Network, calibrate_scale, make_pairs, rhs_batch,
                                              train)
    wl = W.WORKLOADS["box24_N7_lognormal_helmholtz"]
    xi, _ = mx.mxsem_gll(wl.N)
    bm = W.box_mesh(wl.ne, wl.N, xi)
    kf = W.lognormal_k(bm, wl.k_seed)
    mesh = mx.Mesh(ctx, bm.E, wl.N, bm.xyz, bm.glo, bm.bnd, kcoef=kf, helm_h=wl.helm_h)
    nloc = mesh.nloc
    log(f"learned leg: {wl.name} nloc={nloc}")
    t0 = time.perf_counter()
    train_rhs = rhs_batch(bm, mesh, range(5100, 5116))
    R, E = make_pairs(mesh, train_rhs, samples=8, mesh_np=bm, seed=11)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = Network(mesh, seed=3)
    t0 = time.perf_counter()
    losses = train(net, R, E, steps=300, batch=4, lr=2e-3, seed=1, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del R, E
    lam, cal = calibrate_scale(net, mesh, train_rhs[0], log=log)
    net.attach()
    seed = 5900
    b = rhs_batch(bm, mesh, [seed])[0]
    methods = (("learned", dict(mode=mx.MODE_MIXED_IR, pc=mx.PC_LEARNED, method=mx.METHOD_FCG)),
               ("jacobi_mixed_ir", dict(mode=mx.MODE_MIXED_IR)),
               ("fp64_jacobi", dict(mode=mx.MODE_FP64)))
    rec = {}
    xs = {}
    for tol in (wl.tol, 1e-8):
        for name, kw in methods:
            x = torch.zeros_like(b)
            mesh.solve(b, x, tol=tol, max_iter=50000, **kw)  # warm-up
            runs = []
            for _ in range(reps):
                x.zero_()
                _, st = mesh.solve(b, x, tol=tol, max_iter=50000, **kw)
                runs.append(st)
            st = sorted(runs, key=lambda r: r.ms)[len(runs) // 2]
            it = st.iterations + st.outer
            key = f"residual_{tol:.0e}"
            rec.setdefault(key, {})[name] = {
                "ms": round(st.ms, 3), "iterations": it, "rel_res": st.rel_res,
                "gdof_iter_s": round(nloc * it / (st.ms * 1e-3) / 1e9, 3),
                "fallback_steps": st.fallback_used, "median_of": reps}
            xs[f"{key}/{name}"] = x.cpu().numpy()
            log(f"  {key} {name}: {it} it, {st.ms:.1f} ms, res {st.rel_res:.2e}")
    for key in list(rec):
        r = rec[key]
        r["learned_vs_jacobi_time"] = round(r["jacobi_mixed_ir"]["ms"] / r["learned"]["ms"], 3)
        r["learned_vs_fp64_time"] = round(r["fp64_jacobi"]["ms"] / r["learned"]["ms"], 3)
    out = {"workload": wl.name, "E": bm.E, "N": wl.N, "nloc": nloc, "held_out_rhs_seed": seed,
           **rec,
           "training": {"pairs": 128, "rhs_seeds": "5100-5115", "adam_steps": 300,
                        "loss_first": losses[0], "loss_last20": float(np.mean(losses[-20:])),
                        "scale": lam,
                        "calibration_iterations": {str(k): v for k, v in cal.items()},
                        "pairs_s": round(t_data, 2), "train_s": round(t_train, 2)}}
    net.close()
    mesh.close()
    return out, {"rhs_seed": seed, "x": xs}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            return next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        return ""


def _oracle_problem(wl, rhs_seed=None):
    import oracle
    from paper_2503_02134_amd import workloads as W
    xo, _ = oracle.gll(wl.N)
    bm = W.box_mesh(wl.ne, wl.N, xo, seed=wl.deform_seed)
    kf = W.lognormal_k(bm, wl.k_seed) if wl.k_seed is not None else None
    if rhs_seed is None:
        f = W.manufactured(bm)[0] if wl.rhs == "manufactured" else W.random_smooth_rhs(bm, wl.rhs_seed)
    else:
        f = W.random_smooth_rhs(bm, rhs_seed)
    om = oracle.Mesh(bm.E, wl.N, bm.xyz, bm.glo, bm.bnd, kcoef=kf, helm_h=wl.helm_h)
    return om, om.rhs(f)


def _c_err(om, x, xs):
    import numpy as np
    c = om.c
    return float(np.sqrt(np.sum(c * (x - xs) ** 2) / np.sum(c * xs * xs)))


def oracle_leg(wl, sols):
    """The oracle on the host cores: its FP64 Jacobi-PCG solve of the
    workload from x = 0 to relative residual 1e-10 is timed (the CPU
    baseline), then continued from that solution to 1e-13, which gives the
    reference solution x*; every GPU solution in sols gets its relative
    c-norm error against x*."""
    import oracle
    t0 = time.perf_counter()
    om, b = _oracle_problem(wl)
    log(f"oracle: {wl.name} set up in {time.perf_counter() - t0:.1f}s; solving to 1e-10")
    t0 = time.perf_counter()
    x10, st10 = om.pcg(b, tol=1e-10, maxit=20000)
    el = time.perf_counter() - t0
    log(f"oracle: {st10.iterations} iterations to 1e-10 in {el:.1f}s; continuing to 1e-13")
    t1 = time.perf_counter()
    xs, st13 = om.pcg(b, tol=1e-13, maxit=20000, x0=x10)
    el13 = time.perf_counter() - t1
    log(f"oracle: x* after {st13.iterations} more iterations ({el13:.1f}s), "
        f"true residual {st13.rel_res_true:.2e}")
    # the solve ends with one true-residual operator application: counted
    # as an iteration's worth of work
    value = om.nloc * (st10.iterations + 1) / el / 1e9
    base = {"value": round(value, 5), "unit": "GDOF*iter/s", "cores": oracle.max_threads(),
            "cpu_model": _cpu_model(), "kind": "oracle",
            "sample": (f"the whole FP64 Jacobi-PCG solve of {wl.name} from x = 0 to relative "
                       f"residual 1e-10 (plain C oracle, OpenMP over elements): "
                       f"{st10.iterations} iterations, {el:.1f} s"),
            "iterations": st10.iterations, "time_to_solution_s": round(el, 2),
            "rel_res_true": st10.rel_res_true}
    errs = {"reference": (f"oracle FP64 Jacobi-PCG to relative residual 1e-13 "
                          f"({st10.iterations} + {st13.iterations} iterations, true residual "
                          f"{st13.rel_res_true:.1e})"),
            "norm": "relative c-weighted L2 (c = 1/multiplicity)",
            "cpu_solution_1e-10": _c_err(om, x10, xs)}
    for name, x in sols.items():
        errs[name] = _c_err(om, x, xs)
    log(f"errors vs oracle: {errs}")
    return base, errs


def batch_oracle_problems():
    """The batch problems whose solutions the oracle checks: the first one of
    each order on 8^3 elements (the oracle solves each in a few seconds)."""
    from paper_2503_02134_amd import workloads as W
    picked, seen = [], set()
    for p, (ne, N, _) in enumerate(W.batch_draws()):
        if ne == 8 and N not in seen:
            picked.append(p)
            seen.add(N)
    return tuple(picked)


def _oracle_timed(om, b):
    """The oracle's FP64 Jacobi-PCG of one problem from x = 0, timed to
    relative residual 1e-10, then continued from that solution to 1e-13
    (x*, untimed).  Returns x*, the 1e-10 solve's record and seconds, and the
    continuation's record."""
    t0 = time.perf_counter()
    x10, st10 = om.pcg(b, tol=1e-10, maxit=50000)
    el = time.perf_counter() - t0
    xs, st13 = om.pcg(b, tol=1e-13, maxit=50000, x0=x10)
    return xs, st10, el, st13


def _oracle_rate(nloc_its, seconds):
    # a solve ends with one true-residual operator application: counted as
    # an iteration's worth of work, as in oracle_leg
    return round(sum(n * (i + 1) for n, i in nloc_its) / sum(seconds) / 1e9, 5)


def batch_oracle_errors(sols):
    """The oracle on the batch problems in sols (problem -> GPU solution):
    each one's FP64 Jacobi-PCG timed to 1e-10 (a bounded sample of the batch
    workload for the CPU baseline) and continued to 1e-13; returns the
    relative c-norm errors of the GPU solutions against those x* and the
    sample's timing."""
    import oracle
    from paper_2503_02134_amd import workloads as W
    draws = W.batch_draws()
    errs = {"reference": "oracle FP64 Jacobi-PCG of each listed problem to relative residual 1e-13",
            "norm": "relative c-weighted L2 (c = 1/multiplicity)"}
    work, secs, per = [], [], {}
    for p, x in sols.items():
        ne, N, seed = draws[p]
        xo, _ = oracle.gll(N)
        bm = W.box_mesh(ne, N, xo)
        om = oracle.Mesh(bm.E, N, bm.xyz, bm.glo, bm.bnd)
        xs, st10, el, _ = _oracle_timed(om, om.rhs(W.random_smooth_rhs(bm, seed)))
        name = f"problem_{p}_ne{ne}_N{N}"
        errs[name] = _c_err(om, x, xs)
        work.append((om.nloc, st10.iterations))
        secs.append(el)
        per[name] = {"iterations": st10.iterations, "s": round(el, 3)}
    cpu = {"value": _oracle_rate(work, secs), "unit": "GDOF*iter/s", "cores": oracle.max_threads(),
           "kind": "oracle",
           "sample": (f"{len(per)} of the 64 problems, each the oracle's FP64 Jacobi-PCG from "
                      f"x = 0 to relative residual 1e-10, one after another"),
           "problems": per}
    log(f"batch errors vs oracle: {errs}; oracle sample {cpu}")
    return errs, cpu


def oracle_reference_errors(wl, rhs_seed, xs_gpu):
    """The oracle on one right-hand side: its FP64 Jacobi-PCG timed to 1e-10
    (the CPU baseline of this workload) and continued to 1e-13 for x*;
    returns the relative c-norm errors of the given GPU solutions against x*
    and the timing."""
    import oracle
    t0 = time.perf_counter()
    om, b = _oracle_problem(wl, rhs_seed)
    xs, st10, el, st13 = _oracle_timed(om, b)
    log(f"oracle: {wl.name} rhs {rhs_seed}: {st10.iterations} iterations to 1e-10 in {el:.1f}s, "
        f"x* after {st13.iterations} more ({time.perf_counter() - t0:.1f}s in all)")
    errs = {"reference": (f"oracle FP64 Jacobi-PCG of right-hand side {rhs_seed} to relative "
                          f"residual 1e-13 ({st10.iterations} + {st13.iterations} iterations)"),
            "norm": "relative c-weighted L2 (c = 1/multiplicity)"}
    for name, x in xs_gpu.items():
        errs[name] = _c_err(om, x, xs)
    cpu = {"value": _oracle_rate([(om.nloc, st10.iterations)], [el]), "unit": "GDOF*iter/s",
           "cores": oracle.max_threads(), "kind": "oracle",
           "sample": (f"the oracle's FP64 Jacobi-PCG of {wl.name}, right-hand side {rhs_seed}, "
                      f"from x = 0 to relative residual 1e-10: {st10.iterations} iterations, "
                      f"{el:.1f} s"),
           "iterations": st10.iterations, "time_to_solution_s": round(el, 2)}
    log(f"errors vs oracle: {errs}")
    return errs, cpu


if __name__ == "__main__":
    main()
