"""bench.py's host-side contract, no GPU: more than one GPU is refused with a
message, and the energy counter reports why it is unavailable instead of
failing when no GPU counter can be read."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_energy_counter_unavailable_without_gpu():
    sys.path.insert(0, ROOT)
    import bench
    import torch
    if torch.cuda.is_available():
        return  # the GPU tests exercise the counter through the benchmark itself
    read, why = bench.energy_counter()
    assert read is None and isinstance(why, str) and why


def test_oracle_leg_on_a_small_workload():
    """The oracle leg of the default run on the 4^3, N = 7 workload: the
    timed solve to 1e-10, its continuation to the 1e-13 reference x*, and
    the error of a given solution against x* (its own 1e-10 solution is
    close to x*, a perturbed copy is not)."""
    sys.path.insert(0, ROOT)
    import numpy as np

    import bench
    from paper_2503_02134_amd import workloads as W
    wl = W.WORKLOADS["box4_N7"]
    om, b = bench._oracle_problem(wl)
    x10, _ = om.pcg(b, tol=1e-10, maxit=2000)
    base, errs = bench.oracle_leg(wl, {"same": x10, "perturbed": x10 * (1 + 1e-6)})
    assert base["kind"] == "oracle" and base["iterations"] > 0 and "1e-10" in base["sample"]
    assert base["value"] > 0 and base["cores"] >= 1
    assert errs["cpu_solution_1e-10"] < 1e-8 and errs["same"] == errs["cpu_solution_1e-10"]
    assert abs(errs["perturbed"] - 1e-6) < 1e-7
    assert "1e-13" in errs["reference"]


def test_batch_oracle_errors():
    """The batch leg's oracle check: one problem of each order on 8^3
    elements, each solution's error against the oracle's 1e-13 solution of
    that problem (the oracle's own 1e-10 solution is close, a perturbed one
    is off by the perturbation), and the oracle's timed 1e-10 solves of them
    as the batch's CPU sample."""
    sys.path.insert(0, ROOT)
    import oracle

    import bench
    from paper_2503_02134_amd import workloads as W
    picked = bench.batch_oracle_problems()
    draws = W.batch_draws()
    assert sorted(draws[p][1] for p in picked) == [5, 7, 9]
    assert all(draws[p][0] == 8 for p in picked)
    p = picked[1]
    ne, N, seed = draws[p]
    xo, _ = oracle.gll(N)
    bm = W.box_mesh(ne, N, xo)
    om = oracle.Mesh(bm.E, N, bm.xyz, bm.glo, bm.bnd)
    x10, st = om.pcg(om.rhs(W.random_smooth_rhs(bm, seed)), tol=1e-10, maxit=5000)
    errs, cpu = bench.batch_oracle_errors({p: x10 * (1 + 1e-6)})
    assert abs(errs[f"problem_{p}_ne{ne}_N{N}"] - 1e-6) < 1e-7
    one = cpu["problems"][f"problem_{p}_ne{ne}_N{N}"]
    assert abs(one["iterations"] - st.iterations) <= 2 and one["s"] > 0
    assert cpu["kind"] == "oracle" and cpu["value"] > 0 and cpu["cores"] >= 1


def test_learned_oracle_reference_and_timing():
    """The learned leg's oracle check on a small log-normal Helmholtz problem
    (4^3 elements, N = 7): the timed 1e-10 solve is the CPU sample, x* its
    continuation to 1e-13; a perturbed copy of the oracle's own solution is
    off by the perturbation."""
    sys.path.insert(0, ROOT)
    import dataclasses

    import bench
    from paper_2503_02134_amd import workloads as W
    wl = dataclasses.replace(W.WORKLOADS["box24_N7_lognormal_helmholtz"], name="box4_lognormal",
                             ne=4)
    om, b = bench._oracle_problem(wl, 5900)
    x10, st = om.pcg(b, tol=1e-10, maxit=5000)
    errs, cpu = bench.oracle_reference_errors(wl, 5900, {"perturbed": x10 * (1 + 1e-6)})
    assert abs(errs["perturbed"] - 1e-6) < 1e-7
    assert cpu["iterations"] == st.iterations and cpu["value"] > 0
    assert "1e-10" in cpu["sample"] and "1e-13" in errs["reference"]
