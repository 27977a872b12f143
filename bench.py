#!/usr/bin/env python
"""Benchmark: converged columns per second of per-column MALI on one MI355X.

Workload: the synthetic 3D-MHD-like cube (256 x 256 = 65,536 columns, 200-400
depth points each, seed 1), the six-level hydrogen-like atom (10 lines, 5
continua, 510 wavelengths), 5 angles, converged to a maximum relative
population change of 1e-4.  A step solves one batch of columns (default:
the whole cube, streamed through the resident slots) to convergence; K steps
cycle through the cube's batches.
Inputs are resident in HBM before the timed region.

Four forms run on the same batches: the plain FP64 path, the precision
form on the slot scheduler (FP32 formal solution and rate accumulation,
FP64 rate solve, Ng and convergence test) from LTE, the same from the
escape-probability start, and the same from the learned start (a network
trained beforehand on another cube, its inference inside the timed
region).  Every form stops by the change test (1e-4) and the fixed-point
bound (--tol-fp).  The timed steps run on a non-default stream with
profiling off, so the slot scheduler replays each iteration as a captured
graph.  `value` is the learned-start form's rate of converged columns,
times the fraction of the accuracy sample within 1e-3 of the oracle
converged to 1e-10 when that fraction is below 1.  The roofline object
describes the dominant kernel (the formal-solution sweep) from HIP-event
timings taken inside the library on the launch stream during one extra,
profiled step of the same form and batch.  The CPU baseline is the FP64
oracle on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "converged columns/s @1e-3 rel. accuracy: plain FP64 vs batched FP32+warm start"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}
HBM_PEAK_GBS = 8000.0
# HBM bytes per FP32 sweep stage of the learned-start form from rocprofv3
# FETCH_SIZE / WRITE_SIZE (calibrated on a 1 GiB copy), valid only for the kernel source they were
# taken on: the JSON line reports null once that source has changed.
SWEEP_TRAFFIC = {
    "source": "paper_1411_1079_amd/csrc/mali.hip",
    "sha256": "39bd161138b3ce9e151b9d2b80b0922f2f7afe12726526d4a7596ae6b08200c1",
    "read_bytes": 24.20e9,
    "written_bytes": 5.52e9,
    "summary": "profiles/k_sweep_fp32_learned_start_cube256_counters.md",
}


def sweep_traffic():
    import hashlib
    path = os.path.join(ROOT, SWEEP_TRAFFIC["source"])
    with open(path, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != SWEEP_TRAFFIC["sha256"]:
            return None
    return SWEEP_TRAFFIC["read_bytes"] + SWEEP_TRAFFIC["written_bytes"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_batches(rh, cols, dev_fields, batch):
    """DeviceColumns views of consecutive column ranges of the resident cube."""
    out = []
    n = cols.n_columns
    for c0 in range(0, n, batch):
        c1 = min(n, c0 + batch)
        g0, g1 = int(cols.offset[c0]), int(cols.offset[c1])
        off = (cols.offset[c0:c1 + 1] - g0).astype(np.int64)
        views = {k: v[g0:g1] for k, v in dev_fields.items()}
        out.append((c0, c1, rh.DeviceColumns(offset=off, **views)))
    return out


FORMS = {
    # plain FP64 MALI, fixed chunks of columns iterated together
    "fp64": dict(precision=0, scheduler=0),
    # precision form on the slot scheduler (retire converged columns, refill slots), LTE start
    "fp32": dict(precision=1, scheduler=1),
    # the same from the escape-probability start (the paper's third cold start)
    "fp32e": dict(precision=1, scheduler=1, start=3, esc_iter=3),
    # the same started from the network's prediction (columns that fail are redone from LTE)
    "fp32w": dict(precision=1, scheduler=1),
}
FORM_NAMES = {
    "fp64": "plain FP64 MALI, chunked, LTE start",
    "fp32": "slot scheduler, FP32 formal solution + FP64 rate solve, LTE start",
    "fp32e": "slot scheduler, FP32 formal solution + FP64 rate solve, escape-probability start (3 iterations)",
    "fp32w": "slot scheduler, FP32 formal solution + FP64 rate solve, learned start (MLP, BF16 MFMA)",
}
MLP_FLOPS_PER_SAMPLE = 2 * (36 * 256 + 2 * 256 * 256 + 256 * 6)


def train_network(rh, torch, atom, args):
    """Train the start-solution network on columns of another cube (three
    of every four columns, --train-columns), converged by the FP64 form to
    1e-6; not timed with the forms (reported separately)."""
    from paper_1411_1079_amd import synth, warmstart
    t0 = time.perf_counter()
    every = args.nx * args.nx
    pick = [c for c in range(every) if c % 4 != 3][: args.train_columns]
    cols = synth.cube_columns(args.train_seed, args.nx, args.nx).select(pick)
    t1 = time.perf_counter()
    dc = rh.DeviceColumns.from_host(cols)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # a fixed formal-solution shape (not the autotuner's choice), so that the
    # targets, and the trained network, are the same on every run
    res = rh.solve(atom, dc, precision=0, scheduler=1, n_mu=5, tol=1e-6, max_iter=300, profile=0,
                   sweep_mc=1, sweep_pack=1)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    net, rep = warmstart.train(atom, dc, res["pops"], steps=args.train_steps, batch=8192, lr=2e-3, seed=1)
    info = dict(cube_seed=args.train_seed, columns=cols.n_columns, points=rep.points,
                converged=int((res["status"] == 0).sum().item()), generate_s=t1 - t0, converge_s=t3 - t2,
                train_s=rep.seconds, steps=rep.steps, batch=rep.batch, loss_first=rep.loss_first,
                loss_last=rep.loss_last)
    del res, dc
    return net, info


def run_form(rh, torch, atom, batches, form, steps, warmup, ws, net=None, shrink=None, crs_f0=1.0, tol_fp=0.0):
    """Warm-up steps, then `steps` timed steps on a non-default stream with
    profiling off (the slot scheduler replays captured graphs), then one
    profiled step of the first timed batch for the per-kernel times."""
    from paper_1411_1079_amd import warmstart
    st = torch.cuda.Stream()
    opts = rh.default_options(n_mu=5, tol=1e-4, tol_fp=tol_fp, max_iter=200, profile=0, crs_f0=crs_f0,
                              **FORMS[form])
    if form == "fp32w":
        runs = [warmstart.WarmStartSolver(atom, dc, net, opts, workspace=ws,
                                          shrink=warmstart.SHRINK if shrink is None else shrink)
                for _, _, dc in batches]
        solvers = [r.solver for r in runs]
    else:
        runs = solvers = [rh.Solver(atom, dc, opts, want_spectrum=True, workspace=ws) for _, _, dc in batches]
    nb = len(solvers)

    def step(r, stats=None):
        nonlocal refined
        with torch.cuda.stream(st):
            if form == "fp32w":
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(st)
                r.predict(st)
                e1.record(st)
                r.solver.run(st)
                gl = rh.last_stats()["graph_launches"]
                refined += r.refine_failed(st)
                if stats is not None:
                    stats["predict_events"].append((e0, e1))
                    stats["samples"] += r.dc.total_depth
            else:
                r.run(st)
                gl = rh.last_stats()["graph_launches"]
        return gl

    refined = 0
    for i in range(warmup):
        step(runs[i % nb])
    torch.cuda.synchronize()
    refined = 0
    columns = converged = 0
    graph_launches = 0
    mlp = dict(predict_events=[], samples=0)
    t0 = time.perf_counter()
    for i in range(steps):
        r = runs[(warmup + i) % nb]
        graph_launches += step(r, mlp)
        columns += r.dc.n_columns
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    iters = []
    for i in range(steps):
        s = solvers[(warmup + i) % nb]
        converged += int((s.status == 0).sum().item())
        iters.append(s.n_iter.cpu().numpy())
    iters = np.concatenate(iters)
    hist = {f"p{q}": float(np.percentile(iters, q)) for q in (50, 90, 99, 100)}
    out = dict(seconds=t1 - t0, columns=columns, converged=converged, solvers=solvers,
               first_batch=(warmup % nb), iter_percentiles=hist, mean_iterations=float(iters.mean()),
               ran={(warmup + i) % nb for i in range(steps)}, graph_launches=graph_launches)
    if form == "fp32w":
        ms = sum(a.elapsed_time(b) for a, b in mlp["predict_events"])
        out["mlp"] = dict(predict_ms=ms, samples=mlp["samples"], refined_columns=refined,
                          forward_tflops=MLP_FLOPS_PER_SAMPLE * mlp["samples"] / (ms / 1e3) / 1e12)
    # one profiled step (HIP events around the library's launches, eager
    # launches with a host synchronisation per iteration): kernel times
    b = out["first_batch"]
    opts.profile = 1
    if form == "fp32w":
        prof = warmstart.WarmStartSolver(atom, batches[b][2], net, opts, workspace=ws,
                                         shrink=warmstart.SHRINK if shrink is None else shrink)
    else:
        prof = rh.Solver(atom, batches[b][2], opts, want_spectrum=True, workspace=ws)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    with torch.cuda.stream(st):
        prof.run(st)
        pst = rh.last_stats()
    torch.cuda.synchronize()
    out["profiled_seconds"] = time.perf_counter() - tp
    out["stats"] = pst
    return out


def host_cpu():
    """CPU model and logical CPU count of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(atom_path, cols, batches, gpu_first, budget_s, max_cols, threads, tol_fp, seed=1):
    """The FP64 oracle as it stands, one column per task on a thread pool of
    `threads` host threads, on a seeded random sample of the columns of the
    timed batches (so the sample has the cube's mix of fast and slowly
    converging columns), until the time budget or max_cols is reached."""
    import concurrent.futures

    from oracle import oracle as O

    a = O.Atom(atom_path)
    c0, c1 = batches[gpu_first][0], batches[-1][1]
    order = [int(c) for c in c0 + np.random.default_rng(seed).permutation(c1 - c0)[:max_cols]]
    results = []
    t0 = time.perf_counter()
    # a pool: one column per task, a new task as soon as a thread is free,
    # none started after the budget; the columns in flight then finish
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        pending = {}
        nxt = 0

        def submit():
            nonlocal nxt
            c = order[nxt]
            nxt += 1
            pending[ex.submit(O.solve_column, a, cols.column(c), n_mu=5, tol=1e-4, tol_fp=tol_fp,
                              max_iter=200)] = c

        while nxt < len(order) and len(pending) < threads:
            submit()
        while pending:
            done, _ = concurrent.futures.wait(list(pending), return_when=concurrent.futures.FIRST_COMPLETED)
            for f in done:
                results.append((pending.pop(f), f.result()))
                if nxt < len(order) and time.perf_counter() - t0 < budget_s:
                    submit()
    dt = time.perf_counter() - t0
    conv = sum(1 for _, r in results if r["status"] == 0)
    iters = np.array([r["n_iter"] for _, r in results])
    model, ncpu = host_cpu()
    return dict(value=conv / dt, unit="columns/s", cores=threads, kind="oracle",
                cpu_model=model, host_logical_cpus=ncpu,
                sample=f"{len(results)} columns drawn at random (seed {seed}) from columns {c0}..{c1 - 1} of the "
                       f"cube, same stopping rule, mean {iters.mean():.2f} iterations, {dt:.1f} s wall on "
                       f"{threads} threads of {model}"), results


def converged_oracle(atom_path, cols, n, threads, seed=0):
    """The oracle converged to 1e-10 on a seeded random sample of n columns
    of the whole cube (not timed): the reference of the 1e-3 accuracy
    criterion.  The sample includes slowly converging columns in their
    proportion."""
    import concurrent.futures

    from oracle import oracle as O
    a = O.Atom(atom_path)
    picks = sorted(np.random.default_rng(seed).choice(cols.n_columns, size=min(n, cols.n_columns), replace=False))
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(O.solve_column, a, cols.column(int(c)), n_mu=5, tol=1e-10, max_iter=1000) for c in picks]
        return [(int(c), f.result()) for c, f in zip(picks, futs)]


def accuracy(results, form, batches, cols, lockstep=False):
    """Max relative difference of populations and emergent intensity between
    a GPU form and oracle results [(global column, result)], and the
    fraction of those columns within 1e-3 in both.  lockstep: also count
    the columns with the oracle's iteration count and status, and the
    largest difference over those (the FP64 form against the oracle under
    the same stopping rule)."""
    host = {}
    ep = es = 0.0
    within = 0
    n = 0
    same_iter = 0
    worst_same = 0.0
    differ = []
    same_diffs = []
    for c, r in results:
        b = next(i for i, (c0, c1, _) in enumerate(batches) if c0 <= c < c1)
        if b not in form["ran"]:
            continue        # a batch the timed steps did not solve
        n += 1
        if b not in host:
            s = form["solvers"][b]
            host[b] = (s.pops.cpu().numpy(), s.spectrum.cpu().numpy(), s.dc.offset, s.n_iter.cpu().numpy(),
                       s.status.cpu().numpy())
        pops, spec, off, nit, stat = host[b]
        i = c - batches[b][0]
        lo, hi = int(off[i]), int(off[i + 1])
        p = float(np.max(np.abs(pops[lo:hi] / r["pops"] - 1.0)))
        e = float(np.max(np.abs(spec[i] / r["spectrum"] - 1.0)))
        ep, es = max(ep, p), max(es, e)
        within += int(p <= 1e-3 and e <= 1e-3)
        if lockstep:
            if nit[i] == r["n_iter"] and stat[i] == r["status"]:
                same_iter += 1
                worst_same = max(worst_same, p, e)
                same_diffs.append((max(p, e), int(c)))
            else:
                differ.append(dict(column=int(c), gpu_n_iter=int(nit[i]), oracle_n_iter=int(r["n_iter"])))
    out = {"pops": ep, "spectrum": es, "columns": n, "fraction_within_1e-3": within / max(n, 1)}
    if lockstep:
        same_diffs.sort(reverse=True)
        out.update({"same_n_iter_and_status": same_iter, "max_rel_diff_where_same_n_iter": worst_same,
                    "largest_diffs_where_same_n_iter": [dict(column=c, rel_diff=d) for d, c in same_diffs[:5]],
                    "columns_with_other_n_iter": differ[:20]})
    return out


def grid_measure(rh, torch, atom, cols, fields, tol_fp, n_out=300, reps=5):
    """Grid optimisation of the whole cube (every column onto n_out points)
    in one call, timed with HIP events on the launch stream; algorithmic
    bytes = six FP64 values read per input point and written per output
    point, plus the status per column."""
    dc = rh.DeviceColumns(offset=np.ascontiguousarray(cols.offset, dtype=np.int64), **fields)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        rh.optimize_grid(atom, dc, n_out, stream=st)      # warm-up
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(st)
            new, status = rh.optimize_grid(atom, dc, n_out, stream=st)
            b.record(st)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)[reps // 2]
    nbytes = 48.0 * (cols.offset[-1] + cols.n_columns * n_out) + 4.0 * cols.n_columns
    out = dict(columns=cols.n_columns, input_points=int(cols.offset[-1]), output_points_per_column=n_out,
               bad_input_columns=int((status != 0).sum().item()), median_ms=ms,
               algorithmic_bytes=nbytes, achieved_GBps=nbytes / (ms / 1e3) / 1e9,
               hbm_frac=nbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
               timing_note=("median of 5 calls between HIP events on the launch stream; each call also uploads "
                            "the 1 MB of depth offsets and waits for it"))
    # the iteration counts on the new grids (Fig. 1 of the paper compares
    # the original and the optimised grid): the FP32 form from LTE on the
    # re-gridded cube and on the original one
    o = rh.default_options(n_mu=5, tol=1e-4, tol_fp=tol_fp, max_iter=200, **FORMS["fp32"])
    for name, d in (("original", dc), ("optimised", new)):
        r = rh.Solver(atom, d, o, want_spectrum=False, want_history=False)
        r.run()
        torch.cuda.synchronize()
        it = r.n_iter.cpu().numpy()
        stt = r.status.cpu().numpy()
        out[f"iterations_{name}_grid"] = dict(mean=float(it.mean()), p99=float(np.percentile(it, 99)),
                                              max=int(it.max()), converged=int((stt == 0).sum()))
    return out


def cube_field(cols, seed):
    """Magnetic field of the full-stack workload: per column a strength
    uniform in 0-2 kG and an isotropic direction (cosine of the inclination
    uniform in [-1, 1], azimuth uniform in [0, 2 pi)), constant along the
    column."""
    rng = np.random.default_rng(seed)
    n = cols.n_columns
    B = rng.uniform(0.0, 0.2, n)
    inc = np.arccos(rng.uniform(-1.0, 1.0, n))
    az = rng.uniform(0.0, 2.0 * np.pi, n)
    nd = np.diff(cols.offset)
    return tuple(np.repeat(x, nd) for x in (B, inc, az))


def prd_workload(args):
    """The full-stack workload: the Ca II-like atom (two PRD resonance lines
    with Zeeman patterns, three CRD lines, four continua, 985 wavelengths)
    on a synthetic cube of args.prd_nx^2 columns with a magnetic field
    (cube_field), 5 angles, solved to the change test 1e-4 plus the
    fixed-point bound, then the emergent Stokes vector; in FP64 (plain
    path, chunked) and FP32 (slot scheduler).  One JSON line with converged
    columns/s, iterations, statuses, the per-kernel times of a profiled solve
    of the same columns, and the time of the polarised formal solution
    alone (final stage from the converged populations with and without the
    Stokes output)."""
    import torch

    from paper_1411_1079_amd import rh15d as rh
    from paper_1411_1079_amd import synth
    tmp = tempfile.mkdtemp()
    atoms = synth.write_atoms(tmp)
    cols = synth.cube_columns(args.seed, args.prd_nx, args.prd_nx)
    dc = rh.DeviceColumns.from_host(cols, field=cube_field(cols, args.seed + 100))
    atom = rh.Atom(atoms["ca2"])
    res = {}
    for name, kw in (("fp64", dict(precision=0, scheduler=0)), ("fp32", dict(precision=1, scheduler=1))):
        o = rh.default_options(n_mu=5, tol=1e-4, tol_fp=args.tol_fp, max_iter=args.prd_max_iter, prd=1, **kw)
        s = rh.Solver(atom, dc, o, want_stokes=True)
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            s.run(st)                      # warm-up (builds the tables)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(st):
            s.run(st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        status = s.status.cpu().numpy()
        it = s.n_iter.cpu().numpy()
        o.profile = 1
        p = rh.Solver(atom, dc, o, workspace=s.workspace, want_stokes=True)
        p.run()
        torch.cuda.synchronize()
        stats = rh.last_stats()
        res[name] = dict(columns_per_s=int((status == 0).sum()) / dt, seconds=dt, columns=cols.n_columns,
                         converged=int((status == 0).sum()), status_counts=np.bincount(status, minlength=5).tolist(),
                         mean_iterations=float(it.mean()), max_iterations=int(it.max()),
                         profiled_kernel_ms={k: stats[k] for k in ("prep_ms", "sweep_ms", "se_ms", "converge_ms",
                                                                   "final_ms", "total_ms")},
                         sweep_tflops=stats["sweep_flops"] / (stats["sweep_ms"] / 1e3) / 1e12 if stats["sweep_ms"] else 0.0)
        pol = torch.sqrt((s.stokes[:, :, 1:] ** 2).sum(dim=2)) / s.stokes[:, :, 0]
        res[name]["max_polarisation_degree"] = float(torch.nan_to_num(pol, nan=0.0).max().item())
        if name == "fp64":
            # the final stage alone, from the converged populations: with and
            # without the Stokes output
            dcp = rh.DeviceColumns(offset=dc.offset, z=dc.z, T=dc.T, n_e=dc.n_e, n_H=dc.n_H, v_z=dc.v_z,
                                   v_turb=dc.v_turb, init_pops=s.pops.clone(), B=dc.B, B_incl=dc.B_incl,
                                   B_azim=dc.B_azim)
            fin = {}
            for want in (False, True):
                o0 = rh.default_options(n_mu=5, max_iter=0, start=rh.START_PROVIDED, prd=1, profile=1, **kw)
                q = rh.Solver(atom, dcp, o0, want_stokes=want)
                q.run()
                q.run()
                torch.cuda.synchronize()
                fin[want] = rh.last_stats()["final_ms"]
            steps = float(cols.offset[-1]) * atom.n_lambda
            res[name]["stokes_ms"] = fin[True] - fin[False]
            res[name]["stokes_point_wavelengths_per_s"] = steps / ((fin[True] - fin[False]) / 1e3)
        log(f"prd {name}: {res[name]}")
    out = dict(metric="converged columns/s, angle-averaged PRD + Zeeman Stokes (Ca II-like atom)", unit="columns/s",
               value=res["fp64"]["columns_per_s"], n_gpus=1, higher_is_better=True, data="synthetic",
               dtype="f64",
               config={"workload": (f"synthetic 3D cube {args.prd_nx}x{args.prd_nx} columns (seed {args.seed}), "
                                    f"200-400 depth points, Ca II-like 5-level atom (2 PRD lines of 61 wavelengths "
                                    f"with Zeeman patterns, 3 CRD lines, 4 continua, 985 wavelengths), 5 angles, "
                                    f"tol 1e-4, fixed-point bound {args.tol_fp:g}, at most {args.prd_max_iter} "
                                    f"iterations; field 0-2 kG uniform, isotropic direction, per column; emergent "
                                    f"Stokes vector"),
                       "parallelism": "1 GPU"},
               forms=res,
               note=("converge_ms includes the rho update kernels (k_prd_rho, k_prd_psi), which run after the "
                     "convergence test; prep_ms includes the R_II tables (k_prd_tables); final_ms includes the "
                     "emergent spectrum and the Stokes formal solution (k_stokes, FP64 in both forms)"))
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--forms", default="fp64,fp32,fp32e,fp32w")
    ap.add_argument("--tol-fp", type=float, default=1e-4,
                    help="fixed-point bound of the stopping rule (every form and the oracle use it)")
    ap.add_argument("--train-seed", type=int, default=7)
    ap.add_argument("--train-steps", type=int, default=96000)
    ap.add_argument("--train-columns", type=int, default=49152,
                    help="training columns: the first of the seed cube's columns whose index is not 3 mod 4 "
                         "(49,152 = three of every four columns of the 256 x 256 cube)")
    ap.add_argument("--crs", type=float, default=1.0,
                    help="collisional-radiative switching: initial collision factor (1 = off)")
    ap.add_argument("--shrink", type=float, default=0.002,
                    help="shrinkage of the predicted |ln b| toward LTE, about the held-out error of the network "
                         "trained for --train-steps")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="oracle threads: the host CPU share allotted to one GPU (16 on the MI355X boxes)")
    ap.add_argument("--cpu-max-columns", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--accuracy-columns", type=int, default=128,
                    help="seeded random columns of the cube also solved by the oracle to 1e-10")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-grid", action="store_true",
                    help="skip the grid-optimisation measurement (profiler runs of one form)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES of device memory once (a reference kernel of known traffic for "
                         "hardware byte counters) and exit")
    ap.add_argument("--save-network", default="", metavar="NPZ",
                    help="write the trained start-solution network (parameters and input normalisation) here")
    ap.add_argument("--load-network", default="", metavar="NPZ",
                    help="use a network written by --save-network instead of training one (for profiler runs, "
                         "where the training's many small launches would dominate)")
    ap.add_argument("--prd", action="store_true",
                    help="measure the partial-frequency-redistribution workload instead (Ca II-like atom)")
    ap.add_argument("--prd-nx", type=int, default=64)
    ap.add_argument("--prd-max-iter", type=int, default=400)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the columns are independent, so several GPUs would each solve "
              "their own share of them with no exchange; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4}), flush=True)
        return

    if args.prd:
        prd_workload(args)
        return

    import torch

    from paper_1411_1079_amd import rh15d as rh
    from paper_1411_1079_amd import synth

    tmp = tempfile.mkdtemp()
    atom_path = synth.write_atoms(tmp)["h6"]
    t = time.perf_counter()
    cols = synth.cube_columns(args.seed, args.nx, args.nx)
    log(f"cube {args.nx}x{args.nx}: {cols.n_columns} columns, {int(cols.offset[-1])} points "
        f"({time.perf_counter() - t:.1f} s)")
    dev = torch.device("cuda:0")
    fields = {k: torch.as_tensor(getattr(cols, k)).to(dev) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
    batches = make_batches(rh, cols, fields, args.batch)
    atom = rh.Atom(atom_path)
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]

    tune = {}
    if not args.no_autotune:
        sample = cols.select(list(range(0, cols.n_columns, 8)))
        dcs = rh.DeviceColumns.from_host(sample)
        for f in forms:
            key = "fp64" if FORMS[f]["precision"] == 0 else "fp32"
            if key in tune:
                continue
            t = time.perf_counter()
            tune[key] = rh.autotune(atom, dcs, n_mu=5, tol=1e-4, max_iter=200, **FORMS[f])
            tune[key]["seconds"] = time.perf_counter() - t
            tune[key]["sample_columns"] = sample.n_columns
            log(f"autotune {key}: {tune[key]}")
        del dcs
    # sized after the autotuner: the tuned formal-solution shape sets the
    # number of rate keys and so the workspace
    ws_bytes = 0
    for f in forms:
        o = rh.default_options(n_mu=5, tol=1e-4, max_iter=200, **FORMS[f])
        ws_bytes = max(ws_bytes, max(rh.workspace_size(atom, dc, o) for _, _, dc in batches))
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    log(f"workspace {ws_bytes / 2**30:.2f} GiB, {len(batches)} batches of <= {args.batch} columns")
    net = train_info = None
    if "fp32w" in forms and args.load_network:
        z = np.load(args.load_network)
        net = rh.MLP(int(z["n_hidden"]), int(z["n_layers"]), atom.n_levels, 0)
        net.set_params(z["params"])
        net.set_normalization(z["mean"], z["std"])
        train_info = dict(loaded=args.load_network)
        log(f"network loaded from {args.load_network}")
    elif "fp32w" in forms:
        log(f"train the start-solution network on cube seed {args.train_seed}")
        net, train_info = train_network(rh, torch, atom, args)
        log(f"network: {train_info}")
        if args.save_network:
            mean, std = net.get_normalization()
            np.savez(args.save_network, params=net.get_params(), mean=mean, std=std, n_hidden=256, n_layers=3)
    res = {}
    for f in forms:
        log(f"form {f}: warmup {args.warmup}, steps {args.steps}")
        r = run_form(rh, torch, atom, batches, f, args.steps, args.warmup, ws, net=net, shrink=args.shrink,
                     crs_f0=args.crs, tol_fp=args.tol_fp)
        st = r["stats"]
        sweep_s = st["sweep_ms"] / 1e3
        res[f] = r
        log(f"form {f}: {r['converged']}/{r['columns']} converged in {r['seconds']:.3f} s "
            f"-> {r['converged'] / r['seconds']:.1f} columns/s (graph launches {r['graph_launches']}); profiled "
            f"step {r['profiled_seconds']:.3f} s, sweep {st['sweep_ms']:.1f} ms over {st['sweep_launches']} "
            f"launches, {st['sweep_flops'] / sweep_s / 1e12:.2f} TFLOP/s, mean iterations "
            f"{r['mean_iterations']:.2f} {r['iter_percentiles']}")

    headline = next(f for f in ("fp32w", "fp32", "fp32e", "fp64") if f in res)
    h = res[headline]
    hst = h["stats"]
    sweep_s = hst["sweep_ms"] / 1e3
    achieved = hst["sweep_flops"] / sweep_s / 1e12 if sweep_s > 0 else 0.0
    peak = PEAK_TFLOPS["fp64" if headline == "fp64" else "fp32"]
    rate = h["converged"] / h["seconds"]
    out = {
        "metric": METRIC,
        "value": rate,
        "unit": "columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * h["seconds"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if headline == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": (f"synthetic 3D cube {args.nx}x{args.nx} columns (seed {args.seed}), 200-400 depth "
                         f"points, H-like 6-level atom (10 lines, 5 continua, 510 wavelengths), 5 angles, "
                         f"stopped at max relative change < 1e-4 and fixed-point bound < {args.tol_fp:g}, "
                         f"batches of {args.batch} columns"),
            "form": FORM_NAMES[headline] + (f", collisional-radiative switching from {args.crs:g}"
                                             if args.crs > 1.0 else ""),
            "global_batch": args.batch,
            "parallelism": "1 GPU",
        },
        "timing": ("host wall clock between device synchronisations around the timed steps, on a non-default "
                   "stream with profiling off (slot-scheduler iterations replayed as captured graphs: "
                   f"{h['graph_launches']} graph launches in the headline's timed steps)"),
        "roofline": {
            "bound": "alu",
            "kernel": f"k_sweep ({'FP64' if headline == 'fp64' else 'FP32'} formal solution and rate accumulation)",
            "achieved": achieved,
            "peak": peak,
            "peak_note": ("published vector peak of the precision; without packed FP32 instructions (kept out of "
                          "the device code) FP32 vector code can reach 78.6 TFLOP/s"),
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": sweep_traffic() if headline == "fp32w" else None,
            "traffic_note": ("HBM bytes per sweep stage, rocprofv3 FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (factors "
                             "from a 1 GiB copy); null when the kernel source differs from the one measured"),
            "timing_note": ("HIP events recorded by the library on the launch stream around each iteration's "
                            "sweep stage, in one profiled step of the headline form on the first timed batch"),
            "launches": hst["sweep_launches"],
            "avg_launch_ms": hst["sweep_ms"] / max(hst["sweep_launches"], 1),
            "algorithmic_flops_per_launch": hst["sweep_flops"] / max(hst["sweep_launches"], 1),
            "algorithmic_GBps": hst["sweep_bytes"] / sweep_s / 1e9 if sweep_s > 0 else 0.0,
        },
        "forms": {},
    }
    for f, r in res.items():
        st = r["stats"]
        out["forms"][f] = {
            "form": FORM_NAMES[f],
            "columns_per_s": r["converged"] / r["seconds"],
            "converged": r["converged"], "columns": r["columns"], "seconds": r["seconds"],
            "graph_launches": r["graph_launches"],
            "mean_iterations": r["mean_iterations"],
            "iteration_percentiles": r["iter_percentiles"],
            "profiled_step_kernel_ms": {k: st[k] for k in ("prep_ms", "sweep_ms", "se_ms", "converge_ms",
                                                            "final_ms")},
            "profiled_step_seconds": r["profiled_seconds"],
            "sweep_tflops": st["sweep_flops"] / (st["sweep_ms"] / 1e3) / 1e12 if st["sweep_ms"] > 0 else 0.0,
        }
        if "mlp" in r:
            out["forms"][f]["mlp"] = r["mlp"]
    if train_info is not None:
        out["network_training"] = train_info
    if not args.no_grid:
        out["grid_optimisation"] = grid_measure(rh, torch, atom, cols, fields, args.tol_fp)
        log(f"grid optimisation: {out['grid_optimisation']}")
    if tune:
        out["autotune"] = tune
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        base, results = cpu_baseline(atom_path, cols, batches, h["first_batch"], args.cpu_budget,
                                     args.cpu_max_columns, args.cpu_threads, args.tol_fp)
        out["cpu_baseline"] = base
        out["accuracy_vs_oracle_same_stopping_rule"] = {f: accuracy(results, r, batches, cols, lockstep=(f == "fp64"))
                                                        for f, r in res.items()}
        log(f"cpu baseline {base['value']:.2f} columns/s on {base['cores']} threads; accuracy "
            f"{out['accuracy_vs_oracle_same_stopping_rule']}")
        if args.accuracy_columns > 0:
            t = time.perf_counter()
            conv = converged_oracle(atom_path, cols, args.accuracy_columns, base["cores"])
            out["accuracy_vs_converged_oracle"] = {f: accuracy(conv, r, batches, cols) for f, r in res.items()}
            log(f"accuracy against the oracle converged to 1e-10 ({len(conv)} columns, "
                f"{time.perf_counter() - t:.1f} s): {out['accuracy_vs_converged_oracle']}")
            frac = out["accuracy_vs_converged_oracle"][headline]["fraction_within_1e-3"]
            if frac < 1.0:
                out["value"] = rate * frac
                out["value_note"] = (f"converged columns/s {rate:.1f} times the fraction {frac:.4f} of the accuracy "
                                     "sample within 1e-3 of the converged oracle")
            else:
                out["value_note"] = "every column of the accuracy sample is within 1e-3 of the converged oracle"
    if "fp64" in res:
        fp64_rate = res["fp64"]["converged"] / res["fp64"]["seconds"]
        if "accuracy_vs_converged_oracle" in out:
            fp64_rate *= min(1.0, out["accuracy_vs_converged_oracle"]["fp64"]["fraction_within_1e-3"])
        out["speedup_vs_plain_fp64"] = out["value"] / fp64_rate
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
