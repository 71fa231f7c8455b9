"""Benchmark: converged (RHS x shift) solves per second on one MI355X.

One step is one full solve of the workload (every RHS, every shift, to
relative residual 1e-6) by the persistent HIP solver, with H, S, the cluster
maps and all working memory already resident in HBM.  The default form
computes the shifted COCG iterates on the real S-Lanczos basis; the
seed-switching COCG form is timed in the same run and reported beside it.  A pair counts as
converged only if its FP64 residual ||b - (z_k S - H) x|| / ||b|| is
<= 1e-6: the true residual audited on the device after the solve in the
full-x form, the FP64 recursive estimate in the projected form.

Prints one JSON line (see the repository's benchmark contract) including a
roofline object for the solver kernel and a CPU baseline of the oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "converged (RHS×shift) solves/s at rel. res 1e-6 (FP64, batched persistent launch)"
WORKLOADS = {
    "cfg1": dict(cfg=1, desc="generalized shifted COCG, simple-cubic 16^3, 4x4 blocks (M=16384), "
                             "S = I + N(0,0.03) blocks, 128 shifts E in [-8,8] + 0.02i, 256 RHS"),
    "cfg0": dict(cfg=0, desc="shifted COCG S=I, simple-cubic 4^3, 4x4 blocks (M=256), 32 shifts + 0.05i, 8 RHS"),
    "cfg2": dict(cfg=2, desc="order-N clusters r~U[2,4]a on fcc 32^3, 9x9 blocks (M=1179648), "
                             "256 shifts + 0.01i, 4096 RHS"),
    "cfg2r": dict(cfg=2, radius=(1.0, 2.0),
                  desc="configuration 2 with cluster radii r~U[1,2]a (19-135 atoms, M_j 171-1215): fcc 32^3, "
                       "9x9 blocks (M=1179648), 256 shifts + 0.01i, 4096 RHS"),
    "cfg4r": dict(cfg=4, radius=(1.0, 2.0),
                  desc="configuration 4 with cluster radii r~U[1,2]a: 16384 fresh RHS on configuration 2's "
                       "matrices, 256 shifts + 0.01i"),
}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
METHODS = {"cocg": 0, "qmr": 1, "cocg-lanczos": 2}
_FORM_NAMES = {"qmr": "shifted QMR, real Lanczos basis", "lanczos": "COCG iterates on the real Lanczos basis"}


def algorithmic_bytes_qmr(stats, nout, bd, has_S, w_share, gal=False):
    """Algorithmic bytes of one launch of the solvers on the real Lanczos
    basis (8 bytes per vector element).  Per RHS and iteration:
      shifts  80 K_a n + 8 n  QMR: read d_{n-1}, d_{n-2}, x; write d_n, x on n = |I_j| rows; v on them
              64 K_a n + 8 n  COCG iterates: read p, x; write p, x
      Lanczos nb_H b^2 8 / w_share + 96 M_j   (H v; t = u - alpha w - beta w_prev; q^T t; the rescale)
      inner   k_in (nb_S b^2 8 / w_share + 48 M_j)"""
    outer, sum_upd, inner = stats[:, 0].astype(float), stats[:, 1].astype(float), stats[:, 2].astype(float)
    M, nblk = stats[:, 4].astype(float), stats[:, 5].astype(float)
    n = np.asarray(nout, dtype=float)
    blk = nblk * bd * bd * 8
    shifts = sum_upd * n * (64 if gal else 80) + outer * n * 8
    lanczos = outer * (blk / w_share + 96 * M)
    a5 = inner * (blk / w_share + 48 * M) if has_S else 0.0
    return float(np.sum(shifts + lanczos + a5))


def algorithmic_bytes(stats, nout, K, bd, has_S, prec, projected, w_share, audit):
    """Algorithmic bytes of one launch, from the per-unit figures of the
    design notes (FP64; FP32 halves vectors, blocks shrink to 4 or 2 bytes).
    Per RHS and outer iteration:
      sweep  64 K_a n + 16 n        n = M_j (full x) or |I_j| (projected rows)
      A4     (nb_H + nb_S) b^2 8 / w_share + 32 M_j
      A5     k_in ((nb_S b^2 8) / w_share + 96 M_j)
    with w_share the number of RHS sharing the blocks at once (all resident
    RHS for a global system, 1 for order-N clusters); the audit applies each
    shift's operator once."""
    vb = 16 if prec == 0 else 8
    bb = {0: 8, 1: 4, 2: 2}[prec]
    outer, sum_upd, inner = stats[:, 0].astype(float), stats[:, 1].astype(float), stats[:, 2].astype(float)
    M, nblk = stats[:, 4].astype(float), stats[:, 5].astype(float)
    n = np.asarray(nout, dtype=float) if projected else M
    blk = nblk * bd * bd * bb
    nmat = 2 if has_S else 1
    sweep = sum_upd * n * 4 * vb + outer * n * vb
    a4 = outer * (blk * nmat / w_share + 2 * vb * M)
    a5 = inner * (blk / w_share + 6 * vb * M) if has_S else 0.0
    aud = K * (nblk * bd * bd * 8 * nmat / w_share + 32 * M) if (audit and not projected) else 0.0
    return float(np.sum(sweep + a4 + a5 + aud))


def cpu_baseline(prob, gpu_stats, n_rhs_sample, iters_sample, workers, projected):
    """Time the oracle (as it stands) on host cores: `workers` processes, each
    running `iters_sample` outer iterations of one RHS of the same workload
    with the same form of the method (projected rows, full x, or "qmr"); the measured
    time per iteration times the mean outer iteration count the solve needs
    (from the GPU run) gives the time per RHS, hence solves/s."""
    import multiprocessing as mp
    idx = list(range(min(n_rhs_sample, prob.nrhs)))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        per = pool.map(_cpu_worker, [(prob, j, iters_sample, projected) for j in idx])
    wall = time.perf_counter() - t0
    t_iter = float(np.mean(per))                 # seconds per outer iteration, one process
    mean_outer = float(np.mean(gpu_stats[:, 0]))
    t_rhs = t_iter * mean_outer
    rate = prob.nshift * min(workers, len(idx)) / t_rhs
    return dict(value=rate, unit="solves/s", cores=int(min(workers, len(idx))), kind="oracle",
                sample=f"{len(idx)} RHS x {iters_sample} outer iterations of the same workload "
                       f"({_FORM_NAMES.get(projected, 'projected rows, three-term form' if projected else 'full x')}), one RHS per "
                       f"process ({workers} processes, 1 BLAS thread each); t/iteration {t_iter * 1e3:.1f} ms "
                       f"x mean outer iterations {mean_outer:.0f} (GPU run) = {t_rhs:.0f} s per RHS of "
                       f"{prob.nshift} shifts; wall {wall:.1f} s")


def _cpu_worker(args):
    prob, j, iters, projected = args
    qmr = projected == "qmr"
    lanczos = projected == "lanczos"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    from oracle import local_system, scocg, scocg_lanczos, scocg_projected, sqmr
    from synth import bsr_to_scipy
    H = bsr_to_scipy(prob.H)
    S = bsr_to_scipy(prob.S) if prob.S is not None else None
    Hc, Sc, loc, orb = local_system(prob, j, H, S)
    b = np.zeros(orb.size, dtype=np.complex128)
    b[loc] = 1.0
    t0 = time.perf_counter()
    if qmr or lanczos:
        rows = np.searchsorted(orb, prob.outs(j))
        fn = sqmr if qmr else scocg_lanczos
        res = fn(Hc, Sc, prob.shifts, b.real, 1e-6, rows=rows, maxiter=iters)
    elif projected:
        rows = np.searchsorted(orb, prob.outs(j))
        res = scocg_projected(Hc, Sc, prob.shifts, b, rows, 1e-6, maxiter=iters)
    else:
        res = scocg(Hc, Sc, prob.shifts, b, 1e-6, maxiter=iters)
    return (time.perf_counter() - t0) / max(1, res.n_outer)


def _cpu_full_worker(args):
    """One RHS of the workload solved to convergence by the oracle (the
    Lanczos-basis form, requested rows, tol 1e-6); returns (rhs, seconds,
    outer iterations, converged pairs)."""
    prob, j, tol = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    from oracle import local_system, scocg_lanczos
    from synth import bsr_to_scipy
    H = bsr_to_scipy(prob.H)
    S = bsr_to_scipy(prob.S) if prob.S is not None else None
    Hc, Sc, loc, orb = local_system(prob, j, H, S)
    b = np.zeros(orb.size)
    b[loc] = 1.0
    t0 = time.perf_counter()
    res = scocg_lanczos(Hc, Sc, prob.shifts, b, tol, rows=np.searchsorted(orb, prob.outs(j)))
    return j, time.perf_counter() - t0, int(res.n_outer), int(np.sum(res.status == 0))


def cpu_full(prob, args):
    """The CPU baseline without extrapolation: every RHS of the workload
    solved to convergence by the oracle (the Lanczos-basis form the product
    runs, requested rows), one RHS per process, args.cpu_full processes;
    the rate is the converged pairs over the wall time of the whole run."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    done, good, outer = 0, 0, []
    with ctx.Pool(args.cpu_full) as pool:
        for j, sec, n_out, g in pool.imap_unordered(_cpu_full_worker, [(prob, j, args.tol) for j in range(prob.nrhs)]):
            done += 1
            good += g
            outer.append(n_out)
            print(f"[cpu-full] RHS {j}: {sec:.1f} s, {n_out} outer iterations, {g}/{prob.nshift} converged "
                  f"({done}/{prob.nrhs} done, {time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    out = {"metric": METRIC, "value": good / wall, "unit": "solves/s", "kind": "oracle", "cores": args.cpu_full,
           "workload": args.workload, "nrhs": prob.nrhs, "shifts": prob.nshift, "seconds": wall,
           "converged_pairs": good, "pairs": prob.nrhs * prob.nshift,
           "outer_iterations": {"mean": float(np.mean(outer)), "max": int(np.max(outer))},
           "sample": f"every RHS ({prob.nrhs}) of the workload to convergence at tol {args.tol}, no extrapolation; "
                     f"the oracle's Lanczos-basis form on requested rows, {args.cpu_full} processes with 1 BLAS "
                     f"thread each"}
    print(json.dumps(out), flush=True)


def copy_calibration(nbytes):
    """A plain device copy of known size (for scaling FETCH_SIZE / WRITE_SIZE)."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"copy_bytes": n * 8, "seconds": dt, "GB/s": 2 * n * 8 / dt / 1e9}), flush=True)


def plain_baseline(B, P, prob, args, kw):
    """FP64 plain: the same library in FP64, textbook full-x form (every
    shift's x and p over the whole local system, two-term seed), no
    projection and no lower precision; the first args.plain RHS run
    concurrently, one workgroup each (the kernel's per-RHS time does not
    shrink with fewer RHS, so this is the plain form's rate on that many
    compute units)."""
    import torch
    sub = prob.subset(range(min(args.plain, prob.nrhs)))
    kw = dict(kw, out_ptr=sub.out_ptr, out_rows=sub.out_rows)
    if sub.cluster_ptr is not None:
        kw.update(cluster_ptr=sub.cluster_ptr, cluster_atoms=sub.cluster_atoms)
    plan = B.Plan(P, sub.shifts, sub.rhs, tol=args.tol, precision=0, audit=1, projected=0, slots=sub.nrhs,
                  threads=args.threads, **kw)
    bufs = plan.alloc_outputs()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    plan.run(bufs, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    status = bufs["status"].cpu().numpy()
    resid = bufs["resid"].cpu().numpy()
    good = int(np.sum((status == 0) & (resid <= 1e-6)))
    out = {"metric": "FP64 plain baseline (not the product configuration)", "value": good / sec, "unit": "solves/s",
           "workload": args.workload, "rhs_timed": sub.nrhs, "seconds": sec, "converged_pairs": good,
           "form": "full x, FP64, one workgroup per RHS, all RHS concurrent", "threads": plan.info["threads"],
           "slots": plan.info["slots"]}
    print(json.dumps(out), flush=True)


def measure_form(B, P, prob, kw, args, method, stream, warmup, steps, warm_budget, time_budget):
    """Autotune (unless the launch shape is given), build the plan, run the
    warm-up and the timed steps of one form of the solve; returns the plan,
    its buffers, the solves/s and the report fields (iterations, roofline).
    The warm-up stops after warm_budget seconds and the timed region holds
    as many of `steps` whole solves as fit time_budget seconds (at least
    one each); the counts actually run are returned."""
    import torch
    threads, slots, tuned = args.threads, args.slots, None
    lanczos = method in ("qmr", "cocg-lanczos")
    team = dict(team_size=args.team, panel_width=args.panel) if lanczos else {}
    if not args.no_autotune and not args.threads and not args.slots and not (lanczos and (args.team or args.panel)):
        tuned = B.autotune(P, prob.shifts, prob.rhs, probe_iters=50,
                           cache_path=os.path.join(ROOT, "paper_1402_7285_amd", "autotune_cache.json"),
                           key_extra=f"{args.workload}|{args.nrhs}", tol=args.tol, precision=PREC[args.precision],
                           projected=args.projected, method=METHODS[method], **kw)
        threads, slots = tuned["threads"], tuned["slots"]
        if lanczos and "team_size" in tuned:
            team = dict(team_size=tuned["team_size"], panel_width=tuned["panel_width"])
        print(f"[bench] {method}: autotuned {tuned}", file=sys.stderr, flush=True)
    plan = B.Plan(P, prob.shifts, prob.rhs, tol=args.tol, precision=PREC[args.precision], audit=1,
                  threads=threads, slots=slots, projected=args.projected, maxiter=args.maxiter,
                  method=METHODS[method], **team, **kw)
    projected = bool(plan.info["global"] & 2)
    qmr = bool(plan.info["global"] & 4)
    gal = bool(plan.info["global"] & 8)
    bufs = plan.alloc_outputs()
    # warm-up: up to `warmup` steps, stopping once they have used warm_budget seconds (at least one step
    # when warmup >= 1); the first one also gives the step time that sizes the timed region
    warm_done, t_warm, step_est = 0, 0.0, None
    for w in range(warmup):
        t1 = time.perf_counter()
        plan.run(bufs, stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        step_est = dt if step_est is None else min(step_est, dt)
        t_warm += dt
        warm_done += 1
        print(f"[bench] {method}: warmup {w + 1}/{warmup} done ({dt:.2f} s)", file=sys.stderr, flush=True)
        if t_warm + step_est > warm_budget:
            break
    # timed steps: as many of the requested `steps` as fit time_budget seconds (at least one)
    n_steps = steps
    if step_est is not None and time_budget > 0:
        n_steps = max(1, min(steps, int(time_budget // max(step_est, 1e-6))))
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_steps):
        ev[i][0].record(stream)
        plan.run(bufs, stream)
        ev[i][1].record(stream)
        torch.cuda.synchronize()
        print(f"[bench] {method}: step {i + 1}/{n_steps}: {ev[i][0].elapsed_time(ev[i][1]) / 1e3:.2f} s",
              file=sys.stderr, flush=True)
        if step_est is None and time_budget > 0:
            # no warm-up: size the timed region from the first step
            step_est = ev[0][0].elapsed_time(ev[0][1]) / 1e3
            n_steps_fit = max(1, min(steps, int(time_budget // max(step_est, 1e-6))))
            if n_steps_fit < n_steps:
                ev = ev[:n_steps_fit]
                n_steps = n_steps_fit
        if i + 1 >= n_steps:
            break
    wall = time.perf_counter() - t0
    step_ms = [a.elapsed_time(b) for a, b in ev]
    kernel_s = float(np.mean(step_ms)) / 1e3
    status = bufs["status"].cpu().numpy()
    resid = bufs["resid"].cpu().numpy()
    good = int(np.sum((status == 0) & (resid <= 1e-6)))
    stats = plan.stats()
    ms_per_step = wall / n_steps * 1e3
    nout = np.diff(prob.out_ptr)
    # RHS sharing the blocks at once: every resident RHS of a global system (a team holds W of them
    # on team_size workgroups), 1 for order-N clusters
    resident = plan.info["slots"] // plan.info["team_size"] * plan.info["panel_width"]
    w_share = min(resident, prob.nrhs) if prob.cluster_ptr is None else 1
    if qmr:
        alg = algorithmic_bytes_qmr(stats, nout, prob.bdim, prob.S is not None, w_share, gal)
    else:
        alg = algorithmic_bytes(stats, nout, prob.nshift, prob.bdim, prob.S is not None, PREC[args.precision],
                                projected, w_share, True)
    achieved = alg / kernel_s / 1e9
    form_key = "lanczos" if gal else "qmr" if qmr else ("proj" if projected else "full")
    report = {
        "converged_pairs": good, "pairs": int(status.size),
        "outer_iterations": {"mean": float(stats[:, 0].mean()), "max": int(stats[:, 0].max())},
        "inner_per_outer": float(stats[:, 2].sum() / max(1, stats[:, 0].sum())),
        "fallback_iterations": int(stats[:, 7].sum()),
        "step_ms": {"median": float(np.median(step_ms)), "min": float(np.min(step_ms)), "max": float(np.max(step_ms)),
                    "all": [float(v) for v in step_ms]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args, form_key, alg),
                     "kernel": ("k_team (team solver)" if plan.info["global"] & 64 else
                                "k_sqmr (persistent solver)" if qmr else "k_scocg (persistent solver)"),
                     "kernel_ms": kernel_s * 1e3, "algorithmic_bytes": alg},
    }
    form = ("COCG iterates on the real Lanczos basis, requested rows" if gal else
            "shifted QMR, real Lanczos basis, requested rows" if qmr else
            "seed-switching COCG, projected rows (three-term seed)" if projected else "seed-switching COCG, full x")
    cpu_form = "lanczos" if gal else "qmr" if qmr else projected
    return dict(plan=plan, bufs=bufs, value=good / (ms_per_step / 1e3), ms_per_step=ms_per_step, stats=stats,
                report=report, form=form, cpu_form=cpu_form, autotuned=tuned is not None, steps=n_steps,
                warmup=warm_done, wall_s=wall, step_s=kernel_s)


def chunked(B, P, prob, kw, args):
    """A workload too large for one launch within the run limits here: its
    RHS are solved in consecutive launches of args.chunk RHS (each launch a
    persistent solve of its RHS), ordered by decreasing local-pattern size
    so that each launch holds RHS of similar cost; the rate is the total of
    converged pairs over the total time."""
    import torch
    ent = np.diff(prob.cluster_ptr).astype(np.float64) if prob.cluster_ptr is not None else np.ones(prob.nrhs)
    order = longest_first(ent) if args.chunk_order == "size" else np.arange(prob.nrhs)
    stream = torch.cuda.current_stream()
    total_s, total_alg, good, pairs, outer = 0.0, 0.0, 0, 0, []
    launches = []
    for c0 in range(0, prob.nrhs, args.chunk):
        sub = prob.subset(order[c0:c0 + args.chunk])
        skw = dict(out_ptr=sub.out_ptr, out_rows=sub.out_rows)
        if sub.cluster_ptr is not None:
            skw.update(cluster_ptr=sub.cluster_ptr, cluster_atoms=sub.cluster_atoms)
        team = dict(team_size=args.team, panel_width=args.panel) if args.method != "cocg" else {}
        plan = B.Plan(P, sub.shifts, sub.rhs, tol=args.tol, threads=args.threads, slots=args.slots,
                      method=METHODS[args.method], **team, **skw)
        bufs = plan.alloc_outputs()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        plan.run(bufs, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
        st, rs = bufs["status"].cpu().numpy(), bufs["resid"].cpu().numpy()
        g = int(np.sum((st == 0) & (rs <= 1e-6)))
        stats = plan.stats()
        qmr = bool(plan.info["global"] & 4)
        gal = bool(plan.info["global"] & 8)
        nout = np.diff(sub.out_ptr)
        if qmr:
            alg = algorithmic_bytes_qmr(stats, nout, sub.bdim, sub.S is not None, 1, gal)
        else:
            alg = algorithmic_bytes(stats, nout, sub.nshift, sub.bdim, sub.S is not None, PREC[args.precision],
                                    bool(plan.info["global"] & 2), 1, True)
        total_s += sec
        total_alg += alg
        good += g
        pairs += st.size
        outer.append(stats[:, 0])
        launches.append({"rhs": sub.nrhs, "seconds": sec, "max_M": int(stats[:, 4].max()),
                         "status_counts": np.bincount(st.ravel().astype(np.int64), minlength=5).tolist(),
                         "outer_max": int(stats[:, 0].max()), "team_size": plan.info["team_size"],
                         "threads": plan.info["threads"], "workgroups": plan.info["slots"],
                         "algorithmic_GBps": alg / sec / 1e9})
        print(f"[bench] launch {len(launches)}: {sub.nrhs} RHS, {sec:.1f} s, converged {g}/{st.size} "
              f"(status counts {np.bincount(st.ravel().astype(np.int64), minlength=5).tolist()}), "
              f"largest cluster M={int(stats[:, 4].max())}, team {plan.info['team_size']}, "
              f"{alg / sec / 1e9:.0f} GB/s algorithmic", file=sys.stderr, flush=True)
        del plan, bufs
    outer = np.concatenate(outer)
    ach = total_alg / total_s / 1e9
    out = {"metric": METRIC, "value": good / total_s, "unit": "solves/s", "n_gpus": 1, "seconds": total_s,
           "converged_pairs": good, "pairs": pairs, "launches": launches,
           "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": total_alg},
           "outer_iterations": {"mean": float(outer.mean()), "max": int(outer.max())},
           "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]['desc']}", "nrhs": prob.nrhs,
                      "chunk": args.chunk, "order": args.chunk_order, "method": args.method,
                      "sample": (f"the first {prob.nrhs} RHS of the workload in generation order (a random sample: "
                                 f"RHS orbitals and cluster radii are independent draws)"
                                 if args.nrhs else "every RHS"),
                      "form": "persistent launches of chunk RHS each, in order of decreasing cluster size"}}
    print(json.dumps(out), flush=True)


def longest_first(cost):
    """Queue order by decreasing cost (stable for ties)."""
    return np.argsort(-np.asarray(cost, dtype=np.float64), kind="stable").astype(np.int32)


def binning_ab(B, args):
    """Learned binning, measured: solve the training workload and log each
    RHS's outer-iteration count, train the cost network on the GPU on those
    counts (scocg_mlp_train), then time the test workload (args.workload)
    with the work queue in index order, by local-pattern size and by the
    learned cost (both set by scocg_schedule), and by the true cost (known
    from the index-order solve).  Results must be identical in every order;
    only the time changes."""
    import torch
    from synth import make_config, mlp_init_weights, rngs_for

    def setup(name, nrhs=None):
        wl = WORKLOADS[name]
        prob = make_config(wl["cfg"], nrhs=nrhs, radius=wl.get("radius"))
        P = B.Problem(prob.H, prob.S)
        kw = dict(out_ptr=prob.out_ptr, out_rows=prob.out_rows)
        if prob.cluster_ptr is not None:
            kw.update(cluster_ptr=prob.cluster_ptr, cluster_atoms=prob.cluster_atoms)
        return prob, P, kw

    team = dict(team_size=args.team, panel_width=args.panel) if args.method != "cocg" else {}

    def timed(P, prob, kw, order=None, model=None, schedule=False):
        plan = B.Plan(P, prob.shifts, prob.rhs, tol=args.tol, threads=args.threads, slots=args.slots,
                      order=order, method=METHODS[args.method], **team, **kw)
        if schedule:
            plan.schedule(model)
        bufs = plan.alloc_outputs()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.run(bufs)
        e1.record()
        torch.cuda.synchronize()
        return plan, bufs, e0.elapsed_time(e1) / 1e3

    ptr, Ptr, kwtr = setup(args.binning)
    print(f"[binning] training workload {args.binning}: {ptr.nrhs} RHS", file=sys.stderr, flush=True)
    plan, bufs, sec = timed(Ptr, ptr, kwtr)
    st = plan.stats()
    feats = plan.features().cpu().numpy()
    print(f"[binning] training solve {sec:.1f} s", file=sys.stderr, flush=True)
    rg = rngs_for((1402, 7285, 4))
    t0 = time.perf_counter()
    model, best_val = B.scocg_mlp_train(feats, np.log(st[:, 0].astype(np.float64)),
                                        init_weights=mlp_init_weights(rg["mlp_init"]), seed=1402_7285_4,
                                        epochs=args.binning_epochs, batch=256, lr=3e-3)
    t_train = time.perf_counter() - t0
    print(f"[binning] trained in {t_train:.1f} s, best validation MSE {best_val:.3f}", file=sys.stderr, flush=True)
    del plan, bufs, Ptr
    torch.cuda.empty_cache()

    pte, Pte, kwte = setup(args.workload, args.nrhs or None)
    plan0, bufs0, sec_index = timed(Pte, pte, kwte)
    ref = bufs0["out"].cpu()
    st0 = plan0.stats()
    ft = plan0.features().cpu().numpy()
    print(f"[binning] test workload {args.workload}: {pte.nrhs} RHS, index order {sec_index:.1f} s",
          file=sys.stderr, flush=True)
    del bufs0
    pred = B.scocg_mlp_predict(model, ft).astype(np.float64)
    truth = st0[:, 0].astype(np.float64)
    ent = ft[:, 0].astype(np.float64) * ft[:, 1].astype(np.float64)
    corr = float(np.corrcoef(pred, np.log(truth))[0, 1])
    runs = {"by_size": dict(schedule=True), "learned": dict(schedule=True, model=model),
            "true_cost": dict(order=longest_first(truth * ent))}
    times = {"index": sec_index}
    for name, how in runs.items():
        _, b, sec = timed(Pte, pte, kwte, **how)
        same = bool(torch.equal(b["out"].cpu(), ref))
        times[name] = sec
        print(f"[binning] {name} order {sec:.1f} s, results identical: {same}", file=sys.stderr, flush=True)
        if not same:
            raise SystemExit("queue order changed the results")
        del b
    pairs = pte.nrhs * pte.nshift
    out = {"metric": "learned binning: solve time by work-queue order", "unit": "s",
           "train_workload": args.binning, "test_workload": args.workload, "nrhs_test": pte.nrhs,
           "seconds": times, "solves_per_s": {k: pairs / v for k, v in times.items()},
           "gain_learned_vs_index": times["index"] / times["learned"],
           "gain_learned_vs_by_size": times["by_size"] / times["learned"],
           "pred_corr_log_iters": corr, "best_val_mse": best_val, "train_seconds": t_train,
           "slots": plan0.info["slots"], "threads": plan0.info["threads"], "method": args.method,
           "team_size": plan0.info["team_size"], "panel_width": plan0.info["panel_width"]}
    print(json.dumps(out), flush=True)


KERNEL_SOURCES = {
    "proj": ("scocg_kernels.hip", "scocg_device.hpp", "scocg_params.hpp"),
    "full": ("scocg_kernels.hip", "scocg_device.hpp", "scocg_params.hpp"),
    "qmr": ("qmr_kernels.hip", "scocg_device.hpp", "scocg_params.hpp"),
    "lanczos": ("qmr_kernels.hip", "scocg_device.hpp", "scocg_params.hpp"),
}


def _kernel_source_hash(form="proj"):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[form]:
        with open(os.path.join(ROOT, "paper_1402_7285_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(args, form, alg_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this workload and form (FETCH_SIZE + WRITE_SIZE, scaled by a plain
    copy's reading), or None if there is none, the kernel sources changed
    since, or this run is not the profiled one (its algorithmic bytes differ:
    another RHS count, iteration cap or tolerance)."""
    key = f"{args.workload}_{args.precision}_{form}"
    kernel = "k_sqmr" if form in ("qmr", "lanczos") else "k_scocg"
    path = os.path.join(ROOT, "profiles", f"{kernel}_{key}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != _kernel_source_hash(form):
        return None
    ref = t.get("algorithmic_bytes_per_launch")
    if not ref or abs(alg_bytes - ref) > 1e-3 * ref:
        return None
    return t.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--time-budget", type=float, default=75.0,
                    help="seconds for the timed steps: as many of --steps whole solves as fit (at least one)")
    ap.add_argument("--warm-budget", type=float, default=30.0,
                    help="seconds for the warm-up: up to --warmup solves, at least one if --warmup >= 1")
    ap.add_argument("--deadline", type=float, default=480.0,
                    help="wall seconds from start after which the optional legs (seed-switching companion, "
                         "CPU baseline) are skipped")
    ap.add_argument("--companion-ratio", type=float, default=3.0,
                    help="expected solve time of the seed-switching form relative to the headline form")
    ap.add_argument("--workload", default="cfg1", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=sorted(PREC))
    ap.add_argument("--nrhs", type=int, default=0, help="0 = the workload's full RHS set")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--cpu-iters", type=int, default=600)
    ap.add_argument("--cpu-rhs", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--projected", type=int, default=1, help="FP64 SELECTED_G: rows-only solve (default 1)")
    ap.add_argument("--method", default="cocg-lanczos", choices=["cocg", "qmr", "cocg-lanczos"],
                    help="cocg: shifted COCG with seed switching; qmr: shifted QMR over the real Lanczos basis; "
                         "cocg-lanczos: the COCG iterates on that basis")
    ap.add_argument("--copy-calib", type=int, default=0, help="only run a device copy of this many bytes")
    ap.add_argument("--cpu-full", type=int, default=0,
                    help="only run the CPU baseline on every RHS of the workload with this many processes")
    ap.add_argument("--no-autotune", action="store_true", help="use --threads/--slots as given")
    ap.add_argument("--team", type=int, default=0,
                    help="Lanczos-basis forms: workgroups per team (-1 one-workgroup solver, 0 autotuned)")
    ap.add_argument("--panel", type=int, default=0, help="Lanczos-basis forms: RHS per panel (0 autotuned)")
    ap.add_argument("--no-companion", action="store_true",
                    help="do not also time the seed-switching COCG form when --method is another form")
    ap.add_argument("--plain", type=int, default=0,
                    help="measure FP64 plain instead: full x, one RHS at a time, on this many RHS")
    ap.add_argument("--binning", default="",
                    help="measure learned binning: train on this workload's logs, time --workload's queue orders")
    ap.add_argument("--binning-epochs", type=int, default=150)
    ap.add_argument("--chunk", type=int, default=0,
                    help="solve the workload in consecutive launches of this many RHS (large cluster workloads)")
    ap.add_argument("--chunk-order", default="size", choices=["size", "index"])
    ap.add_argument("--maxiter", type=int, default=0,
                    help="diagnostics only: cap outer iterations (changes the workload; not a metric run)")
    args = ap.parse_args()
    if args.copy_calib:
        copy_calibration(args.copy_calib)
        return

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the solver shards over RHS with no "
              f"communication during the solve, but multi-GPU runs are not implemented.", file=sys.stderr)
        sys.exit(2)

    if args.cpu_full:
        from synth import make_config
        wl = WORKLOADS[args.workload]
        return cpu_full(make_config(wl["cfg"], nrhs=args.nrhs or None, radius=wl.get("radius")), args)

    import torch
    from paper_1402_7285_amd import binding as B
    from synth import make_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.binning:
        return binning_ab(B, args)
    wl = WORKLOADS[args.workload]
    prob = make_config(wl["cfg"], nrhs=args.nrhs or None, radius=wl.get("radius"))
    print(f"[bench] {args.workload}: M={prob.M} K={prob.nshift} nrhs={prob.nrhs} precision={args.precision}",
          file=sys.stderr, flush=True)
    P = B.Problem(prob.H, prob.S)
    kw = dict(out_ptr=prob.out_ptr, out_rows=prob.out_rows)
    if prob.cluster_ptr is not None:
        kw.update(cluster_ptr=prob.cluster_ptr, cluster_atoms=prob.cluster_atoms)
    if args.plain:
        return plain_baseline(B, P, prob, args, kw)
    if args.chunk:
        return chunked(B, P, prob, kw, args)
    stream = torch.cuda.current_stream()
    r = measure_form(B, P, prob, kw, args, args.method, stream, args.warmup, args.steps, args.warm_budget,
                     args.time_budget)
    plan, bufs = r["plan"], r["bufs"]
    out = {
        "metric": METRIC, "value": r["value"], "unit": "solves/s", "n_gpus": 1, "steps": r["steps"],
        "warmup": r["warmup"], "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp64": "c128", "fp32": "c64", "bf16": "c64/bf16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}", "nrhs": prob.nrhs, "shifts": prob.nshift,
                   "M": prob.M, "tol": args.tol, "precision": args.precision, "batched": "persistent",
                   "slots": plan.info["slots"], "threads": plan.info["threads"], "form": r["form"],
                   "lds_bytes": plan.info["lds_bytes"], "cg_direction_in_lds": bool(plan.info["global"] & 16),
                   "team_size": plan.info["team_size"], "panel_width": plan.info["panel_width"],
                   "matrix_cores": bool(plan.info["global"] & 128),
                   "cg_vectors_in_registers": bool(plan.info["global"] & 256),
                   "s_blocks_ell": bool(plan.info["global"] & 512),
                   "autotuned": r["autotuned"], "steps_requested": args.steps, "warmup_requested": args.warmup,
                   "time_budget_s": args.time_budget},
        **r["report"],
    }
    print(f"[bench] headline: {r['value']:.1f} solves/s over {r['steps']} timed steps "
          f"({r['ms_per_step'] / 1e3:.2f} s each)", file=sys.stderr, flush=True)
    # the HBM bandwidth a plain device copy reaches on this GPU (1 GiB, best of three): the measured
    # ceiling beside the published 8 TB/s
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b_ = torch.empty_like(a)
    best = float("inf")
    for _ in range(3):
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        b_.copy_(a)
        c1.record()
        torch.cuda.synchronize()
        best = min(best, c0.elapsed_time(c1) / 1e3)
    copy_gbs = 2 * a.numel() * 8 / best / 1e9
    del a, b_
    out["roofline"]["measured_copy_GBps"] = copy_gbs
    out["roofline"]["frac_of_measured_copy"] = out["roofline"]["achieved"] / copy_gbs
    left = args.deadline - (time.perf_counter() - T_START)
    if args.method != "cocg" and not args.no_companion:
        # the seed-switching form of the same method, timed in the same run (one step, no warm-up beyond
        # the autotuner's probes), only if the time left allows it: its solve takes about
        # companion_ratio times the headline form's
        est = r["step_s"] * args.companion_ratio
        if left > 2.0 * est + 60.0:
            c = measure_form(B, P, prob, kw, args, "cocg", stream, 0, 1, 0.0, 0.0)
            out["seed_switching_form"] = {"form": c["form"], "value": c["value"], "ms_per_step": c["ms_per_step"],
                                          "steps": c["steps"], "threads": c["plan"].info["threads"],
                                          "slots": c["plan"].info["slots"], **c["report"]}
            del c
        else:
            out["seed_switching_form"] = {"skipped": f"estimated {est:.0f} s, {left:.0f} s left before the deadline"}
    w = np.zeros(prob.nshift)
    if prob.nshift > 1:
        dE = np.diff(prob.shifts.real)
        w[:-1] += 0.5 * dE
        w[1:] += 0.5 * dE
    plan.integrate(bufs, w, 0.0, 0.1)                     # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    rho, ldos = plan.integrate(bufs, w, 0.0, 0.1, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_int = e0.elapsed_time(e1)
    int_bytes = plan.out_count * 16 + (plan.out_count // prob.nshift) * 8 + prob.nrhs * prob.nshift * 8
    out["energy_integration"] = {"ms": ms_int, "bytes": int_bytes, "GB/s": int_bytes / (ms_int * 1e-3) / 1e9,
                                 "what": "density-matrix rows and local DOS from the computed G (trapezoid, "
                                         "mu = 0, kT = 0.1)"}
    if not args.no_cpu_baseline:
        workers = max(1, min(16, os.cpu_count() or 1))
        left = args.deadline - (time.perf_counter() - T_START)
        if left > 90.0:
            print(f"[bench] cpu baseline: oracle on {workers} processes ...", file=sys.stderr, flush=True)
            out["cpu_baseline"] = cpu_baseline(prob, r["stats"], args.cpu_rhs, args.cpu_iters, workers,
                                               r["cpu_form"])
        else:
            out["cpu_baseline"] = None
            print(f"[bench] cpu baseline skipped: {left:.0f} s left before the deadline", file=sys.stderr,
                  flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
