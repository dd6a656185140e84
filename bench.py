"""Benchmark: ms per full-spectrum cylindrical Poisson solve on one MI355X.

One step = one complete solve (forward azimuthal DFT, V-cycles on every
plane until the relative residual reaches --tol, inverse DFT) of the
paper-scale 400 x 128 x 512 annular grid (65 real-FFT modes), with rho and
phi resident in HBM.  The metric is the time to rel-L2 1e-12 against the
oracle: by default the V-cycles start from the full-multigrid guess (option
fmg), where tol 1e-13 meets it; from a zero start it takes tol 1e-14 (one more
cycle of error per residual), timed beside it as the variant zero_start.  Inputs are synthetic: the seeded manufactured potential
phi_true of the workloads module, and rho = A phi_true / s formed by the CPU
oracle in extended precision (the CPU-baseline leg), so every run also reports
the error against the oracle's exact solution and against phi_true.

Prints one JSON line (see the repository's benchmark contract).
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak
METRIC = "ms per full-spectrum Poisson solve to rel-L2 1e-12; achieved HBM GB/s vs peak"
REL_L2_TARGET = 1e-12
# relative residual tolerance that meets rel-L2 1e-12 at 400 x 128 x 512 from
# each start (error per residual: about 9 after the full-multigrid start, 70
# from zero)
START_TOL = {"fmg": 1e-13, "zero": 1e-14}


def cycle_bytes(direct_level):
    """Algorithmic bytes per finest unknown of one V-cycle: 52 B per unknown of
    each level on fused down and up passes (26 B each), levels weighted 4^-l,
    down to the level solved exactly (32 B per unknown of it: read f, write and
    read w, write u); 52 * 4 / 3 = 69.3 B with every level on passes."""
    if direct_level is None or direct_level < 1:
        return 52.0 * 4.0 / 3.0
    return sum(52.0 * 4.0 ** -l for l in range(direct_level)) + 32.0 * 4.0 ** -direct_level


def fmg_bytes(direct_level):
    """Algorithmic bytes of the full-multigrid start per finest unknown: read f
    (8), write the level-1 right-hand side (2), one V-cycle from level 1 down
    (the cycle's bytes below the finest level); the first finest down pass then
    forms the start from the level-1 answer (2) instead of reading an iterate
    (8), so it is never written."""
    return 8.0 + 2.0 + (cycle_bytes(direct_level) - 52.0) + 2.0 - 8.0
SEQ_FIELDS = 8  # seeded drift directions the 200-step sequence cycles through
FUSED_SOURCES = ("paper_2609_07172_amd/csrc/fused.hip", "paper_2609_07172_amd/csrc/fused_pass.h",
                 "paper_2609_07172_amd/csrc/stencil.h")


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in FUSED_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*msg):
    print("[bench]", *msg, file=sys.stderr, flush=True)


INTERIOR = (slice(None), slice(1, -1), slice(1, -1))


def interior_rel(a, b):
    i = INTERIOR
    return float(np.linalg.norm((a[i] - b[i]).ravel()) / np.linalg.norm(b[i].ravel()))


def accuracy(phi, ref, problem, label):
    """Errors of phi against a reference over interior nodes: rel-L2; rel-L_inf
    (max |e| / max |ref|, Sec. 5.2); Sec. 5.1's epsilon_2 with cylindrical
    weights r_i dr dz; and rel-L2 of the charge-driven part, i.e. relative to
    ref - 300 z / L (the manufactured potential without its blobs), because
    the 300 V background dominates ||phi||."""
    import workloads as W

    _, z, r = W.node_coordinates(problem)
    i = INTERIOR
    e = (phi - ref)[i]
    b = ref[i]
    bg = (problem.phi_zL * z / problem.length)[None, 1:-1, None]
    w = r[None, None, 1:-1]
    return {f"rel_l2_vs_{label}": float(np.linalg.norm(e) / np.linalg.norm(b)),
            f"rel_linf_vs_{label}": float(np.abs(e).max() / np.abs(b).max()),
            f"eps2_vs_{label}": float(np.sqrt(np.sum(w * e * e) / np.sum(w * b * b))),
            f"rel_l2_charge_part_vs_{label}": float(np.linalg.norm(e) / np.linalg.norm(b - bg))}


def cpu_leg(problem, workers: int):
    """The oracle on the host: form rho from phi_true, then solve it (timed)."""
    from oracle import fv, solvers

    t0 = time.perf_counter()
    import workloads as W

    phit = W.manufactured_potential(problem, 12345, np.longdouble)
    rho = fv.charge_from_potential(fv.Grid.of(problem, np.longdouble), phit).astype(np.float64)
    prep = time.perf_counter() - t0
    log(f"cpu: rho formed in {prep:.1f} s")
    grid = fv.Grid.of(problem)
    # repeat the solve for about ten seconds (at least once) and report the mean
    times = []
    while not times or (sum(times) < 10.0 and len(times) < 50):
        t0 = time.perf_counter()
        ref = solvers.solve_separable(grid, rho, problem.bc, workers=workers)
        times.append(time.perf_counter() - t0)
    t_solve = sum(times) / len(times)
    log(f"cpu: oracle solve {t_solve:.3f} s (mean of {len(times)}) on {workers} threads")
    return rho, ref, phit.astype(np.float64), t_solve, len(times)


def cpu_leg_sequence(problem, phit, fields=SEQ_FIELDS):
    """Oracle inputs of the time sequence: the seeded drift directions g_k (unit-RMS
    blob parts of phi_true(97531 + k)) and their charges A g_k / s, formed by the
    oracle's operator, so every step's exact discrete answer is known."""
    from oracle import fv

    import workloads as W

    t0 = time.perf_counter()
    grid = fv.Grid.of(problem)
    _, z, _ = W.node_coordinates(problem)
    blobs = phit[:, 1:-1, 1:-1] - (problem.phi_zL * z / problem.length)[None, 1:-1, None]
    amp = 0.01 * float(np.sqrt(np.mean(blobs * blobs)))
    g = [W.blob_field(problem, 97531 + k) for k in range(fields)]
    drho = [fv.charge_from_potential(grid, f) for f in g]
    log(f"cpu: {fields} drift fields of the sequence formed in {time.perf_counter() - t0:.1f} s")
    return {"amp": amp, "fields": g, "charges": drho}


def cpu_leg_batch(workers: int, count: int = 16):
    """Oracle inputs of the uneven batch: problem i carries phi_true(12345 + i), its
    charge formed by the oracle in extended precision, and the oracle's exact
    separable solve of that charge."""
    from oracle import fv, solvers

    import workloads as W

    t0 = time.perf_counter()
    out = []
    for i, q in enumerate(W.random_problems(count, 24680)):
        phit = W.manufactured_potential(q, 12345 + i, np.longdouble)
        rho = fv.charge_from_potential(fv.Grid.of(q, np.longdouble), phit).astype(np.float64)
        ref = solvers.solve_separable(fv.Grid.of(q), rho, q.bc, workers=workers)
        out.append((rho, ref, phit.astype(np.float64)))
    log(f"cpu: {count} uneven problems formed and solved by the oracle in {time.perf_counter() - t0:.1f} s")
    return out


def alg_bytes(info, nt):
    """Algorithmic HBM bytes of the finest-level fused passes and of one solve."""
    (nr0, nz0), (nr1, nz1) = info["level_shapes"][0], info["level_shapes"][1]
    n0 = nt * (nr0 - 2) * (nz0 - 2)
    n1 = nt * (nr1 - 2) * (nz1 - 2)
    # up pass: read u (8), f (8), coarse correction (8 per coarse unknown); write u (8)
    up = 24 * n0 + 8 * n1
    # down pass: read u (8, skipped on the first cycle), f (8); write u (8), coarse f (8)
    down = 24 * n0 + 8 * n1
    # merged pass (up pass of one cycle, down pass of the next): read u, f, the
    # coarse correction; write u and the coarse right-hand side
    merged = 24 * n0 + 16 * n1
    return {"n0": n0, "n1": n1, "up": up, "down": down, "down_first": down - 8 * n0, "merged": merged}


def traffic_for(kernel: str, launches_bytes: float):
    """HBM bytes per launch measured with rocprofv3 counters, if taken on the current source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash() or kernel not in rec.get("bytes_per_launch", {}):
        return None
    return float(rec["bytes_per_launch"][kernel])


FINE_KERNELS = {  # finest-level FP64 pass symbols -> kernel class
    "k_pass_fine<double, 2, 1, true, true>": "fine_down",
    "k_pass_fine<double, 2, 1, true, false>": "fine_down",
    "k_pass_fine<double, 2, 1, false, false>": "fine_up",
    # the first down pass after the full-multigrid start (forms the start itself)
    "k_pass_fine_pro<double, 2, 1>": "fine_down_pro",
    # the up pass of one cycle and the down pass of the next
    "k_pass_merge<double, 4, 1>": "fine_merged",
}


def _counter_rows(path: str, counter: str):
    import csv

    files = []
    for dirpath, _, names in os.walk(path):
        files += [os.path.join(dirpath, n) for n in names if n.endswith("counter_collection.csv")]
    if len(files) != 1:
        raise SystemExit(f"expected one counter_collection.csv under {path}, found {len(files)}")
    with open(files[0], newline="") as fh:
        return [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]


def ingest_counters(fetch_dir: str, write_dir: str, probe_mib: int):
    """HBM bytes per launch of the finest-level passes from FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by the factor that makes the copy probe (which
    reads and writes probe_mib MiB) count exactly its own size."""
    probe = float(probe_mib) * (1 << 20)
    out = {"source_hash": source_hash(), "copy_probe_bytes": probe, "counters": {},
           "bytes_per_launch": {}}
    for counter, path in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(path, counter)
        copies = [r for r in rows if "cp::" not in r["Kernel_Name"] and "copy" in r["Kernel_Name"]]
        big = max(int(r["Grid_Size"]) for r in copies)
        copies = [float(r["Counter_Value"]) for r in copies if int(r["Grid_Size"]) == big]
        cls_vals = {}
        for r in rows:
            for sym, cls in FINE_KERNELS.items():
                if sym in r["Kernel_Name"]:
                    cls_vals.setdefault(cls, []).append(float(r["Counter_Value"]))
        out["counters"][counter] = {
            "copy_kib_per_dispatch": sum(copies) / len(copies),
            "copy_dispatches": len(copies),
            "kib_per_dispatch": {k: sum(v) / len(v) for k, v in cls_vals.items()},
            "dispatches": {k: len(v) for k, v in cls_vals.items()},
        }
    for cls in sorted(set(FINE_KERNELS.values())):
        if not all(cls in out["counters"][c]["kib_per_dispatch"] for c in ("FETCH_SIZE", "WRITE_SIZE")):
            continue
        total = 0.0
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            c = out["counters"][counter]
            scale = probe / (c["copy_kib_per_dispatch"] * 1024.0)
            c["scale"] = scale
            total += c["kib_per_dispatch"][cls] * 1024.0 * scale
        out["bytes_per_launch"][cls] = total
    dst = os.path.join(ROOT, "profiles", "traffic.json")
    with open(dst, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def time_variant(plan, rho_d, phi_d, args, ref, phit, options):
    """Time the same solve with other solver options (same inputs): the timed loop
    runs without events (graph replay needs them off); one more solve with
    events gives the per-kernel-class breakdown."""
    import torch

    for k, v in options.items():
        plan.set_option(k, v)
    for _ in range(args.warmup):
        plan.solve(rho_d, tol=args.tol, phi=phi_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = plan.solve(rho_d, tol=args.tol, phi=phi_d)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    out = {"options": options, "ms": round(ms, 4), "cycles": st["cycles"],
           "refinements": st["refinements"], "frozen_planes": st["frozen_planes"],
           "rel_residual": st["rel_residual"]}
    if ref is not None:
        phi = phi_d.cpu().numpy()
        out["rel_l2_vs_oracle"] = interior_rel(phi, ref)
        out["rel_l2_vs_phi_true"] = interior_rel(phi, phit)
    plan.set_option("timing", 1)
    _, st = plan.solve(rho_d, tol=args.tol, phi=phi_d)
    plan.set_option("timing", 0)
    out["kernel_ms_one_solve"] = {k: round(v, 4) for k, v in st["kernel_ms"].items()}
    log(f"variant {options}: {ms:.3f} ms/solve, cycles {st['cycles']}, "
        f"refinements {st['refinements']}, rel residual {st['rel_residual']:.3e}")
    for k in options:
        plan.set_option(k, {"precision": 64, "inner_cycles": 2}.get(k, 0))
    return out


def time_autotuned(problem, rho_d, args, ref, phit):
    """A fresh plan tuned by the library's autotuner, then timed like the main solve."""
    import torch

    import paper_2609_07172_amd as P

    plan = P.Plan.for_problem(problem)
    t0 = time.perf_counter()
    plan.autotune()
    tune_s = time.perf_counter() - t0
    chosen = {k: plan.get_option(k) for k in ("chunk_rows", "chunk_rows_coarse", "prefetch", "groups")}
    phi_d = torch.empty_like(rho_d)
    for _ in range(args.warmup):
        plan.solve(rho_d, tol=args.tol, phi=phi_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = plan.solve(rho_d, tol=args.tol, phi=phi_d)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    out = {"chosen": chosen, "tune_s": round(tune_s, 2), "ms": round(ms, 4), "cycles": st["cycles"]}
    if ref is not None:
        out["rel_l2_vs_oracle"] = interior_rel(phi_d.cpu().numpy(), ref)
    log(f"autotuned {chosen} in {tune_s:.1f} s: {ms:.3f} ms/solve")
    plan.close()
    return out


def time_sequence(problem, rho0_d, args, seq, phit, steps=200):
    """The 200-step time sequence of one 400 x 128 x 512 problem: at step t the
    potential moves by sign[t] * 0.01 * rms(blob part of phi_true) times one of
    SEQ_FIELDS seeded unit-RMS blob fields (workloads.sequence_plan), so the
    charge moves by the same multiple of that field's charge (formed by the
    oracle) and the exact answer of every step is known.  Each step is solved
    to tol from the full-multigrid start (cold) or from the previous answer
    (warm start); the timed
    loop includes the charge update on the device.  An untimed replay then
    checks every step's answer against its exact potential.  Without the CPU
    leg (no oracle), the drift is a smooth seeded charge field instead and only
    residuals are reported."""
    import torch

    import paper_2609_07172_amd as P
    import workloads as W

    dev = rho0_d.device
    tol = args.tol
    which, signs = W.sequence_plan(steps, SEQ_FIELDS)
    if seq is not None:
        dq = [torch.from_numpy(f).to(dev) for f in seq["charges"]]
        dphi = [torch.from_numpy(f).to(dev) for f in seq["fields"]]
        amp = seq["amp"]
        kind = "phi_true drift: 0.01 rms(blob part) x seeded unit-RMS blob field per step"
    else:
        dq = [torch.from_numpy(f).to(dev) for f in W.drift_fields(problem, count=SEQ_FIELDS)]
        dphi = None
        amp = 0.01 * float(rho0_d.abs().max())
        kind = "rho drift: 0.01 max|rho0| x smooth seeded field per step (no exact answers)"
    out = {"steps": steps, "tol": tol, "drift": kind, "fields": SEQ_FIELDS}
    for label, warm in (("cold", 0), ("warm", 1)):
        plan = P.Plan.for_problem(problem, warm_start=warm, fmg=1)  # fmg: cold starts only
        rho = rho0_d.clone()
        phi = torch.zeros_like(rho)
        allow = (P.OK, P.NOT_CONVERGED)
        plan.solve(rho, tol=tol, phi=phi, allow=allow)  # converged start, not timed
        torch.cuda.synchronize()
        cycles, not_ok = [], 0
        worst = 0.0
        t0 = time.perf_counter()
        for t in range(steps):
            rho.add_(dq[which[t]], alpha=amp * float(signs[t]))
            _, st = plan.solve(rho, tol=tol, phi=phi, allow=allow)
            cycles.append(st["cycles"])
            worst = max(worst, st["rel_residual"])
            not_ok += st["status"] != P.OK
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        rec = {"ms_per_step": round(ms, 4), "cycles_mean": float(np.mean(cycles)),
               "cycles_max": int(max(cycles)), "worst_rel_residual": worst, "not_converged": int(not_ok)}
        if dphi is not None:
            # untimed replay: every step against its exact potential
            exact = torch.from_numpy(phit).to(dev)
            inner = (slice(None), slice(1, -1), slice(1, -1))
            rho = rho0_d.clone()
            phi.zero_()
            plan.solve(rho, tol=tol, phi=phi, allow=allow)
            errs = []
            for t in range(steps):
                rho.add_(dq[which[t]], alpha=amp * float(signs[t]))
                exact.add_(dphi[which[t]], alpha=amp * float(signs[t]))
                plan.solve(rho, tol=tol, phi=phi, allow=allow)
                e = torch.linalg.vector_norm((phi - exact)[inner]) / torch.linalg.vector_norm(exact[inner])
                errs.append(float(e))
            rec["rel_l2_vs_exact_max"] = max(errs)
            rec["rel_l2_vs_exact_mean"] = float(np.mean(errs))
            rec["steps_over_1e-12"] = int(sum(e > REL_L2_TARGET for e in errs))
        out[label] = rec
        log(f"sequence {label}: {ms:.3f} ms/step, {np.mean(cycles):.2f} cycles/step, "
            f"{not_ok} not converged" + (f", worst rel-L2 {rec['rel_l2_vs_exact_max']:.2e}" if dphi is not None else ""))
        plan.close()
    return out


def time_batch(args, batch):
    """The 16 uneven problems of the batching workload (seeded shapes), each with
    phi_true(12345 + i) and the oracle's charge and answer (blob charges without
    the CPU leg), solved together by cylpoisson_solve_batch (one stream per
    problem) and one after another;
    every problem's answer is compared with the oracle and phi_true."""
    import torch

    import paper_2609_07172_amd as P
    import workloads as W

    probs = W.random_problems(16, 24680)
    if batch is not None:
        rhos = [torch.from_numpy(b[0]).to("cuda:0") for b in batch]
    else:
        rhos = [torch.from_numpy(W.blob_charge(q, 100 + i)).to("cuda:0") for i, q in enumerate(probs)]
    # the full-multigrid start: from zero, tol 1e-14 leaves up to 1.2e-12 on
    # some of these grids (their error runs at about 100 times the residual)
    plans = [P.Plan.for_problem(q, fmg=1) for q in probs]
    phis = [torch.empty_like(r) for r in rhos]
    handles = [p.handle for p in plans]
    P.solve_batch(handles, rhos, phis, tol=args.tol, allow=(P.OK, P.NOT_CONVERGED))
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        status, sts = P.solve_batch(handles, rhos, phis, tol=args.tol, allow=(P.OK, P.NOT_CONVERGED))
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t0) / reps * 1e3
    stats = [p.stats() for p in plans]
    got = [f.cpu().numpy() for f in phis]

    t0 = time.perf_counter()
    for _ in range(reps):
        for p, r, f in zip(plans, rhos, phis):
            p.solve(r, tol=args.tol, phi=f, allow=(P.OK, P.NOT_CONVERGED))
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) / reps * 1e3
    unknowns = sum(q.unknowns for q in probs)
    out = {"problems": [q.name for q in probs], "unknowns": unknowns, "tol": args.tol, "options": {"fmg": 1},
           "rho": "manufactured phi_true(12345 + i)" if batch is not None else "blob",
           "batch_ms": round(batch_ms, 3), "sequential_ms": round(seq_ms, 3),
           "launches": "one stream and host thread per problem", "statuses": sts,
           "cycles": [s["cycles"] for s in stats], "worst_rel_residual": max(s["rel_residual"] for s in stats)}
    if batch is not None:
        out["rel_l2_vs_oracle"] = [interior_rel(g, b[1]) for g, b in zip(got, batch)]
        out["rel_l2_vs_phi_true"] = [interior_rel(g, b[2]) for g, b in zip(got, batch)]
        out["rel_l2_vs_oracle_max"] = max(out["rel_l2_vs_oracle"])
        out["meets_target"] = bool(out["rel_l2_vs_oracle_max"] <= REL_L2_TARGET)
    log(f"batch of 16: {batch_ms:.2f} ms on 16 streams, {seq_ms:.2f} ms one by one"
        + (f", worst rel-L2 vs oracle {out['rel_l2_vs_oracle_max']:.2e}" if batch is not None else ""))
    for p in plans:
        p.close()
    return out


def time_meshes(problem, args):
    """The paper-scale node counts on explicit cell-centred meshes (App. A):
    uniform cells, and cells stretched geometrically 4:1 towards the inner wall
    and towards z = 0 (boundary-layer refinement), each solved by plain
    V-cycles, by plain V-cycles after the autotuner chose omega, by
    V-cycle-preconditioned FGMRES and by V-cycles with the alternating zebra
    line smoother."""
    import torch

    import paper_2609_07172_amd as P
    import workloads as W

    nr, nt, nz = problem.nr, problem.ntheta, problem.nz
    length = problem.length
    meshes = {
        "cell_uniform": (np.linspace(problem.r_in, problem.r_out, nr - 1), np.linspace(0.0, length, nz - 1)),
        "cell_stretched_4to1": (W.stretched_points(problem.r_in, problem.r_out, nr - 2, 4.0 ** (1.0 / (nr - 3))),
                                W.stretched_points(0.0, length, nz - 2, 0.25 ** (1.0 / (nz - 3)))),
    }
    out = {}
    for name, (rf, zf) in meshes.items():
        rho = torch.from_numpy(W.mesh_blob_charge(W.cell_centres(rf), W.cell_centres(zf), nt, seed=11)).to("cuda:0")
        phi = torch.empty_like(rho)
        rec = {}
        for label, opts in (("vcycles", {}), ("vcycles_tuned_omega", {"tune_omega": 1}),
                            ("mg_fgmres", {"krylov": 1, "krylov_precond": 3}),
                            ("alternating_lines", {"smoother": 2})):
            plan = P.Plan.from_mesh(rf, zf, nt, P.CELL, problem.bc, **opts)
            if opts.get("tune_omega"):
                plan.autotune()
            for _ in range(2):
                plan.solve(rho, tol=args.tol, phi=phi)
            torch.cuda.synchronize()
            steps = max(3, args.steps // 4)
            t0 = time.perf_counter()
            for _ in range(steps):
                _, st = plan.solve(rho, tol=args.tol, phi=phi)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
            rec[label] = {"ms": round(ms, 4), "cycles": st["cycles"], "krylov_steps": st["krylov_iterations"],
                          "rel_residual": st["rel_residual"], "fused_levels": plan.info()["fused_levels"],
                          "omega": plan.get_option("omega")}
            log(f"mesh {name} {label}: {ms:.3f} ms/solve, {st['cycles']} V-cycles, "
                f"rel residual {st['rel_residual']:.3e}")
            plan.close()
        out[name] = rec
    return out


def time_learned(problem, rho_d, args, ref, phit):
    """The learned preconditioner at this size: a network trained on the GPU on
    about 20k pairs from a sequence of charges of this grid (the manufactured
    one plus seeded smooth drifts), then the learned solve (FGMRES with the
    network, judged against one V-cycle, V-cycles taking over when it loses),
    timed like the plain solve; the per-step contraction of FGMRES without a
    preconditioner and with the smoother the network imitates beside it; and
    the network's forward pass over all mode pairs (MFMA throughput)."""
    import torch

    import paper_2609_07172_amd as P
    import workloads as W

    fields = [torch.from_numpy(f).to(rho_d.device) for f in W.drift_fields(problem, count=5, seed=4242)]
    amp = 0.05 * float(rho_d.abs().max())
    plan = P.Plan.for_problem(problem)
    net = P.Net(seed=2024)
    t0 = time.perf_counter()
    for k, f in enumerate(fields):
        net.collect(plan, rho_d + amp * f, cycles=8, patches_per_cycle=512, seed=k)
    collect_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    net.train(epochs=30, batch=256, lr=2e-3)
    loss = net.train(epochs=10, batch=256, lr=5e-4)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    out = {"pairs": net.patch_count(), "collect_s": round(collect_s, 2), "train_s": round(train_s, 2),
           "final_loss": loss}
    lplan = P.Plan.for_problem(problem, krylov=1)
    P.plan_set_net(lplan, net)
    phi_d = torch.empty_like(rho_d)
    lplan.solve(rho_d, tol=args.tol, phi=phi_d)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 4)
    t0 = time.perf_counter()
    for _ in range(reps):
        _, st = lplan.solve(rho_d, tol=args.tol, phi=phi_d)
    torch.cuda.synchronize()
    out.update({"ms": round((time.perf_counter() - t0) / reps * 1e3, 4), "status": st["status"],
                "krylov_iterations": st["krylov_iterations"], "vcycles": st["cycles"],
                "fell_back": st["learned_fallback"], "vcycle_rate": st["vcycle_rate"],
                "learned_rate": st["learned_rate"], "rel_residual": st["rel_residual"]})
    if ref is not None:
        got = phi_d.cpu().numpy()
        out["rel_l2_vs_oracle"] = interior_rel(got, ref)
        out["rel_l2_vs_phi_true"] = interior_rel(got, phit)
    rates = {}
    for label, precond in (("none", 0), ("smoother", 2), ("network", 1)):
        pl = P.Plan.for_problem(problem, krylov=1, krylov_precond=precond, fallback=0, krylov_max=8)
        P.plan_set_net(pl, net)
        _, s2 = pl.solve(rho_d, tol=args.tol, phi=phi_d, allow=(P.OK, P.NOT_CONVERGED))
        rates[label] = s2["learned_rate"]
        pl.close()
    out["fgmres_rate_per_step"] = rates
    # the network inside the multigrid preconditioner: FGMRES with one V-cycle
    # (krylov_precond 3) against one V-cycle followed by the network's
    # correction of the residual it leaves (krylov_precond 4), per step and to tol
    inner = {}
    for label, precond, n in (("vcycle", 3, None), ("vcycle_plus_network", 4, net),
                              ("vcycle_plus_nothing", 4, None)):
        pl = P.Plan.for_problem(problem, krylov=1, krylov_precond=precond, fallback=0, krylov_max=8)
        if n is not None:
            P.plan_set_net(pl, n)
        _, s2 = pl.solve(rho_d, tol=1e-30, phi=phi_d, allow=(P.OK, P.NOT_CONVERGED))
        rec = {"rate_per_step": s2["learned_rate"]}
        pl.close()
        if label != "vcycle_plus_nothing":
            pl = P.Plan.for_problem(problem, krylov=1, krylov_precond=precond)
            if n is not None:
                P.plan_set_net(pl, n)
            pl.solve(rho_d, tol=args.tol, phi=phi_d)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                _, s3 = pl.solve(rho_d, tol=args.tol, phi=phi_d)
            torch.cuda.synchronize()
            rec.update({"ms": round((time.perf_counter() - t0) / reps * 1e3, 4), "status": s3["status"],
                        "krylov_iterations": s3["krylov_iterations"], "fell_back": s3["learned_fallback"],
                        "rel_residual": s3["rel_residual"]})
            if ref is not None:
                rec["rel_l2_vs_oracle"] = interior_rel(phi_d.cpu().numpy(), ref)
            pl.close()
        inner[label] = rec
    out["network_inside_vcycle"] = inner
    log(f"learned V-cycle: FGMRES per step {inner['vcycle']['rate_per_step']:.4f} (V-cycle), "
        f"{inner['vcycle_plus_network']['rate_per_step']:.4f} (V-cycle + network), "
        f"{inner['vcycle_plus_nothing']['rate_per_step']:.4f} (V-cycle, judged path without network); "
        f"{inner['vcycle_plus_network']['ms']:.2f} ms against {inner['vcycle']['ms']:.2f} ms")
    # the network's forward pass over every mode pair of this grid
    npairs, H, Wd = problem.ntheta // 2 + 1, problem.nz - 2, problem.nr - 2
    x = torch.randn((npairs, H, Wd, 4), dtype=torch.float32, device=rho_d.device)
    net.forward(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        net.forward(x)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 5
    flops = 2.0 * npairs * H * Wd * (9 * 4 * 16 + 9 * 16 * 16 + 9 * 16 * 2)
    # algorithmic HBM bytes: read 4 FP32 inputs, write 2 FP32 outputs per pixel
    nbytes = 24.0 * npairs * H * Wd
    out["network_forward"] = {"pixels": npairs * H * Wd, "ms": round(fwd_ms, 4),
                              "tflops": round(flops / (fwd_ms * 1e-3) / 1e12, 2),
                              "mfma_bf16_peak_tflops": 2500.0,
                              "hbm_gbs": round(nbytes / (fwd_ms * 1e-3) / 1e9, 1), "hbm_peak_gbs": HBM_PEAK_GBS,
                              "roofline_ms": round(max(flops / 2.5e15, nbytes / (HBM_PEAK_GBS * 1e9)) * 1e3, 4)}
    log(f"learned: {out['ms']:.3f} ms/solve, FGMRES rates {rates}, V-cycle {st['vcycle_rate']:.3f}, "
        f"fell back {st['learned_fallback']}; network forward {fwd_ms:.3f} ms")
    for q in (lplan, plan):
        q.close()
    net.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tol", type=float, default=None,
                    help="relative residual tolerance (default: 1e-13 with --start fmg, 1e-14 from zero)")
    ap.add_argument("--start", choices=["fmg", "zero"], default="fmg",
                    help="first iterate of the V-cycles: full-multigrid guess or zero")
    ap.add_argument("--workload", choices=["paper", "batched", "small"], default="paper")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg (blob rho)")
    ap.add_argument("--option", action="append", default=[], help="solver option key=value")
    ap.add_argument("--no-variants", action="store_true",
                    help="time only the plain FP64 solve (skip the mixed-precision variant)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the timed region, copy MIB MiB on the device three times "
                         "(the reference kernel for the HBM byte counters)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, then WRITE_SIZE) of bench.py --copy-probe, and exit")
    args = ap.parse_args()

    if args.ingest_counters:
        if args.copy_probe <= 0:
            raise SystemExit("--ingest-counters needs the --copy-probe size the runs used")
        ingest_counters(*args.ingest_counters, args.copy_probe)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solve runs on a single MI355X that owns every "
              "Fourier plane; the library has no multi-GPU path (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2609_07172_amd as P
    import workloads as W

    problem = {"paper": W.PAPER_SCALE, "batched": W.BATCHED, "small": W.SMALL}[args.workload]
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    workers = max(1, min(affinity, 16))

    cpu = None
    seq = batch = None
    if args.no_cpu:
        rho = W.blob_charge(problem, 24680)
        ref = phit = None
    else:
        rho, ref, phit, t_cpu, reps = cpu_leg(problem, workers)
        if not args.no_variants:
            seq = cpu_leg_sequence(problem, phit)
            batch = cpu_leg_batch(workers)
        cpu = {"value": t_cpu * 1e3, "unit": "ms", "cores": workers, "kind": "oracle",
               "host_cpus": os.cpu_count(), "affinity_cpus": affinity,
               "sample": f"one full {problem.nr}x{problem.ntheta}x{problem.nz} solve by the oracle's "
                         "exact separable solver (Hockney's FFT / DST-I / tridiagonal method: "
                         "scipy.fft rfft/DST-I with `cores` threads, numpy tridiagonal sweep), "
                         f"same rho; mean of {reps} repetitions.  Threads = the process's CPU "
                         "affinity capped at 16 (the box's CPU share for one GPU).  The oracle's "
                         "plain-definition sparse LU of the 3-D system does not fit this size "
                         "(about 70 min already at 129 x 64 x 129)"}

    dev = torch.device("cuda:0")
    fmg = args.start == "fmg"
    if args.tol is None:
        args.tol = START_TOL[args.start]
    tol = args.tol
    opts = {"fmg": 1} if fmg else {}
    for kv in args.option:
        k, v = kv.split("=")
        opts[k] = float(v)
    plan = P.Plan.for_problem(problem, **opts)
    info = plan.info()
    rho_d = torch.from_numpy(rho).to(dev)
    phi_d = torch.empty_like(rho_d)
    log(f"plan: levels {info['level_shapes']} workspace {info['workspace_bytes'] / 2**30:.2f} GiB")

    for _ in range(args.warmup):
        plan.solve(rho_d, tol=args.tol, phi=phi_d)
    torch.cuda.synchronize()

    # Timed region.  HIP events recorded around every finest-level pass on the
    # solve's stream give those passes' device times (the roofline figures);
    # the other launches run without events between them.
    plan.set_option("timing", 2)
    sums, launches, per = {}, {}, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        _, st = plan.solve(rho_d, tol=args.tol, phi=phi_d)
        torch.cuda.synchronize()
        per.append(time.perf_counter() - a)
        for k, v in st["kernel_ms"].items():
            sums[k] = sums.get(k, 0.0) + v
            launches[k] = launches.get(k, 0) + st["kernel_launches"][k]
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    plan.set_option("timing", 0)
    ms = total / args.steps * 1e3
    log(f"gpu: {ms:.3f} ms/solve over {args.steps} steps, cycles {st['cycles']}, "
        f"rel residual {st['rel_residual']:.3e}")
    phi = phi_d.cpu().numpy()

    # the same loop without events, for the cost of the event records themselves
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.solve(rho_d, tol=args.tol, phi=phi_d)
    torch.cuda.synchronize()
    ms_plain = (time.perf_counter() - t0) / args.steps * 1e3

    # untimed: the device time of every kernel class (events around every launch)
    plan.set_option("timing", 1)
    class_sums = {}
    for _ in range(args.steps):
        _, cst = plan.solve(rho_d, tol=args.tol, phi=phi_d)
        for k, v in cst["kernel_ms"].items():
            class_sums[k] = class_sums.get(k, 0.0) + v
    plan.set_option("timing", 0)
    torch.cuda.synchronize()

    variants = {}
    if not args.no_variants:
        # the other start at its own tolerance for rel-L2 1e-12; every other
        # variant starts from zero at that start's tolerance
        other = "zero" if fmg else "fmg"
        oargs = argparse.Namespace(**{**vars(args), "tol": START_TOL[other]})
        variants[other + "_start"] = time_variant(plan, rho_d, phi_d, oargs, ref, phit,
                                                  {"fmg": 0 if fmg else 1})
        # mixed precision from the same full-multigrid start and tolerance as
        # the headline (three FP32 V-cycles per FP64 refinement step)
        margs = argparse.Namespace(**{**vars(args), "tol": START_TOL["fmg"]})
        variants["mixed_fp32"] = time_variant(plan, rho_d, phi_d, margs, ref, phit,
                                              {"fmg": 1, "precision": 32, "inner_cycles": 3})
        plan.set_option("fmg", 0)
        args = argparse.Namespace(**{**vars(args), "tol": START_TOL["zero"]})
        variants["masks"] = time_variant(plan, rho_d, phi_d, args, ref, phit, {"masks": 1})
        variants["graph"] = time_variant(plan, rho_d, phi_d, args, ref, phit, {"graph": 1})
        variants["autotuned"] = time_autotuned(problem, rho_d, args, ref, phit)
        variants["warm_start_sequence"] = time_sequence(problem, rho_d, args, seq, phit)
        variants["batch_uneven"] = time_batch(args, batch)
        variants["learned_preconditioner"] = time_learned(problem, rho_d, args, ref, phit)
        variants["meshes"] = time_meshes(problem, args)

    if args.copy_probe > 0:
        # a plain device copy of known size: the scale for the HBM byte counters
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe} MiB x 3")

    # practical HBM peak: a plain 1 GiB device-to-device copy (reads and writes 1 GiB)
    csrc = torch.ones((1 << 30) // 8, dtype=torch.float64, device=dev)
    cdst = torch.empty_like(csrc)
    cdst.copy_(csrc)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        cdst.copy_(csrc)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * (1 << 30) * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del csrc, cdst

    b = alg_bytes(info, problem.ntheta)
    if fmg:
        # the first down pass forms the full-multigrid start from the level-1
        # answer (8 B per level-1 unknown) instead of reading an iterate
        b["down_first"] = b["down"] - 8 * b["n0"] + 8 * b["n1"]
    # algorithmic bytes per launch of each finest-level pass class: the first
    # down pass of a solve reads no iterate (or the level-1 answer after the
    # full-multigrid start), the later ones (after a check) read it
    nd = launches.get("fine_down", 0) / args.steps
    first_down = b["down_first"]
    per_launch = {"fine_up": b["up"], "fine_merged": b["merged"],
                  "fine_down": (first_down + b["down"] * max(0.0, nd - 1)) / max(nd, 1.0)}
    fine = {}
    for cls, nbytes in per_launch.items():
        if launches.get(cls, 0) == 0:
            continue
        avg = sums[cls] / launches[cls]
        gbs = nbytes / (avg * 1e-3) / 1e9
        fine[cls] = {"bytes_per_launch": nbytes, "avg_launch_ms": round(avg, 5), "launches_per_solve":
                     launches[cls] / args.steps, "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    dominant = max(fine, key=lambda k: sums[k])
    bytes_launch, avg_ms = fine[dominant]["bytes_per_launch"], fine[dominant]["avg_launch_ms"]
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    traffic = traffic_for(dominant, bytes_launch)

    unknowns = problem.unknowns
    # each merged pass moves 24 B per finest unknown less than the up and down
    # passes it replaces (u and f read once, u written once)
    merges = launches.get("fine_merged", 0) / args.steps
    dlev = info["direct_level"]
    model_bytes = (16.0 * problem.nodes + 16.0 * unknowns + cycle_bytes(dlev) * st["cycles"] * unknowns
                   + (fmg_bytes(dlev) * unknowns if fmg else 0.0) - 24.0 * merges * unknowns)
    out = {
        "metric": METRIC,
        "value": round(ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": problem.name, "nr": problem.nr, "ntheta": problem.ntheta,
                   "nz": problem.nz, "modes": problem.ntheta // 2 + 1, "unknowns": unknowns,
                   "tol": tol, "start": args.start, "rho": "blob" if args.no_cpu else "manufactured",
                   "options": opts},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "bytes_per_launch": bytes_launch,
                     "avg_launch_ms": round(avg_ms, 5)},
        "fine_passes": fine,
        "cpu_baseline": cpu,
        "cycles": st["cycles"],
        "rel_residual": st["rel_residual"],
        "ms_without_events": round(ms_plain, 4),
        "ms_min": round(min(per) * 1e3, 4),
        "ms_p50": round(float(np.median(per)) * 1e3, 4),
        # the whole solve against the algorithmic byte model: 16 B per node and per
        # unknown for the transforms, cycle_bytes per unknown and V-cycle, less 24 B
        # per unknown and merged pass, and for the full-multigrid start fmg_bytes
        # per unknown (restrict f, one V-cycle from level 1 down)
        "solve_roofline": {"model_bytes": model_bytes,
                           "t_roof_ms": round(model_bytes / (HBM_PEAK_GBS * 1e9) * 1e3, 4),
                           "frac": round(model_bytes / (HBM_PEAK_GBS * 1e9) / (ms_plain * 1e-3), 4)},
        "copy_gbs": round(copy_gbs, 1),
        "dof_cycles_per_s": unknowns * st["cycles"] / (ms * 1e-3),
        "poisson_cells_per_s": problem.nodes / (ms * 1e-3),
        "kernel_ms_per_solve": {k: round(v / args.steps, 4) for k, v in class_sums.items()},
        "kernel_launches_per_solve": {k: v / args.steps for k, v in launches.items()},
        "variants": variants,
    }
    if ref is not None:
        out.update(accuracy(phi, ref, problem, "oracle"))
        out.update(accuracy(phi, phit, problem, "phi_true"))
        # the oracle's own FP64 solve against phi_true, the scale of those errors
        out["oracle_rel_l2_vs_phi_true"] = interior_rel(ref, phit)
        # the metric's accuracy target, checked on this run's answer
        out["rel_l2_target"] = REL_L2_TARGET
        out["meets_target"] = bool(out["rel_l2_vs_oracle"] <= REL_L2_TARGET)
    print(json.dumps(out), flush=True)
    if ref is not None and not out["meets_target"]:
        log(f"rel-L2 {out['rel_l2_vs_oracle']:.3e} against the oracle misses the target {REL_L2_TARGET:.0e}")
        sys.exit(1)


if __name__ == "__main__":
    main()
