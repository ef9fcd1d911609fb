#!/usr/bin/env python3
"""Benchmark: GenEO-preconditioned CG on one MI355X.

A step is one pass of the whole path over one synthetic problem: assembly of
A and b (gn_assemble), overlapping decomposition + local factors + batched
GenEO eigensolves + coarse space and factor (gn_setup_geneo), and PCG to a
1e-8 relative residual (gn_solve).  `value` is solved DOFs per second of step
time; the solve-only rate, PCG iterations and the p50/p99 solve latency are
reported beside it.

Default workload: the largest single-GPU configuration, the 384x72x71 ramped
24-ply laminate (6,054,912 free DOFs, 1536 subdomains, 12 GenEO vectors each,
N_H = 18,432), FP64 local factors.  The SPE10-shaped 60x220x85 diffusion
(1,121,354 DOFs) is timed beside it as a secondary workload.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_workload(name):
    from workloads import generate as gen
    if name == "c2":
        return gen.config_c2()
    if name == "c1":
        return gen.config_c1()
    if name == "c3":
        return gen.config_c3()
    if name == "c5":
        return gen.config_c5()
    raise ValueError(name)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _crop_workload(config):
    """A bounded crop of the benched workload for the oracle: the same mesh
    spacing, layers or coefficient field and loads, with fewer elements and
    subdomains."""
    import numpy as np
    from workloads import generate as gen
    if config == "c2":
        w_full = gen.spe10_like()
        ne = (20, 40, 16)
        kc = w_full.elem_k.reshape(85, 220, 60)[:ne[2], :ne[1], :ne[0]]
        w = gen.diffusion_box(ne, kc.ravel(), (2, 2, 2), overlap=2, threshold=0.15, nev_max=32,
                              name="spe10_crop")
        return w, f"a {ne[0]}x{ne[1]}x{ne[2]} crop of the same field, 2x2x2 subdomains, overlap 2, threshold 0.15"
    # the ramped laminate: the clamped end (16 x 6 elements at its 0.5 mm
    # spacing), its bottom four plies and three resin layers, top pressure, 2x1x1
    # subdomains with 12 GenEO vectors each
    layers = []
    for p in range(4):
        layers.append(("ply", [0, 90, 45, -45][p % 4], 2, gen.PLY_T))
        if p != 3:
            layers.append(("resin", 0.0, 1, gen.RESIN_T))
    nx, ny = 16, 6
    w = gen.laminate_plate((nx, ny), (8.0, 3.0), layers, nparts=(2, 1, 1), overlap=1, nev=12, body=None,
                           traction=np.tile(np.array([0.0, 0.0, -0.01]), nx * ny), nrhs=1,
                           resin=gen.iso_consts(162.0, 0.35), name="ramp_laminate_crop")
    return w, ("the clamped end of the same laminate (16x6 elements at its 0.5 mm spacing, the bottom "
               "4 plies + 3 resin layers, 11 element layers), 2x1x1 subdomains, 12 GenEO vectors")


def cpu_baseline(config):
    """Oracle (as written, untuned) on a bounded sample of the benched workload,
    timed end to end (assembly + GenEO set-up + PCG to 1e-8) on the host: once
    with BLAS on every core, once on one core."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import fem, geneo, pcg
    w, what = _crop_workload(config)

    def run():
        t0 = time.perf_counter()
        Ke = fem.element_matrices(w)
        A, b, free = fem.assemble(w, Ke)
        g = geneo.GenEO(w, A, Ke)
        x, info = pcg.pcg(A, b[:, 0], g.apply, rtol=1e-8, maxit=2000)
        return time.perf_counter() - t0, info

    dt_all, info = run()
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    with threadpool_limits(limits=1):
        dt_one, _ = run()
    nproc = os.cpu_count() or 1
    return {"value": w.n_free / dt_all, "unit": "DOFs/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle end-to-end on {what} ({w.n_free} DOFs, {info['iters']} PCG its) "
                      f"in {dt_all:.1f} s with BLAS on {threads} threads",
            "single_core": {"value": w.n_free / dt_one, "seconds": dt_one, "cores": 1},
            "host": {"nproc": nproc, "cpu_model": _cpu_model()}}


TRAFFIC_SOURCE = os.path.join(ROOT, "paper_1901_05188_amd", "csrc", "local_solve.hip")


def traffic_file(workload, prec, threads):
    """Counter summary of the local-solve kernel for a workload, factor precision
    and launch shape (threads per subdomain)."""
    return os.path.join(ROOT, "profiles", f"local_solve_traffic_{workload}_fp{prec}_{threads}t.json")


def _sha256(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def summarize_counters(fetch_csv, write_csv, kernel_prefix="k_local_solve", floor_kib=1024.0):
    """Condense two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch) of the same bench command into HBM bytes per working launch of the
    local-solve kernel.  Each counter is scaled by what it reads for the last
    device-to-device copy of the run (a 1 GiB copy: 2^30 bytes read and written).
    Launches that return at once after convergence (below floor_kib) are left out."""
    import csv

    def read(path, counter):
        kern, copies = [], []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                name = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", "")
                v = float(r["Counter_Value"])
                if name.startswith(kernel_prefix) and v >= floor_kib:
                    kern.append((name.split("(")[0], v))
                if "copyBuffer" in name:
                    copies.append(v)
        if not kern or not copies:
            raise SystemExit(f"{path}: no {kernel_prefix} dispatches or no copy kernel")
        return kern, copies[-1]

    kf, cf = read(fetch_csv, "FETCH_SIZE")
    kw, cw = read(write_csv, "WRITE_SIZE")
    copy_bytes = float(1 << 30)
    fetch_scale, write_scale = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    fetch = sum(v for _, v in kf) / len(kf) * 1024.0 * fetch_scale
    write = sum(v for _, v in kw) / len(kw) * 1024.0 * write_scale
    out = {"kernel": kf[0][0], "source": os.path.relpath(TRAFFIC_SOURCE, ROOT),
           "source_sha256": _sha256(TRAFFIC_SOURCE),
           "working_dispatches": len(kf), "fetch_kib_mean": sum(v for _, v in kf) / len(kf),
           "write_kib_mean": sum(v for _, v in kw) / len(kw),
           "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_scale": fetch_scale, "write_scale": write_scale,
           "hbm_read_bytes_per_launch": fetch, "hbm_write_bytes_per_launch": write,
           "hbm_bytes_per_launch": fetch + write}
    return out


def measured_traffic(workload, prec, threads):
    """HBM bytes per working local-solve launch from the committed counter
    summary, or None if it is missing or was taken on another kernel source."""
    try:
        with open(traffic_file(workload, prec, threads)) as f:
            t = json.load(f)
        if t.get("source_sha256") != _sha256(TRAFFIC_SOURCE):
            return None
        return t
    except (OSError, ValueError):
        return None


def _run_stream(srv, ids, n_free, reqs, loads, rtol):
    """Submit requests at their arrival times; wait for all.  Returns per-request
    latencies, the columns' reports and the wall time."""
    tickets = []
    tstart = time.perf_counter()
    for i, r in enumerate(reqs):
        dt = tstart + r["t"] - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        b, x = loads[i]
        x.zero_()
        tickets.append(srv.submit(ids[r["op"]], n_free[r["op"]], b, x, rtol=rtol, maxit=5000))
    lat, reps, sts = [], [], []
    for t in tickets:
        st, rep, l = srv.wait(t)
        lat.append(l)
        reps.append(rep)
        sts.append(st)
    return lat, reps, sts, time.perf_counter() - tstart


def _stream_summary(reqs, lat, reps, sts, wall, n_free, rtol, rate):
    import numpy as np
    lat_s = sorted(lat)
    q = lambda f: lat_s[min(len(lat_s) - 1, int(round(f * (len(lat_s) - 1))))]
    cols = [c for rep in reps for c in rep]
    dofcols = sum(len(rep) * n_free[r["op"]] for r, rep in zip(reqs, reps))
    at_rtol = sum(1 for c in cols if c["true_rel_res"] <= rtol)
    at_floor = sum(1 for c in cols if c["true_rel_res"] > rtol and c["true_rel_res"] <= 4 * c["res_floor"])
    return {"requests": len(reqs), "columns": len(cols), "arrival_rate_per_s": rate,
            "arrival_span_s": reqs[-1]["t"], "wall_s": wall, "requests_per_s": len(reqs) / wall,
            "dof_rhs_per_s": dofcols / wall,
            "latency_ms": {"p50": 1000 * q(0.5), "p99": 1000 * q(0.99)},
            "pcg_iters": {"mean": float(np.mean([c["iters"] for c in cols])),
                          "max": int(max(c["iters"] for c in cols))},
            "all_converged": all(st == 0 for st in sts) and all(c["converged"] == 1 for c in cols),
            "max_true_rel_res": max(c["true_rel_res"] for c in cols),
            # true residual b - A x at rtol, or (the rest) at the FP64 rounding floor of x
            "columns_true_res_at_rtol": at_rtol, "columns_true_res_at_fp64_floor": at_floor,
            "columns_neither": len(cols) - at_rtol - at_floor}


def serving_leg(gp, n_req, rate, rtol, dev):
    """Serving: the 16-operator laminate catalogue (4 sizes 0.2-2M DOFs x 4
    random layups, FP32 local factors inside FP64 PCG), requests of 1-16
    patch-traction load cases from the Poisson stream, submitted at their
    arrival times; latency is submit to completion of the request's last
    column.  Three streams:
      overloaded   the catalogue resident, the first n_req requests at `rate`
                   (above what one GPU completes: the queue grows);
      sustainable  the same operators, requests at a rate the server keeps up
                   with (latency = service time plus little queueing);
      budgeted     the catalogue registered by description on a server whose
                   HBM budget holds about half of it: operators are built when
                   requested and their footprint fits, idle ones evicted (LRU)."""
    import numpy as np
    import torch
    from workloads import generate as gen
    cat = gen.config_c4_catalogue()
    t0 = time.perf_counter()
    ops = []
    for w in cat:
        prob = gp.Problem.from_workload(w)
        pc = gp.Preconditioner.from_workload(prob, w, local_prec=32)
        ops.append((w, prob, pc))
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    srv = gp.Server(maxit_cap=5000)
    ids = [srv.add(p, pc) for (_, p, pc) in ops]
    n_free = [p.n_free for (_, p, _) in ops]
    resident = sum(gp.resident_bytes(p, pc) for (_, p, pc) in ops)
    est = [gp.footprint(w, local_prec=32) for (w, _, _) in ops]
    # measured footprint of each operator (with the server's batched workspace)
    # against the a-priori estimate
    meas = [srv.info(i)["bytes"] for i in ids]
    log(f"serving: catalogue of {len(ops)} operators built in {t_build:.1f}s, {resident / 1e9:.1f} GB resident")
    reqs = gen.c4_requests(len(ops), n_req=n_req, rate=rate)
    loads = []
    for r in reqs:
        w, p, _ = ops[r["op"]]
        b = torch.zeros((r["k"], p.n_free), dtype=torch.float64, device=dev)
        p.load_vectors(b, traction=gen.patch_tractions(w, r["k"], np.random.default_rng(r["seed"])))
        loads.append((b, torch.zeros_like(b)))
    torch.cuda.synchronize()
    lat, reps, sts, wall = _run_stream(srv, ids, n_free, reqs, loads, rtol)
    over = _stream_summary(reqs, lat, reps, sts, wall, n_free, rtol, rate)
    # one request again, alone on an idle server: the same bits as in the mix
    i0 = max(range(len(reqs)), key=lambda i: reqs[i]["k"])
    b0, x0 = loads[i0]
    x_mix = x0.clone()
    xa = torch.zeros_like(x0)
    torch.cuda.synchronize()
    srv.wait(srv.submit(ids[reqs[i0]["op"]], n_free[reqs[i0]["op"]], b0, xa, rtol=rtol, maxit=5000))
    same = bool(torch.equal(xa, x_mix))
    # a rate the server sustains: about 60 % of the overloaded stream's throughput
    rate2 = round(0.6 * over["requests_per_s"], 2)
    n2 = min(len(reqs), 40)
    reqs2 = [dict(r, t=i / rate2) for i, r in enumerate(reqs[:n2])]
    lat2, reps2, sts2, wall2 = _run_stream(srv, ids, n_free, reqs2, loads[:n2], rtol)
    sustain = _stream_summary(reqs2, lat2, reps2, sts2, wall2, n_free, rtol, rate2)
    sustain["arrivals"] = "evenly spaced, the first requests of the stream"
    srv.close()
    # its error against FP64 local factors on the same operator
    w, p, _ = ops[reqs[i0]["op"]]
    pc64 = gp.Preconditioner.from_workload(p, w, local_prec=64)
    x64 = torch.zeros_like(x_mix)
    gp.solve(p, pc64, b0, x64, rtol=rtol, maxit=5000)
    err64 = float(torch.max(torch.linalg.norm(x_mix - x64, dim=1) / torch.linalg.norm(x64, dim=1)))
    pc64.close()
    for (_, p, pc) in ops:
        pc.close()
        p.close()
    # budgeted: operators registered by description, built on demand
    budget = int(0.5 * sum(est))
    srv = gp.Server(maxit_cap=5000, hbm_budget=budget)
    ids_b = [srv.register(w, local_prec=32)[0] for w in cat]
    n3 = min(len(reqs), 30)
    rate3 = rate2
    reqs3 = [dict(r, t=i / rate3) for i, r in enumerate(reqs[:n3])]
    lat3, reps3, sts3, wall3 = _run_stream(srv, ids_b, n_free, reqs3, loads[:n3], rtol)
    budgeted = _stream_summary(reqs3, lat3, reps3, sts3, wall3, n_free, rtol, rate3)
    infos = [srv.info(i) for i in ids_b]
    budgeted.update({"hbm_budget_GB": budget / 1e9, "catalogue_estimate_GB": sum(est) / 1e9,
                     "builds": sum(i["builds"] for i in infos), "evictions": sum(i["evictions"] for i in infos),
                     "resident_at_end": sum(1 for i in infos if i["resident"])})
    srv.close()
    del loads
    out = {"workload": "laminate catalogue 16 operators (0.2/0.5/1/2 M DOFs x 4 layups), FP32 local factors, "
                       "Poisson arrivals, 1-16 patch tractions per request",
           "overloaded": over, "sustainable": sustain, "budgeted": budgeted,
           "alone_equals_mix_bitwise": same, "rel_err_vs_fp64_local": err64,
           "catalogue_build_s": t_build, "resident_GB": resident / 1e9,
           "footprint_estimate_over_measured": {"min": min(e / m for e, m in zip(est, meas)),
                                                "max": max(e / m for e, m in zip(est, meas))}}
    log(f"serving: overloaded {over['requests']} req at {rate}/s: {over['requests_per_s']:.2f} req/s, p50 "
        f"{over['latency_ms']['p50']:.0f} ms p99 {over['latency_ms']['p99']:.0f} ms; sustainable at {rate2}/s: p50 "
        f"{sustain['latency_ms']['p50']:.0f} ms p99 {sustain['latency_ms']['p99']:.0f} ms; budgeted "
        f"{budget / 1e9:.0f} GB: {budgeted['builds']} builds, {budgeted['evictions']} evictions, p50 "
        f"{budgeted['latency_ms']['p50']:.0f} ms; alone==mix {same}; err vs FP64 {err64:.1e}")
    return out


def robustness_leg(gp, dev):
    """The paper's Example 1b comparison (one-level AS, zero-energy modes,
    GenEO) at a 1e-5 residual reduction: the Example 1 plate (30,240 DOFs)
    split into N = 4, 8, 16, 32 subdomains, and a channelled diffusion box
    (33,759 DOFs, 32 subdomains) with contrast 1 to 1e6.  Iterations,
    CG-Lanczos kappa and coarse dimension per preconditioner."""
    import torch
    from workloads import generate as gen

    def run(w):
        prob = gp.Problem.from_workload(w)
        b = torch.zeros((1, prob.n_free), dtype=torch.float64, device=dev)
        prob.rhs(b)
        row = {"n_free": prob.n_free, "subdomains": list(w.nparts)}
        for name, coarse in (("AS", 0), ("ZEM", 2), ("GenEO", 1)):
            pc = gp.Preconditioner.from_workload(prob, w, coarse=coarse)
            x = torch.zeros_like(b)
            _, rep = gp.solve(prob, pc, b, x, rtol=1e-5, maxit=5000)
            row[name] = {"iters": rep[0]["iters_first"], "kappa": round(rep[0]["cond_est"], 1),
                         "dim_VH": pc.report["coarse_dim"]}
            pc.close()
        prob.close()
        return row

    plate = {}
    for N, parts in ((4, (2, 2, 1)), (8, (8, 1, 1)), (16, (8, 2, 1)), (32, (8, 4, 1))):
        plate[str(N)] = run(gen.example1b_plate(parts))
        r = plate[str(N)]
        log(f"robustness plate N={N}: AS {r['AS']['iters']} it / kappa {r['AS']['kappa']}, "
            f"ZEM {r['ZEM']['iters']} / {r['ZEM']['kappa']} / dim {r['ZEM']['dim_VH']}, "
            f"GenEO {r['GenEO']['iters']} / {r['GenEO']['kappa']} / dim {r['GenEO']['dim_VH']}")
    contrast = {}
    for cst in (1.0, 1e2, 1e4, 1e6):
        contrast[f"{cst:g}"] = run(gen.contrast_box(cst, (4, 4, 2)))
        r = contrast[f"{cst:g}"]
        log(f"robustness contrast {cst:g}: AS {r['AS']['iters']}, ZEM {r['ZEM']['iters']}, "
            f"GenEO {r['GenEO']['iters']} (dim {r['GenEO']['dim_VH']})")
    return {"rtol": 1e-5, "example1b_plate_by_N": plate, "diffusion_32_subdomains_by_contrast": contrast}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--local-prec", type=int, default=64)
    ap.add_argument("--local-kernel", type=int, default=0,
                    help="single-column local-solve kernel: 0 = timed choice of launch shape, 3 / 4 = 512 / "
                         "1024 threads per subdomain (to take counters of the shape a timed run chose)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32-local-factor comparison leg")
    ap.add_argument("--solve-reps", type=int, default=5, help="warm solves per step for latency")
    ap.add_argument("--multi-rhs", type=int, default=16,
                    help="columns of the batched multi-RHS leg (0 = skip)")
    ap.add_argument("--serve", type=int, default=60,
                    help="requests of the serving stream to replay (0 skips the serving leg)")
    ap.add_argument("--no-robustness", action="store_true",
                    help="skip the AS / ZEM / GenEO comparison over subdomain counts and contrasts")
    ap.add_argument("--secondary", default="c2",
                    help="second workload timed end to end beside the headline ('' = none)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="mean arrivals per second")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="end with a device-to-device copy of this many GiB (a reference "
                         "kernel of known traffic for hardware-counter runs)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the local-solve HBM traffic summary of --config/--local-prec from two "
                         "counter runs and exit")
    args = ap.parse_args()
    if args.summarize_counters:
        out = summarize_counters(*args.summarize_counters)
        name = make_workload(args.config).name
        if args.local_kernel not in (3, 4):
            raise SystemExit("--summarize-counters needs --local-kernel 3 or 4: the launch shape the counter runs used")
        threads = 512 if args.local_kernel == 3 else 1024
        if not out["kernel"].endswith(f", {threads // 32}>"):
            raise SystemExit(f"counter runs used {out['kernel']}, not the {threads}-thread shape")
        path = traffic_file(name, args.local_prec, threads)
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(out))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; sharding over several GPUs is not implemented"}))
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1901_05188_amd as gp

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"generating workload {args.config}")
    w = make_workload(args.config)
    log(f"workload {w.name}: ne={w.ne} n_free={w.n_free} subdomains={w.n_sub}")

    def host_assembly(wl):
        """The problem assembled from the workload's host arrays (gn_assemble:
        host checks, upload, device assembly), before any timed step; returns it
        and the wall time of that call."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob = gp.Problem.from_workload(wl)
        torch.cuda.synchronize()
        return prob, time.perf_counter() - t0

    def step(prob, wl, keep):
        """One step with the inputs resident in HBM: assemble A and b on the
        device from them (gn_reassemble), set up, solve.  The preconditioner is
        closed at the end of the step unless keep (the last timed step keeps it
        for the warm measurements)."""
        t0 = time.perf_counter()
        prob.reassemble()
        t_re = time.perf_counter() - t0
        pc = gp.Preconditioner.from_workload(prob, wl, local_prec=args.local_prec, local_kernel=args.local_kernel)
        b = torch.zeros((prob.nrhs, prob.n_free), dtype=torch.float64, device=dev)
        prob.rhs(b)
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, rep = gp.solve(prob, pc, b, x, rtol=args.rtol, maxit=5000, check_every=16)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        report = dict(pc.report)
        report["reassembly_s"] = t_re
        if not keep:
            pc.close()
            pc = b = x = None
        return prob, pc, b, x, rep[0], report, t1 - t0, t2 - t1, t2 - t0

    log("assembly from the host arrays")
    head_prob, host_asm_s = host_assembly(w)
    log(f"  {host_asm_s:.3f}s")
    for i in range(args.warmup):
        log(f"warmup step {i}")
        out = step(head_prob, w, keep=False)
        log(f"  setup {out[6]:.3f}s solve {out[7]:.3f}s iters {out[4]['iters']}")
        del out
    torch.cuda.synchronize()
    times, setups, solves, iters, reasm = [], [], [], [], []
    last = None
    t_start = time.perf_counter()
    for i in range(args.steps):
        prob, pc, b, x, rep, report, ts, tv, tt = step(head_prob, w, keep=(i == args.steps - 1))
        reasm.append(report["reassembly_s"])
        times.append(tt)
        setups.append(ts)
        solves.append(tv)
        iters.append(rep["iters"])
        log(f"step {i}: total {tt:.3f}s setup {ts:.3f}s solve {tv:.3f}s iters {rep['iters']} "
            f"true_rel_res {rep['true_rel_res']:.2e} cond {rep['cond_est']:.1f} NH {report['coarse_dim']}")
        log("  setup report " + json.dumps(report))
        last = (prob, pc, b, x, rep)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    prob, pc, b, x, rep = last
    # warm solve latency (operator and preconditioner resident) with per-kernel events
    gp.profile_enable(True)
    lat = []
    applications = 0      # preconditioner applications that did work (one per PCG iteration)
    for r in range(args.solve_reps):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, prep = gp.solve(prob, pc, b, x, rtol=args.rtol, maxit=5000, check_every=16)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        applications += sum(c["iters"] for c in prep)
    groups = {}
    for gname in ("trsv", "spmv", "prolong", "coarse", "vec"):
        ms, n, by = gp.profile_read(gname)
        groups[gname] = {"ms_total": ms, "launches": n, "bytes": by}
    gp.profile_enable(False)
    lat_plain = []
    for r in range(args.solve_reps):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gp.solve(prob, pc, b, x, rtol=args.rtol, maxit=5000, check_every=16)
        torch.cuda.synchronize()
        lat_plain.append(time.perf_counter() - t0)
    n_dof = prob.n_free * prob.nrhs
    ms_per_step = 1000.0 * t_total / args.steps
    # Roofline of the local solves.  Launches after convergence inside the last
    # chunk of iterations see the done flag and return at once: they count as
    # launches (as in a kernel trace) that move no algorithmic bytes.
    tr = groups["trsv"]
    launches = max(tr["launches"], 1)
    tr_ms = tr["ms_total"] / launches
    bytes_per_app = tr["bytes"] / launches
    bytes_per_launch = bytes_per_app * min(applications, launches) / launches
    tr_gbs = bytes_per_launch / (tr_ms * 1e-3) / 1e9 if tr["launches"] else 0.0
    threads = pc.report["local_threads"]
    ftype = "double" if args.local_prec == 64 else "float"
    nc = 3 if w.pde == 1 else 1
    # template arguments <FT, NC, slots, G> up to the slots, which the band fixes
    instance = (f"k_local_solve_pf<{ftype}, {nc}, *, {threads // 32}>" if threads
                else "k_band_solve_mc (16-column matrix-core kernel)")
    traffic = measured_traffic(w.name, args.local_prec, threads) if threads else None
    if traffic and not (traffic["kernel"].startswith(f"k_local_solve_pf<{ftype}, {nc},")
                        and traffic["kernel"].endswith(f", {threads // 32}>")):
        traffic = None     # counters taken on another kernel
    tile_bytes = pc.report["apply_tile_bytes"]
    roof = {"bound": "hbm", "kernel": "k_local_solve (batched banded fwd+bwd triangular solves)",
            "kernel_instance": instance, "local_threads": threads,
            "achieved": round(tr_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(tr_gbs / HBM_PEAK_GBS, 4),
            # HBM bytes per working launch from the committed counter runs of this
            # kernel source and workload (null when the source changed since)
            "traffic": traffic["hbm_bytes_per_launch"] if traffic else None,
            "avg_launch_ms": round(tr_ms, 4), "launches": tr["launches"],
            "working_launches": applications,
            # algorithmic bytes: both sweeps over the factors' bands, the r gather,
            # the z write and Phi_j (the figure `achieved` divides)
            "bytes_per_working_launch": bytes_per_app,
            # the same launch over the stored whole 32x32 tiles (padding included)
            "tile_bytes_per_working_launch": tile_bytes,
            "tile_over_band": round(tile_bytes / bytes_per_app, 4) if bytes_per_app else None,
            "traffic_over_band": round(traffic["hbm_bytes_per_launch"] / bytes_per_app, 4)
            if traffic and bytes_per_app else None,
            "bytes_per_launch": bytes_per_launch}
    lat_sorted = sorted(lat_plain)
    # mixed-precision leg: the same operator with FP32 local factors inside the
    # FP64 outer PCG (warm solves), its error against the FP64 solution above
    mixed = None
    if args.local_prec == 64 and not args.no_mixed:
        pc32 = gp.Preconditioner.from_workload(prob, w, local_prec=32)
        x32 = torch.zeros_like(b)
        gp.solve(prob, pc32, b, x32, rtol=args.rtol, maxit=5000, check_every=16)   # warm
        mt = []
        for r in range(3):
            x32.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, mrep = gp.solve(prob, pc32, b, x32, rtol=args.rtol, maxit=5000, check_every=16)
            torch.cuda.synchronize()
            mt.append(time.perf_counter() - t0)
        tmix = statistics.median(mt)
        mixed = {"local_prec": 32, "solve_s": tmix, "solve_dofs_per_s": n_dof / tmix,
                 "speedup_vs_fp64_solve": statistics.median(lat_plain) / tmix,
                 "iters": mrep[0]["iters"], "true_rel_res": mrep[0]["true_rel_res"],
                 "rel_diff_vs_fp64_solution": float(torch.linalg.norm(x32 - x) / torch.linalg.norm(x)),
                 "setup_s": pc32.report["t_total_s"]}
        log(f"mixed precision: {tmix:.3f}s per solve, {mrep[0]['iters']} iters, x{mixed['speedup_vs_fp64_solve']:.2f}")
        pc32.close()
    # batched multi-RHS leg: the workload's load plus seeded random loads, all
    # columns in one batched solve (the warm operator and preconditioner)
    multi = None
    if args.multi_rhs > 1:
        k = args.multi_rhs
        gen_t = torch.Generator(device=dev)
        gen_t.manual_seed(1234)
        B = torch.randn((k, prob.n_free), dtype=torch.float64, device=dev, generator=gen_t)
        B[0].copy_(b[0])
        X = torch.zeros_like(B)
        gp.solve(prob, pc, B, X, rtol=args.rtol, maxit=5000, check_every=16)   # warm
        mt = []
        for r in range(2):
            X.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, mrep = gp.solve(prob, pc, B, X, rtol=args.rtol, maxit=5000, check_every=16)
            torch.cuda.synchronize()
            mt.append(time.perf_counter() - t0)
        tm = min(mt)
        multi = {"k": k, "solve_s": tm, "solve_dofs_per_s": prob.n_free * k / tm,
                 "speedup_vs_single": (prob.n_free * k / tm) / (n_dof / statistics.median(lat_plain)),
                 "iters": [c["iters"] for c in mrep],
                 "max_true_rel_res": max(c["true_rel_res"] for c in mrep),
                 "all_converged": all(c["converged"] == 1 for c in mrep)}
        log(f"multi-RHS k={k}: {tm:.3f}s, {multi['solve_dofs_per_s']:.3e} DOFs/s, "
            f"x{multi['speedup_vs_single']:.2f} vs one column")

    def pct(v, q):
        k = min(len(v) - 1, max(0, int(round(q * (len(v) - 1)))))
        return v[k]

    # the headline operator is released before the other legs
    head_report, head_n_free, head_nrhs = dict(pc.report), prob.n_free, prob.nrhs
    pc.close()
    prob.close()
    del pc, prob, b, x
    secondary = None
    if args.secondary:
        w2 = make_workload(args.secondary)
        log(f"secondary workload {w2.name}: n_free={w2.n_free}")
        prob2, _ = host_assembly(w2)
        step(prob2, w2, keep=False)                # warm
        t2s, its2 = [], []
        for i in range(3):
            _, _, _, _, rep2, rp2, ts2, tv2, tt2 = step(prob2, w2, keep=False)
            t2s.append(tt2)
            its2.append(rep2["iters"])
            log(f"  secondary step {i}: total {tt2:.3f}s setup {ts2:.3f}s solve {tv2:.3f}s")
        secondary = {"workload": w2.name, "n_free": w2.n_free, "local_prec": args.local_prec,
                     "value": w2.n_free / statistics.mean(t2s), "unit": "DOFs/s",
                     "ms_per_step": 1000 * statistics.mean(t2s), "steps": 3, "pcg_iters": its2[-1],
                     "setup_s_last": rp2["t_total_s"], "coarse_dim": rp2["coarse_dim"]}
        prob2.close()
    serving = serving_leg(gp, args.serve, args.serve_rate, args.rtol, dev) if args.serve > 0 else None
    robust = None if args.no_robustness else robustness_leg(gp, dev)

    res = {
        "metric": "solved DOFs/s + PCG iters to 1e-8 rel. residual; p50/p99 solve latency",
        "value": n_dof / (t_total / args.steps),
        "unit": "DOFs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.local_prec == 64 else "f64+f32-local",
        "data": "synthetic",
        "config": {"workload": w.name, "ne": list(w.ne), "n_free": head_n_free, "nrhs": head_nrhs,
                   "subdomains": list(w.nparts), "overlap": w.overlap,
                   "geneo": {"nev": w.nev, "threshold": w.threshold, "nev_max": w.nev_max},
                   "local_prec": args.local_prec, "rtol": args.rtol,
                   "parallelism": "1 GPU, all subdomains batched"},
        "pcg_iters": iters[-1],
        "solve_dofs_per_s": n_dof / statistics.median(lat_plain),
        "solve_latency_ms": {"p50": 1000 * pct(lat_sorted, 0.5), "p99": 1000 * pct(lat_sorted, 0.99)},
        "setup_s_median": statistics.median(setups),
        "step_s": {"median": statistics.median(times), "max": max(times),
                   "max_over_median": max(times) / statistics.median(times)},
        "setup_breakdown_s": {"local_factors": head_report["t_local_s"], "eigen": head_report["t_eigen_s"],
                              "coarse": head_report["t_coarse_s"], "device_alloc": head_report["t_alloc_s"]},
        # the step assembles on the device from inputs resident in HBM; the same
        # step with the assembly from the host arrays (checks, PCIe upload)
        "host_inputs": {"assembly_from_host_s": host_asm_s,
                        "reassembly_s_median": statistics.median(reasm),
                        "dofs_per_s_with_host_assembly":
                            n_dof / (statistics.mean(times) - statistics.median(reasm) + host_asm_s)},
        "coarse_dim": head_report["coarse_dim"],
        "eig_iters": head_report["eig_iters"],
        "eig_solves": head_report["eig_solves"],
        "preconditioner_bytes": head_report["hbm_bytes"],
        "cond_est": rep["cond_est"],
        "true_rel_res": rep["true_rel_res"],
        "res_floor": rep["res_floor"],
        "kernel_groups_ms_per_solve": {k: v["ms_total"] / args.solve_reps for k, v in groups.items()},
        "roofline": roof,
    }
    if secondary is not None:
        res["secondary"] = secondary
    if mixed is not None:
        res["mixed_precision"] = mixed
    if multi is not None:
        res["multi_rhs"] = multi
    if serving is not None:
        res["serving"] = serving
    if robust is not None:
        res["coarse_space_comparison"] = robust
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(args.config)
    # streaming reference on the same device: a 1 GiB device-to-device copy
    # (read + write bytes over its event-timed duration), context for the roofline
    nref = (1 << 30) // 8
    src = torch.ones(nref, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    res["hbm_copy_GBps"] = round(5 * 2 * nref * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del src, dst
    if args.copy_calibration_gib > 0:
        n = int(args.copy_calibration_gib * (1 << 30)) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {n * 8} bytes read and written")
        del src, dst
    print(json.dumps(res))


if __name__ == "__main__":
    main()
