"""Benchmark: SGF-preconditioned CG on one MI355X.

One step = one pass of the whole hot path on the resident synthetic problem:
numeric SGF factorization (every level: interior elimination, separator
compression, coarsening, exact top) followed by a CG solve of a fresh
right-hand side to 1e-8 relative residual, preconditioned by the factor.
The level-1 symbolic analysis (integer planning that depends only on the
grid) is done once before timing, as a solver reusing its analysis would;
its host time is reported beside the step.

Prints ONE JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3

WORKLOADS = {
    "varcoef2d_1024": "2D -div(a grad u), 5-point FD on a 1024^2 grid (n=1,048,576), a=exp(g), g a Gaussian "
                      "random field from 64 seeded random Fourier modes (corr. length 0.05, sigma 1), Dirichlet; "
                      "SGF Nest-All-All, q=2, leaf 16x16; rhs U[-1,1]; CG to 1e-8",
    "poisson2d_64": "2D Poisson, 5-point FD on 64^2 (n=4096), a=1; q=1, leaf 8x8; CG to 1e-10",
    "varcoef3d_128": "3D -div(a grad u), 7-point FD on 128^3 (n=2,097,152), a=10^u, u~U(-2,2) constant on 8^3 "
                     "boxes; q=1, leaf 8^3; CG to 1e-8",
    "elasticity3d_48": "3D linear elasticity, Q1 hexahedra on 48^3 nodes (n=324,864), E=1/100 with 20 random "
                       "inclusions, nu=0.3, x=0 clamped; q=1, leaf 6; CG to 1e-8",
    "serving": "request stream with Poisson arrivals at 80% of the measured capacity: operators half 2D "
               "(128^2..1024^2, Fourier field, q=2, leaf 16) and half 3D (32^3..96^3, 10^u box field, q=1, leaf 8); "
               "30% new operators (factorize + solve), 70% 1-16 rhs on operators seen before; 200 GiB HBM "
               "budget; FP32 factor / FP64 CG to 1e-8",
}

SERVE_2D = (128, 256, 512, 1024)
SERVE_3D = (32, 48, 64, 96)


def run_serving(a):
    """Serving workload: the library's request loop (sgf_server_*) fed by a
    seeded open-loop arrival process.  Coefficient fields come from a pool of
    `--pool` seeds per size (generated before the clock starts); every new
    operator is registered afresh (own analysis and factorization)."""
    import torch
    from paper_1907_03406_amd import sgf
    from sgf_inputs.problems import config_problem, random_rhs, poisson_fd, gaussian_field_fourier, blocky_log_field
    from sgf_inputs.rng import uniform
    t0 = time.perf_counter()
    pool = []
    for N in SERVE_2D:
        for k in range(a.pool):
            pool.append((poisson_fd((N, N), gaussian_field_fourier(100 + k, 2)), dict(q=2, leaf=16)))
    for N in SERVE_3D:
        for k in range(a.pool):
            pool.append((poisson_fd((N, N, N), blocky_log_field(200 + k, 3)), dict(q=1, leaf=8)))
    t_gen = time.perf_counter() - t0
    nreq = a.requests
    # seeded request stream: kind, operator pick, pool pick, nrhs (streams 3000..3004)
    u_kind = uniform(a.seed, 3000, nreq + 64)
    u_pick = uniform(a.seed, 3001, nreq + 64)
    u_pool = uniform(a.seed, 3002, nreq + 64)
    u_rhs = uniform(a.seed, 3003, nreq + 64)
    u_gap = uniform(a.seed, 3004, nreq + 64)
    dev = torch.device("cuda:0")
    rhs_cache = {}

    def rhs_for(n, k, j):
        key = (n, k)
        if key not in rhs_cache:
            rhs_cache[key] = torch.from_numpy(np.stack([random_rhs(a.seed, n, c) for c in range(16)], axis=0)).to(dev)
        return rhs_cache[key][:k]

    def stream(srv, count, offset):
        ops = []
        reqs = []
        for i in range(offset, offset + count):
            if not ops or u_kind[i] < 0.3:
                half = u_pool[i] < 0.5
                sizes = len(SERVE_2D) if half else len(SERVE_3D)
                base = 0 if half else len(SERVE_2D) * a.pool
                pidx = base + int(u_pool[i] * 2 % 1.0 * sizes * a.pool) % (sizes * a.pool)
                reqs.append(("new", pidx))
                ops.append(pidx)
            else:
                reqs.append(("old", int(u_pick[i] * len(ops)) % len(ops)))
            reqs[-1] += (1 + int(u_rhs[i] * 16) % 16,)
        return reqs

    def run(srv, reqs, rate):
        ids, opsrc = [], []
        pending = []
        t_start = time.monotonic()
        t_next = t_start
        for i, (kind, ref, k) in enumerate(reqs):
            if rate:
                t_next += -np.log(max(1.0 - u_gap[i], 1e-12)) / rate
                d = t_next - time.monotonic()
                if d > 0:
                    time.sleep(d)
            arrival = time.monotonic()
            if kind == "new":
                prob, kw = pool[ref]
                ids.append(srv.add_operator(prob, precision=sgf.FP32, **kw))
                opsrc.append(prob)
                op = ids[-1]
                prob_n = prob.n
            else:
                op = ids[ref]
                prob_n = opsrc[ref].n
            b = rhs_for(prob_n, k, i)
            x = torch.zeros_like(b)
            pending.append((srv.submit(op, b, x, rtol=1e-8, maxit=2000), arrival, k, x))
        out = []
        for t, arrival, k, x in pending:
            inf = srv.wait(t)
            out.append((inf, arrival, k))
        t_end = time.monotonic()
        return out, t_start, t_end

    srv = sgf.Server(hbm_budget=200 << 30, slots=a.slots, max_batch_rhs=16)
    # capacity: a closed batch submitted at once (all requests queued together)
    cal = stream(srv, a.calibration, nreq)
    res, ts, te = run(srv, cal, None)
    cap_req_s = len(cal) / (te - ts)
    rate = 0.8 * cap_req_s
    srv.close()
    srv = sgf.Server(hbm_budget=200 << 30, slots=a.slots, max_batch_rhs=16)
    reqs = stream(srv, nreq, 0)
    res, ts, te = run(srv, reqs, rate)
    st = srv.stats()
    srv.close()
    bad = [inf for inf, _, _ in res if inf["status"] != 0 or inf["relres_max"] >= 1e-8]
    lat = np.array([(inf["t_end"] - arrival) * 1e3 for inf, arrival, _ in res])
    solves = sum(k for _, _, k in res)
    makespan = te - ts
    # kernel roofline of the serving work: the server's handles are internal,
    # so a profiled pass after the stream runs one request of the most common
    # shape (a 512^2 operator of the 2D pool: factorization + 8-rhs PCG), every
    # launch timed, the apply launched directly
    rl = None
    if not a.no_serving_roofline:
        prob, kw = pool[2 * a.pool]   # 512^2, first field
        s = sgf.Solver.from_problem(prob, precision=sgf.FP32, **kw)
        vals = torch.from_numpy(prob.data).to(dev)
        b = rhs_for(prob.n, 8, 0)
        x = torch.zeros_like(b)
        s.factorize(vals)
        s.pcg(b.T, x.T, rtol=1e-8, maxit=2000)
        s.set_apply_graph(False)
        torch.cuda.synchronize()
        s.profile(True)
        for _ in range(3):
            x.zero_()
            s.factorize(vals)
            s.pcg(b.T, x.T, rtol=1e-8, maxit=2000)
        torch.cuda.synchronize()
        stt = s.profile_read()
        s.profile(False)
        s.close()
        rl = roofline({k: v for k, v in stt.items() if "@" not in k}, {k: v for k, v in stt.items() if "@" in k},
                      "fp32", 3)
        if rl is not None:
            gpu_ms = sum(v["ms"] for k, v in stt.items() if "@" not in k)
            kms = stt.get(rl["kernel"], {"ms": 0})["ms"]
            rl["share_of_gpu_time"] = round(kms / gpu_ms, 3) if gpu_ms else None
            rl["timed_in"] = ("a profiled pass after the stream: three requests of a 512^2 operator of the 2D pool "
                              "(factorization + 8-rhs PCG to 1e-8), every launch timed, apply launched directly")
    cpu = None if a.no_cpu_baseline else cpu_baseline_serving(pool, a, res, reqs)
    out = {
        "metric": "PCG solves/s (serving: factorize/solve request stream, each rhs to 1e-8 relative residual)",
        "value": round(solves / makespan, 3),
        "unit": "solves/s",
        "n_gpus": 1, "steps": nreq, "warmup": a.calibration,
        "ms_per_step": round(makespan / nreq * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serving: {WORKLOADS['serving']}", "requests": nreq, "slots": a.slots,
                   "pool_fields_per_size": a.pool, "seed": a.seed,
                   "step": "one request (arrival to completion); value = right-hand sides solved / makespan"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2), "p99": round(float(np.percentile(lat, 99)), 2),
                       "mean": round(float(lat.mean()), 2)},
        "arrival_rate_req_s": round(rate, 3), "capacity_req_s": round(cap_req_s, 3),
        "requests_failed": len(bad),
        "new_operators": sum(1 for r in reqs if r[0] == "new"),
        "mean_batch_rhs": round(float(np.mean([inf["batch_rhs"] for inf, _, _ in res])), 2),
        "server": st, "problem_gen_s": round(t_gen, 1),
        "roofline": rl, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)



def mark_kernel(torch):
    """One tiny fill kernel of 16-bit integers (no other kernel of the run
    fills that type) before and after the timed steps, so that a kernel
    trace of the run can be cut to exactly the timed steps
    (--summarize-trace); synchronized, outside the timed region."""
    torch.full((4099,), 7, dtype=torch.int16, device="cuda")
    torch.cuda.synchronize()


def summarize_trace(trace_dir, label, command):
    """Per-kernel summary of the timed steps from a rocprofv3 kernel trace
    (CSV) of `bench.py`: the dispatches between the two marker fills."""
    import csv
    import glob
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *kernel_trace.csv under {trace_dir}")
    rows = []
    for f in files:
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    marks = [i for i, r in enumerate(rows) if "FillFunctor<short>" in r["Kernel_Name"]]
    if len(marks) < 2:
        raise SystemExit(f"markers not found ({len(marks)})")
    a, b = marks[0], marks[1]
    sel = rows[a + 1:b]
    t0, t1 = int(rows[a]["End_Timestamp"]), int(rows[b]["Start_Timestamp"])
    stats = {}
    for r in sel:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        k = stats.setdefault(r["Kernel_Name"], [0, 0.0, 0])
        k[0] += 1
        k[1] += d
    tot = sum(v[1] for v in stats.values())
    print(f"# {label}")
    print(f"# command: {command}")
    print(f"# the timed steps only: dispatches between the two marker fills of bench.py "
          f"({len(sel)} dispatches over {(t1 - t0) / 1e6:.2f} ms of wall time)")
    print("# durations in microseconds; pct of the summed kernel time")
    print(f"{'kernel':70s} {'calls':>6s} {'total_us':>10s} {'avg_us':>9s} {'pct':>6s}")
    for name, (n, us, g) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
        nm = name if len(name) <= 70 else name[:67] + "..."
        print(f"{nm:70s} {n:6d} {us:10.1f} {us / n:9.2f} {100 * us / tot:6.2f}")
    print(f"# summed kernel time {tot:.1f} us")


def summarize_pmc(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, kernels, label, commands, out_json):
    """HBM bytes per launch of one launch class from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of this script, scaled by
    what the same counters read for a device copy of 1 GiB
    (--copy-calibration runs); `kernels` are the HIP kernel name prefixes of
    the class.  Writes the record beside the summary into `out_json`."""
    import csv
    import glob

    def per_kernel(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                rows += [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
        acc = {}
        for r in rows:
            k = acc.setdefault(r["Kernel_Name"], [0, 0.0, r.get("Grid_Size", "")])
            k[0] += 1
            k[1] += float(r["Counter_Value"])
        return acc

    def copy_kib(d, counter):
        acc = per_kernel(d, counter)
        vals = [v[1] / v[0] for k, v in acc.items() if "copy" in k.lower()]
        if not vals:
            raise SystemExit(f"no copy kernel in the calibration run {d}")
        return max(vals)

    gib_kib = 1024.0 * 1024.0
    f_scale = gib_kib / copy_kib(cal_fetch_dir, "FETCH_SIZE")
    w_scale = gib_kib / copy_kib(cal_write_dir, "WRITE_SIZE")
    fk, wk = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    sel = [k for k in fk if any(k.startswith(p) for p in kernels)]
    if not sel:
        raise SystemExit(f"no kernel named {kernels}")
    fetch = sum(fk[k][1] / fk[k][0] for k in sel) * 1024 * f_scale
    write = sum(wk[k][1] / wk[k][0] for k in sel if k in wk) * 1024 * w_scale
    print(f"# {label}")
    for c in commands:
        print(f"#   {c}")
    print(f"# calibration: a 1 GiB device copy reads FETCH_SIZE {gib_kib / f_scale:.1f} KiB and WRITE_SIZE "
          f"{gib_kib / w_scale:.1f} KiB per dispatch, so bytes = FETCH_SIZE * 1024 * {f_scale:.4f} + "
          f"WRITE_SIZE * 1024 * {w_scale:.4f}")
    print("# kernels of the launch class (summed per launch):")
    for k in sel:
        print(f"#   {k}: {fk[k][0]} dispatch(es), FETCH_SIZE {fk[k][1] / fk[k][0]:.0f} KiB, "
              f"WRITE_SIZE {wk.get(k, [1, 0.0])[1] / wk.get(k, [1, 0.0])[0]:.0f} KiB")
    print(f"fetch_bytes_per_launch {fetch:.0f}")
    print(f"write_bytes_per_launch {write:.0f}")
    print(f"total_bytes_per_launch {fetch + write:.0f}")
    print()
    print("# every kernel of the counter runs, MB per dispatch (raw counters x 1024):")
    print(f"{'kernel':60s} {'launches':>8s} {'fetch_MB':>10s} {'write_MB':>10s}")
    for k, (n, v, g) in sorted(fk.items(), key=lambda kv: -kv[1][1]):
        w = wk.get(k, [1, 0.0, ""])
        nm = k if len(k) <= 60 else k[:57] + "..."
        print(f"{nm:60s} {n:8d} {v / n * 1024 / 1e6:10.2f} {w[1] / w[0] * 1024 / 1e6:10.2f}")
    return fetch + write


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1907_03406_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    rec = t.get(kernel)
    if not rec or rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def run_form(probs, cfg, precision, steps, warmup, profile, seed=0, log=None, tiled_min_rows=-1, autotune=True,
             graph=True):
    """Steps alternate between the operators in `probs` (same grid and
    pattern, different coefficient fields), all resident on the device.
    Before the steps (untimed, like the analysis): one factorization + solve
    to learn the iteration count, then the autotuner picks each level's
    elimination path weighted by the applies one solve makes."""
    import torch
    from paper_1907_03406_amd import sgf
    dev = torch.device("cuda:0")
    prob = probs[0]
    t0 = time.perf_counter()
    s = sgf.Solver.from_problem(prob, q=cfg["q"], leaf=cfg["leaf"],
                                precision={"fp32": sgf.FP32, "fp32_bf16n": sgf.FP32_BF16N, "fp64": sgf.FP64}[precision],
                                tiled_min_rows=tiled_min_rows)
    t_an = time.perf_counter() - t0
    s.set_apply_graph(graph)
    vals_all = [torch.from_numpy(p.data).to(dev) for p in probs]
    from sgf_inputs.problems import random_rhs
    nrhs = cfg.get("nrhs", 1)
    rhs = [torch.from_numpy(np.ascontiguousarray(
        np.stack([random_rhs(seed, prob.n, j * nrhs + c) for c in range(nrhs)], axis=0))).to(dev)
        for j in range(steps + warmup)]
    x = torch.zeros(nrhs, prob.n, dtype=torch.float64, device=dev)
    tol = cfg["tol"]
    modes, t_tune = None, 0.0
    if autotune:
        t0 = time.perf_counter()
        s.factorize(vals_all[0])
        it0, _ = s.pcg(rhs[0].T, x.T, rtol=tol, maxit=1000)
        modes = s.autotune(vals_all[0], napply=(int(it0.max()) + 1) * nrhs).tolist()
        x.zero_()
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t0
        if log:
            print(f"[bench] {precision} autotune: modes per level {modes} ({t_tune:.1f} s)", file=sys.stderr,
                  flush=True)
    # Kernel timing: every launch is bracketed by events during the warmup
    # steps, which launch the apply kernels directly (not as the captured
    # graph) so that each kernel class of the apply is timed too: the
    # per-kernel table.  The timed steps bracket only the launches of the
    # roofline launch class picked from them, so that the events of the other
    # launches do not slow the measured steps; when that class runs inside
    # the captured apply graph (not visible to events), its launches are
    # timed in a kernel pass of as many steps right after the timed ones,
    # with the apply launched directly.
    its, lat, fac = [], [], []
    warm = {}
    rl0 = None
    for j in range(warmup + steps):
        if profile and j == 0 and warmup > 0:
            torch.cuda.synchronize()
            s.set_apply_graph(False)
            s.profile(True)
        if j == warmup:
            torch.cuda.synchronize()
            if profile:
                s.set_apply_graph(graph)
                if warmup > 0:
                    warm = s.profile_read()
                    s.profile(False)
                    rl0 = roofline({k: v for k, v in warm.items() if "@" not in k},
                                   {k: v for k, v in warm.items() if "@" in k}, precision, warmup)
                    if rl0 is not None:
                        s.profile_select(rl0["kernel"].split("@")[0])
                s.profile(True)
            mark_kernel(torch)   # trace marker: the timed steps start
            t_start = time.perf_counter()
        ts = time.perf_counter()
        s.factorize(vals_all[j % len(vals_all)])
        tf = time.perf_counter()
        it, rel = s.pcg(rhs[j].T, x.T, rtol=tol, maxit=1000)
        te = time.perf_counter()
        if j >= warmup:
            lat.append(te - ts)
            fac.append(tf - ts)
            its.append(int(it.max()))
        if log:
            print(f"[bench] {precision} step {j} factor {1e3 * (tf - ts):.1f} ms solve {1e3 * (te - tf):.1f} ms "
                  f"it {it.tolist()}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    mark_kernel(torch)   # trace marker: the timed steps ended
    raw = s.profile_read() if profile else {}
    kernel_pass = None
    if profile and graph and rl0 is not None and rl0["kernel"].startswith("apply_"):
        # the roofline class runs inside the apply graph: time it in a pass of
        # the same steps with the apply launched directly
        s.profile(False)
        s.set_apply_graph(False)
        s.profile(True)
        t0 = time.perf_counter()
        for j in range(warmup, warmup + steps):
            s.factorize(vals_all[j % len(vals_all)])
            s.pcg(rhs[j].T, x.T, rtol=tol, maxit=1000)
        torch.cuda.synchronize()
        kernel_pass = {"steps": steps, "ms_per_step": round((time.perf_counter() - t0) / steps * 1e3, 3)}
        raw = s.profile_read()
        s.set_apply_graph(graph)
    if profile:
        s.profile(False)
        s.profile_select(None)
    table = warm if warm else raw
    stats = {k: v for k, v in table.items() if "@" not in k}
    by_level = {k: v for k, v in table.items() if "@" in k}
    timed_stats = {k: v for k, v in raw.items() if "@" not in k}
    timed_by_level = {k: v for k, v in raw.items() if "@" in k}
    prof_steps = warmup if warm else steps
    info = s.info()
    # true residual of the last solve
    A = probs[(warmup + steps - 1) % len(probs)].csr()
    xb = x.cpu().numpy()
    bb = rhs[-1].cpu().numpy()
    true_rel = max(np.linalg.norm(bb[c] - A @ xb[c]) / np.linalg.norm(bb[c]) for c in range(nrhs))
    s.close()
    return dict(total=total, lat=lat, fac=fac, its=its, info=info, stats=stats, analyze_s=t_an,
                true_rel=true_rel, nrhs=nrhs, by_level=by_level, modes=modes, tune_s=t_tune,
                timed_stats=timed_stats, timed_by_level=timed_by_level, prof_steps=prof_steps, kernel_pass=kernel_pass)


def roofline(stats, by_level, precision, steps):
    """Roofline of the dominant kernel launch class: the largest event time
    among one kernel at one level ("kernel@L<t>": factorization and apply
    kernels) and the CG kernels.  The class is picked from the warmup steps
    (every launch timed, the apply launched directly); the figures come from
    its launches in the timed steps (only that class timed there), or from
    the kernel pass when the class runs inside the captured apply graph."""
    cand = dict(by_level)
    cand.update({k: v for k, v in stats.items() if k.startswith("cg_")})
    cand = {k: v for k, v in cand.items() if "graph" not in k and v["ms"] > 0}
    if not cand:
        return None
    name, k = max(cand.items(), key=lambda kv: kv[1]["ms"])
    per = k["ms"] / max(k["launches"], 1)
    peak_f = FP64_PEAK_TFLOPS if precision == "fp64" else FP32_PEAK_TFLOPS
    # a kernel with both algorithmic flops and bytes is bound by whichever
    # roof is lower at its arithmetic intensity (ridge = peak flops / HBM peak)
    if k["flops"] > 0 and k["bytes"] > 0 and k["flops"] / k["bytes"] < peak_f * 1e12 / (HBM_PEAK_GBS * 1e9):
        ach = k["bytes"] / (k["ms"] * 1e-3) / 1e9
        return {"kernel": name, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_for(name),
                "intensity_flop_per_byte": round(k["flops"] / k["bytes"], 2),
                "flops_tflops": round(k["flops"] / (k["ms"] * 1e-3) / 1e12, 3),
                "avg_launch_ms": round(per, 4), "launches": k["launches"], "share_of_gpu_time": None}
    if k["flops"] > 0:
        # the elimination kernels' flops are dense contractions on the matrix
        # cores (FP32 / FP64 MFMA peaks equal the vector peaks on this chip)
        peak = FP64_PEAK_TFLOPS if precision == "fp64" else FP32_PEAK_TFLOPS
        ach = k["flops"] / (k["ms"] * 1e-3) / 1e12
        bound = "mfma" if name.startswith(("elim", "top", "comp_update")) else "alu"
        return {"kernel": name, "bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 4), "traffic": traffic_for(name),
                "avg_launch_ms": round(per, 4), "launches": k["launches"], "share_of_gpu_time": None}
    ach = k["bytes"] / (k["ms"] * 1e-3) / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_for(name),
            "avg_launch_ms": round(per, 4), "launches": k["launches"], "share_of_gpu_time": None}


def host_description():
    """Host cores, CPU model and the BLAS behind NumPy."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [f"{i.get('internal_api')} {i.get('version')} ({i.get('num_threads')} threads)"
                for i in threadpool_info() if i.get("user_api") == "blas"]
    except Exception:
        blas = []
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"nproc": usable, "cpu_model": model, "blas": blas or ["unknown"]}


def cpu_baseline(key, seed, sample_grid):
    """The oracle (FP64 NumPy) on a bounded sample of the workload, scaled to
    the full problem by the unknown count (the method is O(n)): one
    factorization and a CG solve of each of the configuration's right-hand
    sides (every one counts as a solve, as on the GPU), once on one thread
    (as the paper's sequential runs) and once with every host core available
    to the BLAS.  `value` is the faster of the two; both are reported."""
    from threadpoolctl import threadpool_limits
    from oracle import sgf_oracle as O
    from sgf_inputs.problems import config_problem, random_rhs
    from sgf_inputs.problems import CONFIGS
    p, cfg = config_problem(key, seed=seed, grid=sample_grid)
    c = CONFIGS[key]
    n_full = int(np.prod(c["grid"])) if "grid" in c else 3 * (c["nodes"] - 1) * c["nodes"] ** 2
    nrhs = int(c.get("nrhs", 1))
    host = host_description()
    legs = {}
    for threads in (1, host["nproc"]):
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            F = O.factorize(p.csr(), p.coords, p.grid, p.dpn, O.Options(q=cfg["q"], leaf=cfg["leaf"]))
            t1 = time.perf_counter()
            its = []
            for j in range(nrhs):
                x, it, rel = O.pcg(p.csr(), random_rhs(seed + j, p.n), lambda r: O.apply_inverse(F, r),
                                   tol=cfg["tol"])
                its.append(int(it))
            t2 = time.perf_counter()
        legs[threads] = {"value": round(n_full and nrhs / ((t2 - t0) * n_full / p.n), 6), "cores": threads,
                         "factorize_s": round(t1 - t0, 2), "cg_s": round(t2 - t1, 2), "it": max(its)}
    best = max(legs.values(), key=lambda v: v["value"])
    return {"value": best["value"], "unit": "solves/s", "cores": best["cores"], "kind": "oracle",
            "sample": f"{key} at " + (f"{sample_grid} nodes per side" if isinstance(sample_grid, int)
                                      else f"grid {tuple(sample_grid)}")
                      + f" (n={p.n}), FP64 NumPy, factorize + CG of {nrhs} right-hand side(s) "
                      f"(at most {legs[1]['it']} it); scaled by n_full/n_sample = {n_full / p.n:.0f}",
            "single_thread": legs[1], "all_cores": legs[host["nproc"]], "host": host}


def cpu_baseline_serving(pool, a, res, reqs):
    """The oracle on a bounded sample of the request mix: a new-operator
    request (factorization + one solve) on the smallest 2D and the smallest 3D
    operator of the pool, timed on one thread; the stream's total oracle time
    is estimated by scaling each request's factorization and solves by its
    operator's unknown count (the method is O(n)) and weighting the
    right-hand sides it carries."""
    from threadpoolctl import threadpool_limits
    from oracle import sgf_oracle as O
    from sgf_inputs.problems import random_rhs
    per_n = {}
    detail = []
    for idx, tag in ((0, "2D"), (len(SERVE_2D) * a.pool, "3D")):
        prob, kw = pool[idx]
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            F = O.factorize(prob.csr(), prob.coords, prob.grid, prob.dpn, O.Options(q=kw["q"], leaf=kw["leaf"]))
            t1 = time.perf_counter()
            x, it, rel = O.pcg(prob.csr(), random_rhs(a.seed, prob.n), lambda r: O.apply_inverse(F, r), tol=1e-8)
            t2 = time.perf_counter()
        per_n[tag] = ((t1 - t0) / prob.n, (t2 - t1) / prob.n)
        detail.append(f"{tag} n={prob.n}: factorize {t1 - t0:.2f} s, solve {t2 - t1:.2f} s ({it} it)")
    total, solves = 0.0, 0
    ops = []
    for (kind, ref, k) in reqs:
        if kind == "new":
            ops.append(ref)
            prob = pool[ref][0]
        else:
            prob = pool[ops[ref]][0]
        tag = "2D" if prob.dim == 2 else "3D"
        fac, sol = per_n[tag]
        total += (fac if kind == "new" else 0.0) * prob.n + k * sol * prob.n
        solves += k
    return {"value": round(solves / total, 6), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": "one new-operator request (factorize + one solve to 1e-8) on the smallest 2D and 3D operator "
                      "of the pool, FP64 NumPy, one thread (" + "; ".join(detail) + "), scaled per request by n "
                      "(factorization for new operators, one solve per right-hand side) over the timed stream"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="varcoef2d_1024", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp32_bf16n", "fp64"])
    ap.add_argument("--no-fp64-form", action="store_true", help="skip the plain FP64 comparison form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--operators", type=int, default=2,
                    help="distinct coefficient fields (seeds seed, seed+1, ...) that the steps cycle through")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--tiled-min-rows", type=int, default=-1,
                    help="levels with fronts of at least this many rows use the tiled elimination (-1: built-in)")
    ap.add_argument("--no-autotune", action="store_true", help="skip the per-level path autotuner")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch the apply kernels directly (per-kernel apply timings) instead of the captured graph")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="print the timed steps' per-kernel summary of a rocprofv3 kernel trace (CSV) of this script")
    ap.add_argument("--label", default="", help="with --summarize-trace / --summarize-pmc: title line")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR", "CAL_WRITE_DIR"),
                    help="HBM bytes per launch of --pmc-class from rocprofv3 FETCH_SIZE / WRITE_SIZE runs")
    ap.add_argument("--pmc-class", default="", help="with --summarize-pmc: launch class (e.g. apply_lsi_bwd@L1)")
    ap.add_argument("--pmc-kernels", default="", help="with --summarize-pmc: HIP kernel name prefixes separated by ';' (template arguments hold commas)")
    ap.add_argument("--command", default="", help="with --summarize-trace: the command that made the trace")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device-to-device copy of 1 GiB (reference for HBM byte counters)")
    ap.add_argument("--requests", type=int, default=300, help="serving: requests in the timed stream")
    ap.add_argument("--calibration", type=int, default=40, help="serving: closed-batch requests to measure capacity")
    ap.add_argument("--slots", type=int, default=4, help="serving: concurrent requests on the device")
    ap.add_argument("--pool", type=int, default=2, help="serving: coefficient fields per operator size")
    ap.add_argument("--no-serving-roofline", action="store_true", help="serving: skip the profiled roofline pass")
    a = ap.parse_args()
    if a.summarize_trace:
        summarize_trace(a.summarize_trace, a.label, a.command)
        return
    if a.summarize_pmc:
        import io
        from contextlib import redirect_stdout
        buf = io.StringIO()
        with redirect_stdout(buf):
            total = summarize_pmc(*a.summarize_pmc, a.pmc_kernels.split(";"), a.label, a.command.split(" ;; "),
                                  None)
        text = buf.getvalue()
        print(text, end="")
        name = a.pmc_class.replace("@", "_at_")
        summary = f"profiles/varcoef2d_1024_fp32_{name}_hbm_counters.txt"
        open(os.path.join(ROOT, summary), "w").write(text)
        path = os.path.join(ROOT, "profiles", "traffic.json")
        t = json.load(open(path)) if os.path.exists(path) else {}
        t[a.pmc_class] = {"bytes_per_launch": int(total), "hip_kernels": a.pmc_kernels.split(";"),
                          "source_hash": source_hash(), "summary": summary}
        json.dump(t, open(path, "w"), indent=1)
        return
    if a.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 4, "launches": 3}))
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 (the multi-GPU sharding "
                                   "of the factor is a design note, not implemented)"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if a.config == "serving":
        run_serving(a)
        return
    from sgf_inputs.problems import config_problem
    t0 = time.perf_counter()
    probs = [config_problem(a.config, seed=a.seed + i)[0] for i in range(a.operators)]
    cfg = config_problem.__globals__["CONFIGS"][a.config]
    prob = probs[0]
    t_gen = time.perf_counter() - t0
    main_form = run_form(probs, cfg, a.precision, a.steps, a.warmup, profile=True, seed=a.seed, log=a.verbose,
                         tiled_min_rows=a.tiled_min_rows, autotune=not a.no_autotune, graph=not a.no_graph)
    other = None
    if not a.no_fp64_form and a.precision != "fp64":
        other = run_form(probs, cfg, "fp64", max(2, a.steps // 2), 1, profile=False, seed=a.seed, log=a.verbose,
                         tiled_min_rows=a.tiled_min_rows, autotune=not a.no_autotune)
    lat = np.array(main_form["lat"]) * 1e3
    steps = a.steps
    ms = main_form["total"] / steps * 1e3
    st = main_form["stats"]              # every launch timed, over main_form["prof_steps"] steps
    psteps = main_form["prof_steps"]
    gpu_ms = sum(v["ms"] for v in st.values())
    apply_ms = sum(v["ms"] for k, v in st.items() if k.startswith("apply_"))
    apply_bytes = sum(v["bytes"] for k, v in st.items() if k.startswith("apply_"))
    elim = st.get("elim", {"ms": 0, "flops": 0})
    fac_flops = main_form["info"]["factor_flops"]
    fac_ms = float(np.mean(main_form["fac"])) * 1e3
    # the roofline class as timed inside the timed steps
    rl = roofline(main_form["timed_stats"], main_form["timed_by_level"], a.precision, steps)
    if rl is not None:
        kms = main_form["timed_by_level"].get(rl["kernel"], main_form["timed_stats"].get(rl["kernel"], {"ms": 0}))["ms"]
        rl["share_of_gpu_time"] = round((kms / steps) / (gpu_ms / psteps), 3) if gpu_ms else None
        rl["timed_in"] = ("a kernel pass of the same steps right after the timed ones, apply launched directly "
                          f"({main_form['kernel_pass']['ms_per_step']} ms per step)" if main_form["kernel_pass"]
                          else "the timed steps")
    out = {
        "metric": "PCG solves/s (numeric SGF factorization + CG solve to 1e-8 relative residual per solve)",
        "value": round(main_form["nrhs"] * 1e3 / ms, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{a.config}: {WORKLOADS[a.config]}",
            "n": prob.n, "nnz": prob.nnz, "q": cfg["q"], "leaf": cfg["leaf"], "tol": cfg["tol"],
            "factor_apply_dtype": {"fp32": "f32", "fp32_bf16n": "f32 (N from bf16 operands)", "fp64": "f64"}[a.precision],
            "cg_dtype": "f64",
            "nrhs": main_form["nrhs"], "seed": a.seed, "operators": a.operators,
            "step": "numeric factorization of operator (step mod operators) + CG solve of nrhs fresh right-hand "
                    "sides (one batched PCG); value counts every right-hand side as a solve",
        },
        "tuning": {"modes_per_level": main_form["modes"], "autotune_s": round(main_form["tune_s"], 2),
                   "legend": "0 tiled multi-workgroup elimination, 1 banded fronts one wavefront each, 8/16/32 one workgroup per front with that "
                             "panel width, -1 no interiors (top)"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3)},
        "it_C": main_form["its"],
        "true_rel_residual": float(main_form["true_rel"]),
        "factor_ms": round(fac_ms, 3),
        "factor_tflops": round(fac_flops / (fac_ms * 1e-3) / 1e12, 4),
        "elim_kernel_tflops": round(elim["flops"] / (elim["ms"] * 1e-3) / 1e12, 4) if elim["ms"] else None,
        "apply_gbs": round(apply_bytes / (apply_ms * 1e-3) / 1e9, 1) if apply_ms else None,
        "pcg_iteration_gbs": (round(st["pcg_iteration_graph"]["bytes"] / (st["pcg_iteration_graph"]["ms"] * 1e-3) / 1e9, 1)
                              if st.get("pcg_iteration_graph", {}).get("ms") else None),
        "pcg_only_solves_per_s": round(1e3 / (ms - fac_ms), 3) if ms > fac_ms else None,
        "gpu_kernel_ms_per_step": round(gpu_ms / psteps, 3),
        "kernel_times_from": ("the warmup steps, every launch timed; the timed steps time only the roofline "
                              "launch class" if psteps != steps else "the timed steps, every launch timed"),
        "levels": main_form["info"]["levels"], "top_size": main_form["info"]["top_size"],
        "factor_bytes": main_form["info"]["factor_bytes"],
        "analyze_s": round(main_form["analyze_s"], 3), "problem_gen_s": round(t_gen, 2),
        "kernels": {k: {"ms_per_step": round(v["ms"] / psteps, 4), "launches_per_step": round(v["launches"] / psteps, 1)}
                    for k, v in sorted(st.items(), key=lambda kv: -kv[1]["ms"])},
        "factor_kernels_by_level_ms_per_step": {k: round(v["ms"] / psteps, 4) for k, v in
                                                 sorted(main_form["by_level"].items(), key=lambda kv: -kv[1]["ms"])
                                                 if v["ms"] / psteps > 0.02},
        "roofline": rl,
    }
    if other is not None:
        oms = other["total"] / len(other["lat"]) * 1e3
        out["fp64_form"] = {"value": round(main_form["nrhs"] * 1e3 / oms, 4), "ms_per_step": round(oms, 3),
                            "it_C": other["its"], "modes_per_level": other["modes"],
                            "factor_ms": round(float(np.mean(other["fac"])) * 1e3, 3),
                            "speedup_of_main_form": round(oms / ms, 3)}
    if not a.no_cpu_baseline:
        sample = {"varcoef2d_1024": (512, 512), "poisson2d_64": (64, 64), "varcoef3d_128": (48, 48, 48),
                  "elasticity3d_48": 16}[a.config]
        out["cpu_baseline"] = cpu_baseline(a.config, a.seed, sample)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
