#!/usr/bin/env python
"""Benchmark of the implicit reaction-diffusion step on one MI355X.

Headline workload: 2-D Allen-Cahn u_t = eps^2 Lap u + u - u^3 on the periodic unit
square, 2048 x 2048 grid, eps = 0.01, backward Euler h_t = 1e-3, 200 steps,
u0 ~ Uniform[-0.1, 0.1] (seed 1), stop at ||F/h_t||_2 <= 1e-6.  The same
trajectory is run in plain FP64 and in the FP32-mixed precision (FP32 inner
PDHG, FP64 residual / update passes).  A step is one rd_step call: the whole
PDHG solve of one implicit time step, inputs already resident in HBM.

Prints ONE JSON line: throughput in grid-point-iterations/s (grid points x PDHG
iterations per second; mixed: FP32 inner iterations), p50/p99 step latency for
both precisions, the PDHG iteration against the HBM roofline (algorithmic bytes
per grid-point-iteration over the iteration's summed kernel durations, HIP events
on the launch stream), the other configurations (64^2 Allen-Cahn, 512^2 Neumann
Cahn-Hilliard, 1024^2 Schnakenberg) with their error against the oracle, the
serving stream, and the CPU oracle timed on bounded samples.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PDHG grid-point-iters/s + p50/p99 step latency, FP32-mixed vs FP64 at 1e-5"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per grid-point-iteration of the whole PDHG iteration, one
# component: the state read and written once (U, P read + write, U^k read; mixed:
# e, P, r, U_b read, e, P written) plus one spectral round trip per transform
# direction (the row pass writes the spectrum, the column pass reads and writes it,
# the inverse row pass reads it).  A mixed outer FP64 pass moves 44 B per point.
ALG_BYTES = {"fp64": 72, "mixed": 40}
OUTER_BYTES = 44
# The same count on an N^3 grid: the x transforms stay in the row passes and each of
# the three line passes (forward y, z with the symbol, inverse y) reads and writes the
# spectrum once, two round trips more than the single 2-D column pass.
ALG_BYTES_3D = {"fp64": 104, "mixed": 56}


def iteration_hbm(kernels, alg_bytes_per_point, pts):
    """Whole-iteration HBM figure from a kernel table: the algorithmic bytes of one
    iteration over the summed kernel durations, and its fraction of the HBM peak."""
    it_ms = sum(v["ms"] for v in kernels.values())
    b = alg_bytes_per_point * pts
    return dict(us=round(it_ms * 1e3, 2), bytes=b, achieved=round(b / (it_ms * 1e-3) / 1e9, 1),
                frac=round(b / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))

# Algorithmic HBM bytes per grid point and launch of each kernel (one component):
# every field the kernel must read or write once, nothing for tables or halos.
#   cols   : read + write the spectrum (N^2 reals)
#   rowinv : read spectrum, read P, write P, write P~
#   upd    : read P~, read U_n (mixed: e_n and the FP32 copy of U), write U_{n+1}
#   rowfwd : read U_{n+1} and U^k (mixed: e, U_b, r), write the spectrum
BYTES_PER_POINT = {
    "fp64": {"cols": 16, "rowinv": 32, "upd": 24, "rowfwd": 24, "yfwd": 16, "zsym": 16, "yinv": 16},
    "mixed": {"cols": 8, "rowinv": 16, "upd": 16, "rowfwd": 16, "yfwd": 8, "zsym": 8, "yinv": 8},
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counted_traffic(prec, kernel, logn):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated), or None when the summary is missing or
    was taken from other kernel sources than the ones built here."""
    import re
    from paper_2305_03945_amd import profsum
    path = os.path.join(ROOT, "profiles", "ac2048_traffic.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```\n(\{.*\})\n```", open(path).read())
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("source_hash") != profsum.source_hash():
        return None
    t = "float" if prec == "mixed" else "double"
    kind = {"mixed": 5, "fp64": 1}[prec]   # 5: the mixed row pass (its inner launches)
    names = {"cols": "k_cols<%s,%d,0,1,%d>" % (t, logn, kind), "rowinv": "k_rowinv<%s,%d,0,1>" % (t, logn),
             "upd": "k_upd<%s,%d,0,0,%d>" % (t, logn, 1 if prec == "mixed" else 0),
             "rowfwd": "k_row_forward<%s,%d,0,0,%d>" % (t, logn, kind)}
    k = d["kernels"].get(names.get(kernel, ""))
    return None if k is None else k["hbm_bytes"]


def percentile(xs, q):
    s = sorted(xs)
    if not s:
        return None
    k = (len(s) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def run_precision(ctx, rd, torch, cfg, u0, prec, steps, warmup):
    p = rd.problem_from_config(cfg)
    o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], omega=cfg["omega"], precision=prec)
    ht = cfg["ht"]
    a = u0.clone()
    b = torch.empty_like(a)
    for _ in range(warmup):
        ctx.step(a, ht, p, o, out=b)
        a, b = b, a
    a.copy_(u0)
    torch.cuda.synchronize()
    lat, iters, outer, first = [], 0, 0, None
    statuses, mass = {}, []
    t0 = time.perf_counter()
    for k in range(steps):
        ts = time.perf_counter()
        _, info = ctx.step(a, ht, p, o, out=b)
        lat.append(time.perf_counter() - ts)
        iters += info["iters"]
        outer += info["outer"]
        statuses[info["status"]] = statuses.get(info["status"], 0) + 1
        mass.append(abs(info["mass_drift"]))
        if k == 0:
            first = b.clone()
        a, b = b, a
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pts = cfg["N"] ** cfg.get("dim", 2)
    return dict(
        pt_iters_per_s=pts * iters / wall, wall_s=wall, ms_per_step=1e3 * wall / steps,
        p50_ms=1e3 * percentile(lat, 50), p99_ms=1e3 * percentile(lat, 99),
        iters_total=iters, iters_per_step=iters / steps, outer_total=outer, outer_per_step=outer / steps,
        status=statuses, max_abs_mass_drift_per_step=max(mass),
    ), first, a


def cpu_oracle_sample(cfg, u0_np, wl):
    """The FP64 oracle (Algorithm 1, numpy, one host core) on the first step of the
    headline workload, plus the serving-stream sample."""
    r, t = oracle_step(cfg, u0_np)
    N = cfg["N"]
    return r, dict(value=t["pt_iters_per_s"], unit="grid-point-iters/s", cores=t["cores"], kind="oracle",
                   wall_s=round(t["step_ms"] / 1e3, 3),
                   sample="first implicit step of the %dx%d Allen-Cahn workload, %d PDHG iterations to the "
                          "workload tolerance; numpy on one host core (the oracle is not parallelised)"
                          % (N, N, r.iters),
                   host=host_info(), serving=oracle_serving_sample(wl))


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(cpu_model=model, nproc=os.cpu_count(), omp_num_threads=os.environ.get("OMP_NUM_THREADS"))


def oracle_step(cfg, u0_np):
    """The FP64 oracle (Algorithm 1, numpy, as it stands) on one step: result and timing."""
    from oracle import pdhg as opdhg
    from tests.rd_cases import oracle_opts, oracle_problem
    # cores: CPU time of this thread over wall time (the oracle's numpy FFTs and scipy
    # sparse products run on the calling thread; process-wide CPU time would also count
    # the GPU runtime's own threads)
    t0, c0 = time.perf_counter(), time.thread_time()
    r = opdhg.step(oracle_problem(cfg), u0_np, cfg["ht"], oracle_opts(cfg))
    wall = time.perf_counter() - t0
    cpu = time.thread_time() - c0
    pts = cfg["N"] ** cfg.get("dim", 2)
    return r, dict(pt_iters_per_s=pts * r.iters / wall, step_ms=1e3 * wall, iters=r.iters,
                   cores=max(1, round(cpu / wall)))


def oracle_serving_sample(wl, n_req=8, max_n=256):
    """The oracle on serving requests alone, one after the other: the first n_req steps
    of the stream (trajectory order) whose grid is at most max_n^2."""
    from oracle import pdhg as opdhg
    from tests.rd_cases import oracle_opts, oracle_problem
    reqs = wl.serving_requests(64, 8, seed=5)
    lat, pts_iters, done = [], 0, 0
    t_all = time.perf_counter()
    for r in reqs:
        if r["cfg"]["N"] > max_n:
            continue
        cfg = r["cfg"]
        t0 = time.perf_counter()
        res = opdhg.step(oracle_problem(cfg), r["u0"], cfg["ht"], oracle_opts(cfg))
        lat.append(time.perf_counter() - t0)
        pts_iters += cfg["N"] ** 2 * res.iters
        done += 1
        if done >= n_req:
            break
    wall = time.perf_counter() - t_all
    return dict(requests=done, p50_ms=1e3 * percentile(lat, 50), max_ms=1e3 * max(lat),
                pt_iters_per_s=pts_iters / wall,
                sample="first %d steps of the serving stream with N <= %d, each alone" % (done, max_n))


def iteration_roofline(kernels, results, N, steps):
    """The PDHG iteration against the HBM roofline: ALG_BYTES per grid-point-iteration
    x N^2 over the summed durations of the iteration's launches (HIP events on the
    launch stream); the same over a whole step (mixed: inner iterations and outer FP64
    passes); and the dominant kernel against its own bytes with its counted traffic."""
    out = {}
    for prec in ("mixed", "fp64"):
        it_ms = sum(v["ms"] for v in kernels[prec].values())
        b = ALG_BYTES[prec] * N * N
        gbs = b / (it_ms * 1e-3) / 1e9
        counted = [counted_traffic(prec, k, N.bit_length() - 1) for k in kernels[prec]]
        r = results[prec]
        step_bytes = (r["iters_per_step"] * ALG_BYTES[prec] + r["outer_per_step"] * OUTER_BYTES) * N * N
        step_gbs = step_bytes / (r["ms_per_step"] * 1e-3) / 1e9
        dom = max(kernels[prec], key=lambda k: kernels[prec][k]["ms"])
        dk = kernels[prec][dom]
        dt = counted_traffic(prec, dom, N.bit_length() - 1)
        out[prec] = dict(
            bytes_per_iteration=b, us_per_iteration=round(it_ms * 1e3, 2), achieved=round(gbs, 1),
            frac=round(gbs / HBM_PEAK_GBS, 4),
            traffic=None if any(c is None for c in counted) else round(sum(counted)),
            launches=list(kernels[prec]),
            step=dict(bytes_per_step=step_bytes, ms_per_step=r["ms_per_step"], achieved=round(step_gbs, 1),
                      frac=round(step_gbs / HBM_PEAK_GBS, 4)),
            dominant_kernel=dict(kernel=dom, bytes_per_launch=dk["bytes"], ms_per_launch=dk["ms"],
                                 achieved=round(dk["gbs"], 1), frac=round(dk["gbs"] / HBM_PEAK_GBS, 4),
                                 traffic=None if dt is None else round(dt)))
    m = out["mixed"]
    return dict(bound="hbm", kernel="PDHG iteration (%s), FP32-mixed inner loop" % ", ".join(m["launches"]),
                achieved=m["achieved"], peak=HBM_PEAK_GBS, unit="GB/s", frac=m["frac"], traffic=m["traffic"],
                traffic_unit="HBM bytes per iteration (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                bytes_per_iteration=m["bytes_per_iteration"], us_per_iteration=m["us_per_iteration"],
                bytes_per_grid_point_iteration=ALG_BYTES, mixed=m, fp64=out["fp64"])


def config_leg(ctx, rd, torch, wl, name, precs, steps=None, oracle=True):
    """One named configuration for its whole step count: per precision p50/p99 step
    latency, grid-point-iterations/s, iterations (and outer passes) per step, the
    largest per-step |mass drift|, and the max-abs difference of step 1 from the
    oracle's step 1; the oracle's own timing of that step."""
    import numpy as np
    cfg = dict(wl.CONFIGS[name])
    n = cfg["steps"] if steps is None else min(steps, cfg["steps"])
    u0_np = wl.initial_field(cfg)
    u0 = torch.tensor(u0_np, dtype=torch.float64, device="cuda")
    out = dict(workload=name, N=cfg["N"], steps=n)
    firsts = {}
    ncomp = 2 if cfg["kind"] == "schnakenberg" else 1
    for prec in precs:
        out[prec], firsts[prec], _ = run_precision(ctx, rd, torch, cfg, u0, prec, n, 2)
        if cfg["N"] > 64:
            # the iteration's launches (HIP events) against ALG_BYTES, the bytes one
            # iteration must move per grid point, times the number of species
            p = rd.problem_from_config(cfg)
            o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], omega=cfg["omega"], precision=prec)
            ms = ctx.profile_iteration(u0, cfg["ht"], p, o, reps=20)
            it_ms = sum(ms.values())
            b = ALG_BYTES[prec] * ncomp * cfg["N"] ** 2
            out[prec]["iteration"] = dict(kernels_us={k: round(v * 1e3, 2) for k, v in ms.items()},
                                          us=round(it_ms * 1e3, 2), bytes=b,
                                          frac=round(b / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    if oracle:
        ref, timing = oracle_step(cfg, u0_np)
        out["oracle_step1"] = dict(timing, residual=ref.residual, status=ref.status)
        for prec in precs:
            out[prec]["step1_maxabs_vs_oracle"] = float(np.max(np.abs(firsts[prec].cpu().numpy() - ref.U)))
    if "fp64" in precs and "mixed" in precs:
        out["speedup_mixed_vs_fp64"] = out["fp64"]["wall_s"] / out["mixed"]["wall_s"]
    del u0
    torch.cuda.empty_cache()
    return out


def serve_stream(ctx, rd, torch, reqs, rate):
    """Serve the request stream: trajectory i's step j arrives at reqs[i]["arrivals"][j]
    (seconds after the start; all zero = closed loop).  A step's latency is its
    completion time minus max(arrival, completion of the trajectory's previous step).
    Trajectories are opened at their first arrival and closed after their last step."""
    n = len(reqs)
    u0s = [torch.tensor(r["u0"], dtype=torch.float64, device="cuda") for r in reqs]
    probs = [rd.problem_from_config(r["cfg"]) for r in reqs]
    opts = [rd.make_opts(tol=r["cfg"]["tol"], tau_u=r["cfg"]["tau"], tau_p=r["cfg"]["tau"], omega=r["cfg"]["omega"],
                         precision="mixed") for r in reqs]
    torch.cuda.synchronize()
    events = sorted((a, i, j) for i, r in enumerate(reqs) for j, a in enumerate(r["arrivals"]))
    trajs = [None] * n
    tickets = {}                      # ticket -> (i, j)
    done_at = {}                      # (i, j) -> completion time
    infos = {}
    ev = 0
    t0 = time.perf_counter()
    total = len(events)
    while len(done_at) < total:
        now = time.perf_counter() - t0
        while ev < total and events[ev][0] <= now:
            _, i, j = events[ev]
            if trajs[i] is None:
                trajs[i] = ctx.open(probs[i], opts[i], u0s[i])
            tickets[trajs[i].submit(reqs[i]["cfg"]["ht"])] = (i, j)
            ev += 1
        ctx.pump()
        now = time.perf_counter() - t0
        for tk, (i, j) in list(tickets.items()):
            info = ctx.poll(tk)
            if info is None:
                continue
            del tickets[tk]
            done_at[(i, j)] = now
            infos[(i, j)] = info
            if j == len(reqs[i]["arrivals"]) - 1:
                trajs[i].close()
        if ev < total and not tickets:
            time.sleep(max(0.0, min(1e-3, events[ev][0] - now)))
    wall = time.perf_counter() - t0
    lat = []
    pts = 0
    statuses = {}
    for (i, j), t in done_at.items():
        start = reqs[i]["arrivals"][j]
        if j > 0:
            start = max(start, done_at[(i, j - 1)])
        lat.append(t - start)
        N = reqs[i]["cfg"]["N"]
        pts += N * N * infos[(i, j)]["iters"]
        st = infos[(i, j)]["status"]
        statuses[st] = statuses.get(st, 0) + 1
    return dict(requests=total, wall_s=wall, req_per_s=total / wall, pt_iters_per_s=pts / wall,
                p50_ms=1e3 * percentile(lat, 50), p99_ms=1e3 * percentile(lat, 99), status=statuses,
                rate_req_per_s=rate)


def serving_leg(rd, torch, wl, n_traj, steps_per_traj):
    """Mixed-precision serving stream: closed-loop pass for the saturation rate,
    then Poisson arrivals at 0.7 x that rate."""
    ctx = rd.Context(0)
    try:
        closed = serve_stream(ctx, rd, torch, wl.serving_requests(n_traj, steps_per_traj, seed=5), None)
        rate = 0.7 * closed["req_per_s"]
        opened = serve_stream(ctx, rd, torch, wl.serving_requests(n_traj, steps_per_traj, seed=5, rate=rate), rate)
    finally:
        ctx.close()
    return dict(closed_loop=closed, poisson=opened,
                stream="%d trajectories x %d steps, Allen-Cahn / Cahn-Hilliard / Schnakenberg uniform, N in "
                       "{64..1024}, periodic/Neumann 50/50, h_t log-uniform [1e-4, 1e-2], FP32-mixed"
                       % (n_traj, steps_per_traj))


ADAPT = dict(ht0=0.4, eta=0.5, n_hi=50, n_lo=40, t_end=2.0)


def adaptive_leg(ctx, rd, torch, cfg, u0):
    """The same trajectory with the adaptive step size of Sec. 2.2 (mixed precision):
    h_t^0 = 0.4, eta = 0.5, N^* = 50, N_* = 40, over t in [0, 2].  From the noise the
    first large step needs many iterations (shrink); as the field coarsens the counts
    fall below N_* (enlarge)."""
    p = rd.problem_from_config(cfg)
    o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], omega=cfg["omega"], precision="mixed")
    ht0 = ADAPT["ht0"]
    a = rd.make_adapt(ht0, ADAPT["eta"], ADAPT["n_hi"], ADAPT["n_lo"])
    t_end = ADAPT["t_end"]
    u = u0.clone()
    ctx.advance(u, 2 * cfg["ht"], p, o, rd.make_adapt(cfg["ht"], 0.5, 1000, 1))   # warm: workspaces, tables
    u.copy_(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info, trace = ctx.advance(u, t_end, p, o, a)
    wall = time.perf_counter() - t0
    N = cfg["N"]
    return dict(t_end=t_end, ht0=ht0, eta=ADAPT["eta"], n_hi=ADAPT["n_hi"], n_lo=ADAPT["n_lo"], wall_s=wall,
                pt_iters_per_s=N * N * info["pdhg_iters"] / wall, **info,
                step_sizes=sorted(set(round(h, 12) for h, _, ok in trace if ok)))


def kernel_table(ctx, rd, cfg, u0, prec, pts, reps=20):
    p = rd.problem_from_config(cfg)
    o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], precision=prec)
    ms = ctx.profile_iteration(u0, cfg["ht"], p, o, reps=reps)
    return {k: dict(ms=t, bytes=BYTES_PER_POINT[prec][k] * pts,
                    gbs=BYTES_PER_POINT[prec][k] * pts / (t * 1e-3) / 1e9) for k, t in ms.items()}


def hbm_leg(ctx, rd, torch, wl, steps):
    """The 2048^2 Allen-Cahn parameters on 4096^2 (working set beyond the last-level
    cache): both precisions, per-kernel durations and the whole-iteration HBM rate."""
    cfg = dict(wl.CONFIGS["ac4096"])
    u0 = torch.tensor(wl.initial_field(cfg), dtype=torch.float64, device="cuda")
    n = min(steps, cfg["steps"])
    out = dict(workload="allen_cahn_4096_periodic", steps=n)
    pts = cfg["N"] ** 2
    for prec in ("fp64", "mixed"):
        out[prec], _, _ = run_precision(ctx, rd, torch, cfg, u0, prec, n, 1)
        k = kernel_table(ctx, rd, cfg, u0, prec, pts)
        it_ms = sum(v["ms"] for v in k.values())
        it_bytes = sum(v["bytes"] for v in k.values())
        out[prec]["kernels"] = k
        out[prec]["iteration_gbs"] = it_bytes / (it_ms * 1e-3) / 1e9
        out[prec]["iteration"] = iteration_hbm(k, ALG_BYTES[prec], pts)
    del u0
    torch.cuda.empty_cache()
    return out


def paper_examples_leg(ctx, rd, torch, wl, steps):
    """The paper's examples at their own sizes (128^2) and parameters: the sixth-order
    FCH equation (Sec. 3.3), Schnakenberg with kappa = 100 (Sec. 3.4.1) and the
    Allen-Cahn shrinking circle (Sec. 3.1.1): iterations per step beside the paper's
    counts, time per step and throughput."""
    import numpy as np
    n = min(steps, 20)
    cases = {
        "fch_sec3.3": (rd.make_problem("fch", 128, L=2 * np.pi, diff=(0.18 ** 2,)), wl.fch_example_field(128),
                       1e-3, dict(tol=0.5e-5, tau_u=0.58, tau_p=0.58, max_iter=3000), ("fp64", "mixed")),
        "schnakenberg_sec3.4.1": (rd.make_problem("schnakenberg", 128, bc="neumann", diff=(0.05, 1.0), a=0.1305,
                                                  sb=0.7695, kappa=100.0), wl.schnakenberg_example_field(128),
                                  1.0 / 5000, dict(tol=1e-7, tau_u=0.9, tau_p=0.9), ("fp64", "mixed")),
        "allen_cahn_circle_sec3.1.1": (rd.make_problem("allen_cahn", 128, L=0.5, diff=(0.01,), b=100.0),
                                       wl.circle_example_field(128), 1e-3, dict(tol=1e-7, tau_u=0.5, tau_p=0.5),
                                       ("fp64", "mixed")),
    }
    out = {}
    for name, (p, u0_np, ht, kw, precs) in cases.items():
        u0 = torch.tensor(u0_np, dtype=torch.float64, device="cuda")
        out[name] = {}
        for prec in precs:
            o = rd.make_opts(precision=prec, **kw)
            a = u0.clone()
            b = torch.empty_like(a)
            ctx.step(a, ht, p, o, out=b)
            torch.cuda.synchronize()
            iters, lat = [], []
            t0 = time.perf_counter()
            for _ in range(n):
                ts = time.perf_counter()
                _, info = ctx.step(a, ht, p, o, out=b)
                lat.append(time.perf_counter() - ts)
                iters.append(info["iters"])
                a, b = b, a
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            pts = u0_np.shape[-1] ** 2
            out[name][prec] = dict(steps=n, iters_per_step=sum(iters) / n, iters_first=iters[0],
                                   iters_last=iters[-1], ms_per_step=1e3 * wall / n,
                                   p50_ms=1e3 * percentile(lat, 50), pt_iters_per_s=pts * sum(iters) / wall)
    out["paper_counts"] = {"schnakenberg_sec3.4.1": "about 30 iterations per step",
                           "allen_cahn_circle_sec3.1.1": "mostly below 200 iterations per step"}
    return out


def grid3d_leg(ctx, rd, torch, wl, steps):
    """The 128^3 Allen-Cahn workload (7-point Laplacian, 3-D FFT preconditioner),
    both precisions, the workload's step count (or ``steps`` if smaller)."""
    cfg = dict(wl.CONFIGS["ac3d128"])
    u0 = torch.tensor(wl.initial_field(cfg), dtype=torch.float64, device="cuda")
    n = min(steps, cfg["steps"])
    out = dict(workload="allen_cahn_128^3_periodic", steps=n)
    finals = {}
    for prec in ("fp64", "mixed"):
        out[prec], _, finals[prec] = run_precision(ctx, rd, torch, cfg, u0, prec, n, 2)
    out["mixed_vs_fp64_final_maxabs"] = float((finals["mixed"] - finals["fp64"]).abs().max().item())
    out["speedup_mixed_vs_fp64"] = out["fp64"]["wall_s"] / out["mixed"]["wall_s"]
    out["kernels"] = {prec: kernel_table(ctx, rd, cfg, u0, prec, cfg["N"] ** 3) for prec in ("fp64", "mixed")}
    for prec in ("fp64", "mixed"):
        out[prec]["iteration"] = iteration_hbm(out["kernels"][prec], ALG_BYTES_3D[prec], cfg["N"] ** 3)
    # the largest 3-D grid, the same parameters: rate and kernels at 16.8 M points
    big = dict(cfg, N=256)
    u1 = torch.tensor(wl.initial_field(big), dtype=torch.float64, device="cuda")
    out["n256"] = {}
    for prec in ("fp64", "mixed"):
        out["n256"][prec], _, _ = run_precision(ctx, rd, torch, big, u1, prec, min(n, 10), 1)
        out["n256"][prec]["kernels"] = kernel_table(ctx, rd, big, u1, prec, 256 ** 3)
        out["n256"][prec]["iteration"] = iteration_hbm(out["n256"][prec]["kernels"], ALG_BYTES_3D[prec], 256 ** 3)
    del u1
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ac2048")
    ap.add_argument("--reps", type=int, default=20, help="launches per kernel for the HIP-event timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-stream leg")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a float32 negation of this many MiB (read + write), the known-size "
                         "kernel that calibrates HBM byte counters")
    ap.add_argument("--serve-traj", type=int, default=64, help="trajectories in the serving stream")
    ap.add_argument("--serve-steps", type=int, default=8, help="steps per trajectory in the serving stream")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (--gpus %d refused)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2305_03945_amd import rd, workloads as wl

    cfg = dict(wl.CONFIGS[args.workload])
    N = cfg["N"]
    u0_np = wl.initial_field(cfg)
    u0 = torch.tensor(u0_np, dtype=torch.float64, device="cuda")
    if args.calib_copy_mb:
        n = args.calib_copy_mb * 1024 * 1024 // 4
        a = torch.rand(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b
    ctx = rd.Context(0)
    results, firsts, finals = {}, {}, {}
    for prec in ("fp64", "mixed"):
        log("timing %s: %d warmup + %d steps on %dx%d" % (prec, args.warmup, args.steps, N, N))
        results[prec], firsts[prec], finals[prec] = run_precision(ctx, rd, torch, cfg, u0, prec, args.steps,
                                                                  args.warmup)
        log("  %s" % json.dumps(results[prec]))

    # Per-kernel launch durations (HIP events on the launch stream).
    kernels = {}
    p = rd.problem_from_config(cfg)
    for prec in ("fp64", "mixed"):
        o = rd.make_opts(tol=cfg["tol"], tau_u=cfg["tau"], tau_p=cfg["tau"], precision=prec)
        ms = ctx.profile_iteration(u0, cfg["ht"], p, o, reps=args.reps)
        kernels[prec] = {}
        for k, t in ms.items():
            nbytes = BYTES_PER_POINT[prec][k] * N * N
            kernels[prec][k] = dict(ms=t, bytes=nbytes, gbs=nbytes / (t * 1e-3) / 1e9)
        log("  kernels %s: %s" % (prec, json.dumps(kernels[prec])))
    roofline = iteration_roofline(kernels, results, N, args.steps)
    log("  roofline %s" % json.dumps(roofline))
    log("adaptive step size: mixed, t in [0, %g]" % ADAPT["t_end"])
    adaptive = adaptive_leg(ctx, rd, torch, cfg, u0)
    log("  %s" % json.dumps(adaptive))

    log("4096^2 Allen-Cahn (working set beyond the last-level cache)")
    hbm4096 = hbm_leg(ctx, rd, torch, wl, args.steps)
    log("  %s" % json.dumps({p: hbm4096[p]["pt_iters_per_s"] for p in ("fp64", "mixed")}))

    log("paper examples (128^2): FCH, Schnakenberg kappa = 100, Allen-Cahn circle")
    examples = paper_examples_leg(ctx, rd, torch, wl, args.steps)
    log("  %s" % json.dumps({k: {p: v[p]["iters_per_step"] for p in v} for k, v in examples.items()
                             if k != "paper_counts"}))

    configs = {}
    for name, precs in (("ac64", ("fp64", "mixed")), ("ch512", ("fp64", "mixed")),
                        ("schnak1024", ("mixed", "fp64"))):
        log("configuration %s: %s" % (name, ", ".join(precs)))
        configs[name] = config_leg(ctx, rd, torch, wl, name, precs, oracle=not args.no_cpu)
        log("  %s" % json.dumps(configs[name]))

    log("3-D grid: 128^3 Allen-Cahn")
    grid3d = grid3d_leg(ctx, rd, torch, wl, args.steps)
    log("  %s" % json.dumps(grid3d))

    serving = None
    if not args.no_serve:
        log("serving stream: %d trajectories x %d steps" % (args.serve_traj, args.serve_steps))
        serving = serving_leg(rd, torch, wl, args.serve_traj, args.serve_steps)
        log("  %s" % json.dumps(serving))

    accuracy = {}
    cpu = None
    if not args.no_cpu:
        log("cpu oracle: first step at %dx%d" % (N, N))
        ref, cpu = cpu_oracle_sample(cfg, u0_np, wl)
        cpu["configs"] = {k: v.get("oracle_step1") for k, v in configs.items()}
        for prec in ("fp64", "mixed"):
            accuracy["%s_step1_maxabs_vs_oracle" % prec] = float(np.max(np.abs(firsts[prec].cpu().numpy() - ref.U)))
        accuracy["oracle_step1_iters"] = ref.iters
    accuracy["mixed_vs_fp64_final_maxabs"] = float((finals["mixed"] - finals["fp64"]).abs().max().item())

    mx, f64 = results["mixed"], results["fp64"]
    line = {
        "metric": METRIC, "value": mx["pt_iters_per_s"], "unit": "grid-point-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": mx["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64 (mixed)", "data": "synthetic",
        "config": {"workload": "allen_cahn_%d_periodic" % N, "N": N, "eps": float(cfg["diff"][0]) ** 0.5,
                   "ht": cfg["ht"], "steps": cfg["steps"], "tol_l2": cfg["tol"], "tau": cfg["tau"],
                   "u0": "uniform[-0.1,0.1] seed %d" % cfg["seed"]},
        "p50_ms": mx["p50_ms"], "p99_ms": mx["p99_ms"],
        "mixed": mx, "fp64": f64,
        "speedup_mixed_vs_fp64": f64["wall_s"] / mx["wall_s"],
        "accuracy": accuracy, "kernels": kernels, "roofline": roofline, "cpu_baseline": cpu, "serving": serving,
        "adaptive": adaptive, "configs": configs, "grid3d": grid3d, "hbm4096": hbm4096,
        "paper_examples": examples,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
