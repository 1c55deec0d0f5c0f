"""Benchmark of the per-solve hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): n = 256 points
per axis on [-1,1)^3 (h = 2/n), the C-infinity bump density
exp(-1/(1 - r^2/0.6^2)) for r < 0.6, padded FFT grid 512^3, 40 Gaussian-sum
terms, FP64.  One step = one psp_solve (all five passes) on a density that is
already resident in HBM.  The FP32 tier of the same workload is timed beside
it.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
# hardware queues for the serving leg's streams (two per size class and one
# for precomputes, beside this script's own): with HIP's default of 4, a
# small request's stream can share a queue with a large solve and wait behind
# it in order.  Read when HIP initialises, so it is set before torch loads;
# the single-solve legs measured the same with 4 and 8.
os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
COPY_CAL_BYTES = 1 << 30   # plain device copy used to calibrate the byte counters
TRAFFIC_FILE = os.path.join(HERE, "profiles", "traffic_passes_n256.txt")
# what decides the pass kernels of a solve: their sources and the shipped
# launch-shape table
KERNEL_SOURCES = ["paper_2506_04489_amd/csrc/fft_core.hpp", "paper_2506_04489_amd/csrc/passes.hpp",
                  "paper_2506_04489_amd/tuning_gfx950.json"]


def _code_only(text: str) -> str:
    """C++ source without its comments and with whitespace runs collapsed,
    so that an edit of the commentary leaves the record of the kernels valid."""
    out = []
    i, n = 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":                      # string or character literal
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of what decides the pass kernels: the code of their sources
    (comments and layout aside) and the launch-shape table."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        path = os.path.join(HERE, rel)
        if os.path.exists(path):
            with open(path, "rb") as f:
                data = f.read()
            if rel.endswith((".hpp", ".h", ".hip", ".cpp")):
                data = _code_only(data.decode("utf-8")).encode("utf-8")
            h.update(data)
    return h.hexdigest()


def measured_traffic():
    """Per-launch HBM bytes of each pass from the committed counter summary,
    or None when the pass kernels changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.loads(next(l for l in f if l.startswith("{")))
    except (OSError, StopIteration, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec


def pass_bytes(n: int, real_bytes: int):
    """Algorithmic HBM bytes of each pass for one solve (half-spectrum axis
    counted as n+1 bins; the multiplier octant is FP64 in both tiers)."""
    c = 2 * real_bytes                     # one complex value
    half = n * n * (n + 1)                 # bins of an n x n x (n+1) array
    return [
        real_bytes * n ** 3 + c * half,                       # H1 forward i3 (R2C)
        c * half + 2 * c * half,                              # H2 forward i2
        2 * (2 * c * half) + 8 * (n + 1) ** 3,                # H3 i1 fwd * m * inv
        2 * c * half + c * half,                              # H4 inverse i2
        c * half + real_bytes * n ** 3,                       # H5 inverse i3 (C2R)
    ]


PASS_NAMES = ["H1_z_r2c", "H2_y_fwd", "H3_x_fused", "H4_y_inv", "H5_z_c2r"]


def time_tier(torch, B, D, n, dtype, steps, warmup, chunk=0, group=0):
    h = 2.0 / n
    td = torch.float64 if dtype == "f64" else torch.float32
    t0 = time.perf_counter()
    plan = B.Plan(n, h, 40, dtype=dtype).precompute()
    plan.set_tuning(chunk, group)
    t_pre = time.perf_counter() - t0
    rho = D.bump(n, h, -1.0, 0.6, xp=torch, device="cuda").to(td).contiguous()
    u = torch.empty_like(rho)
    # the solves run on a stream of their own (default priority): on the
    # legacy null stream every launch also orders against all other streams
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(warmup):
        plan.solve(rho, u, stream=st)
    torch.cuda.synchronize()
    # per-pass HIP events on the last fifth of the timed solves (armed while
    # earlier solves still run): an event record between passes costs a
    # solve a few percent, so the other solves run without them and the
    # wall-clock rate is that of plain solves
    profiled = max(1, steps // 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        if i == steps - profiled:
            plan.profile_enable(profiled)
        plan.solve(rho, u, stream=st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cnt, pass_ms, solve_ms = plan.profile_read()
    assert cnt == profiled
    return {"plan": plan, "wall_s": wall, "pass_ms": pass_ms, "solve_ms_events": solve_ms,
            "precompute_s": t_pre, "u": u, "rho": rho, "stream": st}


def solve_latency(torch, B, plan, rho, u, st, count=50, graph_reps=50):
    """Per-solve latency (HIP events around each solve, on the stream the
    solve runs on): median, p99 and the mean of the first 10 (the paper's
    timing protocol, Section 3); and the rate of the same solve replayed as
    a captured HIP graph."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(count)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(st)
        plan.solve(rho, u, stream=st)
        b.record(st)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    first10 = [a.elapsed_time(b) for a, b in ev[:10]]
    g = B.Graph.capture(plan, rho, u, stream=st)
    for _ in range(3):
        g.launch(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(graph_reps):
        g.launch(st)
    torch.cuda.synchronize()
    graph_ms = 1e3 * (time.perf_counter() - t0) / graph_reps
    g.close()
    return {"median_ms": round(ms[len(ms) // 2], 4), "p99_ms": round(ms[min(len(ms) - 1, int(0.99 * len(ms)))], 4),
            "mean_of_10_ms": round(sum(first10) / 10, 4), "graph_ms_per_solve": round(graph_ms, 4),
            "graph_solves_per_s": round(1e3 / graph_ms, 1)}


def bench_batched(torch, B, D, dtype, reps=5):
    """The batched workload: 64 seeded Gaussian mixtures, n ~ U{32,48,64,96,128}.
    One-at-a-time psp_solve, one psp_solve_batched (grouped launches), the
    batch replayed as a captured graph, and the batch through the persistent
    kernels, in solves/s."""
    td = torch.float64 if dtype == "f64" else torch.float32
    items = D.batched_workload(count=64, seed=D.BATCH_SEED)
    plans = {}
    for it in items:
        if it.n not in plans:
            plans[it.n] = B.Plan(it.n, it.h, 40, dtype=dtype).precompute()
    ps = [plans[it.n] for it in items]
    rhos = [it.mixture.sample(it.n, it.h, it.x0, xp=torch, device="cuda").to(td).contiguous() for it in items]
    us = [torch.empty_like(r) for r in rhos]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_single = timed(lambda: [p.solve(r, u) for p, r, u in zip(ps, rhos, us)])
    t_batch = timed(lambda: B.solve_batched(ps, rhos, us))
    g = B.Graph.capture_batched(ps, rhos, us)
    t_graph = timed(lambda: g.launch())
    g.close()
    # the same batch through the persistent kernels (one launch per pass)
    B.set_batch_mode("persistent")
    try:
        t_pers = timed(lambda: B.solve_batched(ps, rhos, us))
        B.set_batch_mode("flat")
        t_flat = timed(lambda: B.solve_batched(ps, rhos, us))
    finally:
        B.set_batch_mode("grouped")
    # FP32 tier: every result's error against the FP64 tier (whose parity
    # with the oracle is 1e-12), worst per n
    err = None
    if dtype == "f32":
        B.solve_batched(ps, rhos, us)
        p64 = {n: B.Plan(n, 2.0 / n, 40).precompute() for n in plans}
        err = {}
        for it, r, u in zip(items, rhos, us):
            ref = p64[it.n].solve(r.double())
            e = float((u.double() - ref).abs().max() / ref.abs().max())
            err[it.n] = max(err.get(it.n, 0.0), e)
        err = {int(k): float("%.3g" % v) for k, v in sorted(err.items())}
    pts = sum(it.n ** 3 for it in items)
    return {"count": len(items), "sizes": sorted({it.n for it in items}),
            "one_at_a_time_solves_per_s": round(len(items) / t_single, 1),
            "batched_solves_per_s": round(len(items) / t_batch, 1),
            "graph_batched_solves_per_s": round(len(items) / t_graph, 1),
            "persistent_batched_solves_per_s": round(len(items) / t_pers, 1),
            "flat_batched_solves_per_s": round(len(items) / t_flat, 1),
            "batched_mpts_per_s": round(pts / t_batch / 1e6, 1),
            "speedup_batched_vs_single": round(t_single / t_batch, 2),
            **({"max_err_vs_f64_tier_by_n": err} if err is not None else {})}


def bench_serving(torch, B, D, count=2000, rates=(0.25, 0.5, 0.75, 0.9, 1.0, 1.2), budget=200 << 30, slots=64):
    """The serving stream: Poisson arrivals, n from {64..384}, 50/50 tiers and
    density families; spectra cached per (n, h, R) (warmed first).  For each
    rate (a multiple of the measured capacity) the latency percentiles from
    submit to completion and the achieved throughput."""
    import numpy as np
    reqs = D.serving_workload(count=count, rate=1.0, seed=D.SERVE_SEED)
    sv = B.Server(hbm_budget_bytes=budget, max_slots=slots)
    # inputs: a few distinct densities per (n, tier, family), reused; outputs
    # from per-(n, tier) rings of buffers whose previous request must be done
    pool, rings = {}, {}
    for r in reqs:
        key = (r.n, r.tier, r.kind)
        if key not in pool:
            td = torch.float64 if r.tier == "f64" else torch.float32
            pool[key] = [D.request_density(q, xp=torch, device="cuda").to(td).contiguous()
                         for q in [x for x in reqs if (x.n, x.tier, x.kind) == key][:2]]
        rk = (r.n, r.tier)
        if rk not in rings:
            rings[rk] = {"bufs": [torch.empty_like(pool[key][0]) for _ in range(16)], "owner": [None] * 16, "next": 0}
    torch.cuda.synchronize()

    def run(rate):
        t0 = time.perf_counter()
        tickets = []
        for i, r in enumerate(reqs):
            due = t0 + r.t_arrival / rate
            while time.perf_counter() < due:
                pass
            ring = rings[(r.n, r.tier)]
            slot = ring["next"]
            ring["next"] = (slot + 1) % len(ring["bufs"])
            prev = ring["owner"][slot]
            while prev is not None and not sv.poll(prev)[0]:
                time.sleep(0.0002)
            rho = pool[(r.n, r.tier, r.kind)][i % len(pool[(r.n, r.tier, r.kind)])]
            t = sv.submit(r.n, r.h, 40, r.tier, rho, ring["bufs"][slot])
            ring["owner"][slot] = t
            tickets.append(t)
        sv.drain()
        wall = time.perf_counter() - t0
        lat = np.array([sv.poll(t)[2] for t in tickets])
        return wall, lat

    # warm the spectrum cache and workspaces: one request per (n, tier)
    warm = []
    for (n, tier), ring in rings.items():
        key = next(k for k in pool if k[0] == n and k[1] == tier)
        warm.append(sv.submit(n, 2.0 / n, 40, tier, pool[key][0], ring["bufs"][0]))
    sv.drain()
    # capacity: the whole stream submitted at once
    wall, lat = run(1e9)
    cap = count / wall
    # one-at-a-time baseline: the same requests as consecutive psp_solve calls
    plans = {}
    for r in reqs:
        if (r.n, r.tier) not in plans:
            plans[(r.n, r.tier)] = B.Plan(r.n, r.h, 40, dtype=r.tier).precompute()
    def seq():
        for i, r in enumerate(reqs):
            k = (r.n, r.tier, r.kind)
            plans[(r.n, r.tier)].solve(pool[k][i % len(pool[k])], rings[(r.n, r.tier)]["bufs"][0])
    seq()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    out = {"requests": count, "capacity_req_per_s": round(cap, 1),
           "one_at_a_time_req_per_s": round(count / t_seq, 1), "rates": []}
    pts = sum(r.n ** 3 for r in reqs)
    ns = np.array([r.n for r in reqs])
    for f in rates:
        wall, lat = run(cap * f)
        by_n = {int(n): [round(float(np.percentile(lat[ns == n], q)), 3) for q in (50, 99)]
                for n in sorted(set(ns.tolist()))}
        out["rates"].append({"load": f, "rate_req_per_s": round(cap * f, 1),
                             "p50_ms": round(float(np.percentile(lat, 50)), 3),
                             "p99_ms": round(float(np.percentile(lat, 99)), 3),
                             "p50_p99_ms_by_n": by_n,
                             "achieved_req_per_s": round(count / wall, 1),
                             "achieved_mpts_per_s": round(pts / wall / 1e6, 1)})
    # FP32-tier requests: error of each (n, density family) input against the
    # FP64 tier (whose parity with the oracle is 1e-12), worst per n
    err = {}
    for (n, tier, kind), dens in pool.items():
        if tier != "f32":
            continue
        p32, p64 = B.Plan(n, 2.0 / n, 40, dtype="f32").precompute(), B.Plan(n, 2.0 / n, 40).precompute()
        for d in dens:
            u32, ref = p32.solve(d), p64.solve(d.double())
            e = float((u32.double() - ref).abs().max() / ref.abs().max())
            err[n] = max(err.get(n, 0.0), e)
    out["f32_max_err_vs_f64_tier_by_n"] = {int(k): float("%.3g" % v) for k, v in sorted(err.items())}
    st = sv.stats()
    out["bytes_peak_GB"] = round(st["bytes_peak"] / 2 ** 30, 2)
    out["cache_hits"], out["cache_misses"] = st["cache_hits"], st["cache_misses"]
    sv.close()
    return out


EPS_TABLE3 = (7.5e-2, 2.2e-2, 5.7e-3, 1.6e-3, 4.7e-4, 2.0e-4)


def bench_eps(torch, B, sizes=(64, 128), R=461, sigma=0.2, reps=20):
    """Error against the exact potential as the near-field cutoff eps varies
    (Theorem 1, Table 3): the paper's Gaussian (sigma = 0.2) on its node grid
    of [-2, 2]^3 (N nodes per axis, both ends), S = 460 Gaussian-sum terms,
    eps relative to the box width.  Per (N, eps): E, set-up time (plan
    creation + precompute, i.e. Algorithm 1) and solve time; per N the slope
    of log E against log eps over the cutoff-limited rows."""
    import math
    out = {"sizes": list(sizes), "R": R, "sigma": sigma, "rows": [], "slope": {}}
    for N in sizes:
        h = 4.0 / (N - 1)
        x = -2.0 + h * torch.arange(N, dtype=torch.float64, device="cuda")
        r = torch.sqrt(x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2)
        rho = (torch.exp(-r * r / (2 * sigma * sigma)) / ((2 * math.pi) ** 1.5 * sigma ** 3)).contiguous()
        safe = torch.where(r > 0, r, torch.ones_like(r))
        u_star = torch.where(r > 0, torch.special.erf(safe / (math.sqrt(2) * sigma)) / (4 * math.pi * safe),
                             torch.full_like(r, math.sqrt(2 / math.pi) / (4 * math.pi * sigma)))
        logs = []
        for e in EPS_TABLE3:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p = B.Plan(N, h, R, eps=e * 4.0, delta=math.sqrt(3.0) * N * h).precompute()
            torch.cuda.synchronize()
            setup_s = time.perf_counter() - t0
            u = p.solve(rho)
            for _ in range(3):
                p.solve(rho, u)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                p.solve(rho, u)
            torch.cuda.synchronize()
            solve_ms = 1e3 * (time.perf_counter() - t0) / reps
            E = float((u - u_star).abs().max() / u_star.abs().max())
            out["rows"].append({"N": N, "eps": e, "E": float("%.4g" % E), "setup_s": round(setup_s, 3),
                                "solve_ms": round(solve_ms, 4)})
            if 4e-4 < e < 3e-2:
                logs.append((math.log(e), math.log(E)))
            del p
        mx = sum(a for a, _ in logs) / len(logs)
        my = sum(b for _, b in logs) / len(logs)
        out["slope"][N] = round(sum((a - mx) * (b - my) for a, b in logs) / sum((a - mx) ** 2 for a, _ in logs), 3)
    return out


BOX_ROWS = (("Table 4", "gauss", 0.2, ((-3, 2), (-2, 3.5), (-1, 5))),
            ("Table 6", "bump", (2.0, 10.0), ((-3, 1), (-2, 3), (-2, 4))),
            ("Table 8", "anis", 2.0, ((-2, 2), (-4, 4), (-4, 4))),
            ("Table 8", "anis", 32.0, ((-2, 2), (-64, 64), (-64, 64))))


def _box_density(torch, family, par, box, N):
    """(rho, u*) of the paper's rectangular-box benchmarks at the box centre
    on its node grid (N points per side including both ends; N: one count or
    one per axis), on the GPU."""
    import math
    Ns = tuple(N) if isinstance(N, (tuple, list)) else (N, N, N)
    hs = tuple((b - a) / (m - 1) for (a, b), m in zip(box, Ns))
    ax = [a + h * torch.arange(m, dtype=torch.float64, device="cuda") - 0.5 * (a + b)
          for (a, b), h, m in zip(box, hs, Ns)]
    X, Y, Z = ax[0][:, None, None], ax[1][None, :, None], ax[2][None, None, :]
    if family == "gauss":
        s = par
        r = torch.sqrt(X * X + Y * Y + Z * Z)
        rho = torch.exp(-r * r / (2 * s * s)) / ((2 * math.pi) ** 1.5 * s ** 3)
        safe = torch.where(r > 0, r, torch.ones_like(r))
        u = torch.where(r > 0, torch.special.erf(safe / (math.sqrt(2) * s)) / (4 * math.pi * safe),
                        torch.full_like(r, math.sqrt(2 / math.pi) / (4 * math.pi * s)))
    elif family == "bump":
        R, d = par
        r2 = X * X + Y * Y + Z * Z
        inside = r2 < R * R
        den = torch.where(inside, R * R - r2, torch.ones_like(r2))
        u = torch.where(inside, torch.exp(-d * R * R / den), torch.zeros_like(r2))
        rho = torch.where(inside, 2 * d * R ** 2 * (3 * R ** 4 - 2 * R ** 2 * r2 - r2 ** 2 - 2 * d * R ** 2 * r2)
                          / den ** 4 * u, torch.zeros_like(r2))
    else:
        sx, sy, sz = 0.2, 0.2 * par, 0.2 * par
        u = torch.exp(-X * X / sx ** 2 - Y * Y / sy ** 2 - Z * Z / sz ** 2)
        rho = -(4 * X * X / sx ** 4 + 4 * Y * Y / sy ** 4 + 4 * Z * Z / sz ** 4
                - 2 / sx ** 2 - 2 / sy ** 2 - 2 / sz ** 2) * u
    return hs, rho.contiguous(), u


GRID_ROWS = (("grid", "gauss", 0.2, ((-2, 2), (-2, 2), (-2, 2)), (64, 96, 128)),
             ("grid", "gauss", 0.2, ((-2, 2), (-2, 2), (-2, 2)), (128, 192, 256)))


def bench_box(torch, B, sizes=(64, 128), R=461, reps=20):
    """The paper's rectangular-box benchmarks (Section 3, Tables 4, 6, 8):
    E against the exact potential, set-up time (plan creation + precompute)
    and solve time, per table row and N; then the Gaussian on grids with a
    different point count per axis."""
    out = []
    rows = [(t, f, p, b, N) for t, f, p, b in BOX_ROWS for N in sizes] + list(GRID_ROWS)
    for tab, fam, par, box, N in rows:
        hs, rho, u_star = _box_density(torch, fam, par, box, N)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = B.Plan(N, hs, R).precompute()
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        u = p.solve(rho)
        for _ in range(3):
            p.solve(rho, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            p.solve(rho, u)
        torch.cuda.synchronize()
        E = float((u - u_star).abs().max() / u_star.abs().max())
        out.append({"table": tab, "family": fam, "param": par, "N": N, "E": float("%.4g" % E),
                    "setup_s": round(setup_s, 4),
                    "solve_ms": round(1e3 * (time.perf_counter() - t0) / reps, 4)})
        del p
    return out


def cpu_baseline_and_parity(n, rho_big, gpu_u, gpu_u32=None, reps_small=10, reps_mid=3):
    """The oracle (as it stands) timed on the host, solve phase only (the
    set-up of Algorithm 1 excluded, as in the paper's protocol, Section 3),
    with its C naive FFT on one thread and on all of them:
      * n = 32 Gaussian: reps_small solves each way (median and mean);
      * n = 128 oscillatory: reps_mid solves on all threads, one on one;
      * the headline n (bump, rho_big: the density the GPU solved, copied
        back): one whole solve on all threads, whose output is compared
        element by element with the timed GPU result (FP64 tier, and the
        FP32 tier when given): eq. error_infty over every grid point.
    value/unit: the headline solve on all threads, in solves/s."""
    import statistics
    import numpy as np
    from oracle import native
    from oracle import psp_oracle as O
    from paper_2506_04489_amd import densities as D
    all_threads = native.set_threads(0)

    def timed(rho, h, su, reps, threads):
        native.set_threads(threads)
        O.solve(rho[:4, :4, :4], h, 4)                     # warm the library
        ts, u = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            u = O.solve(rho, h, su.R, su=su)
            ts.append(time.perf_counter() - t0)
        return ts, u

    out = {"kind": "oracle", "unit": "solves/s", "cores": all_threads, "host_cpus": os.cpu_count(),
           "protocol": "solve phase only (set-up excluded); C naive radix-2/3 FFT with OpenMP over lines, "
                       "pad/multiply/crop in numpy"}
    runs = {}
    h = 2.0 / 32
    su = O.setup(32, h, 40)
    rho = D.gaussian(32, h, -1.0, 0.15)
    for th in (1, all_threads):
        ts, _ = timed(rho, h, su, reps_small, th)
        runs["n32_gaussian_%dthr" % th] = {"solves": reps_small, "median_s": round(statistics.median(ts), 5),
                                          "mean_s": round(sum(ts) / len(ts), 5)}
    h = 2.0 / 128
    su = O.setup(128, h, 40)
    rho = D.oscillatory(128, h, -1.0, a=0.2, omega=20.0)
    for th, reps in ((all_threads, reps_mid), (1, 1)):
        ts, _ = timed(rho, h, su, reps, th)
        runs["n128_oscillatory_%dthr" % th] = {"solves": reps, "median_s": round(statistics.median(ts), 4),
                                              "mean_s": round(sum(ts) / len(ts), 4)}
    h = 2.0 / n
    su = O.setup(n, h, 40)
    ts, want = timed(rho_big, h, su, 1, all_threads)
    runs["n%d_bump_%dthr" % (n, all_threads)] = {"solves": 1, "median_s": round(ts[0], 3), "mean_s": round(ts[0], 3)}
    native.set_threads(0)
    out["runs"] = runs
    out["value"] = 1.0 / ts[0]
    out["sample"] = ("one whole n=%d bump solve on %d threads (%.1f s); beside it n=32 x%d and n=128 x%d on all "
                     "threads and on one" % (n, all_threads, ts[0], reps_small, reps_mid))
    scale = float(np.max(np.abs(want)))
    parity = {"points": int(want.size), "metric": "max|u_gpu - u_oracle| / max|u_oracle| over every grid point",
              "f64": float(np.max(np.abs(gpu_u - want)) / scale), "tol_f64": 1e-12}
    parity["f64_ok"] = parity["f64"] <= 1e-12
    if gpu_u32 is not None:
        parity["f32"] = float(np.max(np.abs(gpu_u32 - want)) / scale)
        parity["tol_f32"] = 1e-5
        parity["f32_ok"] = parity["f32"] <= 1e-5
    return out, parity


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle CPU baseline and the element-wise check of the timed result")
    ap.add_argument("--no-f32", action="store_true", help="skip the FP32 tier")
    ap.add_argument("--chunk", type=int, default=0, help="k3 tiles per H2-H4 chunk (0: library default)")
    ap.add_argument("--group", type=int, default=0, help="i1 slabs per H1-H2/H4-H5 group (0: library default)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--no-eps", action="store_true", help="skip the near-field cutoff study")
    ap.add_argument("--no-box", action="store_true", help="skip the rectangular-box rows")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        sys.stderr.write("bench.py measures one GPU: the library has no multi-GPU path "
                         "(requested --gpus %d)\n" % args.gpus)
        sys.exit(2)

    import torch
    from paper_2506_04489_amd import densities as D
    from paper_2506_04489_amd import psp as B
    B.lib()                                   # fail loudly if libpsp.so is missing
    n = args.n
    if args.copy_calibration:
        a = torch.ones(COPY_CAL_BYTES // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    res = time_tier(torch, B, D, n, "f64", args.steps, args.warmup, args.chunk, args.group)
    ms = 1e3 * res["wall_s"] / args.steps
    value = args.steps / res["wall_s"]
    pb = pass_bytes(n, 8)
    dom = max(range(5), key=lambda i: res["pass_ms"][i])
    achieved = pb[dom] / (res["pass_ms"][dom] * 1e-3) / 1e9
    b_alg_fused = 16 * n ** 3 + 128 * n * n * (n + 1) + 8 * (n + 1) ** 3
    out = {
        "metric": "FP64 solves/s at 256^3 (<=1e-12 rel err vs oracle); served p50/p99 ms",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single solve, bump exp(-1/(1-r^2/0.36)) r<0.6, n=%d on [-1,1)^3, "
                               "padded %d^3, R=40, FP64" % (n, 2 * n),
                   "n": n, "padded": 2 * n, "R": 40, "global_batch": 1},
        "mpts_per_s": round(value * n ** 3 / 1e6, 1),
        "roofline": {"bound": "hbm", "kernel": PASS_NAMES[dom], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "alg_bytes_per_launch": pb[dom]},
        "kernel_source_sha256": kernel_source_hash(),
        "passes": {PASS_NAMES[i]: {"ms": round(res["pass_ms"][i], 4),
                                   "alg_GBps": round(pb[i] / (res["pass_ms"][i] * 1e-3) / 1e9, 1)}
                   for i in range(5)},
        "solve_ms_events": round(res["solve_ms_events"], 4),
        "solve_frac_of_hbm_roofline_fused_xy_model": round(b_alg_fused / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "solve_frac_of_hbm_roofline_5pass": round(sum(pb) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "precompute_s": round(res["precompute_s"], 3),
        "paper_context": "MATLAB on i7-8565U, FP64, 128^3: 0.536 s/solve (Table 1); no 256^3 or GPU number",
    }
    # set-up of a further plan in the warm process (Algorithm 1: GS fit, 1D
    # tables, spectrum; a new h, so no cached spectrum); precompute_s above is
    # the process's first plan and includes loading the library and its code
    t0 = time.perf_counter()
    p2 = B.Plan(n, 2.0 / n * (1 + 1e-3), 40, dtype="f64").precompute()
    torch.cuda.synchronize()
    out["precompute_warm_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
    del p2
    out["latency"] = solve_latency(torch, B, res["plan"], res["rho"], res["u"].clone(), res["stream"])
    pk = B.device_peaks()
    out["peaks"] = {"hbm_spec_GBps": HBM_PEAK_GBS, "copy_measured_GBps": round(pk["copy_GBps"], 1),
                    "fp64_mfma_spec_TFLOPs": 78.6, "fp64_mfma_measured_TFLOPs": round(pk["fp64_mfma_TFLOPs"], 1)}
    out["roofline"]["frac_of_measured_copy"] = round(achieved / pk["copy_GBps"], 4)
    tr = measured_traffic() if n == 256 else None
    if tr is not None and PASS_NAMES[dom] in tr.get("passes", {}):
        out["roofline"]["traffic"] = tr["passes"][PASS_NAMES[dom]]["bytes"]
        out["roofline"]["traffic_source"] = os.path.relpath(TRAFFIC_FILE, HERE)
    if not args.no_f32:
        r32 = time_tier(torch, B, D, n, "f32", args.steps, args.warmup, args.chunk, args.group)
        # FP32-tier error against the FP64 result of the same workload
        u64 = res["u"]
        err = float((r32["u"].double() - u64).abs().max() / u64.abs().max())
        out["_u32"] = r32["u"].double().cpu().numpy()
        out["f32_tier"] = {"solves_per_s": round(args.steps / r32["wall_s"], 3),
                           "ms_per_step": round(1e3 * r32["wall_s"] / args.steps, 4),
                           "pass_ms": [round(v, 4) for v in r32["pass_ms"]],
                           "err_vs_f64_tier": err}
    if not args.no_batched:
        out["batched"] = {t: bench_batched(torch, B, D, t) for t in ("f64", "f32")}
    if not args.no_serve:
        out["served"] = bench_serving(torch, B, D, count=args.serve_count)
        loads = out["served"]["rates"]
        if loads:
            near = min(loads, key=lambda x: abs(x["load"] - 0.9))
            out["served_p50_ms"], out["served_p99_ms"] = near["p50_ms"], near["p99_ms"]
    if not args.no_eps:
        out["eps_study"] = bench_eps(torch, B)
    if not args.no_box:
        out["box_rows"] = bench_box(torch, B)
    if not args.no_cpu:
        # the timed results themselves, checked against the oracle's
        # whole-grid solve (timed as the CPU baseline)
        u32 = out.pop("_u32", None)
        out["cpu_baseline"], out["parity"] = cpu_baseline_and_parity(n, res["rho"].cpu().numpy(),
                                                                     res["u"].cpu().numpy(), u32)
    out.pop("_u32", None)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
