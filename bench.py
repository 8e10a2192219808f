#!/usr/bin/env python3
"""Benchmark of the k-point ISDF hot path on one MI355X.

One step = the whole path over one batch of synthetic input: the fit
(X^k, Pi^q and eta^q as k convolutions, FP64 pivoted Cholesky), the Coulomb
kernel W^q (grid FFT with 4 pi/|G+q|^2, V^q GEMM, FP64 solves) and the
fragment ERIs of every fragment of the workload, submitted at one instant to
the serving loop and collected by polling (so each fragment has a
submit-to-done latency).  Inputs (orbitals, interpolation points, fragment
coefficients) are resident in HBM before timing starts.

Prints one JSON line: fragment ERIs/s (sum of n_f^4 over fragments per
second of wall time, fit included), p50/p99 latency, the speedup over the
same step in FP64, the max |mixed - FP64| error per result, a roofline entry
for the dominant kernel and the FP64 CPU oracle timed on this host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak rates of MI355X (dense; TFLOP/s and GB/s)
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "hbm": 8000.0}
PREC_PEAK = {"fp64": ("fp64", 78.6), "fp32": ("fp32", 157.3), "bf16x3": ("bf16", 2500.0)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3_k4_32")
    ap.add_argument("--prec", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-fp64-ref", action="store_true")
    ap.add_argument("--poisson-rates", default="200,1000,4000",
                    help="request rates (1/s) of the open-arrival serving sweep after the timed steps; '' skips it")
    ap.add_argument("--poisson-n", type=int, default=256, help="requests per rate of the sweep")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the fragment-batch comparison (eager / HIP graph / tuned tiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=25.0)
    ap.add_argument("--max-batch", type=int, default=0,
                    help="fragments per serving batch (0: all of a step in one batch)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device copy first (reference for HBM byte counters)")
    return ap.parse_args()


def n_classes(kmesh):
    """Number of classes {q, -q} of the k mesh: the stages from the metric on
    run over one q of each (the others are complex conjugates)."""
    m1, m2, m3 = kmesh
    n = 0
    for j1 in range(m1):
        for j2 in range(m2):
            for j3 in range(m3):
                q = (j1 * m2 + j2) * m3 + j3
                mq = (((m1 - j1) % m1) * m2 + (m2 - j2) % m2) * m3 + (m3 - j3) % m3
                n += mq >= q
    return n


def stage_work(stage, cfg, nfs, prec, eta32=False):
    """(bound, algorithmic amount per launch, unit, peak) of a stage; eta32:
    the fit stored T and eta as complex FP32 (8 B a value, else 16).  The
    k-space stages (T^k, k convolutions' inputs) count all N_k; everything
    indexed by q counts the nh classes {q, -q} it runs over."""
    nk, nip, ng, norb = cfg.n_k, cfg.n_ip, cfg.n_g, cfg.n_orb
    nh = n_classes(cfg.kmesh)
    eb = 8 if eta32 else 16
    s2 = sum(n * n for n in nfs)
    dt, pk = PREC_PEAK[prec]
    if stage == "frag_eri":   # Hermitian half of sum_q U^q R^{qH} per fragment
        fl = sum(8.0 * nh * nip * (n * n) * (n * n + 1) / 2 for n in nfs)
        return "mfma", fl / 1e12, "TFLOP", pk
    if stage == "frag_u":     # U^q = W^q R^q
        return "mfma", 8.0 * nh * nip * nip * s2 / 1e12, "TFLOP", pk
    if stage == "v_gemm":     # Hermitian half of eta~ eta~^H
        return "mfma", 8.0 * nh * nip * nip * ng / 2 / 1e12, "TFLOP", pk
    if stage == "grid_fft":
        if prec == "fp64":    # two read+write passes over eta (c128)
            return "hbm", 4.0 * nh * nip * ng * 16 / 1e9, "GB", PEAK["hbm"]
        # one pass: eta read, the split operand written (8 B a point)
        return "hbm", nh * nip * ng * (eb + 8) / 1e9, "GB", PEAK["hbm"]
    if stage == "rhs_t":      # T^k_I(r) = X^k conj(phi^k): written once
        return "hbm", 1.0 * nk * nip * ng * eb / 1e9, "GB", PEAK["hbm"]
    if stage == "rhs_kconv":  # T^k_I(r) read (all k), eta written once (nh classes)
        return "hbm", (nk + nh) * nip * ng * eb / 1e9, "GB", PEAK["hbm"]
    if stage == "metric_kconv":
        return "hbm", (nk + nh) * nip * nip * 16 / 1e9, "GB", PEAK["hbm"]
    if stage == "frag_pair":  # write R^q once (c128 in FP64, 8 B a point in the mixed formats)
        return "hbm", nh * nip * s2 * (16 if prec == "fp64" else 8) / 1e9, "GB", PEAK["hbm"]
    if stage == "chol":       # blocked factor: n^3/3 complex MACs
        return "fp64", 8.0 * nh * nip ** 3 / 3 / 1e12, "TFLOP", PEAK["fp64"]
    if stage == "pinv":       # L^{-1} (n^3/6) and G = Y^H Y lower half (n^3/2) complex MACs
        return "fp64", 8.0 * nh * nip ** 3 * (1 / 6 + 1 / 2) / 1e12, "TFLOP", PEAK["fp64"]
    if stage == "w_solve":    # W' = (G V') G: one full product, one Hermitian (lower half)
        return "fp64", 1.5 * 8.0 * nh * nip ** 3 / 1e12, "TFLOP", PEAK["fp64"]
    if stage == "metric_t":
        return "mfma", 8.0 * nk * nip * nip * norb / 2 / 1e12, "TFLOP", PEAK["fp64"]
    if stage == "frag_t":
        return "mfma", 8.0 * nk * nip * norb * sum(nfs) / 1e12, "TFLOP", PEAK["fp64"]
    return None


KERNEL_OF_STAGE = {"frag_eri": ("zgemm_nt_kernel<0, false, true, 3>", "{x}false, true, 3"),
                   "frag_u": ("zgemm_nt_kernel<0, false, false, 2>", "{x}false, false, 2"),
                   "v_gemm": ("zgemm_nt_kernel<0, false, true, 1>", "{x}false, true, 1"),
                   "frag_pair": ("pair_kernel(PairArgs)", "pair_reg_kernel<"),
                   "rhs_t": ("rhs_t_kernel<", "rhs_t_kernel<"),
                   "rhs_kconv": ("kconv_reg_kernel<", "kconv_reg_kernel<"),
                   "grid_fft": ("slab_kernel_c<", "fft3_reg_kernel<")}


def kernel_name(stage, prec):
    """Name (prefix) of a stage's main kernel as the profiler lists it: the
    FP32 path runs the two-plane big-tile kernel, bf16x3 its own MFMA kernel."""
    if stage not in KERNEL_OF_STAGE:
        return stage
    x = {"fp32": "zgemm_big_kernel<1, ", "bf16x3": "zgemm_x3_kernel<"}.get(prec, "")
    return KERNEL_OF_STAGE[stage][0 if prec == "fp64" else 1].format(x=x)


def counter_traffic(stage, workload, prec):
    """HBM bytes of one step of a stage's main kernel (all its dispatches in
    the step) from the committed rocprofv3 counter summary (FETCH_SIZE +
    WRITE_SIZE, scaled by a 1 GiB copy), or None if there is none or a kernel
    source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (workload, prec))
    if stage not in KERNEL_OF_STAGE or not os.path.exists(path):
        return None
    prof = json.load(open(path))
    csrc = os.path.join(ROOT, "paper_2601_16379_amd", "csrc")
    for f, h in prof.get("sources_sha256", {}).items():
        fp = os.path.join(csrc, f)
        if not os.path.exists(fp) or hashlib.sha256(open(fp, "rb").read()).hexdigest() != h:
            return None
    key = kernel_name(stage, prec)
    for name, v in prof["kernels"].items():
        if key in name:
            return v["step_bytes"]
    return None


STAGES = ["metric_t", "metric_kconv", "rhs_t", "rhs_kconv", "chol", "pinv", "grid_fft", "v_gemm", "w_solve",
          "frag_t", "frag_pair", "frag_u", "frag_eri"]


def cpu_baseline(d, frags, w_gpu, budget_s):
    """The FP64 oracle on a bounded sample of the same step, extrapolated to
    the whole step with the cost model stated in the sample string."""
    import numpy as np
    from oracle import kpoint as ko
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    cfg = d.cfg
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    x = ko.ip_values(d.orbitals, d.ip_index)
    pi = ko.metric_k(x, cfg.kmesh)
    t_metric = time.perf_counter() - t0
    nr = min(2048, cfg.n_g)
    ridx = np.sort(rng.choice(cfg.n_g, nr, replace=False))
    t0 = time.perf_counter()
    ko.rhs(x, d.orbitals, cfg.kmesh, [0], ridx)
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    ko.rhs(x, d.orbitals, cfg.kmesh, [0, 1], ridx)
    t2 = time.perf_counter() - t0
    per_q = max(t2 - t1, 0.0)
    t_rhs = (max(t1 - per_q, 0.0) + cfg.n_k * per_q) * cfg.n_g / nr
    eta_q = (rng.standard_normal((cfg.n_ip, cfg.n_g))
             + 1j * rng.standard_normal((cfg.n_ip, cfg.n_g)))
    t0 = time.perf_counter()
    ko.kernel_v_route(pi, eta_q[None], d.lattice, cfg.grid, cfg.kmesh, qs=[1])
    t_w = (time.perf_counter() - t0) * cfg.n_k
    # fragments: three sizes, cost model t = a n_f^2 + b n_f^4
    nfs = [f.shape[2] for f in frags]
    order = np.argsort(nfs)
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[(3 * len(order)) // 4])]
    ts = []
    for f in pick:
        t0 = time.perf_counter()
        ko.fragment_eri(x, frags[f], w_gpu, cfg.kmesh)
        ts.append(time.perf_counter() - t0)
        if sum(ts) > budget_s:
            break
    done = pick[:len(ts)]
    if len(ts) >= 2 and len(set(nfs[p] for p in done)) >= 2:
        a_ = np.array([[nfs[p] ** 2, nfs[p] ** 4] for p in done], dtype=float)
        coef = np.linalg.lstsq(a_, np.array(ts), rcond=None)[0]
        coef = np.maximum(coef, 0)
        t_frag = float(sum(coef[0] * n ** 2 + coef[1] * n ** 4 for n in nfs))
    else:
        t_frag = ts[0] * sum(n ** 4 for n in nfs) / nfs[pick[0]] ** 4
    t_step = t_metric + t_rhs + t_w + t_frag
    erisum = float(sum(n ** 4 for n in nfs))
    return {
        "value": erisum / t_step, "unit": "ERIs/s", "cores": int(cores), "kind": "oracle",
        "sample": ("FP64 numpy oracle (direct k and R sums) on this host: metric for all q; "
                   "eta on %d sampled grid points for 1 and 2 q, scaled to all points and q; "
                   "W for one q (FFT, V, pseudo-inverse) times N_q; ERIs of fragments with "
                   "n_f = %s given the GPU FP64 W, extrapolated with t = a n_f^2 + b n_f^4 "
                   "to all %d fragments; extrapolated step %.1f s (measured %.1f s)"
                   % (nr, [nfs[p] for p in pick[:len(ts)]], len(nfs), t_step,
                      t_metric + t1 + t2 + t_w / cfg.n_k + sum(ts))),
        "seconds_per_step": t_step,
        "stage_s": {"metric": t_metric, "rhs": t_rhs, "w": t_w, "fragments": t_frag},
    }


def poisson_sweep(ctx, inp, cfg, cdev, outs, prec, rates, n):
    """Open arrivals: requests for the step's fragments (reused cyclically)
    submitted one at a time at Poisson arrival times (seeded), while earlier
    ones run; per rate the offered and served rates and the p50 / p99 latency
    (the library's clock: submit -> completion observed)."""
    import numpy as np
    rows = []
    for rate in rates:
        arr = inp.make_arrivals(cfg, n, rate)
        tickets, pending, lat = [], set(), {}
        i = 0
        t0 = time.perf_counter()
        while i < n or pending:
            now = time.perf_counter() - t0
            while i < n and arr[i] <= now:
                f = i % len(cdev)
                t = ctx.submit_n([cdev[f]], [outs[f]], prec)[0]
                tickets.append(t)
                pending.add(t)
                i += 1
            for t in list(pending):
                st, l = ctx.poll(t)
                if st == "DONE":
                    lat[t] = l
                    pending.discard(t)
                elif st in ("FAILED", "CANCELLED"):
                    raise RuntimeError("request %d %s: %s" % (t, st, ctx.last_error()))
        wall = time.perf_counter() - t0
        lm = 1e3 * np.array([lat[t] for t in tickets])
        rows.append({"rate_per_s": rate, "requests": n, "offered_per_s": n / float(arr[-1]),
                     "served_per_s": n / wall, "p50_ms": float(np.percentile(lm, 50)),
                     "p99_ms": float(np.percentile(lm, 99))})
        print("poisson %g/s: p50 %.2f ms, p99 %.2f ms" % (rate, rows[-1]["p50_ms"], rows[-1]["p99_ms"]),
              file=sys.stderr, flush=True)
    return rows


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    torch.cuda.set_device(0)
    import isdf_inputs as inp
    import paper_2601_16379_amd as pkg

    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        src.fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cfg = inp.get_config(args.workload)
    t_gen = time.perf_counter()
    d = inp.make_inputs(cfg)
    frags = inp.make_fragments(cfg)
    nfs = [int(f.shape[2]) for f in frags]
    t_gen = time.perf_counter() - t_gen
    print("inputs %s generated in %.1f s: N_k=%d grid=%s n_orb=%d n_ip=%d fragments=%d"
          % (cfg.name, t_gen, cfg.n_k, cfg.grid, cfg.n_orb, cfg.n_ip, len(frags)),
          file=sys.stderr, flush=True)

    orb = torch.from_numpy(d.orbitals).cuda()
    ip = torch.from_numpy(d.ip_index).cuda()
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, orb, ip)
    del orb
    cdev = [torch.from_numpy(f).cuda() for f in frags]
    out_mix = [torch.empty((n, n, n, n), dtype=torch.complex128, device="cuda") for n in nfs]
    out_64 = [torch.empty((n, n, n, n), dtype=torch.complex128, device="cuda") for n in nfs]
    torch.cuda.synchronize()
    per_req = 16 * (cfg.n_k * cfg.n_orb * max(nfs) + cfg.n_k * cfg.n_ip * max(nfs)
                    + 2 * cfg.n_k * cfg.n_ip * max(nfs) ** 2)
    batch_bytes = 16 * (cfg.n_k * cfg.n_orb * sum(nfs) + cfg.n_k * cfg.n_ip * sum(nfs)
                        + 2 * cfg.n_k * cfg.n_ip * sum(n * n for n in nfs)) + (1 << 26)
    budget = 2 * max(batch_bytes, per_req)
    ctx.serve_start(max_inflight=2, max_batch=args.max_batch or len(frags), budget_bytes=budget)

    def step(prec, outs):
        ctx.fit(prec)
        ctx.coulomb_kernel(prec)
        tickets = ctx.submit_n(cdev, outs, prec)
        lat = {}
        pending = set(tickets)
        while pending:
            for t in list(pending):
                st, l = ctx.poll(t)
                if st == "DONE":
                    lat[t] = l
                    pending.discard(t)
                elif st in ("FAILED", "CANCELLED"):
                    raise RuntimeError("request %d %s: %s" % (t, st, ctx.last_error()))
        return [lat[t] for t in tickets]

    for i in range(args.warmup):
        step(args.prec, out_mix)
        print("warmup step %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ctx.stage_reset()
    lats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        lats += step(args.prec, out_mix)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    print("timed %d steps: %.2f ms/step" % (args.steps, ms_step), file=sys.stderr, flush=True)
    # device time of each stage per step (HIP events on the stream it runs on)
    # and the number of timed intervals (kernel launches for "*_kernel")
    stage = {}
    for s in STAGES + [s + "_kernel" for s in KERNEL_OF_STAGE]:
        tot, cnt = ctx.stage_total(s)
        if cnt:
            stage[s] = (tot / args.steps, cnt / args.steps)
    erisum = float(sum(n ** 4 for n in nfs))
    value = erisum * args.steps / wall
    lat_ms = 1e3 * np.asarray(lats)

    # a mixed-precision fit stores T and eta as complex FP32 on the one-pass FFT grids
    eta32 = args.prec != "fp64" and pkg.isdf_fit_eta_fp32(cfg.grid)
    # dominant stage and the roofline of its main kernel: algorithmic work of
    # one launch over the average launch duration; where the stage also runs
    # small helper kernels its GEMM launches are timed alone ("<stage>_kernel")
    dom = max((s for s in STAGES if s in stage), key=lambda k: stage[k][0])
    bound, amount, unit, peak = stage_work(dom, cfg, nfs, args.prec, eta32)
    kt, kn = stage.get(dom + "_kernel", stage[dom])
    avg_ms = kt / kn
    achieved = (amount / kn) / (avg_ms / 1e3)
    if unit == "GB":
        roof = {"bound": "hbm", "achieved": achieved, "peak": peak, "unit": "GB/s"}
    elif bound == "mfma":
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s"}
    roof["frac"] = achieved / peak
    tr = counter_traffic(dom, cfg.name, args.prec)
    roof["traffic"] = None if tr is None else tr / kn
    roof["stage"] = dom
    roof["kernel"] = kernel_name(dom, args.prec)
    roof["avg_launch_ms"] = avg_ms
    roof["launches_per_step"] = kn
    roof["algorithmic_per_launch"] = amount / kn * (1e9 if unit == "GB" else 1e12)

    stage_rows = {}
    for s in STAGES:
        if s not in stage:
            continue
        tot, cnt = stage[s]
        w = stage_work(s, cfg, nfs, args.prec, eta32)
        row = {"ms_per_step": tot, "intervals_per_step": cnt,
               "share": tot / sum(stage[k][0] for k in STAGES if k in stage)}
        if w:
            rate = w[1] / (tot / 1e3)
            row["rate"] = rate
            row["unit"] = "GB/s" if w[2] == "GB" else "TFLOP/s"
            row["frac"] = rate / w[3]
        stage_rows[s] = row

    extra = {}
    rates = [float(r) for r in args.poisson_rates.split(",") if r.strip()]
    if rates:
        extra["poisson"] = poisson_sweep(ctx, inp, cfg, cdev, out_mix, args.prec, rates, args.poisson_n)
    if not args.no_fp64_ref and args.prec != "fp64":
        step("fp64", out_64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step("fp64", out_64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        # W is rebuilt by the last call: rebuild the mixed W for consistency of
        # later calls (not timed)
        errs = [float((a - b).abs().max().item()) for a, b in zip(out_mix, out_64)]
        extra["fp64_ms_per_step"] = 1e3 * t64
        extra["speedup_vs_fp64"] = t64 * 1e3 / ms_step
        extra["max_err_eh"] = max(errs)
        extra["max_err_eh_per_result"] = {"min": min(errs), "median": float(np.median(errs)),
                                          "max": max(errs), "n": len(errs)}
        extra["err_bound_eh"] = 1e-6
    cpu = None
    if not args.no_cpu_baseline:
        w_gpu = np.stack([ctx.get_kernel(q) for q in range(cfg.n_k)])
        cpu = cpu_baseline(d, frags, w_gpu, args.cpu_budget_s)
    if not args.no_graph and args.prec != "fp64":
        # the fragment batch alone (after the timed steps): eager
        # isdf_fragment_eri, its captured HIP graph, and the eager batch again
        # with the launch tiling isdf_autotune picks on it
        ctx.fit(args.prec)
        ctx.coulomb_kernel(args.prec)

        def per_call(fn, n=5):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n):
                fn()
            torch.cuda.synchronize()
            return 1e3 * (time.perf_counter() - t0) / n

        eager_ms = per_call(lambda: ctx.fragment_eri(cdev, args.prec, out=out_mix))
        g = ctx.graph(cdev, out_mix, args.prec)
        graph_ms = per_call(g.launch)
        g.close()
        rep = ctx.autotune(cdev, out_mix, args.prec)
        tuned_ms = per_call(lambda: ctx.fragment_eri(cdev, args.prec, out=out_mix))
        extra["fragment_batch"] = {"eager_ms": eager_ms, "graph_ms": graph_ms, "tuned_eager_ms": tuned_ms,
                                   "autotune": rep}
    ctx.serve_stop()
    ctx.close()

    out = {
        "metric": "fragment ERIs/s + p50/p99 latency, mixed vs FP64 at <=1e-6 Eh max error",
        "value": value,
        "unit": "ERIs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": cfg.name, "n_k": cfg.n_k, "kmesh": list(cfg.kmesh),
                   "grid": list(cfg.grid), "n_orb": cfg.n_orb, "n_ip": cfg.n_ip,
                   "fragments": len(nfs), "n_f_range": [min(nfs), max(nfs)],
                   "eris_per_step": erisum, "parallelism": "1 GPU"},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                       "p99": float(np.percentile(lat_ms, 99)), "n": int(lat_ms.size)},
        "fragments_per_s": len(nfs) * args.steps / wall,
        "roofline": roof,
        "stages": stage_rows,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
