#!/usr/bin/env python3
"""Benchmark of the k-point ISDF hot path on one MI355X.

Two kinds of workload:

* the N_k = 1000 cell (10x10x10 mesh, 40^3 grid, 52 orbitals, 1040
  interpolation points, a stream of 500 fragments of 20-120 orbitals; the
  default) and the N_k = 216 cell: the fit and the Coulomb kernel (X^k, Pi^q
  and eta^q as k convolutions, the FP64 pivoted Cholesky, the grid FFT with
  4 pi/|G+q|^2, V^q and W^q) run once and are timed once; every timed step is
  then a fixed slice of the fragment stream (consecutive fragments of the
  seeded stream, cycling), submitted at one instant to the serving loop with
  W^q resident and polled to completion.  After the timed steps the same
  cell is fitted in FP64 and one slice is run in FP64: the speedup of the
  mixed precision over the plain FP64 GPU path and the max |mixed - FP64| of
  every result of that slice.  The same timed slices are also run in a
  second precision (--alt-prec, single bf16 by default) and reported apart
  with their own rate and error against FP64; the headline value stays the
  --prec one.  The N_k = 216 cell can instead be served to
  open Poisson arrivals (--arrivals).
* the small cells (N_k <= 64): one step is the whole path, fit + kernel + all
  fragments of the cell.

Inputs (orbitals, interpolation points, fragment coefficients) are resident
in HBM before timing starts.  Prints one JSON line: fragment ERIs/s (sum of
n_f^4 over the step's fragments per second of wall time), p50/p99 request
latency, the speedup over FP64, the max error per result, a roofline entry for
the dominant kernel and the FP64 CPU oracle timed on this host on a bounded
sample.
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
PREC_PEAK = {"fp64": ("fp64", 78.6), "fp32": ("fp32", 157.3), "bf16x3": ("bf16", 2500.0), "bf16": ("bf16", 2500.0)}
STREAM_MIN_NK = 216


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5_k10_40")
    ap.add_argument("--prec", default="bf16x3", choices=["fp64", "fp32", "bf16x3", "bf16"])
    ap.add_argument("--alt-prec", default="bf16", choices=["", "fp64", "fp32", "bf16x3", "bf16"],
                    help="second precision timed on the same slices of the fragment stream (reported "
                         "apart, with its own error against FP64); '' for none")
    ap.add_argument("--qgroup", type=int, default=0,
                    help="classes {q, -q} per launch of the fragment contraction (0: the context's default)")
    ap.add_argument("--wg-per-cu", type=int, default=0,
                    help="workgroups per CU of the fragment GEMMs (1: ring pipeline; 0: the context's default)")
    ap.add_argument("--slice", type=int, default=4,
                    help="fragments per timed step of the large cells (a fixed slice of the stream)")
    ap.add_argument("--no-fp64-ref", action="store_true")
    ap.add_argument("--arrivals", type=int, default=0,
                    help="large cells: serve this many requests at the cell's Poisson rate instead of slices")
    ap.add_argument("--poisson-rates", default=None,
                    help="small cells: rates (1/s) of the open-arrival sweep after the timed steps; '' skips it")
    ap.add_argument("--poisson-n", type=int, default=256, help="requests per rate of the sweep")
    ap.add_argument("--no-graph", action="store_true",
                    help="small cells: skip the fragment-batch comparison (eager / HIP graph / tuned tiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=25.0)
    ap.add_argument("--max-inflight", type=int, default=0,
                    help="batches in flight at once in the served stream (0: 1 for the stream slices)")
    ap.add_argument("--max-batch", type=int, default=0,
                    help="fragments per serving batch (0: all of a step in one batch)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device copy first (reference for HBM byte counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="large cells: skip the Coulomb/exchange and interpolation-point legs")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the measured HBM / GEMM peaks (timed after the steps)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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


def frag_flops(cfg, n):
    """Algorithmic flops of one fragment's GEMMs: U^q = R^q W^q
    (8 nh N_IP^2 n^2) and the Hermitian half of the contraction
    (8 nh N_IP n^2 (n^2 + 1) / 2)."""
    nh, nip = n_classes(cfg.kmesh), cfg.n_ip
    return 8.0 * nh * nip * nip * n * n + 8.0 * nh * nip * (n * n) * (n * n + 1) / 2


def stage_work(stage, cfg, nfs, prec, passes=1, yform=False):
    """(bound, algorithmic amount, unit, peak) of a stage over the fragments
    nfs (fragment stages) or one fit + kernel.  The k-space stages (T^k, the
    k convolutions' inputs) count all N_k; everything indexed by q counts the
    nh classes {q, -q} it runs over.  The fit and the kernel are FP64 in
    every precision (16 bytes a value).  passes: q batches of a kernel whose
    eta does not fit at once (the RHS is formed again in each).  yform: the
    mixed fragment GEMMs run in the factor form (W = L L^H): U^q = R^q W^q is
    the triangular Y^q = R^q L^q, whose work is the triangle's."""
    nk, nip, ng, norb = cfg.n_k, cfg.n_ip, cfg.n_g, cfg.n_orb
    nh = n_classes(cfg.kmesh)
    s2 = sum(n * n for n in nfs)
    dt, pk = PREC_PEAK[prec]
    if stage == "frag_eri":   # Hermitian half of sum_q U^q R^{qH} per fragment
        fl = sum(8.0 * nh * nip * (n * n) * (n * n + 1) / 2 for n in nfs)
        return "mfma", fl / 1e12, "TFLOP", pk
    if stage == "frag_u":     # U^q = W^q R^q, or the triangular Y^q = R^q L^q
        tri = (nip + 1) / (2.0 * nip) if yform else 1.0
        return "mfma", 8.0 * nh * nip * nip * s2 * tri / 1e12, "TFLOP", pk
    if stage == "frag_pair":  # write R^q once (c128 in FP64, 8 B a point in the mixed formats)
        return "hbm", nh * nip * s2 * (16 if prec == "fp64" else 8) / 1e9, "GB", PEAK["hbm"]
    if stage == "frag_t":
        return "mfma", 8.0 * nk * nip * norb * sum(nfs) / 1e12, "TFLOP", PEAK["fp64"]
    if stage == "v_gemm":     # Hermitian half of eta~ eta~^H, FP64 MFMA
        return "mfma", 8.0 * nh * nip * nip * ng / 2 / 1e12, "TFLOP", PEAK["fp64"]
    if stage == "grid_fft":   # two read+write passes over eta (c128)
        return "hbm", 4.0 * nh * nip * ng * 16 / 1e9, "GB", PEAK["hbm"]
    if stage == "rhs_t":      # T^k_I(r) = X^k conj(phi^k): formed once per q-batch pass (FP64 FMAs)
        return "fp64", passes * 8.0 * nk * nip * ng * norb / 1e12, "TFLOP", PEAK["fp64"]
    if stage == "rhs_kconv":  # T^k_I(r) read (all k) once per q-batch pass, eta written once (nh classes)
        return "hbm", (passes * nk + nh) * nip * ng * 16 / 1e9, "GB", PEAK["hbm"]
    if stage == "metric_kconv":
        return "hbm", (nk + nh) * nip * nip * 16 / 1e9, "GB", PEAK["hbm"]
    if stage == "chol":       # blocked factor: n^3/3 complex MACs
        return "fp64", 8.0 * nh * nip ** 3 / 3 / 1e12, "TFLOP", PEAK["fp64"]
    if stage == "pinv":       # L^{-1} (n^3/6) and G = Y^H Y lower half (n^3/2) complex MACs
        return "fp64", 8.0 * nh * nip ** 3 * (1 / 6 + 1 / 2) / 1e12, "TFLOP", PEAK["fp64"]
    if stage == "w_solve":    # W' = (G V') G: one full product, one Hermitian (lower half)
        return "fp64", 1.5 * 8.0 * nh * nip ** 3 / 1e12, "TFLOP", PEAK["fp64"]
    if stage == "metric_t":
        return "mfma", 8.0 * nk * nip * nip * norb / 2 / 1e12, "TFLOP", PEAK["fp64"]
    return None


KERNEL_OF_STAGE = {"frag_eri": ("zgemm_nt_kernel<0, false, true, 3>", "{x}false, true, 3"),
                   "frag_u": ("zgemm_nt_kernel<0, false, false, 2>", "{x}false, false, 2"),
                   "frag_pair": ("pair_kernel", "pair_kernel"),
                   "v_gemm": ("zgemm_nt_kernel<0, false, true, 1>", "zgemm_nt_kernel<0, false, true, 1>"),
                   "rhs_t": ("rhs_t_kernel<", "rhs_t_kernel<"),
                   "rhs_kconv": ("kconv_", "kconv_"),
                   "grid_fft": ("slab_kernel_c<", "slab_kernel_c<")}


def kernel_name(stage, prec):
    """Name (prefix) of a stage's main kernel as the profiler lists it: the
    FP32 path runs the two-plane big-tile kernel, bf16x3 and bf16 their own
    MFMA kernels."""
    if stage not in KERNEL_OF_STAGE:
        return stage
    x = {"fp32": "zgemm_big_kernel<1, ", "bf16x3": "zgemm_x3_kernel<", "bf16": "zgemm_x1_kernel<"}.get(prec, "")
    if stage == "frag_eri" and prec == "bf16":
        return "zgemm_c2b_kernel<3>"
    return KERNEL_OF_STAGE[stage][0 if prec == "fp64" else 1].format(x=x)


# other kernels of a stage (the contraction of launches with few tiles)
KERNEL_ALT = {("frag_eri", "bf16x3"): "zgemm_c2b_kernel<2>"}


def counter_traffic(stage, workload, prec):
    """HBM bytes per launch of a stage's main kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB
    copy), or None if there is none or a kernel source changed since it was
    taken."""
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
    # bytes per launch over every kernel of the stage, weighted by dispatches
    keys = [kernel_name(stage, prec)] + ([KERNEL_ALT[(stage, prec)]] if (stage, prec) in KERNEL_ALT else [])
    tot = n = 0
    for name, v in prof["kernels"].items():
        if any(k in name for k in keys):
            tot += v.get("launch_bytes", 0.0) * v.get("dispatches", 1)
            n += v.get("dispatches", 1)
    return tot / n if n else None


FIT_STAGES = ["metric_t", "metric_kconv", "rhs_t", "rhs_kconv", "chol", "pinv", "grid_fft", "v_gemm", "w_solve"]
FRAG_STAGES = ["frag_t", "frag_pair", "frag_u", "frag_eri"]
STAGES = FIT_STAGES + FRAG_STAGES


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        return os.cpu_count()


class FixedW:
    """W^q stand-in for timing the oracle's fragment step: the same matrix
    for every q (the oracle's cost does not depend on the values)."""

    def __init__(self, n, seed=0):
        import numpy as np
        rng = np.random.default_rng(seed)
        a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        self.w = a @ a.conj().T / n
        self.shape = (1, n, n)

    def __getitem__(self, q):
        return self.w


def cpu_baseline(d, nfs_step, budget_s):
    """The FP64 oracle on bounded samples of the same workload, extrapolated
    with the cost model stated in the sample string.  The rate is the
    oracle's fragment ERIs/s with W^q given (the step's work on the GPU);
    the whole-job seconds (fit + kernel + every fragment of the cell) are
    reported beside it."""
    import numpy as np
    from oracle import kpoint as ko
    cfg = d.cfg
    nk, nip, ng = cfg.n_k, cfg.n_ip, cfg.n_g
    rng = np.random.default_rng(0)
    t_all = time.perf_counter()
    x = ko.ip_values(d.orbitals, d.ip_index)
    # metric: rows of Pi^q for one and two q (direct k sums), scaled to all
    # rows and all N_k q of the plain form
    rows = list(range(min(8, nip)))
    t0 = time.perf_counter()
    ko.metric_rows(x, cfg.kmesh, rows, [0])
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    ko.metric_rows(x, cfg.kmesh, rows, [0, 1])
    t2 = time.perf_counter() - t0
    per_q = max(t2 - t1, 0.0)
    t_metric = (max(t1 - per_q, 0.0) + nk * per_q) * nip / len(rows)
    # RHS: eta on sampled grid points for one and two q, scaled to all
    # points and N_k q
    nr = min(256, ng)
    ridx = np.sort(rng.choice(ng, nr, replace=False))
    t0 = time.perf_counter()
    ko.rhs(x, d.orbitals, cfg.kmesh, [0], ridx)
    r1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    ko.rhs(x, d.orbitals, cfg.kmesh, [0, 1], ridx)
    r2 = time.perf_counter() - t0
    per_q = max(r2 - r1, 0.0)
    t_rhs = (max(r1 - per_q, 0.0) + nk * per_q) * ng / nr
    # W for one q (FFT, V, pseudo-inverse) on a stand-in eta, times N_k
    eta_q = rng.standard_normal((nip, ng)) + 1j * rng.standard_normal((nip, ng))
    pi_fix = FixedW(nip, 3)        # a Hermitian positive definite stand-in for Pi^q
    t0 = time.perf_counter()
    ko.kernel_v_route(pi_fix, eta_q[None], d.lattice, cfg.grid, cfg.kmesh, qs=[1])
    t_w = (time.perf_counter() - t0) * nk
    del eta_q
    # fragments: two small sizes given a stand-in W, cost t = a n^2 + b n^4
    w_fix = FixedW(nip)
    sizes = [4, 8] if nk >= STREAM_MIN_NK else sorted(set([min(nfs_step), int(np.median(nfs_step))]))
    ts = []
    for n in sizes:
        c = inp_fragment(cfg, n)
        t0 = time.perf_counter()
        ko.fragment_eri(x, c, w_fix, cfg.kmesh)
        ts.append(time.perf_counter() - t0)
    a_ = np.array([[n ** 2, n ** 4] for n in sizes], dtype=float)
    coef = np.maximum(np.linalg.lstsq(a_, np.array(ts), rcond=None)[0], 0)
    t_frag = lambda ns: float(sum(coef[0] * n ** 2 + coef[1] * n ** 4 for n in ns))
    step_s = t_frag(nfs_step)
    import isdf_inputs as inp
    all_nfs = [int(n) for n in inp.fragment_sizes(cfg)]
    whole = t_metric + t_rhs + t_w + t_frag(all_nfs)
    return {
        "value": float(sum(n ** 4 for n in nfs_step)) / step_s, "unit": "ERIs/s", "cores": int(blas_threads()),
        "kind": "oracle",
        "sample": ("FP64 numpy oracle (direct k and R sums) on this host: fragment ERIs of n_f = %s given W^q, "
                   "extrapolated with t = a n_f^2 + b n_f^4 to the step's fragments (n_f %s); whole cell: "
                   "Pi^q rows for 1 and 2 q scaled to all rows and %d q, eta on %d grid points for 1 and 2 q "
                   "scaled to the grid and %d q, W for one q times %d, all %d fragments; measured %.1f s"
                   % (sizes, list(nfs_step), nk, nr, nk, nk, len(all_nfs), time.perf_counter() - t_all)),
        "seconds_per_step": step_s,
        "whole_cell_s": whole,
        "stage_s": {"metric": t_metric, "rhs": t_rhs, "w": t_w, "fragments_all": t_frag(all_nfs)},
    }


def inp_fragment(cfg, n):
    import isdf_inputs as inp
    return inp.make_fragment(cfg, 10_000 + n, n)


def roofline_entry(ctx, stage_tot, cfg, nfs, prec, steps):
    """Roofline of the dominant fragment stage's main kernel: algorithmic
    work of one launch over its average launch duration (HIP events around
    each launch on the stream it runs on)."""
    dom = max((s for s in FRAG_STAGES if s in stage_tot), key=lambda k: stage_tot[k][0])
    bound, amount, unit, peak = stage_work(dom, cfg, nfs, prec)
    kt, kn = stage_tot.get(dom + "_kernel", stage_tot[dom])
    avg_ms = kt / kn
    achieved = (amount / kn) / (avg_ms / 1e3)
    roof = {"bound": "hbm" if unit == "GB" else "mfma", "achieved": achieved, "peak": peak,
            "unit": "GB/s" if unit == "GB" else "TFLOP/s"}
    roof["frac"] = achieved / peak
    roof["traffic"] = counter_traffic(dom, cfg.name, prec)
    roof["stage"] = dom
    roof["kernel"] = kernel_name(dom, prec)
    if roof["kernel"].count("<") > roof["kernel"].count(">"):   # a prefix of the profiler's name
        roof["kernel"] += ">"
    if (dom, prec) in KERNEL_ALT:
        roof["kernel"] += " (" + KERNEL_ALT[(dom, prec)] + " for launches of fewer tiles than two rounds)"
    roof["avg_launch_ms"] = avg_ms
    roof["launches_per_step"] = kn / steps
    roof["algorithmic_per_launch"] = amount / kn * (1e9 if unit == "GB" else 1e12)
    if prec == "bf16x3" and unit != "GB":
        # three bf16 MFMA products per algorithmic real product
        roof["frac_of_x3_ceiling"] = achieved / (peak / 3)
    return roof


def stage_rows(stage_tot, cfg, nfs, prec, per, passes=1, yform=False):
    rows = {}
    tot_ms = sum(stage_tot[k][0] for k in STAGES if k in stage_tot)
    for s in STAGES:
        if s not in stage_tot:
            continue
        tot, cnt = stage_tot[s]
        w = stage_work(s, cfg, nfs if s in FRAG_STAGES else [], prec, passes, yform)
        row = {"ms": tot / per, "intervals": cnt / per, "share": tot / tot_ms if tot_ms else 0.0}
        if w and tot > 0:
            amount = w[1] * (1 if s in FRAG_STAGES else per)
            rate = amount / (tot / 1e3)
            row["rate"] = rate
            row["unit"] = "GB/s" if w[2] == "GB" else "TFLOP/s"
            row["frac"] = rate / w[3]
        rows[s] = row
    return rows


def measured_peaks(torch):
    """Achievable rates on this GPU, timed with events: HBM as a device copy
    of 4 GiB (read + write bytes / time) and dense GEMMs of the vendor BLAS
    (torch.matmul) per dtype, best of three after a warm-up."""
    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            best = min(best, a.elapsed_time(b) / 1e3)
        return best
    out = {}
    src = torch.empty(1 << 29, dtype=torch.float64, device="cuda")   # 4 GiB
    src.fill_(1.0)
    dst = torch.empty_like(src)
    t = timed(lambda: dst.copy_(src))
    out["hbm_copy_GBps"] = 2 * src.numel() * 8 / t / 1e9
    del src, dst
    for name, dt, n in (("fp64", torch.float64, 8192), ("fp32", torch.float32, 8192),
                        ("bf16", torch.bfloat16, 16384)):
        a = torch.randn(n, n, dtype=torch.float32, device="cuda").to(dt)
        b = torch.randn(n, n, dtype=torch.float32, device="cuda").to(dt)
        t = timed(lambda: torch.matmul(a, b))
        out["gemm_%s_TFLOPs" % name] = 2.0 * n ** 3 / t / 1e12
        del a, b
    torch.cuda.empty_cache()
    out["how"] = ("device copy of 4 GiB (2 x 4 GiB moved); torch.matmul of square n x n matrices "
                  "(n = 8192 fp64/fp32, 16384 bf16), best of 3 timed with events")
    return out


HF_STAGES = ["hf_rho", "hf_j", "hf_kconv", "hf_k"]


def hf_leg(ctx, cfg, d, inp, np, torch, reps, oracle):
    """Coulomb and exchange matrices (isdf_hf_jk, eq. (10)) of a seeded
    closed-shell density matrix with W^q resident: one untimed call, then
    `reps` timed calls (device buffers); per-stage times from the library's
    events; the exchange k convolution against its algorithmic bytes (read
    rho and W of every class, write M once); with `oracle`, the oracle's K
    at one k point timed on the host and scaled by N_k."""
    dm = torch.from_numpy(inp.make_density(cfg)).cuda()
    ctx.hf_jk(dm)
    torch.cuda.synchronize()
    before = collect_stages(ctx, HF_STAGES)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.hf_jk(dm)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    after = collect_stages(ctx, HF_STAGES)
    st = {k: (after[k][0] - before.get(k, (0.0, 0))[0]) / reps for k in after}
    nh = n_classes(cfg.kmesh)
    nn = cfg.n_ip * cfg.n_ip
    kconv_bytes = (2 * cfg.n_k + nh) * nn * 16
    gemm_flops = 2 * 8.0 * cfg.n_k * (cfg.n_ip * cfg.n_orb ** 2 + nn * cfg.n_orb)
    out = {"ms_per_call": 1e3 * wall, "stages_ms": st,
           "kconv": {"bytes": kconv_bytes, "GBps": kconv_bytes / (st.get("hf_kconv", 0) / 1e3) / 1e9
                     if st.get("hf_kconv") else None, "bound": "hbm"},
           "rho_and_k_gemm_tflops": gemm_flops / ((st.get("hf_rho", 0) + st.get("hf_k", 0)) / 1e3) / 1e12
           if st.get("hf_rho") else None,
           "density": "closed shell, N_orb/2 occupied per k (seeded)"}
    if oracle:
        from oracle import hf as ohf
        from oracle import kpoint as ko
        x = ko.ip_values(d.orbitals, d.ip_index)
        ks = [0]
        w = np.stack([ctx.get_kernel(q) for q in range(cfg.n_k)])
        dmh = dm.cpu().numpy()
        t0 = time.perf_counter()
        ohf.exchange_at(x, w, dmh, cfg.kmesh, ks)
        tk = time.perf_counter() - t0
        out["oracle"] = {"exchange_one_k_s": tk, "exchange_all_k_s_estimate": tk * cfg.n_k,
                         "sample": "K at one k point (all q), scaled by N_k"}
        del w
    return out


def select_leg(cfg, d, pkg, np, torch, oracle):
    """Interpolation points by pivoted Cholesky (isdf_select_points) on the
    cell's device-resident orbitals, all N_IP points, timed once; the step's
    algorithmic bytes (read the orbitals once, the earlier factor columns at
    their values once) against HBM; with `oracle`, two oracle steps on the
    host scaled to N_IP steps."""
    orb = torch.from_numpy(d.orbitals).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ip, res = pkg.select_points(cfg.grid, cfg.kmesh, orb, cfg.n_ip)
    t = time.perf_counter() - t0
    del orb
    torch.cuda.empty_cache()
    nrows = cfg.n_k * cfg.n_orb
    n = cfg.n_ip
    byts = n * nrows * cfg.n_g * 16.0 + cfg.n_g * 8.0 * (n * (n - 1) / 2 + 3 * n)
    out = {"s": t, "points": n, "ms_per_step": 1e3 * t / n, "bytes": byts, "GBps": byts / t / 1e9,
           "frac_of_8TBps": byts / t / 8e12, "residual_first_last": [float(res[0]), float(res[-1])]}
    if oracle:
        from oracle import ipselect as ips
        t0 = time.perf_counter()
        ips.pivoted_cholesky_points(d.orbitals, 2)
        t2 = time.perf_counter() - t0
        out["oracle"] = {"two_steps_s": t2, "all_steps_s_estimate": t2 / 2 * n,
                         "sample": "two greedy steps (with the residual start), scaled to N_IP steps"}
    return out


MP2_STAGES = ["mp2_green", "mp2_pconv", "mp2_wchi", "mp2_trace"]


def mp2_leg(ctx, cfg, d, inp, np, torch, n_tau, oracle):
    """Opposite-spin MP2 (isdf_sos_mp2) of seeded canonical orbitals on an
    n_tau-point Laplace grid, timed once after an untimed call; per-stage
    times; the W chi products against the FP64 MFMA peak (16 nh N_IP^3 flops
    per tau); with `oracle`, the oracle's Green's functions at 8 k points
    timed on the host and scaled to N_k and n_tau (the dominant host cost)."""
    c, e, n_occ = inp.make_mo(cfg)
    tau, wt = inp.laplace_grid(n_tau, 1.0)
    cdev = torch.from_numpy(c).cuda()
    ctx.sos_mp2(cdev, e, n_occ, tau[:1], wt[:1])
    torch.cuda.synchronize()
    before = collect_stages(ctx, MP2_STAGES)
    t0 = time.perf_counter()
    r = ctx.sos_mp2(cdev, e, n_occ, tau, wt)
    t = time.perf_counter() - t0
    after = collect_stages(ctx, MP2_STAGES)
    st = {k: after[k][0] - before.get(k, (0.0, 0))[0] for k in after}
    nh = n_classes(cfg.kmesh)
    wflops = 16.0 * nh * cfg.n_ip ** 3 * n_tau
    out = {"s": t, "n_tau": n_tau, "ms_per_tau": 1e3 * t / n_tau, "e_os": r["e_os"], "e_sos_mp2": r["e_sos_mp2"],
           "stages_ms": st,
           "w_chi_tflops": wflops / (st["mp2_wchi"] / 1e3) / 1e12 if st.get("mp2_wchi") else None,
           "orbitals": "seeded canonical orbitals, N_orb/2 occupied, gap >= 0.5 Eh; Laplace grid "
                       "Gauss-Legendre mapped by tau = (1 + x)/(1 - x)"}
    if oracle:
        from oracle import kpoint as ko
        from oracle import mp2 as omp2
        ks = list(range(min(8, cfg.n_k)))
        x = ko.ip_values(d.orbitals[ks], d.ip_index)
        y = omp2.mo_at_ips(x, c[ks])
        t0 = time.perf_counter()
        omp2.greens(y, e[ks], n_occ, float(tau[0]), omp2.chemical_potential(e, n_occ))
        tg = time.perf_counter() - t0
        out["oracle"] = {"greens_8k_s": tg, "greens_all_tau_s_estimate": tg * cfg.n_k / len(ks) * n_tau,
                         "sample": "the oracle's Green's functions at 8 k points for one tau, scaled to "
                                   "N_k and n_tau (the k convolutions and traces not included)"}
    return out


DRPA_STAGES = ["mp2_green", "mp2_pconv", "drpa_accum", "drpa_p", "drpa_logdet"]


def drpa_leg(ctx, cfg, inp, np, torch, n_tau, n_omega):
    """Direct RPA (isdf_drpa) of the same seeded canonical orbitals: n_tau
    times (mapped Gauss-Legendre) for the frequency polarisabilities, a
    time-to-frequency transform fitted over the excitation energies, n_omega
    frequency points, timed once; per-stage times."""
    c, e, n_occ = inp.make_mo(cfg)
    tau, _ = inp.laplace_grid(n_tau, 0.5)
    om, ow = inp.laplace_grid(n_omega, 1.0)
    g = inp.fitted_transform(tau, om, *inp.excitation_range(e, n_occ))
    cdev = torch.from_numpy(c).cuda()
    before = collect_stages(ctx, DRPA_STAGES)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.drpa(cdev, e, n_occ, tau, ow, g)
    t = time.perf_counter() - t0
    after = collect_stages(ctx, DRPA_STAGES)
    st = {k: after[k][0] - before.get(k, (0.0, 0))[0] for k in after}
    return {"s": t, "n_tau": n_tau, "n_omega": n_omega, "e_drpa": r["e_drpa"], "e_second": r["e_second"],
            "stages_ms": st}


def collect_stages(ctx, names):
    out = {}
    for s in names:
        tot, cnt = ctx.stage_total(s)
        if cnt:
            out[s] = (tot, cnt)
    return out


def poll_all(ctx, tickets, t_sched=None):
    """Poll tickets to completion; latency from submission (or from the
    scheduled arrival time when t_sched gives one per ticket)."""
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


# --------------------------------------------------------------------------
# large cells: fit + kernel once, then slices of the fragment stream
# --------------------------------------------------------------------------
def run_stream(args, cfg, pkg, inp, np, torch):
    t_gen = time.perf_counter()
    d = inp.make_inputs(cfg)
    t_gen = time.perf_counter() - t_gen
    log("inputs %s generated in %.1f s: N_k=%d grid=%s n_orb=%d n_ip=%d"
        % (cfg.name, t_gen, cfg.n_k, cfg.grid, cfg.n_orb, cfg.n_ip))
    t0 = time.perf_counter()
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, d.orbitals, d.ip_index)
    torch.cuda.synchronize()
    log("context created in %.1f s (orbitals copied to HBM)" % (time.perf_counter() - t0))
    nfs_all = [int(n) for n in inp.fragment_sizes(cfg)]
    S = max(1, args.slice)
    nsl = args.warmup + args.steps
    slices = [[(i * S + j) % len(nfs_all) for j in range(S)] for i in range(nsl)]
    need = sorted(set(f for sl in slices for f in sl))
    coeffs = {f: torch.from_numpy(inp.make_fragment(cfg, f, nfs_all[f])).cuda() for f in need}
    out_elems = max(sum(nfs_all[f] ** 4 for f in sl) for sl in slices)
    out_buf = torch.empty(out_elems, dtype=torch.complex128, device="cuda")

    def outs_of(sl, buf):
        o, off = [], 0
        for f in sl:
            n = nfs_all[f]
            o.append(buf[off:off + n ** 4].view(n, n, n, n))
            off += n ** 4
        return o

    # fit + Coulomb kernel (once per cell), timed
    ctx.stage_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.fit(args.prec)
    t_fit = time.perf_counter() - t0
    ctx.coulomb_kernel(args.prec)
    t_kernel = time.perf_counter() - t0 - t_fit
    fit_stages = collect_stages(ctx, FIT_STAGES)
    st = ctx.stats()
    rhs_passes = -(-st["classes"] // st["q_batch"])   # q batches of the kernel (eta formed in each)
    wfac = bool(st.get("w_factor"))                  # mixed fragment GEMMs in the factor form
    log("fit %.2f s, Coulomb kernel %.2f s" % (t_fit, t_kernel))
    free, total = torch.cuda.mem_get_info()
    budget = int(0.9 * free)
    if args.wg_per_cu or args.qgroup:
        # defaults: the context's initial tiling
        ctx.set_tiling(args.qgroup or st["eri_qgroup_initial"], args.wg_per_cu or 2)
    ctx.serve_start(max_inflight=args.max_inflight or 1, max_batch=args.max_batch or S, budget_bytes=budget)

    def step(sl, prec, buf):
        return poll_all(ctx, ctx.submit_n([coeffs[f] for f in sl], outs_of(sl, buf), prec))

    for i in range(args.warmup):
        step(slices[i], args.prec, out_buf)
        log("warmup slice %d done" % i)
    torch.cuda.synchronize()
    ctx.stage_reset()
    lats, step_s = [], []
    keep = None
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        sl = slices[args.warmup + i]
        lats += step(sl, args.prec, out_buf)
        step_s.append(time.perf_counter() - ts)
        if i == 0:
            keep = out_buf[:sum(nfs_all[f] ** 4 for f in sl)].clone()
        log("slice %d (n_f %s): %.3f s" % (i, [nfs_all[f] for f in sl], step_s[-1]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed_nfs = [nfs_all[f] for i in range(args.steps) for f in slices[args.warmup + i]]
    frag_tot = collect_stages(ctx, FRAG_STAGES + [s + "_kernel" for s in FRAG_STAGES])
    erisum = float(sum(n ** 4 for n in timed_nfs))
    value = erisum / wall
    lat_ms = 1e3 * np.asarray(lats)
    flops_timed = sum(frag_flops(cfg, n) for n in timed_nfs)
    # whole cell (fit + kernel + every fragment of the stream) at the measured
    # fragment rate: an estimate, stated as one
    est_stream_s = sum(frag_flops(cfg, n) for n in nfs_all) / (flops_timed / wall)
    extra = {"fit_s": t_fit, "kernel_s": t_kernel,
             "fit_kernel_stages": stage_rows(fit_stages, cfg, [], args.prec, 1, rhs_passes),
             "rhs_passes": rhs_passes,
             "step_s": {"min": min(step_s), "median": float(np.median(step_s)), "max": max(step_s)},
             "fragment_tflops_per_s": flops_timed / wall / 1e12,
             "whole_cell_estimate": {"fragments": len(nfs_all), "stream_s": est_stream_s,
                                     "total_s": t_fit + t_kernel + est_stream_s,
                                     "eris_per_s": float(sum(n ** 4 for n in nfs_all))
                                     / (t_fit + t_kernel + est_stream_s),
                                     "basis": "fit + kernel measured once; the 500-fragment stream at the "
                                              "measured fragment flop rate of the timed slices"}}
    alt = None
    if args.alt_prec and args.alt_prec != args.prec:
        # the same timed slices in a second precision (reported apart)
        step(slices[0], args.alt_prec, out_buf)
        torch.cuda.synchronize()
        ctx.stage_reset()
        alat, ast = [], []
        t0 = time.perf_counter()
        for i in range(args.steps):
            ts = time.perf_counter()
            sl = slices[args.warmup + i]
            alat += step(sl, args.alt_prec, out_buf)
            ast.append(time.perf_counter() - ts)
            if i == 0:
                alt_keep = out_buf[:sum(nfs_all[f] ** 4 for f in sl)].clone()
        torch.cuda.synchronize()
        awall = time.perf_counter() - t0
        atot = collect_stages(ctx, FRAG_STAGES + [s + "_kernel" for s in FRAG_STAGES])
        aroof = roofline_entry(ctx, atot, cfg, timed_nfs, args.alt_prec, args.steps)
        alt = {"prec": args.alt_prec, "value": erisum / awall, "unit": "ERIs/s", "ms_per_step": 1e3 * awall / args.steps,
               "latency_ms": {"p50": float(np.percentile(1e3 * np.asarray(alat), 50)),
                              "p99": float(np.percentile(1e3 * np.asarray(alat), 99))},
               "slice0_s": ast[0],
               "roofline": {k: aroof[k] for k in ("stage", "kernel", "achieved", "peak", "unit", "frac")},
               "stages": stage_rows(atot, cfg, timed_nfs, args.alt_prec, args.steps, 1,
                                    wfac and args.alt_prec != "fp64")}
        log("%s: %.3e ERIs/s (%.1f ms per step)" % (args.alt_prec, alt["value"], alt["ms_per_step"]))
    ctx.serve_stop()
    roof = roofline_entry(ctx, frag_tot, cfg, timed_nfs, args.prec, args.steps)
    stages = stage_rows(frag_tot, cfg, timed_nfs, args.prec, args.steps, 1, wfac and args.prec != "fp64")
    extra["w_factor"] = wfac
    if not args.no_extras:
        log("Coulomb / exchange matrices and interpolation-point selection")
        extra["hf_jk"] = hf_leg(ctx, cfg, d, inp, np, torch, 3, not args.no_cpu_baseline)
        log("hf_jk %.1f ms per call" % extra["hf_jk"]["ms_per_call"])
        extra["select_points"] = select_leg(cfg, d, pkg, np, torch, not args.no_cpu_baseline)
        log("select_points %.2f s" % extra["select_points"]["s"])
        extra["sos_mp2"] = mp2_leg(ctx, cfg, d, inp, np, torch, 4, not args.no_cpu_baseline)
        log("sos_mp2 %.2f s for 4 tau points" % extra["sos_mp2"]["s"])
        extra["drpa"] = drpa_leg(ctx, cfg, inp, np, torch, 16, 4)
        log("drpa %.2f s for 16 tau and 4 omega points" % extra["drpa"]["s"])
    if not args.no_fp64_ref and args.prec != "fp64":
        # the plain FP64 GPU path on the same cell: fit + kernel, and the
        # first timed slice; speedup on that slice and max error per result
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.fit("fp64")
        t64_fit = time.perf_counter() - t0
        ctx.coulomb_kernel("fp64")
        t64_kernel = time.perf_counter() - t0 - t64_fit
        log("FP64 fit %.2f s, kernel %.2f s" % (t64_fit, t64_kernel))
        sl = slices[args.warmup]
        ctx.serve_start(max_inflight=1, max_batch=args.max_batch or S, budget_bytes=budget)
        t0 = time.perf_counter()
        lat64 = poll_all(ctx, ctx.submit_n([coeffs[f] for f in sl], outs_of(sl, out_buf), "fp64"))
        t64 = time.perf_counter() - t0
        ctx.serve_stop()
        mixed = outs_of(sl, keep)
        ref64 = outs_of(sl, out_buf)
        errs = [float((a - b).abs().max().item()) for a, b in zip(mixed, ref64)]
        vmax = [float(b.abs().max().item()) for b in ref64]
        extra.update({
            "fp64_fit_s": t64_fit, "fp64_kernel_s": t64_kernel,
            "fp64_slice_s": t64, "mixed_slice_s": step_s[0],
            "speedup_vs_fp64": t64 / step_s[0],
            "speedup_vs_fp64_whole_cell": (t64_fit + t64_kernel + est_stream_s * t64 / step_s[0])
            / (t_fit + t_kernel + est_stream_s),
            "fp64_latency_ms": {"p50": float(np.percentile(1e3 * np.asarray(lat64), 50)),
                                "p99": float(np.percentile(1e3 * np.asarray(lat64), 99))},
            "max_err_eh": max(errs),
            "max_err_eh_per_result": [{"n_f": nfs_all[f], "err": e, "max_abs_v": v}
                                      for f, e, v in zip(sl, errs, vmax)],
            "err_bound_eh": 1e-6, "err_reference": "GPU FP64 path, same slice"})
        if alt is not None:
            aerr = [float((a - b).abs().max().item()) for a, b in zip(outs_of(sl, alt_keep), ref64)]
            alt.update({"speedup_vs_fp64": t64 / alt["slice0_s"], "max_err_eh": max(aerr),
                        "max_err_rel_of_max_v": max(e / v for e, v in zip(aerr, vmax))})
    if alt is not None:
        extra["alt_precision"] = alt
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(d, [nfs_all[f] for f in slices[args.warmup]], args.cpu_budget_s)
    ctx.close()
    nh = n_classes(cfg.kmesh)
    cfgd = {"workload": cfg.name, "n_k": cfg.n_k, "kmesh": list(cfg.kmesh), "grid": list(cfg.grid),
            "n_orb": cfg.n_orb, "n_ip": cfg.n_ip, "classes": nh, "stream_fragments": len(nfs_all),
            "n_f_range": [cfg.frag_lo, cfg.frag_hi], "fragments_per_step": S,
            "eris_per_step": erisum / args.steps, "parallelism": "1 GPU",
            "step": "one fixed slice of the fragment stream, W^q resident (fit + kernel once, reported apart)"}
    return value, wall, erisum, lat_ms, roof, stages, cpu, extra, cfgd, len(timed_nfs)


# --------------------------------------------------------------------------
# large cells served to open arrivals
# --------------------------------------------------------------------------
def run_arrivals(args, cfg, pkg, inp, np, torch):
    d = inp.make_inputs(cfg)
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, d.orbitals, d.ip_index)
    t0 = time.perf_counter()
    ctx.fit(args.prec)
    ctx.coulomb_kernel(args.prec)
    t_fk = time.perf_counter() - t0
    n = args.arrivals
    nfs_all = [int(x) for x in inp.fragment_sizes(cfg, n)]
    coeffs = [torch.from_numpy(inp.make_fragment(cfg, f, nfs_all[f])).cuda() for f in range(n)]
    # outputs: a ring large enough for every request that can be queued at once
    outs = [torch.empty((m, m, m, m), dtype=torch.complex128, device="cuda") for m in nfs_all]
    arr = inp.make_arrivals(cfg, n)
    free, _ = torch.cuda.mem_get_info()
    ctx.serve_start(max_inflight=2, max_batch=args.max_batch or 16, budget_bytes=int(0.8 * free))
    tickets, sched = [], []
    i = 0
    lat = {}
    pending = set()
    t0 = time.perf_counter()
    while i < n or pending:
        now = time.perf_counter() - t0
        while i < n and arr[i] <= now:
            t = ctx.submit(coeffs[i], outs[i], args.prec)
            tickets.append(t)
            sched.append(arr[i])
            pending.add(t)
            i += 1
        for t in list(pending):
            st, _ = ctx.poll(t)
            if st == "DONE":
                lat[t] = time.perf_counter() - t0
                pending.discard(t)
            elif st in ("FAILED", "CANCELLED"):
                raise RuntimeError("request %d %s: %s" % (t, st, ctx.last_error()))
    wall = time.perf_counter() - t0
    ctx.serve_stop()
    ctx.close()
    # latency from the scheduled arrival to the observed completion
    lm = np.array([1e3 * (lat[t] - s) for t, s in zip(tickets, sched)])
    erisum = float(sum(m ** 4 for m in nfs_all))
    extra = {"arrivals": {"rate_per_s": cfg.arrival_rate, "requests": n, "offered_per_s": n / float(arr[-1]),
                          "served_per_s": n / wall, "fit_kernel_s": t_fk,
                          "latency_from": "scheduled arrival"}}
    cfgd = {"workload": cfg.name, "n_k": cfg.n_k, "kmesh": list(cfg.kmesh), "grid": list(cfg.grid),
            "n_orb": cfg.n_orb, "n_ip": cfg.n_ip, "requests": n, "n_f_range": [cfg.frag_lo, cfg.frag_hi],
            "parallelism": "1 GPU", "step": "one request of the open-arrival run"}
    return erisum / wall, wall, erisum, lm, None, {}, None, extra, cfgd, n


# --------------------------------------------------------------------------
# small cells: one step = fit + kernel + every fragment
# --------------------------------------------------------------------------
def poisson_sweep(ctx, inp, cfg, cdev, outs, prec, rates, n):
    """Open arrivals: requests for the step's fragments (reused cyclically)
    submitted one at a time at seeded Poisson arrival times while earlier
    ones run; per rate the offered and served rates and the p50 / p99
    latency from the scheduled arrival to the observed completion."""
    import numpy as np
    rows = []
    for rate in rates:
        arr = inp.make_arrivals(cfg, n, rate)
        tickets, sched, pending, done = [], [], set(), {}
        i = 0
        t0 = time.perf_counter()
        while i < n or pending:
            now = time.perf_counter() - t0
            while i < n and arr[i] <= now:
                f = i % len(cdev)
                t = ctx.submit_n([cdev[f]], [outs[f]], prec)[0]
                tickets.append(t)
                sched.append(arr[i])
                pending.add(t)
                i += 1
            for t in list(pending):
                st, _ = ctx.poll(t)
                if st == "DONE":
                    done[t] = time.perf_counter() - t0
                    pending.discard(t)
                elif st in ("FAILED", "CANCELLED"):
                    raise RuntimeError("request %d %s: %s" % (t, st, ctx.last_error()))
        wall = time.perf_counter() - t0
        lm = 1e3 * np.array([done[t] - s for t, s in zip(tickets, sched)])
        rows.append({"rate_per_s": rate, "requests": n, "offered_per_s": n / float(arr[-1]),
                     "served_per_s": n / wall, "p50_ms": float(np.percentile(lm, 50)),
                     "p99_ms": float(np.percentile(lm, 99)), "latency_from": "scheduled arrival"})
        log("poisson %g/s: p50 %.2f ms, p99 %.2f ms" % (rate, rows[-1]["p50_ms"], rows[-1]["p99_ms"]))
    return rows


def run_whole(args, cfg, pkg, inp, np, torch):
    d = inp.make_inputs(cfg)
    frags = inp.make_fragments(cfg)
    nfs = [int(f.shape[2]) for f in frags]
    log("inputs %s: N_k=%d grid=%s n_orb=%d n_ip=%d fragments=%d"
        % (cfg.name, cfg.n_k, cfg.grid, cfg.n_orb, cfg.n_ip, len(frags)))
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, d.orbitals, d.ip_index)
    cdev = [torch.from_numpy(f).cuda() for f in frags]
    out_mix = [torch.empty((n, n, n, n), dtype=torch.complex128, device="cuda") for n in nfs]
    out_64 = [torch.empty((n, n, n, n), dtype=torch.complex128, device="cuda") for n in nfs]
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    ctx.serve_start(max_inflight=2, max_batch=args.max_batch or len(frags), budget_bytes=int(0.8 * free))

    def step(prec, outs):
        ctx.fit(prec)
        ctx.coulomb_kernel(prec)
        return poll_all(ctx, ctx.submit_n(cdev, outs, prec))

    for i in range(args.warmup):
        step(args.prec, out_mix)
        log("warmup step %d done" % i)
    torch.cuda.synchronize()
    ctx.stage_reset()
    lats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        lats += step(args.prec, out_mix)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log("timed %d steps: %.2f ms/step" % (args.steps, 1e3 * wall / args.steps))
    tot = collect_stages(ctx, STAGES + [s + "_kernel" for s in FRAG_STAGES])
    erisum = float(sum(n ** 4 for n in nfs)) * args.steps
    roof = roofline_entry(ctx, tot, cfg, nfs * args.steps, args.prec, args.steps)
    wfac = bool(ctx.stats().get("w_factor"))
    stages = stage_rows(tot, cfg, nfs * args.steps, args.prec, args.steps, 1, wfac and args.prec != "fp64")
    extra = {"w_factor": wfac}
    rates = [float(r) for r in (args.poisson_rates if args.poisson_rates is not None else "200,1000,4000").split(",")
             if r.strip()]
    if rates:
        extra["poisson"] = poisson_sweep(ctx, inp, cfg, cdev, out_mix, args.prec, rates, args.poisson_n)
    if not args.no_fp64_ref and args.prec != "fp64":
        step("fp64", out_64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nfp = 3
        for _ in range(nfp):
            step("fp64", out_64)
        torch.cuda.synchronize()
        t64 = (time.perf_counter() - t0) / nfp
        errs = [float((a - b).abs().max().item()) for a, b in zip(out_mix, out_64)]
        extra["fp64_ms_per_step"] = 1e3 * t64
        extra["speedup_vs_fp64"] = t64 / (wall / args.steps)
        extra["max_err_eh"] = max(errs)
        extra["max_err_eh_per_result"] = {"min": min(errs), "median": float(np.median(errs)),
                                          "max": max(errs), "n": len(errs)}
        extra["err_bound_eh"] = 1e-6
        extra["err_reference"] = "GPU FP64 path, same fragments"
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(d, nfs, args.cpu_budget_s)
    if not args.no_graph and args.prec != "fp64":
        ctx.serve_stop()
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
    else:
        ctx.serve_stop()
    ctx.close()
    cfgd = {"workload": cfg.name, "n_k": cfg.n_k, "kmesh": list(cfg.kmesh), "grid": list(cfg.grid),
            "n_orb": cfg.n_orb, "n_ip": cfg.n_ip, "fragments": len(nfs), "n_f_range": [min(nfs), max(nfs)],
            "eris_per_step": erisum / args.steps, "parallelism": "1 GPU",
            "step": "fit + Coulomb kernel + every fragment of the cell"}
    return erisum / wall, wall, erisum, 1e3 * np.asarray(lats), roof, stages, cpu, extra, cfgd, len(nfs) * args.steps


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
    if cfg.n_k >= STREAM_MIN_NK and args.arrivals > 0:
        res = run_arrivals(args, cfg, pkg, inp, np, torch)
    elif cfg.n_k >= STREAM_MIN_NK:
        res = run_stream(args, cfg, pkg, inp, np, torch)
    else:
        res = run_whole(args, cfg, pkg, inp, np, torch)
    value, wall, erisum, lat_ms, roof, stages, cpu, extra, cfgd, nreq = res
    if not args.no_peaks:
        pk = measured_peaks(torch)
        extra["measured_peaks"] = pk
        if roof and roof["unit"] == "TFLOP/s":
            ref = pk["gemm_bf16_TFLOPs"] if args.prec == "bf16x3" else pk["gemm_%s_TFLOPs" % args.prec]
            roof["frac_of_measured_peak"] = roof["achieved"] / ref
        elif roof:
            roof["frac_of_measured_peak"] = roof["achieved"] / pk["hbm_copy_GBps"]
    steps = args.steps if not (cfg.n_k >= STREAM_MIN_NK and args.arrivals > 0) else nreq
    out = {
        "metric": "fragment ERIs/s + p50/p99 latency, mixed vs FP64 at <=1e-6 Eh max error",
        "value": value,
        "unit": "ERIs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": cfgd,
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "n": int(lat_ms.size)},
        "fragments_per_s": nreq / wall,
        "roofline": roof,
        "stages": stages,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
