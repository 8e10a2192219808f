"""The serving loop (continuous batching): requests that arrive while others
run are admitted into later batches, several batches are in flight on their
own streams, and every result equals the same fragment computed alone."""
import time

import numpy as np
import pytest

import isdf_inputs as inp
from oracle import kpoint as ko

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    import paper_2601_16379_amd as pkg
    d = inp.make_inputs("t_mid_k4")
    cfg = d.cfg
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, d.orbitals, d.ip_index)
    ctx.fit()
    ctx.coulomb_kernel("fp64")
    rng = np.random.default_rng(1)
    sizes = rng.integers(3, 17, size=24)
    frags = [inp.make_fragment(cfg, 100 + i, int(n)) for i, n in enumerate(sizes)]
    alone = {}
    for prec in ("fp64", "bf16x3"):
        alone[prec] = [ctx.fragment_eri([f], prec)[0] for f in frags]
    # the FP64 oracle of every fragment (eqs. (2)-(8), (19)-(20))
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    ref = [ko.fragment_eri(x, f, w, cfg.kmesh) for f in frags]
    return ctx, frags, alone, ref


def _wait(ctx, tickets, timeout=60.0):
    t0 = time.time()
    states = {}
    while len(states) < len(tickets):
        for t in tickets:
            if t in states:
                continue
            st, lat = ctx.poll(t)
            if st in ("DONE", "FAILED", "CANCELLED"):
                states[t] = (st, lat)
        assert time.time() - t0 < timeout, "requests did not finish"
    return states


def test_each_result_equals_alone_in_the_mix(served):
    ctx, frags, alone, ref = served
    # at most 5 requests per batch, two batches in flight
    ctx.serve_start(max_inflight=2, max_batch=5, budget_bytes=512 << 20)
    try:
        rng = np.random.default_rng(2)
        outs, tickets, precs = [], [], []
        for i, f in enumerate(frags):
            prec = "fp64" if i % 3 else "bf16x3"
            n = f.shape[2]
            o = np.empty((n, n, n, n), dtype=np.complex128)
            tickets.append(ctx.submit(f, o, prec))
            outs.append(o)
            precs.append(prec)
            time.sleep(float(rng.exponential(0.002)))   # arrivals while others run
        states = _wait(ctx, tickets)
        for i, t in enumerate(tickets):
            st, lat = states[t]
            assert st == "DONE"
            assert lat > 0
            assert np.array_equal(outs[i], alone[precs[i]][i]), i
        s = ctx.stats()
        assert s["batches"] >= 3          # requests were split over several batches
    finally:
        ctx.serve_stop()


def test_submit_n_one_batch_and_latency(served):
    ctx, frags, alone, ref = served
    ctx.serve_start(max_inflight=1, max_batch=len(frags), budget_bytes=8 << 30)
    try:
        outs = [np.empty((f.shape[2],) * 4, dtype=np.complex128) for f in frags]
        before = ctx.stats()["batches"]
        tickets = ctx.submit_n(frags, outs, "fp64")
        states = _wait(ctx, tickets)
        assert all(states[t][0] == "DONE" for t in tickets)
        assert ctx.stats()["batches"] - before == 1
        lats = [states[t][1] for t in tickets]
        assert max(lats) - min(lats) < 1e-3      # one batch: same completion
        for o, a in zip(outs, alone["fp64"]):
            assert np.array_equal(o, a)
    finally:
        ctx.serve_stop()


def test_cancel_unknown_and_budget_errors(served):
    import paper_2601_16379_amd as pkg
    ctx, frags, alone, ref = served
    # 64 MB per batch: fragments of up to 16 orbitals fit (~21 MB each in
    # FP64), one of 40 (~125 MB) does not
    ctx.serve_start(max_inflight=1, max_batch=1, budget_bytes=64 << 20)
    try:
        f = frags[0]
        n = f.shape[2]
        outs = [np.empty((n,) * 4, dtype=np.complex128) for _ in range(12)]
        tickets = [ctx.submit(f, o, "fp64") for o in outs]
        cancelled = None
        for t in reversed(tickets):
            st, _ = ctx.poll(t)
            if st == "QUEUED":
                ctx.cancel(t)
                cancelled = t
                break
        states = _wait(ctx, tickets)
        if cancelled is not None:
            assert states[cancelled][0] == "CANCELLED"
        for t, o in zip(tickets, outs):
            if t != cancelled:
                assert states[t][0] == "DONE"
                assert np.array_equal(o, alone["fp64"][0])
        with pytest.raises(pkg.IsdfError) as e:
            ctx.poll(10 ** 12)
        assert e.value.status == -7
        big = inp.make_fragment(ctx_cfg(), 999, 40)
        with pytest.raises(pkg.IsdfError) as e:
            ctx.submit(big, np.empty((40,) * 4, dtype=np.complex128), "fp64")
        assert e.value.status == -2
    finally:
        ctx.serve_stop()


def ctx_cfg():
    return inp.get_config("t_mid_k4")


def test_refit_while_serving_idle(served):
    ctx, frags, alone, ref = served
    ctx.serve_start(max_inflight=2, max_batch=8, budget_bytes=8 << 30)
    try:
        ctx.fit()                  # idle: allowed
        ctx.coulomb_kernel("fp64")
        o = np.empty((frags[1].shape[2],) * 4, dtype=np.complex128)
        t = ctx.submit(frags[1], o, "fp64")
        _wait(ctx, [t])
        assert np.array_equal(o, alone["fp64"][1])
    finally:
        ctx.serve_stop()


def test_served_results_match_the_oracle(served):
    """Every served result against the FP64 oracle: FP64 within 1e-10
    relative, bf16x3 within 1e-6 Eh."""
    ctx, frags, alone, ref = served
    ctx.serve_start(max_inflight=2, max_batch=6, budget_bytes=1 << 30)
    try:
        outs, tickets, precs = [], [], []
        rng = np.random.default_rng(4)
        for i, f in enumerate(frags):
            prec = "bf16x3" if i % 2 else "fp64"
            n = f.shape[2]
            o = np.empty((n, n, n, n), dtype=np.complex128)
            tickets.append(ctx.submit(f, o, prec, priority=int(rng.integers(0, 3))))
            outs.append(o)
            precs.append(prec)
        states = _wait(ctx, tickets)
        assert all(states[t][0] == "DONE" for t in tickets)
        for o, r, p in zip(outs, ref, precs):
            if p == "fp64":
                assert float(np.max(np.abs(o - r)) / np.max(np.abs(r))) < 1e-10
            else:
                assert float(np.max(np.abs(o - r))) < 1e-6
    finally:
        ctx.serve_stop()


def test_refit_right_after_submit_is_busy_or_exact(served):
    """A refit issued right after a submit either is refused (the request is
    queued or in flight) or runs after the request's batch completed: the
    served result always equals the fragment computed alone."""
    import paper_2601_16379_amd as pkg
    ctx, frags, alone, ref = served
    ctx.serve_start(max_inflight=2, max_batch=8, budget_bytes=8 << 30)
    try:
        busy = 0
        for i in range(6):
            f = frags[i]
            n = f.shape[2]
            o = np.empty((n, n, n, n), dtype=np.complex128)
            t = ctx.submit(f, o, "fp64")
            try:
                ctx.fit()
                ctx.coulomb_kernel("fp64")
            except pkg.IsdfError as e:
                assert e.status == -6          # ISDF_E_BUSY
                busy += 1
            st = _wait(ctx, [t])[t][0]
            if st == "DONE":
                assert np.array_equal(o, alone["fp64"][i])
            else:
                # admitted only after a refit cleared W^q and before the new
                # kernel existed: the request fails, it never returns stale data
                assert st == "FAILED"
        # leave the context with a current kernel
        ctx.fit()
        ctx.coulomb_kernel("fp64")
    finally:
        ctx.serve_stop()


def test_priority_orders_admission(served):
    """With one batch of one request at a time, queued requests are admitted
    by priority (higher first), submission order among equals."""
    ctx, frags, alone, ref = served
    ctx.serve_start(max_inflight=1, max_batch=1, budget_bytes=1 << 30)
    try:
        f0 = frags[0]
        n0 = f0.shape[2]
        blocker = np.empty((n0,) * 4, dtype=np.complex128)
        tickets = [ctx.submit(f0, blocker, "fp64")]
        order = [0, 2, 1, 2, 0]
        outs, t_sub = [], []
        for j, p in enumerate(order):
            f = frags[1 + j]
            n = f.shape[2]
            o = np.empty((n,) * 4, dtype=np.complex128)
            outs.append(o)
            t_sub.append(time.perf_counter())
            tickets.append(ctx.submit(f, o, "fp64", priority=p))
        _wait(ctx, tickets)
        # completion time = submission + latency (both on the host clock)
        done = {j: t_sub[j] + ctx.poll(tickets[1 + j])[1] for j in range(len(order))}
        # completion order follows (priority desc, submission asc)
        expect = sorted(range(len(order)), key=lambda j: (-order[j], j))
        done_order = sorted(range(len(order)), key=lambda j: done[j])
        assert done_order == expect, (done_order, expect)
        for j, o in enumerate(outs):
            assert np.array_equal(o, alone["fp64"][1 + j])
    finally:
        ctx.serve_stop()
