"""The serving loop (continuous batching): requests that arrive while others
run are admitted into later batches, several batches are in flight on their
own streams, and every result equals the same fragment computed alone."""
import time

import numpy as np
import pytest

import isdf_inputs as inp

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
    return ctx, frags, alone


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
    ctx, frags, alone = served
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
    ctx, frags, alone = served
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
    ctx, frags, alone = served
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
    ctx, frags, alone = served
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
