"""Checkpoint and resume on the GPU: a context restored by isdf_load from the
file isdf_save wrote gives bit-identical X^k, Pi^q, W^q and fragment ERIs
(FP64 and bf16x3, synchronous and served), refuses a refit (it holds no
orbitals), and saves the same bytes again; the header carries the sizes the
format states."""
import struct

import numpy as np
import pytest

import isdf_inputs as inp

pytestmark = pytest.mark.gpu


def test_resumed_context_is_bit_identical(tmp_path):
    import paper_2601_16379_amd as pkg
    d = inp.make_inputs("t_m4_k16")
    cfg = d.cfg
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, d.orbitals, d.ip_index)
    ctx.fit()
    ctx.coulomb_kernel("fp64")
    frags = inp.make_fragments(cfg)
    ref = {p: ctx.fragment_eri(frags, p) for p in ("fp64", "bf16x3")}
    path = tmp_path / "cell.ckp"
    ctx.save(str(path))
    data = path.read_bytes()
    assert data[:8] == b"ISDFCKP1"
    grid = struct.unpack_from("<3i", data, 16)
    kmesh = struct.unpack_from("<3i", data, 28)
    n_orb, n_ip, nh = struct.unpack_from("<3i", data, 40)
    assert (tuple(grid), tuple(kmesh), n_orb, n_ip) == (tuple(cfg.grid), tuple(cfg.kmesh), cfg.n_orb, cfg.n_ip)
    payload = struct.unpack_from("<Q", data, 128)[0]
    assert len(data) == 144 + payload
    assert np.array_equal(np.frombuffer(data, np.int32, n_ip, 144), d.ip_index)

    res = pkg.Isdf.load(str(path))
    for q in range(cfg.n_k):
        assert np.array_equal(res.get_kernel(q), ctx.get_kernel(q))
        assert np.array_equal(res.get_metric(q), ctx.get_metric(q))
    for k in range(cfg.n_k):
        assert np.array_equal(res.get_ivs(k), ctx.get_ivs(k))
    for p in ("fp64", "bf16x3"):
        got = res.fragment_eri(frags, p)
        for a, b in zip(got, ref[p]):
            assert np.array_equal(a, b)
    # served from the restored context
    res.serve_start(max_inflight=2, max_batch=4, budget_bytes=1 << 30)
    try:
        outs = [np.empty((f.shape[2],) * 4, dtype=np.complex128) for f in frags]
        tickets = [res.submit(f, o, "bf16x3") for f, o in zip(frags, outs)]
        import time
        t0 = time.time()
        while any(res.poll(t)[0] != "DONE" for t in tickets):
            assert time.time() - t0 < 60
        for a, b in zip(outs, ref["bf16x3"]):
            assert np.array_equal(a, b)
    finally:
        res.serve_stop()
    with pytest.raises(pkg.IsdfError) as e:
        res.fit()
    assert e.value.status == -3
    path2 = tmp_path / "again.ckp"
    res.save(str(path2))
    assert path2.read_bytes() == data
    res.close()
    ctx.close()
