"""isdf_fragment_eri_static (the entry point for callers that cannot
allocate device memory) through the C ABI: two calls in a row, the second
with a smaller batch, each equal bit for bit to isdf_fragment_eri on the same
fragments (same kernels, same summation order), a (pq)-blocked fragment
among them; a fragment too large for the static array is refused before any
launch, and host pointers are refused."""
import ctypes

import numpy as np
import pytest

import isdf_inputs as inp

pytestmark = pytest.mark.gpu

ISDF_FRAG_DEVICE = 0x1


def _call(ctx, fn, prec, tensors, outs, flags=ISDF_FRAG_DEVICE):
    import paper_2601_16379_amd as pkg
    n = len(tensors)
    nfs = np.array([t.shape[2] for t in tensors], dtype=np.int32)
    cptr = (ctypes.c_void_p * n)(*[t.data_ptr() for t in tensors])
    eptr = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    return getattr(ctx.lib, fn)(ctx.h, pkg.isdf.PRECISIONS[prec], n, nfs.ctypes.data, cptr, eptr, flags)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_static_entry_point_equals_allocating_one(prec):
    import torch
    import paper_2601_16379_amd as pkg
    d = inp.make_inputs("t_mid_k4")
    cfg = d.cfg
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, d.orbitals, d.ip_index)
    ctx.fit(prec)
    ctx.coulomb_kernel(prec)
    rng = np.random.default_rng(3)
    # first call: the workload's fragments plus one of 60 orbitals whose
    # unblocked workspace (R^q and U^q 2 x 55-110 MB, the FP64 contraction
    # 207 MB) exceeds the 252 MiB array, so it runs (pq)-blocked; second
    # call: a smaller batch
    first = inp.make_fragments(cfg) + [inp.make_fragment(cfg, 77, 60)]
    second = [inp.make_fragment(cfg, 90 + i, int(n)) for i, n in enumerate(rng.integers(3, 9, size=3))]
    for batch in (first, second):
        cd = [torch.from_numpy(c).cuda() for c in batch]
        ref = [torch.zeros((c.shape[2],) * 4, dtype=torch.complex128, device="cuda") for c in batch]
        got = [torch.full((c.shape[2],) * 4, float("nan"), dtype=torch.complex128, device="cuda") for c in batch]
        st = _call(ctx, "isdf_fragment_eri", prec, cd, ref)
        assert st == 0, ctx.last_error()
        st = _call(ctx, "isdf_fragment_eri_static", prec, cd, got)
        assert st == 0, ctx.last_error()
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
    # too large for the array even in 32 pair blocks: refused, nothing written
    n = 64                          # its FP64 contraction alone is 268 MB
    big = [torch.from_numpy(inp.make_fragment(cfg, 99, n)).cuda()]
    sentinel = torch.full((n,) * 4, 7.0, dtype=torch.complex128, device="cuda")
    st = _call(ctx, "isdf_fragment_eri_static", prec, big, [sentinel])
    msg = ctx.last_error()
    assert st == -2 and "workspace" in msg, (st, msg)
    torch.cuda.synchronize()
    assert bool((sentinel == 7.0).all())
    # host pointers are refused
    host = [inp.make_fragment(cfg, 5, 4)]
    lib = ctx.lib
    cptr = (ctypes.c_void_p * 1)(host[0].ctypes.data)
    out = np.empty((4,) * 4, dtype=np.complex128)
    eptr = (ctypes.c_void_p * 1)(out.ctypes.data)
    nfs = np.array([4], dtype=np.int32)
    assert lib.isdf_fragment_eri_static(ctx.h, 0, 1, nfs.ctypes.data, cptr, eptr, 0) == -1
    ctx.close()
