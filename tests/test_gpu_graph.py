"""Fragment batches captured as HIP graphs (isdf_graph_*), through the C ABI.

Every replay must equal the eager isdf_fragment_eri of the same batch bit for
bit (the same kernels on the same data), with the program's own eager work
and synchronisations between replays; coefficients updated in place between
replays are read by the next replay; a replay without a current Coulomb
kernel and host pointers are refused."""
import ctypes

import numpy as np
import pytest

import isdf_inputs as inp

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("name", ["t_small_k3", "t_m4_k16"])
def test_graph_replays_equal_eager(name, prec):
    import torch
    import paper_2601_16379_amd as pkg
    print("graph case", name, prec, flush=True)
    d = inp.make_inputs(name)
    cfg = d.cfg
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, d.orbitals, d.ip_index)
    ctx.fit(prec)
    ctx.coulomb_kernel(prec)
    frags = inp.make_fragments(cfg)
    cdev = [torch.from_numpy(f).cuda() for f in frags]
    out = [torch.empty((f.shape[2],) * 4, dtype=torch.complex128, device="cuda") for f in frags]
    ref = [e.cpu().numpy() for e in ctx.fragment_eri(cdev, prec)]
    g = ctx.graph(cdev, out, prec)
    for rep in range(3):
        for e in out:
            e.zero_()
        # eager work on the context between replays
        other = ctx.fragment_eri(cdev[:1], prec)
        torch.cuda.synchronize()
        assert np.array_equal(other[0].cpu().numpy(), ref[0])
        g.launch()
        for f in range(len(frags)):
            assert np.array_equal(out[f].cpu().numpy(), ref[f]), (rep, f)
    # new coefficients in place: the next replay reads them
    rng = np.random.default_rng(7)
    c0 = frags[0] * (1.0 + 0.5 * rng.standard_normal(frags[0].shape))
    cdev[0].copy_(torch.from_numpy(np.ascontiguousarray(c0)))
    ref2 = [e.cpu().numpy() for e in ctx.fragment_eri(cdev, prec)]
    assert not np.array_equal(ref2[0], ref[0])
    g.launch()
    for f in range(len(frags)):
        assert np.array_equal(out[f].cpu().numpy(), ref2[f]), f
    # a new fit invalidates W^q: the replay is refused until the next kernel
    ctx.fit(prec)
    with pytest.raises(pkg.IsdfError) as e:
        g.launch()
    assert e.value.status == -3
    ctx.coulomb_kernel(prec)
    g.launch()
    for f in range(len(frags)):
        assert np.array_equal(out[f].cpu().numpy(), ref2[f]), f
    g.close()
    ctx.close()


def test_graph_refuses_host_pointers():
    import torch
    import paper_2601_16379_amd as pkg
    d = inp.make_inputs("t_small_k2")
    cfg = d.cfg
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, d.orbitals, d.ip_index)
    ctx.fit()
    ctx.coulomb_kernel("fp64")
    frags = inp.make_fragments(cfg)[:1]
    host_out = np.empty((frags[0].shape[2],) * 4, dtype=np.complex128)
    nf = np.array([frags[0].shape[2]], dtype=np.int32)
    cptr = (ctypes.c_void_p * 1)(frags[0].ctypes.data)
    eptr = (ctypes.c_void_p * 1)(host_out.ctypes.data)
    h = ctypes.c_void_p()
    st = ctx.lib.isdf_graph_create(ctx.h, 0, 1, nf.ctypes.data, cptr, eptr, ctypes.byref(h))
    assert st == -1 and not h.value        # ISDF_E_INVALID
    with pytest.raises(ValueError):
        ctx.graph(frags, [host_out], "fp64")
    cdev = torch.from_numpy(frags[0]).cuda()
    with pytest.raises(ValueError):
        ctx.graph([cdev], [host_out], "fp64")
    ctx.close()
