"""Launch tiling of the fragment contraction (isdf_autotune, isdf_set_tiling),
through the C ABI: every tiling the tuner may pick meets the mixed bound
against the FP64 oracle (1e-6 Eh), the tuner's choice is one of its
candidates and sticks to the context, a graph captured after tuning equals
the eager batch with that tiling bit for bit, and bad tilings are refused.
The ring pipeline of the bf16 fragment GEMMs (one workgroup a CU) issues the
same MFMAs in the same order per accumulator as the two-stage pipeline, so
its results are equal bit for bit."""
import numpy as np
import pytest

import isdf_inputs as inp
from oracle import kpoint as ko

pytestmark = pytest.mark.gpu

MIXED_EH = 1e-6


@pytest.mark.parametrize("name", ["t_small_k3", "t_m4_k16"])
def test_every_tiling_within_bound(name):
    import torch
    import paper_2601_16379_amd as pkg
    print("tiling case", name, flush=True)
    d = inp.make_inputs(name)
    cfg = d.cfg
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    frags = inp.make_fragments(cfg)
    ref = [ko.fragment_eri(x, cf, w, cfg.kmesh) for cf in frags]
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, d.orbitals, d.ip_index)
    ctx.fit("bf16x3")
    ctx.coulomb_kernel("bf16x3")
    cdev = [torch.from_numpy(f).cuda() for f in frags]
    nh = (cfg.n_k + sum(1 for q in range(cfg.n_k) if _self_conj(q, cfg.kmesh))) // 2
    for nl in (1, 2, 3):
        for wg in (1, 2, 8):
            ctx.set_tiling((nh + nl - 1) // nl, wg)
            got = ctx.fragment_eri(cdev, "bf16x3")
            for f in range(len(frags)):
                err = float(np.max(np.abs(got[f].cpu().numpy() - ref[f])))
                assert err < MIXED_EH, (nl, wg, f, err)
    out = [torch.empty((f.shape[2],) * 4, dtype=torch.complex128, device="cuda") for f in frags]
    rep = ctx.autotune(cdev, out, "bf16x3")
    print(name, rep, flush=True)
    assert rep["n_tried"] >= 4 and rep["ms"] > 0 and rep["ms_default"] > 0
    assert rep["wg_per_cu"] in (1, 2, 4, 8)
    g0 = ctx.stats()["eri_qgroup_initial"]
    assert 1 <= g0 <= 12
    n_init = -(-nh // g0)                   # launches of the initial tiling (balanced groups)
    assert rep["eri_qgroup"] in {-(-nh // nl) for nl in (1, 2, 3, n_init)}
    assert ctx.stats()["eri_qgroup"] == rep["eri_qgroup"] and ctx.stats()["wg_per_cu"] == rep["wg_per_cu"]
    assert rep["ms"] <= rep["ms_default"]
    eager = [e.cpu().numpy() for e in ctx.fragment_eri(cdev, "bf16x3")]
    for f in range(len(frags)):
        assert float(np.max(np.abs(eager[f] - ref[f]))) < MIXED_EH
    g = ctx.graph(cdev, out, "bf16x3")
    for e in out:
        e.zero_()
    g.launch()
    for f in range(len(frags)):
        assert np.array_equal(out[f].cpu().numpy(), eager[f]), f
    g.close()
    for bad in ((0, 2), (4, -1), (4, 9)):
        with pytest.raises(pkg.IsdfError) as e:
            ctx.set_tiling(*bad)
        assert e.value.status == -1
    ctx.close()


def _self_conj(q, kmesh):
    m1, m2, m3 = kmesh
    j = (q // (m2 * m3), (q // m3) % m2, q % m3)
    return all((2 * jj) % m == 0 for jj, m in zip(j, kmesh))


@pytest.mark.parametrize("name", ["t_small_k3", "t_m4_k16", "t_k6_cube", "t_cond_k8"])
@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
def test_ring_pipeline_equals_two_stage_bitwise(name, prec):
    import torch
    import paper_2601_16379_amd as pkg
    print("ring case", name, prec, flush=True)
    d = inp.make_inputs(name)
    cfg = d.cfg
    frags = inp.make_fragments(cfg)
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, d.orbitals, d.ip_index)
    ctx.fit(prec)
    ctx.coulomb_kernel(prec)
    cdev = [torch.from_numpy(f).cuda() for f in frags]
    nh = (cfg.n_k + sum(1 for q in range(cfg.n_k) if _self_conj(q, cfg.kmesh))) // 2
    nl = -(-nh // ctx.stats()["eri_qgroup_initial"])
    g = -(-nh // nl)                        # the initial tiling's classes per launch
    ctx.set_tiling(g, 2)
    two = [e.cpu().numpy() for e in ctx.fragment_eri(cdev, prec)]
    ctx.set_tiling(g, 1)
    ring = [e.cpu().numpy() for e in ctx.fragment_eri(cdev, prec)]
    ring2 = [e.cpu().numpy() for e in ctx.fragment_eri(cdev, prec)]
    for f in range(len(frags)):
        assert np.array_equal(ring[f], two[f]), (f, frags[f].shape[2])
        assert np.array_equal(ring2[f], two[f]), f
    ctx.close()


def test_initial_classes_per_launch():
    """The initial classes per ERI launch: the most, at most 12, whose K range
    of one operand row (8 bytes an element) stays within 72 KB: 12 up to 768
    interpolation points, 11 at 800, 8 at 1040."""
    import paper_2601_16379_amd as pkg
    rng = np.random.default_rng(5)
    lat = 6.0 * np.eye(3)
    grid = (16, 16, 16)
    orb = (rng.standard_normal((1, 4, 4096)) + 1j * rng.standard_normal((1, 4, 4096))).astype(np.complex128)
    for n_ip, want in ((520, 12), (768, 12), (800, 11), (1040, 8)):
        ctx = pkg.Isdf(lat, grid, (1, 1, 1), orb, np.arange(n_ip, dtype=np.int32) * 3)
        st = ctx.stats()
        print("n_ip %d: %d classes a launch" % (n_ip, st["eri_qgroup_initial"]), flush=True)
        assert st["eri_qgroup_initial"] == want and st["eri_qgroup"] == want and st["wg_per_cu"] == 2
        ctx.close()
