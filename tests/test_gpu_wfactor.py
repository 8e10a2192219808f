"""Factor form of the mixed fragment GEMMs (eq. (19) with W^q = L L^H).

W^q is Hermitian positive semidefinite, so sum_q R^q W^q R^{qH} =
sum_q Y^q Y^{qH} with Y^q = R^q L^q.  With the factor the mixed paths form the
triangular product Y^q instead of U^q = R^q W^q and contract Y with itself.
Checked against the FP64 oracle on every ERI (1e-6 Eh for FP32 and bf16x3,
3e-2 of max |V| for single bf16, the bars of the plain form), against the
plain form of the same context settings (ISDF_W_PLAIN), and: the FP64 path
does not change; a metric of deficient rank (workload 1: Pi^q of rank 36 for
64 points) has a singular W^q and keeps the plain form (its mixed ERIs
equal those of a context with ISDF_W_PLAIN bit for bit)."""
import numpy as np
import pytest

import isdf_inputs as inp
from oracle import kpoint as ko

pytestmark = pytest.mark.gpu

MIXED_EH = 1e-6
BF16_REL = 3e-2


def _ctx(d, **kw):
    import paper_2601_16379_amd as pkg
    return pkg.Isdf(d.lattice, d.cfg.grid, d.cfg.kmesh, d.orbitals, d.ip_index, **kw)


@pytest.mark.parametrize("name", ["t_small_k3", "t_mid_k4", "t_k6_cube", "t_k10_line", "t_cond_k8"])
def test_factor_form_against_oracle_and_plain(name):
    print("case", name, flush=True)
    d = inp.make_inputs(name)
    cfg = d.cfg
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    frags = inp.make_fragments(cfg)
    ref = [ko.fragment_eri(x, cf, w, cfg.kmesh) for cf in frags]
    fac, plain = _ctx(d), _ctx(d, w_plain=True)
    for c in (fac, plain):
        c.fit()
        c.coulomb_kernel("fp64")
    assert fac.stats()["w_factor"] is True
    assert plain.stats()["w_factor"] is False
    for prec in ("fp32", "bf16x3", "bf16"):
        a = fac.fragment_eri(frags, prec)
        b = plain.fragment_eri(frags, prec)
        for i, cf in enumerate(frags):
            vmax = float(np.max(np.abs(ref[i])))
            ea = float(np.max(np.abs(a[i] - ref[i])))
            eb = float(np.max(np.abs(b[i] - ref[i])))
            print("%s %s frag %d n_f %d: factor %.2e Eh, plain %.2e Eh, |factor - plain| %.2e (max|V| %.2e)"
                  % (name, prec, i, cf.shape[2], ea, eb, float(np.max(np.abs(a[i] - b[i]))), vmax))
            if prec == "bf16":
                assert ea < BF16_REL * vmax
            else:
                assert ea < MIXED_EH
    # the FP64 path is the same code in both
    a = fac.fragment_eri(frags, "fp64")
    b = plain.fragment_eri(frags, "fp64")
    for i in range(len(frags)):
        assert np.array_equal(a[i], b[i])
    fac.close()
    plain.close()


def test_rank_deficient_metric_keeps_plain_form():
    d = inp.make_inputs("c1_gamma_16")
    cfg = d.cfg
    ctx, plain = _ctx(d), _ctx(d, w_plain=True)
    for c in (ctx, plain):
        c.fit()
        c.coulomb_kernel("fp64")
    st = ctx.stats()
    print("workload 1: rank", st["rank"][0], "of", cfg.n_ip, "w_factor", st["w_factor"])
    assert st["rank"][0] < cfg.n_ip
    assert st["w_factor"] is False
    frags = inp.make_fragments(cfg)
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    ref = [ko.fragment_eri(x, cf, w, cfg.kmesh) for cf in frags]
    got = ctx.fragment_eri(frags, "fp64")
    for i in range(len(frags)):
        assert float(np.max(np.abs(got[i] - ref[i]))) < 1e-10 * float(np.max(np.abs(ref[i])))
    # the mixed paths are the plain form's, bit for bit
    for prec in ("bf16x3", "bf16", "fp32"):
        a = ctx.fragment_eri(frags, prec)
        b = plain.fragment_eri(frags, prec)
        for i in range(len(frags)):
            assert np.array_equal(a[i], b[i]), (prec, i)
    ctx.close()
    plain.close()


def test_factor_form_blocked_equals_unblocked_bitwise():
    """(pq)-blocked fragments recompute Y of each column block; each output
    element is still summed in the same order."""
    d = inp.make_inputs("t_m4_k16")
    ctx = _ctx(d)
    ctx.fit()
    ctx.coulomb_kernel("fp64")
    assert ctx.stats()["w_factor"] is True
    frags = inp.make_fragments(d.cfg)
    for prec in ("bf16x3", "bf16", "fp32"):
        ref = ctx.fragment_eri(frags, prec)
        blk = ctx.fragment_eri(frags, prec, pair_blocks=4)
        for i in range(len(frags)):
            assert np.array_equal(blk[i], ref[i]), (prec, i)
    ctx.close()
