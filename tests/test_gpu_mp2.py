"""k-point opposite-spin MP2 on the GPU (isdf_sos_mp2, eqs. (11)-(15))
against the oracle.

Given the GPU's own W^q, the integrand F(tau_n) at every quadrature point
and E_OS must match the oracle's direct k sums at 1e-11 relative (FP64
Green's functions, k transforms and N_IP^3 products); with a fine quadrature
E_OS approaches the closed-form sum over ijab (quadrature error only); on
workload 1, whose points span the pair space, it approaches the MP2 energy
from the supercell's FFT-Poisson ERIs."""
import numpy as np
import pytest

import isdf_inputs as inp
from oracle import kpoint as ko
from oracle import mp2
from oracle import supercell as sc

pytestmark = pytest.mark.gpu


def _ctx(d, **kw):
    import paper_2601_16379_amd as pkg
    return pkg.Isdf(d.lattice, d.cfg.grid, d.cfg.kmesh, d.orbitals, d.ip_index, **kw)


def _fitted(name):
    d = inp.make_inputs(name)
    ctx = _ctx(d)
    ctx.fit()
    ctx.coulomb_kernel("fp64")
    x = ko.ip_values(d.orbitals, d.ip_index)
    w = np.stack([ctx.get_kernel(q) for q in range(d.cfg.n_k)])
    return d, ctx, x, w


@pytest.mark.parametrize("name", ["t_small_k2", "t_small_k3", "t_mid_k4", "t_m4_k16", "t_k6_line",
                                  "t_k10_line", "t_k10_cube"])
def test_os_mp2_against_oracle(name):
    import torch
    d, ctx, x, w = _fitted(name)
    cfg = d.cfg
    c, e, n_occ = inp.make_mo(cfg)
    tau, wt = inp.laplace_grid(6, 1.0)
    cin = torch.from_numpy(c).cuda() if name == "t_mid_k4" else c
    r = ctx.sos_mp2(cin, e, n_occ, tau, wt, per_class=True)
    f_ref = np.array([mp2.os_integrand(x, w, c, e, n_occ, cfg.kmesh, t).real for t in tau])
    e_ref = -np.sum(wt * f_ref)
    ef = np.max(np.abs(r["integrand"] - f_ref) / np.abs(f_ref))
    ee = abs(r["e_os"] - e_ref) / abs(e_ref)
    print("%s: F rel %.2e, E_OS %.6e (rel %.2e)" % (name, ef, r["e_os"], ee))
    assert ef < 1e-11 and ee < 1e-11
    assert np.allclose(r["classes"].sum(axis=1), r["integrand"], rtol=1e-13, atol=0)
    assert r["e_os"] < 0 and abs(r["e_sos_mp2"] - 1.3 * r["e_os"]) < 1e-15 * abs(r["e_os"])
    ctx.close()


def test_os_mp2_converges_to_closed_form():
    d, ctx, x, w = _fitted("t_small_k3")
    cfg = d.cfg
    c, e, n_occ = inp.make_mo(cfg)
    exact = mp2.os_closed_form(x, w, c, e, n_occ, cfg.kmesh)
    tau, wt = inp.laplace_grid(36, 1.0)
    r = ctx.sos_mp2(c, e, n_occ, tau, wt)
    rel = abs(r["e_os"] - exact) / abs(exact)
    print("t_small_k3: E_OS %.10e vs closed form %.10e (rel %.1e)" % (r["e_os"], exact, rel))
    assert rel < 1e-9
    ctx.close()


def test_workload1_os_mp2_equals_fft_poisson():
    d, ctx, x, w = _fitted("c1_gamma_16")
    cfg = d.cfg
    c, e, n_occ = inp.make_mo(cfg)
    no = cfg.n_orb
    psi = sc.fragment_orbitals(sc.supercell_orbitals(d.orbitals, cfg.grid, cfg.kmesh), c)
    eri = sc.exact_eri(psi, d.lattice, cfg.grid, cfg.kmesh)
    occ, vir = np.arange(n_occ), np.arange(n_occ, no)
    v = eri[np.ix_(occ, vir, occ, vir)]
    delta = (e[0][vir][None, :, None, None] - e[0][occ][:, None, None, None]
             + e[0][vir][None, None, None, :] - e[0][occ][None, None, :, None])
    exact = -np.sum(np.abs(v) ** 2 / delta)
    tau, wt = inp.laplace_grid(36, 1.0)
    r = ctx.sos_mp2(c, e, n_occ, tau, wt)
    rel = abs(r["e_os"] - exact) / abs(exact)
    print("workload 1: E_OS %.10e vs FFT-Poisson %.10e (rel %.1e)" % (r["e_os"], exact, rel))
    assert rel < 1e-9
    ctx.close()


def test_os_mp2_errors():
    import paper_2601_16379_amd as pkg
    d = inp.make_inputs("t_tiny_k2")
    ctx = _ctx(d)
    c, e, n_occ = inp.make_mo(d.cfg)
    tau, wt = inp.laplace_grid(4, 1.0)
    with pytest.raises(pkg.IsdfError) as ex:
        ctx.sos_mp2(c, e, n_occ, tau, wt)
    assert ex.value.status == -3
    ctx.fit()
    ctx.coulomb_kernel("fp64")
    bad = e.copy()
    bad[0, 0] = 1.0                      # an occupied energy above the virtual ones
    for args in ((c, bad, n_occ, tau, wt), (c, e, d.cfg.n_orb, tau, wt), (c, e, n_occ, -tau, wt)):
        with pytest.raises(pkg.IsdfError) as ex:
            ctx.sos_mp2(*args)
        assert ex.value.status == -1
    lib = pkg.load_library()
    import ctypes
    eos = ctypes.c_double()
    t = np.ascontiguousarray(tau)
    w_ = np.ascontiguousarray(wt)
    st = lib.isdf_sos_mp2(ctx.h, c.ctypes.data, e.ctypes.data, d.cfg.n_orb, n_occ, t.size, t.ctypes.data,
                          w_.ctypes.data, None, None, ctypes.byref(eos), 0x1)
    assert st == -1
    ctx.close()

