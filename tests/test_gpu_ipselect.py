"""Interpolation points by pivoted Cholesky on the GPU (isdf_select_points)
against the oracle's greedy selector.

Pivots are integer results: they must equal the oracle's at every step
whose choice is separated from the runner-up by more than rounding (gap
above 1e-9 of the first residual; the test cells have no closer step, which
is asserted), and each pivot's residual must agree to 1e-10 of the first.
Where the residuals tie exactly (workload 1's symmetric real orbitals) the
pivot order is not unique: there the rank and the exact ERIs on the
selected points are compared instead."""
import numpy as np
import pytest

import isdf_inputs as inp
from oracle import ipselect as ips
from oracle import kpoint as ko
from oracle import supercell as sc

pytestmark = pytest.mark.gpu

GAP = 1e-9      # relative to the first residual
RES = 1e-10


def _select(d, n_ip, device=False):
    import paper_2601_16379_amd as pkg
    import torch
    orb = torch.from_numpy(d.orbitals).cuda() if device else d.orbitals
    ip, res = pkg.select_points(d.cfg.grid, d.cfg.kmesh, orb, n_ip)
    torch.cuda.synchronize()
    return ip, res


def _check_against_oracle(name, gpu_ip, gpu_res, orbitals, n, all_separated=True):
    piv, dmax, lf, d, gap = ips.pivoted_cholesky_points(orbitals, n, with_gaps=True)
    sep = gap > GAP * dmax[0]
    m = n if np.all(sep) else int(np.argmin(sep))
    print("%s: %d pivots, %d separated, min gap %.2e, residual %.3e -> %.3e"
          % (name, n, m, gap.min() / dmax[0], dmax[0], dmax[-1]), flush=True)
    if all_separated:
        assert m == n, "oracle has a near-tie at step %d" % m
    bad = np.nonzero(gpu_ip[:m] != piv[:m])[0]
    assert bad.size == 0, "first differing pivot at step %d" % bad[0]
    assert np.max(np.abs(gpu_res[:m] - dmax[:m])) < RES * dmax[0]


@pytest.mark.parametrize("name", ["t_small_k2", "t_mid_k4", "t_k6_line", "t_k10_line", "t_cond_k8"])
def test_pivots_equal_oracle(name):
    d = inp.make_inputs(name)
    n = d.cfg.n_ip
    ip, res = _select(d, n, device=(name == "t_mid_k4"))
    assert len(set(ip.tolist())) == n
    _check_against_oracle(name, ip, res, d.orbitals, n)


def test_workload1_selection_spans_pair_space():
    """8 real orbitals at Gamma: 36 pair functions, so 36 selected points
    give a full-rank metric and the FFT-Poisson ERIs (ties in the residual
    make the order of equal points arbitrary; the span is not)."""
    import paper_2601_16379_amd as pkg
    d = inp.make_inputs("c1_gamma_16")
    cfg = d.cfg
    ip, res = _select(d, 48)
    assert len(set(ip.tolist())) == 48
    assert res[35] > 1e-8 * res[0]
    assert np.all(res[36:] < 1e-12 * res[0])
    sel = ip[:36].copy()
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, d.orbitals, sel)
    ctx.fit()
    assert ctx.stats()["rank"] == [36]
    ctx.coulomb_kernel("fp64")
    coeffs = inp.make_fragment(cfg, 0, 8)
    v = ctx.fragment_eri([coeffs], "fp64")[0]
    psi = sc.fragment_orbitals(sc.supercell_orbitals(d.orbitals, cfg.grid, cfg.kmesh), coeffs)
    exact = sc.exact_eri(psi, d.lattice, cfg.grid, cfg.kmesh)
    err = float(np.max(np.abs(v - exact)))
    print("workload 1, 36 selected points: max|V - exact| = %.2e Eh" % err)
    assert err < 1e-12
    ctx.close()


def test_selected_points_feed_the_fit():
    """The selected points (in selection order) through the whole path: GPU
    FP64 fragment ERIs against the oracle's on the same points.  The
    conditioning of Pi^q on these points is reported beside that of the
    density-weighted subset: the greedy choice maximises the residual of the
    pair products, not the conditioning of every Pi^q, and on this cell it is
    the larger of the two."""
    import paper_2601_16379_amd as pkg
    d = inp.make_inputs("t_mid_k4")
    cfg = d.cfg
    ip, _ = _select(d, cfg.n_ip)
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, ip, d.lattice, cfg.grid, cfg.kmesh)
    ctx = pkg.Isdf(d.lattice, cfg.grid, cfg.kmesh, d.orbitals, ip)
    ctx.fit()
    ctx.coulomb_kernel("fp64")
    frags = inp.make_fragments(cfg)[:3]
    out = ctx.fragment_eri(frags, "fp64")
    for f, o in zip(frags, out):
        ref = ko.fragment_eri(x, f, w, cfg.kmesh)
        assert float(np.max(np.abs(o - ref)) / np.max(np.abs(ref))) < 1e-10
    ctx.close()
    pi0 = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)[1]
    c_sel = max(np.linalg.cond(p) for p in pi)
    c_rnd = max(np.linalg.cond(p) for p in pi0)
    print("t_mid_k4: max cond(Pi^q) %.2e selected vs %.2e density-weighted subset" % (c_sel, c_rnd))


def test_zero_orbitals_are_a_numeric_error():
    import paper_2601_16379_amd as pkg
    d = inp.make_inputs("t_tiny_k1")
    z = np.zeros_like(d.orbitals)
    with pytest.raises(pkg.IsdfError) as e:
        pkg.select_points(d.cfg.grid, d.cfg.kmesh, z, 4)
    assert e.value.status == -4
    assert "span only 0" in str(e.value)


def test_device_flag_on_host_memory_is_refused():
    import ctypes
    import paper_2601_16379_amd as pkg
    d = inp.make_inputs("t_tiny_k1")
    lib = pkg.load_library()
    g = np.asarray(d.cfg.grid, dtype=np.int32)
    k = np.asarray(d.cfg.kmesh, dtype=np.int32)
    ip = np.zeros(4, dtype=np.int32)
    st = lib.isdf_select_points(g.ctypes.data, k.ctypes.data, d.cfg.n_orb, d.orbitals.ctypes.data, 4,
                                ip.ctypes.data, None, 0x1, None)
    assert st == -1
    assert b"not device memory" in lib.isdf_last_error(None)
    _ = ctypes


@pytest.mark.timeout(600)
def test_workload3_selection_sampled():
    """4x4x4 mesh, 32^3 grid, 26 orbitals: all 520 pivots on the GPU; the
    first 32 against the oracle; every pivot distinct, residuals
    non-increasing (to rounding)."""
    d = inp.make_inputs("c3_k4_32")
    n = d.cfg.n_ip
    ip, res = _select(d, n, device=True)
    assert len(set(ip.tolist())) == n
    assert np.all(res[1:] <= res[:-1] * (1 + 1e-12))
    _check_against_oracle("c3_k4_32", ip, res, d.orbitals, 32)
