"""Parity of the gfx950 library (through the C ABI) with the FP64 oracle.

Bars: integer / index work bit-exact; FP64 path within 1e-10 relative
(max |diff| / max |oracle|) per result; mixed paths within 1e-6 Eh absolute
on fragment ERIs.  Small cases span several 64-wide GEMM tiles with ragged
tails (N_IP = 150, pair counts up to 196) and every mesh shape used by the
workloads (Gamma only, even and odd axes)."""
import numpy as np
import pytest

import isdf_inputs as inp
from oracle import geometry as geo
from oracle import kpoint as ko
from oracle import supercell as sc

pytestmark = pytest.mark.gpu

FP64_REL = 1e-10


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _ctx(d, **kw):
    import paper_2601_16379_amd as pkg
    return pkg.Isdf(d.lattice, d.cfg.grid, d.cfg.kmesh, d.orbitals, d.ip_index, **kw)


class Case:
    """GPU and oracle fits of one small configuration (module cache)."""

    def __init__(self, name):
        self.d = inp.make_inputs(name)
        cfg = self.d.cfg
        print("case", name, flush=True)
        self.x, self.pi, self.eta, self.w = ko.fit_and_kernel(
            self.d.orbitals, self.d.ip_index, self.d.lattice, cfg.grid, cfg.kmesh)
        self.ctx = _ctx(self.d)
        self.ctx.fit()
        self.g_pi = np.stack([self.ctx.get_metric(q) for q in range(cfg.n_k)])
        self.g_x = np.stack([self.ctx.get_ivs(k) for k in range(cfg.n_k)])
        self.g_eta = np.stack([self.ctx.get_rhs(q) for q in range(cfg.n_k)])
        self.ctx.coulomb_kernel("fp64")
        self.g_w = np.stack([self.ctx.get_kernel(q) for q in range(cfg.n_k)])


_CASES = {}


def case(name):
    if name not in _CASES:
        _CASES[name] = Case(name)
    return _CASES[name]


SMALL = ["t_tiny_k1", "t_small_k2", "t_small_k3", "t_mid_k4"]


@pytest.mark.parametrize("name", SMALL)
def test_ivs_bit_exact(name):
    c = case(name)
    assert np.array_equal(c.g_x, c.x)


@pytest.mark.parametrize("name", SMALL)
def test_metric_parity(name):
    c = case(name)
    assert _rel(c.g_pi, c.pi) < 1e-12


@pytest.mark.parametrize("name", SMALL)
def test_rhs_parity(name):
    c = case(name)
    assert _rel(c.g_eta, c.eta) < 1e-12


@pytest.mark.parametrize("name", SMALL)
def test_kernel_parity(name):
    """W^q itself where Pi^q has full rank; where it is singular W^q is not
    unique and the unique quantity A W A^H (A = pair products of the
    interpolating vectors, the fitted Coulomb matrix of orbital pairs) is
    compared instead."""
    c = case(name)
    cfg = c.d.cfg
    ranks = c.ctx.stats()["rank"]
    for q in range(cfg.n_k):
        ev = np.linalg.eigvalsh(c.pi[q])
        assert ranks[q] == int((ev > 1e-13 * ev.max()).sum())
    if all(r == cfg.n_ip for r in ranks):
        for q in range(cfg.n_k):
            # forward-error bound of the two-sided solve: 4 n eps cond(Pi^q)
            tol = max(FP64_REL, 4 * cfg.n_ip * np.finfo(float).eps * np.linalg.cond(c.pi[q]))
            assert _rel(c.g_w[q], c.w[q]) < tol
    kq = geo.k_plus_q(cfg.kmesh)
    for q in range(cfg.n_k):
        for k in range(min(cfg.n_k, 3)):
            # rows: pairs conj(phi^k_mu) phi^{k+q}_nu at the interpolation points
            a = (c.x[k].conj()[:, :, None] * c.x[kq[k, q]][:, None, :]).reshape(cfg.n_ip, -1).T
            assert _rel(a @ c.g_w[q] @ a.conj().T, a @ c.w[q] @ a.conj().T) < FP64_REL


@pytest.mark.parametrize("name", SMALL)
def test_fragment_eri_fp64_parity(name):
    c = case(name)
    cfg = c.d.cfg
    frags = inp.make_fragments(cfg)
    out = c.ctx.fragment_eri(frags, "fp64")
    for f, cf in enumerate(frags):
        ref = ko.fragment_eri(c.x, cf, c.w, cfg.kmesh)
        assert _rel(out[f], ref) < FP64_REL, (f, cf.shape)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name", ["t_small_k3", "t_mid_k4"])
def test_fragment_eri_mixed_within_1e6(name, prec):
    c = case(name)
    cfg = c.d.cfg
    frags = inp.make_fragments(cfg)
    out = c.ctx.fragment_eri(frags, prec)
    for f, cf in enumerate(frags):
        ref = ko.fragment_eri(c.x, cf, c.w, cfg.kmesh)
        err = float(np.max(np.abs(out[f] - ref)))
        print("%s %s frag %d n_f %d max|dV| %.3e Eh" % (name, prec, f, cf.shape[2], err))
        assert err < 1e-6


def test_batch_equals_alone_bitwise():
    c = case("t_mid_k4")
    frags = inp.make_fragments(c.d.cfg)
    batch = c.ctx.fragment_eri(frags, "fp64")
    for f in (0, len(frags) - 1):
        alone = c.ctx.fragment_eri([frags[f]], "fp64")[0]
        assert np.array_equal(alone, batch[f])


def test_device_pointers_match_host():
    import torch
    c = case("t_small_k3")
    frags = inp.make_fragments(c.d.cfg)
    host = c.ctx.fragment_eri(frags, "fp64")
    dev = c.ctx.fragment_eri([torch.from_numpy(f).cuda() for f in frags], "fp64")
    torch.cuda.synchronize()
    for h, g in zip(host, dev):
        assert np.array_equal(h, g.cpu().numpy())


def test_workload1_exact_eris_rank_deficient_metric():
    """16^3 Gamma cell, 8 real orbitals, 64 points: Pi has rank 36, the
    pivoted factorisation finds it and the ERIs equal FFT-Poisson."""
    d = inp.make_inputs("c1_gamma_16")
    cfg = d.cfg
    ctx = _ctx(d)
    ctx.fit()
    assert ctx.stats()["rank"] == [36]
    ctx.coulomb_kernel("fp64")
    coeffs = inp.make_fragment(cfg, 0, 8)
    v = ctx.fragment_eri([coeffs], "fp64")[0]
    phi_s = sc.supercell_orbitals(d.orbitals, cfg.grid, cfg.kmesh)
    psi = sc.fragment_orbitals(phi_s, coeffs)
    exact = sc.exact_eri(psi, d.lattice, cfg.grid, cfg.kmesh)
    assert np.max(np.abs(v - exact)) < 1e-12


def test_no_pivot_singular_metric_is_numeric_error():
    import paper_2601_16379_amd as pkg
    d = inp.make_inputs("c1_gamma_16")
    ctx = _ctx(d, no_pivot=True)
    with pytest.raises(pkg.IsdfError) as e:
        ctx.fit()
    assert e.value.status == -4
    assert "q = 0" in str(e.value)


def test_state_errors():
    import paper_2601_16379_amd as pkg
    d = inp.make_inputs("t_tiny_k1")
    ctx = _ctx(d)
    with pytest.raises(pkg.IsdfError) as e:
        ctx.coulomb_kernel()
    assert e.value.status == -3
    ctx.fit()
    with pytest.raises(pkg.IsdfError) as e:
        ctx.fragment_eri([inp.make_fragment(d.cfg, 0, 2)])
    assert e.value.status == -3
    with pytest.raises(pkg.IsdfError) as e:
        ctx.get_kernel(0)
    assert e.value.status == -3


@pytest.mark.parametrize("name", ["t_grid10_k1", "t_grid18_k2", "t_grid20_k3", "t_grid36_k2",
                                  "t_grid40_k1"])
def test_grid_fft_sizes_kernel_and_eri(name):
    """Every radix pair of the unit-cell FFT (10 = 2x5, 18 = 3x6, 20 = 4x5,
    36 = 6x6, 40 = 5x8) through W^q and the fragment ERIs."""
    d = inp.make_inputs(name)
    cfg = d.cfg
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    ctx = _ctx(d)
    ctx.fit()
    ctx.coulomb_kernel("fp64")
    assert ctx.stats()["rank"] == [cfg.n_ip] * cfg.n_k
    for q in range(cfg.n_k):
        tol = max(FP64_REL, 4 * cfg.n_ip * np.finfo(float).eps * np.linalg.cond(pi[q]))
        assert _rel(ctx.get_kernel(q), w[q]) < tol, q
    frags = inp.make_fragments(cfg)
    out = ctx.fragment_eri(frags, "fp64")
    for f, cf in enumerate(frags):
        assert _rel(out[f], ko.fragment_eri(x, cf, w, cfg.kmesh)) < FP64_REL


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name", ["t_small_k3", "t_mid_k4", "t_grid10_k1", "t_grid18_k2", "t_grid20_k3",
                                  "t_grid36_k2", "t_m4_k16"])
def test_mixed_kernel_and_eri_within_1e6(name, prec):
    """The mixed-precision Coulomb path (one-pass FP32 FFT on cubic grids up to
    32^3 -- here 10, 12, 16, 18, 20 -- the two-pass FFT above that -- 36 --,
    V^q from FP32 / bf16 hi+lo operands) through the fragment ERIs, against
    the FP64 oracle."""
    c = case(name)
    cfg = c.d.cfg
    ctx = _ctx(c.d)
    ctx.fit(prec)
    ctx.coulomb_kernel(prec)
    frags = inp.make_fragments(cfg)
    out = ctx.fragment_eri(frags, prec)
    worst = 0.0
    for f, cf in enumerate(frags):
        ref = ko.fragment_eri(c.x, cf, c.w, cfg.kmesh)
        worst = max(worst, float(np.max(np.abs(out[f] - ref))))
    print("%s %s kernel + ERIs max|dV| %.3e Eh" % (name, prec, worst))
    from test_gpu_meshes import known_bf16x3_limit
    known_bf16x3_limit(name, prec, worst)
    assert worst < 1e-6


@pytest.mark.parametrize("name", ["t_tiny_k2", "t_small_k2", "t_mid_k4", "t_grid10_k1", "t_grid18_k2",
                                  "t_grid20_k3", "t_grid36_k2", "t_grid40_k1"])
def test_eta_tilde_elementwise(name):
    """The grid-FFT stage itself (eq. (7) weighting), element by element for
    every q, within 1e-12 of max."""
    c = case(name)
    cfg = c.d.cfg
    ctx = _ctx(c.d)
    ctx.fit("fp64")
    ctx.coulomb_kernel("fp64")
    for q in range(cfg.n_k):
        ref = ko.eta_tilde(c.eta[q], c.d.lattice, cfg.grid, cfg.kmesh, q)
        got = ctx.get_eta_tilde(q)
        assert float(np.max(np.abs(got - ref))) <= 1e-12 * np.abs(ref).max(), q


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name", ["t_mid_k4", "t_grid20_k3", "t_m4_k16"])
def test_fit_and_kernel_are_fp64_in_every_precision(name, prec):
    """The fit and the Coulomb kernel run in FP64 whatever the precision
    (W^q amplifies their rounding by up to cond(Pi^q) on each side): eta,
    eta~ and W^q of a mixed-precision call equal those of an FP64 call bit for
    bit."""
    c = case(name)
    cfg = c.d.cfg
    got = []
    for p in ("fp64", prec):
        ctx = _ctx(c.d)
        ctx.fit(p)
        eta = np.stack([ctx.get_rhs(q) for q in range(cfg.n_k)])
        ctx.coulomb_kernel(p)
        et = np.stack([ctx.get_eta_tilde(q) for q in range(cfg.n_k)])
        w = np.stack([ctx.get_kernel(q) for q in range(cfg.n_k)])
        got.append((eta, et, w))
        ctx.close()
    for a, b in zip(got[0], got[1]):
        assert np.array_equal(a, b)


def test_fp64_fit_then_mixed_kernel_within_1e6():
    """The FP64 eta also feeds the mixed kernel (the grid FFT converts it)."""
    c = case("t_mid_k4")
    cfg = c.d.cfg
    ctx = _ctx(c.d)
    ctx.fit("fp64")
    ctx.coulomb_kernel("bf16x3")
    frags = inp.make_fragments(cfg)
    out = ctx.fragment_eri(frags, "bf16x3")
    for f, cf in enumerate(frags):
        ref = ko.fragment_eri(c.x, cf, c.w, cfg.kmesh)
        assert float(np.max(np.abs(out[f] - ref))) < 1e-6


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("name,qb", [("t_mid_k4", 5), ("t_small_k3", 4), ("t_m4_k16", 5)])
def test_q_batches_equal_resident_bitwise(name, qb, prec):
    """With eta formed per batch of qb classes inside the kernel (ISDF_Q_BATCH)
    every element goes through the same instructions as with eta resident:
    W^q for every q and the ERIs are bitwise equal; eta is then unavailable
    after the fit and eta~ after the kernel."""
    import paper_2601_16379_amd as pkg
    c = case(name)
    cfg = c.d.cfg
    frags = inp.make_fragments(cfg)
    res = []
    for q_batch in (0, qb):
        ctx = _ctx(c.d, q_batch=q_batch)
        ctx.fit(prec)
        if q_batch:
            with pytest.raises(pkg.IsdfError) as e:
                ctx.get_rhs(0)
            assert e.value.status == -3
        ctx.coulomb_kernel(prec)
        if q_batch:
            with pytest.raises(pkg.IsdfError) as e:
                ctx.get_eta_tilde(0)
            assert e.value.status == -3
        w = np.stack([ctx.get_kernel(q) for q in range(cfg.n_k)])
        res.append((w, ctx.fragment_eri(frags, prec)))
        if q_batch:
            # a q-batched kernel released the fit's transient buffers; a
            # second fit allocates them again and repeats the result
            ctx.fit(prec)
            ctx.coulomb_kernel(prec)
            assert np.array_equal(np.stack([ctx.get_kernel(q) for q in range(cfg.n_k)]), w)
        ctx.close()
    assert np.array_equal(res[0][0], res[1][0])
    for a, b in zip(res[0][1], res[1][1]):
        assert np.array_equal(a, b)
