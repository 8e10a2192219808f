"""Parity at the workloads' own sizes, in the launch configuration the
benchmark times.

Workload 2 (2x2x2 mesh, 24^3 grid, 16 orbitals, 256 points): the whole
oracle runs (all q of Pi, eta and W, the fragment ERIs).  Workload 3
(4x4x4 mesh, 32^3 grid, 26 orbitals, 520 points, 64 fragments): Pi for all
q; eta at sampled grid points of sampled q; W for the q = 0, a generic and a
Brillouin-zone-boundary q; fragment ERIs of the smallest, a median and the
largest fragment from the oracle's eqs. (19)-(20) given the GPU FP64 W^q
(so the fragment step is checked on its own at full size).  Mixed
precision: every result within 1e-6 Eh of the FP64 reference."""
import numpy as np
import pytest

import isdf_inputs as inp
from oracle import geometry as geo
from oracle import kpoint as ko

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _w_tol(pi_q):
    """W^q = Pi^+ V Pi^+ amplifies FP64 rounding (on either side) by the
    condition number of Pi^q: compare W at the forward-error bound of a
    two-sided solve, 4 n eps cond(Pi^q) relative (at least 1e-10).  The
    fragment ERIs, which see W only through the range of Pi, keep 1e-10."""
    n = pi_q.shape[0]
    return max(1e-10, 4 * n * np.finfo(float).eps * np.linalg.cond(pi_q))


def _ctx(d):
    import torch
    import paper_2601_16379_amd as pkg
    return pkg.Isdf(d.lattice, d.cfg.grid, d.cfg.kmesh, torch.from_numpy(d.orbitals).cuda(),
                    torch.from_numpy(d.ip_index).cuda())


def test_workload2_full_oracle():
    d = inp.make_inputs("c2_k2_24")
    cfg = d.cfg
    print("workload 2: oracle fit", flush=True)
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    ctx = _ctx(d)
    ctx.fit()
    assert _rel(np.stack([ctx.get_metric(q) for q in range(cfg.n_k)]), pi) < 1e-12
    assert _rel(np.stack([ctx.get_rhs(q) for q in range(cfg.n_k)]), eta) < 1e-12
    ctx.coulomb_kernel("fp64")
    for q in range(cfg.n_k):
        assert _rel(ctx.get_kernel(q), w[q]) < _w_tol(pi[q]), q
    frags = inp.make_fragments(cfg)
    ref = [ko.fragment_eri(x, f, w, cfg.kmesh) for f in frags]
    out = ctx.fragment_eri(frags, "fp64")
    for o, r in zip(out, ref):
        assert _rel(o, r) < 1e-10
    for prec in ("fp32", "bf16x3"):
        ctx.fit(prec)
        ctx.coulomb_kernel(prec)
        out = ctx.fragment_eri(frags, prec)
        for o, r in zip(out, ref):
            err = float(np.max(np.abs(o - r)))
            print("workload 2 %s max|dV| = %.3e Eh (max|V| = %.3e)" % (prec, err, np.abs(r).max()))
            assert err < 1e-6


@pytest.fixture(scope="module")
def w3():
    d = inp.make_inputs("c3_k4_32")
    ctx = _ctx(d)
    ctx.fit()
    return d, ctx


def test_workload3_metric_all_q(w3):
    d, ctx = w3
    cfg = d.cfg
    x = ko.ip_values(d.orbitals, d.ip_index)
    pi = ko.metric_k(x, cfg.kmesh)
    assert _rel(np.stack([ctx.get_metric(q) for q in range(cfg.n_k)]), pi) < 1e-12
    assert ctx.stats()["rank"] == [cfg.n_ip] * cfg.n_k


QS3 = [0, 21, 42]   # Gamma, generic (1,1,1), Brillouin-zone boundary (2,2,2)


def test_workload3_rhs_sampled(w3):
    d, ctx = w3
    cfg = d.cfg
    x = ko.ip_values(d.orbitals, d.ip_index)
    rng = np.random.default_rng(5)
    ridx = np.sort(rng.choice(cfg.n_g, 700, replace=False))
    ref = ko.rhs(x, d.orbitals, cfg.kmesh, QS3, ridx)
    for i, q in enumerate(QS3):
        g = ctx.get_rhs(q)[:, ridx]
        assert _rel(g, ref[i]) < 1e-12


def test_workload3_kernel_and_fragments(w3):
    d, ctx = w3
    cfg = d.cfg
    x = ko.ip_values(d.orbitals, d.ip_index)
    pi = np.stack([ctx.get_metric(q) for q in range(cfg.n_k)])
    print("workload 3: oracle eta for q = %s on the whole grid" % QS3, flush=True)
    eta = ko.rhs_chunked(x, d.orbitals, cfg.kmesh, QS3)
    w_ref = ko.kernel_v_route(pi, eta, d.lattice, cfg.grid, cfg.kmesh, qs=QS3)
    del eta
    ctx.coulomb_kernel("fp64")
    w_gpu = np.stack([ctx.get_kernel(q) for q in range(cfg.n_k)])
    for i, q in enumerate(QS3):
        err = _rel(w_gpu[q], w_ref[i])
        print("workload 3 W^q q=%d rel %.2e cond(Pi) %.2e" % (q, err, np.linalg.cond(pi[q])))
        assert err < _w_tol(pi[q]), q
    frags = inp.make_fragments(cfg)
    nfs = np.array([f.shape[2] for f in frags])
    order = np.argsort(nfs)
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    ref = {f: ko.fragment_eri(x, frags[f], w_gpu, cfg.kmesh) for f in pick}
    out = ctx.fragment_eri(frags, "fp64")             # the whole batch, as benchmarked
    for f in pick:
        assert _rel(out[f], ref[f]) < 1e-10, f
    # mixed precision (the benchmarked path): W^q and every fragment GEMM in
    # bf16x3 (FP32 eta), against the FP64 results of the same batch
    ctx.fit("bf16x3")
    ctx.coulomb_kernel("bf16x3")
    mixed = ctx.fragment_eri(frags, "bf16x3")
    errs = [float(np.max(np.abs(m - o))) for m, o in zip(mixed, out)]
    print("workload 3 bf16x3 max|dV| over %d fragments: %.3e Eh" % (len(errs), max(errs)))
    assert max(errs) < 1e-6
    for f in pick:
        assert float(np.max(np.abs(mixed[f] - ref[f]))) < 1e-6


# --------------------------------------------------------------------------
# Workloads 4 (6x6x6 mesh, 36^3 grid, 40 orbitals, 800 points) and 5
# (10x10x10 mesh, 40^3 grid, 52 orbitals, 1040 points): sampled checks, the
# plain oracle being too large to run whole (eta of workload 5 is 1 TB).
# * X bit for bit at sampled k; rows of Pi^q at sampled q against the
#   oracle's direct k sums, all rows at three q (q = 0, a generic q, a
#   zone-boundary q);
# * W^q at those q through V^q = Pi^q W^q Pi^q on sampled rows S: the
#   oracle forms eta^q_S on the whole grid and V_SS from it (eqs. (5), (7)),
#   the GPU W^q is contracted with the oracle's rows of Pi^q (eq. (8));
# * fragments of 4 and 8 orbitals from the oracle's eqs. (19)-(20) given the
#   GPU FP64 W^q (the fragment step checked on its own), FP64 and bf16x3;
# * a stream fragment and one of 120 orbitals ((pq)-blocked at this size)
#   in bf16x3 against the GPU FP64 path, 1e-6 Eh.
# --------------------------------------------------------------------------
class Big:
    def __init__(self, name):
        import paper_2601_16379_amd as pkg
        print("%s: generating inputs" % name, flush=True)
        self.d = inp.make_inputs(name)
        cfg = self.d.cfg
        print("%s: creating the context" % name, flush=True)
        self.ctx = pkg.Isdf(self.d.lattice, cfg.grid, cfg.kmesh, self.d.orbitals, self.d.ip_index)
        self.ctx.fit("fp64")
        self.ctx.coulomb_kernel("fp64")
        print("%s: fit + kernel done" % name, flush=True)
        self.x = ko.ip_values(self.d.orbitals, self.d.ip_index)
        self._w = None

    def w_all(self):
        if self._w is None:
            n = self.d.cfg.n_k
            self._w = np.stack([self.ctx.get_kernel(q) for q in range(n)])
        return self._w


BIG = ["c4_k6_36", "c5_k10_40"]


@pytest.fixture(scope="module", params=BIG)
def bigcell(request):
    """One large cell at a time (pytest runs every test of one parameter
    before the next)."""
    b = Big(request.param)
    yield b
    b.ctx.close()


def _qs_of(cfg):
    """q = 0, a generic q and a zone-boundary q (every axis m/2)."""
    m = cfg.kmesh
    gen = geo.mesh_index(np.array([1, 2, 3]) % np.array(m), m)
    bnd = geo.mesh_index(np.array([m[0] // 2, m[1] // 2, m[2] // 2]), m)
    return [0, int(gen), int(bnd)]


@pytest.mark.timeout(900)
def test_large_cell_metric_and_ivs(bigcell):
    b = bigcell
    name = b.d.cfg.name
    cfg = b.d.cfg
    for k in (0, 1, cfg.n_k // 2, cfg.n_k - 1):
        assert np.array_equal(b.ctx.get_ivs(k), b.x[k])
    assert b.ctx.stats()["rank"] == [cfg.n_ip] * cfg.n_k
    rng = np.random.default_rng(7)
    rows = sorted(rng.choice(cfg.n_ip, 6, replace=False).tolist())
    qs = sorted(set(_qs_of(cfg) + rng.choice(cfg.n_k, 13, replace=False).tolist()))
    ref = ko.metric_rows(b.x, cfg.kmesh, rows, qs)
    for i, q in enumerate(qs):
        got = b.ctx.get_metric(q)[rows]
        assert _rel(got, ref[i]) < 1e-12, q


@pytest.mark.timeout(900)
def test_large_cell_select_points(bigcell):
    """All N_IP pivots of the pivoted Cholesky of the pair products at the
    cell's full size; the first three against the oracle (one orbital pass
    each), every pivot distinct, residuals non-increasing to rounding."""
    import time
    import paper_2601_16379_amd as pkg
    from oracle import ipselect as ips
    b = bigcell
    cfg = b.d.cfg
    t0 = time.time()
    ip, res = pkg.select_points(cfg.grid, cfg.kmesh, b.d.orbitals, cfg.n_ip)
    print("%s: %d points selected on the GPU in %.1f s (residual %.3e -> %.3e)"
          % (cfg.name, cfg.n_ip, time.time() - t0, res[0], res[-1]), flush=True)
    assert len(set(ip.tolist())) == cfg.n_ip
    assert np.all(res[1:] <= res[:-1] * (1 + 1e-12))
    piv, dmax, _, _, gap = ips.pivoted_cholesky_points(b.d.orbitals, 3, with_gaps=True)
    print("%s: oracle pivots %s, gaps %s" % (cfg.name, piv.tolist(), (gap / dmax[0]).tolist()), flush=True)
    assert np.all(gap > 1e-9 * dmax[0])
    assert np.array_equal(ip[:3], piv)
    assert np.max(np.abs(res[:3] - dmax)) < 1e-10 * dmax[0]


@pytest.mark.timeout(900)
def test_large_cell_kernel_through_v(bigcell):
    b = bigcell
    name = b.d.cfg.name
    cfg = b.d.cfg
    rng = np.random.default_rng(8)
    rows = sorted(rng.choice(cfg.n_ip, 6, replace=False).tolist())
    qs = _qs_of(cfg)
    print("%s: oracle Pi^q for q = %s" % (name, qs), flush=True)
    pi = ko.metric_rows(b.x, cfg.kmesh, list(range(cfg.n_ip)), qs)
    print("%s: oracle eta^q on rows %s" % (name, rows), flush=True)
    eta_s = ko.rhs_chunked(b.x[:, rows], b.d.orbitals, cfg.kmesh, qs)
    for i, q in enumerate(qs):
        v_ss = ko.coulomb_kernel_of(eta_s[i], b.d.lattice, cfg.grid, cfg.kmesh, q)
        w = b.ctx.get_kernel(q)
        p_s = pi[i][rows]                                  # rows S of Pi^q
        got = p_s @ w @ p_s.conj().T                        # (Pi W Pi)_SS
        cond = np.linalg.cond(pi[i])
        tol = max(1e-10, 8 * cfg.n_ip * np.finfo(float).eps * cond)
        err = _rel(got, v_ss)
        print("%s q=%d: |(Pi W Pi)_SS - V_SS| / max|V_SS| = %.2e (cond(Pi) %.2e, bound %.2e)"
              % (name, q, err, cond, tol))
        assert err < tol, q


@pytest.mark.timeout(900)
def test_large_cell_hf_jk_sampled(bigcell):
    """Coulomb and exchange matrices (eq. (10)) at the cell's full size from
    the GPU's W^q: J at every k against the oracle, K at two sampled k
    against the oracle's direct sum over all q."""
    import torch
    from oracle import hf
    b = bigcell
    cfg = b.d.cfg
    dm = inp.make_density(cfg)
    jd, kd = b.ctx.hf_jk(torch.from_numpy(dm).cuda())
    torch.cuda.synchronize()
    j, k = jd.cpu().numpy(), kd.cpu().numpy()
    del jd, kd
    w = b.w_all()
    ks = [0, cfg.n_k // 2 + 1]
    k_ref = hf.exchange_at(b.x, w, dm, cfg.kmesh, ks)
    j_ref = hf.coulomb(b.x, w, dm)
    ek, ej = _rel(k[ks], k_ref), _rel(j, j_ref)
    print("%s: K at k = %s rel %.2e, J rel %.2e" % (cfg.name, ks, ek, ej), flush=True)
    assert ek < 1e-11 and ej < 1e-11


def _class_of(kmesh, q):
    """Class index of q (classes: the q of the mesh, C order, whose -q is not
    smaller)."""
    mq = geo.minus_q(kmesh)
    reps = [p for p in range(int(np.prod(kmesh))) if mq[p] >= p]
    return reps.index(q if mq[q] >= q else int(mq[q]))


@pytest.mark.timeout(900)
def test_large_cell_sos_mp2_sampled(bigcell):
    """Opposite-spin MP2 at the cell's full size from the GPU's W^q, two
    tau points: the class contributions of q = 0, a generic q and a
    zone-boundary q against the oracle's polarisabilities of those q (their
    k sums over the whole mesh), and the integrand = the sum of the classes."""
    from oracle import mp2
    b = bigcell
    cfg = b.d.cfg
    c, e, n_occ = inp.make_mo(cfg)
    tau = np.array([0.4, 1.3])
    wt = np.array([0.5, 0.5])
    r = b.ctx.sos_mp2(c, e, n_occ, tau, wt, per_class=True)
    assert np.allclose(r["classes"].sum(axis=1), r["integrand"], rtol=1e-12, atol=0)
    w = b.w_all()
    y = mp2.mo_at_ips(b.x, c)
    mu = mp2.chemical_potential(e, n_occ)
    mq = geo.minus_q(cfg.kmesh)
    qs = _qs_of(cfg)
    for n, t in enumerate(tau):
        go, gv = mp2.greens(y, e, n_occ, t, mu)
        chi, chit = mp2.polarisabilities(go, gv, cfg.kmesh, qs)
        del go, gv
        for i, q in enumerate(qs):
            term = np.trace(w[q] @ chi[i] @ w[q] @ chit[i]).real / cfg.n_k * (1 if mq[q] == q else 2)
            got = r["classes"][n, _class_of(cfg.kmesh, q)]
            rel = abs(got - term) / abs(term)
            print("%s tau %.1f q %d: class term %.6e rel %.2e" % (cfg.name, t, q, term, rel), flush=True)
            assert rel < 1e-10


@pytest.mark.timeout(900)
def test_large_cell_drpa_sampled(bigcell):
    """Direct RPA at the cell's full size from the GPU's W^q (two tau and
    two omega points): the class contributions of q = 0, a generic q and a
    zone-boundary q against the oracle's frequency polarisabilities of those
    q and ln det(1 - chi W) by LU."""
    from oracle import mp2
    from oracle import rpa
    b = bigcell
    cfg = b.d.cfg
    c, e, n_occ = inp.make_mo(cfg)
    tau, tw = np.array([0.4, 1.3]), np.array([0.6, 0.9])
    om, ow = np.array([0.0, 0.7]), np.array([0.5, 0.5])
    g = inp.quadrature_transform(tau, tw, om)
    r = b.ctx.drpa(c, e, n_occ, tau, ow, g, per_class=True)
    assert np.allclose(r["classes"].sum(axis=1), r["integrand"], rtol=1e-12, atol=0)
    w = b.w_all()
    y = mp2.mo_at_ips(b.x, c)
    mq = geo.minus_q(cfg.kmesh)
    qs = _qs_of(cfg)
    chis = rpa.chi_omega_from_tau(y, e, n_occ, cfg.kmesh, g, tau, qs)
    for m in range(len(om)):
        for i, q in enumerate(qs):
            full, _ = rpa.rpa_terms(chis[m, i] @ w[q])
            term = full * (1 if mq[q] == q else 2) / (np.pi * cfg.n_k)
            got = r["classes"][m, _class_of(cfg.kmesh, q)]
            rel = abs(got - term) / abs(term)
            print("%s omega %.1f q %d: class term %.6e rel %.2e" % (cfg.name, om[m], q, term, rel), flush=True)
            assert rel < 1e-9


@pytest.mark.timeout(900)
def test_large_cell_small_fragments_oracle(bigcell):
    b = bigcell
    name = b.d.cfg.name
    cfg = b.d.cfg
    frags = [inp.make_fragment(cfg, 20_000 + n, n) for n in (4, 8)]
    w = b.w_all()
    ref = [ko.fragment_eri(b.x, c, w, cfg.kmesh) for c in frags]
    out64 = b.ctx.fragment_eri(frags, "fp64")
    out16 = b.ctx.fragment_eri(frags, "bf16x3")
    out1 = b.ctx.fragment_eri(frags, "bf16")
    for c, r, o64, o16, o1 in zip(frags, ref, out64, out16, out1):
        rel = _rel(o64, r)
        err = float(np.max(np.abs(o16 - r)))
        err1 = float(np.max(np.abs(o1 - r)))
        print("%s n_f %d: FP64 rel %.2e, bf16x3 max|dV| %.2e Eh, bf16 %.2e Eh (max|V| %.2e)"
              % (name, c.shape[2], rel, err, err1, np.abs(r).max()))
        assert rel < 1e-10
        assert err < 1e-6
        assert err1 < 1e-6


@pytest.mark.timeout(900)
def test_large_cell_stream_fragments_mixed_vs_fp64(bigcell):
    import torch
    b = bigcell
    name = b.d.cfg.name
    cfg = b.d.cfg
    nfs = inp.fragment_sizes(cfg)
    frags = [inp.make_fragment(cfg, 0, int(nfs[0])), inp.make_fragment(cfg, 30_000, cfg.frag_hi)]
    dev = [torch.from_numpy(c).cuda() for c in frags]
    o64 = b.ctx.fragment_eri(dev, "fp64")
    o16 = b.ctx.fragment_eri(dev, "bf16x3")
    o1 = b.ctx.fragment_eri(dev, "bf16")
    for c, a, m, m1 in zip(frags, o64, o16, o1):
        err = float((a - m).abs().max().item())
        err1 = float((a - m1).abs().max().item())
        print("%s n_f %d: vs FP64 max|dV| bf16x3 %.2e Eh, bf16 %.2e Eh (max|V| %.2e)"
              % (name, c.shape[2], err, err1, float(a.abs().max().item())))
        assert err < 1e-6
        assert err1 < 1e-6
    del o64, o16, o1, dev
    torch.cuda.empty_cache()
