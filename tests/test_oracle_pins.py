"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test is chosen so that a plausible mistake in the oracle (a dropped
term, a wrong sign or index, a transposed operand, a missing conjugate or
normalisation) fails at least one of them:

* Poisson normalisation: the periodised Gaussian self-energy closed form
  (Ewald identity, Madelung constant from an explicit lattice sum);
* DFT conventions and the G+q box: explicit double sums on tiny cells;
* exactness: interpolation points = the whole grid (or a set spanning the
  pair space) reproduce FFT-Poisson ERIs (eqs. (2)-(3) with zero residual);
* k machinery: k-point results (eqs. (4)-(8), (17)-(20)) equal the plain
  Gamma-point supercell ISDF, which has no k sums at all;
* eq. (8): the xi route equals the Pi W Pi = V route;
* invariants: Hermiticity / PSD, q -> -q conjugation, ERI permutational
  symmetry, crystal-momentum conservation (eq. (9)), covariance.
"""
import math

import numpy as np
import pytest

import isdf_inputs as inp
from oracle import geometry as geo
from oracle import kpoint as ko
from oracle import poisson
from oracle import supercell as sc


def _case(name, n_ip=None):
    d = inp.make_inputs(name, n_ip=n_ip)
    return d


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


# --------------------------------------------------------------------------
# Poisson normalisation
# --------------------------------------------------------------------------
def test_madelung_independent_of_split():
    z1 = poisson.madelung_simple_cubic(eta=2.0)
    z2 = poisson.madelung_simple_cubic(eta=3.0, nreal=5, nrec=10)
    assert abs(z1 - z2) < 1e-11
    assert 2.83 < z1 < 2.84


def test_gaussian_self_energy_closed_form():
    length, sigma, n = 10.0, 0.5, 64
    lattice = np.eye(3) * length
    frac = geo.grid_frac((n, n, n))
    pos = frac * length
    rho = np.zeros(n ** 3)
    norm = (2 * np.pi * sigma ** 2) ** -1.5
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                d = pos - (np.array([i, j, k]) + 0.5) * length
                rho += norm * np.exp(-np.einsum("ij,ij->i", d, d) / (2 * sigma ** 2))
    shape = (n, n, n)
    rhat = np.fft.fftn(rho.reshape(shape)).reshape(-1)
    kern = geo.coulomb_supercell(lattice, shape, (1, 1, 1))
    refl = poisson.reflect_index(shape)
    val = poisson.coulomb_pair_sum(rhat[refl], rhat, kern, length ** 3, n ** 3).real
    ref = poisson.gaussian_self_energy_closed_form(
        sigma, length, poisson.madelung_simple_cubic())
    assert abs(val - ref) / abs(ref) < 1e-10


# --------------------------------------------------------------------------
# DFT conventions / box: explicit sums on a tiny cell
# --------------------------------------------------------------------------
def _symmetric_box(n, qf):
    """(g, weight) of every G_d = g with |g + qf| <= n/2: the box of K_d
    values symmetric about zero, with weight 1/2 on its two faces
    |g + qf| = n/2 (each face point and its opposite are the same DFT
    index).  Enumerated over a range wider than the box, no modular
    arithmetic."""
    out = []
    for g in range(-n, n + 1):
        x = g + qf
        if abs(x) < n / 2 - 1e-9:
            out.append((g, 1.0))
        elif abs(abs(x) - n / 2) < 1e-9:
            out.append((g, 0.5))
    return out


def _explicit_kpoint_box_eri(d, coeffs):
    """(pq|rs) with the G+q box summed explicitly (no FFT, no index tables)."""
    cfg = d.cfg
    lat = d.lattice
    phi_s = sc.supercell_orbitals(d.orbitals, cfg.grid, cfg.kmesh)
    psi = sc.fragment_orbitals(phi_s, coeffs)
    shape = tuple(cfg.grid[i] * cfg.kmesh[i] for i in range(3))
    xs_frac = geo.grid_frac(shape)                      # supercell fractions
    x_cart = xs_frac @ geo.supercell_lattice(lat, cfg.kmesh)
    b = geo.reciprocal(lat)
    nf = psi.shape[0]
    rho = (psi.conj()[:, None, :] * psi[None, :, :]).reshape(nf * nf, -1)
    vol_s = abs(np.linalg.det(geo.supercell_lattice(lat, cfg.kmesh)))
    ns = psi.shape[1]
    eri = np.zeros((nf * nf, nf * nf), dtype=np.complex128)
    for jq in geo.kmesh_indices(cfg.kmesh):
        qf = np.array([((jq[a] + cfg.kmesh[a] // 2) % cfg.kmesh[a] - cfg.kmesh[a] // 2)
                       / cfg.kmesh[a] for a in range(3)])
        for g1, w1 in _symmetric_box(cfg.grid[0], qf[0]):
            for g2, w2 in _symmetric_box(cfg.grid[1], qf[1]):
                for g3, w3 in _symmetric_box(cfg.grid[2], qf[2]):
                    kv = (np.array([g1, g2, g3]) + qf) @ b
                    k2 = kv @ kv
                    if k2 < 1e-14:
                        continue
                    e = np.exp(-1j * (x_cart @ kv))
                    fk = rho @ e                       # rhohat(K)
                    fmk = rho @ e.conj()               # rhohat(-K)
                    eri += (w1 * w2 * w3 * 4 * np.pi / k2) * np.outer(fk, fmk)
    return (vol_s / ns ** 2) * eri.reshape(nf, nf, nf, nf)


def test_exact_eri_matches_explicit_sums_tiny():
    d = _case("t_tiny_k2")
    coeffs = inp.make_fragment(d.cfg, 0, 3)
    phi_s = sc.supercell_orbitals(d.orbitals, d.cfg.grid, d.cfg.kmesh)
    psi = sc.fragment_orbitals(phi_s, coeffs)
    fft_eri = sc.exact_eri(psi, d.lattice, d.cfg.grid, d.cfg.kmesh)
    brute = _explicit_kpoint_box_eri(d, coeffs)
    assert _rel(fft_eri, brute) < 1e-13


def test_coulomb_kernel_matches_explicit_dft_tiny():
    d = _case("t_tiny_k2")
    cfg = d.cfg
    rng = np.random.default_rng(7)
    f = rng.standard_normal((5, cfg.n_g)) + 1j * rng.standard_normal((5, cfg.n_g))
    b = geo.reciprocal(d.lattice)
    r_cart = geo.grid_frac(cfg.grid) @ d.lattice
    for q in range(cfg.n_k):
        w = ko.coulomb_kernel_of(f, d.lattice, cfg.grid, cfg.kmesh, q)
        jq = geo.kmesh_indices(cfg.kmesh)[q]
        qf = np.array([((jq[a] + cfg.kmesh[a] // 2) % cfg.kmesh[a] - cfg.kmesh[a] // 2)
                       / cfg.kmesh[a] for a in range(3)])
        ref = np.zeros((5, 5), dtype=np.complex128)
        for g1, w1 in _symmetric_box(cfg.grid[0], qf[0]):
            for g2, w2 in _symmetric_box(cfg.grid[1], qf[1]):
                for g3, w3 in _symmetric_box(cfg.grid[2], qf[2]):
                    kv = (np.array([g1, g2, g3]) + qf) @ b
                    k2 = kv @ kv
                    if k2 < 1e-14:
                        continue
                    fh = f @ np.exp(-1j * (r_cart @ kv))
                    ref += (w1 * w2 * w3 * 4 * np.pi / k2) * np.outer(fh, fh.conj())
        ref *= cfg.volume / cfg.n_g ** 2
        assert _rel(w, ref) < 1e-13


# --------------------------------------------------------------------------
# Exactness limits
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["t_tiny_k1", "t_tiny_k2"])
def test_full_grid_ips_reproduce_exact_eri(name):
    cfg = inp.get_config(name)
    d = _case(name, n_ip=cfg.n_g)
    coeffs = inp.make_fragment(d.cfg, 0, 3)
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice,
                                      d.cfg.grid, d.cfg.kmesh)
    isdf = ko.fragment_eri(x, coeffs, w, d.cfg.kmesh)
    phi_s = sc.supercell_orbitals(d.orbitals, d.cfg.grid, d.cfg.kmesh)
    psi = sc.fragment_orbitals(phi_s, coeffs)
    exact = sc.exact_eri(psi, d.lattice, d.cfg.grid, d.cfg.kmesh)
    assert _rel(isdf, exact) < 1e-12
    # The Gamma-point supercell form is exact too.
    g_s = sc.gamma_isdf_eri(d.orbitals, d.ip_index, coeffs, d.lattice, d.cfg.grid,
                            d.cfg.kmesh)
    assert _rel(g_s, exact) < 1e-12


def test_c1_ips_span_pair_space_exact():
    """Workload 1 (Gamma, 8 real orbitals, 64 points): the metric has rank
    36 = 8*9/2 and the ISDF ERIs equal the FFT-Poisson ERIs."""
    d = _case("c1_gamma_16")
    coeffs = inp.make_fragment(d.cfg, 0, 8)
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice,
                                      d.cfg.grid, d.cfg.kmesh)
    wv = np.linalg.eigvalsh(pi[0])
    assert int((wv > 1e-12 * wv.max()).sum()) == 36
    isdf = ko.fragment_eri(x, coeffs, w, d.cfg.kmesh)
    phi_s = sc.supercell_orbitals(d.orbitals, d.cfg.grid, d.cfg.kmesh)
    psi = sc.fragment_orbitals(phi_s, coeffs)
    exact = sc.exact_eri(psi, d.lattice, d.cfg.grid, d.cfg.kmesh)
    assert np.max(np.abs(isdf - exact)) < 1e-12
    # real orbitals: 8-fold symmetry and a real tensor
    assert np.max(np.abs(isdf.imag)) < 1e-14
    v = isdf.real
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (1, 0, 3, 2)]:
        assert np.max(np.abs(v - v.transpose(perm))) < 1e-14


# --------------------------------------------------------------------------
# k machinery: k-point form == Gamma-point supercell form
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["t_tiny_k1", "t_tiny_k2", "t_small_k2"])
def test_kpoint_equals_supercell_isdf(name):
    d = _case(name)
    cfg = d.cfg
    coeffs = inp.make_fragment(cfg, 0, min(4, cfg.n_k * cfg.n_orb))
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    kp = ko.fragment_eri(x, coeffs, w, cfg.kmesh)
    gs = sc.gamma_isdf_eri(d.orbitals, d.ip_index, coeffs, d.lattice, cfg.grid,
                           cfg.kmesh)
    assert _rel(kp, gs) < 1e-11


def test_metric_blocks_are_supercell_metric():
    """Pi^q / N_k are the Fourier blocks of the block-circulant supercell
    metric: sum_D Pcal_{(I,D),(J,0)} exp(i q.D) = Pi^q_{IJ} / N_k."""
    d = _case("t_small_k2")
    cfg = d.cfg
    x = ko.ip_values(d.orbitals, d.ip_index)
    pi = ko.metric_k(x, cfg.kmesh)
    phi_s = sc.supercell_orbitals(d.orbitals, cfg.grid, cfg.kmesh)
    psi_c = phi_s.reshape(-1, phi_s.shape[-1]) / np.sqrt(cfg.n_k)
    xs = sc.supercell_ip_index(d.ip_index, cfg.grid, cfg.kmesh).reshape(cfg.n_k, cfg.n_ip)
    j = geo.kmesh_indices(cfg.kmesh)
    m = np.asarray(cfg.kmesh)
    for q in range(cfg.n_k):
        blk = np.zeros((cfg.n_ip, cfg.n_ip), dtype=np.complex128)
        for dd in range(cfg.n_k):
            g = psi_c[:, xs[dd]].T @ psi_c[:, xs[0]].conj()
            ph = np.exp(2j * np.pi * np.sum(j[q] * j[dd] / m))
            blk += np.abs(g) ** 2 * ph
        assert _rel(blk, pi[q] / cfg.n_k) < 1e-12


# --------------------------------------------------------------------------
# eq. (8): both routes to W
# --------------------------------------------------------------------------
def test_zeta_route_equals_v_route():
    d = _case("t_small_k3")
    cfg = d.cfg
    x = ko.ip_values(d.orbitals, d.ip_index)
    pi = ko.metric_k(x, cfg.kmesh)
    eta = ko.rhs(x, d.orbitals, cfg.kmesh, list(range(cfg.n_k)))
    wz = ko.kernel_zeta_route(pi, eta, d.lattice, cfg.grid, cfg.kmesh)
    wv = ko.kernel_v_route(pi, eta, d.lattice, cfg.grid, cfg.kmesh)
    assert _rel(wz, wv) < 1e-10


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_fit():
    d = _case("t_small_k3")
    cfg = d.cfg
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    return d, x, pi, eta, w


def test_metric_and_kernel_hermitian_psd(small_fit):
    d, x, pi, eta, w = small_fit
    # W = Pi^+ V Pi^+ carries the rounding of the pseudo-inverse, amplified by
    # cond(Pi) (~1e3 here): Hermitian to ~1e-11 relative, Pi to ~1e-15.
    for q in range(pi.shape[0]):
        for mat, tol in ((pi[q], 1e-14), (w[q], 1e-11)):
            assert np.max(np.abs(mat - mat.conj().T)) < tol * np.max(np.abs(mat))
            ev = np.linalg.eigvalsh(0.5 * (mat + mat.conj().T))
            assert ev.min() > -1e-12 * ev.max()


def test_minus_q_conjugation(small_fit):
    d, x, pi, eta, w = small_fit
    cfg = d.cfg
    mq = geo.minus_q(cfg.kmesh)
    jq = geo.kmesh_indices(cfg.kmesh)
    m = np.asarray(cfg.kmesh)
    for q in range(cfg.n_k):
        assert _rel(pi[mq[q]], pi[q].conj()) < 1e-13
        assert _rel(eta[mq[q]], eta[q].conj()) < 1e-13
        # the kernel is symmetric under K -> -K, zone-boundary q included
        assert _rel(w[mq[q]], w[q].conj()) < 1e-11


def test_eri_symmetries_and_psd(small_fit):
    d, x, pi, eta, w = small_fit
    coeffs = inp.make_fragment(d.cfg, 1, 7)
    v = ko.fragment_eri(x, coeffs, w, d.cfg.kmesh)
    nf = v.shape[0]
    assert _rel(v.transpose(2, 3, 0, 1), v) < 1e-12           # (pq|rs) = (rs|pq)
    assert _rel(v.transpose(1, 0, 3, 2).conj(), v) < 1e-12    # (qp|sr)^* = (pq|rs)
    m = v.transpose(0, 1, 3, 2).reshape(nf * nf, nf * nf)     # M_{(pq),(sr)}
    assert np.max(np.abs(m - m.conj().T)) < 1e-12 * np.max(np.abs(m))
    ev = np.linalg.eigvalsh(0.5 * (m + m.conj().T))
    assert ev.min() > -1e-12 * ev.max()


def test_crystal_momentum_conservation(small_fit):
    d, x, pi, eta, w = small_fit
    cfg = d.cfg
    nk, norb = cfg.n_k, cfg.n_orb
    rng = np.random.default_rng(3)
    picks = [(int(rng.integers(nk)), int(rng.integers(norb))) for _ in range(5)]
    coeffs = np.zeros((nk, norb, len(picks)), dtype=np.complex128)
    for p, (k, mu) in enumerate(picks):
        coeffs[k, mu, p] = 1.0
    v = ko.fragment_eri(x, coeffs, w, cfg.kmesh)
    j = geo.kmesh_indices(cfg.kmesh)
    m = np.asarray(cfg.kmesh)
    nz = 0
    for p in range(5):
        for q in range(5):
            for r in range(5):
                for s in range(5):
                    kp, kq, kr, ks = (picks[i][0] for i in (p, q, r, s))
                    cons = np.all((j[kq] - j[kp] + j[ks] - j[kr]) % m == 0)
                    if not cons:
                        assert abs(v[p, q, r, s]) < 1e-15
                    else:
                        nz += 1
                        ref = ko.thc_kpoint_eri(x, w, cfg.kmesh, kp, picks[p][1], kq,
                                                picks[q][1], kr, picks[r][1], ks,
                                                picks[s][1]) / nk
                        assert abs(v[p, q, r, s] - ref) < 1e-13 * max(1.0, abs(ref))
    assert nz > 0


def test_covariance(small_fit):
    d, x, pi, eta, w = small_fit
    cfg = d.cfg
    c = inp.make_fragment(cfg, 2, 6)
    v = ko.fragment_eri(x, c, w, cfg.kmesh)
    # lattice translation R0: C^k -> exp(i k.R0) C^k leaves V unchanged
    j = geo.kmesh_indices(cfg.kmesh)
    r0 = np.array([1, 0, 2])
    ph = np.exp(2j * np.pi * (j * r0 / np.asarray(cfg.kmesh)).sum(-1))
    vt = ko.fragment_eri(x, c * ph[:, None, None], w, cfg.kmesh)
    assert _rel(vt, v) < 1e-12
    # unitary rotation of the fragment orbitals
    rng = np.random.default_rng(11)
    z = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    u, _ = np.linalg.qr(z)
    vu = ko.fragment_eri(x, np.einsum("kmp,pa->kma", c, u), w, cfg.kmesh)
    ref = np.einsum("pqrs,pa,qb,rc,sd->abcd", v, u.conj(), u, u.conj(), u)
    assert _rel(vu, ref) < 1e-12
    # sub-fragment = sub-block
    vs = ko.fragment_eri(x, c[:, :, 1:4], w, cfg.kmesh)
    assert _rel(vs, v[1:4, 1:4, 1:4, 1:4]) < 1e-12


def test_eta_tilde_of_plane_waves_closed_form():
    """A plane wave exp(i (G0+q).r) has the single weighted coefficient
    sqrt(Omega c) at G0 (eq. (7)), c = 4 pi/|K|^2 for the representative K
    of G0 + q nearest zero (faces averaged: G0 = (-3, ., -2) sits on the
    faces of the 6 x 5 x 4 grid), and the K = 0 term is dropped: an
    independent check of the phase, the FFT index order, the reciprocal
    lattice and the weight of ``eta_tilde``."""
    lattice = np.array([[4.0, 0.0, 0.0], [1.0, 4.5, 0.0], [0.5, 0.3, 5.0]])
    grid, kmesh = (6, 5, 4), (2, 3, 1)
    vol = abs(np.linalg.det(lattice))
    frac = geo.grid_frac(grid)
    b = geo.reciprocal(lattice)
    g0s = np.array([(0, 0, 0), (1, -2, 1), (-3, 2, -2)])
    for q in range(6):
        qf = geo.q_frac_wrapped(geo.kmesh_indices(kmesh)[q], kmesh)
        f = np.exp(2j * np.pi * (frac @ (g0s + qf).T)).T
        et = ko.eta_tilde(f, lattice, grid, kmesh, q)
        for i, g0 in enumerate(g0s):
            idx = np.ravel_multi_index(tuple(np.mod(g0, grid)), grid)
            # the kernel of K = G0 + q is carried by the representatives of
            # its DFT index in the symmetric box (half weight on a face)
            c = 0.0
            reps = [[(g, w) for g, w in _symmetric_box(grid[a], qf[a]) if (g - g0[a]) % grid[a] == 0]
                    for a in range(3)]
            for g1, w1 in reps[0]:
                for g2, w2 in reps[1]:
                    for g3, w3 in reps[2]:
                        k2 = float(np.sum(((np.array([g1, g2, g3]) + qf) @ b) ** 2))
                        c += 0.0 if k2 < 1e-14 else w1 * w2 * w3 * 4.0 * np.pi / k2
            expect = np.sqrt(vol * c)
            assert abs(et[i, idx] - expect) < 1e-12 * max(1.0, expect), (q, i)
            assert np.max(np.abs(np.delete(et[i], idx))) < 1e-12, (q, i)


# --------------------------------------------------------------------------
# Lattice duality and the reduced forms the sampled GPU references use
# --------------------------------------------------------------------------
def test_reciprocal_duality_non_orthogonal():
    """a_i . b_j = 2 pi delta_ij on a triclinic lattice (explicit dot
    products), and the textbook reciprocal of a hexagonal lattice
    a1 = (a, 0, 0), a2 = (a/2, a sqrt(3)/2, 0), a3 = (0, 0, c):
    b1 = 2 pi/a (1, -1/sqrt(3), 0), b2 = 2 pi/a (0, 2/sqrt(3), 0),
    b3 = 2 pi/c (0, 0, 1).  The hexagonal lattice matrix is not symmetric,
    so a transposed inverse fails it."""
    tri = np.array([[4.0, 0.0, 0.0], [1.0, 4.5, 0.0], [0.5, 0.3, 5.0]])
    b = geo.reciprocal(tri)
    for i in range(3):
        for j in range(3):
            dot = sum(tri[i][c] * b[j][c] for c in range(3))
            assert abs(dot - (2 * np.pi if i == j else 0.0)) < 1e-13
    a, c = 4.7, 7.3
    hexa = np.array([[a, 0.0, 0.0], [a / 2, a * math.sqrt(3) / 2, 0.0], [0.0, 0.0, c]])
    expect = np.array([[2 * np.pi / a, -2 * np.pi / (a * math.sqrt(3)), 0.0],
                       [0.0, 4 * np.pi / (a * math.sqrt(3)), 0.0],
                       [0.0, 0.0, 2 * np.pi / c]])
    assert np.max(np.abs(geo.reciprocal(hexa) - expect)) < 1e-13


def test_rhs_reduced_forms_equal_full_form():
    """rhs on a subset of grid points and of q (in any order) returns the
    matching entries of the full call, and rhs_chunked with a chunk that does
    not divide N_g equals the full call: the forms the sampled GPU
    references rely on."""
    d = _case("t_small_k3")
    cfg = d.cfg
    x = ko.ip_values(d.orbitals, d.ip_index)
    full = ko.rhs(x, d.orbitals, cfg.kmesh, list(range(cfg.n_k)))
    rng = np.random.default_rng(5)
    ridx = np.sort(rng.choice(cfg.n_g, 97, replace=False))
    qs = [7, 0, 13]
    sub = ko.rhs(x, d.orbitals, cfg.kmesh, qs, ridx)
    assert _rel(sub, full[qs][:, :, ridx]) < 1e-15
    assert cfg.n_g % 500 != 0
    ch = ko.rhs_chunked(x, d.orbitals, cfg.kmesh, qs, chunk=500)
    assert _rel(ch, full[qs]) < 1e-15
    # subsets of interpolation points (rows) are rows of the full result
    rows = [3, 40, 11]
    sub_rows = ko.rhs(x[:, rows], d.orbitals, cfg.kmesh, qs, ridx)
    assert _rel(sub_rows, full[qs][:, rows][:, :, ridx]) < 1e-15


def test_kernel_v_route_q_subset_equals_full_call():
    """kernel_v_route with qs = [q2, q0] returns the rows q2, q0 of the full
    call (eta given in the order of qs)."""
    d = _case("t_small_k3")
    cfg = d.cfg
    x = ko.ip_values(d.orbitals, d.ip_index)
    pi = ko.metric_k(x, cfg.kmesh)
    eta = ko.rhs(x, d.orbitals, cfg.kmesh, list(range(cfg.n_k)))
    full = ko.kernel_v_route(pi, eta, d.lattice, cfg.grid, cfg.kmesh)
    qs = [9, 0, 4]
    sub = ko.kernel_v_route(pi, eta[qs], d.lattice, cfg.grid, cfg.kmesh, qs=qs)
    assert _rel(sub, full[qs]) < 1e-15


def test_metric_rows_equal_full_metric():
    """Rows of Pi^q from the rows of X alone (the reduced form used at the
    largest workloads) equal rows of the full metric for every q."""
    d = _case("t_small_k3")
    cfg = d.cfg
    x = ko.ip_values(d.orbitals, d.ip_index)
    pi = ko.metric_k(x, cfg.kmesh)
    rows = [5, 0, 77]
    pr = ko.metric_rows(x, cfg.kmesh, rows)
    assert _rel(pr, pi[:, rows, :]) < 1e-15


# --------------------------------------------------------------------------
# Interpolation-point selection (pivoted Cholesky of the pair products)
# --------------------------------------------------------------------------
from oracle import ipselect as ips


def _pair_product_matrix(orbitals):
    """Z with rows (k_mu, mu, k_nu, nu) and columns r:
    phi^{k_mu}_mu(r) conj(phi^{k_nu}_nu(r)), straight from the definition."""
    phi = orbitals.reshape(-1, orbitals.shape[2])
    return (phi[:, None, :] * phi[None, :, :].conj()).reshape(-1, phi.shape[1])


def test_selector_gram_is_the_pair_product_gram():
    d = _case("t_tiny_k2")
    z = _pair_product_matrix(d.orbitals)
    m = (z.conj().T @ z)
    assert np.max(np.abs(m.imag)) < 1e-12 * np.max(np.abs(m))
    phi = d.orbitals.reshape(-1, d.cfg.n_g)
    for p in (0, 17, 300, 511):
        assert _rel(ips.gram_column(phi, p), m[:, p].real) < 1e-13


def test_selector_is_the_greedy_pivoted_cholesky_of_the_explicit_gram():
    """Against the explicit Gram matrix: every pivot is the largest residual
    diagonal of M - L L^T at its step, L L^T reproduces the pivot columns of
    M, and the residual diagonal is diag(M - L L^T)."""
    d = _case("t_tiny_k2")
    z = _pair_product_matrix(d.orbitals)
    m = (z.conj().T @ z).real
    n = 20
    piv, dmax, lf, res, gap = ips.pivoted_cholesky_points(d.orbitals, n, with_gaps=True)
    for i in range(n):
        resid = np.diag(m) - np.sum(lf[:, :i] ** 2, axis=1)
        resid[piv[:i]] = 0.0                       # chosen points leave the candidate set
        assert piv[i] == int(np.argmax(resid)), i
        assert abs(dmax[i] - resid[piv[i]]) < 1e-12 * np.max(np.diag(m))
        top = np.sort(resid)[::-1]
        assert abs(gap[i] - (top[0] - top[1])) < 1e-12 * np.max(np.diag(m))
    assert _rel(lf @ lf[piv].T, m[:, piv]) < 1e-12
    assert np.max(np.abs(res - (np.diag(m) - np.sum(lf ** 2, axis=1)))) < 1e-12 * np.max(np.diag(m))
    # the first pivot is the densest point (M(r, r) = rho(r)^2)
    rho = np.sum(np.abs(d.orbitals) ** 2, axis=(0, 1))
    assert piv[0] == int(np.argmax(rho))


def test_selected_points_span_the_pair_space_and_reproduce_exact_eris():
    """Workload 1 (8 real orbitals at Gamma): the pair products span
    8 * 9 / 2 = 36 functions, so the residual vanishes after 36 pivots, and
    ISDF on those 36 points reproduces the FFT-Poisson ERIs."""
    d = _case("c1_gamma_16")
    cfg = d.cfg
    piv, dmax, lf, res = ips.pivoted_cholesky_points(d.orbitals, 37)
    assert dmax[35] > 1e-8 * dmax[0]
    assert dmax[36] < 1e-13 * dmax[0]
    ip = np.sort(piv[:36]).astype(np.int32)
    # beyond the rank the residuals are rounding noise, and no point is
    # chosen twice
    piv48, dmax48 = ips.pivoted_cholesky_points(d.orbitals, 48)[:2]
    assert len(set(piv48.tolist())) == 48
    assert np.all(dmax48[36:] < 1e-13 * dmax48[0])
    coeffs = inp.make_fragment(cfg, 0, 8)
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, ip, d.lattice, cfg.grid, cfg.kmesh)
    isdf = ko.fragment_eri(x, coeffs, w, cfg.kmesh)
    phi_s = sc.supercell_orbitals(d.orbitals, cfg.grid, cfg.kmesh)
    psi = sc.fragment_orbitals(phi_s, coeffs)
    exact = sc.exact_eri(psi, d.lattice, cfg.grid, cfg.kmesh)
    assert _rel(isdf, exact) < 1e-12


def test_selection_invariant_under_orbital_rotation_within_k():
    """G(r, r') is invariant under a unitary mixing of the orbitals of each k,
    so the pivots are too."""
    d = _case("t_small_k2")
    rng = np.random.default_rng(9)
    rot = np.empty_like(d.orbitals)
    for k in range(d.cfg.n_k):
        u, _ = np.linalg.qr(rng.standard_normal((d.cfg.n_orb,) * 2)
                            + 1j * rng.standard_normal((d.cfg.n_orb,) * 2))
        rot[k] = u.T @ d.orbitals[k]
    a = ips.pivoted_cholesky_points(d.orbitals, 40)[0]
    b = ips.pivoted_cholesky_points(rot, 40)[0]
    assert np.array_equal(a, b)


# --------------------------------------------------------------------------
# k-point Hartree-Fock Coulomb and exchange matrices (eq. (10))
# --------------------------------------------------------------------------
from oracle import hf


def _supercell_jk(d, dm):
    """J and K of gamma on the supercell from the exact FFT-Poisson ERIs of
    every supercell orbital N_k^{-1/2} phi^k_mu, contracted with the
    block-diagonal density matrix: J_ab = sum_cd (ab|dc) g_cd,
    K_ab = sum_cd (ac|db) g_cd.  Returns full supercell matrices."""
    cfg = d.cfg
    n = cfg.n_k * cfg.n_orb
    ident = np.eye(n, dtype=np.complex128).reshape(cfg.n_k, cfg.n_orb, n)
    phi_s = sc.supercell_orbitals(d.orbitals, cfg.grid, cfg.kmesh)
    psi = sc.fragment_orbitals(phi_s, ident)
    eri = sc.exact_eri(psi, d.lattice, cfg.grid, cfg.kmesh)
    g = np.zeros((n, n), dtype=np.complex128)
    for k in range(cfg.n_k):
        s = slice(k * cfg.n_orb, (k + 1) * cfg.n_orb)
        g[s, s] = dm[k]
    j = np.einsum("abdc,cd->ab", eri, g)
    kk = np.einsum("acdb,cd->ab", eri, g)
    return j, kk


@pytest.mark.parametrize("name", ["t_tiny_k2", "t_k10_line"])
def test_jk_equal_contraction_of_eq9_eris(name):
    """Eq. (10) as a sum over q (and J as the q = 0 term) against the plain
    element-by-element contraction of the crystalline ERIs of eq. (9); the
    10-point mesh axis tells q from -q."""
    d = _case(name)
    cfg = d.cfg
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    dm = inp.make_density(cfg)
    j_ref, k_ref = hf.jk_from_eri(x, w, dm, cfg.kmesh)
    assert _rel(hf.exchange(x, w, dm, cfg.kmesh), k_ref) < 1e-13
    assert _rel(hf.coulomb(x, w, dm), j_ref) < 1e-13
    ks = [cfg.n_k - 1, 1]
    assert _rel(hf.exchange_at(x, w, dm, cfg.kmesh, ks), k_ref[ks]) < 1e-13


@pytest.mark.parametrize("name", ["t_tiny_k2", "t_k10_line"])
def test_jk_with_full_grid_ips_equal_exact_supercell_jk(name):
    """With every grid point an interpolation point the fit is exact, so J
    and K from W^q equal the FFT-Poisson Coulomb and exchange matrices of
    the supercell density matrix; the supercell matrices have no blocks
    between different k (crystal momentum)."""
    cfg = inp.get_config(name)
    d = _case(name, n_ip=cfg.n_g)
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    dm = inp.make_density(cfg)
    j_s, k_s = _supercell_jk(d, dm)
    kk = hf.exchange(x, w, dm, cfg.kmesh)
    jj = hf.coulomb(x, w, dm)
    no = cfg.n_orb
    for k in range(cfg.n_k):
        s = slice(k * no, (k + 1) * no)
        assert _rel(kk[k], k_s[s, s]) < 1e-11
        assert _rel(jj[k], j_s[s, s]) < 1e-11
        for k2 in range(cfg.n_k):
            if k2 != k:
                s2 = slice(k2 * no, (k2 + 1) * no)
                assert np.max(np.abs(k_s[s, s2])) < 1e-13 * np.max(np.abs(k_s))
                assert np.max(np.abs(j_s[s, s2])) < 1e-13 * np.max(np.abs(j_s))


def test_jk_hermitian_and_exchange_psd():
    """For Hermitian PSD P^k: J^k and K^k are Hermitian, K^k is PSD (the
    exchange kernel gamma(x, y) v(x - y) is a product of PSD kernels), and
    the Coulomb and exchange energies sum_k tr(P^k J^k), sum_k tr(P^k K^k)
    are real and positive."""
    d = _case("t_small_k2")
    cfg = d.cfg
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    dm = inp.make_density(cfg)
    kk = hf.exchange(x, w, dm, cfg.kmesh)
    jj = hf.coulomb(x, w, dm)
    for k in range(cfg.n_k):
        assert _rel(kk[k], kk[k].conj().T) < 1e-13
        assert _rel(jj[k], jj[k].conj().T) < 1e-13
        assert np.linalg.eigvalsh(kk[k]).min() > -1e-12 * np.abs(kk[k]).max()
    ej = np.einsum("kab,kba->", dm, jj)
    ek = np.einsum("kab,kba->", dm, kk)
    assert abs(ej.imag) < 1e-12 * abs(ej) and ej.real > 0
    assert abs(ek.imag) < 1e-12 * abs(ek) and ek.real > 0


# --------------------------------------------------------------------------
# k-point SOS-MP2 in the imaginary-time form (eqs. (11)-(15))
# --------------------------------------------------------------------------
from oracle import mp2


@pytest.mark.parametrize("name", ["t_small_k3", "t_k10_line"])
def test_os_integrand_equals_closed_form_at_every_tau(name):
    """F(tau) from the polarisabilities (k convolutions of the Green's
    functions at the points, traces with W^q) equals the closed-form sum
    over ijab of |(ia|jb)|^2 exp(-tau Delta) from the crystalline ERIs of
    eq. (9), with no quadrature; the chemical potential cancels."""
    d = _case(name)
    cfg = d.cfg
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    c, e, n_occ = inp.make_mo(cfg)
    for tau in (0.0, 0.37, 1.9):
        f = mp2.os_integrand(x, w, c, e, n_occ, cfg.kmesh, tau)
        ref = mp2.os_closed_form(x, w, c, e, n_occ, cfg.kmesh, tau)
        assert abs(f.imag) < 1e-12 * abs(ref)
        assert abs(f.real - ref) < 1e-12 * abs(ref), tau
    y = mp2.mo_at_ips(x, c)
    go, gv = mp2.greens(y, e, n_occ, 0.8, 0.1)
    go2, gv2 = mp2.greens(y, e, n_occ, 0.8, -0.2)
    chi, chit = mp2.polarisabilities(go, gv, cfg.kmesh)
    chi2, chit2 = mp2.polarisabilities(go2, gv2, cfg.kmesh)
    assert _rel(chi, chi2) < 1e-12 and _rel(chit, chit2) < 1e-12
    # chit^q = conj(chi^{-q})
    mq = geo.minus_q(cfg.kmesh)
    assert _rel(chit, chi[mq].conj()) < 1e-13


def test_os_energy_quadrature_converges_to_closed_form():
    d = _case("t_small_k3")
    cfg = d.cfg
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    c, e, n_occ = inp.make_mo(cfg)
    exact = mp2.os_closed_form(x, w, c, e, n_occ, cfg.kmesh)
    assert exact < 0
    errs = []
    for n in (12, 24, 36):
        t, wt = inp.laplace_grid(n, 1.0)
        errs.append(abs(mp2.os_energy(x, w, c, e, n_occ, cfg.kmesh, t, wt) - exact) / abs(exact))
    assert errs[2] < 1e-9 and errs[1] < errs[0]


@pytest.mark.parametrize("name", ["t_tiny_k2", "t_k10_line"])
def test_os_energy_with_full_grid_ips_equals_supercell_mp2(name):
    """With every grid point an interpolation point the ISDF ERIs are exact,
    so E_OS equals the opposite-spin MP2 energy of the supercell canonical
    orbitals from the FFT-Poisson ERIs, -sum |(ia|jb)|^2 / Delta, per cell."""
    cfg = inp.get_config(name)
    d = _case(name, n_ip=cfg.n_g)
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    c, e, n_occ = inp.make_mo(cfg)
    nk, no = cfg.n_k, cfg.n_orb
    coeffs = np.zeros((nk, no, nk * no), dtype=np.complex128)
    for k in range(nk):
        coeffs[k, :, k * no:(k + 1) * no] = c[k]
    phi_s = sc.supercell_orbitals(d.orbitals, cfg.grid, cfg.kmesh)
    psi = sc.fragment_orbitals(phi_s, coeffs)
    eri = sc.exact_eri(psi, d.lattice, cfg.grid, cfg.kmesh)
    occ = np.array([k * no + p for k in range(nk) for p in range(n_occ)])
    vir = np.array([k * no + p for k in range(nk) for p in range(n_occ, no)])
    ef = e.reshape(-1)
    v = eri[np.ix_(occ, vir, occ, vir)]
    delta = (ef[vir][None, :, None, None] - ef[occ][:, None, None, None]
             + ef[vir][None, None, None, :] - ef[occ][None, None, :, None])
    e_sc = -np.sum(np.abs(v) ** 2 / delta) / nk
    assert _rel(mp2.os_closed_form(x, w, c, e, n_occ, cfg.kmesh), e_sc) < 1e-11


# --------------------------------------------------------------------------
# k-point direct RPA (eq. (16))
# --------------------------------------------------------------------------
from oracle import rpa


def test_drpa_second_order_term_is_the_os_mp2_energy():
    """The second-order term of the logarithm of eq. (16) is the
    opposite-spin MP2 energy (closed form over ijab), on a frequency
    quadrature fine enough for its Lorentzians; the full dRPA energy is
    negative and smaller in magnitude (screening)."""
    d = _case("t_small_k3")
    cfg = d.cfg
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    c, e, n_occ = inp.make_mo(cfg)
    om, ow = inp.laplace_grid(40, 1.0)
    e_rpa, e_2 = rpa.drpa_energy(x, w, c, e, n_occ, cfg.kmesh, om, ow)
    e_os = mp2.os_closed_form(x, w, c, e, n_occ, cfg.kmesh)
    assert abs(e_2 - e_os) < 1e-8 * abs(e_os)
    assert e_os < e_rpa < 0
    # the same energies from the time polarisabilities with a fitted transform
    tau, _ = inp.laplace_grid(32, 0.5)
    lo, hi = inp.excitation_range(e, n_occ)
    e_rpa_t, e_2_t = rpa.drpa_energy(x, w, c, e, n_occ, cfg.kmesh, om, ow, tau,
                                     inp.fitted_transform(tau, om, lo, hi))
    assert abs(e_rpa_t - e_rpa) < 1e-6 * abs(e_rpa) and abs(e_2_t - e_2) < 1e-6 * abs(e_2)


@pytest.mark.parametrize("name", ["t_k10_line", "t_small_k3"])
def test_chi_omega_from_time_quadrature_matches_closed_form(name):
    """chi^q(iw) as the quadrature of the time integral of the Green's-function
    polarisabilities converges to the Lorentzian closed form (a 128-point
    mapped Gauss-Legendre grid resolves exp(i w tau) up to w = 1.5 Eh);
    chi^q(-iw) is chi^q(iw)^H; chi^{-q}(iw) = conj(chi^q(iw))."""
    d = _case(name)
    cfg = d.cfg
    x = ko.ip_values(d.orbitals, d.ip_index)
    c, e, n_occ = inp.make_mo(cfg)
    y = mp2.mo_at_ips(x, c)
    tau, tw = inp.laplace_grid(128, 1.0)
    omegas = [0.0, 0.6, 1.5]
    qs = [0, 1, cfg.n_k - 1]
    got = rpa.chi_omega_from_tau(y, e, n_occ, cfg.kmesh, inp.quadrature_transform(tau, tw, omegas), tau, qs)
    mq = geo.minus_q(cfg.kmesh)
    for m, om in enumerate(omegas):
        for i, q in enumerate(qs):
            ref = rpa.chi_omega_exact(y, e, n_occ, cfg.kmesh, q, om)
            assert _rel(got[m, i], ref) < 1e-7, (om, q)
            assert _rel(rpa.chi_omega_exact(y, e, n_occ, cfg.kmesh, q, -om), ref.conj().T) < 1e-13
            assert _rel(rpa.chi_omega_exact(y, e, n_occ, cfg.kmesh, int(mq[q]), om), ref.conj()) < 1e-13
    # a fitted transform on 32 times is accurate at every frequency, up to
    # those a plain quadrature cannot resolve
    tau2, _ = inp.laplace_grid(32, 0.5)
    om2, _ = inp.laplace_grid(12, 1.0)
    lo, hi = inp.excitation_range(e, n_occ)
    fit = rpa.chi_omega_from_tau(y, e, n_occ, cfg.kmesh, inp.fitted_transform(tau2, om2, lo, hi), tau2, qs)
    for m, om in enumerate(om2):
        for i, q in enumerate(qs):
            assert _rel(fit[m, i], rpa.chi_omega_exact(y, e, n_occ, cfg.kmesh, q, om)) < 1e-6, (om, q)


def test_drpa_log_det_against_the_ring_series():
    """With W scaled so that the ring series converges, Re ln det(1 - P) +
    Re tr P equals -sum_{n >= 2} Re tr(P^n) / n."""
    d = _case("t_k10_line")
    cfg = d.cfg
    x, pi, eta, w = ko.fit_and_kernel(d.orbitals, d.ip_index, d.lattice, cfg.grid, cfg.kmesh)
    c, e, n_occ = inp.make_mo(cfg)
    y = mp2.mo_at_ips(x, c)
    p = rpa.chi_omega_exact(y, e, n_occ, cfg.kmesh, 3, 0.4) @ w[3]
    p = p * (0.5 / np.max(np.abs(np.linalg.eigvals(p))))
    full, second = rpa.rpa_terms(p)
    series = 0.0
    pn = p @ p
    for n in range(2, 80):
        series -= np.trace(pn).real / n
        pn = pn @ p
    assert abs(full - series) < 1e-12 * abs(series)
    assert abs(second + 0.5 * np.trace(p @ p).real) < 1e-15
