"""Exact ERIs and Gamma-point ISDF on the Born-von Karman supercell (oracle).

A Gamma-centred k mesh m1 x m2 x m3 is equivalent to a supercell of N_k unit
cells (introduction; eq. (1)).  On that supercell the method has a plain,
k-free definition, which is what every k-point quantity must reproduce:

* supercell orbitals  psi_c(x) = N_k^{-1/2} phi^k_mu(x),  c = (k, mu),
  with the Bloch extension phi^k(r + R) = exp(i k.R) phi^k(r) (eq. (1));
* fragment orbitals   psi_p(x) = N_k^{-1/2} sum_k sum_mu C^k_{mu p} phi^k_mu(x)
  (eq. (17));
* exact ERIs (FFT-Poisson on the supercell grid), chemists' notation with the
  conjugate on p and r:  (pq|rs) = (rho_pq | rho_rs),  rho_pq = conj(psi_p) psi_q;
* Gamma-point ISDF (eqs. (2)-(3) with one k point): interpolation points
  x_a = r_I + R, fit every pair product psi_c conj(psi_d) by
  sum_a zeta_a(x) psi_c(x_a) conj(psi_d(x_a)) in the least-squares sense,
  solve the normal equations with the minimum-norm pseudo-inverse, and form
  (pq|rs) = sum_ab P_{a,pq} (zeta_a|zeta_b) P_{b,rs},
  P_{a,pq} = conj(psi_p(x_a)) psi_q(x_a).

Supercell grid: index X_d = t_d n_d + i_d for cell t and unit-cell point i,
M_d = m_d n_d points per axis, C order.
"""
import numpy as np

from . import geometry as geo
from . import poisson


def supercell_orbitals(orbitals, grid, kmesh):
    """phi^k_mu on the supercell grid: [N_k, N_orb, M1*M2*M3] (eq. (1))."""
    nk, norb, _ = orbitals.shape
    n1, n2, n3 = grid
    m1, m2, m3 = kmesh
    jk = geo.kmesh_indices(kmesh)
    phi = orbitals.reshape(nk, norb, n1, n2, n3)
    out = np.empty((nk, norb, m1, n1, m2, n2, m3, n3), dtype=np.complex128)
    for k in range(nk):
        ph = [np.exp(2j * np.pi * jk[k, d] * np.arange(kmesh[d]) / kmesh[d])
              for d in range(3)]
        bloch = ph[0][:, None, None] * ph[1][None, :, None] * ph[2][None, None, :]
        out[k] = (bloch[None, :, None, :, None, :, None]
                  * phi[k][:, None, :, None, :, None, :])
    return out.reshape(nk, norb, -1)


def supercell_ip_index(ip_index, grid, kmesh):
    """Supercell flat indices of x_a = r_I + R, ordered a = (t, I)."""
    n1, n2, n3 = grid
    m1, m2, m3 = kmesh
    i1, i2, i3 = np.unravel_index(np.asarray(ip_index), (n1, n2, n3))
    jt = geo.kmesh_indices(kmesh)
    x1 = jt[:, 0, None] * n1 + i1[None, :]
    x2 = jt[:, 1, None] * n2 + i2[None, :]
    x3 = jt[:, 2, None] * n3 + i3[None, :]
    return np.ravel_multi_index((x1, x2, x3), (m1 * n1, m2 * n2, m3 * n3)).reshape(-1)


def fragment_orbitals(phi_s, coeffs):
    """psi_p(x) = N_k^{-1/2} sum_k sum_mu C^k_{mu p} phi^k_mu(x)  (eq. (17))."""
    nk = phi_s.shape[0]
    return np.einsum("kmp,kmx->px", coeffs, phi_s) / np.sqrt(nk)


def exact_eri(psi, lattice, grid, kmesh):
    """FFT-Poisson ERIs of fragment orbitals psi [n_f, N_S] on the supercell.

    (pq|rs) = (Omega_S/N_S^2) sum_{K != 0} (4 pi/|K|^2) rhohat_pq(K) rhohat_rs(-K)
    with rho_pq = conj(psi_p) psi_q and the nearest-representative kernel of
    ``geometry`` (symmetric under K -> -K, so it does not matter which of the
    two densities carries K).  Returns [n_f]^4 complex128."""
    nf, ns = psi.shape
    shape = tuple(grid[d] * kmesh[d] for d in range(3))
    vol_s = abs(np.linalg.det(geo.supercell_lattice(lattice, kmesh)))
    kern = geo.coulomb_supercell(lattice, grid, kmesh)
    rho = (psi.conj()[:, None, :] * psi[None, :, :]).reshape(nf * nf, *shape)
    rhat = np.fft.fftn(rho, axes=(1, 2, 3)).reshape(nf * nf, -1)
    refl = poisson.reflect_index(shape)
    a = rhat * kern[None, :]
    eri = (vol_s / ns ** 2) * (a @ rhat[:, refl].T)
    return eri.reshape(nf, nf, nf, nf)


def pinv_hermitian(mat, rcond):
    """Minimum-norm pseudo-inverse of a Hermitian PSD matrix: eigenvalues
    below rcond * max eigenvalue are dropped (the least-squares reading of
    "after solving eq. (3)")."""
    w, v = np.linalg.eigh(mat)
    keep = w > rcond * w.max()
    return (v[:, keep] / w[keep]) @ v[:, keep].conj().T, int(keep.sum())


def gamma_isdf(orbitals, ip_index, lattice, grid, kmesh, rcond=1e-13):
    """Gamma-point supercell ISDF: returns (xs, zeta, Wcal, rank).

    xs      supercell indices of the interpolation points (a = (t, I));
    zeta    interpolation functions [N_a, N_S] (real: the normal equations
            are real, see below);
    Wcal    Coulomb kernel (zeta_a|zeta_b) [N_a, N_a];
    rank    numerical rank of the metric.

    Metric  Pcal_ab = |G(x_a, x_b)|^2 and right-hand side
    h_a(x) = |G(x_a, x)|^2 with G(x, y) = sum_c psi_c(x) conj(psi_c(y))
    (eqs. (3)-(5) with a single k point)."""
    nk = orbitals.shape[0]
    phi_s = supercell_orbitals(orbitals, grid, kmesh)
    psi_c = phi_s.reshape(-1, phi_s.shape[-1]) / np.sqrt(nk)      # [N_c, N_S]
    xs = supercell_ip_index(ip_index, grid, kmesh)
    a_vals = psi_c[:, xs]                                         # [N_c, N_a]
    gmat = a_vals.T @ a_vals.conj()                               # G(x_a, x_b)
    pcal = np.abs(gmat) ** 2
    h = np.abs(a_vals.T @ psi_c.conj()) ** 2                      # [N_a, N_S]
    pinv, rank = pinv_hermitian(pcal, rcond)
    zeta = pinv @ h
    shape = tuple(grid[d] * kmesh[d] for d in range(3))
    ns = psi_c.shape[1]
    vol_s = abs(np.linalg.det(geo.supercell_lattice(lattice, kmesh)))
    kern = geo.coulomb_supercell(lattice, grid, kmesh)
    zhat = np.fft.fftn(zeta.reshape(-1, *shape), axes=(1, 2, 3)).reshape(zeta.shape[0], -1)
    refl = poisson.reflect_index(shape)
    # (zeta_a|zeta_b)
    wcal = (vol_s / ns ** 2) * ((zhat * kern[None, :]) @ zhat[:, refl].T)
    return xs, zeta, wcal, rank


def gamma_isdf_eri(orbitals, ip_index, coeffs, lattice, grid, kmesh,
                   rcond=1e-13, isdf=None):
    """(pq|rs) = sum_ab P_{a,pq} Wcal_ab P_{b,rs} on the supercell (eq. (9)
    specialised to one k point and transformed with eq. (17))."""
    if isdf is None:
        isdf = gamma_isdf(orbitals, ip_index, lattice, grid, kmesh, rcond)
    xs, _, wcal, _ = isdf
    phi_s = supercell_orbitals(orbitals, grid, kmesh)
    psi = fragment_orbitals(phi_s, coeffs)                        # [n_f, N_S]
    pv = psi[:, xs]                                               # [n_f, N_a]
    pair = pv.conj()[:, None, :] * pv[None, :, :]                 # [p, q, a]
    nf = psi.shape[0]
    pair = pair.reshape(nf * nf, -1)
    eri = pair @ wcal @ pair.T
    return eri.reshape(nf, nf, nf, nf)
