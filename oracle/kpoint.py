"""k-point ISDF fit, Coulomb kernel and fragment ERIs (oracle, plain form).

Readings of the paper fixed here (each pinned by ``tests/test_oracle_pins.py``):

* a superscript -k on X, phi, C or Y means the complex conjugate of the
  quantity at k (eq. (2) writes phi(r)^* = phi^{-k}(r)); the orbital at mesh
  point -k is never looked up;
* q is the mesh difference of the pair momenta, q = k_mu - k_nu (eq. (2));
  in the Coulomb kernel q is wrapped to [-1/2, 1/2) per axis, and each DFT
  index of the unit-cell grid stands for K = G + q taken at its
  representative nearest zero per axis (the kernel averaged over the two
  representatives where K_d = +-n_d/2), see ``oracle.geometry``;
* the element-wise product of Algorithm 1 is T^R conj(T^R) = |T^R|^2 (what
  the least-squares normal equations of eq. (2) require);
* the normal equations of eq. (3) are solved in the minimum-norm
  least-squares sense (eigenvalues below rcond * max dropped);
* normalisations follow the supercell definitions of ``oracle.supercell``:
  fragment ERIs are in Hartree for fragment orbitals normalised on the
  supercell.

Index conventions of this module (chemists' ERIs, conjugate on p and r):

    T^k_{IJ}   = sum_mu X^k_{I mu} conj(X^k_{J mu})                       (Alg. 1, Y = X)
    Pi^q_{IJ}  = sum_k conj(T^{k+q}_{IJ}) T^k_{IJ}                         (eq. (4))
    T^k_I(r)   = sum_mu X^k_{I mu} conj(phi^k_mu(r))                       (Alg. 1, Y = phi)
    eta^q_I(r) = sum_k conj(T^{k+q}_I(r)) T^k_I(r)                         (eq. (5))
    Pi^q xi^q(r) = eta^q(r)                                                (eq. (3))
    xihat^q_I(G) = sum_r xi^q_I(r) exp(-i (G+q).r)
    W^q_{IJ}   = (Omega/N_g^2) sum_G c(G+q) xihat^q_I(G) conj(xihat^q_J(G)) (eq. (6))
    V^q_{IJ}   = same with eta in place of xi;  W^q = Pi^{q+} V^q Pi^{q+}  (eqs. (7)-(8))
    psi_p(r_I + R) = N_k^{-1/2} sum_k exp(i k.R) sum_mu C^k_{mu p} X^k_{I mu}  (eq. (17), Alg. 2)
    R^q_{I,pq} = N_k^{-1/2} sum_R exp(-i q.R) conj(psi_p(r_I+R)) psi_q(r_I+R)  (eq. (20))
    (pq|rs)    = sum_q sum_IJ R^q_{I,pq} W^q_{IJ} R^{-q}_{J,rs}             (eq. (19))

With these, the k-point results equal the Gamma-point supercell ISDF of
``oracle.supercell`` exactly (both use the G+q box).  The paper's V_pqrs,
which carries the conjugate on the second and fourth index, is (qp|sr) here.
"""
import numpy as np

from . import geometry as geo
from .supercell import pinv_hermitian


def ip_values(orbitals, ip_index):
    """Interpolating vectors X^k_{I mu} = phi^k_mu(r_I)  (below eq. (2)).
    Returns [N_k, N_IP, N_orb]."""
    return np.ascontiguousarray(np.transpose(orbitals[:, :, ip_index], (0, 2, 1)))


def metric_k(x, kmesh):
    """Pi^q_{IJ} = sum_k conj(T^{k+q}_{IJ}) T^k_{IJ}  (eq. (4)), direct k sum."""
    nk = x.shape[0]
    t = np.matmul(x, np.transpose(x.conj(), (0, 2, 1)))           # T^k_{IJ}
    kq = geo.k_plus_q(kmesh)
    pi = np.empty_like(t)
    for q in range(nk):
        pi[q] = np.einsum("kij,kij->ij", t[kq[:, q]].conj(), t)
    return pi


def metric_rows(x, kmesh, rows, qs=None):
    """Rows I in ``rows`` of Pi^q_{IJ} = sum_k conj(T^{k+q}_{IJ}) T^k_{IJ}
    (eq. (4)) for the listed q (all if None), from the rows of T^k alone:
    the same direct k sum as ``metric_k`` at a cost linear in the number of
    rows.  Returns [len(qs), len(rows), N_IP]."""
    nk = x.shape[0]
    qs = list(range(nk)) if qs is None else list(qs)
    t = np.matmul(x[:, rows, :], np.transpose(x.conj(), (0, 2, 1)))   # T^k_{IJ}, I in rows
    kq = geo.k_plus_q(kmesh)
    out = np.empty((len(qs),) + t.shape[1:], dtype=np.complex128)
    for iq, q in enumerate(qs):
        out[iq] = np.einsum("kij,kij->ij", t[kq[:, q]].conj(), t)
    return out


def rhs(x, orbitals, kmesh, qs, r_index=None):
    """eta^q_I(r) = sum_k conj(T^{k+q}_I(r)) T^k_I(r) for the listed q
    (eq. (5); Algorithm 1 with Y = phi), direct k sum, on the grid points
    r_index (all points if None).  Returns [len(qs), N_IP, N_r]."""
    nk = x.shape[0]
    phi = orbitals if r_index is None else orbitals[:, :, r_index]
    t = np.matmul(x, phi.conj())                                  # T^k_I(r)
    kq = geo.k_plus_q(kmesh)
    out = np.empty((len(qs), x.shape[1], phi.shape[2]), dtype=np.complex128)
    for iq, q in enumerate(qs):
        out[iq] = np.einsum("kir,kir->ir", t[kq[:, q]].conj(), t)
    return out


def rhs_chunked(x, orbitals, kmesh, qs, chunk=4096):
    """eta^q_I(r) of eq. (5) for the listed q on the whole grid, computed
    over grid chunks so that T^k_I(r) is never held for all r at once."""
    ng = orbitals.shape[2]
    out = np.empty((len(qs), x.shape[1], ng), dtype=np.complex128)
    for r0 in range(0, ng, chunk):
        idx = np.arange(r0, min(ng, r0 + chunk))
        out[:, :, idx] = rhs(x, orbitals, kmesh, qs, idx)
    return out


def solve(pi_q, eta_q, rcond=1e-13):
    """Minimum-norm solution of Pi^q xi^q(r) = eta^q(r) for every r (eq. (3))."""
    pinv, _ = pinv_hermitian(pi_q, rcond)
    return pinv @ eta_q


def coulomb_kernel_of(f_q, lattice, grid, kmesh, q):
    """(Omega/N_g^2) sum_G c(G+q) fhat_I(G) conj(fhat_J(G)) with
    fhat_I(G) = sum_r f_I(r) exp(-i (G+q).r) (eq. (6) for f = xi, eq. (7)
    for f = eta); q wrapped to [-1/2, 1/2) per axis.  f_q: [N_IP, N_g]."""
    jq = geo.kmesh_indices(kmesh)[q]
    qf = geo.q_frac_wrapped(jq, kmesh)
    frac = geo.grid_frac(grid)
    phase = np.exp(-2j * np.pi * (frac @ qf))                     # exp(-i q.r)
    n1, n2, n3 = grid
    fh = np.fft.fftn((f_q * phase[None, :]).reshape(-1, n1, n2, n3),
                     axes=(1, 2, 3)).reshape(f_q.shape[0], -1)
    c = geo.coulomb_g_plus_q(lattice, grid, qf)
    vol = abs(np.linalg.det(lattice))
    ng = n1 * n2 * n3
    return (vol / ng ** 2) * ((fh * c[None, :]) @ fh.conj().T)


def eta_tilde(f_q, lattice, grid, kmesh, q):
    """The Coulomb-weighted transform whose Hermitian square is V^q (eq. (7)):
    etatilde_I(G) = sqrt(Omega c(G+q)) / N_g * sum_r f_I(r) exp(-i (G+q).r),
    so that (Omega/N_g^2) sum_G c(G+q) fhat_I conj(fhat_J) = etatilde etatilde^H.
    G in the numpy FFT index order of the grid; f_q: [N_IP, N_g]."""
    jq = geo.kmesh_indices(kmesh)[q]
    qf = geo.q_frac_wrapped(jq, kmesh)
    frac = geo.grid_frac(grid)
    phase = np.exp(-2j * np.pi * (frac @ qf))
    n1, n2, n3 = grid
    fh = np.fft.fftn((f_q * phase[None, :]).reshape(-1, n1, n2, n3),
                     axes=(1, 2, 3)).reshape(f_q.shape[0], -1)
    c = geo.coulomb_g_plus_q(lattice, grid, qf)
    vol = abs(np.linalg.det(lattice))
    return fh * (np.sqrt(vol * c) / (n1 * n2 * n3))[None, :]


def kernel_zeta_route(pi, eta_all, lattice, grid, kmesh, rcond=1e-13):
    """W^q for all q from xi^q = Pi^{q+} eta^q (eqs. (3), (6))."""
    out = np.empty_like(pi)
    for q in range(pi.shape[0]):
        xi = solve(pi[q], eta_all[q], rcond)
        out[q] = coulomb_kernel_of(xi, lattice, grid, kmesh, q)
    return out


def kernel_v_route(pi, eta_all, lattice, grid, kmesh, rcond=1e-13, qs=None):
    """W^q = Pi^{q+} V^q Pi^{q+} (eqs. (7)-(8)); eta_all indexed like qs."""
    qs = list(range(pi.shape[0])) if qs is None else list(qs)
    out = np.empty((len(qs),) + pi.shape[1:], dtype=np.complex128)
    for iq, q in enumerate(qs):
        v = coulomb_kernel_of(eta_all[iq], lattice, grid, kmesh, q)
        pinv, _ = pinv_hermitian(pi[q], rcond)
        out[iq] = pinv @ v @ pinv
    return out


def fit_and_kernel(orbitals, ip_index, lattice, grid, kmesh, rcond=1e-13, route="v"):
    """The whole fit of this module at once (small cases): X, Pi, eta, W."""
    x = ip_values(orbitals, ip_index)
    pi = metric_k(x, kmesh)
    nk = x.shape[0]
    eta = rhs(x, orbitals, kmesh, list(range(nk)))
    if route == "v":
        w = kernel_v_route(pi, eta, lattice, grid, kmesh, rcond)
    else:
        w = kernel_zeta_route(pi, eta, lattice, grid, kmesh, rcond)
    return x, pi, eta, w


def fragment_psi_at_ips(x, coeffs, kmesh):
    """psi_p(r_I + R) = N_k^{-1/2} sum_k exp(i k.R) sum_mu C^k_{mu p} X^k_{I mu}
    (eq. (17) at the interpolation points; Algorithm 2 first two steps),
    direct sum over k.  Returns [N_R, N_IP, n_f] with R in mesh C order."""
    nk = x.shape[0]
    t = np.matmul(x, coeffs)                                      # T^k_{Ip} = sum_mu X C
    j = geo.kmesh_indices(kmesh)
    m = np.asarray(kmesh, dtype=np.float64)
    phase = np.exp(2j * np.pi * ((j[:, None, :] * j[None, :, :]) / m).sum(-1))  # [R, k]
    # sum over k as one matrix product: [R, k] x [k, (I p)]
    psi = (phase @ t.reshape(nk, -1)).reshape((nk,) + t.shape[1:])
    return psi / np.sqrt(nk)


def fragment_r(x, coeffs, kmesh):
    """R^q_{I,pq} = N_k^{-1/2} sum_R exp(-i q.R) conj(psi_p) psi_q at r_I + R
    (eq. (20); Algorithm 2 outer product and transform), direct sum over R.
    Returns [N_q, N_IP, n_f, n_f]."""
    nk = x.shape[0]
    psi = fragment_psi_at_ips(x, coeffs, kmesh)                   # [R, I, p]
    pair = psi.conj()[:, :, :, None] * psi[:, :, None, :]        # [R, I, p, q]
    j = geo.kmesh_indices(kmesh)
    m = np.asarray(kmesh, dtype=np.float64)
    phase = np.exp(-2j * np.pi * ((j[:, None, :] * j[None, :, :]) / m).sum(-1))  # [q, R]
    # sum over R as one matrix product: [q, R] x [R, (I p q)]
    r = (phase @ pair.reshape(nk, -1)).reshape(pair.shape)
    return r / np.sqrt(nk)


def fragment_eri(x, coeffs, w, kmesh):
    """(pq|rs) = sum_q sum_IJ R^q_{I,pq} W^q_{IJ} R^{-q}_{J,rs}  (eq. (19))."""
    r = fragment_r(x, coeffs, kmesh)
    nq, nip, nf, _ = r.shape
    mq = geo.minus_q(kmesh)
    eri = np.zeros((nf * nf, nf * nf), dtype=np.complex128)
    for q in range(nq):
        a = r[q].reshape(nip, nf * nf)                            # [I, pq]
        b = r[mq[q]].reshape(nip, nf * nf)                        # [J, rs]
        eri += a.T @ w[q] @ b
    return eri.reshape(nf, nf, nf, nf)


def thc_kpoint_eri(x, w, kmesh, k_mu, mu, k_nu, nu, k_la, la, k_si, si):
    """Crystalline-basis ERI of eq. (9) in this module's convention:
    sum_IJ conj(X^{k_mu}_{I mu}) X^{k_nu}_{I nu} W^{q}_{IJ} conj(X^{k_la}_{J la}) X^{k_si}_{J si}
    with q = k_nu - k_mu (the density conj(phi_mu) phi_nu carries momentum
    k_nu - k_mu).  Zero unless momentum is conserved (handled by caller)."""
    j = geo.kmesh_indices(kmesh)
    q = geo.mesh_index(j[k_nu] - j[k_mu], kmesh)
    a = x[k_mu][:, mu].conj() * x[k_nu][:, nu]
    b = x[k_la][:, la].conj() * x[k_si][:, si]
    return a @ w[q] @ b
