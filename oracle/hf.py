"""k-point Hartree-Fock Coulomb and exchange matrices from W^q (oracle,
plain form).

Test infrastructure only (see ``oracle/__init__``).  The paper's section on
quantum embedding and local correlation evaluates the exact exchange of
k-point Hartree-Fock from the factorised integrals (eq. (10)) as a sum over
q of W^q times the density matrix at the interpolation points, "which can
also be computed as a convolution"; the Coulomb matrix is the q = 0 term of
the same factorisation.

Definitions (fixed here; pinned in ``tests/test_oracle_pins.py``):

* density matrices P^k_{la sg} (one Hermitian matrix per k) describe the
  one-particle density matrix
      gamma(x, y) = N_k^-1 sum_k sum_{la sg} phi^k_la(x) P^k_{la sg} conj(phi^k_sg(y)),
  i.e. the block P^k in the supercell orbitals N_k^{-1/2} phi^k;
* the Coulomb and exchange matrices are those of gamma in the same basis,
      J^k_{mu nu} = N_k^-1 sum_k' sum_{la sg} (mu k, nu k | sg k', la k') P^k'_{la sg}
      K^k_{mu nu} = N_k^-1 sum_k' sum_{la sg} (mu k, la k' | sg k', nu k) P^k'_{la sg}
  with the crystalline ERIs of eq. (9) in this package's convention
  (``kpoint.thc_kpoint_eri``: conjugate on the first and third index, W^q
  with q = (momentum of the second index) - (momentum of the first));
  K is returned without the minus sign with which eq. (10) enters it into
  the Fock matrix;
* with rho^k_{IJ} = sum_{la sg} X^k_{I la} P^k_{la sg} conj(X^k_{J sg}) this
  gives eq. (10) in this convention,
      K^k_{mu nu} = N_k^-1 sum_IJ conj(X^k_{I mu}) X^k_{J nu} sum_q W^q_{IJ} rho^{k+q}_{IJ},
      J^k_{mu nu} = N_k^-1 sum_I conj(X^k_{I mu}) X^k_{I nu} sum_J W^0_{IJ} n_J,
      n_J = sum_k rho^k_{JJ}  (N_k times the density at r_J).
The sums over k and q are direct (no convolution theorem).
"""
import numpy as np

from . import geometry as geo
from .kpoint import thc_kpoint_eri


def density_at_ips(x, dm):
    """rho^k_{IJ} = sum_{la sg} X^k_{I la} P^k_{la sg} conj(X^k_{J sg}).
    x: [N_k, N_IP, N_orb]; dm: [N_k, N_orb, N_orb].  Returns [N_k, N_IP, N_IP]."""
    return np.matmul(np.matmul(x, dm), np.transpose(x.conj(), (0, 2, 1)))


def exchange(x, w, dm, kmesh):
    """K^k_{mu nu} = N_k^-1 sum_IJ conj(X^k_{I mu}) X^k_{J nu}
    sum_q W^q_{IJ} rho^{k+q}_{IJ}  (eq. (10)), direct sum over q.
    w: [N_k, N_IP, N_IP] (every q).  Returns [N_k, N_orb, N_orb]."""
    nk = x.shape[0]
    rho = density_at_ips(x, dm)
    kq = geo.k_plus_q(kmesh)
    out = np.empty((nk, x.shape[2], x.shape[2]), dtype=np.complex128)
    for k in range(nk):
        m = np.zeros_like(rho[0])
        for q in range(nk):
            m += w[q] * rho[kq[k, q]]
        out[k] = x[k].conj().T @ m @ x[k] / nk
    return out


def exchange_at(x, w, dm, kmesh, ks):
    """K^k of ``exchange`` for the listed k only (the same sums).  Returns
    [len(ks), N_orb, N_orb]."""
    nk = x.shape[0]
    kq = geo.k_plus_q(kmesh)
    xh = np.transpose(x.conj(), (0, 2, 1))
    out = np.empty((len(ks), x.shape[2], x.shape[2]), dtype=np.complex128)
    for i, k in enumerate(ks):
        m = np.zeros((x.shape[1], x.shape[1]), dtype=np.complex128)
        for q in range(nk):
            kp = kq[k, q]
            m += w[q] * (x[kp] @ dm[kp] @ xh[kp])
        out[i] = x[k].conj().T @ m @ x[k] / nk
    return out


def coulomb(x, w, dm):
    """J^k_{mu nu} = N_k^-1 sum_I conj(X^k_{I mu}) X^k_{I nu} (W^0 n)_I,
    n_J = sum_k rho^k_{JJ} (the q = 0 term of eq. (9) contracted with P).
    Returns [N_k, N_orb, N_orb]."""
    nk = x.shape[0]
    # diagonal of rho^k only: n_J = sum_k sum_{la sg} X^k_{J la} P^k_{la sg} conj(X^k_{J sg})
    n = np.einsum("kjl,kls,kjs->j", x, dm, x.conj(), optimize=True)
    v = w[0] @ n
    return np.stack([x[k].conj().T @ (v[:, None] * x[k]) for k in range(nk)]) / nk


def jk_from_eri(x, w, dm, kmesh):
    """J and K by contracting the crystalline ERIs of eq. (9)
    (``kpoint.thc_kpoint_eri``) element by element with P: the plain
    definitions above, for tiny cells."""
    nk, _, norb = x.shape
    j = np.zeros((nk, norb, norb), dtype=np.complex128)
    kk = np.zeros((nk, norb, norb), dtype=np.complex128)
    for k in range(nk):
        for mu in range(norb):
            for nu in range(norb):
                sj = sk = 0.0
                for kp in range(nk):
                    for la in range(norb):
                        for sg in range(norb):
                            p = dm[kp, la, sg]
                            sj += thc_kpoint_eri(x, w, kmesh, k, mu, k, nu, kp, sg, kp, la) * p
                            sk += thc_kpoint_eri(x, w, kmesh, k, mu, kp, la, kp, sg, k, nu) * p
                j[k, mu, nu] = sj / nk
                kk[k, mu, nu] = sk / nk
    return j, kk
