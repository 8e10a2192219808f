"""k-point opposite-spin MP2 (SOS-MP2) from W^q in the imaginary-time form
(oracle, plain form).

Test infrastructure only (see ``oracle/__init__``).  The paper's section on
quantum embedding and local correlation writes the opposite-spin MP2 energy
(eqs. (11)-(12)) as an integral over imaginary time of the trace of a product
of two polarisabilities in the interpolation-point basis, each a convolution
over k of two Green's functions (eqs. (13)-(15)), and scales it by
c_SOS = 1.3 (eq. (11)).

Definitions (fixed here; pinned in ``tests/test_oracle_pins.py``).  Canonical
orbitals psi^k_p = sum_mu C^k_{mu p} phi^k_mu with energies e^k_p, the first
n_occ of every k occupied; Y^k_{Ip} = psi^k_p(r_I) = (X^k C^k)_{Ip}.  With a
chemical potential m between the occupied and virtual energies (it cancels)
and tau >= 0:

    Go^k_{IJ}(tau) = sum_{i occ} Y^k_{Ii} exp(+tau (e_i - m)) conj(Y^k_{Ji})
    Gv^k_{IJ}(tau) = sum_{a vir} Y^k_{Ia} exp(-tau (e_a - m)) conj(Y^k_{Ja})
    chi^q_{IJ}     = N_k^-1 sum_k Gv^k_{IJ} conj(Go^{k+q}_{IJ})
    chit^q_{IJ}    = N_k^-1 sum_k Go^k_{IJ} conj(Gv^{k+q}_{IJ})   (= conj(chi^{-q}))
    F(tau)         = N_k^-1 sum_q tr[W^q chi^q W^q chit^q]          (real, >= 0)
    E_OS           = -int_0^inf F(tau) dtau,   E_SOS-MP2 = 1.3 E_OS

per unit cell, in Hartree.  Readings: the Green's functions of eq. (15) are
taken as the decaying ones (occupied propagating with exp(+tau e_i),
virtual with exp(-tau e_a), energies from the chemical potential): the
printed exponents grow with tau; a superscript q - k on a Green's function
is the complex conjugate at k - q, and q is counted as in this package's
W^q, which pairs Gv^k with conj(Go^{k+q}) (as Pi^q pairs T^k with
conj(T^{k+q})); the sign is that of the MP2 energy (E_OS < 0).  In exact
arithmetic this equals the closed form

    E_OS = -N_k^-3 sum_{k_i k_a k_j} sum_{ijab} |(i k_i, a k_a | j k_j, b k_b)|^2
           / (e_a + e_b - e_i - e_j),   k_b = k_j + k_i - k_a,

with the crystalline ERIs of eq. (9) in the canonical orbitals
(``kpoint.thc_kpoint_eri``), i.e. the supercell MP2 opposite-spin energy
-sum |(ia|jb)|^2 / Delta divided by N_k; and F(tau) is the same sum with
exp(-tau Delta) for 1/Delta, for every tau.
"""
import numpy as np

from . import geometry as geo


def mo_at_ips(x, c):
    """Y^k_{Ip} = sum_mu X^k_{I mu} C^k_{mu p}.  Returns [N_k, N_IP, N_mo]."""
    return np.matmul(x, c)


def chemical_potential(e, n_occ):
    """Midpoint between the highest occupied and lowest virtual energy."""
    return 0.5 * (np.max(e[:, :n_occ]) + np.min(e[:, n_occ:]))


def greens(y, e, n_occ, tau, mu):
    """(Go^k(tau), Gv^k(tau)), each [N_k, N_IP, N_IP]."""
    yo, yv = y[:, :, :n_occ], y[:, :, n_occ:]
    do = np.exp(tau * (e[:, :n_occ] - mu))
    dv = np.exp(-tau * (e[:, n_occ:] - mu))
    go = np.matmul(yo * do[:, None, :], np.transpose(yo.conj(), (0, 2, 1)))
    gv = np.matmul(yv * dv[:, None, :], np.transpose(yv.conj(), (0, 2, 1)))
    return go, gv


def polarisabilities(go, gv, kmesh, qs=None):
    """(chi^q, chit^q) for the listed q (all if None), direct sums over k."""
    nk = go.shape[0]
    qs = list(range(nk)) if qs is None else list(qs)
    kq = geo.k_plus_q(kmesh)
    chi = np.empty((len(qs),) + go.shape[1:], dtype=np.complex128)
    chit = np.empty_like(chi)
    for i, q in enumerate(qs):
        kpq = kq[:, q]                          # index of k + q for every k
        chi[i] = np.sum(gv * go[kpq].conj(), axis=0) / nk
        chit[i] = np.sum(go * gv[kpq].conj(), axis=0) / nk
    return chi, chit


def os_integrand(x, w, c, e, n_occ, kmesh, tau):
    """F(tau) = N_k^-1 sum_q tr[W^q chi^q W^q chit^q] (w: [N_k, N_IP, N_IP],
    every q).  Returns the complex value (its imaginary part is rounding)."""
    nk = x.shape[0]
    y = mo_at_ips(x, c)
    go, gv = greens(y, e, n_occ, tau, chemical_potential(e, n_occ))
    chi, chit = polarisabilities(go, gv, kmesh)
    return sum(np.trace(w[q] @ chi[q] @ w[q] @ chit[q]) for q in range(nk)) / nk


def os_energy(x, w, c, e, n_occ, kmesh, tau, weight):
    """E_OS = -sum_n weight_n F(tau_n) on a quadrature of [0, inf)."""
    return -sum(wt * os_integrand(x, w, c, e, n_occ, kmesh, t).real for t, wt in zip(tau, weight))


def os_closed_form(x, w, c, e, n_occ, kmesh, tau=None):
    """The closed form from the crystalline ERIs in the canonical orbitals:
    E_OS (tau None) or F(tau) (exp(-tau Delta) in place of -1/Delta)."""
    nk = x.shape[0]
    y = mo_at_ips(x, c)
    j = geo.kmesh_indices(kmesh)
    tot = 0.0
    for ki in range(nk):
        for ka in range(nk):
            q = int(geo.mesh_index(j[ka] - j[ki], kmesh))
            # pair densities conj(psi_i) psi_a at the points: [I, (i a)]
            a_pair = (y[ki][:, :n_occ].conj()[:, :, None] * y[ka][:, None, n_occ:]).reshape(x.shape[1], -1)
            dia = (e[ka][None, n_occ:] - e[ki][:n_occ, None]).reshape(-1)
            for kj in range(nk):
                kb = int(geo.mesh_index(j[kj] + j[ki] - j[ka], kmesh))
                b_pair = (y[kj][:, :n_occ].conj()[:, :, None] * y[kb][:, None, n_occ:]).reshape(x.shape[1], -1)
                djb = (e[kb][None, n_occ:] - e[kj][:n_occ, None]).reshape(-1)
                v = a_pair.T @ w[q] @ b_pair                   # (i a | j b)
                delta = dia[:, None] + djb[None, :]
                if tau is None:
                    tot -= np.sum(np.abs(v) ** 2 / delta)
                else:
                    tot += np.sum(np.abs(v) ** 2 * np.exp(-tau * delta))
    return tot / nk ** 3
