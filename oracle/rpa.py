"""k-point direct RPA correlation energy from W^q (oracle, plain form).

Test infrastructure only (see ``oracle/__init__``).  The paper's eq. (16)
integrates, over imaginary frequency, ln det(1 - P^q(iw)) + tr P^q(iw) with
the same polarisability-times-W as the opposite-spin MP2 energy, whose
second-order term it is; the integrals are done by quadrature.

Definitions (fixed here; pinned in ``tests/test_oracle_pins.py``), with the
canonical orbitals, Y^k = X^k C^k and the Green's-function polarisabilities
of ``oracle.mp2``:

    chi^q(iw)  = -int_0^inf [exp(+i w tau) chi^q(tau) + exp(-i w tau) chit^q(tau)] dtau
               = -N_k^-1 sum_k [ sum_{a in k, i in k+q} v v^H / (D - i w)
                               + sum_{i in k, a in k+q} u u^H / (D + i w) ],
      v = Y^k_a o conj(Y^{k+q}_i),  u = Y^k_i o conj(Y^{k+q}_a),  D = e_a - e_i > 0,
      evaluated from the time polarisabilities with a transform gamma[m, n]
      that maps exp(-D tau_n) to 1 / (D - i w_m) (a quadrature, or fitted):
      chi^q(iw_m) = -sum_n [gamma[m, n] chi^q(tau_n) + conj(gamma[m, n]) chit^q(tau_n)];
    E_dRPA     = sum_q int_{-inf}^{inf} dw / (2 pi N_k) [ln det(1 - chi^q W^q) + tr(chi^q W^q)]
               = sum_q int_0^inf dw / (pi N_k) Re[ln det(1 - chi^q W^q) + tr(chi^q W^q)]

per unit cell, in Hartree (chi^q(-iw)^H = chi^q(iw), so the integrand at -w
is the conjugate of that at w).  Readings: P^q(iw) = chi^q(iw) W^q with the
sign that makes E_dRPA < 0; the second-order term of the logarithm,
-1/2 tr(P^2), then gives exactly the opposite-spin MP2 energy E_OS of
``oracle.mp2``, as the paper states.  chi^q(iw) is not Hermitian without
time-reversal symmetry (the synthetic orbitals have none).
"""
import numpy as np

from . import geometry as geo
from . import mp2


def chi_omega_exact(y, e, n_occ, kmesh, q, omega):
    """chi^q(iw) from the closed form (Lorentzian sum over i, a)."""
    nk = y.shape[0]
    kq = geo.k_plus_q(kmesh)
    out = np.zeros((y.shape[1], y.shape[1]), dtype=np.complex128)
    for k in range(nk):
        kp = kq[k, q]
        # a at k, i at k + q
        v = (y[k][:, None, n_occ:] * y[kp][:, :n_occ, None].conj()).reshape(y.shape[1], -1)
        dv = (e[k][None, n_occ:] - e[kp][:n_occ, None]).reshape(-1)
        out -= (v / (dv - 1j * omega)) @ v.conj().T
        # i at k, a at k + q
        u = (y[k][:, :n_occ, None] * y[kp][:, None, n_occ:].conj()).reshape(y.shape[1], -1)
        du = (e[kp][None, n_occ:] - e[k][:n_occ, None]).reshape(-1)
        out -= (u / (du + 1j * omega)) @ u.conj().T
    return out / nk


def chi_omega_from_tau(y, e, n_occ, kmesh, transform, tau, qs=None):
    """chi^q(iw_m) = -sum_n [gamma[m, n] chi^q(tau_n) + conj(gamma[m, n])
    chit^q(tau_n)] with the mp2 polarisabilities at the times ``tau`` and the
    time-to-frequency transform gamma = ``transform`` [n_w, n_tau].  Returns
    [n_w, n_q, N_IP, N_IP]."""
    nk = y.shape[0]
    qs = list(range(nk)) if qs is None else list(qs)
    mu = mp2.chemical_potential(e, n_occ)
    out = np.zeros((transform.shape[0], len(qs), y.shape[1], y.shape[1]), dtype=np.complex128)
    for n, t in enumerate(tau):
        go, gv = mp2.greens(y, e, n_occ, t, mu)
        chi, chit = mp2.polarisabilities(go, gv, kmesh, qs)
        for m in range(transform.shape[0]):
            g = transform[m, n]
            out[m] -= g * chi + np.conj(g) * chit
    return out


def rpa_terms(p):
    """(Re ln det(1 - P) + Re tr P, -1/2 Re tr(P^2)) of one matrix P."""
    sgn, ld = np.linalg.slogdet(np.eye(p.shape[0]) - p)
    return (ld + np.log(sgn)).real + np.trace(p).real, -0.5 * np.trace(p @ p).real


def drpa_energy(x, w, c, e, n_occ, kmesh, omega, omega_weight, tau=None, transform=None):
    """(E_dRPA, its second-order term) on the frequency quadrature
    (omega, omega_weight) of [0, inf); chi^q(iw) from the closed form, or,
    with (tau, transform), from the polarisabilities at the times tau and the
    time-to-frequency transform (what the library computes)."""
    nk = x.shape[0]
    y = mp2.mo_at_ips(x, c)
    if tau is not None:
        chis = chi_omega_from_tau(y, e, n_occ, kmesh, transform, tau)
    e_rpa = e_2 = 0.0
    for q in range(nk):
        for m, (om, wo) in enumerate(zip(omega, omega_weight)):
            chi = chis[m, q] if tau is not None else chi_omega_exact(y, e, n_occ, kmesh, q, om)
            full, second = rpa_terms(chi @ w[q])
            e_rpa += wo / (np.pi * nk) * full
            e_2 += wo / (np.pi * nk) * second
    return e_rpa, e_2
