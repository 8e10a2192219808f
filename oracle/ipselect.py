"""Interpolation-point selection by pivoted Cholesky (oracle, plain form).

Test infrastructure only (see ``oracle/__init__``).  The paper's section
"Periodic k-point FFTISDF representation of integrals" selects the
interpolation points by a pivoted Cholesky decomposition of the products
phi^{k_mu}_mu(r) conj(phi^{k_nu}_nu(r)), the grid point r being the column
index, and keeps the first N_IP = c_IP N_AO pivots.

Written out: the products form a matrix Z with rows (mu, k_mu, nu, k_nu) and
columns r; the pivoted Cholesky of Z^H Z picks columns greedily.  Its
entries are

    M(r, r') = sum_{mu k_mu nu k_nu} conj(Z_r) Z_r'
             = | sum_k sum_mu phi^k_mu(r') conj(phi^k_mu(r)) |^2 = |G(r', r)|^2,

real and non-negative, with diagonal M(r, r) = rho(r)^2,
rho(r) = sum_k sum_mu |phi^k_mu(r)|^2.  The greedy (diagonally pivoted)
Cholesky keeps a residual diagonal d (initially diag M); at step i it takes
the point p of largest residual (the lowest index among equals), forms the
new column of the factor from column p of M minus the part already
explained by the previous columns, divides by sqrt(d(p)), and lowers d by
the square of that column:

    L[:, i] = (M[:, p] - sum_{j<i} L[:, j] L[p, j]) / sqrt(d(p))
    d      <- d - L[:, i]^2,   d(p) <- 0.

The chosen point leaves the candidate set, as a pivoted Cholesky moves the
pivot column out of the trailing matrix: its residual is exactly zero in
exact arithmetic (d(p) - L[p, i]^2 = 0) and is set to zero, so that rounding
can never select it again.

M is never formed: column p is |G(:, p)|^2 with G(:, p) one product of the
orbital matrix with the orbital values at p.
"""
import numpy as np


def gram_column(phi, p):
    """Column p of M: |sum_{k mu} phi(x) conj(phi(p))|^2 for every grid point
    x.  phi: [N_k N_orb, N_g] (rows (k, mu))."""
    g = phi.T @ phi[:, p].conj()
    return (g.real * g.real + g.imag * g.imag)


def pivoted_cholesky_points(orbitals, n_ip, with_gaps=False):
    """First n_ip pivots of the greedy pivoted Cholesky of M (in pivot
    order) and the residual diagonal after each step.  orbitals:
    [N_k, N_orb, N_g].  Returns (pivots [n_ip] int, residual_max [n_ip],
    L [N_g, n_ip], d [N_g] after the last step); with_gaps also returns
    gap [n_ip], the largest residual minus the second largest before each
    step (how far each choice is from a tie)."""
    nk, norb, ng = orbitals.shape
    phi = orbitals.reshape(-1, ng)
    rho = np.zeros(ng)
    for k in range(nk):
        ok = orbitals[k]
        rho += np.sum(ok.real * ok.real + ok.imag * ok.imag, axis=0)
    d = rho * rho
    lf = np.zeros((ng, n_ip))
    piv = np.zeros(n_ip, dtype=np.int64)
    dmax = np.zeros(n_ip)
    gap = np.zeros(n_ip)
    for i in range(n_ip):
        p = int(np.argmax(d))          # numpy returns the first index of the maximum
        piv[i] = p
        dmax[i] = d[p]
        if with_gaps:
            gap[i] = d[p] - np.max(np.delete(d, p)) if ng > 1 else d[p]
        if d[p] <= 0.0:
            raise ValueError("the products span only %d columns" % i)
        col = gram_column(phi, p) - lf[:, :i] @ lf[p, :i]
        lf[:, i] = col / np.sqrt(d[p])
        d = d - lf[:, i] ** 2
        d[p] = 0.0
    if with_gaps:
        return piv, dmax, lf, d, gap
    return piv, dmax, lf, d
