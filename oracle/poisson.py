"""FFT-Poisson Coulomb sums and an explicit Ewald lattice sum (oracle).

For densities f, g periodic on a cell of volume Omega sampled at N grid
points x, the Coulomb integral per cell with a neutralising background is

    (f|g) = (Omega / N^2) sum_{K != 0} (4 pi/|K|^2) fhat(-K) ghat(K),
    fhat(K) = sum_x f(x) exp(-i K.x),

which is how the paper evaluates its Coulomb kernels "by FFT" (eqs. (6)-(7);
the grid infrastructure of the section on the crystalline GTO basis).  The
K box and the kernel come from ``geometry``.
"""
import math

import numpy as np


def coulomb_pair_sum(fhat, ghat, kernel, volume, npts):
    """(f|g) from DFTs over one index set: fhat, ghat [..., N] (numpy fftn
    order, flattened), kernel [N] = 4 pi/|K_s|^2 (0 at K = 0).  fhat(-K) is
    taken at the DFT index -s mod N, i.e. as given by the caller through
    ``reflect_index``."""
    return (volume / npts ** 2) * np.sum(fhat * kernel * ghat, axis=-1)


def reflect_index(shape):
    """Flat index of -s (mod shape) for every flat DFT index s (C order)."""
    idx = [(-np.arange(n)) % n for n in shape]
    grid = np.meshgrid(*idx, indexing="ij")
    return np.ravel_multi_index(grid, shape).reshape(-1)


def madelung_simple_cubic(eta=2.0, nreal=6, nrec=8):
    """zeta_SC of the simple-cubic lattice (unit lattice constant), from the
    Ewald split with parameter eta: the potential at a point charge from its
    images plus a neutralising background equals -zeta_SC/L.

        phi = sum_{T != 0} erfc(eta |T|)/|T|
            + (4 pi/Omega) sum_{K != 0} exp(-K^2/(4 eta^2))/K^2
            - 2 eta/sqrt(pi) - pi/(Omega eta^2),

    summed explicitly over integer lattice vectors (no FFT)."""
    phi = 0.0
    rng = range(-nreal, nreal + 1)
    for i in rng:
        for j in rng:
            for k in rng:
                if i == 0 and j == 0 and k == 0:
                    continue
                r = math.sqrt(i * i + j * j + k * k)
                phi += math.erfc(eta * r) / r
    rec = 0.0
    rngk = range(-nrec, nrec + 1)
    for i in rngk:
        for j in rngk:
            for k in rngk:
                if i == 0 and j == 0 and k == 0:
                    continue
                k2 = (2 * math.pi) ** 2 * (i * i + j * j + k * k)
                rec += math.exp(-k2 / (4 * eta * eta)) / k2
    phi += 4 * math.pi * rec - 2 * eta / math.sqrt(math.pi) - math.pi / (eta * eta)
    return -phi


def gaussian_self_energy_closed_form(sigma, length, zeta_sc):
    """Coulomb self-energy per cell of a unit Gaussian charge of standard
    deviation sigma, periodised in a cubic cell of side L with a neutralising
    background (Ewald identity with eta = 1/(2 sigma)):

        1/(sigma sqrt(pi)) - zeta_SC/L + 4 pi sigma^2/L^3  (+ O(erfc(L/2sigma)))."""
    return 1.0 / (sigma * math.sqrt(math.pi)) - zeta_sc / length \
        + 4.0 * math.pi * sigma ** 2 / length ** 3
