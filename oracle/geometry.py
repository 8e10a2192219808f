"""Cell geometry for the oracle: grid points, k mesh, G+q box, Coulomb kernel.

Conventions (paper section "Periodic k-point FFTISDF representation of
integrals"; eq. (1) for the Bloch sums):

* lattice rows a1, a2, a3; reciprocal rows b_i with a_i . b_j = 2 pi delta_ij;
* unit-cell grid in C order, fractional coordinate of index i_d is i_d/n_d;
* Gamma-centred k mesh, mesh integer j_d in [0, m_d), k = sum_d (j_d/m_d) b_d;
  a momentum difference q is the mesh difference modulo m (eq. (2): q is the
  pair momentum shifted into the first Brillouin zone);
* the Coulomb kernel is 4 pi / |K|^2 with the K = 0 term dropped
  (neutralising background), K = G + q.
"""
import numpy as np


def reciprocal(lattice):
    """Rows b_i of 2 pi A^{-T}."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(lattice, dtype=np.float64)).T


def kmesh_indices(kmesh):
    """Mesh integers j of all k points, C order, shape [N_k, 3]."""
    m1, m2, m3 = kmesh
    j = np.stack(np.meshgrid(np.arange(m1), np.arange(m2), np.arange(m3),
                             indexing="ij"), axis=-1)
    return j.reshape(-1, 3)


def mesh_index(j, kmesh):
    """C-order index of mesh integer vectors j (taken modulo the mesh)."""
    j = np.asarray(j) % np.asarray(kmesh)
    return (j[..., 0] * kmesh[1] + j[..., 1]) * kmesh[2] + j[..., 2]


def k_plus_q(kmesh):
    """Table kq[k, q] = index of the mesh point j_k + j_q (modulo m)."""
    j = kmesh_indices(kmesh)
    return mesh_index(j[:, None, :] + j[None, :, :], kmesh)


def minus_q(kmesh):
    """Index of -q for every q of the mesh."""
    return mesh_index(-kmesh_indices(kmesh), kmesh)


def wrap(i, n):
    """Representative of integer i modulo n in [-n/2, n/2) (floor(n/2))."""
    i = np.asarray(i)
    return ((i + n // 2) % n) - n // 2


def grid_frac(grid):
    """Fractional coordinates of the unit-cell grid points, [N_g, 3]."""
    n1, n2, n3 = grid
    i = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3),
                             indexing="ij"), -1).reshape(-1, 3)
    return i / np.asarray(grid, dtype=np.float64)


def q_frac_wrapped(jq, kmesh):
    """Fractional (units of b) momentum of mesh difference jq, wrapped to
    [-1/2, 1/2) per axis (for even m the tie is at -1/2)."""
    m = np.asarray(kmesh)
    return wrap(np.asarray(jq), m) / m


def coulomb_g_plus_q(lattice, grid, qfrac):
    """c(G+q) = 4 pi/|G+q|^2 on the DFT index set of the unit-cell grid.

    G = B g with g in [-n/2, n/2) per axis (numpy FFT index order, C order
    over the grid), q = B qfrac; the term with G+q = 0 is 0.  Returns the
    kernel as a float64 array of shape [N_g]."""
    b = reciprocal(lattice)
    n1, n2, n3 = grid
    g = np.stack(np.meshgrid(wrap(np.arange(n1), n1), wrap(np.arange(n2), n2),
                             wrap(np.arange(n3), n3), indexing="ij"), -1).reshape(-1, 3)
    kf = g + np.asarray(qfrac)[None, :]
    kv = kf @ b
    k2 = np.einsum("ij,ij->i", kv, kv)
    out = np.zeros_like(k2)
    nz = k2 > 1e-24
    out[nz] = 4.0 * np.pi / k2[nz]
    return out


def supercell_lattice(lattice, kmesh):
    """Lattice of the Born-von Karman supercell, rows m_d a_d."""
    return np.asarray(lattice) * np.asarray(kmesh)[:, None]


def supercell_box(grid, kmesh, mode):
    """Integer representative (units of the supercell reciprocal vectors) of
    every DFT index s of the supercell grid, per axis, M_d = m_d n_d.

    mode "supercell": s -> wrap(s, M)  (the plain supercell FFT box);
    mode "kpoint":    s -> m wrap((s - jw)/m, n) + jw with jw = wrap(s mod m, m),
                      i.e. K = G + q with G in the unit-cell box and q wrapped,
                      the box the k-point Coulomb kernel sums over.
    Returns three integer arrays (one per axis)."""
    out = []
    for d in range(3):
        n, m = grid[d], kmesh[d]
        big = n * m
        s = np.arange(big)
        if mode == "supercell":
            out.append(wrap(s, big))
        elif mode == "kpoint":
            jw = wrap(s % m, m)
            g = ((s - jw) // m) % n
            out.append(m * wrap(g, n) + jw)
        else:
            raise ValueError(mode)
    return out


def coulomb_supercell(lattice, grid, kmesh, mode):
    """4 pi/|K|^2 on the supercell DFT index set (C order), K = 0 dropped."""
    bs = reciprocal(supercell_lattice(lattice, kmesh))
    r1, r2, r3 = supercell_box(grid, kmesh, mode)
    g = np.stack(np.meshgrid(r1, r2, r3, indexing="ij"), -1).reshape(-1, 3)
    kv = g @ bs
    k2 = np.einsum("ij,ij->i", kv, kv)
    out = np.zeros_like(k2)
    nz = k2 > 1e-24
    out[nz] = 4.0 * np.pi / k2[nz]
    return out
