"""Cell geometry for the oracle: grid points, k mesh, G+q box, Coulomb kernel.

Conventions (paper section "Periodic k-point FFTISDF representation of
integrals"; eq. (1) for the Bloch sums):

* lattice rows a1, a2, a3; reciprocal rows b_i with a_i . b_j = 2 pi delta_ij;
* unit-cell grid in C order, fractional coordinate of index i_d is i_d/n_d;
* Gamma-centred k mesh, mesh integer j_d in [0, m_d), k = sum_d (j_d/m_d) b_d;
  a momentum difference q is the mesh difference modulo m (eq. (2): q is the
  pair momentum shifted into the first Brillouin zone);
* the Coulomb kernel is 4 pi / |K|^2 with the K = 0 term dropped
  (neutralising background), K = G + q.  On the DFT grid K is known only
  modulo n b per axis; each index takes the representative of its class
  nearest zero per axis, |K_d| <= n_d / 2 (fractional units), and where two
  representatives tie (K_d = +-n_d/2: the Nyquist plane of an even grid, or
  a zone-boundary q on an odd one) the kernel is their average.  That
  reading is symmetric under K -> -K, so the kernels at q and -q are
  reflections of each other and Pi^{-q}, V^{-q}, W^{-q} are the complex
  conjugates of those at q; it is the same kernel for the k-point form and
  for the Gamma-point supercell form.
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


def coulomb_nearest(frac, period, brows):
    """4 pi/|K|^2 for fractional vectors frac [N, 3] (units of the rows of
    brows) taken modulo period[d] per axis: the representative with
    |K_d| <= period_d / 2 per axis, averaged over the two where K_d sits at
    +-period_d/2 (2, 4 or 8 vectors); 0 where K = 0."""
    frac = np.asarray(frac, dtype=np.float64)
    per = np.asarray(period, dtype=np.float64)
    x = np.mod(frac + per / 2, per) - per / 2          # in [-p/2, p/2)
    tie = np.abs(x + per / 2) < 1e-9                    # K_d = -p/2 = +p/2 (mod p)
    acc = np.zeros(frac.shape[0])
    cnt = np.zeros(frac.shape[0])
    for s in range(8):
        sh = np.array([(s >> d) & 1 for d in range(3)], dtype=np.float64)
        ok = np.all(tie | (sh == 0), axis=1)            # shift only tied axes
        kv = (x + sh * per) @ brows
        k2 = np.einsum("ij,ij->i", kv, kv)
        nz = ok & (k2 > 1e-24)
        acc[nz] += 4.0 * np.pi / k2[nz]
        cnt[ok] += 1
    return acc / cnt


def coulomb_g_plus_q(lattice, grid, qfrac):
    """c(G+q) = 4 pi/|G+q|^2 on the DFT index set of the unit-cell grid.

    Index s_d of axis d stands for the class G_d = s_d (mod n_d); K = G + q
    with q = B qfrac takes the representative nearest zero per axis (ties
    averaged, see the module notes); the term with K = 0 is 0.  Returns the
    kernel as a float64 array of shape [N_g] (numpy FFT index order, C
    order over the grid)."""
    b = reciprocal(lattice)
    n1, n2, n3 = grid
    g = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3),
                             indexing="ij"), -1).reshape(-1, 3)
    return coulomb_nearest(g + np.asarray(qfrac)[None, :], grid, b)


def supercell_lattice(lattice, kmesh):
    """Lattice of the Born-von Karman supercell, rows m_d a_d."""
    return np.asarray(lattice) * np.asarray(kmesh)[:, None]


def coulomb_supercell(lattice, grid, kmesh):
    """4 pi/|K|^2 on the supercell DFT index set (C order), K = 0 dropped,
    with the same nearest-representative reading: supercell index s_d is
    the class K_d = s_d (mod m_d n_d) in units of the supercell reciprocal
    rows, i.e. K = G + q of the k-point form with the same representative."""
    bs = reciprocal(supercell_lattice(lattice, kmesh))
    shape = [grid[d] * kmesh[d] for d in range(3)]
    s = np.stack(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij"), -1).reshape(-1, 3)
    return coulomb_nearest(s, shape, bs)
