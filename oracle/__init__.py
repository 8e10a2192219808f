"""Plain FP64 CPU oracle of the k-point ISDF path (test infrastructure only).

This package is the slow, obviously correct reference against which the HIP
library is checked.  It is test infrastructure: only ``tests/``, the smoke
check of ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may
import it.  The library never does, and this package imports nothing from the
library; the two share only the seeded input generators of ``isdf_inputs``.

Everything is complex128 / float64 numpy, written in the paper's order and
notation (section "Periodic k-point FFTISDF representation of integrals",
eqs. (2)-(8), Algorithm 1; fragment Hamiltonian, eqs. (17)-(20), Algorithm 2),
with direct sums over k and over lattice translations R instead of the
convolution theorem, so that each step can be checked against its equation by
eye.  Modules:

* ``geometry``  -- lattice, grid, k mesh, G+q box and the Coulomb kernel;
* ``poisson``   -- FFT-Poisson Coulomb sums and an explicit Ewald sum;
* ``supercell`` -- exact ERIs and Gamma-point ISDF on the Born-von Karman
  supercell (the plain definitions every k-point result must reproduce);
* ``kpoint``    -- the k-point fit, the Coulomb kernel and the fragment ERIs;
* ``ipselect``  -- interpolation points by pivoted Cholesky of the pair products;
* ``hf``        -- k-point Hartree-Fock Coulomb and exchange matrices from W^q
  (eq. (10));
* ``mp2``       -- k-point opposite-spin MP2 in the imaginary-time form
  (eqs. (11)-(15));
* ``rpa``       -- k-point direct RPA correlation energy (eq. (16)).

Every function is pinned by ``tests/test_oracle_pins.py``; none is
"parity unpinned" except the size of the ISDF approximation error itself on
synthetic orbitals, which the paper's accuracy figures (diamond, GTOs) cannot
fix.
"""
