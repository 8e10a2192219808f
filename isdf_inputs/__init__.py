"""Seeded synthetic inputs for the k-point ISDF path.

This module is shared by the FP64 oracle (``oracle/``) and by the HIP path's
tests and benchmark.  It holds no ISDF arithmetic: it only draws the cell,
the Bloch orbitals on the unit-cell grid, the interpolation-point indices, the
fragment coefficients and the request arrival times, all from fixed seeds.

Recipe (stand-ins for the paper's GTO/GTH workloads, which need PySCF):

* cell: cubic, lattice constant ``a`` bohr, uniform grid ``n^3`` in C order,
  ``r = (i1/n1) a1 + (i2/n2) a2 + (i3/n3) a3``;
* k-mesh: Gamma-centred ``m1 x m2 x m3``, ``k_j = sum_i (j_i/m_i) b_i`` with
  ``b = 2 pi A^-T``; k index in C order over ``j``;
* orbitals: ``phi^k_mu(r) = exp(i k.r) u^k_mu(r)`` with
  ``u = sum_{|g| <= gmax} c_g exp(i G.r)``, ``G = (2 pi/a) g``,
  ``c_g ~ N(0,1) exp(-|G|^2 / env)`` (complex normal with Re, Im ~ N(0,1/2)
  for complex orbitals; real orbitals take Re of the sum), then Loewdin
  orthonormalised per k with the grid metric ``S = (Omega/N_g) Phi^H Phi``;
* interpolation points: ``N_IP`` grid indices drawn without replacement with
  probability proportional to ``rho(r) = sum_k sum_mu |phi^k_mu(r)|^2``,
  returned sorted;
* fragments: ``C = Q`` of the QR factorisation of a complex Gaussian
  ``(N_k N_orb) x n_f`` matrix with the column phases fixed by ``diag(R)``
  (Haar-distributed orthonormal columns); ``C^k_{mu p} = Q[(k, mu), p]``;
  sizes uniform on the stated inclusive range;
* arrivals: exponential inter-arrival times at the stated rate (Poisson).

Every stream is seeded from ``numpy.random.SeedSequence([cfg_id, stream, ...])``.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import hashlib
import os
from typing import Optional

import numpy as np

__all__ = ["Config", "CONFIGS", "get_config", "Inputs", "make_inputs",
           "make_fragments", "make_arrivals", "kmesh_indices"]

STREAM_ORBITALS = 1
STREAM_IPS = 2
STREAM_FRAG_SIZES = 3
STREAM_FRAG_COEFFS = 4
STREAM_ARRIVALS = 5
STREAM_DENSITY = 6
STREAM_MO = 7


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    cfg_id: int
    a: float                 # cubic lattice constant, bohr
    grid: tuple              # (n1, n2, n3)
    kmesh: tuple             # (m1, m2, m3)
    n_orb: int
    n_ip: int
    gmax: float = 8.0        # plane-wave cutoff |g| <= gmax (integer units)
    env: float = 4.0         # envelope exp(-|G|^2/env), |G| in bohr^-1
    real: bool = False       # real orbitals (Gamma-only workloads)
    n_frag: int = 1
    frag_lo: int = 0         # fragment sizes uniform on [frag_lo, frag_hi]
    frag_hi: int = 0
    arrival_rate: float = 0.0

    @property
    def n_k(self) -> int:
        return int(np.prod(self.kmesh))

    @property
    def n_g(self) -> int:
        return int(np.prod(self.grid))

    @property
    def volume(self) -> float:
        return self.a ** 3


# The five workload shapes, plus small cases that the oracle finishes in
# seconds while still spanning several GPU tiles and ragged tails.
CONFIGS = {
    "c1_gamma_16": Config("c1_gamma_16", 1, 6.0, (16, 16, 16), (1, 1, 1), 8, 64,
                          real=True, n_frag=1, frag_lo=8, frag_hi=8),
    "c2_k2_24": Config("c2_k2_24", 2, 6.0, (24, 24, 24), (2, 2, 2), 16, 256,
                       n_frag=1, frag_lo=16, frag_hi=16),
    "c3_k4_32": Config("c3_k4_32", 3, 6.0, (32, 32, 32), (4, 4, 4), 26, 520,
                       n_frag=64, frag_lo=12, frag_hi=40),
    "c4_k6_36": Config("c4_k6_36", 4, 6.0, (36, 36, 36), (6, 6, 6), 40, 800,
                       n_frag=2000, frag_lo=20, frag_hi=80, arrival_rate=200.0),
    "c5_k10_40": Config("c5_k10_40", 5, 6.0, (40, 40, 40), (10, 10, 10), 52, 1040,
                        n_frag=500, frag_lo=20, frag_hi=120),
    # small parity cases
    "t_tiny_k1": Config("t_tiny_k1", 101, 4.0, (6, 6, 6), (1, 1, 1), 3, 12,
                        gmax=1.5, env=2.0, n_frag=1, frag_lo=3, frag_hi=3),
    "t_tiny_k2": Config("t_tiny_k2", 102, 4.0, (8, 8, 8), (2, 1, 2), 3, 14,
                        gmax=1.5, env=2.0, n_frag=2, frag_lo=2, frag_hi=4),
    "t_small_k2": Config("t_small_k2", 103, 5.0, (12, 12, 12), (2, 2, 2), 6, 72,
                         gmax=2.0, env=3.0, n_frag=3, frag_lo=5, frag_hi=9),
    "t_small_k3": Config("t_small_k3", 104, 5.0, (12, 12, 12), (3, 2, 3), 7, 90,
                         gmax=2.0, env=3.0, n_frag=4, frag_lo=4, frag_hi=11),
    "t_mid_k4": Config("t_mid_k4", 105, 6.0, (16, 16, 16), (2, 2, 4), 10, 150,
                       gmax=5.0, env=4.0, n_frag=6, frag_lo=6, frag_hi=14),
    # grid sizes of every FFT code path (radix pairs 2x5, 4x5, 3x6, 6x6, 5x8)
    "t_grid10_k1": Config("t_grid10_k1", 110, 5.0, (10, 10, 10), (1, 1, 1), 8, 30,
                          gmax=2.0, env=3.0, n_frag=1, frag_lo=4, frag_hi=4),
    "t_grid20_k3": Config("t_grid20_k3", 111, 5.0, (20, 20, 20), (3, 1, 1), 4, 40,
                          gmax=3.0, env=3.0, n_frag=1, frag_lo=6, frag_hi=6),
    "t_grid18_k2": Config("t_grid18_k2", 112, 5.0, (18, 18, 18), (1, 2, 1), 6, 36,
                          gmax=3.0, env=3.0, n_frag=1, frag_lo=5, frag_hi=5),
    "t_grid36_k2": Config("t_grid36_k2", 113, 6.0, (36, 36, 36), (2, 1, 1), 6, 40,
                          gmax=4.0, env=4.0, n_frag=1, frag_lo=6, frag_hi=6),
    "t_grid40_k1": Config("t_grid40_k1", 114, 6.0, (40, 40, 40), (1, 1, 1), 8, 36,
                          gmax=4.0, env=4.0, n_frag=1, frag_lo=4, frag_hi=4),
    # first mesh axis of length 4 (four lanes per element in the register k
    # convolution and pair transform) with axes of 2, odd n_orb, ragged tiles
    "t_m4_k16": Config("t_m4_k16", 115, 5.0, (10, 10, 10), (4, 2, 2), 7, 90,
                       gmax=2.0, env=3.0, n_frag=3, frag_lo=4, frag_hi=9),
    # mesh axes of 6 and 10 (the k-mesh shapes of workloads 4 and 5): the LDS
    # k transforms with axis lengths up to 8 and up to 16
    "t_k6_line": Config("t_k6_line", 116, 5.0, (10, 10, 10), (6, 1, 1), 5, 60,
                        gmax=2.0, env=3.0, n_frag=2, frag_lo=4, frag_hi=9),
    "t_k10_line": Config("t_k10_line", 117, 5.0, (8, 8, 8), (1, 10, 1), 4, 48,
                         gmax=1.5, env=2.0, n_frag=2, frag_lo=3, frag_hi=7),
    "t_k6_cube": Config("t_k6_cube", 118, 4.0, (6, 6, 6), (6, 6, 6), 2, 16,
                        gmax=1.5, env=2.0, n_frag=2, frag_lo=3, frag_hi=6),
    "t_k10_cube": Config("t_k10_cube", 119, 4.0, (4, 4, 4), (10, 10, 10), 2, 10,
                         gmax=1.0, env=2.0, n_frag=2, frag_lo=2, frag_hi=4),
    # ill-conditioned metrics like the large workloads (cond(Pi^q) 4e4-5e5,
    # workloads 3 and 4 measure 1e4-2e5): 33 interpolation points per
    # orbital on smooth orbitals
    "t_cond_k8": Config("t_cond_k8", 120, 6.0, (16, 16, 16), (2, 2, 2), 6, 200,
                        gmax=4.0, env=2.0, n_frag=2, frag_lo=6, frag_hi=10),
}


def get_config(name: str) -> Config:
    return CONFIGS[name]


def kmesh_indices(kmesh) -> np.ndarray:
    """Mesh integers ``j`` of every k point, C order, shape ``[N_k, 3]``."""
    m1, m2, m3 = kmesh
    j = np.stack(np.meshgrid(np.arange(m1), np.arange(m2), np.arange(m3),
                             indexing="ij"), axis=-1)
    return j.reshape(-1, 3)


@dataclasses.dataclass
class Inputs:
    cfg: Config
    lattice: np.ndarray      # [3, 3] rows a1, a2, a3 (bohr)
    orbitals: np.ndarray     # complex128 [N_k, N_orb, N_g]
    ip_index: np.ndarray     # int32 [N_IP], sorted grid indices

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.orbitals).view(np.uint8).tobytes())
        h.update(self.ip_index.astype(np.int32).tobytes())
        return h.hexdigest()


def _seed(cfg: Config, *stream) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg.cfg_id, *stream]))


def _plane_wave_set(cfg: Config):
    gm = int(np.floor(cfg.gmax))
    rng = np.arange(-gm, gm + 1)
    g = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), -1).reshape(-1, 3)
    g = g[np.einsum("ij,ij->i", g, g) <= cfg.gmax ** 2 + 1e-9]
    gvec = g * (2.0 * np.pi / cfg.a)
    envelope = np.exp(-np.einsum("ij,ij->i", gvec, gvec) / cfg.env)
    return g, envelope


def _orbitals_at_k(cfg: Config, kidx: int, jk: np.ndarray, g, envelope) -> np.ndarray:
    n1, n2, n3 = cfg.grid
    rng = _seed(cfg, STREAM_ORBITALS, kidx)
    npw = g.shape[0]
    if cfg.real:
        coef = rng.standard_normal((cfg.n_orb, npw)) * envelope
    else:
        coef = (rng.standard_normal((cfg.n_orb, npw))
                + 1j * rng.standard_normal((cfg.n_orb, npw))) * np.sqrt(0.5) * envelope
    # Evaluate sum_g c_g exp(2 pi i g.i/n) on the grid by placing the
    # coefficients (aliased modulo n) and taking an unnormalised inverse DFT.
    box = np.zeros((cfg.n_orb, n1, n2, n3), dtype=np.complex128)
    np.add.at(box, (slice(None), g[:, 0] % n1, g[:, 1] % n2, g[:, 2] % n3), coef)
    u = np.fft.ifftn(box, axes=(1, 2, 3)) * (n1 * n2 * n3)
    if cfg.real:
        u = u.real.astype(np.complex128)
    # Bloch phase exp(i k.r) = exp(2 pi i sum_d j_d i_d / (m_d n_d))
    m = cfg.kmesh
    ph = [np.exp(2j * np.pi * jk[d] * np.arange(cfg.grid[d]) / (m[d] * cfg.grid[d]))
          for d in range(3)]
    phase = ph[0][:, None, None] * ph[1][None, :, None] * ph[2][None, None, :]
    phi = (u * phase[None]).reshape(cfg.n_orb, -1)
    # Loewdin orthonormalisation with the grid metric (Omega/N_g) Phi^H Phi
    s = (cfg.volume / cfg.n_g) * (phi.conj() @ phi.T)
    w, v = np.linalg.eigh(s)
    s_inv_half = (v * (1.0 / np.sqrt(w))) @ v.conj().T
    return (s_inv_half.T @ phi)


def _workers(cfg: Config, nk: int) -> int:
    """Threads for the per-k generation: one for small cells, up to 16 for
    large ones (each k point is independent; BLAS runs single-threaded inside
    a worker, which gives the same numbers as a serial run)."""
    if nk * cfg.n_orb * cfg.n_g < (1 << 24):
        return 1
    return max(1, min(16, os.cpu_count() or 1, nk))


def make_orbitals(cfg: Config, k_subset: Optional[np.ndarray] = None,
                  out: Optional[np.ndarray] = None) -> np.ndarray:
    """Bloch orbitals ``[len(k_subset) or N_k, N_orb, N_g]`` (complex128),
    written into ``out`` when given."""
    g, envelope = _plane_wave_set(cfg)
    jks = kmesh_indices(cfg.kmesh)
    ks = np.arange(cfg.n_k) if k_subset is None else np.asarray(k_subset)
    if out is None:
        out = np.empty((len(ks), cfg.n_orb, cfg.n_g), dtype=np.complex128)

    def one(i):
        out[i] = _orbitals_at_k(cfg, int(ks[i]), jks[ks[i]], g, envelope)

    nw = _workers(cfg, len(ks))
    if nw == 1:
        for i in range(len(ks)):
            one(i)
    else:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1), cf.ThreadPoolExecutor(nw) as ex:
            list(ex.map(one, range(len(ks))))
    return out


def density(cfg: Config, orbitals: np.ndarray) -> np.ndarray:
    """rho(r) = sum_k sum_mu |phi^k_mu(r)|^2, summed per k and then over k in
    k order (threads over k for large cells)."""
    nk = orbitals.shape[0]
    part = np.empty((nk, orbitals.shape[2]))

    def one(k):
        o = orbitals[k]
        part[k] = (o.real * o.real + o.imag * o.imag).sum(axis=0)

    nw = _workers(cfg, nk)
    if nw == 1:
        for k in range(nk):
            one(k)
    else:
        with cf.ThreadPoolExecutor(nw) as ex:
            list(ex.map(one, range(nk)))
    rho = np.zeros(orbitals.shape[2])
    for k in range(nk):
        rho += part[k]
    return rho


def make_ip_index(cfg: Config, orbitals: np.ndarray) -> np.ndarray:
    rho = density(cfg, orbitals)
    p = rho / rho.sum()
    rng = _seed(cfg, STREAM_IPS)
    idx = rng.choice(cfg.n_g, size=cfg.n_ip, replace=False, p=p)
    return np.sort(idx).astype(np.int32)


def make_inputs(cfg, n_ip: Optional[int] = None) -> Inputs:
    """Cell, orbitals and interpolation points of a workload.

    ``n_ip`` overrides the configured count (``n_ip = N_g`` selects the whole
    grid, in order)."""
    if isinstance(cfg, str):
        cfg = get_config(cfg)
    orb = make_orbitals(cfg)
    if n_ip is not None and n_ip != cfg.n_ip:
        cfg = dataclasses.replace(cfg, n_ip=int(n_ip))
    if cfg.n_ip == cfg.n_g:
        ip = np.arange(cfg.n_g, dtype=np.int32)
    else:
        ip = make_ip_index(cfg, orb)
    lattice = np.eye(3) * cfg.a
    return Inputs(cfg, lattice, orb, ip)


def fragment_sizes(cfg: Config, n_frag: Optional[int] = None) -> np.ndarray:
    n = cfg.n_frag if n_frag is None else n_frag
    rng = _seed(cfg, STREAM_FRAG_SIZES)
    return rng.integers(cfg.frag_lo, cfg.frag_hi + 1, size=n).astype(np.int64)


def make_fragment(cfg: Config, f: int, n_f: int) -> np.ndarray:
    """Coefficients ``C[k, mu, p]`` (complex128 ``[N_k, N_orb, n_f]``)."""
    rng = _seed(cfg, STREAM_FRAG_COEFFS, f)
    n = cfg.n_k * cfg.n_orb
    if n_f > n:
        raise ValueError("fragment larger than the orbital space")
    z = (rng.standard_normal((n, n_f)) + 1j * rng.standard_normal((n, n_f))) * np.sqrt(0.5)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    q = q * (d / np.abs(d))[None, :]
    if cfg.real and cfg.n_k == 1:
        # Real Gamma-only workloads: the fragment of all orbitals is the
        # identity; smaller ones use real orthonormal coefficients.
        if n_f == n:
            return np.eye(n, dtype=np.complex128).reshape(1, n, n)
        zr = rng.standard_normal((n, n_f))
        q, r = np.linalg.qr(zr)
        q = (q * np.sign(np.diag(r))[None, :]).astype(np.complex128)
    return q.reshape(cfg.n_k, cfg.n_orb, n_f)


def make_density(cfg: Config, n_occ: Optional[int] = None, seed: int = 0) -> np.ndarray:
    """Closed-shell k-point density matrices ``P[k, mu, nu]`` (complex128
    ``[N_k, N_orb, N_orb]``): per k, 2 U U^H with U the first n_occ columns of
    a Haar-random unitary (QR of a complex Gaussian with the phases of R's
    diagonal removed); n_occ = N_orb // 2 (at least 1) unless given.
    Hermitian, positive semidefinite, trace 2 n_occ per k."""
    n = cfg.n_orb
    n_occ = max(1, n // 2) if n_occ is None else int(n_occ)
    rng = _seed(cfg, STREAM_DENSITY, seed)
    out = np.empty((cfg.n_k, n, n), dtype=np.complex128)
    for k in range(cfg.n_k):
        z = (rng.standard_normal((n, n_occ)) + 1j * rng.standard_normal((n, n_occ))) * np.sqrt(0.5)
        q, r = np.linalg.qr(z)
        q = q * (np.diag(r) / np.abs(np.diag(r)))[None, :]
        out[k] = 2.0 * (q @ q.conj().T)
    return out


def make_mo(cfg: Config, n_occ: Optional[int] = None, seed: int = 0):
    """Synthetic canonical orbitals of a k-point mean-field calculation:
    per k a Haar-random unitary ``C[k, mu, p]`` (complex128
    ``[N_k, N_orb, N_orb]``) and sorted energies ``e[k, p]`` (float64
    ``[N_k, N_orb]``), the first n_occ (N_orb // 2, at least 1) occupied,
    uniform in [-1.0, -0.3] Eh, the rest uniform in [0.2, 1.5] Eh (a gap of
    at least 0.5 Eh, as an insulator's).  Returns (C, e, n_occ)."""
    n = cfg.n_orb
    n_occ = max(1, n // 2) if n_occ is None else int(n_occ)
    rng = _seed(cfg, STREAM_MO, seed)
    c = np.empty((cfg.n_k, n, n), dtype=np.complex128)
    e = np.empty((cfg.n_k, n))
    for k in range(cfg.n_k):
        z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * np.sqrt(0.5)
        q, r = np.linalg.qr(z)
        c[k] = q * (np.diag(r) / np.abs(np.diag(r)))[None, :]
        e[k, :n_occ] = np.sort(rng.uniform(-1.0, -0.3, n_occ))
        e[k, n_occ:] = np.sort(rng.uniform(0.2, 1.5, n - n_occ))
    return c, e, n_occ


def laplace_grid(n: int, scale: float):
    """Quadrature for integrals over tau in [0, inf) of decaying exponentials:
    n-point Gauss-Legendre on x in (-1, 1) mapped by tau = scale (1 + x)/(1 - x)
    (weights times dtau/dx = 2 scale/(1 - x)^2).  Returns (tau, weight)."""
    x, w = np.polynomial.legendre.leggauss(int(n))
    tau = scale * (1.0 + x) / (1.0 - x)
    return tau, w * 2.0 * scale / (1.0 - x) ** 2


def quadrature_transform(tau, tau_weight, omega):
    """Time-to-frequency transform of a plain quadrature:
    gamma[m, n] = tau_weight[n] exp(i omega[m] tau[n]) (complex128
    [n_omega, n_tau]), so that sum_n gamma[m, n] exp(-D tau_n) approximates
    int_0^inf exp(-(D - i omega_m) tau) dtau = 1 / (D - i omega_m); accurate
    only while the grid resolves exp(i omega tau)."""
    return np.asarray(tau_weight)[None, :] * np.exp(1j * np.outer(omega, tau))


def fitted_transform(tau, omega, d_min: float, d_max: float, n_d: int = 400):
    """Time-to-frequency transform fitted by least squares: for every omega_m
    the coefficients gamma[m, :] minimise the relative error of
    sum_n gamma[m, n] exp(-D tau_n) against 1 / (D - i omega_m) over D on
    n_d log-spaced points of [d_min, d_max] (the range of the excitation
    energies), singular values below 1e-14 of the largest dropped.  Accurate
    at every omega, including those a plain quadrature cannot resolve.
    Returns complex128 [n_omega, n_tau]."""
    tau = np.asarray(tau, dtype=np.float64)
    d = np.geomspace(d_min, d_max, int(n_d))
    basis = np.exp(-np.outer(d, tau))
    out = np.empty((len(omega), tau.size), dtype=np.complex128)
    for m, w in enumerate(omega):
        target = 1.0 / (d - 1j * w)
        scale = 1.0 / np.abs(target)
        u, sv, vh = np.linalg.svd(basis * scale[:, None], full_matrices=False)
        keep = sv > 1e-14 * sv[0]
        out[m] = vh[keep].conj().T @ ((u[:, keep].conj().T @ (target * scale)) / sv[keep])
    return out


def excitation_range(e: np.ndarray, n_occ: int):
    """(smallest, largest) e_a - e_i over all k of canonical energies e[k, p]."""
    occ, vir = e[:, :n_occ], e[:, n_occ:]
    return float(vir.min() - occ.max()), float(vir.max() - occ.min())


def make_fragments(cfg: Config, n_frag: Optional[int] = None):
    sizes = fragment_sizes(cfg, n_frag)
    return [make_fragment(cfg, f, int(nf)) for f, nf in enumerate(sizes)]


def make_arrivals(cfg: Config, n: int, rate: Optional[float] = None) -> np.ndarray:
    """Arrival times (seconds, from 0) of ``n`` requests, Poisson at ``rate``/s."""
    lam = cfg.arrival_rate if rate is None else rate
    rng = _seed(cfg, STREAM_ARRIVALS)
    if lam <= 0:
        return np.zeros(n)
    return np.cumsum(rng.exponential(1.0 / lam, size=n)) - 0.0
