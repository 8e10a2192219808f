"""Tiles of the right-hand side (eq. (5), Algorithm 1 with Y = phi).

The library forms T^k_I(r) and its k convolution on tiles of grid points
and, where the whole range of interpolation points would leave fewer than
256 grid points a tile (the 1000-k workload), of interpolation points too.
Each element (I, r) is computed by the same operations in the same order
whatever tile holds it, so W^q from a context whose tile budget
(ISDF_RHS_TILE_BYTES, read at create) forces small tiles, with ragged last
tiles, must equal W^q of the default tiles bit for bit.  The cells cover the
register k convolution (meshes of axes <= 4), the LDS one and the
register-line one (6^3 mesh); the 10^3 mesh's tiles are checked against the
oracle by the large-cell tests."""
import os

import numpy as np
import pytest

import isdf_inputs as inp

pytestmark = pytest.mark.gpu

# a 6^3 mesh with more points than one point tile (60 = 3 x 16 + 12)
K6_IPS = inp.Config("t_k6_cube_ips", 121, 4.0, (8, 8, 8), (6, 6, 6), 3, 60, gmax=1.5, env=2.0)


def _kernel_and_tiles(d, budget=None):
    import paper_2601_16379_amd as pkg
    old = os.environ.get("ISDF_RHS_TILE_BYTES")
    try:
        if budget is not None:
            os.environ["ISDF_RHS_TILE_BYTES"] = str(budget)
        ctx = pkg.Isdf(d.lattice, d.cfg.grid, d.cfg.kmesh, d.orbitals, d.ip_index)
    finally:
        if old is None:
            os.environ.pop("ISDF_RHS_TILE_BYTES", None)
        else:
            os.environ["ISDF_RHS_TILE_BYTES"] = old
    st = ctx.stats()
    ctx.fit()
    ctx.coulomb_kernel("fp64")
    w = np.stack([ctx.get_kernel(q) for q in range(d.cfg.n_k)])
    ctx.close()
    return w, st["r_tile"], st["ip_tile"]


@pytest.mark.parametrize("cell,budget", [("t_mid_k4", 1 << 20), ("t_cond_k8", 1 << 20),
                                         ("t_k6_line", 1 << 18), ("k6_ips", 1 << 21)])
def test_point_tiles_equal_default_bitwise(cell, budget):
    d = inp.make_inputs(K6_IPS if cell == "k6_ips" else cell)
    cfg = d.cfg
    w0, rc0, ri0 = _kernel_and_tiles(d)
    w1, rc1, ri1 = _kernel_and_tiles(d, budget)
    print("%s: default tile %d grid points x %d points, forced %d x %d"
          % (cfg.name, rc0, ri0, rc1, ri1))
    assert ri0 == cfg.n_ip
    assert ri1 < cfg.n_ip and ri1 % 16 == 0 and cfg.n_ip % ri1 != 0
    assert rc1 == min(cfg.n_g, 256)
    assert np.array_equal(w0, w1)
