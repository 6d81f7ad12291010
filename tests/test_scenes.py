"""Seeded input generator: mesh topology, shapes, packing."""
import math

import numpy as np
import pytest

from paper_1812_04719_amd import scenes as S


@pytest.mark.parametrize("p", [4, 16, 24, 32])
def test_grid_mesh_counts_and_euler(p):
    t = S.grid_topology(p)
    assert t.nv == 2 * p * (p + 1) + 2
    assert t.nt == 4 * p * (p + 1)
    assert t.ne == 6 * p * (p + 1)
    assert t.nv - t.ne + t.nt == 2
    # every edge is shared by exactly two triangles (closed manifold)
    e = np.sort(np.concatenate([t.tri[:, [0, 1]], t.tri[:, [1, 2]], t.tri[:, [2, 0]]]), axis=1)
    _, cnt = np.unique(e, axis=0, return_counts=True)
    assert np.all(cnt == 2)


@pytest.mark.parametrize("p", [8, 32])
def test_outward_orientation(p):
    t = S.grid_topology(p)
    x = S.spheroid_body_points(p, 1.9, 1.0)
    a, b, c = x[t.tri[:, 0]], x[t.tri[:, 1]], x[t.tri[:, 2]]
    vol6 = np.einsum("ij,ij->i", a, np.cross(b, c))
    assert np.all(vol6 > 0)
    assert 0 < 4 / 3 * math.pi * 1.9 - vol6.sum() / 6 < 0.06 * 4 / 3 * math.pi * 1.9  # inscribed


def test_gauss_legendre_polar_nodes():
    th, _ = S.grid_angles(8)
    x, _ = np.polynomial.legendre.leggauss(9)
    assert np.allclose(np.cos(th[:-2:16]), x[::-1])


def test_spheroid_reduced_volume():
    a, b = S.spheroid_axes(0.91, 1.34)
    e = math.sqrt(1 - b * b / (a * a))
    area = 2 * math.pi * b * b * (1 + a / (b * e) * math.asin(e))
    vol = 4 / 3 * math.pi * a * b * b
    r0 = math.sqrt(area / (4 * math.pi))
    assert abs(r0 - 1.34) < 1e-12
    assert abs(vol / (4 / 3 * math.pi * r0 ** 3) - 0.91) < 1e-12


def test_fcc_config_volume_fraction_and_determinism():
    sc = S.make_config(3)
    assert sc.n_ves == 1440
    assert abs(np.prod(sc.box_len[0]) - 28.4 ** 3) < 1e-6
    assert abs(sc.meta["vf"] - 0.5766) < 1e-3
    assert np.abs(sc.x1 - sc.x0).max() <= 0.1
    sc2 = S.make_config(3)
    assert sc.sha256() == sc2.sha256()
