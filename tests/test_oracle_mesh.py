"""Pins of the oracle's meshes, counts and blending map (CPU only)."""
import os

import numpy as np
import pytest

from oracle.fem import blend_jacobian, blend_map, volume
from oracle.mesh import (RefinedMesh, cube_macros, kuhn_cube, micro_tets,
                         shell_counts, shell_macros)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_dof_counts.txt")


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        t = line.split()
        rows.append((int(t[0]), int(t[1]), int(t[2]), int(t[3]), float(t[4]),
                     float(t[5]), float(t[6]), t[7]))
    return rows


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: r[7])
def test_closed_form_reproduces_printed_counts(row):
    nt, nr, L, cores, up, T, tol, _ = row
    n2, n1 = shell_counts(nt, nr, L)
    assert abs((3 * n2 + n1) / cores - up) <= tol * up
    assert abs(n2 / cores - T) <= tol * T


@pytest.mark.parametrize("nt,nr,L", [(1, 1, 0), (1, 1, 1), (2, 1, 0), (2, 1, 1), (1, 2, 1), (2, 1, 2), (3, 2, 0)])
def test_shell_node_counts_match_closed_form(nt, nr, L):
    mac = shell_macros(nt, nr, 0.55, 1.0)
    assert mac.n_macros == 60 * nt * nt * nr
    m = RefinedMesh(mac, L)
    assert (m.n2, m.n1) == shell_counts(nt, nr, L)
    assert m.ne == mac.n_macros * 8 ** L


@pytest.mark.parametrize("L", [0, 1, 2, 3])
def test_structured_refinement_of_kuhn_macros_is_the_kuhn_grid(L):
    """Bey refinement (octahedra cut along b <-> a+c) of the six Kuhn-ordered
    cube macros equals the Kuhn grid built directly."""
    m = RefinedMesh(cube_macros(), L)
    x2k, e2k, x1k, e1k = kuhn_cube(L)
    assert m.n2 == len(x2k) and m.n1 == len(x1k)
    s = 2 ** (L + 1)

    def tetset(x, e):
        key = np.round(x[e] * s).astype(np.int64)                 # (ne,10,3)
        key = key[:, :4]
        key = np.sort(key[..., 0] * 10 ** 6 + key[..., 1] * 10 ** 3 + key[..., 2], axis=1)
        return set(map(tuple, key))

    assert tetset(m.x2, m.e2) == tetset(x2k, e2k)


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_micro_tets_fill_the_macro(n):
    mt = micro_tets(n).astype(np.float64)
    d = np.linalg.det(np.stack([mt[:, 1] - mt[:, 0], mt[:, 2] - mt[:, 0], mt[:, 3] - mt[:, 0]], axis=2))
    assert np.all(np.abs(d) > 0.5)                     # lattice volume 1 (x 1/6)
    assert np.isclose(np.abs(d).sum(), n ** 3)


def test_conforming_faces():
    """Every face of the refined shell is shared by 2 elements or lies on a sphere."""
    m = RefinedMesh(shell_macros(1, 2, 0.55, 1.0), 1)
    faces = np.sort(np.concatenate([m.e1[:, [0, 1, 2]], m.e1[:, [0, 1, 3]],
                                    m.e1[:, [0, 2, 3]], m.e1[:, [1, 2, 3]]]), axis=1)
    u, cnt = np.unique(faces, axis=0, return_counts=True)
    assert cnt.max() == 2
    bnd = u[cnt == 1]
    f = m.flag1[bnd]
    assert np.all((f == f[:, :1]) & (f > 0))


def test_blending_fixes_vertices_and_spheres():
    mac = shell_macros(2, 2, 0.55, 1.0)
    m = RefinedMesh(mac, 1)
    for k in range(4):
        v = mac.vertices[mac.tets[:, k]]
        assert np.allclose(blend_map(v, m.blend_g, m.blend_s0), v, atol=1e-15)
    r = np.linalg.norm(m.X2, axis=1)
    assert np.allclose(r[m.flag2 == 1], 0.55, atol=1e-15)
    assert np.allclose(r[m.flag2 == 2], 1.0, atol=1e-15)
    # the middle layer r = 0.775 is a sphere too (radius interpolated per macro)
    x = m.x2
    assert r.min() >= 0.55 - 1e-15 and r.max() <= 1.0 + 1e-15


def test_blending_jacobian_matches_finite_differences():
    mac = shell_macros(1, 1, 0.55, 1.0)
    m = RefinedMesh(mac, 0)
    rng = np.random.default_rng(0)
    lam = rng.dirichlet(np.ones(4), size=len(mac.tets))
    xt = np.einsum("mk,mkd->md", lam, mac.vertices[mac.tets])
    J = blend_jacobian(xt, m.blend_g, m.blend_s0)
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (blend_map(xt + e, m.blend_g, m.blend_s0) - blend_map(xt - e, m.blend_g, m.blend_s0)) / (2 * h)
        assert np.allclose(J[:, :, d], fd, atol=1e-8)
    g, s0 = m.blend_g, m.blend_s0
    r = np.linalg.norm(xt, axis=1)
    d_ = xt / r[:, None]
    alpha = (np.einsum("mk,mk->m", g, xt) + s0) / r
    assert np.allclose(np.linalg.det(J), alpha ** 2 * np.einsum("mk,mk->m", g, d_), rtol=1e-12)


def test_blended_volume_converges_to_shell_volume():
    exact = 4.0 / 3.0 * np.pi * (1.0 - 0.55 ** 3)
    errs = [abs(volume(RefinedMesh(shell_macros(1, 1, 0.55, 1.0), L)) - exact) for L in range(3)]
    assert errs[2] < errs[1] < errs[0]
    assert errs[1] / errs[2] > 3.5            # O(h^2) quadrature/geometry error
    # unblended (flat) macro mesh misses the curved volume by far more
    flat = abs(volume(RefinedMesh(cube_macros(), 0)) - 1.0)
    assert flat < 1e-14
