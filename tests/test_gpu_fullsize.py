"""GPU parity at the full benchmark size (icosahedral 10x2 shell, 12,000
macro-tets, level 4, N_u = 2.0e8) in the launch configuration the benchmark
times, on sampled outputs the oracle can compute on its own: the rows of A and
B at the nodes inside one macro-tet depend only on that macro's micro-tets, so
a one-macro oracle mesh reproduces them exactly.  Inputs are smooth functions
of the node coordinates, evaluated by each side at its own nodes.  Also the
symmetry of the projected A at full size.
"""
import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

import inputs
from oracle.fem import assemble_A, assemble_B
from oracle.mesh import MacroMesh, RefinedMesh, shell_macros

pytestmark = pytest.mark.gpu

L, NT, NR = 4, 10, 2


def _eta(X):
    return np.exp(1.5 * np.sin(3.0 * X[:, 0]) * np.cos(2.0 * X[:, 1]) + X[:, 2])


@pytest.fixture(scope="module")
def full():
    print("\n[full size: shell 10x2 level 4]", flush=True)
    from paper_2506_04157_amd import StokesContext
    sc = StokesContext("shell", level=L, min_level=0, n_tan=NT, n_rad=NR)
    X2, _ = sc.coords(which=2)
    X1, _ = sc.coords(which=1)
    sc.set_fields(torch.tensor(_eta(X1), device="cuda"))
    yield sc, X2, X1
    sc.close()


def _one_macro(mac_id):
    mm = shell_macros(NT, NR, 0.55, 1.0)
    t = mm.tets[mac_id]
    one = MacroMesh("shell", mm.vertices[t], [[0, 1, 2, 3]], mm.layer[t], 0.55, 1.0, NR)
    return RefinedMesh(one, L)


def _block_match(Xg, n_block, Xo):
    """Indices into Xg of the points Xo: the macro-interior nodes are numbered
    macro by macro, n_block per macro, so the block is found first."""
    nm = 60 * NT * NT * NR
    means = Xg[:nm * n_block].reshape(nm, n_block, 3).mean(axis=1)
    b = int(np.argmin(np.linalg.norm(means - Xo.mean(axis=0), axis=1)))
    d, j = cKDTree(Xg[b * n_block:(b + 1) * n_block]).query(Xo)
    assert d.max() < 1e-12, "macro-interior nodes not found"
    return b * n_block + j


@pytest.mark.parametrize("mac_id", [0, 5432, 11999])
def test_sampled_rows_of_A_and_B(full, mac_id):
    sc, X2, X1 = full
    m = _one_macro(mac_id)
    n2, n1 = m.n2, m.n1
    # macro-interior nodes of the one-macro mesh (all barycentric weights > 0)
    in2 = (m.keys2[:, 4:] > 0).all(axis=1)
    in1 = (m.keys1[:, 4:] > 0).all(axis=1)
    g2 = _block_match(X2, int(in2.sum()), m.X2[in2])
    g1 = _block_match(X1, int(in1.sum()), m.X1[in1])
    u_or = inputs.smooth_vector_field(7, m.X2).T.ravel()
    A = assemble_A(m, _eta(m.X1))
    B = assemble_B(m)
    # a smooth input makes A u and B u small differences of large terms, so
    # each row's error is measured against its scale sum_j |a_ij u_j|
    yA = (A @ u_or).reshape(3, n2)[:, in2]
    sA = (abs(A) @ abs(u_or)).reshape(3, n2)[:, in2]
    yB = (B @ u_or)[in1]
    sB = (abs(B) @ abs(u_or))[in1]
    N2 = len(X2)
    u = torch.tensor(inputs.smooth_vector_field(7, X2).T.ravel(), device="cuda")
    for dtype, tol in [(torch.float64, 1e-13), (torch.float32, 1e-5)]:
        y = sc.apply_A(u.to(dtype), bc=0).double().cpu().numpy().reshape(3, N2)[:, g2]
        err = np.abs(y - yA) / sA
        print(mac_id, dtype, err.max())
        assert err.max() <= tol, (mac_id, dtype)
    q = sc.apply_B(u, bc=0).cpu().numpy()[g1]
    assert (np.abs(q - yB) / sB).max() <= 1e-13


def test_projected_A_is_symmetric_at_full_size(full):
    sc, X2, X1 = full
    n = 3 * len(X2)
    x = torch.tensor(inputs.uniform(1, n), device="cuda")
    y = torch.tensor(inputs.uniform(2, n), device="cuda")
    xAy = torch.dot(x, sc.apply_A(y, bc=3)).item()
    yAx = torch.dot(y, sc.apply_A(x, bc=3)).item()
    assert abs(xAy - yAx) <= 1e-12 * abs(xAy)
