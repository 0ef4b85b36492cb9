"""Test helpers: node matching by coordinates and oracle problem setup."""
import numpy as np
import torch
from scipy.spatial import cKDTree

from oracle.fem import assemble_A, assemble_B, assemble_M_inv_eta
from oracle.mesh import RefinedMesh, cube_macros, shell_macros
from oracle.system import velocity_basis


def match(x_or, x_lib, tol=1e-11):
    """perm with x_or[perm[i]] == x_lib[i]; asserts a bijection."""
    d, perm = cKDTree(x_or).query(x_lib)
    assert d.max() < tol, f"unmatched node, distance {d.max():.3e}"
    assert len(np.unique(perm)) == len(perm) == len(x_or)
    return perm


class Pair:
    """A library context and the oracle mesh of the same problem."""

    def __init__(self, kind, level, min_level=0, n_tan=1, n_rad=1, bc_inner=1, bc_outer=2):
        from paper_2506_04157_amd import StokesContext
        self.kind = kind
        self.ctx = StokesContext(kind, level=level, min_level=min_level, n_tan=n_tan, n_rad=n_rad,
                                 bc_inner=bc_inner, bc_outer=bc_outer)
        mac = cube_macros() if kind == "cube" else shell_macros(n_tan, n_rad, 0.55, 1.0)
        self.meshes = {l: RefinedMesh(mac, l) for l in range(min_level, level + 1)}
        self.perm2, self.perm1 = {}, {}
        for l, m in self.meshes.items():
            X2, f2 = self.ctx.coords(l, 2)
            X1, f1 = self.ctx.coords(l, 1)
            self.perm2[l] = match(m.X2, X2)
            self.perm1[l] = match(m.X1, X1)
            assert np.array_equal(m.flag2[self.perm2[l]], f2)
            assert np.array_equal(m.flag1[self.perm1[l]], f1)
        self.dir_flags = {1} if kind == "cube" else ({1} if bc_inner == 1 else set()) | ({2} if bc_outer == 1 else set())
        self.fs_flags = set() if kind == "cube" else ({1} if bc_inner == 2 else set()) | ({2} if bc_outer == 2 else set())
        self.L = level

    # vectors: oracle order (numpy) <-> library order (torch, device)
    def u_to_lib(self, v, l=None, dtype=torch.float64):
        p = self.perm2[self.L if l is None else l]
        return torch.tensor(v.reshape(3, -1)[:, p].ravel(), dtype=dtype, device="cuda")

    def u_to_or(self, t, l=None):
        p = self.perm2[self.L if l is None else l]
        a = t.detach().double().cpu().numpy().reshape(3, -1)
        out = np.empty_like(a)
        out[:, p] = a
        return out.ravel()

    def p_to_lib(self, v, l=None, dtype=torch.float64):
        return torch.tensor(v[self.perm1[self.L if l is None else l]], dtype=dtype, device="cuda")

    def p_to_or(self, t, l=None):
        p = self.perm1[self.L if l is None else l]
        a = t.detach().double().cpu().numpy()
        out = np.empty_like(a)
        out[p] = a
        return out

    def s2_to_lib(self, v, l=None):
        return torch.tensor(v[self.perm2[self.L if l is None else l]], dtype=torch.float64, device="cuda")

    def s2_to_or(self, t, l=None):
        p = self.perm2[self.L if l is None else l]
        a = t.detach().cpu().numpy()
        out = np.empty_like(a)
        out[p] = a
        return out

    def projector(self, l=None):
        m = self.meshes[self.L if l is None else l]
        Q, dm, fs = velocity_basis(m, self.dir_flags, self.fs_flags)
        return Q @ Q.T, Q


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def rowerr(y, ref, scale):
    """Largest per-entry error relative to the entry's own scale (for an
    operator row: sum_j |a_ij x_j|), so that one wrong node cannot hide in a
    norm over all nodes."""
    return float(np.max(np.abs(y - ref) / np.maximum(scale, 1e-300)))
