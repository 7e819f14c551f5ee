"""Small hand-built systems used by the oracle pins."""
import numpy as np

from paper_2603_22274_amd import gen


def point_charges(pos, q, box, r_cut, alpha, grid=(16, 16, 16), sigma=None, eps=None, lig=None):
    n = len(pos)
    return gen.System(
        name='pins', box=np.asarray(box, np.float64), pos=np.asarray(pos, np.float32),
        charge=np.asarray(q, np.float32),
        sigma=np.full(n, 3.0, np.float32) if sigma is None else np.asarray(sigma, np.float32),
        epsilon=np.zeros(n, np.float32) if eps is None else np.asarray(eps, np.float32),
        mass=np.full(n, 12.0, np.float32),
        is_ligand=np.zeros(n, np.uint8) if lig is None else np.asarray(lig, np.uint8),
        bonds=np.zeros((0, 2), np.int32), bond_k=np.zeros(0, np.float32),
        bond_r0=np.zeros(0, np.float32), waters=np.zeros((0, 3), np.int32),
        excl=np.zeros((0, 2), np.int32), lambdas=np.array([[1.0, 1.0, 0.0]]),
        r_cut=r_cut, skin=0.0, ewald_alpha=alpha, grid=tuple(grid))


def rocksalt(n_side=8, r0=2.82):
    g = np.arange(n_side) * r0
    P = np.stack(np.meshgrid(g, g, g, indexing='ij'), -1).reshape(-1, 3)
    idx = np.stack(np.meshgrid(*[np.arange(n_side)] * 3, indexing='ij'), -1).reshape(-1, 3)
    q = np.where(idx.sum(1) % 2 == 0, 1.0, -1.0)
    return P + 0.5 * r0, q, np.array([n_side * r0] * 3)
