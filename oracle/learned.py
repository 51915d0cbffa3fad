"""Learned block preconditioner: features, targets and the scaled-gradient step, FP64.

Test infrastructure only (like the rest of `oracle/`): the GPU library computes all of this
itself; the tests compare the two.

The paper preconditions the gradient by solving Eq. precond, K^c H^u G - G H^o K^v = g,
with an inner CG (Sec. III.B).  The learned replacement predicts, for every
(u-atom I, o-atom J) block of the response pattern, an elementwise scaling c_IJ of the
gradient block, G_IJ = c_IJ * g_IJ, from features that only involve the two atoms:

  * the upper triangles (row-major, diagonal included) of S^u_II, H^u_II, S^o_JJ, H^o_JJ;
  * the generalised eigenvalues of (H^u_II, S^u_II) and (H^o_JJ, S^o_JJ), ascending: local
    estimates of the Kohn-Sham energies of Sec. III.B's preconditioner;
  * their differences eps^u_a - eps^o_b (a outer, b inner), local estimates of the
    energy differences that Eq. precond divides by;
  * the minimum-image distance between the centres of the two atoms' function boxes.

A second output t_IJ, fitted to log10 of the block's share of sum_i ||P^q_i||^2 over
converged vectors (+1e-8), scales a random initial guess: L0_IJ ~ N(0, 1) * sqrt(10^t_IJ).
The scaled gradient is used only when it is a descent direction for every state
(<g_i, G_i>_S > 0); otherwise the CG preconditioner of Eq. precond is used instead.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def n_features(bu: int, bo: int) -> int:
    return bu * (bu + 1) + bo * (bo + 1) + bu + bo + bu * bo + 1


def _upper(A):
    i, j = np.triu_indices(A.shape[0])
    return A[i, j]


def _box_centres(fs, h):
    """Centre of each atom's function box in bohr, (z, y, x) order (the distance below is
    symmetric in the axes)."""
    return (np.asarray(fs.origin, dtype=np.float64) + 0.5 * (np.asarray(fs.extent) - 1)) * h


def block_features(sysm, blocks: np.ndarray) -> np.ndarray:
    """[number of true entries of `blocks`, n_features] in row-major block order."""
    cfg = sysm.cfg
    bu, bo = sysm.vir.n_per_atom, sysm.occ.n_per_atom
    nA = cfg.n_atoms
    fu, fo = [], []
    for I in range(nA):
        s = slice(I * bu, (I + 1) * bu)
        S, H = sysm.S_u[s, s], sysm.H_u[s, s]
        fu.append((_upper(S), _upper(H), scipy.linalg.eigh(H, S, eigvals_only=True)))
    for J in range(nA):
        s = slice(J * bo, (J + 1) * bo)
        S, H = sysm.S_o[s, s], sysm.H_o[s, s]
        fo.append((_upper(S), _upper(H), scipy.linalg.eigh(H, S, eigvals_only=True)))
    cu = _box_centres(sysm.vir, cfg.h)
    co = _box_centres(sysm.occ, cfg.h)
    rows = []
    for I in range(nA):
        for J in np.nonzero(blocks[I])[0]:
            su, hu, eu = fu[I]
            so, ho, eo = fo[J]
            d = cu[I] - co[J]
            d -= cfg.L * np.round(d / cfg.L)
            rows.append(np.concatenate([su, hu, so, ho, eu, eo, (eu[:, None] - eo[None, :]).ravel(),
                                        [np.sqrt(np.sum(d * d))]]))
    return np.array(rows)


def block_view(sysm, X: np.ndarray, blocks: np.ndarray) -> np.ndarray:
    """[k, n_u, n_o] -> [k, number of blocks, n_u_per_atom * n_o_per_atom] (row-major blocks)."""
    bu, bo = sysm.vir.n_per_atom, sysm.occ.n_per_atom
    nA = sysm.cfg.n_atoms
    Xb = X.reshape(X.shape[0], nA, bu, nA, bo).transpose(0, 1, 3, 2, 4)
    I, J = np.nonzero(blocks)
    return Xb[:, I, J].reshape(X.shape[0], len(I), bu * bo)


def expand_blocks(sysm, vals: np.ndarray, blocks: np.ndarray) -> np.ndarray:
    """[number of blocks, n_u_per_atom * n_o_per_atom] -> dense [n_u, n_o] (zero outside)."""
    bu, bo = sysm.vir.n_per_atom, sysm.occ.n_per_atom
    nA = sysm.cfg.n_atoms
    out = np.zeros((nA, nA, bu, bo))
    I, J = np.nonzero(blocks)
    out[I, J] = vals.reshape(-1, bu, bo)
    return out.transpose(0, 2, 1, 3).reshape(nA * bu, nA * bo)


def guess_target(sysm, Pq: np.ndarray, blocks: np.ndarray) -> np.ndarray:
    """t_IJ = log10(share of sum_i ||P^q_i,IJ||^2 + 1e-8) for converged vectors Pq [k, n_u, n_o]."""
    w = np.sum(block_view(sysm, Pq, blocks) ** 2, axis=(0, 2))
    return np.log10(w / np.sum(w) + 1e-8)


def guess_scale(t: np.ndarray) -> np.ndarray:
    return np.sqrt(10.0 ** t)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32).copy()
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
