"""Convert a synthetic system to the array layout of the libtddft C-ABI (BSR matrices with
atom blocks, function boxes with (x, y, z) origins) and move response kernels between dense
[n_states, n_u, n_o] form and the [n_states, values of the response pattern] layout.  Pure layout; no
arithmetic of the method.

Response kernels P^p, P^q live on the response pattern: the blocks K^c S^u L S^o K^v can
reach from auxiliary matrices L on the truncation pattern M (Eq. auxiliary), or M itself
when the response kernels are truncated too (the linear-scaling mode)."""
from __future__ import annotations

import numpy as np


def _offsets(n_blocks: int, per: int) -> np.ndarray:
    return (np.arange(n_blocks + 1) * per).astype(np.int32)


def dense_to_bsr(A: np.ndarray, bmask: np.ndarray, br: int, bc: int):
    """Dense matrix -> (rowptr, colind, val) on the blocks where bmask is true."""
    nbr, nbc = bmask.shape
    rowptr = np.zeros(nbr + 1, dtype=np.int64)
    cols = []
    vals = []
    for i in range(nbr):
        js = np.nonzero(bmask[i])[0]
        rowptr[i + 1] = rowptr[i] + len(js)
        cols.append(js.astype(np.int32))
        if len(js):
            blk = A[i * br:(i + 1) * br].reshape(br, nbc, bc)[:, js, :]     # [br, k, bc]
            vals.append(np.transpose(blk, (1, 0, 2)).ravel())
    colind = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    val = np.concatenate(vals) if vals else np.zeros(0)
    return rowptr, colind.astype(np.int32), np.ascontiguousarray(val, dtype=np.float64)


def _nonzero_blocks(A, nb, b):
    return np.abs(A.reshape(nb, b, nb, b)).max(axis=(1, 3)) > 0


def matrix_blocks(A, nb, b):
    """Block pattern a symmetric matrix is passed with: nonzero blocks, the diagonal, and
    the transpose pattern."""
    mask = _nonzero_blocks(A, nb, b)
    np.fill_diagonal(mask, True)
    return mask | mask.T


def _functions(fs, N):
    nA, per = fs.n_atoms, fs.n_per_atom
    origin = np.zeros((nA * per, 3), dtype=np.int32)
    extent = np.zeros((nA * per, 3), dtype=np.int32)
    sizes = []
    chunks = []
    for I in range(nA):
        oz, oy, ox = fs.origin[I]
        ez, ey, ex = fs.extent[I]
        for k in range(per):
            f = I * per + k
            origin[f] = (ox, oy, oz)
            extent[f] = (ex, ey, ez)
            v = np.ascontiguousarray(fs.vals[I][k], dtype=np.float64).ravel()
            sizes.append(v.size)
            chunks.append(v)
    off = np.zeros(nA * per + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return dict(n_fn=nA * per, origin=origin.ravel(), extent=extent.ravel(), off=off,
                val=np.concatenate(chunks))


def system_arrays(sysm) -> dict:
    """Everything tddft_create needs, as contiguous numpy arrays."""
    cfg = sysm.cfg
    nA = cfg.n_atoms
    no, nu = sysm.occ.n_per_atom, sysm.vir.n_per_atom
    out = dict(n=np.array([cfg.N] * 3, dtype=np.int32), L=np.array([cfg.L] * 3))
    out["occ"] = _functions(sysm.occ, cfg.N)
    out["vir"] = _functions(sysm.vir, cfg.N)
    ooff, uoff = _offsets(nA, no), _offsets(nA, nu)
    for name, A, b, off in (("S_o", sysm.S_o, no, ooff), ("H_o", sysm.H_o, no, ooff),
                            ("K_v", sysm.K_v, no, ooff), ("S_u", sysm.S_u, nu, uoff),
                            ("H_u", sysm.H_u, nu, uoff), ("K_c", sysm.K_c, nu, uoff)):
        rowptr, colind, val = dense_to_bsr(A, matrix_blocks(A, nA, b), b, b)
        out[name] = dict(nbr=nA, nbc=nA, row_off=off, col_off=off, rowptr=rowptr,
                         colind=colind, val=val)
    rowptr, colind, _ = dense_to_bsr(np.zeros((nA * nu, nA * no)), sysm.M, nu, no)
    out["M"] = dict(nbr=nA, nbc=nA, row_off=uoff, col_off=ooff, rowptr=rowptr, colind=colind,
                    val=None)
    return out


def response_blocks(sysm) -> np.ndarray:
    """Atom pairs (u-atom, o-atom) of the response pattern: M itself when the response
    kernels are truncated to it (the system's mask_p), else the blocks reachable in
    K^c S^u L S^o K^v from L on M (graph reachability over the nonzero blocks)."""
    if getattr(sysm.cfg, "mask_p", False):
        return np.asarray(sysm.M, dtype=bool)
    nA = sysm.cfg.n_atoms

    def nz(A, b):
        return matrix_blocks(A, nA, b)

    def bmul(X, Y):
        return (X.astype(np.int32) @ Y.astype(np.int32)) > 0
    nu, no = sysm.vir.n_per_atom, sysm.occ.n_per_atom
    left = bmul(nz(sysm.K_c, nu), nz(sysm.S_u, nu))
    right = bmul(nz(sysm.S_o, no), nz(sysm.K_v, no))
    return bmul(bmul(left, sysm.M), right)


def _index(sysm, blocks) -> np.ndarray:
    cfg = sysm.cfg
    nu, no = sysm.vir.n_per_atom, sysm.occ.n_per_atom
    idx = []
    nofn = sysm.occ.n_fn
    for I in range(cfg.n_atoms):
        for J in np.nonzero(blocks[I])[0]:
            r = I * nu + np.arange(nu)
            c = J * no + np.arange(no)
            idx.append((r[:, None] * nofn + c[None, :]).ravel())
    return np.concatenate(idx)


def p_index(sysm) -> np.ndarray:
    """Flat dense indices (into [n_u, n_o]) of the values of a response kernel in C-ABI
    order (blocks of the response pattern, row-major inside each block)."""
    return _index(sysm, response_blocks(sysm))


def dense_to_p(sysm, X: np.ndarray) -> np.ndarray:
    """[n, n_u, n_o] -> [n, values of the response pattern]"""
    idx = p_index(sysm)
    X = np.asarray(X)
    return np.ascontiguousarray(X.reshape(X.shape[0], -1)[:, idx])


def p_to_dense(sysm, V: np.ndarray) -> np.ndarray:
    idx = p_index(sysm)
    V = np.asarray(V)
    out = np.zeros((V.shape[0], sysm.vir.n_fn * sysm.occ.n_fn))
    out[:, idx] = V
    return out.reshape(V.shape[0], sysm.vir.n_fn, sysm.occ.n_fn)
