"""Brute-force dense Casida problem, the definition the method must reproduce.

Sec. II.A, Eq. TDDFT_ham: [[A, B], [-B, -A]] (X, Y) = omega (X, Y) with
A_{cv,c'v'} = delta (eps_c - eps_v) + K_{cv,c'v'}, B = K and
K_{cv,c'v'} = int int psi_c psi_v [1/|r - r'| + f_xc] psi_c' psi_v'  (spin dropped).

The Kohn-Sham-like states are the generalised eigenvectors of (H, S) in each function set
that the density kernels K^v and K^c project onto (K = sum a a^T, Sec. II.C).  The Coulomb
kernel is the periodic one with G = 0 dropped and f_xc the ALDA exchange kernel at rho0, on
the same grid as the method.  Valid only for untruncated (exactly idempotent) kernels.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import grid


def kernel_states(H, S, K, tol=1e-8):
    """Eigenpairs of (H, S) spanned by the density kernel K: weights w = a^T S K S a are
    1 for states in K and 0 otherwise.  When K projects onto a subspace that no set of
    eigenvectors of (H, S) spans (the complement projector of the joint representation,
    Sec. II.C, Eq. proj), the states are those of H restricted to range(K): with C an
    S-orthonormal basis of the range, the eigenpairs of C^T H C."""
    eps, C = scipy.linalg.eigh(H, S)
    w = np.einsum("ia,ij,jk,kl,la->a", C, S, K, S, C)
    sel = np.nonzero(w > 0.5)[0]
    if np.max(np.abs(w[sel] - 1.0)) <= tol and (len(sel) == len(w) or
                                                np.max(np.abs(w[w <= 0.5])) <= tol):
        return eps[sel], C[:, sel]
    return projected_states(H, S, K)


def projected_states(H, S, K, tol=1e-8):
    """States of H in range(K) for an S-idempotent K (K S K = K)."""
    if np.linalg.norm(K @ S @ K - K) > tol * np.linalg.norm(K):
        raise ValueError("density kernel is not idempotent")
    wk, V = scipy.linalg.eigh(S @ K @ S, S)          # S-orthonormal; 1 on range(K), 0 off it
    B = V[:, wk > 0.5]
    Hp = B.T @ H @ B
    e, U = np.linalg.eigh(0.5 * (Hp + Hp.T))
    return e, B @ U


class Casida:
    def __init__(self, sysm, xc: bool = True, hartree: bool = True, rho_floor: float = 1e-10,
                 coupling_scale: float = 1.0):
        N, L, h = sysm.cfg.N, sysm.cfg.L, sysm.cfg.h
        self.eps_v, Bv = kernel_states(sysm.H_o, sysm.S_o, sysm.K_v)
        self.eps_c, Ac = kernel_states(sysm.H_u, sysm.S_u, sysm.K_c)
        self.a, self.b = Ac, Bv
        uo = grid.to_global(N, sysm.vir).reshape(sysm.vir.n_fn, -1)
        oo = grid.to_global(N, sysm.occ).reshape(sysm.occ.n_fn, -1)
        psi_c = Ac.T @ uo                                   # [nc, N^3]
        psi_v = Bv.T @ oo                                   # [nv, N^3]
        rho0 = 2.0 * np.sum(psi_v ** 2, axis=0)             # closed shell
        fxc = grid.fxc_alda(rho0, rho_floor) if xc else np.zeros_like(rho0)
        nc, nv = len(self.eps_c), len(self.eps_v)
        pair = (psi_c[:, None, :] * psi_v[None, :, :]).reshape(nc * nv, -1)
        pot = fxc[None, :] * pair
        if hartree:
            pot = pot + grid.poisson_periodic(pair.reshape(-1, N, N, N), L).reshape(nc * nv, -1)
        K = h ** 3 * pair @ pot.T
        self.K = coupling_scale * 0.5 * (K + K.T)
        self.D = (self.eps_c[:, None] - self.eps_v[None, :]).ravel()
        self.rho0 = rho0.reshape(N, N, N)

    @property
    def A(self):
        return np.diag(self.D) + self.K

    @property
    def B(self):
        return self.K

    def omega_nonhermitian(self):
        """Positive eigenvalues of the 2n x 2n non-Hermitian Casida matrix, ascending."""
        A, B = self.A, self.B
        Mfull = np.block([[A, B], [-B, -A]])
        w = np.linalg.eigvals(Mfull)
        w = np.sort(w.real[w.real > 0])
        return w

    def omega_hermitian(self):
        """sqrt of eig(D^1/2 (A+B) D^1/2), valid because A - B = D > 0."""
        d = np.sqrt(self.D)
        Mh = d[:, None] * (self.A + self.B) * d[None, :]
        return np.sqrt(np.linalg.eigvalsh(0.5 * (Mh + Mh.T)))

    def omega_tda(self):
        return np.linalg.eigvalsh(self.A)

    def to_ngwf(self, x: np.ndarray) -> np.ndarray:
        """P = sum_cv a_c x_cv b_v^T for x of shape [..., nc, nv]."""
        return np.einsum("ic,...cv,jv->...ij", self.a, x, self.b)
