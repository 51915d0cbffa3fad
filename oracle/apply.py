"""The full-TDDFT operator in mixed unoccupied-occupied NGWF space, FP64.

Follows Sec. III.A, Eq. operator_RPA: for response kernels P^p, P^q (rows: u-set, columns:
o-set)

    f_p = K^c H^u P^p - P^p H^o K^v
    f_q = K^c H^u P^q - P^q H^o K^v + 2 K^c V_SCF[P^q] K^v

where V_SCF[P]_ab = h^3 sum_r u_a(r) (V_H[rho] + f_xc rho)(r) o_b(r) and
rho(r) = sum_ab u_a(r) P_ab o_b(r) (Sec. III.A, response densities).  The factor 2 is
A + B = D + 2K (Sec. II.A).  Contravariant quantities; the metric is
<X, Y> = Tr[X^T S^u Y S^o] (Sec. II.C).

Truncation (Sec. III.A, Eq. auxiliary): the auxiliary matrices L are truncated to the
block pattern M; the response kernels are P = K^c S^u L S^o K^v, whose block pattern Mp is
that of the product (wider than M).  In the linear-scaling mode of Sec. IV.C the response
kernels are truncated as well, to M itself, so Mp = M and the invariance constraint holds
only approximately.  Every product is exact; results are restricted to Mp.
"""
from __future__ import annotations

import numpy as np

from . import grid


class Operator:
    """Dense FP64 form of the operator for one system (inputs as produced by the
    synthetic generator: S, H, K for both sets, the function sets and the pattern M)."""

    def __init__(self, sysm, xc: bool = True, hartree: bool = True, rho_floor: float = 1e-10,
                 coupling_scale: float = 1.0, tda: bool = False):
        self.sys = sysm
        self.N = sysm.cfg.N
        self.L = sysm.cfg.L
        self.h = sysm.cfg.h
        self.Su, self.Hu, self.Kc = sysm.S_u, sysm.H_u, sysm.K_c
        self.So, self.Ho, self.Kv = sysm.S_o, sysm.H_o, sysm.K_v
        nb = (sysm.vir.n_per_atom, sysm.occ.n_per_atom)
        self.mask_L = np.kron(sysm.M, np.ones(nb))
        self.mask = np.kron(response_pattern(sysm), np.ones(nb))
        self.xc = xc
        self.hartree = hartree
        self.coupling_scale = coupling_scale
        # Tamm-Dancoff approximation (Sec. II.B): B = 0, both halves see A = D + K
        self.tda = tda
        self.rho_floor = rho_floor
        self.KcHu = self.Kc @ self.Hu
        self.HoKv = self.Ho @ self.Kv
        self.KcSu = self.Kc @ self.Su
        self.SoKv = self.So @ self.Kv
        # ground-state density of a closed shell: rho0 = 2 sum_bb' o_b K^v_bb' o_b'
        self.rho0 = 2.0 * grid.density(self.N, sysm.occ, sysm.occ, self.Kv[None])[0]
        self.fxc = grid.fxc_alda(self.rho0, rho_floor) if xc else np.zeros_like(self.rho0)

    # -- pieces ---------------------------------------------------------------------------
    def T(self, X: np.ndarray) -> np.ndarray:
        """Kohn-Sham-difference part: mask_M(K^c H^u X - X H^o K^v)."""
        return self.mask * (self.KcHu @ X - X @ self.HoKv)

    def response_density(self, Pq: np.ndarray) -> np.ndarray:
        return grid.density(self.N, self.sys.vir, self.sys.occ, Pq)

    def potential(self, rho: np.ndarray) -> np.ndarray:
        V = np.zeros_like(rho)
        if self.hartree:
            V += grid.poisson_periodic(rho, self.L)
        V += self.fxc[None] * rho
        return V

    def vscf(self, Pq: np.ndarray) -> np.ndarray:
        rho = self.response_density(Pq)
        V = self.potential(rho)
        return grid.potential_integrals(self.N, self.h, self.sys.vir, self.sys.occ, V)

    def coupling(self, Pq: np.ndarray) -> np.ndarray:
        """2 mask_M(K^c V_SCF[P^q] K^v) (times the optional test coupling scale); the factor
        is 1 in the Tamm-Dancoff mode (A = D + K instead of A + B = D + 2K)."""
        Vm = self.vscf(Pq)
        factor = 1.0 if self.tda else 2.0
        return self.coupling_scale * factor * self.mask * (self.Kc @ Vm @ self.Kv)

    # -- the operator ---------------------------------------------------------------------
    def apply(self, Pp: np.ndarray, Pq: np.ndarray):
        """(f_p, f_q) for stacks [n_states, n_u_fn, n_o_fn]."""
        Pp = np.asarray(Pp, dtype=np.float64)
        Pq = np.asarray(Pq, dtype=np.float64)
        fp = np.stack([self.T(x) for x in Pp])
        fq = np.stack([self.T(x) for x in Pq])
        if self.xc or self.hartree:
            fq = fq + self.coupling(Pq)
            if self.tda:
                fp = fp + self.coupling(Pp)
        return fp, fq

    # -- metric and projection -------------------------------------------------------------
    def metric(self, X: np.ndarray, Y: np.ndarray) -> float:
        """<X, Y> = Tr[X^T S^u Y S^o] (contravariant X, Y; Sec. II.C)."""
        return float(np.sum(X * (self.Su @ Y @ self.So)))

    def truncate(self, X: np.ndarray) -> np.ndarray:
        """Restriction of an auxiliary matrix to the truncation pattern M."""
        return self.mask_L * X

    def project(self, X: np.ndarray) -> np.ndarray:
        """Pi(L) = K^c S^u L S^o K^v for L on M (Sec. III.A, Eqs. invariance and
        auxiliary); exact, on Mp."""
        return self.mask * (self.KcSu @ self.truncate(X) @ self.SoKv)


def response_pattern(sysm) -> np.ndarray:
    """Atom-block pattern Mp of the response kernels.  In the linear-scaling mode (Sec.
    IV.C: every density matrix, the response kernels included, is truncated) it is M.
    Otherwise it is the pattern of K^c S^u L S^o K^v for L on M (boolean products of the
    block patterns of the factors).  A factor's pattern is its nonzero blocks plus every
    atom's own block: density matrices are truncated by a radius (Sec. IV.C: the truncation
    gives them the pattern of the overlap matrices), so an atom's own block belongs to the
    pattern even where its values vanish (an atom that carries no occupied or no
    unoccupied weight)."""
    if getattr(sysm.cfg, "mask_p", False):
        return np.asarray(sysm.M, dtype=bool)
    nA = sysm.cfg.n_atoms

    def blocks(A, b):
        m = (np.abs(A.reshape(nA, b, nA, b)).max(axis=(1, 3)) > 0).astype(np.int64)
        np.fill_diagonal(m, 1)
        return m
    nu, no = sysm.vir.n_per_atom, sysm.occ.n_per_atom
    pu = blocks(sysm.K_c, nu) @ blocks(sysm.S_u, nu)
    po = blocks(sysm.S_o, no) @ blocks(sysm.K_v, no)
    return ((pu > 0).astype(np.int64) @ sysm.M.astype(np.int64) @ (po > 0).astype(np.int64)) > 0
