"""The full-TDDFT operator in mixed unoccupied-occupied NGWF space, FP64.

Follows Sec. III.A, Eq. operator_RPA: for response kernels P^p, P^q (rows: u-set, columns:
o-set)

    f_p = K^c H^u P^p - P^p H^o K^v
    f_q = K^c H^u P^q - P^q H^o K^v + 2 K^c V_SCF[P^q] K^v

where V_SCF[P]_ab = h^3 sum_r u_a(r) (V_H[rho] + f_xc rho)(r) o_b(r) and
rho(r) = sum_ab u_a(r) P_ab o_b(r) (Sec. III.A, response densities).  The factor 2 is
A + B = D + 2K (Sec. II.A).  Every product is exact; only the results are restricted to
the block pattern M of the response kernels (the paper truncates P^p, P^q, P^v and P^c,
Sec. IV.C).  Contravariant quantities; the metric is <X, Y> = Tr[X^T S^u Y S^o] (Sec. II.C).
"""
from __future__ import annotations

import numpy as np

from . import grid


class Operator:
    """Dense FP64 form of the operator for one system (inputs as produced by the
    synthetic generator: S, H, K for both sets, the function sets and the pattern M)."""

    def __init__(self, sysm, xc: bool = True, hartree: bool = True, rho_floor: float = 1e-10,
                 coupling_scale: float = 1.0):
        self.sys = sysm
        self.N = sysm.cfg.N
        self.L = sysm.cfg.L
        self.h = sysm.cfg.h
        self.Su, self.Hu, self.Kc = sysm.S_u, sysm.H_u, sysm.K_c
        self.So, self.Ho, self.Kv = sysm.S_o, sysm.H_o, sysm.K_v
        self.mask = np.kron(sysm.M, np.ones((sysm.cfg.n_u, sysm.cfg.n_o)))
        self.xc = xc
        self.hartree = hartree
        self.coupling_scale = coupling_scale
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
        """2 mask_M(K^c V_SCF[P^q] K^v) (times the optional test coupling scale)."""
        Vm = self.vscf(Pq)
        return self.coupling_scale * 2.0 * self.mask * (self.Kc @ Vm @ self.Kv)

    # -- the operator ---------------------------------------------------------------------
    def apply(self, Pp: np.ndarray, Pq: np.ndarray):
        """(f_p, f_q) for stacks [n_states, n_u_fn, n_o_fn]."""
        Pp = np.asarray(Pp, dtype=np.float64)
        Pq = np.asarray(Pq, dtype=np.float64)
        fp = np.stack([self.T(x) for x in Pp])
        fq = np.stack([self.T(x) for x in Pq])
        if self.xc or self.hartree:
            fq = fq + self.coupling(Pq)
        return fp, fq

    # -- metric and projection -------------------------------------------------------------
    def metric(self, X: np.ndarray, Y: np.ndarray) -> float:
        """<X, Y> = Tr[X^T S^u Y S^o] (contravariant X, Y; Sec. II.C)."""
        return float(np.sum(X * (self.Su @ Y @ self.So)))

    def project(self, X: np.ndarray) -> np.ndarray:
        """Pi(X) = mask_M(K^c S^u X S^o K^v): the invariance projection applied to auxiliary
        matrices (Sec. III.A, Eqs. invariance and auxiliary)."""
        return self.mask * (self.KcSu @ X @ self.SoKv)
