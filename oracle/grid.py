"""Real-space grid pieces of the response operator, FP64, plain NumPy.

Grid: N^3 points of a periodic cube of side L, spacing h = L / N; arrays are indexed
[z, y, x].  Every localised function lives on a box of grid points (origin, extent),
wrapped periodically; a global point belongs to a box iff each of its coordinates does.

  response density     rho(r) = sum_ab u_a(r) P_ab o_b(r)         (Sec. III.A, rho^{p/q})
  Hartree potential    V_H = IFFT[4 pi / |G|^2 FFT rho], G = 0 dropped   (Sec. II.A, the
                       1/|r - r'| part of the coupling kernel; periodic cell)
  ALDA kernel          f_xc(r) = d^2 e_x / d rho^2 at rho0, LDA exchange
                       e_x = -(3/4)(3/pi)^{1/3} rho^{4/3}            (Sec. II.A, xc part)
  potential integrals  V_ab = h^3 sum_r u_a(r) V(r) o_b(r)         (Sec. II.C, V_SCF^{chi phi})
"""
from __future__ import annotations

import numpy as np


def box_global_index(origin, extent, N: int) -> np.ndarray:
    """Flat global indices (z-major, x fastest) of every point of a box, in box order."""
    z = (origin[0] + np.arange(extent[0])) % N
    y = (origin[1] + np.arange(extent[1])) % N
    x = (origin[2] + np.arange(extent[2])) % N
    return ((z[:, None, None] * N + y[None, :, None]) * N + x[None, None, :]).ravel()


class _Lookup:
    """Global point -> position inside one chosen box (or -1)."""

    def __init__(self, N: int):
        self.table = np.full(N ** 3, -1, dtype=np.int64)
        self.current = None

    def set_box(self, gidx: np.ndarray):
        if self.current is not None:
            self.table[self.current] = -1
        self.table[gidx] = np.arange(len(gidx))
        self.current = gidx

    def find(self, gidx: np.ndarray):
        """For points gidx (of another box): (positions in gidx, positions in chosen box)."""
        loc = self.table[gidx]
        sel = np.nonzero(loc >= 0)[0]
        return sel, loc[sel]


def _flat(fs, I):
    v = fs.vals[I]
    return v.reshape(v.shape[0], -1)


def density(N: int, left, right, P: np.ndarray) -> np.ndarray:
    """rho_s(r) = sum_{a in left, b in right} f^left_a(r) P_s[a, b] f^right_b(r).

    left/right: function sets grouped by atom; P: [n_states, n_left_fn, n_right_fn].
    Returns [n_states, N, N, N]."""
    P = np.asarray(P, dtype=np.float64)
    ns = P.shape[0]
    nl, nr = left.n_per_atom, right.n_per_atom
    rho = np.zeros((ns, N ** 3))
    look = _Lookup(N)
    gl = [box_global_index(left.origin[I], left.extent[I], N) for I in range(left.n_atoms)]
    gr = [box_global_index(right.origin[J], right.extent[J], N) for J in range(right.n_atoms)]
    for I in range(left.n_atoms):
        look.set_box(gl[I])
        psi = np.zeros((ns, nl, len(gl[I])))        # psi_a(r) = sum_b P_ab f_b(r) on box I
        for J in range(right.n_atoms):
            blk = P[:, I * nl:(I + 1) * nl, J * nr:(J + 1) * nr]
            if not np.any(blk):
                continue
            selJ, posI = look.find(gr[J])
            if len(selJ) == 0:
                continue
            fJ = _flat(right, J)[:, selJ]
            psi[:, :, posI] += np.einsum("sab,bp->sap", blk, fJ)
        fI = _flat(left, I)
        rho[:, gl[I]] += np.einsum("ap,sap->sp", fI, psi)
    return rho.reshape(ns, N, N, N)


def poisson_periodic(rho: np.ndarray, L: float) -> np.ndarray:
    """Hartree potential of a periodic density: V(G) = 4 pi rho(G) / |G|^2, V(0) = 0."""
    N = rho.shape[-1]
    k = 2.0 * np.pi * np.fft.fftfreq(N, d=L / N)
    G2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    kern = np.zeros_like(G2)
    nz = G2 > 0
    kern[nz] = 4.0 * np.pi / G2[nz]
    rg = np.fft.fftn(rho, axes=(-3, -2, -1))
    return np.real(np.fft.ifftn(rg * kern, axes=(-3, -2, -1)))


CX = (3.0 / np.pi) ** (1.0 / 3.0)


def ex_lda(rho):
    """LDA exchange energy density per volume (unpolarised): -(3/4)(3/pi)^{1/3} rho^{4/3}."""
    return -0.75 * CX * np.asarray(rho) ** (4.0 / 3.0)


def fxc_alda(rho0: np.ndarray, rho_floor: float = 1e-10) -> np.ndarray:
    """Second derivative of the LDA exchange energy density: -(1/3)(3/pi)^{1/3} rho^{-2/3};
    zero where rho0 < rho_floor."""
    rho0 = np.asarray(rho0, dtype=np.float64)
    out = np.zeros_like(rho0)
    ok = rho0 >= rho_floor
    out[ok] = -(1.0 / 3.0) * CX * rho0[ok] ** (-2.0 / 3.0)
    return out


def potential_integrals(N: int, h: float, left, right, V: np.ndarray) -> np.ndarray:
    """V_s[a, b] = h^3 sum_r f^left_a(r) V_s(r) f^right_b(r) for every overlapping pair.

    V: [n_states, N, N, N].  Returns [n_states, n_left_fn, n_right_fn]."""
    V = np.asarray(V, dtype=np.float64).reshape(V.shape[0], -1)
    ns = V.shape[0]
    nl, nr = left.n_per_atom, right.n_per_atom
    out = np.zeros((ns, left.n_fn, right.n_fn))
    look = _Lookup(N)
    gl = [box_global_index(left.origin[I], left.extent[I], N) for I in range(left.n_atoms)]
    gr = [box_global_index(right.origin[J], right.extent[J], N) for J in range(right.n_atoms)]
    h3 = h ** 3
    for I in range(left.n_atoms):
        look.set_box(gl[I])
        W = _flat(left, I)[None, :, :] * V[:, gl[I]][:, None, :]      # [s, a, p]
        for J in range(right.n_atoms):
            selJ, posI = look.find(gr[J])
            if len(selJ) == 0:
                continue
            fJ = _flat(right, J)[:, selJ]
            out[:, I * nl:(I + 1) * nl, J * nr:(J + 1) * nr] = \
                h3 * np.einsum("sap,bp->sab", W[:, :, posI], fJ)
    return out


def to_global(N: int, fs) -> np.ndarray:
    """Every function of a set on the full grid, [n_fn, N, N, N] (small systems only)."""
    out = np.zeros((fs.n_fn, N ** 3))
    for I in range(fs.n_atoms):
        g = box_global_index(fs.origin[I], fs.extent[I], N)
        out[I * fs.n_per_atom:(I + 1) * fs.n_per_atom, g] = _flat(fs, I)
    return out.reshape(fs.n_fn, N, N, N)
