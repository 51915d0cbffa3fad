"""Oscillator strengths of converged excitations, velocity (momentum) form, FP64.

The paper lists oscillator strengths beside the excitation energies (Sec. IV.A, Table
tab:azo) and broadens them into absorption spectra (Sec. IV.B) without printing the
formula.  In a periodic cell the position operator has no matrix elements between the
delocalised functions, so the velocity form is used: for an excitation n of energy
omega_n with p_n = X_n - Y_n normalised by X^T X - Y^T Y = 1 (the Tsiper normalisation
<p_n, q_n> = 1 of Sec. III.C), the transition moment of the gradient operator is
sum_cv <psi_c| d_alpha |psi_v> p_n,cv and

    f_n = 2 / (3 omega_n) * sum_alpha ( sum_cv <psi_c| d_alpha |psi_v> p_n,cv )^2 .

With the response kernel P^p = sum_cv a_c p_cv b_v^T in the mixed function space (Sec.
III.A) the sum is sum_ab P^p_ab G^alpha_ab with G^alpha_ab = <u_a| d_alpha |o_b>.  The
derivative is the second-order central difference on the periodic grid, the discrete
counterpart of the generator's second-order Laplacian: on the grid it is exactly
antisymmetric (summation by parts), as d_alpha is.
"""
from __future__ import annotations

import numpy as np

from . import grid


def central_derivative(f: np.ndarray, h: float, axis: int) -> np.ndarray:
    """(f(r + h e_axis) - f(r - h e_axis)) / 2h on a periodic grid (arrays [..., z, y, x])."""
    return (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis)) / (2.0 * h)


def gradient_integrals(N: int, h: float, left, right) -> np.ndarray:
    """G[alpha, a, b] = h^3 sum_r f^left_a(r) (d_alpha f^right_b)(r), alpha = x, y, z, from
    every function on the full grid (small systems)."""
    fl = grid.to_global(N, left).reshape(left.n_fn, -1)
    fr = grid.to_global(N, right)
    G = np.zeros((3, left.n_fn, right.n_fn))
    for alpha, axis in ((0, 3), (1, 2), (2, 1)):          # x is the last array axis
        d = central_derivative(fr, h, axis).reshape(right.n_fn, -1)
        G[alpha] = h ** 3 * fl @ d.T
    return G


def oscillator_strengths(omega: np.ndarray, Pp: np.ndarray, G: np.ndarray):
    """(f [n], moments [n, 3]) for response kernels Pp [n, n_u, n_o] of energies omega."""
    D = np.einsum("nab,kab->nk", Pp, G)
    f = 2.0 / (3.0 * np.asarray(omega)) * np.sum(D * D, axis=1)
    return f, D


def casida_oscillator_strengths(cs, G: np.ndarray, n: int):
    """The same from the brute-force Casida eigenvectors (oracle/casida.py): with A - B = D
    diagonal, the Hermitian form D^1/2 (A+B) D^1/2 Z = omega^2 Z (Z^T Z = 1) gives
    X - Y = omega^1/2 D^-1/2 Z.  Returns (omega, f, moments) of the n lowest."""
    d = np.sqrt(cs.D)
    Mh = d[:, None] * (cs.A + cs.B) * d[None, :]
    w2, Z = np.linalg.eigh(0.5 * (Mh + Mh.T))
    omega = np.sqrt(w2[:n])
    nc, nv = len(cs.eps_c), len(cs.eps_v)
    p = (np.sqrt(omega)[None, :] * Z[:, :n] / d[:, None]).T.reshape(n, nc, nv)
    grad_cv = np.einsum("ac,kab,bv->kcv", cs.a, G, cs.b)
    D = np.einsum("ncv,kcv->nk", p, grad_cv)
    return omega, 2.0 / (3.0 * omega) * np.sum(D * D, axis=1), D
