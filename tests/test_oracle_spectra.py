"""Pins for the oscillator strengths of oracle/spectra.py (velocity form)."""
import numpy as np
import pytest

from oracle import grid
from oracle.apply import Operator
from oracle.casida import Casida
from oracle.pcg import Options, Solver
from oracle.spectra import (casida_oscillator_strengths, central_derivative,
                            gradient_integrals, oscillator_strengths)


def test_central_derivative_of_a_plane_wave():
    """On a periodic grid the central difference of sin(k x) is sin(k h)/h cos(k x)."""
    N, L = 16, 8.0
    h = L / N
    x = np.arange(N) * h
    k = 2 * np.pi * 3 / L
    f = np.broadcast_to(np.sin(k * x), (N, N, N))
    d = central_derivative(f, h, axis=2)
    assert np.allclose(d, np.sin(k * h) / h * np.cos(k * x)[None, None, :], atol=1e-13)
    assert np.allclose(central_derivative(f, h, axis=0), 0.0)


def test_gradient_integrals_antisymmetric(small_dense):
    """Summation by parts on the periodic grid: <u|d o> = -<d u|o> exactly, and
    <f|d f> = 0 for every function."""
    s = small_dense
    G_uo = gradient_integrals(s.cfg.N, s.cfg.h, s.vir, s.occ)
    G_ou = gradient_integrals(s.cfg.N, s.cfg.h, s.occ, s.vir)
    assert np.max(np.abs(G_uo + np.transpose(G_ou, (0, 2, 1)))) < 1e-12 * np.max(np.abs(G_uo))
    G_oo = gradient_integrals(s.cfg.N, s.cfg.h, s.occ, s.occ)
    assert np.max(np.abs(np.diagonal(G_oo, axis1=1, axis2=2))) < 1e-12
    assert np.max(np.abs(G_uo)) > 1e-3


def test_no_coupling_closed_form(small_dense):
    """Without coupling X = e_cv, Y = 0: f = 2 / (3 (e_c - e_v)) |<psi_c|d|psi_v>|^2."""
    s = small_dense
    cs = Casida(s, xc=False, hartree=False)
    G = gradient_integrals(s.cfg.N, s.cfg.h, s.vir, s.occ)
    w, f, _ = casida_oscillator_strengths(cs, G, 3)
    grad_cv = np.einsum("ac,kab,bv->kcv", cs.a, G, cs.b)
    order = np.argsort(cs.D)[:3]
    nv = len(cs.eps_v)
    ref = [2.0 / (3.0 * cs.D[i]) * np.sum(grad_cv[:, i // nv, i % nv] ** 2) for i in order]
    assert np.allclose(w, cs.D[order], rtol=1e-12)
    assert np.allclose(f, ref, rtol=1e-10)


@pytest.mark.parametrize("coupling", [1.0, 25.0])
def test_method_vectors_give_casida_strengths(small_dense, coupling):
    """The converged response kernels of the PCG solve (mixed function space) give the
    oscillator strengths of the brute-force Casida eigenvectors; strong coupling makes
    Y large, so the (X - Y) in the velocity form is exercised."""
    s = small_dense
    n = s.cfg.n_states
    op = Operator(s, coupling_scale=coupling)
    cs = Casida(s, coupling_scale=coupling)
    r = Solver(op, Options(n_states=n, tol_omega=1e-11, max_iter=400)).solve(s.guess())
    G = gradient_integrals(s.cfg.N, s.cfg.h, s.vir, s.occ)
    f, D = oscillator_strengths(r.omega, r.P[0], G)
    w_ref, f_ref, _ = casida_oscillator_strengths(cs, G, n)
    assert np.max(np.abs(r.omega - w_ref)) < 1e-9
    # eigenvectors converge as the square root of the energies (omega to ~1e-11 Ha)
    assert np.max(np.abs(f - f_ref)) < 1e-4 * np.max(f_ref)
    assert np.max(f_ref) > 0
    if coupling > 1.0:
        # the velocity form takes p = X - Y; with this coupling q = X + Y differs enough
        # that using it instead fails the comparison (the pin tells the two apart)
        fq, _ = oscillator_strengths(r.omega, r.P[1], G)
        assert np.max(np.abs(fq - f_ref)) > 1e-2 * np.max(f_ref)
