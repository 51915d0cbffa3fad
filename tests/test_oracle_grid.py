"""Pins for the oracle's grid pieces: closed forms, sum rules, brute force on the full grid."""
import numpy as np
import pytest

from oracle import grid
from synth import build_system, configs


def _global_density(sysm, P):
    N = sysm.cfg.N
    U = grid.to_global(N, sysm.vir).reshape(sysm.vir.n_fn, -1)
    O = grid.to_global(N, sysm.occ).reshape(sysm.occ.n_fn, -1)
    return np.einsum("ar,sab,br->sr", U, P, O).reshape(P.shape[0], N, N, N)


@pytest.mark.parametrize("name", ["small_dense", "small_odd"])
def test_density_matches_full_grid_sum(name, request):
    s = request.getfixturevalue(name)
    rng = np.random.default_rng(1)
    P = rng.standard_normal((2, s.vir.n_fn, s.occ.n_fn)) * s.fn_mask()[None]
    rho = grid.density(s.cfg.N, s.vir, s.occ, P)
    ref = _global_density(s, P)
    assert np.max(np.abs(rho - ref)) < 1e-12 * np.max(np.abs(ref))


def test_density_sum_rule(small_odd):
    """h^3 sum_r rho(r) = sum_ab P_ab S^uo_ab (S^uo built by the generator's own code)."""
    s = small_odd
    rng = np.random.default_rng(2)
    P = rng.standard_normal((3, s.vir.n_fn, s.occ.n_fn))
    rho = grid.density(s.cfg.N, s.vir, s.occ, P)
    lhs = s.cfg.h ** 3 * rho.reshape(3, -1).sum(1)
    rhs = np.einsum("sab,ab->s", P, s.S_uo)
    assert np.allclose(lhs, rhs, rtol=1e-11, atol=1e-12)


def test_potential_integrals_unit_potential_is_overlap(small_odd):
    s = small_odd
    N = s.cfg.N
    V = np.ones((1, N, N, N))
    Vm = grid.potential_integrals(N, s.cfg.h, s.vir, s.occ, V)[0]
    assert np.max(np.abs(Vm - s.S_uo)) < 1e-12


def test_potential_integrals_match_full_grid(small_dense):
    s = small_dense
    N = s.cfg.N
    rng = np.random.default_rng(3)
    V = rng.standard_normal((2, N, N, N))
    Vm = grid.potential_integrals(N, s.cfg.h, s.vir, s.occ, V)
    U = grid.to_global(N, s.vir).reshape(s.vir.n_fn, -1)
    O = grid.to_global(N, s.occ).reshape(s.occ.n_fn, -1)
    ref = s.cfg.h ** 3 * np.einsum("ar,sr,br->sab", U, V.reshape(2, -1), O)
    assert np.max(np.abs(Vm - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("N,L", [(16, 10.0), (20, 7.5), (45, 15.0)])
def test_poisson_plane_wave(N, L):
    """cos(G.r) maps to (4 pi / |G|^2) cos(G.r); a constant maps to zero."""
    h = L / N
    z, y, x = np.meshgrid(*(np.arange(N) * h,) * 3, indexing="ij")
    for (kx, ky, kz) in [(1, 0, 0), (2, -3, 1), (0, 0, N // 2 - 1)]:
        G = 2 * np.pi / L * np.array([kx, ky, kz])
        f = np.cos(G[0] * x + G[1] * y + G[2] * z)
        V = grid.poisson_periodic(f[None], L)[0]
        assert np.max(np.abs(V - 4 * np.pi / (G @ G) * f)) < 1e-10
    assert np.max(np.abs(grid.poisson_periodic(np.ones((1, N, N, N)), L))) < 1e-12


def test_poisson_matches_explicit_dft():
    """Explicit O(N^6) Fourier sum on a 6^3 grid (no FFT library involved)."""
    N, L = 6, 5.0
    rng = np.random.default_rng(4)
    rho = rng.standard_normal((N, N, N))
    idx = np.arange(N)
    kk = np.where(idx < (N + 1) // 2, idx, idx - N)        # wrapped wave numbers
    r = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), -1).reshape(-1, 3)
    k = np.stack(np.meshgrid(kk, kk, kk, indexing="ij"), -1).reshape(-1, 3)
    phase = np.exp(-2j * np.pi * (r @ k.T) / N)          # [r, k]
    rhok = rho.reshape(-1) @ phase
    G2 = (2 * np.pi / L) ** 2 * np.sum(k * k, 1)
    kern = np.where(G2 > 0, 4 * np.pi / np.where(G2 > 0, G2, 1), 0.0)
    V = (phase.conj() @ (kern * rhok)).real / N ** 3
    assert np.max(np.abs(V.reshape(N, N, N) - grid.poisson_periodic(rho[None], L)[0])) < 1e-12


def test_fxc_closed_form_and_finite_difference():
    rho = np.array([1e-6, 1e-3, 0.05, 0.3, 2.0])
    f = grid.fxc_alda(rho)
    cx = (3 / np.pi) ** (1 / 3)
    assert np.allclose(f, -(1 / 3) * cx * rho ** (-2 / 3), rtol=1e-14)
    hstep = 1e-4 * rho
    fd = (grid.ex_lda(rho + hstep) - 2 * grid.ex_lda(rho) + grid.ex_lda(rho - hstep)) / hstep ** 2
    assert np.allclose(f, fd, rtol=1e-5)
    assert np.all(grid.fxc_alda(np.array([0.0, 1e-12, 9.9e-11])) == 0.0)


def test_box_index_wraps():
    g = grid.box_global_index((3, 0, 5), (2, 1, 3), 6)
    # points (z, y, x) = (3..4, 0, 5, 0, 1)
    exp = [(z * 6 + 0) * 6 + x for z in (3, 4) for x in (5, 0, 1)]
    assert list(g) == exp


def test_generator_self_overlap_consistent():
    """The generator's S (box intersections) equals the full-grid overlap."""
    s = build_system(configs.small_odd())
    N = s.cfg.N
    U = grid.to_global(N, s.vir).reshape(s.vir.n_fn, -1)
    O = grid.to_global(N, s.occ).reshape(s.occ.n_fn, -1)
    h3 = s.cfg.h ** 3
    assert np.max(np.abs(h3 * U @ U.T - s.S_u)) < 1e-12
    assert np.max(np.abs(h3 * O @ O.T - s.S_o)) < 1e-12
    assert np.max(np.abs(h3 * U @ O.T - s.S_uo)) < 1e-12
