"""The joint unoccupied representation (Eq. proj): the u-set holds every o- and u-function
of an atom and K^c projects onto the complement of the occupied space within it.  Pinned by
the projector's defining properties, independent of how it was formed."""
import numpy as np
import pytest

from conftest import cached_system


@pytest.fixture(scope="module")
def joint():
    return cached_system("small_joint")


def test_joint_u_set_contains_the_o_set(joint):
    s = joint
    nf = s.vir.n_per_atom
    assert nf == s.occ.n_per_atom + 3
    for I in range(s.cfg.n_atoms):
        assert np.array_equal(s.vir.vals[I][:s.occ.n_per_atom], s.occ.vals[I])
    # so the o-block of the joint overlap is S^o itself
    o_sel = (np.arange(s.cfg.n_atoms)[:, None] * nf + np.arange(s.occ.n_per_atom)[None, :]).ravel()
    assert np.allclose(s.S_u[np.ix_(o_sel, o_sel)], s.S_o, atol=1e-14)


def test_complement_projector(joint):
    s = joint
    K, S = s.K_c, s.S_u
    # idempotent in the S metric, symmetric
    assert np.linalg.norm(K @ S @ K - K) < 1e-10 * np.linalg.norm(K)
    assert np.allclose(K, K.T, atol=1e-12)
    # annihilates the occupied space: K^c S^{uo} K^v = 0
    assert np.max(np.abs(K @ s.S_uo @ s.K_v)) < 1e-10
    # rank = dim(joint space) - number of occupied states
    assert abs(np.trace(K @ S) - (s.vir.n_fn - s.cfg.n_occ)) < 1e-8
    # together with the occupied projector it resolves the identity of the joint space:
    # K^c + E K^v E^T = S^-1 (E embeds the o-set)
    nf = s.vir.n_per_atom
    o_sel = (np.arange(s.cfg.n_atoms)[:, None] * nf + np.arange(s.occ.n_per_atom)[None, :]).ravel()
    full = K.copy()
    full[np.ix_(o_sel, o_sel)] += s.K_v
    assert np.max(np.abs(full @ S - np.eye(S.shape[0]))) < 1e-9


def test_projected_states_reduce_to_eigenstates():
    """For an eigenstate projector (the plain u-set) the projected-state construction gives
    the same levels as the eigenstates K^c is built from."""
    from oracle.casida import projected_states
    s = cached_system("small_dense")
    e, C = projected_states(s.H_u, s.S_u, s.K_c)
    assert np.allclose(e, s.eps_u[s.vir_idx], atol=1e-10)
    assert np.allclose(C.T @ s.S_u @ C, np.eye(len(e)), atol=1e-10)


def test_joint_brute_force_and_solver(joint):
    """Joint representation with a gapped complement: the Casida spectrum from the projected
    states is positive, its two forms agree, and the oracle's PCG reaches it."""
    from oracle.apply import Operator
    from oracle.casida import Casida
    from oracle.pcg import Options, Solver
    s = joint
    assert s.eps_u[0] > s.eps_o[s.cfg.n_occ - 1] + s.cfg.gap_margin
    c = Casida(s)
    assert c.D.min() > 0
    n = s.cfg.n_states
    w = c.omega_hermitian()[:n]
    assert np.allclose(w, c.omega_nonhermitian()[:n], atol=1e-10)
    res = Solver(Operator(s), Options(n_states=n, tol_omega=1e-10, max_iter=300)).solve(s.guess(n))
    assert np.max(np.abs(np.asarray(res.omega) - w)) < 1e-9
