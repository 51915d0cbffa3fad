"""Pins for the oracle PCG eigensolver: brute force, closed forms and invariants."""
import numpy as np
import pytest

from oracle.apply import Operator
from oracle.casida import Casida
from oracle.pcg import Options, Solver


@pytest.fixture(scope="module")
def dense(small_dense):
    return small_dense, Operator(small_dense), Casida(small_dense)


@pytest.mark.parametrize("precond", ["cg", "none"])
def test_pcg_matches_brute_force(dense, precond):
    s, op, cs = dense
    n = s.cfg.n_states
    r = Solver(op, Options(n_states=n, precond=precond, tol_omega=1e-10, max_iter=300)).solve(
        s.guess())
    assert r.converged
    assert np.max(np.abs(r.omega - cs.omega_hermitian()[:n])) < 1e-9


def test_pcg_closed_form_without_coupling(small_dense):
    s = small_dense
    op = Operator(s, xc=False, hartree=False)
    cs = Casida(s, xc=False, hartree=False)
    r = Solver(op, Options(n_states=3, tol_omega=1e-11)).solve(s.guess())
    assert np.max(np.abs(r.omega - np.sort(cs.D)[:3])) < 1e-9


def test_pcg_strong_coupling_differs_from_tda(small_dense):
    s = small_dense
    op = Operator(s, coupling_scale=25.0)
    cs = Casida(s, coupling_scale=25.0)
    n = 3
    r = Solver(op, Options(n_states=n, tol_omega=1e-10, max_iter=300)).solve(s.guess())
    wf = cs.omega_hermitian()[:n]
    assert np.max(np.abs(r.omega - wf)) < 1e-9
    assert np.max(np.abs(cs.omega_tda()[:n] - wf)) > 1e-3     # the test is not vacuous


def test_final_vectors_orthonormal_and_eigen(dense):
    s, op, cs = dense
    sol = Solver(op, Options(n_states=3, tol_omega=1e-11))
    r = sol.solve(s.guess())
    C = sol.pq_gram(r.P)
    assert np.max(np.abs(0.5 * (C + C.T) - np.eye(3))) < 1e-10
    Nm = sol.n_matrix(r.P, r.F)
    assert np.max(np.abs(Nm - np.diag(r.omega))) < 1e-8


def test_gradient_orthogonal_to_all_trial_vectors(dense):
    """sum_s <P^s_k, g^s_i> = 0 for all i, k (Sec. III.C)."""
    s, op, cs = dense
    sol = Solver(op, Options(n_states=3))
    p = sol.project(s.guess())
    P = np.stack([p, 0.7 * p + 0.1 * np.roll(p, 1, axis=0)])
    Tp, Tq = sol.orthonormalise(sol.pq_gram(P))
    P = sol.transform(P, Tp, Tq)
    F = sol.apply(P)
    Nm = sol.n_matrix(P, F)
    g = F - np.stack([np.einsum("ij,jkl->ikl", Nm, P[1]), np.einsum("ij,jkl->ikl", Nm, P[0])])
    dots = sol.gram(g[0], sol.cov(P[0])) + sol.gram(g[1], sol.cov(P[1]))
    assert np.max(np.abs(dots)) < 1e-12 * np.max(np.abs(F))


def test_sign_rule_and_gram_schmidt():
    """A forced negative <p_i, q_i> is flipped, then Eq. ortho holds."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 4))
    C = A @ A.T + 4 * np.eye(4)
    C[2, :] *= -1.0                       # q_2 enters with the wrong sign
    C = C.T.copy()                        # C_ij = <p_i, q_j>: flip column 2 (q_2)
    assert C[2, 2] < 0
    Tp, Tq = Solver.orthonormalise(C)
    Cp = Tp @ C @ Tq.T
    assert np.max(np.abs(0.5 * (Cp + Cp.T) - np.eye(4))) < 1e-12
    assert Tq[2, 2] < 0 < Tp[2, 2]


def test_preconditioner_tight_is_inverse_ks_difference(dense):
    """Solving Eq. precond tightly gives G = sum a_c g_cv / (eps_c - eps_v) b_v^T."""
    s, op, cs = dense
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, len(cs.eps_c), len(cs.eps_v)))
    g = cs.to_ngwf(x)
    ref = cs.to_ngwf(x / cs.D.reshape(x.shape[1:]))
    sol = Solver(op, Options(n_states=2, eps_tol=1e-13, max_inner=200))
    G, it = sol.precondition_p(g)
    assert np.max(np.abs(G - ref)) < 1e-9 * np.max(np.abs(ref))
    assert it > 1
    # the same operator expressed on the auxiliary matrices: Pi(z) solves Eq. precond
    sol = Solver(op, Options(n_states=2, eps_tol=1e-14, max_inner=2000))
    z, it = sol.precondition(sol.grad_L(g))
    assert np.max(np.abs(sol.project(z) - ref)) < 1e-7 * np.max(np.abs(ref))


def test_line_search_minimises_trace_functional(dense):
    s, op, cs = dense
    sol = Solver(op, Options(n_states=2))
    rng = np.random.default_rng(6)
    Nc = [np.diag([0.2, 0.3]), 0.01 * rng.standard_normal((2, 2)), np.diag([0.5, 0.4])]
    Nc = [0.5 * (m + m.T) for m in Nc]
    Bc = [np.eye(2), np.zeros((2, 2)), np.eye(2)]
    Nc[1] = Nc[1] - 0.3 * np.eye(2)
    lam = sol.line_search(Nc, Bc, 1.0)
    grid = np.linspace(0, 3, 30001)
    vals = [sol.phi(x, Nc, Bc) for x in grid]
    assert abs(sol.phi(lam, Nc, Bc) - min(vals)) < 1e-9


def _aux_range(s, cs):
    """Matrix of the map L (entries on M) -> KS-basis coefficients of K^c S^u L S^o K^v:
    x = a^T S^u L S^o b for the kernel states a (u-set) and b (o-set)."""
    Mf = np.kron(s.M, np.ones((s.cfg.n_u, s.cfg.n_o))).astype(bool)
    ii, jj = np.nonzero(Mf)
    left = cs.a.T @ s.S_u
    right = s.S_o @ cs.b
    return (left[:, ii][:, None, :] * right[jj, :].T[None, :, :]).reshape(-1, len(ii))


def test_truncated_auxiliary_of_full_rank_reaches_brute_force(small_odd):
    """M truncated (the L-space branch of the solver), but the truncated auxiliary matrices
    still reach every KS pair, so the minimum is the Casida spectrum itself."""
    s = small_odd
    op = Operator(s)
    cs = Casida(s)
    assert not np.all(op.mask_L == 1)
    sv = np.linalg.svd(_aux_range(s, cs), compute_uv=False)
    assert sv[-1] > 1e-3 * sv[0] and len(sv) == len(cs.D)
    n = s.cfg.n_states
    solver = Solver(op, Options(n_states=n, tol_omega=1e-10, max_iter=300))
    assert not solver.complete
    r = solver.solve(s.guess())
    assert r.converged
    assert np.max(np.abs(r.omega - cs.omega_hermitian()[:n])) < 1e-8


def test_truncated_iterates_are_variational(small_trunc):
    """With a rank-deficient auxiliary space every iterate's Tsiper sum lies above the
    minimum over that subspace (brute force: the Casida pencil restricted to the range of
    L -> K^c S^u L S^o K^v), which lies above the untruncated minimum; the line search
    lowers the sum at every step."""
    s = small_trunc
    op = Operator(s)
    cs = Casida(s)
    n = s.cfg.n_states
    U, sv, _ = np.linalg.svd(_aux_range(s, cs), full_matrices=False)
    U = U[:, sv > 0]
    assert U.shape[1] < len(cs.D)
    am = U.T @ (cs.A - cs.B) @ U
    ap = U.T @ (cs.A + cs.B) @ U
    w_sub = np.sort(np.sqrt(np.linalg.eigvals(am @ ap).real))[:n]
    w_all = cs.omega_hermitian()[:n]
    assert np.sum(w_sub) > np.sum(w_all)
    r = Solver(op, Options(n_states=n, max_iter=8)).solve(s.guess())
    sums = np.array([np.sum(h) for h in r.history])
    assert np.all(sums >= np.sum(w_sub) - 1e-10)
    assert np.all(np.diff(sums) <= 1e-12 * np.abs(sums[:-1]))


def test_adaptive_inner_tolerance_reaches_brute_force(dense):
    """A loose inner tolerance early on, tightened with the gradient, changes the path but
    not the minimum."""
    s, op, cs = dense
    n = s.cfg.n_states
    r = Solver(op, Options(n_states=n, eps_loose=0.1, tol_omega=1e-10, max_iter=300)).solve(s.guess())
    assert r.converged
    assert np.max(np.abs(r.omega - cs.omega_hermitian()[:n])) < 1e-9


def test_tamm_dancoff_mode_reaches_tda_brute_force(dense):
    """B = 0: the Tsiper functional of p = q is the Rayleigh quotient of A, so the solver
    returns the lowest eigenvalues of A (dense TDA diagonalisation), which lie above the
    full-TDDFT ones."""
    s, _, cs = dense
    n = s.cfg.n_states
    op = Operator(s, tda=True)
    r = Solver(op, Options(n_states=n, tol_omega=1e-10, max_iter=300)).solve(s.guess())
    assert r.converged
    ref = cs.omega_tda()[:n]
    assert np.max(np.abs(r.omega - ref)) < 1e-9
    assert np.all(ref >= cs.omega_hermitian()[:n] - 1e-12)


def test_response_pattern_keeps_blocks_of_atoms_without_weight():
    """Well-separated atoms: the occupied states sit on two of four atoms, so K^v has
    vanishing diagonal blocks.  The response pattern still holds every atom's own block
    (density matrices are truncated by radius, Sec. IV.C), and on P = Pi(L) the blocks that
    only this reading adds are exactly zero, as is the operator there: the reading changes
    nothing for the P the method produces, only which blocks an arbitrary P may occupy."""
    from conftest import cached_system
    from oracle.apply import response_pattern
    s = cached_system("separated")
    nA = s.cfg.n_atoms
    no, nu = s.occ.n_per_atom, s.vir.n_per_atom
    kv = np.abs(s.K_v.reshape(nA, no, nA, no)).max(axis=(1, 3))
    kc = np.abs(s.K_c.reshape(nA, nu, nA, nu)).max(axis=(1, 3))
    assert (np.diag(kv) == 0).any() and (np.diag(kc) == 0).any()
    assert (kv[~np.eye(nA, dtype=bool)] == 0).all()
    R = response_pattern(s)
    assert R.all()
    # blocks the numerical pattern of the factors would drop
    num = np.outer(np.diag(kc) > 0, np.diag(kv) > 0)
    extra = np.kron(R & ~num, np.ones((nu, no), dtype=bool))
    assert extra.any()
    op = Operator(s, xc=True, hartree=True)
    rng = np.random.default_rng(4)
    L = op.truncate(rng.standard_normal((nA * nu, nA * no)))
    P = op.project(L)
    assert np.abs(P).max() > 0 and (P[extra] == 0).all()
    fp, fq = op.apply(P[None], P[None])
    assert (fp[0][extra] == 0).all() and (fq[0][extra] == 0).all()


def test_learned_scaling_without_progress_is_switched_off(dense):
    """A learned scaling that is a descent direction but a poor preconditioner (random
    factors over six decades) is dropped once the largest gradient norm has not halved in
    ten learned iterations; the solve then finishes with the CG preconditioner and reaches
    brute force.  A constant scaling (steepest descent) keeps halving and stays on."""
    s, op, cs = dense
    n = s.cfg.n_states
    ref = cs.omega_hermitian()[:n]
    rng = np.random.default_rng(1)
    bad = np.exp(rng.uniform(np.log(1e-3), np.log(1e3), (s.vir.n_fn, s.occ.n_fn)))
    r = Solver(op, Options(n_states=n, precond="learned", scaling=bad, tol_omega=1e-10,
                           max_iter=300)).solve(s.guess())
    assert r.converged and r.fallbacks == 1
    assert np.max(np.abs(r.omega - ref)) < 1e-9
    const = np.full((s.vir.n_fn, s.occ.n_fn), 20.0)
    r = Solver(op, Options(n_states=n, precond="learned", scaling=const, tol_omega=1e-10,
                           max_iter=300)).solve(s.guess())
    assert r.converged and r.fallbacks == 0
    assert np.max(np.abs(r.omega - ref)) < 1e-9
