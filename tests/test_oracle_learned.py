"""Pins for the learned-preconditioner oracle: features against the generator's own
geometry and spectral bounds, targets against closed forms, BF16 rounding against torch,
and solver correctness that does not depend on the scaling."""
import numpy as np
import pytest
import scipy.linalg

from oracle import learned
from oracle.apply import Operator, response_pattern
from oracle.casida import Casida
from oracle.pcg import Options, Solver


def test_feature_layout_and_closed_forms(small_odd):
    s = small_odd
    R = response_pattern(s)
    F = learned.block_features(s, R)
    bu, bo = s.cfg.n_u, s.cfg.n_o
    assert F.shape == (int(R.sum()), learned.n_features(bu, bo)) and F.shape[1] == 30
    # normalised functions: unit diagonals of both overlaps
    assert np.allclose(F[:, [0, 3, 5]], 1.0) and np.allclose(F[:, [12, 14]], 1.0)
    # eigenvalue differences are the differences of the listed eigenvalues
    eu, eo = F[:, 18:21], F[:, 21:23]
    assert np.allclose(F[:, 23:29], (eu[:, :, None] - eo[:, None, :]).reshape(-1, 6))


def test_local_eigenvalues_lie_inside_the_global_spectrum(small_odd):
    """Rayleigh quotients: the eigenvalues of a principal sub-pencil lie within the extreme
    eigenvalues of the whole pencil (H, S)."""
    s = small_odd
    F = learned.block_features(s, response_pattern(s))
    wu = scipy.linalg.eigh(s.H_u, s.S_u, eigvals_only=True)
    wo = scipy.linalg.eigh(s.H_o, s.S_o, eigvals_only=True)
    assert np.all(F[:, 18:21] >= wu[0] - 1e-10) and np.all(F[:, 18:21] <= wu[-1] + 1e-10)
    assert np.all(F[:, 21:23] >= wo[0] - 1e-10) and np.all(F[:, 21:23] <= wo[-1] + 1e-10)


def test_distance_feature_matches_atom_positions(small_odd):
    """Box centres sit within one grid step per axis of the atoms they belong to."""
    s = small_odd
    R = response_pattern(s)
    F = learned.block_features(s, R)
    I, J = np.nonzero(R)
    d = s.pos[I] - s.pos[J]
    d -= s.cfg.L * np.round(d / s.cfg.L)
    dist = np.sqrt(np.sum(d * d, axis=1))
    assert np.max(np.abs(F[:, 29] - dist)) <= 2.0 * np.sqrt(3.0) * s.cfg.h


def test_guess_target_closed_form(small_dense):
    s = small_dense
    R = response_pattern(s)
    rng = np.random.default_rng(3)
    P = rng.standard_normal((2, s.vir.n_fn, s.occ.n_fn))
    t = learned.guess_target(s, P, R)
    assert abs(np.sum(10.0 ** t - 1e-8) - 1.0) < 1e-12
    # all weight in one block: that block gets log10(1 + 1e-8), the others -8
    Q = np.zeros_like(P)
    Q[0, :s.cfg.n_u, :s.cfg.n_o] = 1.0
    t1 = learned.guess_target(s, Q, R)
    assert abs(t1[0] - np.log10(1 + 1e-8)) < 1e-15 and np.allclose(t1[1:], -8.0)


def test_block_view_round_trip(small_odd):
    s = small_odd
    R = response_pattern(s)
    rng = np.random.default_rng(4)
    v = rng.standard_normal((int(R.sum()), s.cfg.n_u * s.cfg.n_o))
    X = learned.expand_blocks(s, v, R)
    assert np.array_equal(learned.block_view(s, X[None], R)[0], v)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-8, 8, 1000),
                        [1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(learned.bf16_round(x), ref)


@pytest.mark.parametrize("kind", ["constant", "negative"])
def test_learned_solver_reaches_brute_force_whatever_the_scaling(small_dense, kind):
    """A positive scaling is a valid preconditioner; a negative one is never a descent
    direction and every iteration falls back to the CG preconditioner.  Both reach the
    Casida spectrum."""
    s = small_dense
    op = Operator(s)
    n = s.cfg.n_states
    c = np.full((s.vir.n_fn, s.occ.n_fn), 5.0 if kind == "constant" else -5.0)
    res = Solver(op, Options(n_states=n, precond="learned", scaling=c, tol_omega=1e-10,
                             max_iter=300)).solve(s.guess())
    assert res.converged
    assert np.max(np.abs(res.omega - Casida(s).omega_hermitian()[:n])) < 1e-9
    if kind == "negative":
        assert res.fallbacks == res.iterations
    else:
        assert res.fallbacks == 0
