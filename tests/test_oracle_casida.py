"""Pins for the brute-force Casida oracle and the NGWF-space operator oracle."""
import numpy as np
import pytest

from oracle.apply import Operator
from oracle.casida import Casida, kernel_states


@pytest.fixture(scope="module")
def pair(small_dense):
    return Operator(small_dense), Casida(small_dense)


def test_two_casida_forms_agree(pair):
    _, cs = pair
    w1 = cs.omega_nonhermitian()
    w2 = cs.omega_hermitian()
    assert len(w1) == len(cs.D)
    assert np.max(np.abs(w1 - w2)) < 1e-10


def test_no_coupling_gives_ks_differences(small_dense):
    cs = Casida(small_dense, xc=False, hartree=False)
    assert np.max(np.abs(cs.omega_hermitian() - np.sort(cs.D))) < 1e-13


def test_full_below_tda(pair):
    """Thouless functional with Y = 0 is the TDA functional, so sums of the lowest k
    full-TDDFT energies never exceed the TDA ones (Sec. II.B)."""
    _, cs = pair
    wf = cs.omega_hermitian()
    wt = cs.omega_tda()
    for k in range(1, 6):
        assert np.sum(wf[:k]) <= np.sum(wt[:k]) + 1e-12


def test_kernel_states_are_projector_eigenstates(small_dense):
    s = small_dense
    eps, b = kernel_states(s.H_o, s.S_o, s.K_v)
    assert len(eps) == s.cfg.n_occ
    assert np.allclose(b.T @ s.S_o @ b, np.eye(len(eps)), atol=1e-12)
    assert np.allclose(b @ b.T, s.K_v, atol=1e-12)


@pytest.mark.parametrize("scale", [1.0, 25.0])
def test_ngwf_operator_is_casida_in_ks_basis(small_dense, scale):
    """For P = sum a_c x_cv b_v^T: <P', f_p(P)>_S = x'^T (A-B) x and
    <P', f_q(P)>_S = x'^T (A+B) x (Sec. III.A, Eq. operator_RPA)."""
    op = Operator(small_dense, coupling_scale=scale)
    cs = Casida(small_dense, coupling_scale=scale)
    rng = np.random.default_rng(7)
    nc, nv = len(cs.eps_c), len(cs.eps_v)
    x = rng.standard_normal((2, nc, nv))
    P = cs.to_ngwf(x)
    fp, fq = op.apply(P, P)
    AmB = cs.A - cs.B
    ApB = cs.A + cs.B
    for i in range(2):
        for j in range(2):
            assert abs(op.metric(P[j], fp[i]) - x[j].ravel() @ AmB @ x[i].ravel()) < 1e-11
            assert abs(op.metric(P[j], fq[i]) - x[j].ravel() @ ApB @ x[i].ravel()) < 1e-11


def test_kohn_sham_part_is_diagonal(pair):
    """T(P) has KS-basis components (eps_c - eps_v) x_cv (closed form)."""
    op, cs = pair
    rng = np.random.default_rng(8)
    x = rng.standard_normal((len(cs.eps_c), len(cs.eps_v)))
    P = cs.to_ngwf(x)
    t = op.T(P)
    s = op.sys
    comp = cs.a.T @ s.S_u @ t @ s.S_o @ cs.b
    assert np.max(np.abs(comp - cs.D.reshape(x.shape) * x)) < 1e-12


def test_projection_is_idempotent_and_keeps_invariant(pair):
    """Pi(Pi(L)) = Pi(L) and Pi(P) = P for P = K^c S L S K^v with exact kernels
    (Sec. III.A, Eq. invariance)."""
    op, cs = pair
    rng = np.random.default_rng(9)
    Lx = rng.standard_normal(op.mask.shape)
    P = op.project(Lx)
    assert np.max(np.abs(op.project(P) - P)) < 1e-12 * np.max(np.abs(P))
    x = rng.standard_normal((len(cs.eps_c), len(cs.eps_v)))
    Q = cs.to_ngwf(x)
    assert np.max(np.abs(op.project(Q) - Q)) < 1e-12 * np.max(np.abs(Q))


def test_operator_preserves_invariance(pair):
    """f of an invariant P is invariant (Sec. III.A: the gradient obeys Eq. invariance)."""
    op, cs = pair
    rng = np.random.default_rng(10)
    P = cs.to_ngwf(rng.standard_normal((1, len(cs.eps_c), len(cs.eps_v))))
    fp, fq = op.apply(P, P)
    for f in (fp[0], fq[0]):
        assert np.linalg.norm(op.project(f) - f) < 1e-12 * np.linalg.norm(f)


def test_metric_symmetric(pair):
    op, _ = pair
    rng = np.random.default_rng(11)
    X, Y = rng.standard_normal((2,) + op.mask.shape)
    assert abs(op.metric(X, Y) - op.metric(Y, X)) < 1e-12 * abs(op.metric(X, X))
