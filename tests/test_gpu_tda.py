"""Tamm-Dancoff mode (B = 0, A = D + K on both halves): apply parity against the FP64
oracle and solves against the dense TDA diagonalisation."""
import numpy as np
import pytest

from helpers import gpu_handle, random_p, rel_err, to_dev
from oracle.apply import Operator
from oracle.casida import Casida
from synth import abi as sabi

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,precision,tol", [("small_odd", "fp64", 1e-11),
                                                ("small_trunc", "fp64", 1e-11),
                                                ("small_trunc", "fp32", 2e-5)])
def test_tda_apply(name, precision, tol, request):
    s = request.getfixturevalue(name)
    op = Operator(s, tda=True)
    Pp = random_p(s, 3, 51)
    Pq = random_p(s, 3, 52)
    fp_ref, fq_ref = op.apply(Pp, Pq)
    h = gpu_handle(s, precision=precision, tda=1)
    fp, fq = h.tddft_apply(to_dev(sabi.dense_to_p(s, Pp)), to_dev(sabi.dense_to_p(s, Pq)))
    h.close()
    assert rel_err(sabi.p_to_dense(s, fp.cpu().numpy()), fp_ref) < tol
    assert rel_err(sabi.p_to_dense(s, fq.cpu().numpy()), fq_ref) < tol


@pytest.mark.parametrize("name", ["small_dense", "tiny"])
def test_tda_solve_matches_dense_tda(name, request):
    from conftest import cached_system
    from paper_1507_08157_amd import binding
    s = cached_system(name)
    n = s.cfg.n_states
    h = gpu_handle(s, precision="fp64", tda=1)
    L0 = to_dev(sabi.dense_to_p(s, s.guess(n)))
    Pp, Pq = L0.clone() * 3.0, L0.clone()     # the TDA solve starts from Pq in both halves
    o = binding.tddft_default_options(tda=1, tol_omega=1e-10, max_iter=300)
    w, rc, st = h.tddft_pcg_solve(n, o, Pp, Pq)
    h.close()
    cs = Casida(s)
    assert rc == 0 and st["converged"]
    assert np.max(np.abs(w - cs.omega_tda()[:n])) < 1e-9
    assert np.all(w >= cs.omega_hermitian()[:n] - 1e-9)
    assert np.array_equal(Pp.cpu().numpy(), Pq.cpu().numpy())


def test_tda_must_match_handle(small_dense):
    from paper_1507_08157_amd import binding
    h = gpu_handle(small_dense, precision="fp64")
    with pytest.raises(binding.TddftError) as e:
        h.tddft_pcg_solve(2, binding.tddft_default_options(tda=1))
    h.close()
    assert e.value.code == binding.TDDFT_E_INVALID
