"""GPU parity of the operator application in the joint unoccupied representation (Eq. proj:
5 u-functions per atom, K^c the complement projector) against the FP64 oracle."""
import numpy as np
import pytest

from helpers import gpu_handle, random_p, rel_err, to_dev
from oracle.apply import Operator
from synth import abi as sabi

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 2e-5)])
def test_joint_apply(precision, tol):
    from conftest import cached_system
    s = cached_system("small_joint")
    print(f"[joint] apply {precision}", flush=True)
    op = Operator(s)
    Pp = random_p(s, 3, 31)
    Pq = random_p(s, 3, 131)
    fp_ref, fq_ref = op.apply(Pp, Pq)
    h = gpu_handle(s, precision=precision)
    info = h.tddft_get_info()
    fp, fq = h.tddft_apply(to_dev(sabi.dense_to_p(s, Pp)), to_dev(sabi.dense_to_p(s, Pq)))
    fp = sabi.p_to_dense(s, fp.cpu().numpy())
    fq = sabi.p_to_dense(s, fq.cpu().numpy())
    h.close()
    assert info["block_rows"] == 5 and info["block_cols"] == 2
    assert rel_err(fp, fp_ref) < tol
    if precision == "fp64":
        assert rel_err(fq, fq_ref) < tol
    else:
        assert np.max(np.abs(fq - fq_ref)) < tol * np.max(np.abs(fq_ref))


def test_joint_solve_reaches_brute_force():
    """FP64 PCG in the joint representation converges to the brute-force Casida spectrum
    built from the states of H in the complement of the occupied space."""
    from conftest import cached_system
    from oracle.casida import Casida
    from paper_1507_08157_amd import binding
    s = cached_system("small_joint")
    n = s.cfg.n_states
    print("[joint] solve fp64", flush=True)
    h = gpu_handle(s, precision="fp64")
    w, rc, st = h.tddft_pcg_solve(n, binding.tddft_default_options(tol_omega=1e-10, max_iter=300))
    h.close()
    ref = Casida(s).omega_hermitian()[:n]
    assert st["converged"] and np.max(np.abs(w - ref)) < 1e-9
