"""Parity at the full size of the throughput workload (200 atoms, 128^3 grid, 400 / 600
functions, 8 states) in the launch configuration the benchmark times: one tddft_apply of
all 8 states.

* f_p = T(P^p) (Eq. operator_RPA, no grid work) is compared element by element for every
  state: the oracle's T-term is two dense products per state;
* f_q of one sampled state (the last: imaginary half of the last complex field pair) is
  compared element by element with the oracle's full apply;
* for all 8 states, the coupling part C(P) = f_q - T(P) = 2 K^c V_SCF[P] K^v must give a
  symmetric matrix <P_j, C(P_i)>_S, a property that holds at any size: for invariant
  P = K^c S^u L S^o K^v it is x_j^T 2K x_i with the symmetric Casida coupling K.
The inputs are such invariant kernels (random L, exact products).
"""
import sys

import numpy as np
import pytest

from helpers import gpu_handle, random_p, rel_err, to_dev
from oracle.apply import Operator
from synth import abi as sabi

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

N_STATES = 8
SAMPLED = 7
TOLS = {"fp64": (1e-11, 1e-11, 1e-11), "fp32": (2e-5, 2e-5, 1e-4)}


@pytest.fixture(scope="module")
def full():
    from conftest import cached_system
    print("[full] generating the 200-atom system", flush=True)
    s = cached_system("prec")
    print("[full] oracle set-up", flush=True)
    op = Operator(s)
    Pp = np.stack([op.project(x) for x in random_p(s, N_STATES, 31)])
    Pq = np.stack([op.project(x) for x in random_p(s, N_STATES, 32)])
    print("[full] oracle apply of the sampled state", flush=True)
    _, fq_ref = op.apply(Pp[SAMPLED:SAMPLED + 1], Pq[SAMPLED:SAMPLED + 1])
    tp = np.stack([op.T(x) for x in Pp])
    tq = np.stack([op.T(x) for x in Pq])
    sys.stdout.flush()
    return s, op, Pp, Pq, tp, tq, fq_ref[0]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_full_size_apply(full, precision):
    s, op, Pp, Pq, tp, tq, fq_ref = full
    print(f"[full] GPU apply {precision}, {N_STATES} states", flush=True)
    h = gpu_handle(s, precision=precision)
    fp, fq = h.tddft_apply(to_dev(sabi.dense_to_p(s, Pp)), to_dev(sabi.dense_to_p(s, Pq)))
    fp = sabi.p_to_dense(s, fp.cpu().numpy())
    fq = sabi.p_to_dense(s, fq.cpu().numpy())
    h.close()
    tol_t, tol_q, tol_sym = TOLS[precision]
    assert rel_err(fp, tp) < tol_t
    coup_ref = fq_ref - tq[SAMPLED]
    err_q = np.max(np.abs(fq[SAMPLED] - fq_ref))
    assert err_q < tol_q * np.max(np.abs(fq_ref)), (err_q, np.max(np.abs(coup_ref)))
    # coupling of all states: <P_j, C(P_i)>_S symmetric
    C = fq - tq
    cov = np.stack([op.Su @ x @ op.So for x in Pq])
    G = np.einsum("jab,iab->ij", cov, C)
    assert np.max(np.abs(G - G.T)) < tol_sym * np.max(np.abs(G))
