"""GPU parity of tddft_pcg_solve: converged excitation energies against brute-force Casida
(dense kernels) and against the oracle PCG (truncated kernels)."""
import sys

import numpy as np
import pytest

from helpers import gpu_handle, to_dev
from oracle.apply import Operator
from oracle.casida import Casida
from oracle.pcg import Options, Solver
from synth import abi as sabi

pytestmark = pytest.mark.gpu


def _solve(sysm, precision="fp64", n=None, guess=True, **kw):
    from paper_1507_08157_amd import binding
    n = n or sysm.cfg.n_states
    print(f"[pcg] {sysm.cfg.name} {precision} n={n} {kw}", flush=True)
    sys.stdout.flush()
    h = gpu_handle(sysm, precision=precision)
    o = binding.tddft_default_options(precision=precision, **kw)
    if guess:
        L0 = to_dev(sabi.dense_to_m(sysm, sysm.guess(n)))
        Pp, Pq = L0.clone(), L0.clone()
    else:
        Pp = Pq = None
    w, rc, st = h.tddft_pcg_solve(n, o, Pp, Pq, log_capacity=1000)
    h.close()
    return w, rc, st, Pp, Pq


@pytest.mark.parametrize("precond", [1, 0])
def test_pcg_dense_matches_brute_force(small_dense, precond):
    s = small_dense
    w, rc, st, _, _ = _solve(s, tol_omega=1e-10, precond=precond)
    ref = Casida(s).omega_hermitian()[:s.cfg.n_states]
    assert rc == 0 and st["converged"]
    assert np.max(np.abs(w - ref)) < 1e-9


def test_pcg_tiny_matches_brute_force():
    from conftest import cached_system
    s = cached_system("tiny")
    w, rc, st, _, _ = _solve(s, tol_omega=1e-10)
    ref = Casida(s).omega_hermitian()[:3]
    assert rc == 0
    assert np.max(np.abs(w - ref)) < 1e-9


def test_pcg_no_coupling_is_ks_difference(small_dense):
    s = small_dense
    w, rc, st, _, _ = _solve(s, tol_omega=1e-11, xc=2)
    D = np.sort(Casida(s, xc=False, hartree=False).D)
    assert np.max(np.abs(w - D[:3])) < 1e-9


def test_pcg_random_guess_converges(small_dense):
    s = small_dense
    w, rc, st, _, _ = _solve(s, tol_omega=1e-10, guess=False)
    ref = Casida(s).omega_hermitian()[:3]
    assert np.max(np.abs(w - ref)) < 1e-9


def test_pcg_truncated_matches_oracle_pcg(small_trunc):
    s = small_trunc
    n = s.cfg.n_states
    w, rc, st, Pp, Pq = _solve(s, tol_omega=1e-10)
    ref = Solver(Operator(s), Options(n_states=n, tol_omega=1e-11, max_iter=400)).solve(s.guess())
    assert np.max(np.abs(w - ref.omega)) < 1e-8


@pytest.mark.parametrize("precision,bound", [("fp32", 1e-6), ("bf16", 1e-4)])
def test_pcg_reduced_precision_error(small_trunc, precision, bound):
    s = small_trunc
    w64, _, _, _, _ = _solve(s, tol_omega=1e-10)
    w, rc, st, _, _ = _solve(s, precision=precision, tol_omega=1e-9, max_iter=150)
    print(f"[pcg] {precision} omega error vs fp64: {np.max(np.abs(w - w64)):.3e}", flush=True)
    assert np.max(np.abs(w - w64)) < bound


def test_pcg_stats_and_log(small_dense):
    w, rc, st, _, _ = _solve(small_dense, tol_omega=1e-8)
    assert st["applies"] >= st["iterations"]
    assert st["log_omega"].shape[1] == 3
    assert np.all(np.diff(st["log_time_ms"]) >= 0)


def test_pcg_no_convergence_status(small_dense):
    from paper_1507_08157_amd import binding
    w, rc, st, _, _ = _solve(small_dense, tol_omega=1e-12, max_iter=2)
    assert rc == binding.TDDFT_E_NO_CONVERGENCE
    assert np.all(np.isfinite(w)) and not st["converged"]
