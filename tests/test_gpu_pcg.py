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


CREATE_KEYS = ("xc", "coupling_scale", "rho_floor")


def _solve(sysm, precision="fp64", n=None, guess=True, **kw):
    from paper_1507_08157_amd import binding
    n = n or sysm.cfg.n_states
    print(f"[pcg] {sysm.cfg.name} {precision} n={n} {kw}", flush=True)
    sys.stdout.flush()
    h = gpu_handle(sysm, precision=precision, **{k: v for k, v in kw.items() if k in CREATE_KEYS})
    o = binding.tddft_default_options(precision=precision,
                                      truncate_p=int(getattr(sysm.cfg, "mask_p", False)), **kw)
    if guess:
        L0 = to_dev(sabi.dense_to_p(sysm, sysm.guess(n)))
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


def test_pcg_truncated_trajectory_matches_oracle(small_trunc):
    """Truncated auxiliary pattern M (auxiliary-space gradient and preconditioner): the
    first 15 iterations (three inner CG steps each) reproduce the oracle's energies (stored
    by tests/golden/make_golden.py), iteration by iteration."""
    import json
    import os
    s = small_trunc
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "small_trunc_pcg.json")))
    w, rc, st, Pp, Pq = _solve(s, tol_omega=1e-12, max_iter=gold["iterations"],
                               max_inner=gold["max_inner"])
    ref = np.array(gold["omega_history"])
    got = st["log_omega"]
    assert got.shape == ref.shape
    err = np.max(np.abs(got - ref), axis=1)
    print("[pcg] trajectory error per iteration:", np.array2string(err, precision=2), flush=True)
    assert np.all(err < 1e-7)
    # variational: never below the untruncated (brute-force) energies
    assert np.all(w >= Casida(s).omega_hermitian()[:s.cfg.n_states] - 1e-9)


@pytest.mark.parametrize("name", ["small_kt", "small_kt_exactp"])
def test_pcg_truncated_kernels_trajectory_matches_oracle(name, request):
    """Density kernels truncated at 7.5 bohr and re-purified: the linear-scaling form with
    response kernels truncated to M (`small_kt`, Sec. IV.C) and the exact-response form
    (`small_kt_exactp`, Eq. auxiliary).  FP64 excitation energies of the first 15
    iterations against the oracle's (tests/golden/<name>_pcg.json, written by
    tests/golden/make_golden.py), iteration by iteration."""
    import json
    import os
    s = request.getfixturevalue(name)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", f"{name}_pcg.json")))
    w, rc, st, Pp, Pq = _solve(s, tol_omega=1e-12, max_iter=gold["iterations"],
                               max_inner=gold["max_inner"])
    ref = np.array(gold["omega_history"])
    got = st["log_omega"]
    assert got.shape == ref.shape
    err = np.max(np.abs(got - ref), axis=1)
    print(f"[pcg] {name} trajectory error per iteration:", np.array2string(err, precision=2),
          flush=True)
    assert np.all(err < 1e-7)
    # the sum functional decreases along the trajectory
    sums = ref.sum(axis=1)
    assert sums[-1] < sums[0]


@pytest.mark.parametrize("name", ["small_dense", "tiny"])
@pytest.mark.parametrize("precision,bound", [("fp32", 1e-6), ("bf16", 1e-5)])
def test_pcg_reduced_precision_error(name, precision, bound):
    """Mixed precision (FP32 or BF16 grid samples, FP32 sparse products, FP64 traces and
    control) against the FP64 solve of the same system; the error is printed."""
    from conftest import cached_system
    s = cached_system(name)
    w64, rc64, _, _, _ = _solve(s, tol_omega=1e-10)
    w, rc, st, _, _ = _solve(s, precision=precision, tol_omega=1e-9, max_iter=300)
    print(f"[pcg] {name} {precision} omega error vs fp64: {np.max(np.abs(w - w64)):.3e} "
          f"({st['iterations']} iterations)", flush=True)
    assert rc64 == 0
    assert np.max(np.abs(w - w64)) < bound


def test_pcg_stats_and_log(small_dense):
    w, rc, st, _, _ = _solve(small_dense, tol_omega=1e-8)
    assert st["applies"] >= st["iterations"]
    assert st["log_omega"].shape[1] == 3
    assert np.all(np.diff(st["log_time_ms"]) >= 0)


def test_pcg_rejects_create_time_option_mismatch(small_dense):
    from paper_1507_08157_amd import binding
    h = gpu_handle(small_dense, precision="fp64")
    o = binding.tddft_default_options(precision="fp64", xc=2)
    with pytest.raises(binding.TddftError) as e:
        h.tddft_pcg_solve(3, o)
    assert e.value.code == binding.TDDFT_E_INVALID
    h.close()


def test_pcg_strong_coupling_matches_brute_force(small_dense):
    """Coupling scaled by 25: full and TDA energies differ by > 1e-3 Ha, the solver still
    reproduces the full (non-TDA) Casida eigenvalues."""
    s = small_dense
    w, rc, st, _, _ = _solve(s, tol_omega=1e-10, coupling_scale=25.0)
    cs = Casida(s, coupling_scale=25.0)
    ref = cs.omega_hermitian()[:3]
    assert np.max(np.abs(w - ref)) < 1e-9
    assert np.max(np.abs(cs.omega_tda()[:3] - ref)) > 1e-3


def test_pcg_no_convergence_status(small_dense):
    from paper_1507_08157_amd import binding
    w, rc, st, _, _ = _solve(small_dense, tol_omega=1e-12, max_iter=2)
    assert rc == binding.TDDFT_E_NO_CONVERGENCE
    assert np.all(np.isfinite(w)) and not st["converged"]


@pytest.mark.parametrize("name", ["small_dense", "tiny"])
def test_pcg_adaptive_inner_tolerance(name, request):
    from conftest import cached_system
    from oracle.casida import Casida
    s = cached_system(name)
    w, rc, st, _, _ = _solve(s, tol_omega=1e-10, eps_loose=0.1)
    assert st["converged"]
    assert np.max(np.abs(w - Casida(s).omega_hermitian()[:s.cfg.n_states])) < 1e-9


@pytest.mark.parametrize("name", ["small_dense", "small_kt"])
def test_pcg_graph_replay_is_identical(name, request):
    """Operator applications replayed from captured HIP graphs give bit-identical
    trajectories to direct launches (same kernels, same order of every sum)."""
    s = request.getfixturevalue(name)
    wg, rcg, stg, _, _ = _solve(s, precision="fp32", tol_omega=1e-9, max_iter=60, graphs=1)
    wd, rcd, std, _, _ = _solve(s, precision="fp32", tol_omega=1e-9, max_iter=60, graphs=0)
    assert stg["graph_replays"] > 0 and std["graph_replays"] == 0
    assert stg["iterations"] == std["iterations"]
    assert np.array_equal(stg["log_omega"], std["log_omega"])
    assert np.array_equal(wg, wd)
