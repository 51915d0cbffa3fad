"""GPU oscillator strengths (tddft_oscillator_strengths, velocity form) against the oracle:
the library's gradient integrals through the same converged vectors, and the full
solve-then-strengths path against brute-force Casida eigenvectors."""
import sys

import numpy as np
import pytest

from helpers import gpu_handle, random_p, to_dev
from oracle.casida import Casida
from oracle.spectra import casida_oscillator_strengths, gradient_integrals, oscillator_strengths
from synth import abi as sabi

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["small_dense", "small_odd", "small_kt", "separated"])
def test_moments_match_oracle(name, request):
    """Transition moments sum_ab P_ab G_ab of random kernels on the response pattern:
    the library's FP64 gradient integrals (per-function boxes grown by one point) against
    the oracle's full-grid central differences."""
    s = request.getfixturevalue(name)
    print(f"[spectra] moments {name}", flush=True)
    sys.stdout.flush()
    P = random_p(s, 3, 41)
    omega = np.array([0.1, 0.2, 0.3])
    h = gpu_handle(s, precision="fp64")
    f, D = h.tddft_oscillator_strengths(omega, to_dev(sabi.dense_to_p(s, P)))
    h.close()
    G = gradient_integrals(s.cfg.N, s.cfg.h, s.vir, s.occ)
    f_ref, D_ref = oscillator_strengths(omega, P, G)
    assert np.max(np.abs(D - D_ref)) < 1e-11 * np.max(np.abs(D_ref))
    assert np.max(np.abs(f - f_ref)) < 1e-10 * np.max(f_ref)


@pytest.mark.parametrize("coupling", [1.0, 25.0])
def test_solve_then_strengths_match_brute_force(small_dense, coupling):
    from paper_1507_08157_amd import binding
    s = small_dense
    n = s.cfg.n_states
    print(f"[spectra] solve + strengths, coupling {coupling}", flush=True)
    h = gpu_handle(s, precision="fp64", coupling_scale=coupling)
    o = binding.tddft_default_options(coupling_scale=coupling, tol_omega=1e-11, max_iter=400)
    L0 = to_dev(sabi.dense_to_p(s, s.guess(n)))
    Pp, Pq = L0.clone(), L0.clone()
    w, rc, st = h.tddft_pcg_solve(n, o, Pp, Pq)
    f, D = h.tddft_oscillator_strengths(w, Pp)
    h.close()
    G = gradient_integrals(s.cfg.N, s.cfg.h, s.vir, s.occ)
    w_ref, f_ref, _ = casida_oscillator_strengths(Casida(s, coupling_scale=coupling), G, n)
    assert rc == 0 and np.max(np.abs(w - w_ref)) < 1e-9
    assert np.max(np.abs(f - f_ref)) < 1e-4 * np.max(f_ref)


def test_strengths_reject_bad_arguments(small_dense):
    from paper_1507_08157_amd import binding
    s = small_dense
    h = gpu_handle(s, precision="fp64")
    P = to_dev(sabi.dense_to_p(s, random_p(s, 2, 1)))
    with pytest.raises(binding.TddftError) as e:
        h.tddft_oscillator_strengths(np.array([0.1, -0.2]), P)
    h.close()
    assert e.value.code == binding.TDDFT_E_INVALID
