"""The linear-scaling form of the method (Sec. IV.C) in the oracle and the generator:
density kernels truncated at a radius and re-purified, response kernels truncated to the
pattern M, energy zero mid-gap.  CPU only.

Pins:
  * the mid-gap energy zero leaves the exact method unchanged: for invariant response
    kernels (P = K^c S^u P S^o K^v with idempotent kernels) the operator of Eq.
    operator_RPA does not see H -> H - mu S, and the brute-force Casida energies
    (Sec. II.A) of the shifted and unshifted systems agree;
  * truncation (Sec. IV.C) only restricts: the masked operator applied to kernels on M is
    the exact-pattern operator's result restricted to M, the truncated density kernels
    vanish beyond R_K, stay symmetric and near-idempotent (Sec. III.A after Eq.
    auxiliary);
  * with every radius beyond the cell the truncated form is the exact one.
"""
import dataclasses

import numpy as np
import pytest

from oracle.apply import Operator, response_pattern
from oracle.casida import Casida
from synth import build_system, configs
from synth.system import atom_distances


@pytest.fixture(scope="module")
def kt():
    return build_system(configs.small_kt())


@pytest.fixture(scope="module")
def kt_exact():
    return build_system(configs.small_kt_exactp())


def _shifted(cfg, zero):
    return dataclasses.replace(cfg, energy_zero=zero)


def test_midgap_zero_leaves_brute_force_unchanged():
    c = configs.small_dense()
    s0 = build_system(c)
    s1 = build_system(_shifted(c, "midgap"))
    mu = 0.5 * (s0.eps_o[c.n_occ - 1] + s0.eps_u[s0.vir_idx[0]])
    assert np.allclose(s1.eps_o, s0.eps_o - mu, atol=1e-12)
    assert np.allclose(s1.H_u, s0.H_u - mu * s0.S_u, atol=1e-13)
    # symmetric about zero: the highest occupied and lowest kept conduction level
    assert abs(s1.eps_o[c.n_occ - 1] + s1.eps_u[s1.vir_idx[0]]) < 1e-12
    w0 = Casida(s0).omega_hermitian()
    w1 = Casida(s1).omega_hermitian()
    assert np.max(np.abs(w0 - w1)) < 1e-10


def test_midgap_zero_leaves_operator_unchanged_on_invariant_kernels():
    c = configs.small_dense()
    s0 = build_system(c)
    s1 = build_system(_shifted(c, "midgap"))
    o0, o1 = Operator(s0, xc=False, hartree=False), Operator(s1, xc=False, hartree=False)
    rng = np.random.default_rng(5)
    L = rng.standard_normal((s0.vir.n_fn, s0.occ.n_fn))
    P = o0.project(L)                       # invariant: K^c S P S K^v = P
    t0, t1 = o0.T(P), o1.T(P)
    assert np.max(np.abs(t0 - t1)) < 1e-11 * np.max(np.abs(t0))
    # a kernel outside the invariant space does see the shift (the pin is not vacuous)
    X = rng.standard_normal(P.shape)
    assert np.max(np.abs(o0.T(X) - o1.T(X))) > 1e-3 * np.max(np.abs(o0.T(X)))


def test_truncated_kernels(kt):
    c = kt.cfg
    d = atom_distances(kt.pos, c.L)
    for K, b in ((kt.K_v, c.n_o), (kt.K_c, c.n_u)):
        blk = np.abs(K.reshape(c.n_atoms, b, c.n_atoms, b)).max(axis=(1, 3))
        assert np.all(blk[d > c.R_K] == 0)
        assert np.array_equal(K, K.T)
    assert kt.idem_err["K_v"] < 0.1 and kt.idem_err["K_c"] < 0.1
    assert np.array_equal(kt.M, d <= c.R_M)
    assert 0.05 < kt.M.mean() < 0.5


def test_masked_operator_restricts_the_exact_one(kt, kt_exact):
    """Same inputs (same seed and generator), two response patterns: M and the blocks the
    exact product reaches.  On kernels supported on M the two operators differ only in
    the final restriction."""
    assert np.array_equal(kt.K_c, kt_exact.K_c) and np.array_equal(kt.H_o, kt_exact.H_o)
    assert np.array_equal(response_pattern(kt), kt.M)
    Rx = response_pattern(kt_exact)
    assert Rx.sum() > kt.M.sum() and np.all(Rx[kt.M])
    om, ox = Operator(kt), Operator(kt_exact)
    rng = np.random.default_rng(9)
    P = rng.standard_normal((2, kt.vir.n_fn, kt.occ.n_fn)) * kt.fn_mask()[None]
    fpm, fqm = om.apply(P[:1], P[1:])
    fpx, fqx = ox.apply(P[:1], P[1:])
    mask = kt.fn_mask()
    assert np.max(np.abs(fpm - fpx * mask)) < 1e-13 * np.max(np.abs(fpx))
    assert np.max(np.abs(fqm - fqx * mask)) < 1e-13 * np.max(np.abs(fqx))
    assert np.all(fqm[:, ~mask] == 0)
    # the projection of Eq. auxiliary likewise
    L = rng.standard_normal((kt.vir.n_fn, kt.occ.n_fn))
    assert np.max(np.abs(om.project(L) - ox.project(L) * mask)) < 1e-13 * np.max(np.abs(ox.project(L)))


def test_radii_beyond_the_cell_give_the_exact_form():
    c = dataclasses.replace(configs.small_kt(), n_atoms=12, n_occ=8, n_vir=12, R_K=100.0,
                            R_M=100.0)
    s = build_system(c)
    e = build_system(dataclasses.replace(c, R_K=None, R_M=None, mask_p=False))
    assert np.allclose(s.K_v, e.K_v, atol=1e-10) and np.allclose(s.K_c, e.K_c, atol=1e-10)
    assert np.all(s.M)
    rng = np.random.default_rng(3)
    P = rng.standard_normal((1, s.vir.n_fn, s.occ.n_fn))
    fs = Operator(s).apply(P, P)[1]
    fe = Operator(e).apply(P, P)[1]
    assert np.max(np.abs(fs - fe)) < 1e-9 * np.max(np.abs(fe))
