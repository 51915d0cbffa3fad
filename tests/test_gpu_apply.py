"""GPU parity of tddft_apply (Eq. operator_RPA) against the FP64 oracle, element by element
on M, for every coupling mode, precision mode and test geometry (dense and truncated
patterns, grids of 40^3 (radix 2, 5), 45^3 (radix 3, 5; ragged tiles), 70^3 (radix 2, 5, 7;
ragged tiles), 64^3 and 320^3 (two-buffer FFT passes), and well-separated atoms), and in
the linear-scaling form of Sec. IV.C: density kernels truncated at a radius, response
kernels truncated to M (`small_kt`) or exact on the blocks they reach (`small_kt_exactp`)."""
import sys

import numpy as np
import pytest

from helpers import XC_MODES, gpu_handle, random_p, rel_err, response_mask, to_dev
from oracle.apply import Operator
from synth import abi as sabi

pytestmark = pytest.mark.gpu

# FP64: every product/sum is exact up to rounding of O(10^3)-term FP64 sums.
TOL_FP64 = 1e-11


def _run(sysm, xc, precision, n, seed=1):
    print(f"[apply] {sysm.cfg.name} N={sysm.cfg.N} xc={xc} {precision} n={n}", flush=True)
    sys.stdout.flush()
    op = Operator(sysm, **XC_MODES[xc])
    Pp = random_p(sysm, n, seed)
    Pq = random_p(sysm, n, seed + 100)
    fp_ref, fq_ref = op.apply(Pp, Pq)
    h = gpu_handle(sysm, precision=precision, xc=xc)
    fp, fq = h.tddft_apply(to_dev(sabi.dense_to_p(sysm, Pp)), to_dev(sabi.dense_to_p(sysm, Pq)))
    fp = sabi.p_to_dense(sysm, fp.cpu().numpy())
    fq = sabi.p_to_dense(sysm, fq.cpu().numpy())
    h.close()
    return fp, fq, fp_ref, fq_ref, op, Pq


@pytest.mark.parametrize("name", ["small_dense", "small_odd", "small_trunc", "separated",
                                  "small_kt", "small_kt_exactp"])
@pytest.mark.parametrize("xc", [2, 1, 0])
def test_apply_fp64(name, xc, request):
    s = request.getfixturevalue(name)
    fp, fq, fp_ref, fq_ref, _, _ = _run(s, xc, "fp64", 3)
    assert rel_err(fp, fp_ref) < TOL_FP64
    assert rel_err(fq, fq_ref) < TOL_FP64
    outside = ~response_mask(s)
    assert np.all(fp[:, outside] == 0) and np.all(fq[:, outside] == 0)


@pytest.mark.parametrize("name", ["small_dense", "small_odd", "small_trunc", "separated",
                                  "small_kt", "small_kt_exactp"])
def test_response_pattern_matches_independent_constructions(name, request):
    """The library's response pattern equals the generator's and the oracle's (`separated`:
    block-diagonal factors with vanishing diagonal blocks of K^v and K^c)."""
    from oracle.apply import response_pattern
    from synth import abi as sabi
    s = request.getfixturevalue(name)
    h = gpu_handle(s, precision="fp64")
    rowptr, colind = h.tddft_response_pattern()
    h.close()
    lib = np.zeros((s.cfg.n_atoms, s.cfg.n_atoms), dtype=bool)
    for i in range(s.cfg.n_atoms):
        lib[i, colind[rowptr[i]:rowptr[i + 1]]] = True
    assert np.array_equal(lib, sabi.response_blocks(s))
    assert np.array_equal(lib, response_pattern(s))


@pytest.mark.parametrize("n", [1, 2, 5, 8, 13, 32])
def test_apply_fp64_state_counts(small_trunc, n):
    fp, fq, fp_ref, fq_ref, _, _ = _run(small_trunc, 0, "fp64", n, seed=n)
    assert rel_err(fp, fp_ref) < TOL_FP64
    assert rel_err(fq, fq_ref) < TOL_FP64


@pytest.mark.parametrize("name", ["small_trunc", "small_kt"])
@pytest.mark.parametrize("precision,bound", [("fp32", 2e-5), ("bf16", 2e-2)])
def test_apply_reduced_precision(name, precision, bound, request):
    """FP32: T-term and coupling both at FP32 rounding (sums of ~10^3 terms, relative
    2^-24 * 10^3 ~ 6e-5 worst case, typically far lower).  BF16 grid samples (relative
    2^-9 each, entering twice: rho and the integrals) bound the coupling part by ~1e-2 of its
    own size; the T-term stays FP32."""
    s = request.getfixturevalue(name)
    fp, fq, fp_ref, fq_ref, op, Pq = _run(s, 0, precision, 4)
    assert rel_err(fp, fp_ref) < 2e-5
    coup = op.coupling(Pq)
    err_q = np.max(np.abs(fq - fq_ref))
    assert err_q < bound * np.max(np.abs(coup)) + 2e-5 * np.max(np.abs(fq_ref))


@pytest.mark.parametrize("precision,tol", [("fp64", TOL_FP64), ("fp32", 2e-5)])
def test_apply_crowded_tiles(precision, tol):
    """Tiles with 6 to 18 o-atoms (the grid kernels stage per-tile operands in batches
    sized by the atom count) and 5 states (a partial last pass of the density in both
    precisions)."""
    from conftest import cached_system
    s = cached_system("small_crowded")
    fp, fq, fp_ref, fq_ref, op, Pq = _run(s, 0, precision, 5, seed=21)
    assert rel_err(fp, fp_ref) < tol
    if precision == "fp64":
        assert rel_err(fq, fq_ref) < tol
    else:
        err_q = np.max(np.abs(fq - fq_ref))
        assert err_q < 2e-5 * np.max(np.abs(fq_ref))


def test_apply_tiny_power_of_two_grid():
    from conftest import cached_system
    s = cached_system("tiny")
    fp, fq, fp_ref, fq_ref, _, _ = _run(s, 0, "fp64", 3, seed=7)
    assert rel_err(fq, fq_ref) < TOL_FP64


def test_apply_320_grid_in_place_on_1024_threads():
    """320^3 grid (radix 8, 8, 5): each FFT pass runs in place in one LDS buffer on
    workgroups of 1024 threads (16 x 321 complex values: 82 KB in FP64, 41 KB in FP32);
    FP64 and FP32 parity against the oracle."""
    from conftest import cached_system
    s = cached_system("wide_grid")
    for precision, tol in (("fp64", TOL_FP64), ("fp32", 2e-5)):
        fp, fq, fp_ref, fq_ref, _, _ = _run(s, 0, precision, 1, seed=5)
        assert rel_err(fp, fp_ref) < tol
        assert rel_err(fq, fq_ref) < tol


def test_grid_beyond_lds_is_refused():
    """448^3 (radix 7 and 64): an axis with a factor 7 takes two LDS line buffers per
    workgroup, 2 x 16 x 449 x 16 B = 230 KB in FP64, beyond the 160 KiB of a gfx950
    workgroup: creation refuses it with a clear error, before any transform runs; FP32
    (115 KB) is accepted."""
    import dataclasses
    from paper_1507_08157_amd import binding
    from synth import build_system, configs
    s = build_system(dataclasses.replace(configs.separated(), N=448))
    print("[apply] 448^3 fp64 creation", flush=True)
    with pytest.raises(binding.TddftError) as e:
        gpu_handle(s, precision="fp64")
    assert e.value.code == binding.TDDFT_E_INVALID and "LDS" in str(e.value)
    gpu_handle(s, precision="fp32").close()


@pytest.mark.parametrize("n", [0, 33])
def test_apply_rejects_state_count_outside_range(small_dense, n):
    """0 states (empty input) and more than the maximum of 32 are refused on the host."""
    import torch
    from paper_1507_08157_amd import binding
    s = small_dense
    h = gpu_handle(s, precision="fp64")
    P = torch.zeros((n, h.nnz_p), dtype=torch.float64, device="cuda")
    with pytest.raises(binding.TddftError) as e:
        h.tddft_apply(P, P.clone())
    h.close()
    assert e.value.code == binding.TDDFT_E_INVALID


def test_info_counts_nonzero_work(small_kt):
    """tddft_get_info's nonzero-sample and pair-point counts (the work units the benchmark
    reports) against a direct count on the full grid."""
    from oracle.grid import to_global
    s = small_kt
    h = gpu_handle(s, precision="fp32")
    info = h.tddft_get_info()
    h.close()
    nu = (to_global(s.cfg.N, s.vir) != 0).sum(axis=0)
    no = (to_global(s.cfg.N, s.occ) != 0).sum(axis=0)
    assert info["samples_u_nz"] == int(nu.sum())
    assert info["samples_o_nz"] == int(no.sum())
    assert info["pair_points_nz"] == int((nu.astype(np.int64) * no).sum())
    assert info["pair_points"] >= info["pair_points_nz"]


@pytest.mark.parametrize("name,precision", [("small_kt", "fp32"), ("small_trunc", "fp64"),
                                            ("small_dense", "bf16")])
def test_autotuned_launch_shapes_give_identical_results(name, precision, request):
    """The launch shapes the creation-time tuner picks (FFT threads per axis, density tiles
    per workgroup, sparse-product columns per thread) change no arithmetic: the apply is
    bit-identical to the fixed defaults."""
    s = request.getfixturevalue(name)
    print(f"[apply] autotune {name} {precision}", flush=True)
    Pp = to_dev(sabi.dense_to_p(s, random_p(s, 4, 61)))
    Pq = to_dev(sabi.dense_to_p(s, random_p(s, 4, 62)))
    out = {}
    for tune in (0, 1):
        h = gpu_handle(s, precision=precision, autotune=tune)
        info = h.tddft_get_info()
        fp, fq = h.tddft_apply(Pp, Pq)
        out[tune] = (fp.cpu().numpy(), fq.cpu().numpy(), info)
        h.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    info = out[1][2]
    assert all(t in (0, 256, 512, 1024) for t in info["fft_threads"])
    assert info["density_waves"] in (2, 4, 8) and all(c in (1, 2, 4) for c in info["kshift_cw"])
    assert all(p in (1, 2, 4, 8) for p in info["kshift_pairs"])
    assert info["density_pbcast"] in (0, 1)
    assert all(t in (0, 1, 2) for t in info["kshift_tile"])


@pytest.mark.parametrize("name,precision", [("small_kt", "fp32"), ("small_odd", "fp32"),
                                            ("small_joint", "fp32"), ("small_crowded", "fp32"),
                                            ("small_dense", "bf16"), ("small_kt", "fp64"),
                                            ("small_joint", "fp64"), ("small_odd", "fp64")])
def test_density_p_forms_are_identical(name, precision):
    """The response density keeps a pass's P block either in scalar registers or in vector
    registers read through DPP row broadcasts; both run the same FMAs in the same order, so
    applies are bit-identical (the scalar form is the one the parity tests pin), over the
    block shapes 3x2 (small_kt), the odd-sized grid, 5x2 (joint u-set) and crowded tiles."""
    from conftest import cached_system
    s = cached_system(name)
    print(f"[apply] density P forms {name} {precision}", flush=True)
    Pp = to_dev(sabi.dense_to_p(s, random_p(s, 4, 71)))
    Pq = to_dev(sabi.dense_to_p(s, random_p(s, 4, 72)))
    out = {}
    for form in (0, 1):
        h = gpu_handle(s, precision=precision, density_pbcast=form)
        assert h.tddft_get_info()["density_pbcast"] == form
        fp, fq = h.tddft_apply(Pp, Pq)
        out[form] = (fp.cpu().numpy(), fq.cpu().numpy())
        # 2 states (the two-state kernel) and 3 (a pass with fewer states than its kernel)
        for m in (2, 3):
            fpm, fqm = h.tddft_apply(Pp[:m].contiguous(), Pq[:m].contiguous())
            out[form] += (fpm.cpu().numpy(), fqm.cpu().numpy())
        h.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dense_product_tiles_are_identical(small_dense, precision):
    """The dense (complete-pattern) MFMA products run in three output tile shapes that share
    the k-slab depth, so each MFMA sums the same products: applies and a whole solve are
    bit-identical across the shapes."""
    s = small_dense
    print(f"[apply] dense product tiles {precision}", flush=True)
    Pp = to_dev(sabi.dense_to_p(s, random_p(s, 4, 81)))
    Pq = to_dev(sabi.dense_to_p(s, random_p(s, 4, 82)))
    L0 = to_dev(sabi.dense_to_p(s, s.guess()))
    from paper_1507_08157_amd import binding
    out = {}
    for tile in (0, 1, 2):
        h = gpu_handle(s, precision=precision, gemm_tile=tile)
        info = h.tddft_get_info()
        assert info["kshift_tile"] == [tile, tile]
        fp, fq = h.tddft_apply(Pp, Pq)
        o = binding.tddft_default_options(precision=precision, tol_omega=1e-8)
        w, rc, st = h.tddft_pcg_solve(3, o, L0.clone(), L0.clone())
        out[tile] = (fp.cpu().numpy(), fq.cpu().numpy(), w)
        h.close()
    for tile in (1, 2):
        for a, b in zip(out[0], out[tile]):
            assert np.array_equal(a, b)


SPARSE_VARIANTS = [(1, 1), (1, 2), (1, 4), (1, 8), (2, 1), (2, 2), (2, 4), (4, 1), (4, 2)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sparse_product_variants_are_identical(small_kt, precision):
    """Every (columns per thread, operand pairs per round trip) form of the sparse-pattern
    products sums the pairs in list order: applies and a 15-iteration truncated solve are
    bit-identical across the forms."""
    s = small_kt
    print(f"[apply] sparse product variants {precision}", flush=True)
    Pp = to_dev(sabi.dense_to_p(s, random_p(s, 4, 83)))
    Pq = to_dev(sabi.dense_to_p(s, random_p(s, 4, 84)))
    from paper_1507_08157_amd import binding
    out = {}
    for cw, pb in SPARSE_VARIANTS:
        h = gpu_handle(s, precision=precision, autotune=0, sparse_cw=cw, sparse_pairs=pb)
        info = h.tddft_get_info()
        assert info["kshift_cw"] == [cw, cw] and info["kshift_pairs"] == [pb, pb]
        fp, fq = h.tddft_apply(Pp, Pq)
        L0 = to_dev(sabi.dense_to_p(s, s.guess(4)))
        o = binding.tddft_default_options(precision=precision, truncate_p=int(s.cfg.mask_p),
                                          max_iter=15, tol_omega=1e-12)
        w, rc, st = h.tddft_pcg_solve(4, o, L0.clone(), L0.clone())
        out[(cw, pb)] = (fp.cpu().numpy(), fq.cpu().numpy(), np.asarray(w))
        h.close()
    assert np.max(np.abs(out[(1, 1)][1])) > 0
    for v in SPARSE_VARIANTS[1:]:
        for a, b in zip(out[(1, 1)], out[v]):
            assert np.array_equal(a, b), v
