"""The allocation-free application (tddft_apply_noalloc) against tddft_apply: same
results on two calls in a row, the second with fewer states and another system, and a
clear refusal when the workspace would exceed the library's per-GPU array."""
import sys

import numpy as np
import pytest

from helpers import gpu_handle, random_p, to_dev
from synth import abi as sabi

pytestmark = pytest.mark.gpu


def _pair(sysm, precision, n, seed):
    print(f"[noalloc] {sysm.cfg.name} {precision} n={n}", flush=True)
    sys.stdout.flush()
    import torch
    h = gpu_handle(sysm, precision=precision)
    Pp = to_dev(sabi.dense_to_p(sysm, random_p(sysm, n, seed)))
    Pq = to_dev(sabi.dense_to_p(sysm, random_p(sysm, n, seed + 1)))
    ref = h.tddft_apply(Pp, Pq)
    fp, fq = torch.empty_like(Pp), torch.empty_like(Pq)
    h.tddft_apply_noalloc(Pp, Pq, fp, fq)
    torch.cuda.synchronize()
    h.close()
    return [x.cpu().numpy() for x in (*ref, fp, fq)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_apply_on_two_calls(small_kt, small_dense, precision):
    # first call: 6 states of the 32-atom truncated system; second: 2 states of a smaller
    # system, so the second call reuses the array with a smaller input
    for sysm, n, seed in ((small_kt, 6, 3), (small_dense, 2, 4)):
        rp, rq, fp, fq = _pair(sysm, precision, n, seed)
        # same kernels, same order of every sum: identical results
        assert np.array_equal(fp, rp) and np.array_equal(fq, rq)
        assert np.max(np.abs(rq)) > 0


def test_noalloc_refuses_oversized_workspace():
    from conftest import cached_system
    from paper_1507_08157_amd import binding
    import torch
    s = cached_system("wide_grid")         # 320^3 grid: 32 FP32 states need > 256 MiB
    print("[noalloc] wide_grid fp32 n=32 refusal", flush=True)
    h = gpu_handle(s, precision="fp32")
    P = torch.zeros((32, h.nnz_p), dtype=torch.float64, device="cuda")
    f1, f2 = torch.empty_like(P), torch.empty_like(P)
    with pytest.raises(binding.TddftError) as e:
        h.tddft_apply_noalloc(P, P.clone(), f1, f2)
    h.close()
    assert e.value.code == binding.TDDFT_E_INVALID and "limit" in str(e.value)
    assert binding.tddft_apply_noalloc_limit() == 256 << 20


def test_noalloc_under_graph_capture(small_kt):
    """tddft_apply_noalloc captured into a HIP graph on the handle's own stream: every replay
    (new inputs copied into the captured buffers, eager work and synchronisation between
    replays) equals tddft_apply on those inputs."""
    import torch
    s = small_kt
    print("[noalloc] graph capture small_kt fp32 n=4", flush=True)
    st = torch.cuda.Stream()
    h = gpu_handle(s, precision="fp32", stream=st.cuda_stream)
    n = 4
    Pp = to_dev(sabi.dense_to_p(s, random_p(s, n, 91)))
    Pq = to_dev(sabi.dense_to_p(s, random_p(s, n, 92)))
    fp, fq = torch.empty_like(Pp), torch.empty_like(Pq)
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        h.tddft_apply_noalloc(Pp, Pq, fp, fq)          # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        h.tddft_apply_noalloc(Pp, Pq, fp, fq)
    torch.cuda.synchronize()
    for seed in (93, 95, 97):
        Pp.copy_(to_dev(sabi.dense_to_p(s, random_p(s, n, seed))))
        Pq.copy_(to_dev(sabi.dense_to_p(s, random_p(s, n, seed + 1))))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        rp, rq = h.tddft_apply(Pp, Pq)                  # eager reference between replays
        torch.cuda.synchronize()
        assert np.array_equal(fp.cpu().numpy(), rp.cpu().numpy())
        assert np.array_equal(fq.cpu().numpy(), rq.cpu().numpy())
        print(f"[noalloc] replay with inputs {seed} equals the eager apply", flush=True)
    del g
    h.close()
