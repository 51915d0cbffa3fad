"""Shared test helpers: systems, C-ABI handles, oracle operators."""
from __future__ import annotations

import numpy as np

from synth import abi as sabi


XC_MODES = {  # C-ABI coupling kernel -> oracle switches
    0: dict(xc=True, hartree=True),
    1: dict(xc=False, hartree=True),
    2: dict(xc=False, hartree=False),
}


def random_m(sysm, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, sysm.vir.n_fn, sysm.occ.n_fn))
    return X * sysm.fn_mask()[None]


def gpu_handle(sysm, **opts):
    from paper_1507_08157_amd import binding
    return binding.tddft_create(sabi.system_arrays(sysm), **opts)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
