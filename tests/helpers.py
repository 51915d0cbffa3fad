"""Shared test helpers: systems, C-ABI handles, oracle operators."""
from __future__ import annotations

import numpy as np

from synth import abi as sabi


XC_MODES = {  # C-ABI coupling kernel -> oracle switches
    0: dict(xc=True, hartree=True),
    1: dict(xc=False, hartree=True),
    2: dict(xc=False, hartree=False),
}


def response_mask(sysm):
    """Function-level mask of the response pattern (blocks of K^c S^u L S^o K^v, L on M;
    M itself in the linear-scaling mode)."""
    return np.kron(sabi.response_blocks(sysm), np.ones((sysm.vir.n_per_atom, sysm.occ.n_per_atom))).astype(bool)


def random_p(sysm, n, seed):
    """Random response kernels on the response pattern, [n, n_u, n_o]."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, sysm.vir.n_fn, sysm.occ.n_fn))
    return X * response_mask(sysm)[None]


def gpu_handle(sysm, **opts):
    """C-ABI handle of a synthetic system; the response kernels are truncated to M (the
    linear-scaling mode) when the system is built that way."""
    from paper_1507_08157_amd import binding
    opts.setdefault("truncate_p", int(getattr(sysm.cfg, "mask_p", False)))
    return binding.tddft_create(sabi.system_arrays(sysm), **opts)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
