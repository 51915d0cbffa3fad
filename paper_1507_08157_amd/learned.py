"""Training of the learned block preconditioner (the network behind TDDFT_PC_LEARNED).

Every step runs in libtddft's kernels; this module only moves device tensors between the
calls:

  collect(handle, ...)   converged vectors of one system (plain FP64 PCG) give the guess
                         targets t_IJ (tddft_guess_targets); random auxiliary matrices L
                         give sample gradients g = Pi(L) (tddft_project, Eq. auxiliary)
                         and their tight Eq. precond solutions G* (tddft_precondition);
                         rows pair the block features of R with (g, G*, t) block by block
  train(datasets, ...)   normalisation fitted on the features, then minibatch Adam steps
                         of tddft_mlp_train_step on the loss
                         1/2 ||c * g - G*||^2 / scale + 1/2 (y_guess - t)^2
  model blob             Mlp.export(), passed to a solve as tddft_options.model

    python -m paper_1507_08157_amd.learned --out model.bin [--systems 8] [--atoms 100]

trains on synthetic systems of the benchmark's density (seeded generator, see synth/).
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np

from . import binding


def collect(h, n_states: int, n_samples: int = 4, seed: int = 0, eps_tol: float = 1e-8,
            max_inner: int = 400, solve_options=None):
    """Training rows of one system (device tensors): X [rows, features], g and G* [rows, E],
    t [rows].  Rows are (sample, block of R); blocks must all have the padded shape."""
    import torch
    nf = int(binding.lib().tddft_n_features(h._h))
    F = h.tddft_block_features()
    nb = F.shape[0]
    E = h.nnz_p // nb
    if E * nb != h.nnz_p:
        raise ValueError("collect needs blocks of one shape (uniform atoms)")
    o = solve_options or binding.tddft_default_options(precision="fp64", tol_omega=1e-9,
                                                       max_iter=400)
    Pp = torch.zeros((n_states, h.nnz_p), dtype=torch.float64, device="cuda")
    Pq = torch.zeros_like(Pp)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    L0 = torch.randn((n_states, h.nnz_p), dtype=torch.float64, device="cuda", generator=gen)
    Pp.copy_(L0)
    Pq.copy_(L0)
    w, rc, st = h.tddft_pcg_solve(n_states, o, Pp, Pq)
    t = h.tddft_guess_targets(Pq)
    L = torch.randn((n_samples, h.nnz_p), dtype=torch.float64, device="cuda", generator=gen)
    g = h.tddft_project(L)
    G = h.tddft_precondition(g, eps_tol=eps_tol, max_inner=max_inner)
    X = F.repeat(n_samples, 1)
    return dict(X=X.contiguous(), g=g.reshape(n_samples * nb, E).float().contiguous(),
                gstar=G.reshape(n_samples * nb, E).float().contiguous(),
                t=t.repeat(n_samples).contiguous(), n_features=nf, E=E, omega=w,
                iterations=st["iterations"])


def train(datasets, width: int = 128, epochs: int = 30, batch: int = 4096, lr: float = 2e-3,
          seed: int = 0, log=None):
    """An Mlp fitted to the concatenated rows of `datasets` (from collect)."""
    import torch
    X = torch.cat([d["X"] for d in datasets])
    g = torch.cat([d["g"] for d in datasets])
    gs = torch.cat([d["gstar"] for d in datasets])
    t = torch.cat([d["t"] for d in datasets])
    nf, E = datasets[0]["n_features"], datasets[0]["E"]
    m = binding.Mlp(nf, width, E + 1, seed=seed)
    m.fit_normalisation(X)
    scale = float(gs.square().mean().item())
    rows = X.shape[0]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(rows, device="cuda", generator=gen)
        tot = 0.0
        for b0 in range(0, rows, batch):
            idx = perm[b0:b0 + batch]
            tot += m.train_step(X[idx].contiguous(), g[idx].contiguous(), gs[idx].contiguous(),
                                t[idx].contiguous(), loss_scale=scale, lr=lr)
        hist.append(tot / rows)
        if log:
            log(f"epoch {ep}: mean loss {hist[-1]:.4e}")
    return m, hist


def _main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--systems", type=int, default=8)
    ap.add_argument("--atoms", type=int, default=100)
    ap.add_argument("--states", type=int, default=8)
    ap.add_argument("--samples", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--seed", type=int, default=300000)
    a = ap.parse_args()
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from synth import abi as sabi
    from synth import build_system, configs

    def log(msg):
        print(f"[train] {msg}", flush=True)

    data = []
    for i in range(a.systems):
        t0 = time.perf_counter()
        s = build_system(configs.training_member(i, a.atoms, a.seed))
        h = binding.tddft_create(sabi.system_arrays(s), precision="fp64")
        d = collect(h, a.states, a.samples, seed=a.seed + i)
        h.close()
        data.append(d)
        log(f"system {i}: {s.cfg.n_atoms} atoms, {d['X'].shape[0]} rows, solve "
            f"{d['iterations']} iterations, {time.perf_counter() - t0:.1f} s")
    m, hist = train(data, epochs=a.epochs, seed=a.seed, log=log)
    with open(a.out, "wb") as f:
        f.write(m.export())
    log(f"wrote {a.out}; loss {hist[0]:.4e} -> {hist[-1]:.4e}")


if __name__ == "__main__":
    _main()
