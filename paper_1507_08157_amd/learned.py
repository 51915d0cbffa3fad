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

trains on synthetic systems of the benchmark's density (seeded generator, see synth/);

    python -m paper_1507_08157_amd.learned --evaluate model.bin [--systems 50]
        [--seed 400000] [--json out.json]

solves held-out systems (seeds outside the training range) with the plain Eq. precond
preconditioner and with the model, from the same guess, and reports the iteration and
wall-time ratios with bootstrap confidence intervals.
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


def _gen_member(args):
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from synth import abi as sabi
    from synth import build_system, configs
    i, atoms, seed0, n = args
    s = build_system(configs.training_member(i, atoms, seed0))
    return s.cfg.seed, sabi.system_arrays(s), sabi.dense_to_p(s, s.guess(n))


def evaluate(model: bytes, systems: int = 50, atoms: int = 100, seed0: int = 400000,
             states: int = 4, precision: str = "fp32", tol_omega: float = 1e-8, log=None):
    """Plain Eq. precond against the learned preconditioner on held-out systems: per system
    the outer iterations, wall time, fallbacks and the largest |omega_learned -
    omega_plain|; summary ratios (learned / plain) with 95 % bootstrap intervals.  The
    systems are generated by worker processes forked before this process touches the
    GPU."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    members = []
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1),
                                mp_context=mp.get_context("fork")) as ex:
        for m in ex.map(_gen_member, [(i, atoms, seed0, states) for i in range(systems)]):
            members.append(m)
            if log:
                log(f"held-out system {len(members)} of {systems} generated")
    import torch
    rows = []
    for seed, arrays, guess in members:
        h = binding.tddft_create(arrays, precision=precision)
        L0 = torch.from_numpy(np.ascontiguousarray(guess)).cuda()
        res = {}
        for kind in ("plain", "learned"):
            kw = dict(precision=precision, tol_omega=tol_omega, max_iter=300)
            if kind == "learned":
                kw.update(precond="learned", model=model)
            o = binding.tddft_default_options(**kw)
            w, rc, st = h.tddft_pcg_solve(states, o, L0.clone(), L0.clone())
            res[kind] = (w, rc, st)
        h.close()
        (wp, rcp, sp), (wl, rcl, sl) = res["plain"], res["learned"]
        row = {"seed": int(seed), "plain_iterations": sp["iterations"],
               "learned_iterations": sl["iterations"], "plain_s": sp["solve_ms"] / 1e3,
               "learned_s": sl["solve_ms"] / 1e3, "plain_converged": sp["converged"],
               "learned_converged": sl["converged"], "fallbacks": sl["fallbacks"],
               "omega_diff_Ha": float(np.max(np.abs(wl - wp)))}
        rows.append(row)
        if log:
            log(f"seed {seed}: {row}")
    it = np.array([r["learned_iterations"] / r["plain_iterations"] for r in rows])
    tm = np.array([r["learned_s"] / r["plain_s"] for r in rows])
    rng = np.random.default_rng(0)

    def ci(x):
        b = [np.mean(rng.choice(x, len(x))) for _ in range(2000)]
        return [float(np.percentile(b, 2.5)), float(np.percentile(b, 97.5))]
    return {"systems": len(rows), "atoms": atoms, "states": states, "precision": precision,
            "tol_omega": tol_omega, "iteration_ratio_mean": float(it.mean()),
            "iteration_ratio_ci95": ci(it), "time_ratio_mean": float(tm.mean()),
            "time_ratio_ci95": ci(tm),
            "learned_fewer_iterations": int(np.sum(it < 1.0)),
            "fallback_engaged": int(sum(1 for r in rows if r["fallbacks"] > 0)),
            "all_converged": bool(all(r["plain_converged"] and r["learned_converged"] for r in rows)),
            "max_omega_diff_Ha": float(max(r["omega_diff_Ha"] for r in rows)), "rows": rows}


def _main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out")
    ap.add_argument("--evaluate", metavar="MODEL")
    ap.add_argument("--json")
    ap.add_argument("--systems", type=int, default=8)
    ap.add_argument("--atoms", type=int, default=100)
    ap.add_argument("--states", type=int, default=8)
    ap.add_argument("--samples", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--seed", type=int, default=300000)
    a = ap.parse_args()
    import json
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    def log(msg):
        print(f"[train] {msg}", flush=True)

    if a.evaluate:
        model = open(a.evaluate, "rb").read()
        out = evaluate(model, systems=a.systems, atoms=a.atoms, seed0=a.seed, log=log)
        summary = {k: v for k, v in out.items() if k != "rows"}
        log(json.dumps(summary))
        if a.json:
            with open(a.json, "w") as f:
                json.dump(out, f, indent=1)
        return
    if not a.out:
        ap.error("--out (training) or --evaluate MODEL")

    # the systems are generated by worker processes forked before this process touches
    # the GPU; the solves that label them run here, one after another
    import concurrent.futures as cf
    import multiprocessing as mp
    t0 = time.perf_counter()
    members = []
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1),
                                mp_context=mp.get_context("fork")) as ex:
        for m in ex.map(_gen_member, [(i, a.atoms, a.seed, a.states) for i in range(a.systems)]):
            members.append(m)
            log(f"system {len(members)} of {a.systems} generated")
    log(f"{len(members)} systems generated in {time.perf_counter() - t0:.1f} s")
    data = []
    for i, (seed, arrays, _) in enumerate(members):
        t0 = time.perf_counter()
        h = binding.tddft_create(arrays, precision="fp64")
        d = collect(h, a.states, a.samples, seed=a.seed + i)
        h.close()
        data.append(d)
        log(f"system {i} (seed {seed}): {d['X'].shape[0]} rows, solve "
            f"{d['iterations']} iterations, {time.perf_counter() - t0:.1f} s")
    m, hist = train(data, epochs=a.epochs, seed=a.seed, log=log)
    with open(a.out, "wb") as f:
        f.write(m.export())
    log(f"wrote {a.out}; loss {hist[0]:.4e} -> {hist[-1]:.4e}")


if __name__ == "__main__":
    _main()
