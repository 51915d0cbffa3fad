"""Write the stored expected values used by the GPU tests.  Calls only the FP64 oracle and
the synthetic-input generator.

    python tests/golden/make_golden.py

<name>_pcg.json: the excitation-energy trajectory of the first 15 iterations of the
preconditioned CG (truncated auxiliary pattern M, auxiliary-space preconditioner) from the
seeded initial guess, with three inner CG steps per iteration (a longer inner solve of
these ill-conditioned auxiliary-space systems amplifies rounding differences between
implementations), for
  small_trunc      exact density kernels, M at 6 bohr;
  small_kt         density kernels truncated at 7.5 bohr and re-purified, response
                   kernels truncated to M (the linear-scaling form of Sec. IV.C);
  small_kt_exactp  the same kernels with exact response kernels (Eq. auxiliary).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.apply import Operator  # noqa: E402
from oracle.pcg import Options, Solver  # noqa: E402
from synth import build_system, configs  # noqa: E402


def trajectory(name, it=15, max_inner=3):
    s = build_system(configs.BY_NAME[name]())
    r = Solver(Operator(s), Options(n_states=s.cfg.n_states, max_iter=it, max_inner=max_inner,
                                    tol_omega=1e-12)).solve(s.guess())
    out = {"system": name, "iterations": it, "max_inner": max_inner,
           "omega_history": [list(map(float, w)) for w in r.history],
           "inner_iterations": list(map(int, r.inner_iters)),
           "source": "oracle/pcg.py Solver, FP64"}
    with open(os.path.join(HERE, f"{name}_pcg.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, json.dumps(out["omega_history"][-1]))


def main():
    for name in ("small_trunc", "small_kt", "small_kt_exactp"):
        trajectory(name)


if __name__ == "__main__":
    main()
