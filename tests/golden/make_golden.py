"""Write the stored expected values used by the GPU tests.  Calls only the FP64 oracle and
the synthetic-input generator.

    python tests/golden/make_golden.py

small_trunc_pcg.json: the excitation-energy trajectory of the first 15 iterations of the
preconditioned CG (truncated auxiliary pattern M at 6 bohr, auxiliary-space preconditioner)
on the `small_trunc` system, from the seeded initial guess, with three inner CG steps per
iteration (a longer inner solve of this ill-conditioned auxiliary-space system amplifies
rounding differences between implementations).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.apply import Operator  # noqa: E402
from oracle.pcg import Options, Solver  # noqa: E402
from synth import build_system, configs  # noqa: E402


def main():
    s = build_system(configs.small_trunc())
    it = 15
    r = Solver(Operator(s), Options(n_states=s.cfg.n_states, max_iter=it, max_inner=3,
                                    tol_omega=1e-12)).solve(s.guess())
    out = {"system": "small_trunc", "iterations": it, "max_inner": 3,
           "omega_history": [list(map(float, w)) for w in r.history],
           "inner_iterations": list(map(int, r.inner_iters)),
           "source": "oracle/pcg.py Solver, FP64"}
    with open(os.path.join(HERE, "small_trunc_pcg.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["omega_history"][-1]))


if __name__ == "__main__":
    main()
