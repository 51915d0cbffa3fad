"""The sampled oracle outputs that the 2000-atom GPU parity test compares against (rows of
the Kohn-Sham-difference term; the coupling of single-block response kernels at their own
block, from the density of that block, the full-grid Poisson solve and only the potential
integrals the sandwich needs there) equal the full oracle apply restricted to the same
entries, on the 32-atom truncated system.  CPU only."""
import numpy as np

from oracle.apply import Operator
from test_gpu_full_scale import sampled_case


def test_sampled_outputs_equal_full_oracle(small_kt):
    s = small_kt
    nu, no = s.cfg.n_u, s.cfg.n_o
    _, blocks, rows, Pp, Pq, tp, tq, coup = sampled_case(s, n_states=3, seed=5, extra_rows=4)
    op = Operator(s, xc=False, hartree=True)
    fp, fq = op.apply(Pp, Pq)
    assert np.max(np.abs(fp[:, rows] - tp)) < 1e-12 * np.max(np.abs(tp))
    C = fq - np.stack([op.T(x) for x in Pq])
    for k, (I, J) in enumerate(blocks):
        full = C[k, I * nu:(I + 1) * nu, J * no:(J + 1) * no]
        # rounding relative to the state's whole coupling (a block can be small)
        assert np.max(np.abs(full - coup[k])) < 1e-12 * np.max(np.abs(C[k]))
        assert np.max(np.abs(full)) > 0
