"""FP64 CPU oracle for full (non-Tamm-Dancoff) linear-response TDDFT in two localised
function sets (arXiv:1507.08157).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke entry point and the CPU-baseline leg
of the benchmark may import or run anything in this package.  The GPU library never calls
it, shares no code with it, and fails loudly instead of falling back to it.

Modules
  grid    response density, periodic Poisson solve, ALDA kernel, potential integrals
  apply   the Tsiper operator in NGWF space (Sec. III.A, Eq. operator_RPA)
  casida  brute-force dense Casida eigenproblem (Sec. II.A, Eq. TDDFT_ham)
  pcg     preconditioned CG for the lowest N_omega excitations (Secs. III.A-III.C)
  mlp     FP64 reference MLP (forward, backward, Adam) for the learned preconditioner

Everything is plain NumPy/SciPy in float64, written for clarity, not speed.
"""
