"""libtddft for MI355X: full (non-Tamm-Dancoff) linear-response TDDFT in two localised
function sets (arXiv:1507.08157) as hand-written gfx950 HIP kernels behind a C-ABI.

    from paper_1507_08157_amd import binding
    h = binding.tddft_create(arrays, precision="fp64")
    fp, fq = h.tddft_apply(Pp, Pq)
    omega, status, stats = h.tddft_pcg_solve(n_states)
"""
