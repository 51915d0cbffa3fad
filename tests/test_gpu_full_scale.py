"""Parity at the size of the linear-scaling workload the benchmark times (2000 atoms in an
80 bohr cell, 256^3 grid, 4000 / 6000 functions, density kernels truncated at 15 bohr and
re-purified, response kernels on the 15-bohr pattern M) in its launch configuration: one
tddft_apply of 4 states, in FP64, FP32 and BF16 samples.

The oracle's grid loops visit every atom pair, too slow for a whole 2000-atom apply in a
test, so the outputs are checked where the oracle computes them one by one:
  * the Kohn-Sham-difference term f_p = mask_M(K^c H^u P - P H^o K^v) of every state on
    the rows of sampled u-atoms, exactly (dense row products; P random on all of M);
  * the coupling (Hartree kernel; the ALDA term is compared at small sizes) of states
    whose P^q holds one block each, so that rho is local: the oracle forms rho from that
    block, solves the periodic Poisson problem on the full 256^3 grid, takes the
    potential integrals V_KL of every block the sandwich 2 K^c V K^v needs at a sampled
    output block (u-atoms K in the support of K^c's row, o-atoms L in the support of
    K^v's column) and forms the sandwich there.
"""
import sys

import numpy as np
import pytest

from helpers import gpu_handle, to_dev
from synth import abi as sabi

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N_STATES = 4
TOLS = {"fp64": (1e-11, 1e-10), "fp32": (2e-5, 2e-5), "bf16": (2e-5, 2e-2)}


def _say(msg):
    print(f"[full-scale] {msg}", flush=True)
    sys.stdout.flush()


def _sub(fs, atoms):
    from synth.system import FunctionSet
    atoms = np.asarray(atoms)
    return FunctionSet(fs.n_per_atom, fs.origin[atoms], fs.extent[atoms],
                       [fs.vals[i] for i in atoms])


def _rows(atoms, per):
    return np.concatenate([np.arange(a * per, (a + 1) * per) for a in atoms])


def sampled_case(s, n_states=N_STATES, seed=77, extra_rows=6):
    """Inputs and the oracle's sampled outputs (see the module docstring) for system s."""
    from oracle import grid
    c = s.cfg
    nu, no = c.n_u, c.n_o
    rng = np.random.default_rng(seed)
    mask = s.fn_mask()
    Pp = rng.standard_normal((n_states, s.vir.n_fn, s.occ.n_fn)) * mask[None]
    # P^q: one block (I_k, J_k) of M per state
    Mi, Mj = np.nonzero(s.M)
    pick = rng.choice(len(Mi), n_states, replace=False)
    blocks = [(int(Mi[k]), int(Mj[k])) for k in pick]
    Pq = np.zeros_like(Pp)
    for k, (I, J) in enumerate(blocks):
        Pq[k, I * nu:(I + 1) * nu, J * no:(J + 1) * no] = rng.standard_normal((nu, no))
    # T-term on sampled u-atom rows
    _say("oracle: Kohn-Sham-difference rows")
    samp = np.unique(np.concatenate([rng.choice(c.n_atoms, extra_rows, replace=False),
                                     [b[0] for b in blocks]]))
    rows = _rows(samp, nu)
    KcHu_rows = s.K_c[rows] @ s.H_u
    HoKv = s.H_o @ s.K_v
    tp = np.stack([mask[rows] * (KcHu_rows @ x - x[rows] @ HoKv) for x in Pp])
    tq = np.stack([mask[rows] * (KcHu_rows @ x - x[rows] @ HoKv) for x in Pq])
    # coupling at each state's own block (I_k, J_k)
    coup = []
    for k, (I, J) in enumerate(blocks):
        _say(f"oracle: coupling of state {k} at block {(I, J)}")
        blk = Pq[k, I * nu:(I + 1) * nu, J * no:(J + 1) * no][None]
        rho = grid.density(c.N, _sub(s.vir, [I]), _sub(s.occ, [J]), blk)
        V = grid.poisson_periodic(rho, c.L)
        kc_blk = np.abs(s.K_c[I * nu:(I + 1) * nu].reshape(nu, c.n_atoms, nu)).max(axis=(0, 2)) > 0
        kv_blk = np.abs(s.K_v[:, J * no:(J + 1) * no].reshape(c.n_atoms, no, no)).max(axis=(1, 2)) > 0
        Ks, Ls = np.nonzero(kc_blk)[0], np.nonzero(kv_blk)[0]
        Vm = grid.potential_integrals(c.N, c.h, _sub(s.vir, Ks), _sub(s.occ, Ls), V)[0]
        cq = 2.0 * s.K_c[I * nu:(I + 1) * nu][:, _rows(Ks, nu)] @ Vm @ \
            s.K_v[_rows(Ls, no)][:, J * no:(J + 1) * no]
        coup.append(cq)
    return s, blocks, rows, Pp, Pq, tp, tq, coup


@pytest.fixture(scope="module")
def case():
    from conftest import cached_system
    _say("generating the 2000-atom system")
    return sampled_case(cached_system("scale2000"))


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_full_scale_apply(case, precision):
    s, blocks, rows, Pp, Pq, tp, tq, coup = case
    c = s.cfg
    nu, no = c.n_u, c.n_o
    _say(f"GPU apply {precision}, {N_STATES} states")
    h = gpu_handle(s, precision=precision, xc=1)
    fp, fq = h.tddft_apply(to_dev(sabi.dense_to_p(s, Pp)), to_dev(sabi.dense_to_p(s, Pq)))
    h.close()
    fp = sabi.p_to_dense(s, fp.cpu().numpy())
    fq = sabi.p_to_dense(s, fq.cpu().numpy())
    tol_t, tol_c = TOLS[precision]
    # Kohn-Sham-difference term of every state on the sampled rows (f_p has no coupling)
    assert np.max(np.abs(fp[:, rows] - tp)) < tol_t * np.max(np.abs(tp))
    # coupling: f_q - T(P^q) at each state's block; elsewhere on the sampled rows f_q
    # is the T-term plus a coupling the oracle does not form here
    for k, (I, J) in enumerate(blocks):
        r0 = int(np.nonzero(rows == I * nu)[0][0])
        t_blk = tq[k, r0:r0 + nu, J * no:(J + 1) * no]
        got = fq[k, I * nu:(I + 1) * nu, J * no:(J + 1) * no] - t_blk
        err = np.max(np.abs(got - coup[k]))
        _say(f"{precision} state {k}: coupling max {np.max(np.abs(coup[k])):.3e}, error {err:.2e}")
        assert err < tol_c * np.max(np.abs(coup[k])) + tol_t * np.max(np.abs(t_blk))
    # nothing outside M
    assert np.all(fq[:, ~s.fn_mask()] == 0) and np.all(fp[:, ~s.fn_mask()] == 0)
