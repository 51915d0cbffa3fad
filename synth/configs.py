"""Named workloads.

tiny   : 12 atoms, 20 bohr cube, 64^3, 24 o / 36 u functions, r_c 6, dense kernels,
         8 occupied / 16 virtual states, 3 excitations (plain FP64 parity case).
prec   : 200 atoms, 40 bohr, 128^3, 400 o / 600 u, r_c 7, 8 excitations (precision study;
         the throughput workload); complete auxiliary pattern M (see below).
batch  : 64 systems of 50..300 atoms (uniform), box scaled to keep the density of `prec`,
         grid edge a multiple of 16 in [64, 128], r_c 6, R 20, 4 excitations each.
scale  : 2000 atoms, 80 bohr, 256^3, 4000 o / 6000 u, r_c 6, every density matrix
         truncated at 15 bohr (~3 % block fill), 4 excitations; 500- and 1000-atom
         companions at equal density (scale500, scale1000, scale2000).
Small test systems (several grid tiles, ragged tile tails, non-power-of-two FFTs) are
defined here too.

n_occ / n_vir beyond `tiny` follow n_occ = round(2 * atoms / 3), n_vir = 2 n_occ.
`prec` and the batch keep exact density kernels (these synthetic systems have level
spacings of ~1e-3 Ha and no spectral gap at the Fermi level, so their exact P is
delocalised).  The linear-scaling family (`scale*`, `small_kt`) truncates every density
matrix at a radius as Sec. IV.C does: K^v and K^c at R_K with two masked McWeeny steps, and
the response kernels to the pattern M; with the energy zero mid-gap the non-invariant
remainder this truncation leaves carries positive energy.
Seeds: base = 1000 * config_index + system_index.
"""
from __future__ import annotations

from .system import Config


def tiny(seed: int = 0) -> Config:
    return Config(name="tiny", n_atoms=12, L=20.0, N=64, r_c=6.0, n_occ=8, n_vir=16,
                  R_K=None, R_M=None, n_states=3, seed=seed)


def prec(seed: int = 1000) -> Config:
    return Config(name="prec", n_atoms=200, L=40.0, N=128, r_c=7.0, n_occ=133, n_vir=266,
                  R_K=None, R_M=None, n_states=8, seed=seed)


def _occ(n_atoms: int) -> int:
    return int(round(2 * n_atoms / 3))


def batch_member(i: int, n_atoms: int) -> Config:
    h = 0.3125
    L = 40.0 * (n_atoms / 200.0) ** (1.0 / 3.0)
    N = int(min(128, max(64, 16 * round(L / (16 * h)))))
    L = N * h
    return Config(name=f"batch{i}", n_atoms=n_atoms, L=L, N=N, r_c=6.0,
                  n_occ=_occ(n_atoms), n_vir=2 * _occ(n_atoms), R_K=None, R_M=None,
                  n_states=4, seed=2000 + i)


def batch(n_systems: int = 64):
    import numpy as np
    rng = np.random.default_rng(2000)
    atoms = rng.integers(50, 301, n_systems)
    return [batch_member(i, int(a)) for i, a in enumerate(atoms)]


def training_member(i: int, n_atoms: int = 100, seed0: int = 300000) -> Config:
    """Training systems of the learned preconditioner: the density, radius and spacing of
    `prec` (h = 0.3125 bohr) in a smaller cell, grid edge rounded to a multiple of 4."""
    h = 0.3125
    L = 40.0 * (n_atoms / 200.0) ** (1.0 / 3.0)
    N = int(4 * round(L / (4 * h)))
    return Config(name=f"train{i}", n_atoms=n_atoms, L=N * h, N=N, r_c=7.0,
                  n_occ=_occ(n_atoms), n_vir=2 * _occ(n_atoms), R_K=None, R_M=None,
                  n_states=8, seed=seed0 + i)


def scale(n_atoms: int = 2000) -> Config:
    """Linear-scaling size (Sec. IV.C): density kernels truncated at 15 bohr and re-purified,
    response kernels truncated to the same 15-bohr pattern M, energy zero mid-gap, atoms
    numbered along a space-filling curve."""
    table = {500: (50.0, 160), 1000: (62.5, 200), 2000: (80.0, 256)}
    L, N = table[n_atoms]
    return Config(name=f"scale{n_atoms}", n_atoms=n_atoms, L=L, N=N, r_c=6.0,
                  n_occ=_occ(n_atoms), n_vir=2 * _occ(n_atoms), R_K=15.0, R_M=15.0,
                  n_states=4, seed=4000 + n_atoms, mask_p=True, energy_zero="midgap",
                  order="morton")


def scale500(seed: int | None = None) -> Config:
    return scale(500)


def scale1000(seed: int | None = None) -> Config:
    return scale(1000)


def scale2000(seed: int | None = None) -> Config:
    return scale(2000)


def small_kt(seed: int = 21) -> Config:
    """The linear-scaling mode at parity size: 32 atoms at the density of `scale` in a
    21.875 bohr cube, 70^3 (radix 2, 5, 7; ragged tiles), density kernels truncated at
    7.5 bohr and re-purified, response kernels truncated to M (7.5 bohr), mid-gap zero."""
    return Config(name="small_kt", n_atoms=32, L=21.875, N=70, r_c=4.5, n_occ=_occ(32),
                  n_vir=2 * _occ(32), R_K=7.5, R_M=7.5, n_states=4, seed=seed, mask_p=True,
                  energy_zero="midgap", order="morton")


def small_kt_exactp(seed: int = 21) -> Config:
    """`small_kt` with exact response kernels (P = K^c S^u L S^o K^v on the blocks it
    reaches): truncated density kernels in the variational form of Eq. auxiliary."""
    c = small_kt(seed)
    d = dict(c.__dict__)
    d.update(name="small_kt_exactp", mask_p=False)
    return Config(**d)


# ---- small cases for parity tests ----------------------------------------------------

def small_dense(seed: int = 11) -> Config:
    """6 atoms in a 14 bohr cube, 40^3 (radix 2 and 5 FFT), dense."""
    return Config(name="small_dense", n_atoms=6, L=14.0, N=40, r_c=4.5, n_occ=4, n_vir=8,
                  R_K=None, R_M=None, n_states=3, seed=seed)


def small_trunc(seed: int = 12) -> Config:
    """24 atoms in a 22 bohr cube, 70^3 (radix 2, 5, 7; ragged 4^3 tiles), M at 6 bohr."""
    return Config(name="small_trunc", n_atoms=24, L=22.0, N=70, r_c=4.5, n_occ=16,
                  n_vir=32, R_K=None, R_M=6.0, n_states=4, seed=seed)


def small_odd(seed: int = 13) -> Config:
    """8 atoms in a 15 bohr cube, 45^3 (radix 3 and 5, ragged tiles), truncated M only."""
    return Config(name="small_odd", n_atoms=8, L=15.0, N=45, r_c=4.0, n_occ=5, n_vir=10,
                  R_K=None, R_M=8.0, n_states=2, seed=seed)


def small_crowded(seed: int = 17) -> Config:
    """24 atoms in a 12 bohr cube, 48^3 (radix 2 and 3), dense: 6 to 18 o-atoms per grid
    tile (the other small systems stay below 10), for the per-tile staging of the grid
    kernels."""
    return Config(name="small_crowded", n_atoms=24, L=12.0, N=48, r_c=4.0, n_occ=16,
                  n_vir=32, R_K=None, R_M=None, n_states=5, seed=seed)


def prec_joint(seed: int = 1000) -> Config:
    """`prec` in the joint unoccupied representation (u-set = o- and u-functions of every
    atom, 5 per atom; K^c the complement projector of Eq. proj)."""
    c = prec(seed)
    d = dict(c.__dict__)
    d.update(name="prec_joint", joint=True)
    return Config(**d)


def small_joint(seed: int = 13) -> Config:
    """`small_dense` geometry in the joint unoccupied representation, u-functions 0.4 x as
    wide as the o-functions: with this seed the complement's lowest level (0.335 Ha) lies
    above the HOMO (0.243 Ha), so A - B is positive definite and the solve is defined."""
    c = small_dense(seed)
    d = dict(c.__dict__)
    d.update(name="small_joint", joint=True, u_width_scale=0.4)
    return Config(**d)


def separated(seed: int = 3, N: int = 64) -> Config:
    """4 atoms with narrow function boxes (r_c 1.5 bohr) in a 20 bohr cell: no two atoms
    overlap, every matrix is block-diagonal, and the 2 occupied states sit on two of the
    atoms, so K^v (and K^c) have vanishing diagonal blocks."""
    return Config(name="separated", n_atoms=4, L=20.0, N=N, r_c=1.5, n_occ=2, n_vir=4,
                  R_K=None, R_M=None, n_states=1, seed=seed)


def wide_grid(seed: int = 3) -> Config:
    """`separated` on a 320^3 grid (radix 8, 8, 5): an axis too long for the in-place FFT
    passes, so the transforms take the two-buffer form with line buffers of 2 x 16 x 321
    complex values per workgroup."""
    c = separated(seed, N=320)
    d = dict(c.__dict__)
    d.update(name="wide_grid")
    return Config(**d)


BY_NAME = {"tiny": tiny, "prec": prec, "small_dense": small_dense, "small_kt": small_kt,
           "small_kt_exactp": small_kt_exactp, "scale500": scale500, "scale1000": scale1000,
           "scale2000": scale2000,
           "small_trunc": small_trunc, "small_odd": small_odd, "small_crowded": small_crowded,
           "prec_joint": prec_joint, "small_joint": small_joint, "separated": separated,
           "wide_grid": wide_grid}
