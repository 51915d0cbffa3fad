"""Seeded synthetic systems for linear-response TDDFT in two localised function sets.

This module only builds *inputs*: atoms in a periodic cube, grid-sampled localised
functions for the occupied set (o-set) and the unoccupied set (u-set), their overlap and
Hamiltonian matrices, the valence and conduction density kernels K^v and K^c, the block
sparsity pattern M of the response kernels and a random initial guess.  It performs none
of the response-operator arithmetic (no response density, no potential, no Casida
matrix).  Both the FP64 oracle and the GPU library consume what it writes.

Paper correspondence (arXiv:1507.08157):
  * o-set {phi_beta} spans the occupied space, K^v is its density kernel (Sec. II.C,
    density-matrix expansion of rho^{v}).
  * u-set {chi_alpha} spans the low unoccupied space, K^c is its kernel (Sec. II.C).
  * Density kernels truncated at a radius, as in Sec. IV.C; idempotency is restored
    approximately by masked McWeeny steps (the paper relies on near-idempotent kernels,
    Sec. III.A, discussion after Eq. auxiliary).

Recipe (the paper's molecules, pseudopotentials and optimised NGWFs are not available,
so every system is synthetic):
  * atoms uniform in [0, L)^3, minimum-image separation >= min_sep (rejection), numbered
    in placement order or along a Z-order curve;
  * each atom carries n_o o-functions and n_u u-functions; each function is
    exp(-r^2 / (2 w^2)) times a random polynomial of degree <= 2 in (r - R) (10 monomials,
    N(0,1) coefficients), w ~ U[w_lo, w_hi], cut to zero beyond r_c, normalised so that
    h^3 sum f^2 = 1;
  * Hamiltonian: 2nd-order 7-point finite-difference kinetic energy plus Gaussian wells
    -d exp(-r^2 / 2 sigma^2) (d ~ U[1,3] Ha, sigma = 1 bohr, each well cut at 6 sigma);
  * S_ab = h^3 sum f_a f_b, H_ab = h^3 sum f_a (H f_b), both symmetrised;
  * K^v = sum_v b_v b_v^T over the n_occ lowest generalised eigenvectors of (H^o, S^o);
    K^c = sum_c a_c a_c^T over the n_vir lowest eigenvectors of (H^u, S^u) whose
    eigenvalue exceeds eps_HOMO + gap_margin (the literal "next" states can lie below the
    occupied ones in a second, independent basis, which would make A-B indefinite);
  * optional energy zero mid-gap: H <- H - mu S with mu halfway between the highest
    occupied o-set level and the lowest level K^c keeps;
  * optional truncation of K at radius R_K followed by masked McWeeny steps
    K <- mask(3 K S K - 2 K S K S K);
  * pattern M: (u-atom I, o-atom J) blocks with minimum-image distance <= R_M (dense if
    R_M is None); in the linear-scaling mode (mask_p) the response kernels are truncated
    to M as well (Sec. IV.C), otherwise they live on the blocks K^c S^u L S^o K^v reaches;
  * initial guess L0 ~ N(0,1) on M for each state.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg


@dataclass
class Config:
    name: str
    n_atoms: int
    L: float
    N: int
    r_c: float
    n_occ: int
    n_vir: int
    R_K: float | None
    R_M: float | None
    n_states: int
    seed: int
    n_o: int = 2
    n_u: int = 3
    w_lo: float = 1.0
    w_hi: float = 1.6
    sigma_well: float = 1.0
    depth_lo: float = 1.0
    depth_hi: float = 3.0
    well_cut_sigmas: float = 6.0
    min_sep: float = 2.5
    gap_margin: float = 0.05
    mcweeny_steps: int = 2
    # joint unoccupied representation (Eq. proj): the u-set is every function of an atom,
    # o-functions first (n_o + n_u per atom), and K^c is the complement projector
    # S^-1 - S^-1 S^{.o} K^v S^{o.} S^-1 of the occupied space within that set
    joint: bool = False
    # width factor of the u-functions (the o-functions keep w_lo..w_hi): narrower
    # u-functions carry more kinetic energy and leave the lowest joint states o-like
    u_width_scale: float = 1.0
    # linear-scaling mode (Sec. IV.C): the response kernels P^p, P^q are truncated to the
    # pattern M as well (P = mask_M(K^c S^u L S^o K^v)); False keeps P exact on the blocks
    # the product reaches
    mask_p: bool = False
    # energy zero of the cell: "none" keeps the finite-difference Hamiltonian as built;
    # "midgap" subtracts mu S with mu halfway between the highest occupied o-set level and
    # the lowest level K^c keeps (the method is invariant under this shift while the
    # response kernels obey the invariance constraint; once they are truncated it fixes
    # the sign of the operator on the non-invariant remainder)
    energy_zero: str = "none"
    # atom numbering: "placement" (the order atoms were drawn in) or "morton" (along a
    # Z-order space-filling curve of their positions, as linear-scaling codes number atoms
    # so that nearby atoms have nearby indices and the sparse matrices cluster near their
    # diagonal)
    order: str = "placement"

    @property
    def h(self) -> float:
        return self.L / self.N


@dataclass
class FunctionSet:
    """Functions of one set, grouped by atom (every function of an atom shares its box)."""
    n_per_atom: int
    origin: np.ndarray          # [n_atoms, 3] (z, y, x) grid index of box corner (wrapped)
    extent: np.ndarray          # [n_atoms, 3] (ez, ey, ex)
    vals: list                  # per atom: array [n_per_atom, ez, ey, ex], x fastest

    @property
    def n_atoms(self) -> int:
        return len(self.vals)

    @property
    def n_fn(self) -> int:
        return self.n_atoms * self.n_per_atom


@dataclass
class System:
    cfg: Config
    pos: np.ndarray             # [n_atoms, 3] (x, y, z) bohr
    occ: FunctionSet
    vir: FunctionSet
    S_o: np.ndarray
    H_o: np.ndarray
    K_v: np.ndarray
    S_u: np.ndarray
    H_u: np.ndarray
    K_c: np.ndarray
    S_uo: np.ndarray            # cross overlap u-set x o-set (tests only)
    M: np.ndarray               # [n_atoms, n_atoms] bool, u-atom rows x o-atom cols
    maskK: np.ndarray           # [n_atoms, n_atoms] bool, truncation pattern of K
    eps_o: np.ndarray           # all generalised eigenvalues of (H^o, S^o)
    eps_u: np.ndarray           # all generalised eigenvalues of (H^u, S^u)
    occ_idx: np.ndarray         # selected o-set states (eigen-index)
    vir_idx: np.ndarray         # selected u-set states
    idem_err: dict = field(default_factory=dict)
    tries: int = 0

    @property
    def N(self) -> int:
        return self.cfg.N

    @property
    def h(self) -> float:
        return self.cfg.h

    def guess(self, n_states: int | None = None) -> np.ndarray:
        """Initial auxiliary matrices L0 ~ N(0,1) on M, [n_states, n_u_fn, n_o_fn] FP64."""
        n = self.cfg.n_states if n_states is None else n_states
        rng = np.random.default_rng(np.random.SeedSequence(self.cfg.seed).spawn(4)[3])
        g = rng.standard_normal((n, self.vir.n_fn, self.occ.n_fn))
        return g * self.fn_mask()[None]

    def fn_mask(self) -> np.ndarray:
        """Function-level mask of M, [n_u_fn, n_o_fn]."""
        return np.kron(self.M, np.ones((self.vir.n_per_atom, self.occ.n_per_atom))).astype(bool)


def _min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def atom_distances(pos: np.ndarray, L: float) -> np.ndarray:
    d = _min_image(pos[:, None, :] - pos[None, :, :], L)
    return np.sqrt((d * d).sum(-1))


def _place_atoms(cfg: Config, rng: np.random.Generator) -> np.ndarray:
    pos = np.zeros((cfg.n_atoms, 3))
    n = 0
    attempts = 0
    while n < cfg.n_atoms:
        attempts += 1
        if attempts > 1000 * cfg.n_atoms:
            raise RuntimeError("cannot place atoms with the requested minimum separation")
        p = rng.uniform(0.0, cfg.L, 3)
        if n:
            d = _min_image(pos[:n] - p, cfg.L)
            if np.min((d * d).sum(-1)) < cfg.min_sep ** 2:
                continue
        pos[n] = p
        n += 1
    return pos


def _morton_order(pos: np.ndarray, L: float) -> np.ndarray:
    """Permutation that sorts positions along a Z-order curve (10 bits per axis)."""
    q = np.clip((pos / L * 1024).astype(np.int64), 0, 1023)
    code = np.zeros(len(pos), dtype=np.int64)
    for b in range(10):
        for d in range(3):
            code |= ((q[:, d] >> b) & 1) << (3 * b + d)
    return np.argsort(code, kind="stable")


def _box(center: float, radius: float, h: float, N: int):
    """Grid box along one axis covering [center - radius, center + radius] plus one zero
    layer on each side (so finite differences of the function vanish outside the box)."""
    lo = int(np.ceil((center - radius) / h)) - 1
    hi = int(np.floor((center + radius) / h)) + 1
    ext = hi - lo + 1
    if ext > N:
        raise ValueError("function box larger than the cell")
    return lo, ext


_MONOMIALS = ((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2),
              (1, 1, 0), (1, 0, 1), (0, 1, 1))


def _atom_functions(cfg: Config, R: np.ndarray, n_fn: int, rng: np.random.Generator):
    h, N = cfg.h, cfg.N
    lo = np.zeros(3, dtype=np.int64)
    ext = np.zeros(3, dtype=np.int64)
    for d in range(3):           # d indexes x, y, z
        lo[d], ext[d] = _box(R[d], cfg.r_c, h, N)
    x = (lo[0] + np.arange(ext[0])) * h - R[0]
    y = (lo[1] + np.arange(ext[1])) * h - R[1]
    z = (lo[2] + np.arange(ext[2])) * h - R[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    r2 = X * X + Y * Y + Z * Z
    inside = r2 <= cfg.r_c * cfg.r_c
    widths = np.zeros(n_fn)
    coefs = np.zeros((n_fn, len(_MONOMIALS)))
    for k in range(n_fn):
        widths[k] = rng.uniform(cfg.w_lo, cfg.w_hi) * (cfg.u_width_scale if k >= cfg.n_o else 1.0)
        coefs[k] = rng.standard_normal(len(_MONOMIALS))
    mono = np.stack([X ** px * Y ** py * Z ** pz for (px, py, pz) in _MONOMIALS])
    poly = np.tensordot(coefs, mono, axes=(1, 0))            # [n_fn, ez, ey, ex]
    vals = np.exp(-r2[None] / (2.0 * widths[:, None, None, None] ** 2)) * poly
    vals[:, ~inside] = 0.0
    vals /= np.sqrt(h ** 3 * np.sum(vals * vals, axis=(1, 2, 3)))[:, None, None, None]
    origin = np.array([lo[2] % N, lo[1] % N, lo[0] % N])      # (z, y, x)
    extent = np.array([ext[2], ext[1], ext[0]])
    return origin, extent, vals


def _well_potential(cfg: Config, pos: np.ndarray, depth: np.ndarray) -> np.ndarray:
    h, N = cfg.h, cfg.N
    V = np.zeros((N, N, N))
    rcut = cfg.well_cut_sigmas * cfg.sigma_well
    for I in range(cfg.n_atoms):
        R = pos[I]
        idx = []
        disp = []
        for d in range(3):
            lo = int(np.ceil((R[d] - rcut) / h))
            hi = int(np.floor((R[d] + rcut) / h))
            g = np.arange(lo, hi + 1)
            if len(g) > N:
                g = g[:N]
            idx.append(g % N)
            disp.append(g * h - R[d])
        Z, Y, X = np.meshgrid(disp[2], disp[1], disp[0], indexing="ij")
        r2 = X * X + Y * Y + Z * Z
        v = -depth[I] * np.exp(-r2 / (2.0 * cfg.sigma_well ** 2))
        v[r2 > rcut * rcut] = 0.0
        V[np.ix_(idx[2], idx[1], idx[0])] += v
    return V


def _laplacian_box(f: np.ndarray, h: float) -> np.ndarray:
    """7-point Laplacian on boxes [n, ez, ey, ex]; values beyond the box are zero."""
    out = -6.0 * f
    out[:, 1:] += f[:, :-1]
    out[:, :-1] += f[:, 1:]
    out[:, :, 1:] += f[:, :, :-1]
    out[:, :, :-1] += f[:, :, 1:]
    out[:, :, :, 1:] += f[:, :, :, :-1]
    out[:, :, :, :-1] += f[:, :, :, 1:]
    return out / (h * h)


def _axis_overlap(oa: int, ea: int, ob: int, eb: int, N: int):
    i = np.arange(ea)
    rel = (oa + i - ob) % N
    ok = rel < eb
    return i[ok], rel[ok]


def _as_index(ix):
    """A contiguous index run as a slice (a view instead of a copy), else the array."""
    if len(ix) and ix[-1] - ix[0] + 1 == len(ix):
        return slice(int(ix[0]), int(ix[-1]) + 1)
    return ix


def _box_overlap(oa, ea, ob, eb, N):
    res = []
    for d in range(3):
        ia, ib = _axis_overlap(int(oa[d]), int(ea[d]), int(ob[d]), int(eb[d]), N)
        if len(ia) == 0:
            return None
        res.append((_as_index(ia), _as_index(ib)))
    return res


def _sub(v, z, y, x):
    """v[:, z, y, x] for per-axis slices or index arrays, flattened to [n, points]."""
    v = v[:, z]
    v = v[:, :, y]
    v = v[:, :, :, x]
    return v.reshape(v.shape[0], -1)


def _mask_dense(A: np.ndarray, atom_mask: np.ndarray, br: int, bc: int) -> np.ndarray:
    return A * np.kron(atom_mask, np.ones((br, bc)))


def _mcweeny(K, S, atom_mask, b, steps):
    for _ in range(steps):
        KS = K @ S
        KSK = KS @ K
        K = _mask_dense(3.0 * KSK - 2.0 * KS @ KSK, atom_mask, b, b)
        K = 0.5 * (K + K.T)
    return K


def build_system(cfg: Config, max_tries: int = 8, progress=None) -> System:
    """Build a system; redraw with seed+1 if too few u-states lie above the threshold.
    progress(msg), if given, is called as the stages of a build complete."""
    last = None
    for t in range(max_tries):
        try:
            sysm = _build(cfg, cfg.seed + t, progress)
            sysm.tries = t
            return sysm
        except _NotEnoughStates as e:
            last = e
    raise RuntimeError(f"no valid system after {max_tries} seeds: {last}")


class _NotEnoughStates(Exception):
    pass


def _build(cfg: Config, seed: int, progress=None) -> System:
    def report(msg):
        if progress is not None:
            progress(f"{cfg.name}: {msg}")
    ss = np.random.SeedSequence(seed).spawn(4)
    rng_geo, rng_fn, rng_well = (np.random.default_rng(s) for s in ss[:3])
    h, N = cfg.h, cfg.N
    nA = cfg.n_atoms
    pos = _place_atoms(cfg, rng_geo)
    if cfg.order == "morton":
        pos = pos[_morton_order(pos, cfg.L)]
    elif cfg.order != "placement":
        raise ValueError(f"unknown atom order {cfg.order!r}")
    nf = cfg.n_o + cfg.n_u
    origins = np.zeros((nA, 3), dtype=np.int64)
    extents = np.zeros((nA, 3), dtype=np.int64)
    allv = []
    for I in range(nA):
        o, e, v = _atom_functions(cfg, pos[I], nf, rng_fn)
        origins[I], extents[I] = o, e
        allv.append(v)
    depth = rng_well.uniform(cfg.depth_lo, cfg.depth_hi, nA)
    Vw = _well_potential(cfg, pos, depth)
    report(f"{nA} atoms, functions and wells on the {N}^3 grid")

    # H f on each atom box
    Hv = []
    for I in range(nA):
        o, e = origins[I], extents[I]
        idx = [(o[d] + np.arange(e[d])) % N for d in range(3)]
        vloc = Vw[np.ix_(idx[0], idx[1], idx[2])]
        Hv.append(-0.5 * _laplacian_box(allv[I], h) + vloc[None] * allv[I])

    # pairwise integrals over box intersections
    dist = atom_distances(pos, cfg.L)
    reach = 2.0 * cfg.r_c + 4.0 * h
    S = np.zeros((nA * nf, nA * nf))
    H = np.zeros((nA * nf, nA * nf))
    h3 = h ** 3
    quarter = max(1, nA // 4)
    for I in range(nA):
        if I and I % quarter == 0:
            report(f"overlap and Hamiltonian integrals of {I} of {nA} atoms")
        for J in np.nonzero(dist[I] <= reach)[0]:
            if J < I:
                continue
            ov = _box_overlap(origins[I], extents[I], origins[J], extents[J], N)
            if ov is None:
                continue
            (za, zb), (ya, yb), (xa, xb) = ov
            FI = _sub(allv[I], za, ya, xa)
            FJ = _sub(allv[J], zb, yb, xb)
            GJ = _sub(Hv[J], zb, yb, xb)
            GI = _sub(Hv[I], za, ya, xa)
            sIJ = h3 * FI @ FJ.T
            hIJ = 0.5 * h3 * (FI @ GJ.T + GI @ FJ.T)
            S[I * nf:(I + 1) * nf, J * nf:(J + 1) * nf] = sIJ
            H[I * nf:(I + 1) * nf, J * nf:(J + 1) * nf] = hIJ
            if J != I:
                S[J * nf:(J + 1) * nf, I * nf:(I + 1) * nf] = sIJ.T
                H[J * nf:(J + 1) * nf, I * nf:(I + 1) * nf] = hIJ.T
    S = 0.5 * (S + S.T)
    H = 0.5 * (H + H.T)
    o_sel = (np.arange(nA)[:, None] * nf + np.arange(cfg.n_o)[None, :]).ravel()
    u_sel = (np.arange(nA)[:, None] * nf + cfg.n_o + np.arange(cfg.n_u)[None, :]).ravel()
    S_o, H_o = S[np.ix_(o_sel, o_sel)], H[np.ix_(o_sel, o_sel)]
    S_u, H_u = S[np.ix_(u_sel, u_sel)], H[np.ix_(u_sel, u_sel)]
    S_uo = S[np.ix_(u_sel, o_sel)]

    report("integrals done")
    eps_o, B = scipy.linalg.eigh(H_o, S_o)
    occ_idx = np.arange(cfg.n_occ)
    homo = eps_o[cfg.n_occ - 1]
    K_v = B[:, occ_idx] @ B[:, occ_idx].T
    if cfg.joint:
        if cfg.R_K is not None:
            raise ValueError("joint representation: untruncated kernels only")
        # the u-set is the whole per-atom function list; S^-1 S^{.o} selects the o-positions
        S_u, H_u, S_uo = S, H, S[:, o_sel]
        K_c = np.linalg.inv(S)
        K_c[np.ix_(o_sel, o_sel)] -= K_v
        # levels of the complement: H projected onto range(K^c) in an S-orthonormal basis.
        # With independently drawn o- and u-functions these reach below the HOMO (mixing in
        # the u-functions lowers the joint spectrum), so A - B is not positive definite and
        # only the operator application is meaningful on such systems
        eps_u = complement_levels(H_u, S_u, K_c)
        vir_idx = np.arange(len(eps_u))
    else:
        eps_u, A = scipy.linalg.eigh(H_u, S_u)
        above = np.nonzero(eps_u > homo + cfg.gap_margin)[0]
        if len(above) < cfg.n_vir:
            raise _NotEnoughStates(f"seed {seed}: {len(above)} u-states above threshold")
        vir_idx = above[:cfg.n_vir]
        K_c = A[:, vir_idx] @ A[:, vir_idx].T

    if cfg.energy_zero == "midgap":
        if cfg.joint:
            raise ValueError("joint representation: energy zero as built only")
        mu = 0.5 * (homo + eps_u[vir_idx[0]])
        H_o = H_o - mu * S_o
        H_u = H_u - mu * S_u
        eps_o = eps_o - mu
        eps_u = eps_u - mu
    elif cfg.energy_zero != "none":
        raise ValueError(f"unknown energy zero {cfg.energy_zero!r}")

    if cfg.R_K is None:
        maskK = np.ones((nA, nA), dtype=bool)
    else:
        maskK = dist <= cfg.R_K
    idem = {}
    if cfg.R_K is not None:
        K_v = _mcweeny(_mask_dense(K_v, maskK, cfg.n_o, cfg.n_o), S_o, maskK, cfg.n_o,
                       cfg.mcweeny_steps)
        K_c = _mcweeny(_mask_dense(K_c, maskK, cfg.n_u, cfg.n_u), S_u, maskK, cfg.n_u,
                       cfg.mcweeny_steps)
    for name, K, Sx in (("K_v", K_v, S_o), ("K_c", K_c, S_u)):
        idem[name] = float(np.linalg.norm(K @ Sx @ K - K) / np.linalg.norm(K))
    K_v = 0.5 * (K_v + K_v.T)
    K_c = 0.5 * (K_c + K_c.T)

    if cfg.R_M is None:
        M = np.ones((nA, nA), dtype=bool)
    else:
        M = dist <= cfg.R_M

    occ = FunctionSet(cfg.n_o, origins.copy(), extents.copy(),
                      [v[:cfg.n_o].copy() for v in allv])
    if cfg.joint:
        vir = FunctionSet(nf, origins.copy(), extents.copy(), [v.copy() for v in allv])
    else:
        vir = FunctionSet(cfg.n_u, origins.copy(), extents.copy(),
                          [v[cfg.n_o:].copy() for v in allv])
    cfg_used = cfg if seed == cfg.seed else _with_seed(cfg, seed)
    return System(cfg=cfg_used, pos=pos, occ=occ, vir=vir, S_o=S_o, H_o=H_o, K_v=K_v,
                  S_u=S_u, H_u=H_u, K_c=K_c, S_uo=S_uo, M=M, maskK=maskK, eps_o=eps_o,
                  eps_u=eps_u, occ_idx=occ_idx, vir_idx=vir_idx, idem_err=idem)


def complement_levels(H: np.ndarray, S: np.ndarray, K: np.ndarray) -> np.ndarray:
    """Eigenvalues of H restricted to range(K) for an S-idempotent K (K S K = K): with
    C an S-orthonormal basis of that range, the eigenvalues of C^T H C, ascending."""
    w, V = scipy.linalg.eigh(S @ K @ S, S)
    C = V[:, w > 0.5]
    return np.linalg.eigvalsh(0.5 * (C.T @ H @ C + (C.T @ H @ C).T))


def _with_seed(cfg: Config, seed: int) -> Config:
    d = dict(cfg.__dict__)
    d["seed"] = seed
    return Config(**d)
