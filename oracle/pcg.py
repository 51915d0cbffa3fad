"""Preconditioned conjugate-gradient minimisation of the multi-state Tsiper functional,
FP64 (arXiv:1507.08157, Secs. III.A-III.C).

The paper's own listings (its supplementary algorithms 1 and 2) are not available; the
steps below follow the equations of the main text, and every choice the text leaves open
is one of the documented readings:

  * trial vectors P_i = (p_i, q_i) on the response pattern Mp, Tsiper orthonormality
    B_ij = 1/2 (<p_i, q_j> + <p_j, q_i>) = delta_ij (Eq. ortho), sign rule
    q_i -> -q_i when <p_i, q_i> < 0 before orthonormalising (Sec. III.C), Gram-Schmidt in
    index order;
  * N_ij = 1/2 (<p_j, f^p_i> + <q_j, f^q_i>), symmetrised; omega = eig(N B^-1) (the
    subspace matrix Q of Sec. III.C);
  * gradient g_i = F_i - sum_j N_ij (q_j, p_j) (Sec. III.C, multi-state gradient; with
    B_jj = 1 its coefficient carries the factor 1/2 of the functional);
  * the optimisation variable is the auxiliary matrix L on the truncation pattern M; trial
    vectors are P = Pi(L) = K^c S^u L S^o K^v, exact (Sec. III.A, Eq. auxiliary), so P never
    leaves the invariant space and P itself is never re-projected;
  * learned (optional): G = c * g with a per-block elementwise scaling c predicted from
    two-atom features (oracle/learned.py), used when it is a descent direction for every
    state, else the CG preconditioner below; once the largest gradient norm has not halved
    over `learned_window` iterations with the learned scaling on, the rest of the solve
    uses the CG preconditioner (one more fallback);
  * M complete (no truncation): Eq. precond, K^c H^u G - G H^o K^v = g, is solved by CG in
    the S metric to a relative residual eps_tol (Sec. III.B) and the direction is
    d = -Pi(G) + beta d_prev (Pi(G) = G for invariant G); none -> G = g;
  * M truncated: the gradient with respect to L is r = mask_M(Pi^T(mask_Mp(S^u g S^o)))
    (chain rule through P = Pi(L), whose entries lie on Mp) and Eq. precond is expressed on
    L, H_L(X) = mask_M(Pi^T mask_Mp(S^u T(Pi X) S^o));
    H_L z = r is solved by CG (Euclidean inner product on M) to relative residual eps_tol
    and d = -Pi(z) + beta d_prev, a descent direction by construction; none -> z = r;
  * Polak-Ribiere(+) conjugation, common step lambda for all states, exact line search on
    Tr[N(lambda) B(lambda)^-1] (the sum functional, Eq. Tsiper_multiple, invariant under
    re-orthonormalisation), F carried by linearity F += lambda F(d) and refreshed every
    `refresh` iterations;
  * stop when max |d omega| < tol_omega and max ||g_i|| < sqrt(tol_omega); final omega from
    the subspace diagonalisation, vectors rotated to its eigenvectors.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.optimize


@dataclass
class Options:
    n_states: int
    precond: str = "cg"          # "cg" (Eq. precond solved by CG), "none" or "learned"
    scaling: np.ndarray | None = None   # learned: elementwise gradient scaling [n_u, n_o]
    eps_tol: float = 1e-4
    eps_loose: float = 0.0       # > eps_tol: inner tolerance eps_loose |g|/|g_0| in [eps_tol, eps_loose]
    tol_omega: float = 1e-7
    max_iter: int = 300
    max_inner: int = 50
    refresh: int = 10
    restart: int = 20
    learned_window: int = 10


@dataclass
class Result:
    omega: np.ndarray
    P: np.ndarray                # [2, n, nu, no]: p and q
    F: np.ndarray
    iterations: int
    converged: bool
    history: list = field(default_factory=list)
    inner_iters: list = field(default_factory=list)
    fallbacks: int = 0


class Solver:
    def __init__(self, op, opts: Options):
        self.op = op
        self.o = opts
        self.complete = bool(np.all(op.mask_L == 1))
        self.fallbacks = 0
        self.eps = opts.eps_tol
        self.learned_on = opts.precond == "learned"
        self.learned_gmax = []

    # -- metric helpers -------------------------------------------------------------------
    def cov(self, X):
        """S^u X S^o for a stack [k, nu, no] (then <X, Y> = sum X * cov(Y))."""
        return self.op.Su @ X @ self.op.So

    @staticmethod
    def gram(X, Yc):
        """[k1, k2] matrix of sum(X_a * Yc_b)."""
        return np.einsum("aij,bij->ab", X, Yc)

    # -- operator pieces ------------------------------------------------------------------
    def apply(self, P):
        fp, fq = self.op.apply(P[0], P[1])
        return np.stack([fp, fq])

    def project(self, X):
        return np.stack([self.op.project(x) for x in X])

    def pi_t(self, Y):
        """Pi^T(Y) = mask_M(S^u K^c Y K^v S^o): the adjoint of the projection, onto M."""
        return self.op.mask_L[None] * (self.op.KcSu.T @ Y @ self.op.SoKv.T)

    def grad_L(self, g):
        """Gradient with respect to L of the functional whose P-gradient is g: P has entries
        only on its pattern Mp, so the covariant gradient counts there only
        (mask_M(Pi^T(mask_Mp(S^u g S^o))); the inner mask changes nothing when Mp is the
        pattern the exact product reaches, and matters when P is truncated to M)."""
        return self.pi_t(self.op.mask[None] * self.cov(g))

    def hess_L(self, X):
        """H_L(X) = mask_M(Pi^T(mask_Mp(S^u T(Pi X) S^o))) for X on M."""
        P = self.project(X)
        return self.pi_t(self.op.mask[None] * self.cov(np.stack([self.op.T(x) for x in P])))

    def precondition_p(self, g):
        """Columns of g: [k, nu, no].  CG on T(G) = g in the S metric, G0 = 0, stop at
        ||res|| <= eps_tol ||g||, after max_inner steps or on non-positive curvature."""
        if self.o.precond == "none":
            return g.copy(), 0
        if self.learned_on:
            # learned block scaling, kept only if it is a descent direction for every column
            z = self.o.scaling[None] * g
            if np.all(np.einsum("kij,kij->k", z, self.cov(g)) > 0):
                return z, 0
            self.fallbacks += 1
        G = np.zeros_like(g)
        r = g.copy()
        d = r.copy()
        rr = np.einsum("kij,kij->k", r, self.cov(r))
        rr0 = rr.copy()
        active = rr0 > 0
        steps = np.zeros(len(g), dtype=int)
        for _ in range(self.o.max_inner):
            active &= rr > (self.eps ** 2) * rr0
            if not np.any(active):
                break
            Ld = np.stack([self.op.T(x) for x in d])
            dLd = np.einsum("kij,kij->k", d, self.cov(Ld))
            active &= dLd > 0
            if not np.any(active):
                break
            alpha = np.where(active, rr / np.where(active, dLd, 1.0), 0.0)
            G += alpha[:, None, None] * d
            r -= alpha[:, None, None] * Ld
            rr_new = np.einsum("kij,kij->k", r, self.cov(r))
            beta = np.where(active, rr_new / np.where(rr > 0, rr, 1.0), 0.0)
            d = np.where(active[:, None, None], r + beta[:, None, None] * d, d)
            rr = np.where(active, rr_new, rr)
            steps += active
        G = np.where((steps > 0)[:, None, None], G, g)
        return G, int(steps.max()) if len(steps) else 0

    def precondition(self, r):
        """Columns of r: [k, nu, no] on M.  CG on H_L z = r (Euclidean inner product on
        M), z0 = 0, stop at ||res|| <= eps_tol ||r||, after max_inner steps, or on
        non-positive curvature; none -> z = r."""
        if self.o.precond == "none":
            return r.copy(), 0
        if self.learned_on:
            z = self.op.truncate(self.o.scaling)[None] * r
            if np.all(np.einsum("kij,kij->k", z, r) > 0):
                return z, 0
            self.fallbacks += 1
        z = np.zeros_like(r)
        res = r.copy()
        d = res.copy()
        rr = np.einsum("kij,kij->k", res, res)
        rr0 = rr.copy()
        active = rr0 > 0
        steps = np.zeros(len(r), dtype=int)
        for _ in range(self.o.max_inner):
            active &= rr > (self.eps ** 2) * rr0
            if not np.any(active):
                break
            Hd = self.hess_L(d)
            dHd = np.einsum("kij,kij->k", d, Hd)
            active &= dHd > 0
            if not np.any(active):
                break
            alpha = np.where(active, rr / np.where(active, dHd, 1.0), 0.0)
            z += alpha[:, None, None] * d
            res -= alpha[:, None, None] * Hd
            rr_new = np.einsum("kij,kij->k", res, res)
            beta = np.where(active, rr_new / np.where(rr > 0, rr, 1.0), 0.0)
            d = np.where(active[:, None, None], res + beta[:, None, None] * d, d)
            rr = np.where(active, rr_new, rr)
            steps += active
        z = np.where((steps > 0)[:, None, None], z, r)
        return z, int(steps.max()) if len(steps) else 0

    # -- subspace algebra ------------------------------------------------------------------
    def pq_gram(self, P):
        """C_ij = <p_i, q_j>."""
        return self.gram(P[0], self.cov(P[1]))

    def n_matrix(self, P, F):
        """N_ij = 1/2 (<p_j, f^p_i> + <q_j, f^q_i>), symmetrised."""
        Nm = 0.5 * (self.gram(F[0], self.cov(P[0])) + self.gram(F[1], self.cov(P[1])))
        return 0.5 * (Nm + Nm.T)

    @staticmethod
    def orthonormalise(C):
        """Transforms (Tp, Tq) with p' = Tp p, q' = Tq q such that
        1/2 (C'_ij + C'_ji) = delta_ij for C' = Tp C Tq^T.  Sign rule first (q_i -> -q_i
        when C_ii < 0), then Gram-Schmidt in index order."""
        n = C.shape[0]
        Tp = np.eye(n)
        Tq = np.eye(n)
        for i in range(n):
            if C[i, i] < 0:
                Tq[i] = -Tq[i]
        for i in range(n):
            for j in range(i):
                Cp = Tp @ C @ Tq.T
                c = 0.5 * (Cp[i, j] + Cp[j, i])
                Tp[i] -= c * Tp[j]
                Tq[i] -= c * Tq[j]
            Cp = Tp @ C @ Tq.T
            b = Cp[i, i]
            if not b > 0:
                raise FloatingPointError("Tsiper metric not positive in Gram-Schmidt")
            Tp[i] /= np.sqrt(b)
            Tq[i] /= np.sqrt(b)
        return Tp, Tq

    @staticmethod
    def transform(X, Tp, Tq):
        return np.stack([np.einsum("ij,jkl->ikl", Tp, X[0]),
                         np.einsum("ij,jkl->ikl", Tq, X[1])])

    def combined_dot(self, X, Y):
        """sum_i (<x^p_i, y^p_i> + <x^q_i, y^q_i>)."""
        return float(np.sum(X[0] * self.cov(Y[0])) + np.sum(X[1] * self.cov(Y[1])))

    # -- line search -------------------------------------------------------------------------
    def line_coeffs(self, P, F, D, FD):
        def nmat(Xa, Fb):
            m = 0.5 * (self.gram(Fb[0], self.cov(Xa[0])) + self.gram(Fb[1], self.cov(Xa[1])))
            return m

        def bmat(Xa, Xb):
            m = self.gram(Xa[0], self.cov(Xb[1]))      # <xa^p_i, xb^q_j>
            return m

        N0 = nmat(P, F)
        N1 = nmat(D, F) + nmat(P, FD)
        N2 = nmat(D, FD)
        sym = lambda m: 0.5 * (m + m.T)  # noqa: E731
        C0 = bmat(P, P)
        C1 = bmat(P, D) + bmat(D, P)
        C2 = bmat(D, D)
        return [sym(N0), sym(N1), sym(N2)], [sym(C0), sym(C1), sym(C2)]

    @staticmethod
    def phi(lam, Nc, Bc):
        Nl = Nc[0] + lam * Nc[1] + lam * lam * Nc[2]
        Bl = Bc[0] + lam * Bc[1] + lam * lam * Bc[2]
        try:
            L = np.linalg.cholesky(Bl)
        except np.linalg.LinAlgError:
            return np.inf
        Li = np.linalg.inv(L)
        return float(np.trace(Li @ Nl @ Li.T))

    def line_search(self, Nc, Bc, scale):
        """argmin over lambda > 0 of Tr[N(lambda) B(lambda)^-1] inside the region where
        B(lambda) stays positive definite: coarse log scan, then bounded Brent."""
        lams = scale * np.geomspace(1e-8, 1e4, 241)
        vals = np.array([self.phi(l, Nc, Bc) for l in lams])
        first_bad = np.nonzero(~np.isfinite(vals))[0]
        end = first_bad[0] if len(first_bad) else len(vals)
        if end == 0:
            return 0.0
        k = int(np.argmin(vals[:end]))
        if not vals[k] < self.phi(0.0, Nc, Bc):
            return 0.0
        lo = lams[k - 1] if k > 0 else 0.0
        hi = lams[k + 1] if k + 1 < end else lams[k]
        if hi <= lo:
            return lams[k]
        res = scipy.optimize.minimize_scalar(lambda l: self.phi(l, Nc, Bc), bounds=(lo, hi),
                                             method="bounded",
                                             options={"xatol": 1e-14 * max(hi, 1e-300)})
        lam = float(res.x)
        return lam if self.phi(lam, Nc, Bc) <= vals[k] else float(lams[k])

    # -- driver --------------------------------------------------------------------------------
    def solve(self, L0: np.ndarray) -> Result:
        n = self.o.n_states
        p0 = self.project(np.asarray(L0, dtype=np.float64)[:n])
        P = np.stack([p0, p0.copy()])
        Tp, Tq = self.orthonormalise(self.pq_gram(P))
        P = self.transform(P, Tp, Tq)
        F = self.apply(P)
        hist = []
        inner = []
        omega_prev = None
        D = z_prev = r_prev = None
        restart_next = False
        stalls = 0
        converged = False
        it = 0
        for it in range(self.o.max_iter + 1):
            Nm = self.n_matrix(P, F)
            omega = np.sort(np.linalg.eigvalsh(Nm))
            g = F - np.stack([np.einsum("ij,jkl->ikl", Nm, P[1]),
                              np.einsum("ij,jkl->ikl", Nm, P[0])])
            gnorm = np.sqrt(np.einsum("sikl,sikl->i", g, np.stack([self.cov(g[0]),
                                                                   self.cov(g[1])])))
            hist.append(omega.copy())
            # inner tolerance: constant, or loose while the gradient is large (Sec. IV.A)
            if it == 0:
                g0 = float(np.max(gnorm))
            self.eps = self.o.eps_tol
            if self.o.eps_loose > self.o.eps_tol and g0 > 0:
                self.eps = min(self.o.eps_loose,
                               max(self.o.eps_tol, self.o.eps_loose * float(np.max(gnorm)) / g0))
            if omega_prev is not None and np.max(np.abs(omega - omega_prev)) < self.o.tol_omega \
                    and np.max(gnorm) < np.sqrt(self.o.tol_omega):
                converged = True
                break
            if it == self.o.max_iter:
                break
            omega_prev = omega
            if self.learned_on:
                self.learned_gmax.append(float(np.max(gnorm)))
                k = self.o.learned_window
                if len(self.learned_gmax) > k and self.learned_gmax[-1] > 0.5 * self.learned_gmax[-1 - k]:
                    self.learned_on = False
                    self.fallbacks += 1
            shape = g.shape
            if self.complete:
                # r, z in the S metric on the trial-vector space (M complete)
                r = g.reshape(2 * n, *shape[2:])
                z, ninner = self.precondition_p(r)
                Dz = -self.project(z).reshape(shape)
                num_fn = lambda a, b: float(np.sum(a * self.cov(b)))  # noqa: E731
            else:
                r = self.grad_L(g.reshape(2 * n, *shape[2:]))
                z, ninner = self.precondition(r)
                Dz = -self.project(z).reshape(shape)
                num_fn = lambda a, b: float(np.sum(a * b))  # noqa: E731
            inner.append(ninner)
            if D is None or restart_next or it % self.o.restart == 0:
                beta = 0.0
            else:
                num = num_fn(z, r) - num_fn(z, r_prev)
                den = num_fn(z_prev, r_prev)
                beta = max(0.0, num / den) if den > 0 else 0.0
            D = Dz + beta * D if beta > 0 else Dz
            if self.combined_dot(D, g) >= 0:
                D = Dz
            FD = self.apply(D)
            Nc, Bc = self.line_coeffs(P, F, D, FD)
            scale = 1.0 / np.sqrt(max(self.combined_dot(D, D), 1e-300))
            lam = self.line_search(Nc, Bc, scale)
            if lam == 0.0:          # no decrease along d: restart without a step
                D = None
                stalls += 1
                if stalls >= 3:
                    break
                continue
            stalls = 0
            # a step longer than the trial vectors themselves, or one that does not lower
            # the functional, invalidates the conjugation history
            phi0 = self.phi(0.0, Nc, Bc)
            restart_next = (lam * np.sqrt(self.combined_dot(D, D)) > np.sqrt(self.combined_dot(P, P))
                            or not self.phi(lam, Nc, Bc) < phi0 - 1e-14 * abs(phi0))
            P = P + lam * D
            F = F + lam * FD
            if (it + 1) % self.o.refresh == 0:
                F = self.apply(P)
            Tp, Tq = self.orthonormalise(self.pq_gram(P))
            P = self.transform(P, Tp, Tq)
            F = self.transform(F, Tp, Tq)
            D = self.transform(D, Tp, Tq)
            z_prev = self.transform(z.reshape(shape), Tp, Tq).reshape(z.shape)
            r_prev = self.transform(r.reshape(shape), Tp, Tq).reshape(r.shape)
        # subspace diagonalisation (B = I after Gram-Schmidt)
        Nm = self.n_matrix(P, F)
        w, U = np.linalg.eigh(Nm)
        P = self.transform(P, U.T, U.T)
        F = self.transform(F, U.T, U.T)
        return Result(omega=w, P=P, F=F, iterations=it, converged=converged, history=hist,
                      inner_iters=inner, fallbacks=self.fallbacks)
