// Preconditioned conjugate-gradient minimisation of the multi-state Tsiper functional
// (Secs. III.A-III.C).  Trial vectors, operator images and search directions stay on the
// GPU as column sets in the working precision; every trace is reduced in FP64 and the
// small N_omega x N_omega algebra (orthonormalisation, line search, subspace
// diagonalisation) runs in FP64 on the host.
//
// Choices the main text leaves open (its listings are in unavailable supplementary
// material):
//  * Tsiper orthonormality B_ij = 1/2 (<p_i,q_j> + <p_j,q_i>) = delta_ij (Eq. ortho), sign
//    rule q_i -> -q_i when <p_i,q_i> < 0, then Gram-Schmidt in index order;
//  * N_ij = 1/2 (<p_j,f^p_i> + <q_j,f^q_i>) symmetrised, omega = eig(N) when B = I;
//  * gradient g_i = F_i - sum_j N_ij (q_j, p_j) (Sec. III.C);
//  * the optimisation variable is the auxiliary matrix L on the truncation pattern M and the
//    trial vectors are P = K^c S^u L S^o K^v, exact (Eq. auxiliary), so P stays in the
//    invariant space; the gradient with respect to L is r = mask_M(Pi^T(S^u g S^o));
//  * preconditioner: the KS-difference operator of Eq. precond expressed on L,
//    H_L(X) = mask_M(Pi^T(S^u T(Pi X) S^o)), H_L z = r solved by CG to relative residual
//    eps_tol (Sec. III.B); without truncation Pi z solves Eq. precond itself;
//  * direction d = -Pi(z) + beta d_prev (Polak-Ribiere(+) in L), a common step for all states
//    from an exact line search on Tr[N(lambda) B(lambda)^-1]; history dropped after a step
//    longer than the trial vectors or one without decrease; F carried by linearity and
//    refreshed periodically.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <functional>
#include <limits>

#include "handle.h"
#include "learned.h"

namespace tddft {

namespace {

using Mat = std::vector<double>;   // row-major n x n

// ---- small dense FP64 linear algebra ------------------------------------------------------
bool cholesky(const Mat &A, int n, Mat &L) {
  L.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 0.0)) return false;
    L[j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = s / L[j * n + j];
    }
  }
  return true;
}

// cyclic Jacobi eigen-decomposition of a symmetric matrix; V columns are eigenvectors,
// eigenvalues ascending
void sym_eig(const Mat &A0, int n, std::vector<double> &w, Mat &V) {
  Mat A = A0;
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[a * n + a] < A[b * n + b]; });
  w.resize(n);
  Mat V2((size_t)n * n);
  for (int k = 0; k < n; ++k) {
    w[k] = A[idx[k] * n + idx[k]];
    for (int i = 0; i < n; ++i) V2[i * n + k] = V[i * n + idx[k]];
  }
  V = V2;
}

Mat sym(const Mat &A, int n) {
  Mat S(A.size());
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) S[i * n + j] = 0.5 * (A[i * n + j] + A[j * n + i]);
  return S;
}

// Tr[N B^-1] via B = L L^T; +inf when B is not positive definite
double trace_nbinv(const Mat &N, const Mat &B, int n) {
  Mat L;
  if (!cholesky(B, n, L)) return std::numeric_limits<double>::infinity();
  // X = L^-1 N L^-T; trace
  Mat Y((size_t)n * n);  // Y = L^-1 N
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double s = N[i * n + c];
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * Y[k * n + c];
      Y[i * n + c] = s / L[i * n + i];
    }
  double tr = 0.0;  // trace of Y L^-T = sum_i (L^-1 Y^T)_ii
  Mat Z((size_t)n * n);  // Z = L^-1 Y^T
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double s = Y[c * n + i];
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * Z[k * n + c];
      Z[i * n + c] = s / L[i * n + i];
    }
  for (int i = 0; i < n; ++i) tr += Z[i * n + i];
  return tr;
}

// Brent's minimiser on [a, b]: golden-section steps with parabolic interpolation where it
// is safe (R. P. Brent, Algorithms for Minimization without Derivatives, 1973, ch. 5)
double brent_min(const std::function<double(double)> &f, double a, double b, double tol) {
  const double cg = 0.3819660112501051;
  double x = a + cg * (b - a), w = x, v = x;
  double fx = f(x), fw = fx, fv = fx;
  double d = 0.0, e = 0.0;
  for (int it = 0; it < 200; ++it) {
    const double m = 0.5 * (a + b);
    const double t1 = tol * std::fabs(x) + 1e-300, t2 = 2.0 * t1;
    if (std::fabs(x - m) <= t2 - 0.5 * (b - a)) break;
    bool golden = true;
    if (std::fabs(e) > t1) {
      double r = (x - w) * (fx - fv);
      double q = (x - v) * (fx - fw);
      double p = (x - v) * q - (x - w) * r;
      q = 2.0 * (q - r);
      if (q > 0) p = -p;
      q = std::fabs(q);
      const double etmp = e;
      e = d;
      if (std::fabs(p) < std::fabs(0.5 * q * etmp) && p > q * (a - x) && p < q * (b - x)) {
        d = p / q;
        const double u = x + d;
        if (u - a < t2 || b - u < t2) d = (m >= x) ? t1 : -t1;
        golden = false;
      }
    }
    if (golden) {
      e = (x >= m) ? a - x : b - x;
      d = cg * e;
    }
    const double u = std::fabs(d) >= t1 ? x + d : x + (d > 0 ? t1 : -t1);
    const double fu = f(u);
    if (fu <= fx) {
      if (u >= x) a = x; else b = x;
      v = w; fv = fw; w = x; fw = fx; x = u; fx = fu;
    } else {
      if (u < x) a = u; else b = u;
      if (fu <= fw || w == x) { v = w; fv = fw; w = u; fw = fu; }
      else if (fu <= fv || v == x || v == w) { v = u; fv = fu; }
    }
  }
  return x;
}

// Tsiper Gram-Schmidt: transforms with p' = Tp p, q' = Tq q and 1/2 (C' + C'^T) = I
bool orthonormalise(const Mat &C, int n, Mat &Tp, Mat &Tq) {
  Tp.assign((size_t)n * n, 0.0);
  Tq.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    Tp[i * n + i] = 1.0;
    Tq[i * n + i] = C[i * n + i] < 0 ? -1.0 : 1.0;   // sign rule before orthogonalising
  }
  auto cprime = [&](int i, int j) {  // (Tp C Tq^T)_ij
    double s = 0.0;
    for (int a = 0; a < n; ++a) {
      if (Tp[i * n + a] == 0.0) continue;
      for (int b = 0; b < n; ++b) s += Tp[i * n + a] * C[a * n + b] * Tq[j * n + b];
    }
    return s;
  };
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < i; ++j) {
      const double c = 0.5 * (cprime(i, j) + cprime(j, i));
      for (int k = 0; k < n; ++k) {
        Tp[i * n + k] -= c * Tp[j * n + k];
        Tq[i * n + k] -= c * Tq[j * n + k];
      }
    }
    const double b = cprime(i, i);
    if (!(b > 0.0)) return false;
    const double sc = 1.0 / std::sqrt(b);
    for (int k = 0; k < n; ++k) {
      Tp[i * n + k] *= sc;
      Tq[i * n + k] *= sc;
    }
  }
  return true;
}

// ---- device helpers ------------------------------------------------------------------------
// Column sets live on two block patterns: R (trial vectors, operator images, search
// directions) and M (auxiliary matrices L and their gradients).
template <class T>
struct Solver {
  Handle &h;
  int n, nc;                 // states, columns (2n)
  int64_t nR, nM;
  int E;
  hipStream_t s;
  std::vector<T *> sets;
  DevBuf<unsigned char> arena;
  double *hstage = nullptr;  // pinned staging of coefficients
  DevBuf<double> dstage;
  size_t stage_cap = 1 << 17, stage_off = 0;   // doubles
  DevBuf<double> dres;
  size_t res_off = 0;

  Solver(Handle &h_, int n_) : h(h_), n(n_), nc(2 * n_), nR(h_.nR), nM(h_.nM), E(h_.E), s(h_.stream) {
    TD_HIP(hipHostMalloc((void **)&hstage, stage_cap * sizeof(double), hipHostMallocDefault));
    dstage.alloc(stage_cap);
    dres.alloc(1 << 16);
  }
  ~Solver() {
    if (hstage) (void)hipHostFree(hstage);
  }
  size_t elems(int64_t nblk) const { return (size_t)nblk * nc * E; }
  // sets [0, nr) on R, [nr, nr + nm) on M
  void alloc_sets(int nr, int nm) {
    const size_t br = elems(nR) * sizeof(T), bm = elems(nM) * sizeof(T);
    arena.alloc(br * nr + bm * nm);
    sets.resize(nr + nm);
    for (int i = 0; i < nr; ++i) sets[i] = (T *)(arena.p + br * i);
    for (int i = 0; i < nm; ++i) sets[nr + i] = (T *)(arena.p + br * nr + bm * i);
  }
  void sync() {
    TD_HIP(hipStreamSynchronize(s));
    stage_off = 0;
  }
  const double *coef(const Mat &c) {
    if (stage_off + c.size() > stage_cap) sync();
    double *hp = hstage + stage_off;
    std::copy(c.begin(), c.end(), hp);
    double *dp = dstage.p + stage_off;
    TD_HIP(hipMemcpyAsync(dp, hp, c.size() * sizeof(double), hipMemcpyHostToDevice, s));
    stage_off += (c.size() + 31) & ~(size_t)31;
    return dp;
  }
  // Y = sum of up to 3 sources with coefficient matrices [nc][nc] (+ diag(beta) Y when beta
  // is given: host values, one per column), all on nblk blocks.  When every matrix is
  // diagonal the streaming form runs with the coefficients in its kernel arguments (no
  // upload); otherwise the matrices are staged to the device.
  void lc(int64_t nblk, T *Y, const std::vector<double> *beta,
          std::initializer_list<std::pair<const T *, Mat>> src) {
    bool diagonal = nc <= kLcDiagMax && src.size() <= 3;
    for (auto &sr : src)
      for (int i = 0; i < nc && diagonal; ++i)
        for (int j = 0; j < nc; ++j)
          if (i != j && sr.second[(size_t)i * nc + j] != 0.0) {
            diagonal = false;
            break;
          }
    h.prof.begin(ST_LINCOMB, s);
    if (diagonal) {
      LcDiagArgs a{};
      a.Y = Y;
      a.has_beta = beta != nullptr;
      for (int c = 0; c < nc; ++c) a.beta[c] = beta ? (*beta)[c] : 0.0;
      a.nsrc = 0;
      for (auto &sr : src) {
        a.X[a.nsrc] = sr.first;
        for (int c = 0; c < nc; ++c) a.d[a.nsrc][c] = sr.second[(size_t)c * nc + c];
        ++a.nsrc;
      }
      lincomb_diag<T>(nblk, E, nc, a, s);
    } else {
      LcArgs a{};
      a.Y = Y;
      a.ldy = nc;
      a.yc0 = 0;
      a.nout = nc;
      a.beta = beta ? coef(*beta) : nullptr;
      a.nsrc = 0;
      for (auto &sr : src) {
        LcSrc &x = a.src[a.nsrc++];
        x.X = sr.first;
        x.ldx = nc;
        x.xc0 = 0;
        x.nin = nc;
        x.C = coef(sr.second);
      }
      lincomb<T>(nblk, E, a, s);
    }
    h.prof.end(ST_LINCOMB, s);
  }
  Mat eye(double v = 1.0) {
    Mat I((size_t)nc * nc, 0.0);
    for (int i = 0; i < nc; ++i) I[i * nc + i] = v;
    return I;
  }
  Mat diag(const std::vector<double> &d) {
    Mat D((size_t)nc * nc, 0.0);
    for (int i = 0; i < nc; ++i) D[i * nc + i] = d[i];
    return D;
  }
  void copy(int64_t nblk, T *Y, const T *X) { lc(nblk, Y, nullptr, {{X, eye()}}); }
  void axpy(int64_t nblk, T *Y, double a, const T *X) {   // Y += a X
    const std::vector<double> one(nc, 1.0);
    lc(nblk, Y, &one, {{X, eye(a)}});
  }
  // block-diagonal transform [[Tp,0],[0,Tq]] of the columns, in place (via tmp)
  void transform(int64_t nblk, T *X, T *tmp, const Mat &Tp, const Mat &Tq) {
    Mat B((size_t)nc * nc, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        B[i * nc + j] = Tp[i * n + j];
        B[(n + i) * nc + n + j] = Tq[i * n + j];
      }
    lc(nblk, tmp, nullptr, {{X, B}});
    copy(nblk, X, tmp);
  }
  // FP64 reductions, queued into dres and fetched together
  size_t gram_q(int64_t nblk, const T *X, int xc0, int n1, const T *Y, int yc0, int n2, bool dg) {
    const int np = dg ? n1 : n1 * n2;
    if (res_off + np > dres.n) throw Error{TDDFT_E_DEVICE, "result staging overflow"};
    const size_t at = res_off;
    h.prof.begin(ST_GRAM, s);
    gram<T>(nblk, E, X, nc, xc0, n1, Y, nc, yc0, n2, dg, h.partial.p, h.max_parts, dres.p + at, s);
    h.prof.end(ST_GRAM, s);
    res_off += np;
    return at;
  }
  std::vector<double> fetch() {
    std::vector<double> out(res_off);
    if (res_off) TD_HIP(hipMemcpyAsync(out.data(), dres.p, res_off * sizeof(double), hipMemcpyDeviceToHost, s));
    sync();
    res_off = 0;
    return out;
  }
};

// Eq. precond by CG in the S metric, per column, from z = 0 (vectors on R with M complete):
// T(z) = g with T(X) = K^c H^u X - X H^o K^v.  gc = S^u g S^o.  Stops at relative residual
// eps_tol, after max_inner steps, or on non-positive curvature; columns that never step keep
// z = g.  Returns the number of CG steps taken.
template <class T>
int ksdiff_cg(Solver<T> &S, Handle &h, const T *g, const T *gc, T *zk, T *res, T *resc, T *dk,
              T *dkc, T *Lk, T *Lkc, T *tmp, double eps_tol, int max_inner) {
  const int nc = S.nc;
  const int64_t nb = S.nR;
  hipStream_t s = S.s;
  int iters = 0;
  S.copy(nb, res, g);
  S.copy(nb, resc, gc);
  S.copy(nb, dk, g);
  S.copy(nb, dkc, gc);
  fill<T>(zk, (int64_t)S.elems(nb), T(0), s);
  const size_t q0 = S.gram_q(nb, res, 0, nc, resc, 0, nc, true);
  std::vector<double> r = S.fetch();
  std::vector<double> rr(r.begin() + q0, r.begin() + q0 + nc), rr0 = rr;
  std::vector<char> active(nc);
  for (int c = 0; c < nc; ++c) active[c] = rr0[c] > 0.0;
  std::vector<int> steps(nc, 0);
  const double tol2 = eps_tol * eps_tol;
  for (int k = 0; k < max_inner; ++k) {
    bool any = false;
    for (int c = 0; c < nc; ++c) {
      if (active[c] && !(rr[c] > tol2 * rr0[c])) active[c] = 0;
      any |= (bool)active[c];
    }
    if (!any) break;
    kshift_sets<T>(h, nc, dk, nc, 0, Lk, nc, 0);
    const size_t qd = S.gram_q(nb, Lk, 0, nc, dkc, 0, nc, true);
    r = S.fetch();
    std::vector<double> alpha(nc, 0.0), nalpha(nc, 0.0);
    any = false;
    for (int c = 0; c < nc; ++c) {
      if (active[c] && !(r[qd + c] > 0.0)) active[c] = 0;
      if (active[c]) {
        alpha[c] = rr[c] / r[qd + c];
        nalpha[c] = -alpha[c];
      }
      any |= (bool)active[c];
    }
    if (!any) break;
    covariant_sets<T>(h, nc, Lk, nc, 0, Lkc, nc, 0);
    const std::vector<double> ones(nc, 1.0);
    const std::vector<double> *b1 = &ones;
    S.lc(nb, zk, b1, {{dk, S.diag(alpha)}});
    S.lc(nb, res, b1, {{Lk, S.diag(nalpha)}});
    S.lc(nb, resc, b1, {{Lkc, S.diag(nalpha)}});
    const size_t qr = S.gram_q(nb, res, 0, nc, resc, 0, nc, true);
    r = S.fetch();
    std::vector<double> keep(nc), take(nc);
    for (int c = 0; c < nc; ++c) {
      double beta = 1.0;
      if (active[c]) {
        beta = rr[c] > 0.0 ? r[qr + c] / rr[c] : 0.0;
        rr[c] = r[qr + c];
        steps[c]++;
      }
      keep[c] = active[c] ? beta : 1.0;
      take[c] = active[c] ? 1.0 : 0.0;
    }
    const std::vector<double> *bk = &keep;
    S.lc(nb, dk, bk, {{res, S.diag(take)}});
    S.lc(nb, dkc, bk, {{resc, S.diag(take)}});
    ++iters;
  }
  std::vector<double> fromz(nc), fromr(nc);
  for (int c = 0; c < nc; ++c) {
    fromz[c] = steps[c] > 0 ? 1.0 : 0.0;
    fromr[c] = steps[c] > 0 ? 0.0 : 1.0;
  }
  S.lc(nb, tmp, nullptr, {{zk, S.diag(fromz)}, {g, S.diag(fromr)}});
  S.copy(nb, zk, tmp);
  return iters;
}

}  // namespace

// ---------------------------------------------------------------------------------------
template <class T>
static int solve_impl(Handle &h, int n, const tddft_options &o, double *omega, double *Pp,
                      double *Pq, tddft_stats *st) {
  const auto t_start = std::chrono::steady_clock::now();
  auto elapsed_ms = [&]() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  };
  Solver<T> S(h, n);
  const int nc = 2 * n;
  // sets on R: trial vectors P, images F, covariant Pc, direction D, FD, Dc, gradient g, gc,
  // two scratch sets; sets on M: L-gradient r, preconditioned z, their previous values, the
  // inner-CG residual, direction and operator image, scratch
  enum { P, F, Pc, D, FD, Dc, G, Gc, T1, T2, NR_SETS };
  enum { Lr = NR_SETS, Lz, Lrp, Lzp, Lres, Ld, LHd, Ltmp, Lresc, Ldc, LHdc, NSETS };
  S.alloc_sets(NR_SETS, NSETS - NR_SETS);
  auto set = [&](int i) { return S.sets[i]; };
  const int64_t nR = h.nR, nM = h.nM;
  // M complete: the auxiliary matrices and the trial vectors share one full pattern
  const bool complete = h.m_complete;
  hipStream_t s = h.stream;
  int applies = 0, inner_total = 0, fallbacks = 0;
  // the learned scaling stays on while it makes progress: once the largest gradient norm
  // has not halved over kLearnedWindow learned iterations, the rest of the solve uses the
  // plain preconditioner (counted as a fallback)
  bool learned_on = o.precond == TDDFT_PC_LEARNED;
  constexpr int kLearnedWindow = 10;
  std::vector<double> learned_gmax;
  // learned preconditioner: the network evaluated once on the block features gives the
  // elementwise scaling of every R block (and of M's blocks) and the guess weights
  DevBuf<T> cscale, cscale_m;
  std::vector<float> guess_t;
  if (o.precond == TDDFT_PC_LEARNED) {
    Mlp net;
    net.from_blob(o.model, o.model_bytes, s);
    TD_REQUIRE(net.n_in == h.nfeat && net.n_out == h.E + 1,
               "learned-preconditioner model does not match this system's feature or block size");
    DevBuf<float> Y((size_t)nR * (h.E + 1)), tdev(nR);
    net.forward(nR, h.features.p, Y.p);
    cscale.alloc((size_t)nR * h.E);
    split_outputs<T>(nR, h.E, Y.p, cscale.p, tdev.p, s);
    cscale_m.alloc((size_t)nM * h.E);
    gather_blocks<T>(nM, h.E, h.m_in_r.p, cscale.p, cscale_m.p, s);
    guess_t.resize(nR);
    TD_HIP(hipMemcpyAsync(guess_t.data(), tdev.p, nR * sizeof(float), hipMemcpyDeviceToHost, s));
    TD_HIP(hipStreamSynchronize(s));
  }
  float apply_ms = 0.0f;
  // Operator applications replay HIP graphs: the sets a solve applies the operator to
  // (trial vectors, directions) keep their addresses for the whole solve, so each (X, F)
  // pair is captured once (all of its launches, the K-shift products' fork to the handle's
  // second stream included) and replayed afterwards.  Profiling runs stay direct launches
  // (their events are recorded between stages), as does any capture the runtime refuses.
  struct Captured {
    const T *X;
    T *F;
    hipGraphExec_t exec;
  };
  std::vector<Captured> graphs;
  struct GraphGuard {
    std::vector<Captured> &g;
    ~GraphGuard() {
      for (auto &c : g) (void)hipGraphExecDestroy(c.exec);
    }
  } graph_guard{graphs};
  bool use_graphs = o.graphs != 0 && !h.prof.on;
  auto launch_apply = [&](const T *X, T *Fo) {
    // Tamm-Dancoff: p and q hold the same vectors throughout (same start, same updates)
    apply_sets<T>(h, n, X, nc, 0, n, Fo, nc, 0, n, true, h.opts.tda != 0);
  };
  int graph_replays = 0;
  auto apply_graph = [&](const T *X, T *Fo) -> bool {
    for (auto &c : graphs)
      if (c.X == X && c.F == Fo) {
        TD_HIP(hipGraphLaunch(c.exec, s));
        ++graph_replays;
        return true;
      }
    // the workspace is sized before capture, so no allocation happens inside it
    (void)h.w_apply.get(apply_layout(h, n, sizeof(T)).total);
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    bool ok = true;
    try {
      launch_apply(X, Fo);
    } catch (const Error &) {
      ok = false;
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &g);
    hipGraphExec_t ex = nullptr;
    if (ok && ec == hipSuccess && g && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) {
      (void)hipGraphDestroy(g);
      graphs.push_back({X, Fo, ex});
      TD_HIP(hipGraphLaunch(ex, s));
      return true;
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return false;
  };
  auto apply = [&](const T *X, T *Fo) {
    TD_HIP(hipEventRecord(h.ev0, s));
    if (!(use_graphs && apply_graph(X, Fo))) {
      use_graphs = false;
      launch_apply(X, Fo);
    }
    TD_HIP(hipEventRecord(h.ev1, s));
    TD_HIP(hipEventSynchronize(h.ev1));
    float ms = 0.0f;
    TD_HIP(hipEventElapsedTime(&ms, h.ev0, h.ev1));
    apply_ms += ms;
    ++applies;
  };
  auto cov = [&](const T *X, T *Y) { covariant_sets<T>(h, nc, X, nc, 0, Y, nc, 0); };
  auto proj = [&](const T *Lm, T *Y) { project_sets<T>(h, nc, Lm, nc, 0, Y, nc, 0); };
  auto proj_t = [&](const T *Y, T *Lm) { project_t_sets<T>(h, nc, Y, nc, 0, Lm, nc, 0); };

  // ---- initial auxiliary matrices L0 on M -> P = Pi(L0)
  {
    T *tmpR = set(T1);
    if (Pp && Pq) {
      pack<T>(nR, h.BU, h.BO, n, h.opts.tda ? Pq : Pp, h.nnzR, h.r_voff.p, h.r_shape.p, tmpR, nc, 0, s);
      pack<T>(nR, h.BU, h.BO, n, Pq, h.nnzR, h.r_voff.p, h.r_shape.p, tmpR, nc, n, s);
    } else {
      // seeded N(0,1) (SplitMix64 + Box-Muller), the same matrix for p and q
      std::vector<double> g((size_t)n * h.nnzR);
      uint64_t x = o.seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
      auto next = [&]() {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
      };
      for (size_t i = 0; i < g.size(); i += 2) {
        const double u1 = ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        const double u2 = ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        const double r = std::sqrt(-2.0 * std::log(u1));
        g[i] = r * std::cos(2.0 * M_PI * u2);
        if (i + 1 < g.size()) g[i + 1] = r * std::sin(2.0 * M_PI * u2);
      }
      if (!guess_t.empty()) {   // learned guess: block (I, J) scaled by sqrt(10^t_IJ)
        for (int64_t b = 0; b < nR; ++b) {
          const double f = std::sqrt(std::pow(10.0, (double)guess_t[b]));
          const int sz = (h.r_shape_host[b] & 0xff) * (h.r_shape_host[b] >> 8);
          for (int i = 0; i < n; ++i) {
            double *v = g.data() + (size_t)i * h.nnzR + h.r_voff_host[b];
            for (int e = 0; e < sz; ++e) v[e] *= f;
          }
        }
      }
      DevBuf<double> dg(g.size());
      dg.upload(g, s);
      pack<T>(nR, h.BU, h.BO, n, dg.p, h.nnzR, h.r_voff.p, h.r_shape.p, tmpR, nc, 0, s);
      pack<T>(nR, h.BU, h.BO, n, dg.p, h.nnzR, h.r_voff.p, h.r_shape.p, tmpR, nc, n, s);
      S.sync();
    }
    h.prof.begin(ST_GATHER, s);
    gather_blocks<T>(nM, nc * h.E, h.m_in_r.p, tmpR, set(Ltmp), s);
    h.prof.end(ST_GATHER, s);
    proj(set(Ltmp), set(P));
    cov(set(P), set(Pc));
  }
  Mat Tp, Tq;
  // Tsiper Gram-Schmidt of P (and the same transform of F, Pc and the carried history)
  auto gs_step = [&](bool with_history) -> bool {
    S.gram_q(nR, set(P), 0, n, set(Pc), n, n, false);
    std::vector<double> C = S.fetch();
    if (!orthonormalise(C, n, Tp, Tq)) return false;
    S.transform(nR, set(P), set(T1), Tp, Tq);
    S.transform(nR, set(Pc), set(T1), Tp, Tq);
    S.transform(nR, set(F), set(T1), Tp, Tq);
    if (with_history) {
      S.transform(nR, set(D), set(T1), Tp, Tq);
      S.transform(nR, set(Dc), set(T1), Tp, Tq);
      S.transform(nM, set(Lrp), set(Ltmp), Tp, Tq);
      S.transform(nM, set(Lzp), set(Ltmp), Tp, Tq);
    }
    return true;
  };
  if (!gs_step(false)) throw Error{TDDFT_E_NOT_PD, "initial trial vectors are linearly dependent in the Tsiper metric"};
  apply(set(P), set(F));

  std::vector<double> w(n), w_prev(n, 0.0);
  bool converged = false, have_prev = false, have_dir = false, restart_next = false;
  int it = 0, stalls = 0;
  double gmax0 = 0.0;
  const double sqrt_tol = std::sqrt(o.tol_omega);
  Mat Nm((size_t)n * n);
  for (it = 0; it <= o.max_iter; ++it) {
    // N, omega, gradient g = F - N (q, p), its covariant form and norms
    const size_t qN = S.gram_q(nR, set(F), 0, nc, set(Pc), 0, nc, false);
    std::vector<double> r = S.fetch();
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        Nm[i * n + j] = 0.5 * (r[qN + (size_t)i * nc + j] + r[qN + (size_t)(n + i) * nc + n + j]);
    Nm = sym(Nm, n);
    Mat V;
    sym_eig(Nm, n, w, V);
    {
      Mat Cg((size_t)nc * nc, 0.0);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          Cg[i * nc + n + j] = -Nm[i * n + j];
          Cg[(n + i) * nc + j] = -Nm[i * n + j];
        }
      S.lc(nR, set(G), nullptr, {{set(F), S.eye()}, {set(P), Cg}});
      cov(set(G), set(Gc));
    }
    const size_t qg = S.gram_q(nR, set(G), 0, nc, set(Gc), 0, nc, true);
    r = S.fetch();
    double gmax = 0.0;
    for (int i = 0; i < n; ++i) gmax = std::max(gmax, std::sqrt(std::max(0.0, r[qg + i] + r[qg + n + i])));
    if (st && st->log_omega && st->log_len < st->log_capacity) {
      for (int i = 0; i < n; ++i) st->log_omega[(size_t)st->log_len * n + i] = w[i];
      if (st->log_time_ms) st->log_time_ms[st->log_len] = elapsed_ms();
      if (st->log_gnorm) st->log_gnorm[st->log_len] = gmax;
      st->log_len++;
    }
    for (double v : w)
      if (!std::isfinite(v)) throw Error{TDDFT_E_NOT_PD, "non-finite Tsiper functional"};
    // inner tolerance: constant, or loose while the gradient is still large and tightened as
    // it falls (Sec. IV.A: loose and tight tolerances converge alike in the first iterations)
    if (it == 0) gmax0 = gmax;
    double eps_cur = o.eps_tol;
    if (o.eps_loose > o.eps_tol && gmax0 > 0.0)
      eps_cur = std::min(o.eps_loose, std::max(o.eps_tol, o.eps_loose * gmax / gmax0));
    if (have_prev) {
      double dw = 0.0;
      for (int i = 0; i < n; ++i) dw = std::max(dw, std::fabs(w[i] - w_prev[i]));
      if (dw < o.tol_omega && gmax < sqrt_tol) {
        converged = true;
        break;
      }
    }
    if (it == o.max_iter) break;
    w_prev = w;
    have_prev = true;
    if (learned_on) {
      learned_gmax.push_back(gmax);
      const size_t m = learned_gmax.size();
      if (m > (size_t)kLearnedWindow && gmax > 0.5 * learned_gmax[m - 1 - kLearnedWindow]) {
        learned_on = false;
        ++fallbacks;
      }
    }

    if (complete) {
      // ---- M complete: CG on Eq. precond T(z) = g in the S metric (vectors on R = M);
      //      the conjugation uses r = S^u g S^o with Euclidean dots, i.e. S-metric dots of g
      S.copy(nM, set(Lr), set(Gc));
      bool done = false;
      if (learned_on) {
        // learned block scaling, kept if it is a descent direction for every column
        block_scale<T>(nM, nc, h.E, cscale.p, set(G), set(Lz), s);
        const size_t qd = S.gram_q(nM, set(Lz), 0, nc, set(Gc), 0, nc, true);
        r = S.fetch();
        done = true;
        for (int c = 0; c < nc; ++c) done = done && r[qd + c] > 0.0;
        if (!done) ++fallbacks;
      }
      if (!done) {
        if (o.precond == TDDFT_PC_NONE) {
          S.copy(nM, set(Lz), set(G));
        } else {
          inner_total += ksdiff_cg(S, h, set(G), set(Gc), set(Lz), set(Lres), set(Lresc), set(Ld),
                                   set(Ldc), set(LHd), set(LHdc), set(Ltmp), eps_cur, o.max_inner);
        }
      }
    } else {
    // ---- gradient with respect to L: r = mask_M(Pi^T(S^u g S^o))
    proj_t(set(Gc), set(Lr));
    // ---- preconditioner: CG on H_L z = r, H_L(X) = mask_M(Pi^T(S^u T(Pi X) S^o)),
    //      Euclidean inner product on M, per column
    bool done = false;
    if (learned_on) {
      block_scale<T>(nM, nc, h.E, cscale_m.p, set(Lr), set(Lz), s);
      const size_t qd = S.gram_q(nM, set(Lz), 0, nc, set(Lr), 0, nc, true);
      r = S.fetch();
      done = true;
      for (int c = 0; c < nc; ++c) done = done && r[qd + c] > 0.0;
      if (!done) ++fallbacks;
    }
    if (done) {
    } else if (o.precond == TDDFT_PC_NONE) {
      S.copy(nM, set(Lz), set(Lr));
    } else {
      T *res = set(Lres), *dk = set(Ld), *Hd = set(LHd), *zk = set(Lz);
      S.copy(nM, res, set(Lr));
      S.copy(nM, dk, set(Lr));
      fill<T>(zk, (int64_t)S.elems(nM), T(0), s);
      const size_t q0 = S.gram_q(nM, res, 0, nc, res, 0, nc, true);
      r = S.fetch();
      std::vector<double> rr(r.begin() + q0, r.begin() + q0 + nc), rr0 = rr;
      std::vector<char> active(nc);
      for (int c = 0; c < nc; ++c) active[c] = rr0[c] > 0.0;
      std::vector<int> steps(nc, 0);
      const double tol2 = eps_cur * eps_cur;
      for (int k = 0; k < o.max_inner; ++k) {
        bool any = false;
        for (int c = 0; c < nc; ++c) {
          if (active[c] && !(rr[c] > tol2 * rr0[c])) active[c] = 0;
          any |= (bool)active[c];
        }
        if (!any) break;
        proj(dk, set(T1));
        kshift_sets<T>(h, nc, set(T1), nc, 0, set(T2), nc, 0);
        cov(set(T2), set(T1));
        proj_t(set(T1), Hd);
        const size_t qd = S.gram_q(nM, dk, 0, nc, Hd, 0, nc, true);
        r = S.fetch();
        std::vector<double> alpha(nc, 0.0), nalpha(nc, 0.0);
        any = false;
        for (int c = 0; c < nc; ++c) {
          if (active[c] && !(r[qd + c] > 0.0)) active[c] = 0;
          if (active[c]) {
            alpha[c] = rr[c] / r[qd + c];
            nalpha[c] = -alpha[c];
          }
          any |= (bool)active[c];
        }
        if (!any) break;
        const std::vector<double> ones(nc, 1.0);
        const std::vector<double> *b1 = &ones;
        S.lc(nM, zk, b1, {{dk, S.diag(alpha)}});
        S.lc(nM, res, b1, {{Hd, S.diag(nalpha)}});
        const size_t qr = S.gram_q(nM, res, 0, nc, res, 0, nc, true);
        r = S.fetch();
        std::vector<double> keep(nc), take(nc);
        for (int c = 0; c < nc; ++c) {
          double beta = 1.0;
          if (active[c]) {
            beta = rr[c] > 0.0 ? r[qr + c] / rr[c] : 0.0;
            rr[c] = r[qr + c];
            steps[c]++;
          }
          keep[c] = active[c] ? beta : 1.0;
          take[c] = active[c] ? 1.0 : 0.0;
        }
        S.lc(nM, dk, &keep, {{res, S.diag(take)}});
        inner_total++;
      }
      // columns that never stepped keep z = r
      std::vector<double> fromz(nc), fromr(nc);
      for (int c = 0; c < nc; ++c) {
        fromz[c] = steps[c] > 0 ? 1.0 : 0.0;
        fromr[c] = steps[c] > 0 ? 0.0 : 1.0;
      }
      S.lc(nM, set(Ltmp), nullptr, {{zk, S.diag(fromz)}, {set(Lr), S.diag(fromr)}});
      S.copy(nM, zk, set(Ltmp));
    }
    }
    // ---- Polak-Ribiere(+) in L: beta = <z, r - r_prev> / <z_prev, r_prev>
    double beta = 0.0;
    const bool restart = !have_dir || restart_next || (o.restart > 0 && it % o.restart == 0);
    if (!restart) {
      const size_t qa = S.gram_q(nM, set(Lz), 0, nc, set(Lr), 0, nc, true);
      const size_t qb = S.gram_q(nM, set(Lz), 0, nc, set(Lrp), 0, nc, true);
      const size_t qc = S.gram_q(nM, set(Lzp), 0, nc, set(Lrp), 0, nc, true);
      r = S.fetch();
      double num = 0.0, den = 0.0;
      for (int c = 0; c < nc; ++c) {
        num += r[qa + c] - r[qb + c];
        den += r[qc + c];
      }
      if (den > 0.0) beta = std::max(0.0, num / den);
    }
    // ---- direction D = -Pi(z) + beta D_prev on R and its covariant form
    proj(set(Lz), set(T2));
    cov(set(T2), set(T1));
    if (beta > 0.0) {
      const std::vector<double> bv(nc, beta);
      const std::vector<double> *bb = &bv;
      S.lc(nR, set(D), bb, {{set(T2), S.eye(-1.0)}});
      S.lc(nR, set(Dc), bb, {{set(T1), S.eye(-1.0)}});
      const size_t qd = S.gram_q(nR, set(D), 0, nc, set(Gc), 0, nc, true);
      r = S.fetch();
      double dd = 0.0;
      for (int c = 0; c < nc; ++c) dd += r[qd + c];
      if (dd >= 0.0) {   // not a descent direction: steepest (preconditioned) descent
        S.lc(nR, set(D), nullptr, {{set(T2), S.eye(-1.0)}});
        S.lc(nR, set(Dc), nullptr, {{set(T1), S.eye(-1.0)}});
      }
    } else {
      S.lc(nR, set(D), nullptr, {{set(T2), S.eye(-1.0)}});
      S.lc(nR, set(Dc), nullptr, {{set(T1), S.eye(-1.0)}});
    }
    have_dir = true;
    apply(set(D), set(FD));

    // ---- exact line search on Tr[N(lambda) B(lambda)^-1]
    const size_t q1 = S.gram_q(nR, set(F), 0, nc, set(Dc), 0, nc, false);
    const size_t q2 = S.gram_q(nR, set(FD), 0, nc, set(Pc), 0, nc, false);
    const size_t q3 = S.gram_q(nR, set(FD), 0, nc, set(Dc), 0, nc, false);
    const size_t c0 = S.gram_q(nR, set(P), 0, n, set(Pc), n, n, false);
    const size_t c1a = S.gram_q(nR, set(P), 0, n, set(Dc), n, n, false);
    const size_t c1b = S.gram_q(nR, set(D), 0, n, set(Pc), n, n, false);
    const size_t c2 = S.gram_q(nR, set(D), 0, n, set(Dc), n, n, false);
    const size_t dn = S.gram_q(nR, set(D), 0, nc, set(Dc), 0, nc, true);
    const size_t pn = S.gram_q(nR, set(P), 0, nc, set(Pc), 0, nc, true);
    r = S.fetch();
    auto nblock = [&](size_t q) {
      Mat m((size_t)n * n);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          m[i * n + j] = 0.5 * (r[q + (size_t)i * nc + j] + r[q + (size_t)(n + i) * nc + n + j]);
      return m;
    };
    Mat N0 = Nm, N1 = nblock(q1), N1b = nblock(q2), N2 = nblock(q3);
    for (size_t k = 0; k < N1.size(); ++k) N1[k] += N1b[k];
    N1 = sym(N1, n);
    N2 = sym(N2, n);
    Mat B0((size_t)n * n), B1((size_t)n * n), B2((size_t)n * n);
    for (int k = 0; k < n * n; ++k) {
      B0[k] = r[c0 + k];
      B1[k] = r[c1a + k] + r[c1b + k];
      B2[k] = r[c2 + k];
    }
    B0 = sym(B0, n);
    B1 = sym(B1, n);
    B2 = sym(B2, n);
    double dnorm = 0.0, pnorm = 0.0;
    for (int c = 0; c < nc; ++c) {
      dnorm += r[dn + c];
      pnorm += r[pn + c];
    }
    auto phi = [&](double l) {
      Mat Nl((size_t)n * n), Bl((size_t)n * n);
      for (int k = 0; k < n * n; ++k) {
        Nl[k] = N0[k] + l * N1[k] + l * l * N2[k];
        Bl[k] = B0[k] + l * B1[k] + l * l * B2[k];
      }
      return trace_nbinv(Nl, Bl, n);
    };
    const double scale = 1.0 / std::sqrt(std::max(std::fabs(dnorm), 1e-300));
    const int NL = 241;
    const double phi0 = phi(0.0);
    double best = phi0, lam = 0.0;
    int kbest = -1, end = NL;
    std::vector<double> lams(NL), vals(NL);
    for (int k = 0; k < NL; ++k) {
      lams[k] = scale * std::pow(10.0, -8.0 + 12.0 * k / (NL - 1));
      vals[k] = phi(lams[k]);
      if (!std::isfinite(vals[k])) { end = k; break; }
      if (vals[k] < best) { best = vals[k]; kbest = k; }
    }
    if (kbest < 0) {
      if (++stalls >= 3) break;
      have_dir = false;
      continue;
    }
    stalls = 0;
    {
      const double lo = kbest > 0 ? lams[kbest - 1] : 0.0;
      const double hi = kbest + 1 < end ? lams[kbest + 1] : lams[kbest];
      lam = lams[kbest];
      if (hi > lo) {
        const double lb = brent_min(phi, lo, hi, 1e-12);
        if (phi(lb) <= best) lam = lb;
      }
    }
    // a step longer than the trial vectors themselves, or one that does not lower the
    // functional, invalidates the conjugation history
    restart_next = lam * std::sqrt(std::max(dnorm, 0.0)) > std::sqrt(std::max(pnorm, 0.0)) ||
                   !(phi(lam) < phi0 - 1e-14 * std::fabs(phi0));
    // ---- update, periodic refresh, keep history, orthonormalise
    S.axpy(nR, set(P), lam, set(D));
    S.axpy(nR, set(F), lam, set(FD));
    S.axpy(nR, set(Pc), lam, set(Dc));
    if (o.refresh > 0 && (it + 1) % o.refresh == 0) {
      apply(set(P), set(F));
      cov(set(P), set(Pc));
    }
    S.copy(nM, set(Lrp), set(Lr));
    S.copy(nM, set(Lzp), set(Lz));
    if (!gs_step(true)) throw Error{TDDFT_E_NOT_PD, "Tsiper metric lost positivity"};
  }
  // ---- subspace diagonalisation: rotate to eigenvectors of N (B = I)
  {
    const size_t qN = S.gram_q(nR, set(F), 0, nc, set(Pc), 0, nc, false);
    std::vector<double> r = S.fetch();
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        Nm[i * n + j] = 0.5 * (r[qN + (size_t)i * nc + j] + r[qN + (size_t)(n + i) * nc + n + j]);
    Nm = sym(Nm, n);
    Mat V;
    sym_eig(Nm, n, w, V);
    Mat U((size_t)n * n);   // new_k = sum_i V_ik old_i
    for (int k = 0; k < n; ++k)
      for (int i = 0; i < n; ++i) U[k * n + i] = V[i * n + k];
    S.transform(nR, set(P), set(T1), U, U);
    if (Pp) unpack<T>(nR, h.BU, h.BO, n, set(P), nc, 0, h.r_voff.p, h.r_shape.p, Pp, h.nnzR, s);
    if (Pq) unpack<T>(nR, h.BU, h.BO, n, set(P), nc, n, h.r_voff.p, h.r_shape.p, Pq, h.nnzR, s);
    S.sync();
  }
  for (int i = 0; i < n; ++i) omega[i] = w[i];
  if (st) {
    st->iterations = it;
    st->converged = converged ? 1 : 0;
    st->inner_total = inner_total;
    st->applies = applies;
    st->graph_replays = graph_replays;
    st->fallbacks = fallbacks;
    st->setup_ms = h.setup_ms;
    st->solve_ms = elapsed_ms();
    st->apply_ms = apply_ms;
  }
  if (!converged) return TDDFT_E_NO_CONVERGENCE;
  return fallbacks > 0 ? TDDFT_W_FALLBACK : TDDFT_OK;
}

// Eq. precond alone, for n states in the C-ABI layout (complete M only)
template <class T>
static void precondition_impl(Handle &h, int n, const double *g, double *G, double eps_tol,
                              int max_inner) {
  TD_REQUIRE(h.m_complete, "tddft_precondition needs a complete M");
  Solver<T> S(h, n);
  const int nc = 2 * n;
  enum { X, Xc, Z, RES, RESC, DK, DKC, LK, LKC, TMP, NS };
  S.alloc_sets(NS, 0);
  fill<T>(S.sets[X], (int64_t)S.elems(h.nR), T(0), h.stream);
  pack<T>(h.nR, h.BU, h.BO, n, g, h.nnzR, h.r_voff.p, h.r_shape.p, S.sets[X], nc, 0, h.stream);
  covariant_sets<T>(h, nc, S.sets[X], nc, 0, S.sets[Xc], nc, 0);
  ksdiff_cg(S, h, S.sets[X], S.sets[Xc], S.sets[Z], S.sets[RES], S.sets[RESC], S.sets[DK],
            S.sets[DKC], S.sets[LK], S.sets[LKC], S.sets[TMP], eps_tol, max_inner);
  unpack<T>(h.nR, h.BU, h.BO, n, S.sets[Z], nc, 0, h.r_voff.p, h.r_shape.p, G, h.nnzR, h.stream);
  S.sync();
}

void precondition(Handle &h, int n, const double *g, double *G, double eps_tol, int max_inner) {
  if (h.precision == TDDFT_FP64) precondition_impl<double>(h, n, g, G, eps_tol, max_inner);
  else precondition_impl<float>(h, n, g, G, eps_tol, max_inner);
}

int pcg_solve(Handle &h, int n, const tddft_options &o, double *omega, double *Pp, double *Pq,
              tddft_stats *stats) {
  if (h.precision == TDDFT_FP64) return solve_impl<double>(h, n, o, omega, Pp, Pq, stats);
  return solve_impl<float>(h, n, o, omega, Pp, Pq, stats);
}

}  // namespace tddft
