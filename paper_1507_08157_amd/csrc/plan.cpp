// Host-side symbolic work done once per system: block patterns, the pair lists of every
// masked product, exact host products of the fixed matrices, grid tiles, and
// FFT plans.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.h"
#include "handle.h"

namespace tddft {

int64_t Pattern::find(int r, int c) const {
  const int32_t *b = col.data() + rowptr[r];
  const int32_t *e = col.data() + rowptr[r + 1];
  const int32_t *it = std::lower_bound(b, e, c);
  if (it != e && *it == c) return (int64_t)(it - col.data());
  return -1;
}

Pattern Pattern::dense(int nr, int nc) {
  Pattern p;
  p.nbr = nr;
  p.nbc = nc;
  p.rowptr.resize(nr + 1);
  p.col.resize((size_t)nr * nc);
  for (int i = 0; i <= nr; ++i) p.rowptr[i] = (int64_t)i * nc;
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nc; ++j) p.col[(size_t)i * nc + j] = j;
  return p;
}

Pattern transpose(const Pattern &A) {
  Pattern T;
  T.nbr = A.nbc;
  T.nbc = A.nbr;
  T.rowptr.assign(T.nbr + 1, 0);
  for (int32_t c : A.col) T.rowptr[c + 1]++;
  for (int i = 0; i < T.nbr; ++i) T.rowptr[i + 1] += T.rowptr[i];
  T.col.resize(A.col.size());
  std::vector<int64_t> pos(T.rowptr.begin(), T.rowptr.end() - 1);
  for (int i = 0; i < A.nbr; ++i)
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) T.col[pos[A.col[k]]++] = i;
  return T;
}

Pattern product_pattern(const Pattern &A, const Pattern &B) {
  Pattern C;
  C.nbr = A.nbr;
  C.nbc = B.nbc;
  C.rowptr.assign(C.nbr + 1, 0);
  std::vector<int> mark(B.nbc, -1);
  std::vector<int32_t> row;
  for (int i = 0; i < A.nbr; ++i) {
    row.clear();
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
      const int kk = A.col[k];
      for (int64_t q = B.rowptr[kk]; q < B.rowptr[kk + 1]; ++q) {
        const int j = B.col[q];
        if (mark[j] != i) {
          mark[j] = i;
          row.push_back(j);
        }
      }
    }
    std::sort(row.begin(), row.end());
    C.col.insert(C.col.end(), row.begin(), row.end());
    C.rowptr[i + 1] = (int64_t)C.col.size();
  }
  return C;
}

Pattern intersect(const Pattern &A, const Pattern &B) {
  Pattern C;
  C.nbr = A.nbr;
  C.nbc = A.nbc;
  C.rowptr.assign(C.nbr + 1, 0);
  for (int i = 0; i < A.nbr; ++i) {
    int64_t a = A.rowptr[i], ae = A.rowptr[i + 1], b = B.rowptr[i], be = B.rowptr[i + 1];
    while (a < ae && b < be) {
      if (A.col[a] < B.col[b]) ++a;
      else if (B.col[b] < A.col[a]) ++b;
      else { C.col.push_back(A.col[a]); ++a; ++b; }
    }
    C.rowptr[i + 1] = (int64_t)C.col.size();
  }
  return C;
}

Plan plan_product(const Pattern &A, const Pattern &B, const Pattern &out) {
  Plan p;
  p.out = out;
  const int64_t nout = out.nnzb();
  p.ptr.assign(nout + 1, 0);
  std::vector<int64_t> omap(B.nbc, -1);
  // pass 1: count, pass 2: fill (pairs of one output block ordered by k)
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int64_t> fillpos;
    if (pass == 1) {
      for (int64_t k = 0; k < nout; ++k) p.ptr[k + 1] += p.ptr[k];
      p.pa.resize(p.ptr[nout]);
      p.pb.resize(p.ptr[nout]);
      fillpos.assign(p.ptr.begin(), p.ptr.end() - 1);
    }
    for (int i = 0; i < A.nbr; ++i) {
      for (int64_t q = out.rowptr[i]; q < out.rowptr[i + 1]; ++q) omap[out.col[q]] = q;
      for (int64_t ka = A.rowptr[i]; ka < A.rowptr[i + 1]; ++ka) {
        const int k = A.col[ka];
        for (int64_t kb = B.rowptr[k]; kb < B.rowptr[k + 1]; ++kb) {
          const int64_t o = omap[B.col[kb]];
          if (o < 0) continue;
          if (pass == 0) {
            p.ptr[o + 1]++;
          } else {
            const int64_t w = fillpos[o]++;
            p.pa[w] = (int32_t)ka;
            p.pb[w] = (int32_t)kb;
          }
        }
      }
      for (int64_t q = out.rowptr[i]; q < out.rowptr[i + 1]; ++q) omap[out.col[q]] = -1;
    }
  }
  auto complete = [](const Pattern &P) { return P.nnzb() == (int64_t)P.nbr * P.nbc; };
  if (complete(A) && complete(B) && complete(out) && out.nbr == A.nbr && out.nbc == B.nbc &&
      A.nbc == B.nbr) {
    p.di = A.nbr;
    p.dk = A.nbc;
    p.dj = B.nbc;
  }
  return p;
}

HostBsr host_product(const HostBsr &A, const HostBsr &B, const Pattern &out) {
  if (A.bc != B.br) throw Error{TDDFT_E_INVALID, "host_product: block shape mismatch"};
  Plan pl = plan_product(A.pat, B.pat, out);
  HostBsr C;
  C.pat = out;
  C.br = A.br;
  C.bc = B.bc;
  const int br = A.br, bk = A.bc, bc = B.bc;
  C.val.assign((size_t)out.nnzb() * br * bc, 0.0);
  for (int64_t o = 0; o < out.nnzb(); ++o) {
    double *c = C.val.data() + (size_t)o * br * bc;
    for (int64_t q = pl.ptr[o]; q < pl.ptr[o + 1]; ++q) {
      const double *a = A.val.data() + (size_t)pl.pa[q] * br * bk;
      const double *b = B.val.data() + (size_t)pl.pb[q] * bk * bc;
      for (int r = 0; r < br; ++r)
        for (int t = 0; t < bk; ++t) {
          const double ar = a[r * bk + t];
          if (ar == 0.0) continue;
          for (int cc = 0; cc < bc; ++cc) c[r * bc + cc] += ar * b[t * bc + cc];
        }
    }
  }
  return C;
}

HostBsr host_transpose(const HostBsr &A) {
  HostBsr T;
  T.pat = transpose(A.pat);
  T.br = A.bc;
  T.bc = A.br;
  T.val.assign(A.val.size(), 0.0);
  for (int i = 0; i < A.pat.nbr; ++i)
    for (int64_t k = A.pat.rowptr[i]; k < A.pat.rowptr[i + 1]; ++k) {
      const int64_t kt = T.pat.find(A.pat.col[k], i);
      for (int r = 0; r < A.br; ++r)
        for (int c = 0; c < A.bc; ++c)
          T.val[((size_t)kt * T.br + c) * T.bc + r] = A.val[((size_t)k * A.br + r) * A.bc + c];
    }
  return T;
}

void DevPlan::upload(const Plan &p, hipStream_t s) {
  nout = p.out.nnzb();
  npairs = (int64_t)p.pa.size();
  di = p.di;
  dk = p.dk;
  dj = p.dj;
  ptr.upload(p.ptr, s);
  std::vector<int2> pr(npairs);
  for (int64_t i = 0; i < npairs; ++i) pr[i] = make_int2(p.pa[i], p.pb[i]);
  pairs.upload(pr, s);
  TD_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------------------
// FFT plan: radices (8, 4, 2, 3, 5, 7 preferred in that order) and twiddles
// w[pass][k * (R - 1) + r - 1] = exp(-2 pi i r k / (Ns R)), k < Ns, 1 <= r < R
bool fft_factor(int n, std::vector<int> &radix) {
  radix.clear();
  int m = n;
  const int pref[6] = {8, 4, 2, 3, 5, 7};
  for (int r : pref)
    while (m % r == 0) {
      radix.push_back(r);
      m /= r;
    }
  return m == 1 && (int)radix.size() <= 12;
}

void build_fft_plan(FFTPlan &pl, const int n[3], hipStream_t s) {
  std::vector<double> tw;
  for (int d = 0; d < 3; ++d) {
    AxisFFT &a = pl.ax[d];
    a.n = n[d];
    if (!fft_factor(n[d], a.radix))
      throw Error{TDDFT_E_INVALID, "grid dimension " + std::to_string(n[d]) +
                                       " is not a product of 2, 3, 5 and 7"};
    a.tw_off.clear();
    int Ns = 1, len = 0;
    std::vector<double> axis;
    for (int R : a.radix) {
      a.tw_off.push_back(len);
      for (int k = 0; k < Ns; ++k)
        for (int r = 1; r < R; ++r) {
          const double ang = -2.0 * M_PI * (double)r * k / ((double)Ns * R);
          axis.push_back(std::cos(ang));
          axis.push_back(std::sin(ang));
          ++len;
        }
      Ns *= R;
    }
    a.tw_len = len;
    tw.insert(tw.end(), axis.begin(), axis.end());
    const std::vector<int> ip = fft_inplace_threads(a);
    pl.nt[d] = ip.empty() ? 0 : ip.front();
  }
  pl.tw64.upload(tw, s);
  std::vector<float> twf(tw.begin(), tw.end());
  pl.tw32.upload(twf, s);
  TD_HIP(hipStreamSynchronize(s));
}

}  // namespace tddft

namespace tddft {

const char *const kStageNames[ST_COUNT] = {
    "kshift_left", "kshift_right", "density", "fft_x_fwd", "fft_y_fwd", "fft_z_poisson",
    "fft_y_inv", "fft_x_inv", "vint", "vint_reduce", "sandwich_left", "sandwich_right",
    "project", "covariant", "gram", "lincomb", "project_t", "gather"};

void Prof::init() {
  for (int k = 0; k < ST_COUNT; ++k) {
    if (!a[k]) TD_HIP(hipEventCreate(&a[k]));
    if (!b[k]) TD_HIP(hipEventCreate(&b[k]));
  }
}

void Prof::destroy() {
  for (int k = 0; k < ST_COUNT; ++k) {
    if (a[k]) (void)hipEventDestroy(a[k]);
    if (b[k]) (void)hipEventDestroy(b[k]);
    a[k] = b[k] = nullptr;
  }
}

static void prof_take(Prof &p, int k) {
  TD_HIP(hipEventSynchronize(p.b[k]));
  float t = 0.0f;
  TD_HIP(hipEventElapsedTime(&t, p.a[k], p.b[k]));
  p.ms[k] += t;
  p.count[k] += 1;
  p.pending[k] = false;
}

void Prof::begin(int k, hipStream_t s) {
  if (!on) return;
  if (pending[k]) prof_take(*this, k);
  TD_HIP(hipEventRecord(a[k], s));
}

void Prof::end(int k, hipStream_t s) {
  if (!on) return;
  TD_HIP(hipEventRecord(b[k], s));
  pending[k] = true;
}

void Prof::collect() {
  for (int k = 0; k < ST_COUNT; ++k)
    if (pending[k]) prof_take(*this, k);
}

void Prof::reset() {
  for (int k = 0; k < ST_COUNT; ++k) {
    ms[k] = 0.0;
    count[k] = 0;
    pending[k] = false;
  }
}

}  // namespace tddft
