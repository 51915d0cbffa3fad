// Launch-shape autotuner.  At tddft_create it times the candidate launch shapes of the
// hot kernels on the handle's own data (tile lists, samples, pair lists), keeps the
// fastest in the handle, and remembers it in a process-wide table keyed by the shapes
// that decide it, so that handles of like systems reuse the choice without timing:
//   * FFT passes: threads per workgroup of each axis (256, 512 or 1024 in place, or the
//     two-buffer form), per axis from the stage times of the five passes;
//   * response density: tiles (waves) per workgroup, 2, 4 or 8, and P blocks in scalar
//     registers or in vector registers shared by DPP row broadcasts;
//   * sparse products: columns per thread (1, 2 or 4) and operand pairs per memory round
//     trip (1 to 8), per product plan, at the column count a 4-state application passes it;
//   * dense (complete-pattern) MFMA products: output tile shape (three shapes with the same
//     k-slab depth), per product plan.
// No candidate changes an arithmetic operation or the order of any sum, so results are the
// same whatever is chosen.
#include <map>
#include <mutex>
#include <sstream>

#include "handle.h"

namespace tddft {

namespace {

std::mutex g_tune_mu;
std::map<std::string, std::vector<int>> g_tune_cache;

bool cached(const std::string &key, std::vector<int> &out) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune_cache.find(key);
  if (it == g_tune_cache.end()) return false;
  out = it->second;
  return true;
}

void remember(const std::string &key, const std::vector<int> &v) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache[key] = v;
}

// device milliseconds of f() on stream s, best of `reps` after one warm-up run
template <class F>
float best_ms(hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, F f) {
  f();
  float best = 1e30f;
  for (int r = 0; r < reps; ++r) {
    TD_HIP(hipEventRecord(e0, s));
    f();
    TD_HIP(hipEventRecord(e1, s));
    TD_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    TD_HIP(hipEventElapsedTime(&ms, e0, e1));
    best = std::min(best, ms);
  }
  return best;
}

template <class T>
void tune_typed(Handle &h) {
  hipStream_t s = h.stream;
  const int n = 4, nc = 2 * n;
  const int prec = h.precision;
  // scratch: one column set of 8 columns on R for X and F, the application workspace of 4
  // states (fields, FFT work), zero-filled
  const size_t elems = (size_t)h.nR * nc * h.E;
  T *X = (T *)h.w_pcg.get(2 * elems * sizeof(T));
  T *F = X + elems;
  fill<T>(X, (int64_t)(2 * elems), T(0), s);
  const ApplyLayout lay = apply_layout(h, n, sizeof(T));
  unsigned char *ws = (unsigned char *)h.w_apply.get(lay.total);
  T *fields = (T *)ws;
  T *work = (T *)(ws + lay.fields);
  fill<T>(fields, (int64_t)((lay.fields + lay.work) / sizeof(T)), T(0), s);
  const int64_t pstride = (int64_t)h.nt * TP * 2;
  const int st = std::is_same<T, double>::value ? SAMPLE_F64 : h.stype;
  DevTiles tl = h.tiles_uo;
  tl.usamp = h.usamp();
  tl.osamp = h.osamp();

  // ---- FFT threads per axis
  {
    std::ostringstream k;
    k << "fft " << prec << " " << h.n[0] << " " << h.n[1] << " " << h.n[2] << " " << h.lds_limit;
    std::vector<int> choice;
    if (!cached(k.str(), choice)) {
      std::vector<int> cand[3];
      const size_t elem = 2 * sizeof(T);
      for (int d = 0; d < 3; ++d) {
        cand[d] = fft_inplace_threads(h.fft.ax[d]);
        const int lines = 16;
        if (2 * (size_t)lines * (h.fft.ax[d].n + 1) * elem <= h.lds_limit) cand[d].push_back(0);
        if (cand[d].empty()) cand[d].push_back(h.fft.nt[d]);
      }
      const size_t ncand = std::max({cand[0].size(), cand[1].size(), cand[2].size()});
      std::vector<double> t[3];
      const int saved[3] = {h.fft.nt[0], h.fft.nt[1], h.fft.nt[2]};
      for (size_t c = 0; c < ncand; ++c) {
        for (int d = 0; d < 3; ++d) h.fft.nt[d] = cand[d][std::min(c, cand[d].size() - 1)];
        Prof pf;
        pf.init();
        pf.on = true;
        hartree_xc<T>(h.geom, h.fft, 2, fields, work, h.fxc<T>(), true, s, nullptr);
        for (int r = 0; r < 3; ++r) hartree_xc<T>(h.geom, h.fft, 2, fields, work, h.fxc<T>(), true, s, &pf);
        pf.collect();
        t[0].push_back(pf.ms[ST_FFT_X_FWD] + pf.ms[ST_FFT_X_INV]);
        t[1].push_back(pf.ms[ST_FFT_Y_FWD] + pf.ms[ST_FFT_Y_INV]);
        t[2].push_back(pf.ms[ST_FFT_Z_POISSON]);
        pf.destroy();
      }
      choice.assign(3, 0);
      for (int d = 0; d < 3; ++d) {
        size_t best = 0;
        for (size_t c = 1; c < ncand; ++c)
          if (c < cand[d].size() && t[d][c] < t[d][best]) best = c;
        choice[d] = cand[d][std::min(best, cand[d].size() - 1)];
        h.fft.nt[d] = saved[d];
      }
      remember(k.str(), choice);
    }
    for (int d = 0; d < 3; ++d) h.fft.nt[d] = choice[d];
  }

  // ---- density: waves per workgroup
  {
    std::ostringstream k;
    k << "density " << prec << " " << h.nt << " " << h.BU << "x" << h.BO << " "
      << h.pair_points << " " << h.nR;
    std::vector<int> choice;
    if (!cached(k.str(), choice)) {
      float best = 1e30f;
      choice = {tl.waves, tl.pbcast};
      for (int pb : {0, 1}) {
        for (int wv : {2, 4, 8}) {
          tl.waves = wv;
          tl.pbcast = pb;
          const float ms = best_ms(s, h.ev0, h.ev1, 3, [&]() {
            density<T>(tl, st, h.BU, h.BO, X, nc, n, n, fields, pstride, 1.0, s);
          });
          if (ms < best) {
            best = ms;
            choice = {wv, pb};
          }
        }
      }
      remember(k.str(), choice);
    }
    h.tiles_uo.waves = choice[0];
    h.tiles_uo.pbcast = choice[1];
  }

  // ---- sparse products: columns per thread and pairs per batch, per plan
  // columns per trial: what an application of n = 4 states passes (the K-shift and the
  // solver's products take the p and q sets together, the coupling sandwich the q set)
  struct PlanRef {
    DevPlan *pl;
    bool left;
    const T *op;
    int64_t out_blocks;
    int cols;
  };
  const PlanRef plans[] = {
      {&h.pT_left, true, h.KcHu.ptr<T>(), h.nR, nc}, {&h.pT_right, false, h.HoKv.ptr<T>(), h.nR, nc},
      {&h.pSw1, true, h.Kc.ptr<T>(), h.nM2, n},      {&h.pSw2, false, h.Kv.ptr<T>(), h.nR, n},
      {&h.pPi1, true, h.KcSu.ptr<T>(), h.nM3, nc},   {&h.pPi2, false, h.SoKv.ptr<T>(), h.nR, nc},
      {&h.pPt1, true, h.KcSuT.ptr<T>(), h.nM5, nc},  {&h.pPt2, false, h.SoKvT.ptr<T>(), h.nM, nc},
      {&h.pCov1, true, h.Su.ptr<T>(), h.nM4, nc},    {&h.pCov2, false, h.So.ptr<T>(), h.nR, nc}};
  // operands: a column set that covers every input block index of these plans
  const int64_t maxblk = std::max({h.nR, h.nM, h.nM2, h.nM3, h.nM4, h.nM5, h.nO});
  const size_t big = (size_t)maxblk * nc * h.E;
  T *A = (T *)h.w_small.get(2 * big * sizeof(T));
  T *B = A + big;
  fill<T>(A, (int64_t)(2 * big), T(0), s);
  for (const PlanRef &r : plans) {
    DevPlan &pl = *r.pl;
    if (pl.nout == 0 || pl.di > 0) continue;   // empty, or the dense MFMA form
    std::ostringstream k;
    k << "spmm " << prec << " " << (r.left ? "L " : "R ") << h.BU << "x" << h.BO << " "
      << pl.nout << " " << pl.npairs << " " << r.cols;
    std::vector<int> choice;
    if (!cached(k.str(), choice)) {
      float best = 1e30f;
      choice = {1, 1};
      const int variants[][2] = {{1, 1}, {1, 2}, {1, 4}, {1, 8}, {2, 1}, {2, 2}, {2, 4}, {4, 1}, {4, 2}};
      for (const auto &v : variants) {
        pl.cw = v[0];
        pl.pb = v[1];
        const float ms = best_ms(s, h.ev0, h.ev1, 3, [&]() {
          if (r.left)
            spmm_left<T>(pl, h.BU, h.BO, r.op, A, r.cols, 0, B, r.cols, 0, r.cols, 1.0, false, s);
          else
            spmm_right<T>(pl, h.BU, h.BO, A, r.cols, 0, r.op, B, r.cols, 0, r.cols, 1.0, false, s);
        });
        if (ms < best) {
          best = ms;
          choice = {v[0], v[1]};
        }
      }
      remember(k.str(), choice);
    }
    pl.cw = choice[0];
    pl.pb = choice[1];
  }

  // ---- dense (complete-pattern) products: output tile shape, per plan
  for (const PlanRef &r : plans) {
    DevPlan &pl = *r.pl;
    if (pl.nout == 0 || pl.di == 0) continue;   // empty, or the sparse form (tuned above)
    std::ostringstream k;
    k << "gemm " << prec << " " << (r.left ? "L " : "R ") << h.BU << "x" << h.BO << " "
      << pl.di << " " << pl.dk << " " << pl.dj << " " << r.cols;
    std::vector<int> choice;
    if (!cached(k.str(), choice)) {
      float best = 1e30f;
      int pick = 0;
      for (int tile : {0, 1, 2}) {
        pl.tile = tile;
        const float ms = best_ms(s, h.ev0, h.ev1, 3, [&]() {
          if (r.left)
            spmm_left<T>(pl, h.BU, h.BO, r.op, A, r.cols, 0, B, r.cols, 0, r.cols, 1.0, false, s);
          else
            spmm_right<T>(pl, h.BU, h.BO, A, r.cols, 0, r.op, B, r.cols, 0, r.cols, 1.0, false, s);
        });
        if (ms < best) {
          best = ms;
          pick = tile;
        }
      }
      choice = {pick};
      remember(k.str(), choice);
    }
    pl.tile = choice[0];
  }
  TD_HIP(hipStreamSynchronize(s));
}

}  // namespace

void autotune(Handle &h) {
  if (h.precision == TDDFT_FP64) tune_typed<double>(h);
  else tune_typed<float>(h);
}

}  // namespace tddft
