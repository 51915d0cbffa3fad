// C-ABI entry points of libtddft: argument checks, error conversion, dispatch on the
// handle's precision.  No exception crosses this boundary.
#include <atomic>
#include <new>
#include <set>
#include <thread>

#include "handle.h"
#include "learned.h"

using namespace tddft;

struct tddft_handle {
  Handle h;
};

struct tddft_mlp {
  Mlp m;
};

namespace {
// run f() converting library errors into a status code and the handle's error text
template <class F>
int guarded(std::string &err, F &&f) {
  err.clear();
  try {
    f();
    return TDDFT_OK;
  } catch (const Error &e) {
    err = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    err = "host allocation failed";
    return TDDFT_E_NOMEM;
  } catch (const std::exception &e) {
    err = e.what();
    return TDDFT_E_INVALID;
  } catch (...) {
    err = "unexpected exception";
    return TDDFT_E_INVALID;
  }
}

template <class T>
void project_abi(Handle &h, int n, const double *L, double *P) {
  const size_t eR = (size_t)h.nR * n * h.E, eM = (size_t)h.nM * n * h.E;
  T *A = (T *)h.w_pcg.get((2 * eR + eM) * sizeof(T));
  T *Lm = A + eR, *B = Lm + eM;
  pack<T>(h.nR, h.BU, h.BO, n, L, h.nnzR, h.r_voff.p, h.r_shape.p, A, n, 0, h.stream);
  gather_blocks<T>(h.nM, n * h.E, h.m_in_r.p, A, Lm, h.stream);
  project_sets<T>(h, n, Lm, n, 0, B, n, 0);
  unpack<T>(h.nR, h.BU, h.BO, n, B, n, 0, h.r_voff.p, h.r_shape.p, P, h.nnzR, h.stream);
  TD_HIP(hipStreamSynchronize(h.stream));
}
}  // namespace

static thread_local std::string g_create_error;

extern "C" {

void tddft_default_options(tddft_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = TDDFT_FP64;
  o->xc = TDDFT_XC_ALDA_X;
  o->rho_floor = 1e-10;
  o->coupling_scale = 1.0;
  o->precond = TDDFT_PC_KSDIFF_CG;
  o->eps_tol = 1e-4;
  o->tol_omega = 1e-7;
  o->max_iter = 300;
  o->max_inner = 50;
  o->refresh = 10;
  o->restart = 20;
  o->seed = 0;
  o->model = nullptr;
  o->model_bytes = 0;
  o->stream = nullptr;
  o->eps_loose = 0.0;
  o->tda = 0;
  o->truncate_p = 0;
  o->graphs = 1;
  o->autotune = 1;
  o->density_pbcast = -1;
  o->gemm_tile = -1;
  o->sparse_cw = -1;
  o->sparse_pairs = -1;
}

int tddft_abi_version(void) { return TDDFT_ABI_VERSION; }

const char *tddft_strerror(int code) {
  switch (code) {
    case TDDFT_OK: return "ok";
    case TDDFT_E_INVALID: return "invalid argument";
    case TDDFT_E_NOMEM: return "out of memory";
    case TDDFT_E_DEVICE: return "device error";
    case TDDFT_E_NOT_PD: return "not positive definite";
    case TDDFT_E_NO_CONVERGENCE: return "no convergence";
    case TDDFT_W_FALLBACK: return "learned preconditioner fallback used";
    default: return "unknown status";
  }
}

const char *tddft_last_error(const tddft_handle *h) {
  if (!h) return g_create_error.c_str();
  return h->h.last_error.c_str();
}

int tddft_create(const tddft_system *sys, const tddft_options *opts, tddft_handle **out) {
  g_create_error.clear();
  if (!sys || !out) {
    g_create_error = "null system or output pointer";
    return TDDFT_E_INVALID;
  }
  *out = nullptr;
  tddft_options o;
  if (opts) o = *opts; else tddft_default_options(&o);
  tddft_handle *hd = nullptr;
  try {
    hd = new tddft_handle();
    create_handle(hd->h, *sys, o);
    *out = hd;
    return TDDFT_OK;
  } catch (const Error &e) {
    g_create_error = e.msg;
    delete hd;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_create_error = "host allocation failed";
    delete hd;
    return TDDFT_E_NOMEM;
  } catch (const std::exception &e) {
    g_create_error = e.what();
    delete hd;
    return TDDFT_E_INVALID;
  }
}

int64_t tddft_nnz_p(const tddft_handle *h) { return h ? h->h.nnzR : -1; }

int64_t tddft_response_pattern(const tddft_handle *hd, int64_t *rowptr, int32_t *colind) {
  if (!hd) return TDDFT_E_INVALID;
  const Handle &h = hd->h;
  if (rowptr) std::copy(h.R.rowptr.begin(), h.R.rowptr.end(), rowptr);
  if (colind) std::copy(h.R.col.begin(), h.R.col.end(), colind);
  return h.R.nnzb();
}

int tddft_get_info(const tddft_handle *hd, tddft_info *o) {
  if (!hd || !o) return TDDFT_E_INVALID;
  const Handle &h = hd->h;
  std::memset(o, 0, sizeof(*o));
  for (int d = 0; d < 3; ++d) o->n[d] = h.n[d];
  o->tiles = h.nt;
  o->block_rows = h.BU;
  o->block_cols = h.BO;
  o->max_rows_o = h.maxrows_o;
  o->precision = h.precision;
  o->sample_rows_u = h.sample_rows_u;
  o->sample_rows_o = h.sample_rows_o;
  o->pair_points = h.pair_points;
  o->blocks_m = h.nM;
  o->blocks_r = h.nR;
  o->blocks_o = h.nO;
  o->blocks_m2 = h.nM2;
  o->blocks_m3 = h.nM3;
  o->blocks_m4 = h.nM4;
  o->pairs_kshift = h.pT_left.npairs + h.pT_right.npairs;
  o->pairs_project = h.pPi1.npairs + h.pPi2.npairs;
  o->pairs_project_t = h.pPt1.npairs + h.pPt2.npairs;
  o->pairs_covariant = h.pCov1.npairs + h.pCov2.npairs;
  o->pairs_sandwich = h.pSw1.npairs + h.pSw2.npairs;
  o->partial_pairs = h.partials.total;
  o->setup_ms = h.setup_ms;
  o->samples_u_nz = h.samples_u_nz;
  o->samples_o_nz = h.samples_o_nz;
  o->pair_points_nz = h.pair_points_nz;
  for (int d = 0; d < 3; ++d) o->fft_threads[d] = h.fft.nt[d];
  o->density_waves = h.tiles_uo.waves;
  o->kshift_cw[0] = h.pT_left.cw;
  o->kshift_cw[1] = h.pT_right.cw;
  o->density_pbcast = h.tiles_uo.pbcast;
  o->kshift_tile[0] = h.pT_left.tile;
  o->kshift_tile[1] = h.pT_right.tile;
  o->kshift_pairs[0] = h.pT_left.pb;
  o->kshift_pairs[1] = h.pT_right.pb;
  return TDDFT_OK;
}

int tddft_apply(tddft_handle *hd, int32_t n, const double *Pp, const double *Pq, double *fp,
                double *fq) {
  if (!hd) return TDDFT_E_INVALID;
  Handle &h = hd->h;
  h.last_error.clear();
  if (n < 1 || n > 32 || !Pp || !Pq || !fp || !fq) {
    h.last_error = "tddft_apply: n_states must be in [1, 32] and all arrays non-null";
    return TDDFT_E_INVALID;
  }
  try {
    const int nc = 2 * n;
    auto run = [&](auto tag) {
      using T = decltype(tag);
      const size_t elems = (size_t)h.nR * nc * h.E;
      T *X = (T *)h.w_pcg.get(2 * elems * sizeof(T));
      T *F = X + elems;
      pack<T>(h.nR, h.BU, h.BO, n, Pp, h.nnzR, h.r_voff.p, h.r_shape.p, X, nc, 0, h.stream);
      pack<T>(h.nR, h.BU, h.BO, n, Pq, h.nnzR, h.r_voff.p, h.r_shape.p, X, nc, n, h.stream);
      apply_sets<T>(h, n, X, nc, 0, n, F, nc, 0, n, true);
      unpack<T>(h.nR, h.BU, h.BO, n, F, nc, 0, h.r_voff.p, h.r_shape.p, fp, h.nnzR, h.stream);
      unpack<T>(h.nR, h.BU, h.BO, n, F, nc, n, h.r_voff.p, h.r_shape.p, fq, h.nnzR, h.stream);
      TD_HIP(hipStreamSynchronize(h.stream));
    };
    if (h.precision == TDDFT_FP64) run(double{}); else run(float{});
    return TDDFT_OK;
  } catch (const Error &e) {
    h.last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    h.last_error = "host allocation failed";
    return TDDFT_E_NOMEM;
  } catch (...) {
    h.last_error = "tddft_apply: unexpected exception";
    return TDDFT_E_INVALID;
  }
}

int tddft_apply_noalloc(tddft_handle *hd, int32_t n, const double *Pp, const double *Pq,
                        double *fp, double *fq) {
  if (!hd) return TDDFT_E_INVALID;
  Handle &h = hd->h;
  h.last_error.clear();
  if (n < 1 || n > 32 || !Pp || !Pq || !fp || !fq) {
    h.last_error = "tddft_apply_noalloc: n_states must be in [1, 32] and all arrays non-null";
    return TDDFT_E_INVALID;
  }
  try {
    int dev = -1;
    TD_HIP(hipGetDevice(&dev));
    TD_REQUIRE(dev == h.device && h.scratch, "tddft_apply_noalloc: the handle's GPU must be current");
    const int nc = 2 * n;
    auto run = [&](auto tag) {
      using T = decltype(tag);
      const size_t elems = (size_t)h.nR * nc * h.E;
      const size_t xf = (2 * elems * sizeof(T) + 255) & ~(size_t)255;
      const ApplyLayout lay = apply_layout(h, n, sizeof(T));
      if (xf + lay.total > scratch_capacity())
        throw Error{TDDFT_E_INVALID, "tddft_apply_noalloc: " + std::to_string(n) + " states need " +
                                         std::to_string(xf + lay.total) + " bytes of workspace; the limit is " +
                                         std::to_string(scratch_capacity()) + " (use tddft_apply)"};
      unsigned char *base = (unsigned char *)h.scratch;
      T *X = (T *)base;
      T *F = X + elems;
      pack<T>(h.nR, h.BU, h.BO, n, Pp, h.nnzR, h.r_voff.p, h.r_shape.p, X, nc, 0, h.stream);
      pack<T>(h.nR, h.BU, h.BO, n, Pq, h.nnzR, h.r_voff.p, h.r_shape.p, X, nc, n, h.stream);
      apply_sets<T>(h, n, X, nc, 0, n, F, nc, 0, n, true, false, base + xf);
      unpack<T>(h.nR, h.BU, h.BO, n, F, nc, 0, h.r_voff.p, h.r_shape.p, fp, h.nnzR, h.stream);
      unpack<T>(h.nR, h.BU, h.BO, n, F, nc, n, h.r_voff.p, h.r_shape.p, fq, h.nnzR, h.stream);
      // under stream capture the kernels are recorded into the caller's graph: no wait
      hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
      TD_HIP(hipStreamIsCapturing(h.stream, &cap));
      if (cap == hipStreamCaptureStatusNone) TD_HIP(hipStreamSynchronize(h.stream));
    };
    if (h.precision == TDDFT_FP64) run(double{}); else run(float{});
    return TDDFT_OK;
  } catch (const Error &e) {
    h.last_error = e.msg;
    return e.code;
  } catch (...) {
    h.last_error = "tddft_apply_noalloc: unexpected exception";
    return TDDFT_E_INVALID;
  }
}

int64_t tddft_apply_noalloc_limit(void) { return (int64_t)scratch_capacity(); }

int tddft_oscillator_strengths(tddft_handle *hd, int32_t n, const double *omega, const double *Pp,
                               double *f, double *moments) {
  if (!hd) return TDDFT_E_INVALID;
  Handle &h = hd->h;
  h.last_error.clear();
  if (n < 1 || n > 32 || !omega || !Pp || !f) {
    h.last_error = "tddft_oscillator_strengths: n_states in [1, 32], omega, Pp and f non-null";
    return TDDFT_E_INVALID;
  }
  for (int i = 0; i < n; ++i)
    if (!(omega[i] > 0.0)) {
      h.last_error = "tddft_oscillator_strengths: excitation energies must be positive";
      return TDDFT_E_INVALID;
    }
  return guarded(h.last_error, [&] { oscillator_strengths(h, n, omega, Pp, f, moments); });
}

int tddft_pcg_solve(tddft_handle *hd, int32_t n, const tddft_options *opts, double *omega,
                    double *Pp, double *Pq, tddft_stats *stats) {
  if (!hd) return TDDFT_E_INVALID;
  Handle &h = hd->h;
  h.last_error.clear();
  if (n < 1 || n > 32 || !omega) {
    h.last_error = "tddft_pcg_solve: n_states must be in [1, 32] and omega non-null";
    return TDDFT_E_INVALID;
  }
  if ((Pp == nullptr) != (Pq == nullptr)) {
    h.last_error = "tddft_pcg_solve: give both Pp and Pq or neither";
    return TDDFT_E_INVALID;
  }
  tddft_options o = opts ? *opts : h.opts;
  if (o.precision != h.opts.precision || o.xc != h.opts.xc || o.rho_floor != h.opts.rho_floor ||
      o.coupling_scale != h.opts.coupling_scale || o.tda != h.opts.tda ||
      o.truncate_p != h.opts.truncate_p) {
    h.last_error = "tddft_pcg_solve: precision, xc, rho_floor, coupling_scale, tda and "
                   "truncate_p are fixed at tddft_create and must match the handle's";
    return TDDFT_E_INVALID;
  }
  if (!(o.eps_tol > 0.0) || !(o.tol_omega > 0.0) || o.max_iter < 0 || o.max_inner < 0) {
    h.last_error = "tddft_pcg_solve: tolerances must be positive";
    return TDDFT_E_INVALID;
  }
  if (o.precond == TDDFT_PC_LEARNED && !o.model) o.precond = TDDFT_PC_KSDIFF_CG;
  if (stats) stats->log_len = 0;
  try {
    // the solve runs on the handle's stream; work the caller queued on another stream
    // (the options') is waited for first
    hipStream_t os = (hipStream_t)o.stream;
    if (os != h.stream) {
      TD_HIP(hipEventRecord(h.ev_fork, os));
      TD_HIP(hipStreamWaitEvent(h.stream, h.ev_fork, 0));
    }
    // graph capture needs a stream other than the legacy default one: a handle on the
    // default stream solves on a private non-blocking stream ordered after it (the solve
    // returns only once its stream has finished)
    if (h.stream == nullptr && o.graphs) {
      if (!h.solve_stream) TD_HIP(hipStreamCreateWithFlags(&h.solve_stream, hipStreamNonBlocking));
      TD_HIP(hipEventRecord(h.ev_fork, nullptr));
      TD_HIP(hipStreamWaitEvent(h.solve_stream, h.ev_fork, 0));
      struct Swap {
        Handle &h;
        ~Swap() { h.stream = nullptr; }
      } swap{h};
      h.stream = h.solve_stream;
      const int rc = pcg_solve(h, n, o, omega, Pp, Pq, stats);
      TD_HIP(hipStreamSynchronize(h.solve_stream));
      return rc;
    }
    return pcg_solve(h, n, o, omega, Pp, Pq, stats);
  } catch (const Error &e) {
    h.last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    h.last_error = "host allocation failed";
    return TDDFT_E_NOMEM;
  } catch (const std::exception &e) {
    h.last_error = std::string("tddft_pcg_solve: ") + e.what();
    return TDDFT_E_INVALID;
  } catch (...) {
    h.last_error = "tddft_pcg_solve: unexpected exception";
    return TDDFT_E_INVALID;
  }
}

int tddft_pcg_solve_batched(tddft_handle *const *hs, int32_t n_sys, const int32_t *n_states,
                            const tddft_options *opts, double *const *omega, double *const *Pp,
                            double *const *Pq, tddft_stats *stats, int32_t *status,
                            int32_t max_workers) {
  if (!hs || n_sys < 0 || !n_states || !omega || !status || max_workers < 0) return TDDFT_E_INVALID;
  {
    std::set<const tddft_handle *> seen;
    for (int k = 0; k < n_sys; ++k)
      if (!hs[k] || !seen.insert(hs[k]).second) return TDDFT_E_INVALID;
  }
  const int workers = std::max(1, std::min<int>(n_sys, max_workers > 0 ? max_workers : 16));
  std::atomic<int> next{0};
  auto work = [&]() {
    hipStream_t st = nullptr;
    int dev = -1;
    for (int k = next++; k < n_sys; k = next++) {
      Handle &h = hs[k]->h;
      if (h.device != dev) {
        if (st) (void)hipStreamDestroy(st);
        st = nullptr;
        dev = h.device;
        if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
          h.last_error = "tddft_pcg_solve_batched: stream creation failed";
          status[k] = TDDFT_E_DEVICE;
          st = nullptr;
          dev = -1;
          continue;
        }
      }
      // the handle works on this worker's stream for the solve and gets its own stream
      // back however the solve ends
      struct StreamSwap {
        Handle &h;
        hipStream_t saved;
        StreamSwap(Handle &hh, hipStream_t s) : h(hh), saved(hh.stream) { h.stream = s; }
        ~StreamSwap() { h.stream = saved; }
      } swap(h, st);
      tddft_options o = opts ? *opts : h.opts;
      o.stream = st;
      status[k] = tddft_pcg_solve(hs[k], n_states[k], &o, omega[k], Pp ? Pp[k] : nullptr,
                                  Pq ? Pq[k] : nullptr, stats ? &stats[k] : nullptr);
      (void)hipStreamSynchronize(st);
    }
    if (st) (void)hipStreamDestroy(st);
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < workers; ++t) pool.emplace_back(work);
  work();
  for (auto &t : pool) t.join();
  return TDDFT_OK;
}

void tddft_destroy(tddft_handle *h) { delete h; }

int tddft_project(tddft_handle *hd, int32_t n, const double *L, double *P) {
  if (!hd) return TDDFT_E_INVALID;
  Handle &h = hd->h;
  if (n < 1 || n > 32 || !L || !P) {
    h.last_error = "tddft_project: n_states must be in [1, 32] and arrays non-null";
    return TDDFT_E_INVALID;
  }
  return guarded(h.last_error, [&] {
    if (h.precision == TDDFT_FP64) project_abi<double>(h, n, L, P);
    else project_abi<float>(h, n, L, P);
  });
}

int tddft_precondition(tddft_handle *hd, int32_t n, const double *g, double *G, double eps_tol,
                       int32_t max_inner) {
  if (!hd) return TDDFT_E_INVALID;
  Handle &h = hd->h;
  if (n < 1 || n > 32 || !g || !G || !(eps_tol > 0.0) || max_inner < 0) {
    h.last_error = "tddft_precondition: n_states in [1, 32], non-null arrays, eps_tol > 0";
    return TDDFT_E_INVALID;
  }
  return guarded(h.last_error, [&] { precondition(h, n, g, G, eps_tol, max_inner); });
}

int32_t tddft_n_features(const tddft_handle *h) { return h ? h->h.nfeat : TDDFT_E_INVALID; }

int tddft_block_features(tddft_handle *hd, float *out) {
  if (!hd || !out) return TDDFT_E_INVALID;
  Handle &h = hd->h;
  return guarded(h.last_error, [&] {
    TD_HIP(hipMemcpyAsync(out, h.features.p, (size_t)h.nR * h.nfeat * sizeof(float),
                          hipMemcpyDeviceToDevice, h.stream));
    TD_HIP(hipStreamSynchronize(h.stream));
  });
}

int tddft_guess_targets(tddft_handle *hd, int32_t n, const double *Pq, float *t) {
  if (!hd) return TDDFT_E_INVALID;
  Handle &h = hd->h;
  if (n < 1 || n > 32 || !Pq || !t) {
    h.last_error = "tddft_guess_targets: n_states in [1, 32] and non-null arrays";
    return TDDFT_E_INVALID;
  }
  return guarded(h.last_error, [&] {
    DevBuf<double> w(h.nR);
    block_sqnorm(h.nR, n, h.nnzR, h.r_voff.p, h.r_shape.p, Pq, w.p, h.stream);
    std::vector<double> hw(h.nR);
    TD_HIP(hipMemcpyAsync(hw.data(), w.p, h.nR * sizeof(double), hipMemcpyDeviceToHost, h.stream));
    TD_HIP(hipStreamSynchronize(h.stream));
    double tot = 0.0;
    for (double x : hw) tot += x;
    TD_REQUIRE(tot > 0.0, "tddft_guess_targets: the vectors are zero");
    guess_from_weights(h.nR, w.p, 1.0 / tot, t, h.stream);
    TD_HIP(hipStreamSynchronize(h.stream));
  });
}

// ---- network ---------------------------------------------------------------------------
int tddft_mlp_create(int32_t n_in, int32_t width, int32_t n_out, uint64_t seed, void *stream,
                     tddft_mlp **out) {
  g_create_error.clear();
  if (!out) return TDDFT_E_INVALID;
  *out = nullptr;
  tddft_mlp *m = nullptr;
  try {
    m = new tddft_mlp();
    m->m.init(n_in, width, n_out, (hipStream_t)stream);
    m->m.randomize(seed);
    *out = m;
    return TDDFT_OK;
  } catch (const Error &e) {
    g_create_error = e.msg;
    delete m;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_create_error = "host allocation failed";
    delete m;
    return TDDFT_E_NOMEM;
  }
}

void tddft_mlp_destroy(tddft_mlp *m) { delete m; }

int64_t tddft_mlp_n_params(const tddft_mlp *m) { return m ? m->m.nparams : TDDFT_E_INVALID; }

int tddft_mlp_set_params(tddft_mlp *m, const float *params, const float *mean, const float *stdv) {
  if (!m) return TDDFT_E_INVALID;
  return guarded(m->m.last_error, [&] { m->m.set(params, mean, stdv); });
}

int tddft_mlp_get_params(const tddft_mlp *m, float *params, float *mean, float *stdv) {
  if (!m) return TDDFT_E_INVALID;
  std::string err;
  return guarded(err, [&] { m->m.get(params, mean, stdv); });
}

int tddft_mlp_fit_normalisation(tddft_mlp *m, int64_t rows, const float *X) {
  if (!m) return TDDFT_E_INVALID;
  return guarded(m->m.last_error, [&] { m->m.fit_normalisation(rows, X); });
}

int tddft_mlp_forward(tddft_mlp *m, int64_t rows, const float *X, float *Y) {
  if (!m) return TDDFT_E_INVALID;
  return guarded(m->m.last_error, [&] {
    m->m.forward(rows, X, Y);
    TD_HIP(hipStreamSynchronize(m->m.s));
  });
}

int tddft_mlp_train_step(tddft_mlp *m, int64_t rows, const float *X, const float *g,
                         const float *gstar, const float *t, double loss_scale, double lr,
                         double *loss, float *grad) {
  if (!m) return TDDFT_E_INVALID;
  return guarded(m->m.last_error, [&] {
    const double l = m->m.train_step(rows, X, g, gstar, t, loss_scale, lr, grad);
    if (loss) *loss = l;
  });
}

int tddft_mlp_export(const tddft_mlp *m, void *blob, int64_t cap, int64_t *size) {
  if (!m || !size) return TDDFT_E_INVALID;
  std::string err;
  return guarded(err, [&] {
    const std::vector<unsigned char> b = m->m.blob();
    *size = (int64_t)b.size();
    if (blob) {
      TD_REQUIRE(cap >= (int64_t)b.size(), "tddft_mlp_export: buffer too small");
      std::memcpy(blob, b.data(), b.size());
    }
  });
}

int tddft_mlp_import(const void *blob, int64_t size, void *stream, tddft_mlp **out) {
  g_create_error.clear();
  if (!out) return TDDFT_E_INVALID;
  *out = nullptr;
  tddft_mlp *m = nullptr;
  try {
    m = new tddft_mlp();
    m->m.from_blob(blob, size, (hipStream_t)stream);
    *out = m;
    return TDDFT_OK;
  } catch (const Error &e) {
    g_create_error = e.msg;
    delete m;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_create_error = "host allocation failed";
    delete m;
    return TDDFT_E_NOMEM;
  }
}

const char *tddft_mlp_last_error(const tddft_mlp *m) {
  if (!m) return g_create_error.c_str();
  return m->m.last_error.c_str();
}

int tddft_profile(tddft_handle *hd, int enable) {
  if (!hd) return TDDFT_E_INVALID;
  Handle &h = hd->h;
  try {
    h.prof.collect();
    if (enable) h.prof.init();
    h.prof.reset();
    h.prof.on = enable != 0;
    return TDDFT_OK;
  } catch (const Error &e) {
    h.last_error = e.msg;
    return e.code;
  }
}

int tddft_profile_read(tddft_handle *hd, int cap, double *ms, int64_t *count) {
  if (!hd || cap < 0 || (cap > 0 && (!ms || !count))) return TDDFT_E_INVALID;
  Handle &h = hd->h;
  try {
    h.prof.collect();
  } catch (const Error &e) {
    h.last_error = e.msg;
    return e.code;
  }
  for (int k = 0; k < cap && k < ST_COUNT; ++k) {
    ms[k] = h.prof.ms[k];
    count[k] = h.prof.count[k];
  }
  return ST_COUNT;
}

const char *tddft_profile_stage_name(int k) {
  if (k < 0 || k >= ST_COUNT) return nullptr;
  return kStageNames[k];
}

}  // extern "C"
