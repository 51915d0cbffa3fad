// The per-system handle: device-resident inputs, plans and workspaces.
#pragma once

#include <chrono>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace tddft {

Pattern transpose(const Pattern &A);
Pattern intersect(const Pattern &A, const Pattern &B);
bool fft_factor(int n, std::vector<int> &radix);
void build_fft_plan(FFTPlan &pl, const int n[3], hipStream_t s);

// fixed matrix on device in both working precisions
struct DevMat {
  Pattern pat;
  int br = 0, bc = 0;
  DevBuf<double> d;
  DevBuf<float> f;
  void upload(const HostBsr &m, hipStream_t s);
  template <class T> const T *ptr() const;
};
template <> inline const double *DevMat::ptr<double>() const { return d.p; }
template <> inline const float *DevMat::ptr<float>() const { return f.p; }

// growable device workspace
struct Work {
  DevBuf<unsigned char> buf;
  void *get(size_t bytes) {
    if (bytes > buf.n) buf.alloc(bytes + bytes / 4);
    return buf.p;
  }
};

// allocation-free application: the per-device workspace array (noalloc.hip)
size_t scratch_capacity();
void *scratch_address(int device);

struct Handle {
  int device = 0;
  void *scratch = nullptr;     // this device's copy of the allocation-free workspace
  hipStream_t stream = nullptr;
  tddft_options opts{};
  int precision = TDDFT_FP64;
  int stype = SAMPLE_F64;
  size_t lds_limit = 65536;
  std::string last_error;
  double setup_ms = 0.0;

  // geometry
  int n[3] = {0, 0, 0};
  double L[3] = {0, 0, 0};
  double dV = 0.0;
  GridGeom geom{};
  int nt = 0;

  // blocks
  int nbu = 0, nbo = 0, BU = 0, BO = 0, E = 0;
  std::vector<int> uoff, ooff;
  int n_u = 0, n_o = 0;

  // truncation pattern M of the auxiliary matrices L, response pattern R of P, f
  Pattern M, R;
  int64_t nnzR = 0;            // values of one response kernel in the C-ABI layout
  DevBuf<int64_t> r_voff;      // per R block: offset into the C-ABI values
  DevBuf<int32_t> r_shape;     // per R block: rows | cols << 8
  DevBuf<int32_t> m_in_r;      // per M block: its index in R

  // fixed matrices
  DevMat KcHu, HoKv, KcSu, SoKv, KcSuT, SoKvT, Su, So, Kc, Kv;
  // masked-product plans
  DevPlan pT_left, pT_right, pPi1, pPi2, pPt1, pPt2, pCov1, pCov2, pSw1, pSw2;
  int64_t nM = 0, nR = 0, nM2 = 0, nM3 = 0, nM4 = 0, nM5 = 0, nO = 0;
  bool m_complete = false;     // M holds every (u-block, o-block) pair (then R == M)

  // tiles and partial-sum tables
  DevBuf<int32_t> t_uptr, t_optr, t_pidx_uo, t_pidx_oo;
  DevBuf<double> zero_block;   // kZeroBlock zeros
  DevBuf<int32_t> t_order;     // tiles along a Z-order curve of their coordinates
  DevBuf<int64_t> t_pptr_uo, t_pptr_oo;
  DevBuf<double> us64, os64;
  DevBuf<float> us32, os32;
  DevBuf<__hip_bfloat16> us16, os16;
  DevTiles tiles_uo{}, tiles_oo{};
  int maxrows_uo = 0, maxrows_oo = 0;
  int maxrows_o = 0;           // max over tiles of o-rows (o-atoms * BO)
  DevBuf<int64_t> pa_tbase, pa_cptr;
  DevBuf<int32_t> pa_cidx;
  DevPartials partials{};
  double mean_u_per_tile = 0, mean_o_per_tile = 0;
  int64_t pair_points = 0;     // sum over tiles of (u rows * o rows) * TP (work measure)
  int64_t sample_rows_u = 0, sample_rows_o = 0;
  int64_t samples_u_nz = 0, samples_o_nz = 0, pair_points_nz = 0;  // nonzero-sample counts

  // learned preconditioner: two-atom features of every R block
  int nfeat = 0;
  DevBuf<float> features;      // [nR][nfeat]
  std::vector<int64_t> r_voff_host;
  std::vector<int32_t> r_shape_host;

  // gradient integrals G^alpha_ab = <u_a| d_alpha |o_b> on R (C-ABI layout, alpha-major),
  // for the oscillator strengths
  DevBuf<double> grad_uo;

  // ground state
  DevBuf<double> fxc64;
  DevBuf<float> fxc32;
  FFTPlan fft;

  // workspaces
  Work w_apply, w_pcg, w_small;
  DevBuf<double> partial;      // gram partial sums
  DevBuf<double> small_dev;    // coefficient / result staging
  int max_parts = 1024;        // gram: workgroups of partial sums (x 4096 pairs)

  // second stream of the handle: the K-shift products of an application run there beside
  // the grid pipeline of the coupling term (fork and join through ev_fork / ev_join)
  hipStream_t side = nullptr;
  // private stream of solves on a handle created on the default stream (graph capture)
  hipStream_t solve_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  // timing
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  Prof prof;

  ~Handle();
  template <class T> const T *fxc() const;
  const void *usamp() const;
  const void *osamp() const;
};
template <> inline const double *Handle::fxc<double>() const { return fxc64.p; }
template <> inline const float *Handle::fxc<float>() const { return fxc32.p; }

void create_handle(Handle &h, const tddft_system &sys, const tddft_options &o);

// ---- operator application on column sets (internal precision T) ---------------------------
// Device workspace of one application of n states with elements of `elem` bytes: grid
// fields, FFT work buffer, potential-integral matrices on O, sandwich intermediate on M2
// and the per-tile partial sums, each on a 256-byte boundary.
struct ApplyLayout {
  size_t fields = 0, work = 0, vset = 0, y = 0, part = 0, total = 0;
  int chunk = 0;
};
ApplyLayout apply_layout(const Handle &h, int n, size_t elem);
// X: column set on R with ld columns; p columns [xp0, xp0 + n), q columns [xq0, xq0 + n).
// ws: device workspace of apply_layout(h, n, sizeof(T)).total bytes, or nullptr for the
// handle's own (grown on demand).
template <class T>
void apply_sets(Handle &h, int n, const T *X, int ldx, int xp0, int xq0, T *F, int ldf, int fp0,
                int fq0, bool coupling, bool p_is_q = false, unsigned char *ws = nullptr);
template <class T>
void kshift_sets(Handle &h, int ncol, const T *X, int ldx, int x0, T *F, int ldf, int f0);
// Pi(L) = K^c S^u L S^o K^v: L on M, result on R
template <class T>
void project_sets(Handle &h, int ncol, const T *X, int ldx, int x0, T *F, int ldf, int f0);
template <class T>
void covariant_sets(Handle &h, int ncol, const T *X, int ldx, int x0, T *F, int ldf, int f0);
// Pi^T(Y) = mask_M(S^u K^c Y K^v S^o): Y on R, result on M
template <class T>
void project_t_sets(Handle &h, int ncol, const T *X, int ldx, int x0, T *F, int ldf, int f0);

int pcg_solve(Handle &h, int n, const tddft_options &o, double *omega, double *Pp, double *Pq,
              tddft_stats *stats);
// launch-shape autotuner (tune.cpp): FFT threads per axis, density waves, sparse-product
// columns per thread, timed on the handle's data at creation
void autotune(Handle &h);
// oscillator strengths, velocity form (spectra.hip)
void build_gradient_integrals(Handle &h, const tddft_functions &vir, const tddft_functions &occ);
void oscillator_strengths(Handle &h, int n, const double *omega, const double *Pp, double *f,
                          double *moments);
// Eq. precond by CG in the S metric for n states in the C-ABI layout (complete M)
void precondition(Handle &h, int n, const double *g, double *G, double eps_tol, int max_inner);

}  // namespace tddft
