// Handle construction (validation, upload, tiles, partial-sum tables, plans, rho0 and f_xc) and the
// operator application of Eq. operator_RPA on column sets.
#include <algorithm>
#include <cmath>
#include <thread>

#include "handle.h"
#include "learned.h"

namespace tddft {

Handle::~Handle() {
  prof.destroy();
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  if (side) (void)hipStreamDestroy(side);
  if (solve_stream) (void)hipStreamDestroy(solve_stream);
}

const void *Handle::usamp() const {
  return stype == SAMPLE_F64 ? (const void *)us64.p
                             : (stype == SAMPLE_F32 ? (const void *)us32.p : (const void *)us16.p);
}
const void *Handle::osamp() const {
  return stype == SAMPLE_F64 ? (const void *)os64.p
                             : (stype == SAMPLE_F32 ? (const void *)os32.p : (const void *)os16.p);
}

void DevMat::upload(const HostBsr &m, hipStream_t s) {
  pat = m.pat;
  br = m.br;
  bc = m.bc;
  d.upload(m.val, s);
  std::vector<float> v(m.val.begin(), m.val.end());
  f.upload(v, s);
  TD_HIP(hipStreamSynchronize(s));
}

template <class F>
static void parallel_for(int64_t n, F fn) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 64 || nt == 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      for (int64_t i = t; i < n; i += nt) fn(i);
    });
  for (auto &x : th) x.join();
}

// ---------------------------------------------------------------------------------------
// validation and conversion of the C-ABI inputs
static std::vector<int> read_offsets(const int32_t *off, int nb, const char *what) {
  TD_REQUIRE(off != nullptr && nb > 0, std::string(what) + ": missing block offsets");
  std::vector<int> v(off, off + nb + 1);
  TD_REQUIRE(v[0] == 0, std::string(what) + ": block offsets must start at 0");
  for (int i = 0; i < nb; ++i) {
    const int sz = v[i + 1] - v[i];
    TD_REQUIRE(sz >= 1 && sz <= 5, std::string(what) + ": block sizes must be 1..5");
  }
  return v;
}

static Pattern read_pattern(const tddft_bsr &m, const char *what) {
  TD_REQUIRE(m.rowptr != nullptr, std::string(what) + ": missing rowptr");
  Pattern p;
  p.nbr = m.nbr;
  p.nbc = m.nbc;
  p.rowptr.assign(m.rowptr, m.rowptr + m.nbr + 1);
  TD_REQUIRE(p.rowptr[0] == 0, std::string(what) + ": rowptr must start at 0");
  for (int i = 0; i < m.nbr; ++i)
    TD_REQUIRE(p.rowptr[i + 1] >= p.rowptr[i], std::string(what) + ": rowptr not monotone");
  const int64_t nnzb = p.rowptr[m.nbr];
  TD_REQUIRE(nnzb == 0 || m.colind != nullptr, std::string(what) + ": missing colind");
  p.col.assign(m.colind, m.colind + nnzb);
  for (int i = 0; i < m.nbr; ++i)
    for (int64_t k = p.rowptr[i]; k < p.rowptr[i + 1]; ++k) {
      TD_REQUIRE(p.col[k] >= 0 && p.col[k] < m.nbc, std::string(what) + ": column out of range");
      TD_REQUIRE(k == p.rowptr[i] || p.col[k] > p.col[k - 1],
                 std::string(what) + ": columns not strictly increasing");
    }
  return p;
}

static HostBsr read_bsr(const tddft_bsr &m, const std::vector<int> &roff,
                        const std::vector<int> &coff, int BR, int BC, const char *what) {
  TD_REQUIRE(m.nbr == (int)roff.size() - 1 && m.nbc == (int)coff.size() - 1,
             std::string(what) + ": block counts differ from the function sets");
  TD_REQUIRE(m.row_off && m.col_off, std::string(what) + ": missing block offsets");
  for (int i = 0; i <= m.nbr; ++i)
    TD_REQUIRE(m.row_off[i] == roff[i], std::string(what) + ": row offsets differ from S");
  for (int i = 0; i <= m.nbc; ++i)
    TD_REQUIRE(m.col_off[i] == coff[i], std::string(what) + ": column offsets differ from S");
  HostBsr h;
  h.pat = read_pattern(m, what);
  h.br = BR;
  h.bc = BC;
  TD_REQUIRE(m.val != nullptr, std::string(what) + ": missing values");
  h.val.assign((size_t)h.pat.nnzb() * BR * BC, 0.0);
  int64_t pos = 0;
  for (int i = 0; i < m.nbr; ++i) {
    const int rs = roff[i + 1] - roff[i];
    for (int64_t k = h.pat.rowptr[i]; k < h.pat.rowptr[i + 1]; ++k) {
      const int j = h.pat.col[k];
      const int cs = coff[j + 1] - coff[j];
      for (int r = 0; r < rs; ++r)
        for (int c = 0; c < cs; ++c) {
          const double v = m.val[pos++];
          TD_REQUIRE(std::isfinite(v), std::string(what) + ": non-finite value");
          h.val[((size_t)k * BR + r) * BC + c] = v;
        }
    }
  }
  return h;
}

static void check_symmetric(const HostBsr &A, const char *what) {
  double amax = 0.0;
  for (double v : A.val) amax = std::max(amax, std::fabs(v));
  const double tol = 1e-10 * std::max(amax, 1e-300);
  for (int i = 0; i < A.pat.nbr; ++i)
    for (int64_t k = A.pat.rowptr[i]; k < A.pat.rowptr[i + 1]; ++k) {
      const int j = A.pat.col[k];
      const int64_t kt = A.pat.find(j, i);
      TD_REQUIRE(kt >= 0, std::string(what) + ": pattern not symmetric");
      for (int r = 0; r < A.br; ++r)
        for (int c = 0; c < A.bc; ++c) {
          const double a = A.val[((size_t)k * A.br + r) * A.bc + c];
          const double b = A.val[((size_t)kt * A.br + c) * A.bc + r];
          TD_REQUIRE(std::fabs(a - b) <= tol, std::string(what) + ": matrix not symmetric");
        }
    }
}

static void check_functions(const tddft_functions &fs, int nfn, const int n[3], const char *what) {
  TD_REQUIRE(fs.n_fn == nfn, std::string(what) + ": n_fn differs from the matrices");
  TD_REQUIRE(fs.origin && fs.extent && fs.off && fs.val, std::string(what) + ": missing arrays");
  TD_REQUIRE(fs.off[0] == 0, std::string(what) + ": off must start at 0");
  for (int f = 0; f < nfn; ++f) {
    int64_t cnt = 1;
    for (int d = 0; d < 3; ++d) {
      const int o = fs.origin[3 * f + d], e = fs.extent[3 * f + d];
      TD_REQUIRE(o >= 0 && o < n[d], std::string(what) + ": origin outside the grid");
      TD_REQUIRE(e >= 1 && e <= n[d], std::string(what) + ": box larger than the cell");
      cnt *= e;
    }
    TD_REQUIRE(fs.off[f + 1] - fs.off[f] == cnt, std::string(what) + ": off inconsistent with extent");
  }
  const int64_t tot = fs.off[nfn];
  for (int64_t i = 0; i < tot; ++i)
    TD_REQUIRE(std::isfinite(fs.val[i]), std::string(what) + ": non-finite sample");
}

// ---------------------------------------------------------------------------------------
// tiles of one function set: atoms touching each tile (nonzero samples) and sample rows
struct HostSetTiles {
  std::vector<int32_t> ptr;      // [nt + 1]
  std::vector<int32_t> atoms;
  std::vector<double> samples;   // [ptr[nt] * B * TP]
  int B = 0;
};

// Tiles (raster numbering x fastest) listed along a Z-order curve of their coordinates:
// consecutive entries are spatial neighbours, so the waves in flight share atom pairs and
// their P blocks stay in cache.
static std::vector<int32_t> tile_order(int ntx, int nty, int ntz) {
  const int64_t nt = (int64_t)ntx * nty * ntz;
  auto spread = [](uint64_t v) {  // bits of v at every third position
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
  };
  std::vector<std::pair<uint64_t, int32_t>> key((size_t)nt);
  for (int z = 0; z < ntz; ++z)
    for (int y = 0; y < nty; ++y)
      for (int x = 0; x < ntx; ++x) {
        const int32_t t = x + ntx * (y + nty * z);
        key[t] = {spread(x) | (spread(y) << 1) | (spread(z) << 2), t};
      }
  std::sort(key.begin(), key.end());
  std::vector<int32_t> order((size_t)nt);
  for (int64_t k = 0; k < nt; ++k) order[k] = key[k].second;
  return order;
}

static HostSetTiles build_set_tiles(const tddft_functions &fs, const std::vector<int> &off,
                                    int B, const int n[3], int ntx, int nty, int ntz) {
  const int nt = ntx * nty * ntz;
  const int nb = (int)off.size() - 1;
  std::vector<int> fatom(fs.n_fn);
  for (int a = 0; a < nb; ++a)
    for (int f = off[a]; f < off[a + 1]; ++f) fatom[f] = a;
  // pass 1: atom lists (functions are ordered by atom, so lists come out sorted)
  std::vector<std::vector<int32_t>> lists(nt);
  std::vector<int32_t> stamp(nt, -1);
  for (int f = 0; f < fs.n_fn; ++f) {
    const int a = fatom[f];
    const int ox = fs.origin[3 * f], oy = fs.origin[3 * f + 1], oz = fs.origin[3 * f + 2];
    const int ex = fs.extent[3 * f], ey = fs.extent[3 * f + 1], ez = fs.extent[3 * f + 2];
    const double *v = fs.val + fs.off[f];
    for (int k = 0; k < ez; ++k) {
      const int z = (oz + k) % n[2];
      for (int j = 0; j < ey; ++j) {
        const int y = (oy + j) % n[1];
        const double *row = v + ((int64_t)k * ey + j) * ex;
        for (int i = 0; i < ex; ++i) {
          if (row[i] == 0.0) continue;
          const int x = (ox + i) % n[0];
          const int t = (x >> 2) + ntx * ((y >> 2) + nty * (z >> 2));
          if (stamp[t] != a) {
            stamp[t] = a;
            lists[t].push_back(a);
          }
        }
      }
    }
  }
  HostSetTiles r;
  r.B = B;
  r.ptr.assign(nt + 1, 0);
  for (int t = 0; t < nt; ++t) r.ptr[t + 1] = r.ptr[t] + (int32_t)lists[t].size();
  r.atoms.resize(r.ptr[nt]);
  for (int t = 0; t < nt; ++t) std::copy(lists[t].begin(), lists[t].end(), r.atoms.begin() + r.ptr[t]);
  r.samples.assign((size_t)r.ptr[nt] * B * TP, 0.0);
  // pass 2: samples (each function writes its own rows)
  parallel_for(fs.n_fn, [&](int64_t f) {
    const int a = fatom[f];
    const int row_in_blk = (int)f - off[a];
    const int ox = fs.origin[3 * f], oy = fs.origin[3 * f + 1], oz = fs.origin[3 * f + 2];
    const int ex = fs.extent[3 * f], ey = fs.extent[3 * f + 1], ez = fs.extent[3 * f + 2];
    const double *v = fs.val + fs.off[f];
    for (int k = 0; k < ez; ++k) {
      const int z = (oz + k) % n[2];
      for (int j = 0; j < ey; ++j) {
        const int y = (oy + j) % n[1];
        const double *row = v + ((int64_t)k * ey + j) * ex;
        for (int i = 0; i < ex; ++i) {
          if (row[i] == 0.0) continue;
          const int x = (ox + i) % n[0];
          const int t = (x >> 2) + ntx * ((y >> 2) + nty * (z >> 2));
          const int p = (x & 3) + 4 * ((y & 3) + 4 * (z & 3));
          const int32_t *lb = r.atoms.data() + r.ptr[t];
          const int32_t *le = r.atoms.data() + r.ptr[t + 1];
          const int idx = (int)(std::lower_bound(lb, le, a) - lb);
          r.samples[((size_t)(r.ptr[t] + idx) * B + row_in_blk) * TP + p] = row[i];
        }
      }
    }
  });
  return r;
}

template <class T>
static void upload_converted(DevBuf<T> &dst, const std::vector<double> &src, hipStream_t s) {
  std::vector<T> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = (T)src[i];
  dst.upload(tmp, s);
  TD_HIP(hipStreamSynchronize(s));
}

static void upload_bf16(DevBuf<__hip_bfloat16> &dst, const std::vector<double> &src, hipStream_t s) {
  std::vector<__hip_bfloat16> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = __float2bfloat16((float)src[i]);  // RNE
  dst.upload(tmp, s);
  TD_HIP(hipStreamSynchronize(s));
}

// Per-tile partial sums of the potential integrals: tile t owns u-rows x o-rows function
// pairs from tbase[t] on, contribution-major ((u-atom i, o-atom j) outer, then the block's
// rows and columns); every (tile, u-atom i, o-atom j) is one contribution to its overlap
// block (I, J) in O, listed per block in tile order (a fixed summation order, so results
// are reproducible).  Tiles write contiguously; the per-block sums gather.
static void build_partials(Handle &h, const HostSetTiles &tu, const HostSetTiles &to,
                           const Pattern &O) {
  const int nt = h.nt;
  std::vector<int64_t> tbase(nt, 0), cptr(O.nnzb() + 1, 0);
  std::vector<int64_t> cblk;   // per (tile, i, j) in order: the O block
  int64_t total = 0;
  for (int t = 0; t < nt; ++t) {
    const int nua = tu.ptr[t + 1] - tu.ptr[t], noa = to.ptr[t + 1] - to.ptr[t];
    tbase[t] = total;
    total += (int64_t)nua * h.BU * noa * h.BO;
    for (int i = 0; i < nua; ++i)
      for (int j = 0; j < noa; ++j) {
        const int64_t k = O.find(tu.atoms[tu.ptr[t] + i], to.atoms[to.ptr[t] + j]);
        TD_REQUIRE(k >= 0, "internal: tile pair outside the overlap pattern");
        cblk.push_back(k);
        cptr[k + 1]++;
      }
  }
  TD_REQUIRE((int64_t)cblk.size() < INT32_MAX, "too many partial-sum contributions");
  for (int64_t k = 0; k < O.nnzb(); ++k) cptr[k + 1] += cptr[k];
  // contribution q (tile order) is function pair q * E of the buffer
  std::vector<int32_t> cidx(cptr[O.nnzb()]);
  std::vector<int64_t> fillp(cptr.begin(), cptr.end() - 1);
  for (size_t q = 0; q < cblk.size(); ++q) cidx[fillp[cblk[q]]++] = (int32_t)q;
  hipStream_t s = h.stream;
  h.pa_tbase.upload(tbase, s);
  h.pa_cptr.upload(cptr, s);
  h.pa_cidx.upload(cidx, s);
  TD_HIP(hipStreamSynchronize(s));
  h.partials = DevPartials{total, h.pa_tbase.p, h.pa_cptr.p, h.pa_cidx.p};
}

// ---------------------------------------------------------------------------------------
void create_handle(Handle &h, const tddft_system &sys, const tddft_options &o) {
  const auto t0 = std::chrono::steady_clock::now();
  h.opts = o;
  h.precision = o.precision;
  TD_REQUIRE(o.precision >= TDDFT_FP64 && o.precision <= TDDFT_BF16_GRID, "unknown precision mode");
  TD_REQUIRE(o.density_pbcast >= -1 && o.density_pbcast <= 1, "density_pbcast must be -1, 0 or 1");
  TD_REQUIRE(o.gemm_tile >= -1 && o.gemm_tile <= 2, "gemm_tile must be -1, 0, 1 or 2");
  {
    const int cw = o.sparse_cw, pb = o.sparse_pairs;
    const bool tuned = cw == -1 && pb == -1;
    const bool known = (cw == 1 && (pb == 1 || pb == 2 || pb == 4 || pb == 8)) ||
                       (cw == 2 && (pb == 1 || pb == 2 || pb == 4)) || (cw == 4 && (pb == 1 || pb == 2));
    TD_REQUIRE(tuned || known,
               "sparse_cw/sparse_pairs must both be -1 or one of (1,1) (1,2) (1,4) (1,8) (2,1) (2,2) (2,4) (4,1) (4,2)");
  }
  TD_REQUIRE(o.xc >= TDDFT_XC_ALDA_X && o.xc <= TDDFT_HXC_NONE, "unknown coupling kernel");
  h.stype = o.precision == TDDFT_FP64 ? SAMPLE_F64 : (o.precision == TDDFT_FP32 ? SAMPLE_F32 : SAMPLE_BF16);
  h.stream = (hipStream_t)o.stream;
  hipStream_t s = h.stream;

  // ---- geometry
  for (int d = 0; d < 3; ++d) {
    TD_REQUIRE(sys.n[d] >= 2 && sys.n[d] <= 4096, "grid dimensions must be in [2, 4096]");
    TD_REQUIRE(std::isfinite(sys.L[d]) && sys.L[d] > 0.0, "cell lengths must be positive");
    h.n[d] = sys.n[d];
    h.L[d] = sys.L[d];
    std::vector<int> rad;
    TD_REQUIRE(fft_factor(sys.n[d], rad), "grid dimensions must be products of 2, 3, 5 and 7");
  }
  h.dV = (h.L[0] / h.n[0]) * (h.L[1] / h.n[1]) * (h.L[2] / h.n[2]);
  h.geom.n[0] = h.n[0]; h.geom.n[1] = h.n[1]; h.geom.n[2] = h.n[2];
  h.geom.L[0] = h.L[0]; h.geom.L[1] = h.L[1]; h.geom.L[2] = h.L[2];
  h.geom.ntx = (h.n[0] + TILE - 1) / TILE;
  h.geom.nty = (h.n[1] + TILE - 1) / TILE;
  h.geom.ntz = (h.n[2] + TILE - 1) / TILE;
  h.nt = h.geom.ntx * h.geom.nty * h.geom.ntz;

  // ---- blocks and matrices
  h.ooff = read_offsets(sys.S_o.row_off, sys.S_o.nbr, "S_o");
  h.uoff = read_offsets(sys.S_u.row_off, sys.S_u.nbr, "S_u");
  h.nbo = sys.S_o.nbr;
  h.nbu = sys.S_u.nbr;
  h.n_o = h.ooff.back();
  h.n_u = h.uoff.back();
  int bo = 0, bu = 0;
  for (int i = 0; i < h.nbo; ++i) bo = std::max(bo, h.ooff[i + 1] - h.ooff[i]);
  for (int i = 0; i < h.nbu; ++i) bu = std::max(bu, h.uoff[i + 1] - h.uoff[i]);
  // padded shapes supported by the kernels: (1,1) (2,2) (3,2) (3,3) (5,2) (4,4); every
  // block is copied into a padded one, so the padded shape must cover the largest block
  if (bu <= 1 && bo <= 1) { h.BU = 1; h.BO = 1; }
  else if (bu <= 2 && bo <= 2) { h.BU = 2; h.BO = 2; }
  else if (bu <= 3 && bo <= 2) { h.BU = 3; h.BO = 2; }
  else if (bu <= 3 && bo <= 3) { h.BU = 3; h.BO = 3; }
  else if (bu <= 5 && bo <= 2) { h.BU = 5; h.BO = 2; }
  else { h.BU = 4; h.BO = 4; }
  TD_REQUIRE(bu <= h.BU && bo <= h.BO,
             "unsupported block sizes: at most 4 u- and 4 o-functions per atom, or 5 and 2");
  h.E = h.BU * h.BO;

  HostBsr So = read_bsr(sys.S_o, h.ooff, h.ooff, h.BO, h.BO, "S_o");
  HostBsr Ho = read_bsr(sys.H_o, h.ooff, h.ooff, h.BO, h.BO, "H_o");
  HostBsr Kv = read_bsr(sys.K_v, h.ooff, h.ooff, h.BO, h.BO, "K_v");
  HostBsr Su = read_bsr(sys.S_u, h.uoff, h.uoff, h.BU, h.BU, "S_u");
  HostBsr Hu = read_bsr(sys.H_u, h.uoff, h.uoff, h.BU, h.BU, "H_u");
  HostBsr Kc = read_bsr(sys.K_c, h.uoff, h.uoff, h.BU, h.BU, "K_c");
  check_symmetric(So, "S_o");
  check_symmetric(Ho, "H_o");
  check_symmetric(Kv, "K_v");
  check_symmetric(Su, "S_u");
  check_symmetric(Hu, "H_u");
  check_symmetric(Kc, "K_c");
  for (int i = 0; i < h.nbo; ++i) TD_REQUIRE(So.pat.find(i, i) >= 0, "S_o: missing diagonal block");
  for (int i = 0; i < h.nbu; ++i) TD_REQUIRE(Su.pat.find(i, i) >= 0, "S_u: missing diagonal block");

  TD_REQUIRE(sys.M.nbr == h.nbu && sys.M.nbc == h.nbo, "M: must be u-blocks x o-blocks");
  if (sys.M.row_off)
    for (int i = 0; i <= h.nbu; ++i) TD_REQUIRE(sys.M.row_off[i] == h.uoff[i], "M: row offsets differ from S_u");
  if (sys.M.col_off)
    for (int i = 0; i <= h.nbo; ++i) TD_REQUIRE(sys.M.col_off[i] == h.ooff[i], "M: column offsets differ from S_o");
  h.M = read_pattern(sys.M, "M");
  h.nM = h.M.nnzb();
  TD_REQUIRE(h.nM > 0, "M: empty pattern");
  check_functions(sys.occ, h.n_o, h.n, "occ");
  check_functions(sys.vir, h.n_u, h.n, "vir");

  // ---- every host-side check passed: from here on the device is used
  TD_HIP(hipGetDevice(&h.device));
  h.scratch = scratch_address(h.device);
  int lds = 0;
  TD_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h.device));
  h.lds_limit = (size_t)lds;
  TD_HIP(hipEventCreate(&h.ev0));
  TD_HIP(hipEventCreate(&h.ev1));
  TD_HIP(hipStreamCreateWithFlags(&h.side, hipStreamNonBlocking));
  TD_HIP(hipEventCreateWithFlags(&h.ev_fork, hipEventDisableTiming));
  TD_HIP(hipEventCreateWithFlags(&h.ev_join, hipEventDisableTiming));

  // ---- fixed products (exact, host FP64) and the response pattern R of K^c S^u L S^o K^v
  HostBsr KcHu = host_product(Kc, Hu, product_pattern(Kc.pat, Hu.pat));
  HostBsr HoKv = host_product(Ho, Kv, product_pattern(Ho.pat, Kv.pat));
  HostBsr KcSu = host_product(Kc, Su, product_pattern(Kc.pat, Su.pat));
  HostBsr SoKv = host_product(So, Kv, product_pattern(So.pat, Kv.pat));
  // linear-scaling mode (Sec. IV.C): the response kernels are truncated to M as well
  h.R = o.truncate_p ? h.M : product_pattern(product_pattern(KcSu.pat, h.M), SoKv.pat);
  h.nR = h.R.nnzb();
  {
    std::vector<int64_t> voff(h.nR);
    std::vector<int32_t> shape(h.nR);
    int64_t pos = 0;
    for (int i = 0; i < h.nbu; ++i)
      for (int64_t k = h.R.rowptr[i]; k < h.R.rowptr[i + 1]; ++k) {
        const int j = h.R.col[k];
        const int rs = h.uoff[i + 1] - h.uoff[i], cs = h.ooff[j + 1] - h.ooff[j];
        voff[k] = pos;
        shape[k] = rs | (cs << 8);
        pos += rs * cs;
      }
    h.nnzR = pos;
    h.r_voff.upload(voff, s);
    h.r_shape.upload(shape, s);
    h.r_voff_host = voff;
    h.r_shape_host = shape;
    std::vector<int32_t> mir(h.nM);
    for (int i = 0; i < h.nbu; ++i)
      for (int64_t k = h.M.rowptr[i]; k < h.M.rowptr[i + 1]; ++k) {
        const int64_t r = h.R.find(i, h.M.col[k]);
        TD_REQUIRE(r >= 0, "M is not contained in the response pattern (missing diagonal blocks)");
        mir[k] = (int32_t)r;
      }
    h.m_in_r.upload(mir, s);
    h.m_complete = h.nM == (int64_t)h.nbu * h.nbo;
    if (h.m_complete) TD_REQUIRE(h.R.col == h.M.col && h.nR == h.nM, "complete M must equal R");
  }

  build_features(h, Su, Hu, So, Ho, sys);
  build_gradient_integrals(h, sys.vir, sys.occ);

  // ---- functions and tiles
  HostSetTiles tu = build_set_tiles(sys.vir, h.uoff, h.BU, h.n, h.geom.ntx, h.geom.nty, h.geom.ntz);
  HostSetTiles to = build_set_tiles(sys.occ, h.ooff, h.BO, h.n, h.geom.ntx, h.geom.nty, h.geom.ntz);
  const int nt = h.nt;
  std::vector<int64_t> pptr_uo(nt + 1, 0), pptr_oo(nt + 1, 0);
  std::vector<int32_t> pidx_uo, pidx_oo;
  std::vector<std::vector<int32_t>> orows(h.nbu);
  h.maxrows_uo = h.maxrows_oo = 0;
  int maxpairs_uo = 0, maxpairs_oo = 0, maxrows_r = 0;
  int64_t pp = 0;
  for (int t = 0; t < nt; ++t) {
    const int nua = tu.ptr[t + 1] - tu.ptr[t], noa = to.ptr[t + 1] - to.ptr[t];
    h.maxrows_uo = std::max(h.maxrows_uo, nua * h.BU + noa * h.BO);
    h.maxrows_oo = std::max(h.maxrows_oo, 2 * noa * h.BO);
    maxpairs_uo = std::max(maxpairs_uo, nua * noa);
    maxpairs_oo = std::max(maxpairs_oo, noa * noa);
    maxrows_r = std::max(maxrows_r, noa * h.BO);
    pp += (int64_t)nua * h.BU * noa * h.BO;
    for (int i = 0; i < nua; ++i)
      for (int j = 0; j < noa; ++j) {
        const int I = tu.atoms[tu.ptr[t] + i], J = to.atoms[to.ptr[t] + j];
        pidx_uo.push_back((int32_t)h.R.find(I, J));
        orows[I].push_back(J);
      }
    for (int i = 0; i < noa; ++i)
      for (int j = 0; j < noa; ++j)
        pidx_oo.push_back((int32_t)Kv.pat.find(to.atoms[to.ptr[t] + i], to.atoms[to.ptr[t] + j]));
    pptr_uo[t + 1] = (int64_t)pidx_uo.size();
    pptr_oo[t + 1] = (int64_t)pidx_oo.size();
  }
  pidx_uo.insert(pidx_uo.end(), kPairPad, -1);
  pidx_oo.insert(pidx_oo.end(), kPairPad, -1);
  h.pair_points = pp * TP;
  h.sample_rows_u = (int64_t)tu.ptr[nt] * h.BU;
  h.sample_rows_o = (int64_t)to.ptr[nt] * h.BO;
  // work of the method itself: per grid point, (u-functions nonzero there) x (o-functions
  // nonzero there), without the padding of tiles and blocks
  {
    int64_t nzu = 0, nzo = 0, ppnz = 0;
    for (int t = 0; t < nt; ++t) {
      int cu[TP] = {}, co[TP] = {};
      for (int64_t r = (int64_t)tu.ptr[t] * h.BU; r < (int64_t)tu.ptr[t + 1] * h.BU; ++r)
        for (int p = 0; p < TP; ++p) cu[p] += tu.samples[(size_t)r * TP + p] != 0.0;
      for (int64_t r = (int64_t)to.ptr[t] * h.BO; r < (int64_t)to.ptr[t + 1] * h.BO; ++r)
        for (int p = 0; p < TP; ++p) co[p] += to.samples[(size_t)r * TP + p] != 0.0;
      for (int p = 0; p < TP; ++p) {
        nzu += cu[p];
        nzo += co[p];
        ppnz += (int64_t)cu[p] * co[p];
      }
    }
    h.samples_u_nz = nzu;
    h.samples_o_nz = nzo;
    h.pair_points_nz = ppnz;
  }
  h.mean_u_per_tile = (double)tu.ptr[nt] / nt;
  h.mean_o_per_tile = (double)to.ptr[nt] / nt;
  // pattern O: (u-atom, o-atom) pairs sharing a tile
  Pattern O;
  O.nbr = h.nbu;
  O.nbc = h.nbo;
  O.rowptr.assign(h.nbu + 1, 0);
  for (int I = 0; I < h.nbu; ++I) {
    auto &r = orows[I];
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    O.col.insert(O.col.end(), r.begin(), r.end());
    O.rowptr[I + 1] = (int64_t)O.col.size();
    std::vector<int32_t>().swap(r);
  }
  h.nO = O.nnzb();

  h.t_uptr.upload(tu.ptr, s);
  h.t_optr.upload(to.ptr, s);
  h.t_pptr_uo.upload(pptr_uo, s);
  h.t_pptr_oo.upload(pptr_oo, s);
  h.t_pidx_uo.upload(pidx_uo, s);
  h.t_pidx_oo.upload(pidx_oo, s);
  TD_HIP(hipStreamSynchronize(s));
  upload_converted(h.os64, to.samples, s);   // FP64 o-samples for rho0 (freed below if unused)
  if (h.stype == SAMPLE_F64) {
    upload_converted(h.us64, tu.samples, s);
  } else if (h.stype == SAMPLE_F32) {
    upload_converted(h.us32, tu.samples, s);
    upload_converted(h.os32, to.samples, s);
  } else {
    upload_bf16(h.us16, tu.samples, s);
    upload_bf16(h.os16, to.samples, s);
  }
  const std::vector<double> zeros(kZeroBlock, 0.0);
  h.zero_block.upload(zeros, s);
  const std::vector<int32_t> order = tile_order(h.geom.ntx, h.geom.nty, h.geom.ntz);
  h.t_order.upload(order, s);
  TD_HIP(hipStreamSynchronize(s));
  h.tiles_uo = DevTiles{nt, h.maxrows_uo, maxpairs_uo, maxrows_r, h.t_uptr.p, h.t_optr.p,
                        h.t_pptr_uo.p, h.t_pidx_uo.p, h.usamp(), h.osamp(), h.lds_limit};
  h.tiles_oo = DevTiles{nt, h.maxrows_oo, maxpairs_oo, maxrows_r, h.t_optr.p, h.t_optr.p,
                        h.t_pptr_oo.p, h.t_pidx_oo.p, h.os64.p, h.os64.p, h.lds_limit};
  h.tiles_uo.zero = h.tiles_oo.zero = h.zero_block.p;
  h.tiles_uo.order = h.tiles_oo.order = h.t_order.p;
  TD_REQUIRE((size_t)maxrows_r * TP * sizeof(double) <= h.lds_limit,
             "too many functions per grid tile for the LDS budget");

  h.maxrows_o = maxrows_r;
  build_partials(h, tu, to, O);

  // ---- plans
  HostBsr KcSuT = host_transpose(KcSu);
  HostBsr SoKvT = host_transpose(SoKv);
  h.KcHu.upload(KcHu, s);
  h.HoKv.upload(HoKv, s);
  h.KcSu.upload(KcSu, s);
  h.SoKv.upload(SoKv, s);
  h.KcSuT.upload(KcSuT, s);
  h.SoKvT.upload(SoKvT, s);
  h.Su.upload(Su, s);
  h.So.upload(So, s);
  h.Kc.upload(Kc, s);
  h.Kv.upload(Kv, s);
  const Pattern &M = h.M;
  const Pattern &R = h.R;
  h.pT_left.upload(plan_product(KcHu.pat, R, R), s);
  h.pT_right.upload(plan_product(R, HoKv.pat, R), s);
  Pattern M3 = intersect(product_pattern(KcSu.pat, M), product_pattern(R, transpose(SoKv.pat)));
  h.nM3 = M3.nnzb();
  h.pPi1.upload(plan_product(KcSu.pat, M, M3), s);
  h.pPi2.upload(plan_product(M3, SoKv.pat, R), s);
  Pattern M5 = intersect(product_pattern(KcSuT.pat, R), product_pattern(M, transpose(SoKvT.pat)));
  h.nM5 = M5.nnzb();
  h.pPt1.upload(plan_product(KcSuT.pat, R, M5), s);
  h.pPt2.upload(plan_product(M5, SoKvT.pat, M), s);
  Pattern M4 = intersect(product_pattern(Su.pat, R), product_pattern(R, transpose(So.pat)));
  h.nM4 = M4.nnzb();
  h.pCov1.upload(plan_product(Su.pat, R, M4), s);
  h.pCov2.upload(plan_product(M4, So.pat, R), s);
  Pattern M2 = intersect(product_pattern(Kc.pat, O), product_pattern(R, transpose(Kv.pat)));
  h.nM2 = M2.nnzb();
  h.pSw1.upload(plan_product(Kc.pat, O, M2), s);
  h.pSw2.upload(plan_product(M2, Kv.pat, R), s);

  // ---- FFT plan, rho0 = 2 sum o K^v o and f_xc (FP64 from FP64 samples)
  build_fft_plan(h.fft, h.n, s);
  TD_REQUIRE(fft_lds_bytes(h.fft, h.precision == TDDFT_FP64 ? 16 : 8) <= h.lds_limit,
             "grid dimensions too large for the FFT's line buffers in LDS");
  h.partial.alloc((size_t)h.max_parts * 4096);
  h.small_dev.alloc(8192);
  {
    DevBuf<double> rho((size_t)nt * TP * 2);
    density<double>(h.tiles_oo, SAMPLE_F64, h.BO, h.BO, h.Kv.d.p, 1, 0, 1, rho.p,
                    (int64_t)nt * TP * 2, 2.0, s);
    h.fxc64.alloc((size_t)nt * TP);
    alda_kernel<double>((int64_t)nt * TP, rho.p, o.rho_floor, h.fxc64.p, s);
    TD_HIP(hipStreamSynchronize(s));
    if (h.stype != SAMPLE_F64) {
      std::vector<double> tmp((size_t)nt * TP);
      TD_HIP(hipMemcpy(tmp.data(), h.fxc64.p, tmp.size() * sizeof(double), hipMemcpyDeviceToHost));
      upload_converted(h.fxc32, tmp, s);
    }
  }
  if (h.stype != SAMPLE_F64) {
    h.os64.release();
    h.tiles_oo.usamp = h.tiles_oo.osamp = nullptr;
  }
  if (o.autotune) autotune(h);
  if (o.density_pbcast >= 0) h.tiles_uo.pbcast = o.density_pbcast;
  if (o.gemm_tile >= 0)
    for (DevPlan *pl : {&h.pT_left, &h.pT_right, &h.pSw1, &h.pSw2, &h.pPi1, &h.pPi2, &h.pPt1,
                        &h.pPt2, &h.pCov1, &h.pCov2})
      pl->tile = o.gemm_tile;
  if (o.sparse_cw > 0)
    for (DevPlan *pl : {&h.pT_left, &h.pT_right, &h.pSw1, &h.pSw2, &h.pPi1, &h.pPi2, &h.pPt1,
                        &h.pPt2, &h.pCov1, &h.pCov2}) {
      pl->cw = o.sparse_cw;
      pl->pb = o.sparse_pairs;
    }
  h.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------------------------------
template <class T>
static int stype_of(const Handle &h) {
  return std::is_same<T, double>::value ? SAMPLE_F64 : h.stype;
}

template <class T>
static void kshift_on(Handle &h, hipStream_t s, int ncol, const T *X, int ldx, int x0, T *F, int ldf,
                      int f0) {
  h.prof.begin(ST_KSHIFT_LEFT, s);
  spmm_left<T>(h.pT_left, h.BU, h.BO, h.KcHu.ptr<T>(), X, ldx, x0, F, ldf, f0, ncol, 1.0, false, s);
  h.prof.end(ST_KSHIFT_LEFT, s);
  h.prof.begin(ST_KSHIFT_RIGHT, s);
  spmm_right<T>(h.pT_right, h.BU, h.BO, X, ldx, x0, h.HoKv.ptr<T>(), F, ldf, f0, ncol, -1.0, true, s);
  h.prof.end(ST_KSHIFT_RIGHT, s);
}

template <class T>
void kshift_sets(Handle &h, int ncol, const T *X, int ldx, int x0, T *F, int ldf, int f0) {
  kshift_on<T>(h, h.stream, ncol, X, ldx, x0, F, ldf, f0);
}

template <class T>
void project_sets(Handle &h, int ncol, const T *X, int ldx, int x0, T *F, int ldf, int f0) {
  T *Y = (T *)h.w_small.get((size_t)h.nM3 * ncol * h.E * sizeof(T));
  h.prof.begin(ST_PROJECT, h.stream);
  spmm_left<T>(h.pPi1, h.BU, h.BO, h.KcSu.ptr<T>(), X, ldx, x0, Y, ncol, 0, ncol, 1.0, false, h.stream);
  spmm_right<T>(h.pPi2, h.BU, h.BO, Y, ncol, 0, h.SoKv.ptr<T>(), F, ldf, f0, ncol, 1.0, false, h.stream);
  h.prof.end(ST_PROJECT, h.stream);
}

template <class T>
void project_t_sets(Handle &h, int ncol, const T *X, int ldx, int x0, T *F, int ldf, int f0) {
  T *Y = (T *)h.w_small.get((size_t)h.nM5 * ncol * h.E * sizeof(T));
  h.prof.begin(ST_PROJECT_T, h.stream);
  spmm_left<T>(h.pPt1, h.BU, h.BO, h.KcSuT.ptr<T>(), X, ldx, x0, Y, ncol, 0, ncol, 1.0, false, h.stream);
  spmm_right<T>(h.pPt2, h.BU, h.BO, Y, ncol, 0, h.SoKvT.ptr<T>(), F, ldf, f0, ncol, 1.0, false, h.stream);
  h.prof.end(ST_PROJECT_T, h.stream);
}

template <class T>
void covariant_sets(Handle &h, int ncol, const T *X, int ldx, int x0, T *F, int ldf, int f0) {
  T *Y = (T *)h.w_small.get((size_t)h.nM4 * ncol * h.E * sizeof(T));
  h.prof.begin(ST_COVARIANT, h.stream);
  spmm_left<T>(h.pCov1, h.BU, h.BO, h.Su.ptr<T>(), X, ldx, x0, Y, ncol, 0, ncol, 1.0, false, h.stream);
  spmm_right<T>(h.pCov2, h.BU, h.BO, Y, ncol, 0, h.So.ptr<T>(), F, ldf, f0, ncol, 1.0, false, h.stream);
  h.prof.end(ST_COVARIANT, h.stream);
}

ApplyLayout apply_layout(const Handle &h, int n, size_t elem) {
  // sub-buffers start on 256-byte boundaries (vector loads of the partial sums)
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const int npair = (n + 1) / 2;
  ApplyLayout l;
  l.fields = al((size_t)npair * h.nt * TP * 2 * elem);
  l.work = al((size_t)npair * h.n[0] * h.n[1] * h.n[2] * 2 * elem);
  l.vset = al((size_t)h.nO * n * h.E * elem);
  l.y = al((size_t)h.nM2 * n * h.E * elem);
  // potential integrals in chunks of at most 8 states (chunk starts stay even), which
  // bounds the per-tile partial-sum buffer
  l.chunk = std::min(n, 8);
  l.part = al((size_t)h.partials.total * l.chunk * elem);
  l.total = l.fields + l.work + l.vset + l.y + l.part + 1024;
  return l;
}

template <class T>
void apply_sets(Handle &h, int n, const T *X, int ldx, int xp0, int xq0, T *F, int ldf, int fp0,
                int fq0, bool coupling, bool p_is_q, unsigned char *ws) {
  hipStream_t s = h.stream;
  // The K-shift term writes F and the coupling term adds into it last; up to that add the
  // two read only X. With a coupling term the K-shift products run on the handle's second
  // stream, forked once the first response density is queued on s (so that they overlap
  // the FFTs, the integrals and their reduce rather than the density) and joined before the
  // first add.  While stage profiling is on, everything stays on s, so that each stage's
  // event time is its own.
  const bool with_coupling = coupling && h.opts.xc != TDDFT_HXC_NONE;
  const bool fork = with_coupling && !h.prof.on;
  auto kshift_all = [&](hipStream_t ks) {
    if (xq0 == xp0 + n && fq0 == fp0 + n) {
      kshift_on<T>(h, ks, 2 * n, X, ldx, xp0, F, ldf, fp0);
    } else {
      kshift_on<T>(h, ks, n, X, ldx, xp0, F, ldf, fp0);
      kshift_on<T>(h, ks, n, X, ldx, xq0, F, ldf, fq0);
    }
  };
  if (!fork) kshift_all(s);
  if (!with_coupling) return;
  bool forked = !fork, joined = !fork;
  auto fork_kshift = [&]() {
    if (forked) return;
    TD_HIP(hipEventRecord(h.ev_fork, s));
    TD_HIP(hipStreamWaitEvent(h.side, h.ev_fork, 0));
    kshift_all(h.side);
    TD_HIP(hipEventRecord(h.ev_join, h.side));
    forked = true;
  };
  const int npair = (n + 1) / 2;
  const int64_t pstride = (int64_t)h.nt * TP * 2;
  const ApplyLayout lay = apply_layout(h, n, sizeof(T));
  const int chunk = lay.chunk;
  const size_t bytes_f = lay.fields, bytes_w = lay.work, bytes_v = lay.vset, bytes_y = lay.y;
  unsigned char *base = ws ? ws : (unsigned char *)h.w_apply.get(lay.total);
  T *fields = (T *)base;
  T *work = (T *)(base + bytes_f);
  T *Vset = (T *)(base + bytes_f + bytes_w);
  T *Y = (T *)(base + bytes_f + bytes_w + bytes_v);
  T *part = (T *)(base + bytes_f + bytes_w + bytes_v + bytes_y);
  const int st = stype_of<T>(h);
  DevTiles tl = h.tiles_uo;
  tl.usamp = h.usamp();
  tl.osamp = h.osamp();
  // the coupling term K^c V_SCF[X] K^v of a group of n columns, added to F columns f0s
  // with factor: full TDDFT 2 s on the q half (A + B = D + 2K); Tamm-Dancoff s on both
  // halves (A = D + K), computed once when p and q hold the same vectors
  auto couple = [&](int xc0, std::initializer_list<int> f0s, double factor) {
    h.prof.begin(ST_DENSITY, s);
    density<T>(tl, st, h.BU, h.BO, X, ldx, xc0, n, fields, pstride, 1.0, s);
    h.prof.end(ST_DENSITY, s);
    fork_kshift();
    hartree_xc<T>(h.geom, h.fft, npair, fields, work, h.fxc<T>(), h.opts.xc == TDDFT_XC_ALDA_X, s, &h.prof);
    for (int s0 = 0; s0 < n; s0 += chunk) {
      const int ns = std::min(chunk, n - s0);
      // Vout columns s0.. of a set with n columns: offset the pointer by s0 * E
      potential_integrals<T>(tl, h.partials, st, h.BU, h.BO, fields + (int64_t)(s0 / 2) * pstride, pstride,
                             ns, part, Vset + (size_t)s0 * h.E, n, h.nO, h.dV, s, &h.prof);
    }
    h.prof.begin(ST_SANDWICH_LEFT, s);
    spmm_left<T>(h.pSw1, h.BU, h.BO, h.Kc.ptr<T>(), Vset, n, 0, Y, n, 0, n, 1.0, false, s);
    h.prof.end(ST_SANDWICH_LEFT, s);
    if (!joined) {
      TD_HIP(hipStreamWaitEvent(s, h.ev_join, 0));
      joined = true;
    }
    for (int f0 : f0s) {
      h.prof.begin(ST_SANDWICH_RIGHT, s);
      spmm_right<T>(h.pSw2, h.BU, h.BO, Y, n, 0, h.Kv.ptr<T>(), F, ldf, f0, n, factor, true, s);
      h.prof.end(ST_SANDWICH_RIGHT, s);
    }
  };
  if (!h.opts.tda) {
    couple(xq0, {fq0}, 2.0 * h.opts.coupling_scale);
  } else if (p_is_q) {
    couple(xq0, {fp0, fq0}, h.opts.coupling_scale);
  } else {
    couple(xp0, {fp0}, h.opts.coupling_scale);
    couple(xq0, {fq0}, h.opts.coupling_scale);
  }
}

#define TD_INST_APPLY(T)                                                                      \
  template void apply_sets<T>(Handle &, int, const T *, int, int, int, T *, int, int, int, bool, bool, \
                              unsigned char *);                                              \
  template void kshift_sets<T>(Handle &, int, const T *, int, int, T *, int, int);             \
  template void project_sets<T>(Handle &, int, const T *, int, int, T *, int, int);            \
  template void project_t_sets<T>(Handle &, int, const T *, int, int, T *, int, int);          \
  template void covariant_sets<T>(Handle &, int, const T *, int, int, T *, int, int);

TD_INST_APPLY(double)
TD_INST_APPLY(float)

}  // namespace tddft
