// Launch wrappers of the HIP kernels (host-callable).
#pragma once

#include "internal.h"

namespace tddft {

// Division by a run-time divisor d through a host-computed multiplier m = ceil(2^32 / d)
// (m = 0 for d = 1): floor(q / d) = mulhi(q, m).  With e = m d - 2^32 < d, the quotient is
// exact whenever q e < 2^32, e.g. for all q, d < 2^16, or whenever q d <= 2^32.  A
// run-time 32-bit division costs about fifteen instructions, a 64-bit one several times that.
__host__ __device__ inline uint32_t div_magic(int d) {
  return d <= 1 ? 0u : (uint32_t)((((uint64_t)1 << 32) + (uint64_t)d - 1) / (uint64_t)d);
}
#ifdef __HIPCC__
__device__ __forceinline__ uint32_t fdiv(uint32_t q, uint32_t m) { return m ? __umulhi(q, m) : q; }

// Workgroups are dispatched round-robin over the chip's 8 XCDs, each with its own L2.  This
// renumbers workgroup b of G so that XCD x runs the x-th contiguous eighth of [0, G): work
// items that are neighbours in the numbering (and share operands) then meet in one L2.
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int x = b & 7, per = G >> 3, rem = G & 7;
  return x * per + min(x, rem) + (b >> 3);
}
#endif

// ---- column-set linear combinations ------------------------------------------------------
struct LcSrc {
  const void *X;
  int ldx, xc0, nin;
  const double *C;   // device [nout][nin]
};
struct LcArgs {
  void *Y;
  int ldy, yc0, nout;
  const double *beta;  // device [nout] or nullptr (overwrite)
  int nsrc;
  LcSrc src[3];
};

template <class T>
void spmm_left(const DevPlan &pl, int bu, int bo, const T *A, const T *X, int ldx, int xc0,
               T *C, int ldc, int cc0, int ncol, double alpha, bool acc, hipStream_t s);
template <class T>
void spmm_right(const DevPlan &pl, int bu, int bo, const T *X, int ldx, int xc0, const T *B,
                T *C, int ldc, int cc0, int ncol, double alpha, bool acc, hipStream_t s);
template <class T>
void lincomb(int64_t nblk, int E, const LcArgs &a, hipStream_t s);

// Diagonal form: every source and the output share one column-set layout (ld = nc, column
// offset 0) and the coefficient matrices are diagonal, so
//   Y[k] = beta[c] Y[k] + sum_s d_s[c] X_s[k],   c = (k / E) % nc,
// over the flat element index k; the coefficients travel in the kernel arguments.
constexpr int kLcDiagMax = 64;
struct LcDiagArgs {
  void *Y;
  const void *X[3];
  int nsrc, has_beta;
  double beta[kLcDiagMax];
  double d[3][kLcDiagMax];
};
template <class T>
void lincomb_diag(int64_t nblk, int E, int nc, const LcDiagArgs &a, hipStream_t s);
template <class T>
void gram(int64_t nblk, int E, const T *X, int ldx, int xc0, int n1, const T *Y, int ldy,
          int yc0, int n2, bool diag, double *partial, int max_parts, double *out,
          hipStream_t s);
template <class T>
void pack(int64_t nblk, int BU, int BO, int ns, const double *src, int64_t nnz,
          const int64_t *voff, const int32_t *shape, T *X, int ldx, int xc0, hipStream_t s);
template <class T>
void unpack(int64_t nblk, int BU, int BO, int ns, const T *X, int ldx, int xc0,
            const int64_t *voff, const int32_t *shape, double *dst, int64_t nnz, hipStream_t s);
template <class T>
void fill(T *p, int64_t n, T v, hipStream_t s);
template <class T>
void gather_blocks(int64_t nout, int blk_elems, const int32_t *map, const T *X, T *Y, hipStream_t s);

// ---- grid ----------------------------------------------------------------------------------
// entries of -1 after the end of a tile set's pair table, so that a kernel may read a few
// indices past a tile's last pair without a bounds test
constexpr int kPairPad = 16;
// doubles in the zero block that stands in for a missing P block (NS * BL * BR values of the
// density's widest pass, at most 48)
constexpr int kZeroBlock = 64;
// device view of a tile set (lists and sample rows of two function sets)
struct DevTiles {
  int nt = 0;
  int maxrows = 0;          // max over tiles of (n_left_atoms * BL + n_right_atoms * BR)
  int maxpairs = 0;         // max over tiles of n_left_atoms * n_right_atoms
  int maxrows_r = 0;        // max over tiles of n_right_atoms * BR
  const int32_t *uptr = nullptr, *optr = nullptr;   // [nt + 1]
  const int64_t *pptr = nullptr;                    // [nt + 1]
  const int32_t *pidx = nullptr;                    // pair -> block index (or -1), followed
                                                    // by kPairPad entries of -1
  const void *usamp = nullptr, *osamp = nullptr;    // rows of TP samples
  size_t lds_limit = 65536;                          // device LDS bytes per workgroup
  int waves = 4;                                     // density: tiles (waves) per workgroup
  int pbcast = 0;                                    // density: P blocks in vector registers
                                                     // with DPP row broadcasts (1) or in
                                                     // scalar registers (0)
  const void *zero = nullptr;                        // kZeroBlock zeros (the block read for
                                                     // a pair with no P block)
  const int32_t *order = nullptr;                    // [nt] density: tiles in processing
                                                     // order (Z-order of tile coordinates)
};

// Per-tile partial sums of the potential integrals ([function pair][state], tiles in order,
// contribution-major within a tile) and the fixed-order table that sums them per overlap
// block.
struct DevPartials {
  int64_t total = 0;                  // function pairs over all tiles (values per state)
  const int64_t *tbase = nullptr;     // [nt] first function pair of each tile
  const int64_t *cptr = nullptr;      // [n_out_blocks + 1] contributions per overlap block
  const int32_t *cidx = nullptr;      // per contribution: its index in the partial-sum buffer
                                      // (function pair of its (0, 0) element / E)
};

enum SampleType { SAMPLE_F64 = 0, SAMPLE_F32 = 1, SAMPLE_BF16 = 2 };

// rho_s(r) = scale * sum_{a,b} left_a(r) X_s[a,b] right_b(r), written tile-major as complex
// pairs: out[(s/2) * pair_stride + (t * TP + p) * 2 + (s & 1)]
template <class T>
void density(const DevTiles &tl, int stype, int BL, int BR, const T *X, int ldx, int xc0,
             int ns, T *out, int64_t pair_stride, double scale, hipStream_t s);

// Vout[blk][ldv][E] = scale * sum_r left_a(r) V_s(r) right_b(r) for the nblk_out overlap
// blocks (V tile-major complex pairs); partial: [pa.total][ns] scratch
template <class T>
void potential_integrals(const DevTiles &tl, const DevPartials &pa, int stype, int BL, int BR,
                         const T *V, int64_t pair_stride, int ns, T *partial, T *Vout, int ldv,
                         int64_t nblk_out, double scale, hipStream_t s, Prof *prof);

// f_xc from rho0 (real parts of a tile-major pair array): ALDA exchange kernel
template <class T>
void alda_kernel(int64_t npts, const T *rho_pairs, double floor, T *fxc, hipStream_t s);

// ---- FFT / Poisson --------------------------------------------------------------------------
struct GridGeom {
  int n[3];
  double L[3];
  int ntx, nty, ntz;
};

// V = (V_H[rho] + fxc * rho) for npair complex-packed fields, tile-major in/out:
// fields[pair][tile][TP] complex; work: [pair][n_z][n_y][n_x] complex
template <class T>
void hartree_xc(const GridGeom &g, const FFTPlan &plan, int npair, T *fields, T *work,
                const T *fxc, bool use_fxc, hipStream_t s, Prof *prof);

// largest LDS request of the FFT passes for complex values of `elem` bytes
size_t fft_lds_bytes(const FFTPlan &plan, size_t elem);
// thread counts per workgroup with which an axis's passes run in place (ascending; empty
// when none), and the default choice
std::vector<int> fft_inplace_threads(const AxisFFT &a);

}  // namespace tddft
