// Block-sparse kernels on the atom-block pattern of the response kernels.
//
// A "column set" is an array X[blk][ld][BU*BO] holding `ld` matrices on one block pattern
// (u-atom rows x o-atom columns, blocks padded to BU x BO, row-major); column c of the set
// is the c-th matrix.  All matrices of a solve share the pattern, so a block's values for
// every column are contiguous.
//
//  * masked products  C = alpha * mask(A X) (+ C)  and  C = alpha * mask(X B) (+ C) with a
//    precomputed pair list per output block: every product is exact and only the result
//    is restricted to the output pattern (Sec. III.A: K^c H^u P, P H^o K^v, the
//    K^c V K^v sandwich and the projection K^c S^u L S^o K^v of Eq. auxiliary);
//  * linear combinations of columns (updates, Gram-Schmidt transforms, gradients);
//  * Gram matrices sum_e X[.,i,e] Y[.,j,e] accumulated in FP64 (the traces Tr[X^T S Y S]
//    of Secs. II.C and III.C once Y holds the covariant S^u Y S^o);
//  * conversion between the C-ABI layout [state][values of M] and column sets.
#include <type_traits>

#include "internal.h"
#include "kernels.h"

namespace tddft {

// ---------------------------------------------------------------------------------------
// One thread per (output block, group of CW columns): every operand block pair is read once
// for CW columns (the fixed block of A or B is shared, the column-set blocks are contiguous),
// U pairs at a time.
template <class T, int BU, int BO, int CW, int U>
__global__ __launch_bounds__(256) void k_spmm_left(int64_t nout, int ncol,
                                                   const int64_t *__restrict__ ptr,
                                                   const int2 *__restrict__ pairs,
                                                   const T *__restrict__ A,
                                                   const T *__restrict__ X, int ldx, int xc0,
                                                   T *__restrict__ C, int ldc, int cc0,
                                                   double alpha, int accumulate) {
  constexpr int E = BU * BO;
  const int ng = (ncol + CW - 1) / CW;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nout * ng) return;
  const int64_t k = gid / ng;
  const int m0 = (int)(gid - k * ng) * CW;
  const int nm = min(CW, ncol - m0);
  T acc[CW][E];
#pragma unroll
  for (int u = 0; u < CW; ++u)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[u][e] = T(0);
  const int64_t q0 = ptr[k], q1 = ptr[k + 1];
  // pairs in batches of U: the operand loads of a batch (and the next batch's indices) are
  // issued before its first FMA, so a batch costs one memory round trip; the FMAs still
  // take the pairs one after another in list order (the sum's order depends on neither U
  // nor CW).  Loads past the list's end re-read its last pair, and columns past the call's
  // re-read its last column; neither enters a sum.
  int2 prn[U];
  if (q0 < q1) {
#pragma unroll
    for (int u = 0; u < U; ++u) prn[u] = pairs[min(q0 + u, q1 - 1)];
  }
  for (int64_t qb = q0; qb < q1; qb += U) {
    T av[U][BU * BU], xv[U][CW][E];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T *a = A + (int64_t)prn[u].x * (BU * BU);
#pragma unroll
      for (int i = 0; i < BU * BU; ++i) av[u][i] = a[i];
      const T *x = X + ((int64_t)prn[u].y * ldx + xc0 + m0) * E;
#pragma unroll
      for (int w = 0; w < CW; ++w)
#pragma unroll
        for (int e = 0; e < E; ++e) xv[u][w][e] = x[min(w, nm - 1) * E + e];
    }
    if (qb + U < q1) {
#pragma unroll
      for (int u = 0; u < U; ++u) prn[u] = pairs[min(qb + U + u, q1 - 1)];
    }
    // keeps the compiler from sinking the loads down to their first use
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (qb + u < q1) {
#pragma unroll
        for (int w = 0; w < CW; ++w) {
          if (w < nm) {
#pragma unroll
            for (int r = 0; r < BU; ++r)
#pragma unroll
              for (int t = 0; t < BU; ++t)
#pragma unroll
                for (int c = 0; c < BO; ++c) acc[w][r * BO + c] += av[u][r * BU + t] * xv[u][w][t * BO + c];
          }
        }
      }
    }
  }
  const T al = (T)alpha;
#pragma unroll
  for (int u = 0; u < CW; ++u) {
    if (u < nm) {
      T *c = C + (k * ldc + cc0 + m0 + u) * E;
#pragma unroll
      for (int e = 0; e < E; ++e) c[e] = accumulate ? c[e] + al * acc[u][e] : al * acc[u][e];
    }
  }
}

template <class T, int BU, int BO, int CW, int U>
__global__ __launch_bounds__(256) void k_spmm_right(int64_t nout, int ncol,
                                                    const int64_t *__restrict__ ptr,
                                                    const int2 *__restrict__ pairs,
                                                    const T *__restrict__ X, int ldx, int xc0,
                                                    const T *__restrict__ B,
                                                    T *__restrict__ C, int ldc, int cc0,
                                                    double alpha, int accumulate) {
  constexpr int E = BU * BO;
  const int ng = (ncol + CW - 1) / CW;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nout * ng) return;
  const int64_t k = gid / ng;
  const int m0 = (int)(gid - k * ng) * CW;
  const int nm = min(CW, ncol - m0);
  T acc[CW][E];
#pragma unroll
  for (int u = 0; u < CW; ++u)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[u][e] = T(0);
  const int64_t q0 = ptr[k], q1 = ptr[k + 1];
  // pairs in batches of U, as in k_spmm_left
  int2 prn[U];
  if (q0 < q1) {
#pragma unroll
    for (int u = 0; u < U; ++u) prn[u] = pairs[min(q0 + u, q1 - 1)];
  }
  for (int64_t qb = q0; qb < q1; qb += U) {
    T bv[U][BO * BO], xv[U][CW][E];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T *b = B + (int64_t)prn[u].y * (BO * BO);
#pragma unroll
      for (int i = 0; i < BO * BO; ++i) bv[u][i] = b[i];
      const T *x = X + ((int64_t)prn[u].x * ldx + xc0 + m0) * E;
#pragma unroll
      for (int w = 0; w < CW; ++w)
#pragma unroll
        for (int e = 0; e < E; ++e) xv[u][w][e] = x[min(w, nm - 1) * E + e];
    }
    if (qb + U < q1) {
#pragma unroll
      for (int u = 0; u < U; ++u) prn[u] = pairs[min(qb + U + u, q1 - 1)];
    }
    // keeps the compiler from sinking the loads down to their first use
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (qb + u < q1) {
#pragma unroll
        for (int w = 0; w < CW; ++w) {
          if (w < nm) {
#pragma unroll
            for (int t = 0; t < BO; ++t)
#pragma unroll
              for (int c = 0; c < BO; ++c)
#pragma unroll
                for (int r = 0; r < BU; ++r) acc[w][r * BO + c] += xv[u][w][r * BO + t] * bv[u][t * BO + c];
          }
        }
      }
    }
  }
  const T al = (T)alpha;
#pragma unroll
  for (int u = 0; u < CW; ++u) {
    if (u < nm) {
      T *c = C + (k * ldc + cc0 + m0 + u) * E;
#pragma unroll
      for (int e = 0; e < E; ++e) c[e] = accumulate ? c[e] + al * acc[u][e] : al * acc[u][e];
    }
  }
}

// ---------------------------------------------------------------------------------------
// Dense path (FP32 and FP64).  When both operands and the output of a masked product have
// complete block patterns, the product is a plain dense matrix product; it runs on MFMA
// (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64) straight from the padded-block layouts:
//   left  C = A X:  A [di*BU x dk*BU] in BU x BU blocks, X a column set on dk x dj blocks;
//                   rows (I, r), columns (J, m, c), k = (K, t)
//   right C = X B:  X a column set on di x dk blocks, B [dk*BO x dj*BO] in BO x BO blocks;
//                   rows (I, r, m), columns (J, c), k = (L, t)
// A workgroup of WMW x WNW waves computes a GM x GN output tile over k-slabs of GK, each
// wave (GM / WMW) x (GN / WNW) as 16 x 16 MFMA blocks.  Operand order inside a slab: the
// sum over k is order-free, so in MFMA step s lane group q = lane / 16 supplies
// k = (GK / 4) q + s for both operands; every lane reads GK / 4 consecutive k of one row of
// A and one column of B, stored k-contiguous in LDS ([row][k], rows padded to GK + 4,
// which keeps the 16-byte reads of neighbouring rows on distinct banks).  Two LDS buffers:
// the next slab's global loads are in flight while the current slab is multiplied, one
// barrier per slab.  Global loads of A go along k (AROW = false) or along the tile rows
// (AROW = true: the right product's rows (I, r, m) are 24 bytes apart in memory, its k
// steps a whole block row apart).  Measured at 600 x 6400 x 600 (left) and 9600 x 400 x 400
// (right, FP32): 64 x 64 x 32 tiles 96 / 100 us; these shapes 78 / 82 us.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d_g __attribute__((ext_vector_type(4)));

template <class T> struct MfmaAcc;
template <> struct MfmaAcc<float> { using type = v4f; };
template <> struct MfmaAcc<double> { using type = v4d_g; };

template <class T>
__device__ __forceinline__ typename MfmaAcc<T>::type mfma16x16x4(T a, T b, typename MfmaAcc<T>::type c) {
  if constexpr (std::is_same<T, float>::value) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// tile shapes of the two products
struct GemmLeft { static constexpr int GM = 128, GN = 64, GK = 16, WMW = 4, WNW = 2; static constexpr bool AROW = false; };
struct GemmRight { static constexpr int GM = 64, GN = 64, GK = 16, WMW = 2, WNW = 2; static constexpr bool AROW = true; };
// alternative output tiles the creation-time tuner may pick per product (DevPlan::tile).
// The k-slab depth GK fixes which products each MFMA sums, so every shape here keeps
// GK = 16 and gives bit-identical results.
struct GemmLeft64 { static constexpr int GM = 64, GN = 64, GK = 16, WMW = 2, WNW = 2; static constexpr bool AROW = false; };
struct GemmLeftWide { static constexpr int GM = 64, GN = 128, GK = 16, WMW = 2, WNW = 2; static constexpr bool AROW = false; };
struct GemmRightTall { static constexpr int GM = 128, GN = 64, GK = 16, WMW = 4, WNW = 2; static constexpr bool AROW = true; };
struct GemmRightWide { static constexpr int GM = 64, GN = 128, GK = 16, WMW = 2, WNW = 2; static constexpr bool AROW = true; };

template <class T, int BU, int BO, bool LEFT, class G>
__global__ __launch_bounds__(64 * G::WMW * G::WNW) void k_gemm_blocks(int di, int dk, int dj, int ncol,
                                                                       const T *__restrict__ A,
                                                                       const T *__restrict__ B, int ldx, int xc0,
                                                                       T *__restrict__ C, int ldc, int cc0,
                                                                       T alpha, int accumulate) {
  constexpr int GM = G::GM, GN = G::GN, GK = G::GK, WMW = G::WMW, WNW = G::WNW;
  constexpr bool AROW = G::AROW;
  constexpr int NT = 64 * WMW * WNW;
  constexpr int GKP = GK + 4;
  constexpr int KQ = GK / 4;                           // k per lane group and slab
  constexpr int TM = GM / WMW / 16, TN = GN / WNW / 16;
  constexpr int E = BU * BO;
  static_assert(NT % GK == 0 && GM % (NT / GK) == 0 && NT % GN == 0 && GK % (NT / GN) == 0 &&
                NT % GM == 0 && GK % (NT / GM) == 0 && KQ % 2 == 0, "tile shape");
  using VA = typename MfmaAcc<T>::type;
  __shared__ __align__(16) T As[2][GM][GKP];
  __shared__ __align__(16) T Bs[2][GN][GKP];
  const int M = LEFT ? di * BU : di * BU * ncol;
  const int N = LEFT ? dj * ncol * BO : dj * BO;
  const int K = LEFT ? dk * BU : dk * BO;
  const int i0 = blockIdx.y * GM, n0 = blockIdx.x * GN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t ldxE = (int64_t)ldx * E, ldcE = (int64_t)ldc * E;
  // row part of an A address, k part of an A address, column / k parts of a B address
  auto rowA = [&](int i) -> int64_t {
    if (LEFT) return (int64_t)(i / BU) * dk * (BU * BU) + (i % BU) * BU;
    const int I = i / (BU * ncol), rem = i - I * (BU * ncol), r = rem / ncol, m = rem - r * ncol;
    return ((int64_t)I * dk * ldx + xc0 + m) * E + r * BO;
  };
  auto kA = [&](int k) -> int64_t {
    if (LEFT) return (int64_t)(k / BU) * (BU * BU) + k % BU;
    return (int64_t)(k / BO) * ldxE + k % BO;
  };
  auto colB = [&](int n) -> int64_t {
    if (LEFT) {
      const int J = n / (ncol * BO), rem = n - J * (ncol * BO), m = rem / BO, c = rem - m * BO;
      return ((int64_t)J * ldx + xc0 + m) * E + c;
    }
    return (int64_t)(n / BO) * (BO * BO) + n % BO;
  };
  auto kB = [&](int k) -> int64_t {
    if (LEFT) return (int64_t)(k / BU) * dj * ldxE + (k % BU) * BO;
    return (int64_t)(k / BO) * dj * (BO * BO) + (k % BO) * BO;
  };
  // global staging of A: along k, thread -> k = tid % GK, rows tid / GK + (NT / GK) q; or
  // along rows, thread -> row tid % GM, k = tid / GM + (NT / GM) q.  B: thread -> column
  // tid % GN, k = tid / GN + (NT / GN) q
  constexpr int APER = GM * GK / NT, BPER = GN * GK / NT;
  constexpr int AR = NT / GK, AKP = NT / GM, BK = NT / GN;
  const int ak = AROW ? tid / GM : tid % GK, ar = AROW ? tid % GM : tid / GK;
  int64_t arow[AROW ? 1 : APER];
  bool aval[AROW ? 1 : APER];
#pragma unroll
  for (int q = 0; q < (AROW ? 1 : APER); ++q) {
    const int i = i0 + ar + AR * q;
    aval[q] = i < M;
    arow[q] = aval[q] ? rowA(i) : 0;
  }
  const int bnl = tid % GN, bkl = tid / GN;
  const bool bval = n0 + bnl < N;
  const int64_t bcol = bval ? colB(n0 + bnl) : 0;
  T ra[APER], rb[BPER];
  auto fetch = [&](int k0) {
    if (AROW) {
#pragma unroll
      for (int q = 0; q < APER; ++q) {
        const int k = k0 + ak + AKP * q;
        ra[q] = (k < K && aval[0]) ? A[arow[0] + kA(k)] : T(0);
      }
    } else {
      const int k = k0 + ak;
      const bool kv = k < K;
      const int64_t kp = kv ? kA(k) : 0;
#pragma unroll
      for (int q = 0; q < APER; ++q) ra[q] = (kv && aval[q]) ? A[arow[q] + kp] : T(0);
    }
#pragma unroll
    for (int q = 0; q < BPER; ++q) {
      const int kb = k0 + bkl + BK * q;
      rb[q] = (kb < K && bval) ? B[bcol + kB(kb)] : T(0);
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int q = 0; q < APER; ++q) {
      if (AROW) As[buf][ar][ak + AKP * q] = ra[q];
      else As[buf][ar + AR * q][ak] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < BPER; ++q) Bs[buf][bnl][bkl + BK * q] = rb[q];
  };
  const int wm = (w / WNW) * (GM / WMW), wn = (w % WNW) * (GN / WNW);
  const int q4 = lane >> 4, c16 = lane & 15;
  VA acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = VA{T(0), T(0), T(0), T(0)};
  fetch(0);
  stage(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += GK) {
    const bool more = k0 + GK < K;
    if (more) fetch(k0 + GK);
    T af[TM][KQ], bf[TN][KQ];
    using T2 = T __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int kk = 0; kk < KQ; kk += 2) {
        const T2 v = *reinterpret_cast<const T2 *>(&As[buf][wm + 16 * a + c16][KQ * q4 + kk]);
        af[a][kk] = v.x;
        af[a][kk + 1] = v.y;
      }
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int kk = 0; kk < KQ; kk += 2) {
        const T2 v = *reinterpret_cast<const T2 *>(&Bs[buf][wn + 16 * b + c16][KQ * q4 + kk]);
        bf[b][kk] = v.x;
        bf[b][kk + 1] = v.y;
      }
#pragma unroll
    for (int st = 0; st < KQ; ++st)
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = mfma16x16x4<T>(af[a][st], bf[b][st], acc[a][b]);
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // D of 16x16x4: lane holds column lane % 16 and, in register j, row 4 (lane / 16) + j
  // (FP32) or row 4 j + lane / 16 (FP64)
#pragma unroll
  for (int nb = 0; nb < TN; ++nb) {
    const int n = n0 + wn + nb * 16 + (lane & 15);
    if (n >= N) continue;
    int64_t ccol;
    if (LEFT) {
      const int J = n / (ncol * BO), rem = n - J * (ncol * BO), m = rem / BO, c = rem - m * BO;
      ccol = ((int64_t)J * ldc + cc0 + m) * E + c;
    } else {
      ccol = (int64_t)(n / BO) * ldcE + n % BO;
    }
#pragma unroll
    for (int mb = 0; mb < TM; ++mb) {
      // the lane's rows in this 16-row block: ib + j (FP32) or ib + 4 j (FP64)
      constexpr int step = std::is_same<T, float>::value ? 1 : 4;
      const int ib = i0 + wm + mb * 16 + (std::is_same<T, float>::value ? 4 * (lane >> 4) : (lane >> 4));
      // right product: row i = (I BU + r) ncol + m, decomposed once and then advanced row by
      // row (a run-time division per row would dominate the epilogue)
      int I = 0, r = 0, m = 0;
      if (!LEFT) {
        I = ib / (BU * ncol);
        const int rem = ib - I * (BU * ncol);
        r = rem / ncol;
        m = rem - r * ncol;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = ib + step * j;
        if (i < M) {
          int64_t crow;
          if (LEFT) crow = (int64_t)(i / BU) * dj * ldcE + (i % BU) * BO;
          else crow = ((int64_t)I * dj * ldc + cc0 + m) * E + r * BO;
          T *cp = C + crow + ccol;
          const T v = alpha * acc[mb][nb][j];
          *cp = accumulate ? *cp + v : v;
        }
        if (!LEFT) {
          m += step;
          while (m >= ncol) {
            m -= ncol;
            if (++r == BU) {
              r = 0;
              ++I;
            }
          }
        }
      }
    }
  }
}

#define TD_BDIM_DISPATCH(BU_, BO_, ...)                                     \
  do {                                                                     \
    if (BU_ == 3 && BO_ == 2) { constexpr int BU = 3, BO = 2; __VA_ARGS__; } \
    else if (BU_ == 1 && BO_ == 1) { constexpr int BU = 1, BO = 1; __VA_ARGS__; } \
    else if (BU_ == 2 && BO_ == 2) { constexpr int BU = 2, BO = 2; __VA_ARGS__; } \
    else if (BU_ == 3 && BO_ == 3) { constexpr int BU = 3, BO = 3; __VA_ARGS__; } \
    else if (BU_ == 4 && BO_ == 4) { constexpr int BU = 4, BO = 4; __VA_ARGS__; } \
    else if (BU_ == 5 && BO_ == 2) { constexpr int BU = 5, BO = 2; __VA_ARGS__; } \
    else throw Error{TDDFT_E_INVALID, "unsupported padded block shape"};     \
  } while (0)

static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// the sparse form's (columns per thread, pairs per batch) variants: (1, 1), (1, 2), (1, 4),
// (1, 8), (2, 1), (2, 2), (2, 4), (4, 1), (4, 2)
template <class F>
static void spmm_variant(const DevPlan &pl, F &&launch) {
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I4 = std::integral_constant<int, 4>;
  if (pl.cw == 4) {
    if (pl.pb >= 2) launch(I4{}, I2{});
    else launch(I4{}, I1{});
  } else if (pl.cw == 2) {
    if (pl.pb >= 4) launch(I2{}, I4{});
    else if (pl.pb == 2) launch(I2{}, I2{});
    else launch(I2{}, I1{});
  } else {
    if (pl.pb >= 8) launch(I1{}, std::integral_constant<int, 8>{});
    else if (pl.pb == 4) launch(I1{}, I4{});
    else if (pl.pb == 2) launch(I1{}, I2{});
    else launch(I1{}, I1{});
  }
}

template <class T>
void spmm_left(const DevPlan &pl, int bu, int bo, const T *A, const T *X, int ldx, int xc0,
               T *C, int ldc, int cc0, int ncol, double alpha, bool acc, hipStream_t s) {
  if (pl.nout == 0 || ncol == 0) return;
  if (pl.di > 0) {
    auto launch = [&](auto g) {
      using G = decltype(g);
      const dim3 grid((unsigned)((pl.dj * ncol * bo + G::GN - 1) / G::GN), (unsigned)((pl.di * bu + G::GM - 1) / G::GM));
      TD_BDIM_DISPATCH(bu, bo, hipLaunchKernelGGL((k_gemm_blocks<T, BU, BO, true, G>), grid, dim3(64 * G::WMW * G::WNW), 0, s,
                                                  pl.di, pl.dk, pl.dj, ncol, A, X, ldx, xc0, C, ldc,
                                                  cc0, (T)alpha, acc ? 1 : 0));
    };
    if (pl.tile == 1) launch(GemmLeft64{});
    else if (pl.tile == 2) launch(GemmLeftWide{});
    else launch(GemmLeft{});
    TD_HIP(hipGetLastError());
    return;
  }
  // columns per thread and pairs per batch from the plan (tuned at creation; the sum over
  // pairs has the same order for every choice)
  const int64_t n = pl.nout * ((ncol + pl.cw - 1) / pl.cw);
  auto launch = [&](auto cw, auto u) {
    TD_BDIM_DISPATCH(bu, bo, hipLaunchKernelGGL((k_spmm_left<T, BU, BO, decltype(cw)::value, decltype(u)::value>), dim3(nblocks(n, 256)), dim3(256), 0, s, pl.nout, ncol, pl.ptr.p, pl.pairs.p, A, X, ldx, xc0, C, ldc, cc0, alpha, acc ? 1 : 0));
  };
  spmm_variant(pl, launch);
  TD_HIP(hipGetLastError());
}

template <class T>
void spmm_right(const DevPlan &pl, int bu, int bo, const T *X, int ldx, int xc0, const T *B,
                T *C, int ldc, int cc0, int ncol, double alpha, bool acc, hipStream_t s) {
  if (pl.nout == 0 || ncol == 0) return;
  if (pl.di > 0) {
    auto launch = [&](auto g) {
      using G = decltype(g);
      const dim3 grid((unsigned)((pl.dj * bo + G::GN - 1) / G::GN), (unsigned)((pl.di * bu * ncol + G::GM - 1) / G::GM));
      TD_BDIM_DISPATCH(bu, bo, hipLaunchKernelGGL((k_gemm_blocks<T, BU, BO, false, G>), grid, dim3(64 * G::WMW * G::WNW), 0, s,
                                                  pl.di, pl.dk, pl.dj, ncol, X, B, ldx, xc0, C, ldc,
                                                  cc0, (T)alpha, acc ? 1 : 0));
    };
    if (pl.tile == 1) launch(GemmRightTall{});
    else if (pl.tile == 2) launch(GemmRightWide{});
    else launch(GemmRight{});
    TD_HIP(hipGetLastError());
    return;
  }
  const int64_t n = pl.nout * ((ncol + pl.cw - 1) / pl.cw);
  auto launch = [&](auto cw, auto u) {
    TD_BDIM_DISPATCH(bu, bo, hipLaunchKernelGGL((k_spmm_right<T, BU, BO, decltype(cw)::value, decltype(u)::value>), dim3(nblocks(n, 256)), dim3(256), 0, s, pl.nout, ncol, pl.ptr.p, pl.pairs.p, X, ldx, xc0, B, C, ldc, cc0, alpha, acc ? 1 : 0));
  };
  spmm_variant(pl, launch);
  TD_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------------------
// Y[blk][yc0 + j][e] = beta_j Y + sum_s sum_i C_s[j][i] X_s[blk][xc0_s + i][e]
// One thread per (block, element) computes a chunk of 8 output columns at a time in FP64;
// the coefficients are wave-uniform and arrive through scalar loads.
template <class T>
__global__ __launch_bounds__(256) void k_lincomb(int64_t nblk, int E, LcArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nblk * E) return;
  const int64_t blk = gid / E;
  const int e = (int)(gid - blk * E);
  constexpr int JC = 8;
  for (int j0 = 0; j0 < a.nout; j0 += JC) {
    const int nj = min(JC, a.nout - j0);
    double acc[JC];
    T *y = (T *)a.Y + ((blk * a.ldy + a.yc0 + j0) * E + e);
#pragma unroll
    for (int jj = 0; jj < JC; ++jj)
      acc[jj] = (jj < nj && a.beta) ? a.beta[j0 + jj] * (double)y[(int64_t)jj * E] : 0.0;
    for (int si = 0; si < a.nsrc; ++si) {
      const LcSrc &src = a.src[si];
      const T *x = (const T *)src.X + ((blk * src.ldx + src.xc0) * E + e);
      const double *c = src.C + (int64_t)j0 * src.nin;
      // source columns in steps of four loads in flight (a loop with one load per step
      // would wait on every load); the sum order over i is unchanged
      int i = 0;
      for (; i + 4 <= src.nin; i += 4) {
        double xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = (double)x[(int64_t)(i + u) * E];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int jj = 0; jj < JC; ++jj)
            if (jj < nj) acc[jj] += c[(int64_t)jj * src.nin + i + u] * xv[u];
      }
      for (; i < src.nin; ++i) {
        const double xv = (double)x[(int64_t)i * E];
#pragma unroll
        for (int jj = 0; jj < JC; ++jj)
          if (jj < nj) acc[jj] += c[(int64_t)jj * src.nin + i] * xv;
      }
    }
#pragma unroll
    for (int jj = 0; jj < JC; ++jj)
      if (jj < nj) y[(int64_t)jj * E] = (T)acc[jj];
  }
}

template <class T>
void lincomb(int64_t nblk, int E, const LcArgs &a, hipStream_t s) {
  const int64_t n = nblk * E;
  if (n == 0 || a.nout == 0) return;
  hipLaunchKernelGGL((k_lincomb<T>), dim3(nblocks(n, 256)), dim3(256), 0, s, nblk, E, a);
  TD_HIP(hipGetLastError());
}

// Diagonal linear combination, streaming: four consecutive elements per thread (16-byte
// accesses when the sets allow), FP64 arithmetic in the same order as k_lincomb (beta Y
// first, then the sources in order), so both forms round alike.  The coefficients are
// copied from the kernel arguments into LDS once per workgroup.
template <class T, bool VEC, bool FAST>
__global__ __launch_bounds__(256) void k_lincomb_diag(int64_t n, int E, int nc, uint32_t mE,
                                                      uint32_t mnc, LcDiagArgs a) {
  __shared__ double cb[kLcDiagMax];
  __shared__ double cd[3][kLcDiagMax];
  for (int i = threadIdx.x; i < nc; i += blockDim.x) {
    cb[i] = a.beta[i];
    cd[0][i] = a.d[0][i];
    cd[1][i] = a.d[1][i];
    cd[2][i] = a.d[2][i];
  }
  __syncthreads();
  const int64_t k0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (k0 >= n) return;
  T *Y = (T *)a.Y;
  T y[4], x[3][4];
  if (VEC) {
    using T4 = T __attribute__((ext_vector_type(4)));
    const T4 yv = a.has_beta ? *reinterpret_cast<const T4 *>(Y + k0) : T4(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) y[u] = yv[u];
#pragma unroll
    for (int si = 0; si < 3; ++si)
      if (si < a.nsrc) {
        const T4 xv = *reinterpret_cast<const T4 *>((const T *)a.X[si] + k0);
#pragma unroll
        for (int u = 0; u < 4; ++u) x[si][u] = xv[u];
      }
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = k0 + u;
      y[u] = (a.has_beta && k < n) ? Y[k] : T(0);
#pragma unroll
      for (int si = 0; si < 3; ++si)
        if (si < a.nsrc) x[si][u] = k < n ? ((const T *)a.X[si])[k] : T(0);
    }
  }
  // column of each element: ((k0 + u) / E) % nc, with one division per thread when the host
  // has checked that the multiply-high form is exact (FAST), then stepped element by element
  int cols[4];
  if (FAST) {
    const uint32_t q = fdiv((uint32_t)k0, mE);
    int rem = (int)((uint32_t)k0 - q * (uint32_t)E);
    int col = (int)(q - fdiv(q, mnc) * (uint32_t)nc);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      cols[u] = col;
      if (++rem == E) {
        rem = 0;
        col = col + 1 == nc ? 0 : col + 1;
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) cols[u] = (int)(((k0 + u) / E) % nc);
  }
  T out[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = cols[u];
    double acc = a.has_beta ? cb[c] * (double)y[u] : 0.0;
#pragma unroll
    for (int si = 0; si < 3; ++si)
      if (si < a.nsrc) acc += cd[si][c] * (double)x[si][u];
    out[u] = (T)acc;
  }
  if (VEC) {
    using T4 = T __attribute__((ext_vector_type(4)));
    T4 ov;
#pragma unroll
    for (int u = 0; u < 4; ++u) ov[u] = out[u];
    *reinterpret_cast<T4 *>(Y + k0) = ov;
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k0 + u < n) Y[k0 + u] = out[u];
  }
}

template <class T>
void lincomb_diag(int64_t nblk, int E, int nc, const LcDiagArgs &a, hipStream_t s) {
  const int64_t n = nblk * nc * E;
  if (n == 0) return;
  if (nc > kLcDiagMax || a.nsrc < 0 || a.nsrc > 3) throw Error{TDDFT_E_INVALID, "lincomb_diag: bad arguments"};
  const uintptr_t al = 4 * sizeof(T);   // four-element vectors, naturally aligned
  bool vec = n % 4 == 0 && (uintptr_t)a.Y % al == 0;
  for (int i = 0; i < a.nsrc; ++i) vec = vec && (uintptr_t)a.X[i] % al == 0;
  const unsigned grid = nblocks((n + 3) / 4, 256);
  // multiply-high divisions are exact when q d <= 2^32 for both: k < n by E, k / E by nc
  const bool fast = (double)n * E <= 4294967296.0 && ((double)(n / E) + 1.0) * nc <= 4294967296.0;
  const uint32_t mE = div_magic(E), mnc = div_magic(nc);
  if (vec && fast) hipLaunchKernelGGL((k_lincomb_diag<T, true, true>), dim3(grid), dim3(256), 0, s, n, E, nc, mE, mnc, a);
  else if (vec) hipLaunchKernelGGL((k_lincomb_diag<T, true, false>), dim3(grid), dim3(256), 0, s, n, E, nc, mE, mnc, a);
  else if (fast) hipLaunchKernelGGL((k_lincomb_diag<T, false, true>), dim3(grid), dim3(256), 0, s, n, E, nc, mE, mnc, a);
  else hipLaunchKernelGGL((k_lincomb_diag<T, false, false>), dim3(grid), dim3(256), 0, s, n, E, nc, mE, mnc, a);
  TD_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------------------
// FP64 Gram matrix of two column sets: out[i * n2 + j] = sum X[., xc0+i, .] Y[., yc0+j, .]
// (diag: out[i] = sum X[., xc0+i, .] Y[., yc0+i, .]).  Each workgroup takes a 16 x 16 tile
// of column pairs and a contiguous range of elements; the four waves run
// v_mfma_f64_16x16x4f64 over interleaved 4-element steps (FP64 products and sums), the
// wave results are added in LDS in a fixed order, and a second kernel adds the
// workgroups' partial tiles in a fixed order.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kGramMaxPairs = 4096;   // up to 64 x 64 columns

template <class T, bool FAST>
__global__ __launch_bounds__(256) void k_gram_partial(int64_t nelem, int E, uint32_t mE,
                                                      const T *__restrict__ X,
                                                      int ldx, int xc0, int n1,
                                                      const T *__restrict__ Y, int ldy, int yc0,
                                                      int n2, int diag, int64_t per_part,
                                                      double *__restrict__ partial) {
  __shared__ double red[4][256];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = lane >> 4, m = lane & 15;
  const int i0 = blockIdx.y * 16, j0 = diag ? i0 : blockIdx.z * 16;
  const int ii = i0 + m, jj = j0 + m;
  const bool xi = ii < n1, yj = jj < n2;
  const int64_t k0 = (int64_t)blockIdx.x * per_part;
  const int64_t k1 = k0 + per_part < nelem ? k0 + per_part : nelem;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  // four steps of four elements per wave in flight: loads first, then the products
  for (int64_t kb = k0 + 4 * w; kb < k1; kb += 64) {
    double av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = kb + 16 * u + q;
      av[u] = 0.0;
      bv[u] = 0.0;
      if (k < k1) {
        // block of element k: multiply-high when exact (FAST), else a 64-bit division
        const int64_t blk = FAST ? (int64_t)fdiv((uint32_t)k, mE) : k / E;
        const int e = (int)(k - blk * E);
        if (xi) av[u] = (double)X[(blk * ldx + xc0 + ii) * E + e];
        if (yj) bv[u] = (double)Y[(blk * ldy + yc0 + jj) * E + e];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
  }
  // D of the FP64 16x16x4 product: lane holds column lane % 16 and, in its r-th register,
  // row 4 r + lane / 16 (the FP32 variant interleaves rows the other way)
#pragma unroll
  for (int r = 0; r < 4; ++r) red[w][(4 * r + q) * 16 + m] = acc[r];
  __syncthreads();
  const int npair = diag ? n1 : n1 * n2;
  const int t = threadIdx.x;   // tile entry (row t / 16, column t % 16)
  const int ti = i0 + t / 16, tj = j0 + t % 16;
  if (ti < n1 && tj < n2 && (!diag || ti == tj)) {
    const double v = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    const int qo = diag ? ti : ti * n2 + tj;
    partial[(int64_t)blockIdx.x * npair + qo] = v;
  }
}

// one wave per pair: lanes take parts lane, lane + 64, ... and a fixed butterfly adds them
__global__ __launch_bounds__(256) void k_gram_reduce(int nparts, int npair,
                                                     const double *__restrict__ partial,
                                                     double *__restrict__ out) {
  const int q = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= npair) return;
  double s = 0.0;
  for (int p = lane; p < nparts; p += 64) s += partial[(size_t)p * npair + q];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) out[q] = s;
}

// Diagonal Gram (out[c] = sum X[., xc0+c, .] Y[., yc0+c, .], n1 <= 64 columns), streaming:
// thread (b, c) of a workgroup takes column c of blocks p0 + b, p0 + b + R, ... of the
// workgroup's block range (R = 256 / n1 rows of threads; the n1 threads of a row read one
// block's columns, contiguous), four blocks of loads in flight, products summed in FP64 in
// a fixed order; the rows are then added in row order through LDS.
template <class T, int E>
__global__ __launch_bounds__(256) void k_gram_diag_partial(int64_t nblk, const T *__restrict__ X,
                                                           int ldx, int xc0,
                                                           const T *__restrict__ Y, int ldy, int yc0,
                                                           int n1, int64_t per_part,
                                                           double *__restrict__ partial) {
  __shared__ double red[256];
  const int R = 256 / n1;
  const int b = (int)threadIdx.x / n1, c = (int)threadIdx.x - b * n1;
  const int64_t p0 = (int64_t)blockIdx.x * per_part;
  const int64_t p1 = p0 + per_part < nblk ? p0 + per_part : nblk;
  double acc = 0.0;
  if (b < R) {
    for (int64_t blk0 = p0 + b; blk0 < p1; blk0 += 4 * (int64_t)R) {
      T xv[4][E], yv[4][E];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t blk = blk0 + (int64_t)u * R;
        const T *x = X + (blk * ldx + xc0 + c) * E;
        const T *y = Y + (blk * ldy + yc0 + c) * E;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          xv[u][e] = blk < p1 ? x[e] : T(0);
          yv[u][e] = blk < p1 ? y[e] : T(0);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < E; ++e) acc += (double)xv[u][e] * (double)yv[u][e];
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if ((int)threadIdx.x < n1) {
    double t = 0.0;
    for (int r = 0; r < R; ++r) t += red[r * n1 + threadIdx.x];
    partial[(size_t)blockIdx.x * n1 + threadIdx.x] = t;
  }
}

template <class T>
void gram(int64_t nblk, int E, const T *X, int ldx, int xc0, int n1, const T *Y, int ldy,
          int yc0, int n2, bool diag, double *partial, int max_parts, double *out,
          hipStream_t s) {
  const int npair = diag ? n1 : n1 * n2;
  if (npair > kGramMaxPairs) throw Error{TDDFT_E_INVALID, "gram: too many column pairs"};
  if (diag && n1 >= 1 && n1 <= 64 && (E == 1 || E == 4 || E == 6 || E == 9 || E == 10 || E == 16)) {
    // about eight blocks per thread
    const int R = 256 / n1;
    int64_t per = std::max<int64_t>((int64_t)8 * R, (nblk + max_parts - 1) / max_parts);
    const int parts = (int)std::max<int64_t>(1, (nblk + per - 1) / per);
#define TD_GRAM_DIAG(EE)                                                                              \
  hipLaunchKernelGGL((k_gram_diag_partial<T, EE>), dim3(parts), dim3(256), 0, s, nblk, X, ldx, xc0, Y, \
                     ldy, yc0, n1, per, partial)
    if (E == 1) TD_GRAM_DIAG(1);
    else if (E == 4) TD_GRAM_DIAG(4);
    else if (E == 6) TD_GRAM_DIAG(6);
    else if (E == 9) TD_GRAM_DIAG(9);
    else if (E == 10) TD_GRAM_DIAG(10);
    else TD_GRAM_DIAG(16);
#undef TD_GRAM_DIAG
    TD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((npair + 3) / 4)), dim3(256), 0, s, parts, npair,
                       partial, out);
    TD_HIP(hipGetLastError());
    return;
  }
  const int64_t nelem = nblk * E;
  // element ranges per workgroup: multiples of 64 (four waves x four steps of four elements)
  int parts = (int)std::min<int64_t>(max_parts, std::max<int64_t>(1, nelem / 256));
  int64_t per = (nelem + parts - 1) / parts;
  per = std::max<int64_t>(64, (per + 63) / 64 * 64);
  parts = (int)std::max<int64_t>(1, (nelem + per - 1) / per);
  const int ti = (n1 + 15) / 16, tj = diag ? 1 : (n2 + 15) / 16;
  const uint32_t mE = div_magic(E);
  if ((double)nelem * E <= 4294967296.0)
    hipLaunchKernelGGL((k_gram_partial<T, true>), dim3(parts, ti, tj), dim3(256), 0, s, nelem, E, mE, X, ldx,
                       xc0, n1, Y, ldy, yc0, n2, diag ? 1 : 0, per, partial);
  else
    hipLaunchKernelGGL((k_gram_partial<T, false>), dim3(parts, ti, tj), dim3(256), 0, s, nelem, E, mE, X, ldx,
                       xc0, n1, Y, ldy, yc0, n2, diag ? 1 : 0, per, partial);
  TD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((npair + 3) / 4)), dim3(256), 0, s, parts, npair,
                     partial, out);
  TD_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------------------
// C-ABI layout [state][values of M, natural block sizes] <-> column set (padded blocks)
template <class T>
__global__ __launch_bounds__(256) void k_pack(int64_t nblk, int BU, int BO, int ns,
                                              const double *__restrict__ src, int64_t nnz,
                                              const int64_t *__restrict__ voff,
                                              const int32_t *__restrict__ shape,
                                              T *__restrict__ X, int ldx, int xc0) {
  const int E = BU * BO;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nblk * ns * E) return;
  const int64_t blk = gid / (ns * E);
  const int rem = (int)(gid - blk * ns * E);
  const int s = rem / E, e = rem - s * E;
  const int r = e / BO, c = e - r * BO;
  const int br = shape[blk] & 0xff, bc = shape[blk] >> 8;
  double v = 0.0;
  if (r < br && c < bc) v = src[(int64_t)s * nnz + voff[blk] + r * bc + c];
  X[(blk * ldx + xc0 + s) * E + e] = (T)v;
}

template <class T>
__global__ __launch_bounds__(256) void k_unpack(int64_t nblk, int BU, int BO, int ns,
                                                const T *__restrict__ X, int ldx, int xc0,
                                                const int64_t *__restrict__ voff,
                                                const int32_t *__restrict__ shape,
                                                double *__restrict__ dst, int64_t nnz) {
  const int E = BU * BO;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nblk * ns * E) return;
  const int64_t blk = gid / (ns * E);
  const int rem = (int)(gid - blk * ns * E);
  const int s = rem / E, e = rem - s * E;
  const int r = e / BO, c = e - r * BO;
  const int br = shape[blk] & 0xff, bc = shape[blk] >> 8;
  if (r < br && c < bc) dst[(int64_t)s * nnz + voff[blk] + r * bc + c] = (double)X[(blk * ldx + xc0 + s) * E + e];
}

template <class T>
void pack(int64_t nblk, int BU, int BO, int ns, const double *src, int64_t nnz,
          const int64_t *voff, const int32_t *shape, T *X, int ldx, int xc0, hipStream_t s) {
  const int64_t n = nblk * ns * BU * BO;
  if (n == 0) return;
  hipLaunchKernelGGL((k_pack<T>), dim3(nblocks(n, 256)), dim3(256), 0, s, nblk, BU, BO, ns, src,
                     nnz, voff, shape, X, ldx, xc0);
  TD_HIP(hipGetLastError());
}

template <class T>
void unpack(int64_t nblk, int BU, int BO, int ns, const T *X, int ldx, int xc0,
            const int64_t *voff, const int32_t *shape, double *dst, int64_t nnz, hipStream_t s) {
  const int64_t n = nblk * ns * BU * BO;
  if (n == 0) return;
  hipLaunchKernelGGL((k_unpack<T>), dim3(nblocks(n, 256)), dim3(256), 0, s, nblk, BU, BO, ns, X,
                     ldx, xc0, voff, shape, dst, nnz);
  TD_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------------------
// Y[k][...] = X[map[k]][...]: blocks of a column set on a sub-pattern (truncation to M)
template <class T>
__global__ __launch_bounds__(256) void k_gather_blocks(int64_t nout, int blk_elems,
                                                       const int32_t *__restrict__ map,
                                                       const T *__restrict__ X,
                                                       T *__restrict__ Y) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nout * blk_elems) return;
  const int64_t k = gid / blk_elems;
  const int r = (int)(gid - k * blk_elems);
  Y[gid] = X[(int64_t)map[k] * blk_elems + r];
}

template <class T>
void gather_blocks(int64_t nout, int blk_elems, const int32_t *map, const T *X, T *Y, hipStream_t s) {
  const int64_t n = nout * blk_elems;
  if (n == 0) return;
  hipLaunchKernelGGL((k_gather_blocks<T>), dim3(nblocks(n, 256)), dim3(256), 0, s, nout, blk_elems,
                     map, X, Y);
  TD_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------------------
template <class T>
__global__ void k_fill(int64_t n, T *p, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <class T>
void fill(T *p, int64_t n, T v, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_fill<T>), dim3(nblocks(n, 256)), dim3(256), 0, s, n, p, v);
  TD_HIP(hipGetLastError());
}

// explicit instantiations
#define TD_INST_SPARSE(T)                                                                        \
  template void spmm_left<T>(const DevPlan &, int, int, const T *, const T *, int, int, T *, int, \
                             int, int, double, bool, hipStream_t);                               \
  template void spmm_right<T>(const DevPlan &, int, int, const T *, int, int, const T *, T *,    \
                              int, int, int, double, bool, hipStream_t);                         \
  template void lincomb<T>(int64_t, int, const LcArgs &, hipStream_t);                          \
  template void lincomb_diag<T>(int64_t, int, int, const LcDiagArgs &, hipStream_t);            \
  template void gram<T>(int64_t, int, const T *, int, int, int, const T *, int, int, int, bool,  \
                        double *, int, double *, hipStream_t);                                   \
  template void pack<T>(int64_t, int, int, int, const double *, int64_t, const int64_t *,        \
                        const int32_t *, T *, int, int, hipStream_t);                            \
  template void unpack<T>(int64_t, int, int, int, const T *, int, int, const int64_t *,         \
                          const int32_t *, double *, int64_t, hipStream_t);                      \
  template void fill<T>(T *, int64_t, T, hipStream_t);                                          \
  template void gather_blocks<T>(int64_t, int, const int32_t *, const T *, T *, hipStream_t);

TD_INST_SPARSE(double)
TD_INST_SPARSE(float)

}  // namespace tddft
