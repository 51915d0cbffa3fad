// Real-space grid kernels on 4x4x4 point tiles.
//
// Samples of both function sets are stored tile-major: for every tile, the rows (one per
// function of every atom touching the tile, 64 values each) are contiguous, so a tile's
// samples are read with fully coalesced vector loads, or, when every lane needs the same
// row, with scalar loads into SGPRs.
//
//  * response density (Sec. III.A):   rho_s(r) = sum_ab u_a(r) P_s,ab o_b(r)
//    per tile: psi_a = sum_b P_ab o_b, then rho = sum_a u_a psi_a, P blocks read with
//    wave-uniform (scalar) loads; also used once for rho0 = 2 sum o K^v o.
//  * potential integrals (Sec. II.C, V_SCF^{chi phi}):  V_s,ab = h^3 sum_r u_a V_s o_b
//    per tile, one lane per (o-row, state) reduces over the 64 points in registers; the
//    per-tile sums are added per overlap block in a fixed order (no atomics, reproducible).
//  * ALDA exchange kernel f_xc = -(1/3)(3/pi)^{1/3} rho0^{-2/3} (Sec. II.A, xc part).
// Grid fields are tile-major complex pairs: state 2k in the real part, 2k+1 in the
// imaginary part of field k, so the Hartree FFT transforms two states at once.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "internal.h"
#include "kernels.h"

namespace tddft {

template <class T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <class T, class S>
__device__ __forceinline__ T cvt(S v) { return (T)v; }
template <>
__device__ __forceinline__ float cvt<float, __hip_bfloat16>(__hip_bfloat16 v) {
  return __bfloat162float(v);
}
template <>
__device__ __forceinline__ double cvt<double, __hip_bfloat16>(__hip_bfloat16 v) {
  return (double)__bfloat162float(v);
}

// two consecutive samples (q even, p 4-byte aligned); BF16 pairs come in one 32-bit word so
// that wave-uniform rows are fetched with scalar loads and widened with integer shifts
template <class T, class S>
__device__ __forceinline__ void load2(const S *p, int q, T &a, T &b) {
  a = (T)p[q];
  b = (T)p[q + 1];
}
template <class T>
__device__ __forceinline__ void load2_bf16(const __hip_bfloat16 *p, int q, T &a, T &b) {
  const uint32_t w = reinterpret_cast<const uint32_t *>(p)[q >> 1];
  a = (T)__uint_as_float(w << 16);
  b = (T)__uint_as_float(w & 0xffff0000u);
}
template <>
__device__ __forceinline__ void load2<float, __hip_bfloat16>(const __hip_bfloat16 *p, int q, float &a, float &b) {
  load2_bf16<float>(p, q, a, b);
}
template <>
__device__ __forceinline__ void load2<double, __hip_bfloat16>(const __hip_bfloat16 *p, int q, double &a, double &b) {
  load2_bf16<double>(p, q, a, b);
}

// ---------------------------------------------------------------------------------------
// Response density.  One wave per tile, one lane per grid point.  The tile's o-atoms are
// taken in chunks of JC whose o-rows are loaded once into registers; for every left atom i
// the partial sums psi_s,r = sum_j P_s[(i,r),(j,.)] . o_j over the chunk are built from
// wave-uniform P blocks (all NS states of a block are contiguous, so they arrive in SGPRs
// through a few scalar loads and feed the FMAs as scalar operands), then
// rho_s += u_(i,r) psi_s,r.  The pair loop thus issues only the scalar loads of P: the
// o-rows are not re-read per left atom.  No LDS, so occupancy is set by registers alone.
template <class T, class S, int NS, int BL, int BR, int JC, bool FULL>
__device__ __forceinline__ void density_chunk(const int32_t *__restrict__ pid, int nj,
                                              const T *__restrict__ X, int64_t xoff, int ldx,
                                              const T *__restrict__ zero, int nk,
                                              const T (&o)[JC][BR], T (&tmp)[NS][BL]) {
  constexpr int E = BL * BR;
  // The chunk's block indices arrive in one batch of scalar loads (the pair table carries
  // padding past its end, so all JC are readable), then each pair costs one round trip for
  // its P block; a pair with no P block reads the zero block.
  int pbs[JC];
#pragma unroll
  for (int j = 0; j < JC; ++j) pbs[j] = pid[j];
#pragma unroll
  for (int j = 0; j < JC; ++j) {
    if (j >= nj) break;
    const int pb = pbs[j];
    const T *Pj = pb >= 0 ? X + ((int64_t)pb * ldx) * E + xoff : zero;
    if constexpr (FULL) {
      T pv[NS * E];
#pragma unroll
      for (int q = 0; q < NS * E; ++q) pv[q] = Pj[q];
#pragma unroll
      for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int r = 0; r < BL; ++r)
#pragma unroll
          for (int c = 0; c < BR; ++c) tmp[k][r] += pv[k * E + r * BR + c] * o[j][c];
    } else {
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        if (k >= nk) break;
#pragma unroll
        for (int r = 0; r < BL; ++r)
#pragma unroll
          for (int c = 0; c < BR; ++c) tmp[k][r] += Pj[k * E + r * BR + c] * o[j][c];
      }
    }
  }
}

// Pair loop with P in vector registers (FP32 and FP64).  Every 16-lane row of the wave
// loads the same NS * BL * BR values of a P block, value q in lane q % 16 of register q / 16,
// and each FMA takes its P factor from lane q % 16 of its own row by a DPP row broadcast
// (row_newbcast), so the P operand costs no extra instruction.  The loads are vector loads, which complete
// in order: the P blocks of all pairs of the chunk are requested before the first FMA,
// where the scalar form waits for each block in turn.  A DPP read needs its source register
// written by a load, not by an ALU instruction, in the two cycles before it; the P registers
// are only ever written by loads.
template <int K>
__device__ __forceinline__ void fmac_row_bcast(float &acc, float v, float o) {
  asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
      : "+v"(acc) : "v"(v), "v"(o), "n"(K));
}
// the FP64 ALU takes DPP with the row broadcast on its 64-bit operands as well
template <int K>
__device__ __forceinline__ void fmac_row_bcast(double &acc, double v, double o) {
  asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
      : "+v"(acc) : "v"(v), "v"(o), "n"(K));
}

template <class T, int NS, int BL, int BR, int JC, int NV, int Q0, int... Q>
__device__ __forceinline__ void bcast_pair(std::integer_sequence<int, Q...>, const T (&pv)[NV],
                                           const T (&o)[BR], T (&tmp)[NS][BL]) {
  constexpr int E = BL * BR;
  (fmac_row_bcast<(Q0 + Q) % 16>(tmp[(Q0 + Q) / E][((Q0 + Q) % E) / BR], pv[(Q0 + Q) / 16],
                                 o[(Q0 + Q) % BR]), ...);
}

template <class T, int NS, int BL, int BR, int JC>
__device__ __forceinline__ void density_chunk_bcast(int (&pbs)[JC], const int32_t *__restrict__ pid_next,
                                                    int nj, const T *__restrict__ X,
                                                    int64_t xoff, int ldx,
                                                    const T *__restrict__ zero, int l16,
                                                    const T (&o)[JC][BR],
                                                    T (&tmp)[NS][BL]) {
  constexpr int E = BL * BR, Q = NS * E, NV = (Q + 15) / 16;
  // lane l16 of a row holds values l16, 16 + l16, ...; lanes past the block's end repeat
  // its last value (never broadcast), so every load stays inside the block
  int qi[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) qi[v] = min(16 * v + l16, Q - 1);
  // all JC blocks requested in one straight run (pairs past the chunk's end read the zero
  // block), so the wait before pair j's FMAs counts only the loads issued after it
  T pv[JC][NV];
#pragma unroll
  for (int j = 0; j < JC; ++j) {
    const T *Pj = j < nj && pbs[j] >= 0 ? X + ((int64_t)pbs[j] * ldx) * E + xoff : zero;
#pragma unroll
    for (int v = 0; v < NV; ++v) pv[j][v] = Pj[qi[v]];
  }
  // the next left atom's block indices are in flight during this atom's FMAs
  if (pid_next) {
#pragma unroll
    for (int j = 0; j < JC; ++j) pbs[j] = pid_next[j];
  }
  // keeps the compiler from sinking the loads down to their first use
  asm volatile("" ::: "memory");
#pragma unroll
  for (int j = 0; j < JC; ++j) {
    if (j >= nj) break;
    bcast_pair<T, NS, BL, BR, JC, NV, 0>(std::make_integer_sequence<int, Q>{}, pv[j], o[j], tmp);
  }
}

template <class T, class S, int BL, int BR, int NSC, bool PB>
__global__ __launch_bounds__(512) void k_density(DevTiles tl, const S *__restrict__ usamp,
                                                 const S *__restrict__ osamp,
                                                 const int32_t *__restrict__ pidx,
                                                 const T *__restrict__ X, int ldx, int xc0, int ns,
                                                 T *__restrict__ out, int64_t pair_stride, T scale) {
  // states per pass: a P block (NS * BL * BR values) within 48 SGPRs, NS even (fields hold
  // state pairs): 8 in FP32 and 4 in FP64 for 3 x 2 blocks, capped at NSC (the launch takes
  // the smallest even cap that covers the call's states, so a 4-state call loads 4-state
  // P blocks and runs the unrolled full-pass path)
  constexpr int kSlots = sizeof(T) == 8 ? 24 : 48, kMax = sizeof(T) == 8 ? 4 : 8;
  constexpr int NSe = (kSlots / (BL * BR)) & ~1;
  constexpr int NSf = NSe < 2 ? 2 : (NSe > kMax ? kMax : NSe);
  constexpr int NS = NSf < NSC ? NSf : NSC;
  // o-atoms per register chunk: 8 x BR rows in FP32, 4 x BR in FP64
  constexpr int JC = sizeof(T) == 8 ? 4 : 8;
  static_assert(NS * BL * BR * sizeof(T) <= kZeroBlock * sizeof(double), "zero block too small");
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // each XCD takes one contiguous eighth of the Z-ordered tile list, so its L2 holds the P
  // blocks of one compact region
  const int lt = xcd_block(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + w;
  if (lt >= tl.nt) return;
  const int t = tl.order[lt];
  const int u0 = tl.uptr[t], nua = tl.uptr[t + 1] - u0;
  const int o0 = tl.optr[t], noa = tl.optr[t + 1] - o0;
  const S *os = osamp + (int64_t)o0 * BR * TP;
  using T2 = typename Vec2<T>::type;
  const int32_t *pid = pidx + tl.pptr[t];
  const T *zero = reinterpret_cast<const T *>(tl.zero);
  for (int s0 = 0; s0 < ns; s0 += NS) {
    const int nk = min(NS, ns - s0);
    const int64_t xoff = (int64_t)(xc0 + s0) * BL * BR;
    T acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = T(0);
    for (int j0 = 0; j0 < noa; j0 += JC) {
      const int nj = min(JC, noa - j0);
      // the chunk's o-rows in one run of loads (rows past the chunk's end re-read its last
      // row and are zeroed after conversion), so a chunk costs one memory round trip
      S oraw[JC][BR];
#pragma unroll
      for (int j = 0; j < JC; ++j)
#pragma unroll
        for (int c = 0; c < BR; ++c) oraw[j][c] = os[((j0 + min(j, nj - 1)) * BR + c) * TP + lane];
      T o[JC][BR];
#pragma unroll
      for (int j = 0; j < JC; ++j)
#pragma unroll
        for (int c = 0; c < BR; ++c) o[j][c] = j < nj ? cvt<T>(oraw[j][c]) : T(0);
      // u-rows of the next left atom are requested before this atom's pair loop, so their
      // round trip overlaps the scalar loads and FMAs of the pairs
      const S *us = usamp + ((int64_t)u0 * BL) * TP + lane;
      S un[BL];
      if (nua > 0) {
#pragma unroll
        for (int r = 0; r < BL; ++r) un[r] = us[r * TP];
      }
      // block indices of the first left atom's pairs (the bcast form requests each next
      // atom's indices during the current atom's FMAs; the table is padded past its end)
      int pbs[JC];
      if constexpr (PB) {
        if (nk == NS && nua > 0) {
#pragma unroll
          for (int j = 0; j < JC; ++j) pbs[j] = pid[j0 + j];
        }
      }
      for (int i = 0; i < nua; ++i) {
        T u[BL];
#pragma unroll
        for (int r = 0; r < BL; ++r) u[r] = cvt<T>(un[r]);
        if (i + 1 < nua) {
#pragma unroll
          for (int r = 0; r < BL; ++r) un[r] = us[((i + 1) * BL + r) * TP];
        }
        T tmp[NS][BL];
#pragma unroll
        for (int k = 0; k < NS; ++k)
#pragma unroll
          for (int r = 0; r < BL; ++r) tmp[k][r] = T(0);
        if constexpr (PB) {
          if (nk == NS)
            density_chunk_bcast<T, NS, BL, BR, JC>(pbs, i + 1 < nua ? pid + (i + 1) * noa + j0 : nullptr,
                                                nj, X, xoff, ldx, zero, lane & 15, o, tmp);
          else
            density_chunk<T, S, NS, BL, BR, JC, false>(pid + i * noa + j0, nj, X, xoff, ldx, zero, nk, o, tmp);
        } else if (nk == NS)
          density_chunk<T, S, NS, BL, BR, JC, true>(pid + i * noa + j0, nj, X, xoff, ldx, zero, nk, o, tmp);
        else
          density_chunk<T, S, NS, BL, BR, JC, false>(pid + i * noa + j0, nj, X, xoff, ldx, zero, nk, o, tmp);
#pragma unroll
        for (int r = 0; r < BL; ++r)
#pragma unroll
          for (int k = 0; k < NS; ++k) acc[k] += u[r] * tmp[k][r];
      }
    }
    T *dst = out + (int64_t)(s0 / 2) * pair_stride + ((int64_t)t * TP + lane) * 2;
#pragma unroll
    for (int m = 0; m < NS / 2; ++m) {
      if (2 * m < nk) {
        T2 v;
        v.x = scale * acc[2 * m];
        v.y = 2 * m + 1 < nk ? scale * acc[2 * m + 1] : T(0);
        *reinterpret_cast<T2 *>(dst + (int64_t)m * pair_stride) = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// Potential integrals.  One wave per tile, one lane per (o-row b of the tile, state s),
// looping over 64-item chunks when the tile has more.  The lane forms w(r) = V_s(r) o_b(r)
// for the tile's 64 points in registers (wide loads of the o-row and of the complex-pair
// field), then for every u-row a of the tile sums u_a(r) w(r); u_a's row is wave-uniform and
// arrives in SGPRs through scalar loads, so the inner loop is FMAs with one scalar and one
// vector operand.  Each tile writes its sums to its own range of a partial-sum buffer,
// contribution-major ([(u-atom, o-atom)][r][c][state], so every contribution is one
// contiguous run); k_vint_reduce adds them per overlap block in a fixed order (no
// atomics, reproducible).
template <class T, class S>
__device__ __forceinline__ void load4(const S *p, T (&o)[4]) {
  o[0] = cvt<T>(p[0]); o[1] = cvt<T>(p[1]); o[2] = cvt<T>(p[2]); o[3] = cvt<T>(p[3]);
}
template <>
__device__ __forceinline__ void load4<float, float>(const float *p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4 *>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <>
__device__ __forceinline__ void load4<double, double>(const double *p, double (&o)[4]) {
  const double2 a = reinterpret_cast<const double2 *>(p)[0];
  const double2 b = reinterpret_cast<const double2 *>(p)[1];
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
template <>
__device__ __forceinline__ void load4<float, __hip_bfloat16>(const __hip_bfloat16 *p, float (&o)[4]) {
  const uint2 v = *reinterpret_cast<const uint2 *>(p);
  o[0] = __uint_as_float(v.x << 16); o[1] = __uint_as_float(v.x & 0xffff0000u);
  o[2] = __uint_as_float(v.y << 16); o[3] = __uint_as_float(v.y & 0xffff0000u);
}
// component c (0 real, 1 imaginary) of two consecutive complex values (p 4-element aligned)
template <class T>
__device__ __forceinline__ void load_comp2(const T *p, int c, T &a, T &b) {
  using T2 = typename Vec2<T>::type;
  const T2 x = reinterpret_cast<const T2 *>(p)[0];
  const T2 y = reinterpret_cast<const T2 *>(p)[1];
  a = c ? x.y : x.x;
  b = c ? y.y : y.x;
}

template <class T, class S, int BL, int BR>
__global__ __launch_bounds__(256) void k_vint(DevTiles tl, const int64_t *__restrict__ tbase,
                                              const S *__restrict__ usamp,
                                              const S *__restrict__ osamp,
                                              const T *__restrict__ V, int64_t pair_stride,
                                              int ns, T *__restrict__ partial, T scale) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * (blockDim.x >> 6) + w;
  if (t >= tl.nt) return;
  const int u0 = tl.uptr[t], nua = tl.uptr[t + 1] - u0;
  const int o0 = tl.optr[t], noa = tl.optr[t + 1] - o0;
  const int rows_o = noa * BR;
  const int items = rows_o * ns;
  T *dst = partial + tbase[t] * ns;
  const T *vt = V + (int64_t)t * TP * 2;
  for (int c0 = 0; c0 < items; c0 += 64) {
    const int item = c0 + lane;
    const bool active = item < items;
    const int b = active ? item / ns : 0;
    const int s = active ? item - (item / ns) * ns : 0;
    const S *orow = osamp + ((int64_t)o0 * BR + b) * TP;
    const T *vs = vt + (int64_t)(s >> 1) * pair_stride;
    T wv[TP];
#pragma unroll
    for (int q = 0; q < TP; q += 4) {
      T o[4], v0, v1, v2, v3;
      load4<T, S>(orow + q, o);
      load_comp2<T>(vs + 2 * q, s & 1, v0, v1);
      load_comp2<T>(vs + 2 * q + 4, s & 1, v2, v3);
      wv[q] = o[0] * v0;
      wv[q + 1] = o[1] * v1;
      wv[q + 2] = o[2] * v2;
      wv[q + 3] = o[3] * v3;
    }
    for (int i = 0; i < nua; ++i) {
#pragma unroll
      for (int r = 0; r < BL; ++r) {
        const S *urow = usamp + ((int64_t)(u0 + i) * BL + r) * TP;
        T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
#pragma unroll
        for (int q = 0; q < TP; q += 4) {
          T a0, a1, a2, a3;
          load2<T, S>(urow, q, a0, a1);
          load2<T, S>(urow, q + 2, a2, a3);
          s0 += a0 * wv[q];
          s1 += a1 * wv[q + 1];
          s2 += a2 * wv[q + 2];
          s3 += a3 * wv[q + 3];
        }
        if (active)
          dst[((((int64_t)i * noa + b / BR) * BL + r) * BR + b % BR) * ns + s] = scale * ((s0 + s1) + (s2 + s3));
      }
    }
  }
}

// FP32 variant on MFMA.  Per tile the integrals are a small matrix product
//   Out[a][(b, s)] = sum_r u_a(r) w_(b,s)(r),   w_(b,s)(r) = o_b(r) V_s(r),
// with the 64 points as the contraction.  One wave per tile runs it as 16 x 16 output
// blocks of v_mfma_f32_16x16x4f32; the sum over points is order-free, so lane group
// q = lane / 16 takes points 16 q .. 16 q + 15 and every operand fragment is a run of 16
// consecutive samples (wide loads).  Up to 32 u-rows of A stay in registers while the
// (o-row, state) blocks stream by.
typedef float v4f __attribute__((ext_vector_type(4)));

// Each wave stages into and reads back from its own LDS region only, so after staging it
// waits for its own LDS writes (and keeps the compiler from hoisting the reads above them)
// instead of meeting the workgroup's other waves at a barrier.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <class S>
__device__ __forceinline__ void load16(const S *p, float (&o)[16]) {
#pragma unroll
  for (int k = 0; k < 16; k += 4) {
    float t[4];
    load4<float, S>(p + k, t);
    o[k] = t[0]; o[k + 1] = t[1]; o[k + 2] = t[2]; o[k + 3] = t[3];
  }
}

template <class S, int BL, int BR>
__global__ __launch_bounds__(256) void k_vint_mfma(DevTiles tl, const int64_t *__restrict__ tbase,
                                                   const S *__restrict__ usamp,
                                                   const S *__restrict__ osamp,
                                                   const float *__restrict__ V, int64_t pair_stride,
                                                   int ns, float *__restrict__ partial, float scale) {
  extern __shared__ unsigned char lds_raw[];
  constexpr int LD = TP + 4;   // padded rows: the 16-byte reads of different rows use different banks
  constexpr int MG = 2;        // 16-row blocks of u-rows held in registers at a time
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * (blockDim.x >> 6) + w;
  float *lo = reinterpret_cast<float *>(lds_raw) + (size_t)w * (tl.maxrows_r + ns) * LD;
  float *lv = lo + (size_t)tl.maxrows_r * LD;
  int u0 = 0, nua = 0, o0 = 0, noa = 0;
  if (t < tl.nt) {
    u0 = tl.uptr[t];
    nua = tl.uptr[t + 1] - u0;
    o0 = tl.optr[t];
    noa = tl.optr[t + 1] - o0;
  }
  const int rows_u = nua * BL, rows_o = noa * BR;
  const int items = rows_o * ns;
  const int q = lane >> 4, c16 = lane & 15;
  const S *ut = usamp + (int64_t)u0 * BL * TP;
  float a[MG][16];
  auto load_u = [&](int mg) {
#pragma unroll
    for (int mb = 0; mb < MG; ++mb) {
      const int m = mg + mb * 16 + c16;
      if (m < rows_u) {
        load16<S>(ut + (int64_t)m * TP + 16 * q, a[mb]);
      } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) a[mb][k] = 0.0f;
      }
    }
  };
  // the first u-row blocks are requested before the staging loads, so that both are in
  // flight together
  load_u(0);
  // stage the tile's o-rows (four samples per load) and the states' potentials (one complex
  // pair per load, de-interleaved into the two real states).  Loads go out in batches of
  // four per lane before any LDS write, so a batch costs one memory round trip.
  {
    const S *ot = osamp + (int64_t)o0 * BR * TP;
    const float *vt = V + (int64_t)t * TP * 2;
    const int n_o4 = rows_o * (TP / 4);
    const int n_v2 = t < tl.nt ? ((ns + 1) / 2) * TP : 0;
    for (int i0 = lane; i0 < n_o4 || i0 < n_v2; i0 += 4 * 64) {
      float o4[4][4];
      float2 v2[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 64 * u;
        if (i < n_o4) load4<float, S>(ot + 4 * i, o4[u]);
        if (i < n_v2) {
          const int sp = i / TP, p = i % TP;
          v2[u] = *reinterpret_cast<const float2 *>(vt + (int64_t)sp * pair_stride + 2 * p);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 64 * u;
        if (i < n_o4) {
          float *d = lo + (i / (TP / 4)) * LD + 4 * (i % (TP / 4));
          *reinterpret_cast<float4 *>(d) = make_float4(o4[u][0], o4[u][1], o4[u][2], o4[u][3]);
        }
        if (i < n_v2) {
          const int sp = i / TP, p = i % TP;
          lv[(2 * sp) * LD + p] = v2[u].x;
          if (2 * sp + 1 < ns) lv[(2 * sp + 1) * LD + p] = v2[u].y;
        }
      }
    }
  }
  wave_lds_sync();
  if (t >= tl.nt) return;
  float *dst = partial + tbase[t] * ns;
  for (int mg = 0; mg < rows_u; mg += 16 * MG) {
    if (mg > 0) load_u(mg);
    for (int n0 = 0; n0 < items; n0 += 16) {
      const int n = n0 + c16;
      const bool active = n < items;
      const int b = active ? n / ns : 0;
      const int sidx = active ? n - (n / ns) * ns : 0;
      float bf[16];
      {
        const float *orow = lo + b * LD + 16 * q;
        const float *vrow = lv + sidx * LD + 16 * q;
#pragma unroll
        for (int k = 0; k < 16; k += 4) {
          const float4 o4 = *reinterpret_cast<const float4 *>(orow + k);
          const float4 v4 = *reinterpret_cast<const float4 *>(vrow + k);
          bf[k] = active ? o4.x * v4.x : 0.0f;
          bf[k + 1] = active ? o4.y * v4.y : 0.0f;
          bf[k + 2] = active ? o4.z * v4.z : 0.0f;
          bf[k + 3] = active ? o4.w * v4.w : 0.0f;
        }
      }
#pragma unroll
      for (int mb = 0; mb < MG; ++mb) {
        if (mg + mb * 16 >= rows_u) break;
        v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 16; ++k) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mb][k], bf[k], acc, 0, 0, 0);
        if (active) {
          // contribution-major: [(u-atom, o-atom)][r][c][state]
          const int jo = b / BR, c = b - (b / BR) * BR;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int m = mg + mb * 16 + 4 * q + j;
            if (m < rows_u) {
              const int io = m / BL, r = m - (m / BL) * BL;
              dst[((((int64_t)io * noa + jo) * BL + r) * BR + c) * ns + sidx] = scale * acc[j];
            }
          }
        }
      }
    }
  }
}

// FP64 variant on v_mfma_f64_16x16x4f64: the same per-tile product with FP64 samples, LDS
// rows and potentials (two samples per 16-byte load; rows padded by two values so that the
// 16-byte reads of neighbouring rows fall on different banks).  The FP64 accumulator holds
// rows 4 j + lane / 16 of the 16 x 16 block (FP32: 4 (lane / 16) + j).  One 16-row block of
// u-rows is held in registers at a time.
typedef double v4d_vint __attribute__((ext_vector_type(4)));

template <int BL, int BR>
__global__ __launch_bounds__(128) void k_vint_mfma64(DevTiles tl, const int64_t *__restrict__ tbase,
                                                     const double *__restrict__ usamp,
                                                     const double *__restrict__ osamp,
                                                     const double *__restrict__ V,
                                                     int64_t pair_stride, int ns,
                                                     double *__restrict__ partial, double scale) {
  extern __shared__ unsigned char lds_raw[];
  constexpr int LD = TP + 2;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * (blockDim.x >> 6) + w;
  double *lo = reinterpret_cast<double *>(lds_raw) + (size_t)w * (tl.maxrows_r + ns) * LD;
  double *lv = lo + (size_t)tl.maxrows_r * LD;
  int u0 = 0, nua = 0, o0 = 0, noa = 0;
  if (t < tl.nt) {
    u0 = tl.uptr[t];
    nua = tl.uptr[t + 1] - u0;
    o0 = tl.optr[t];
    noa = tl.optr[t + 1] - o0;
  }
  const int rows_u = nua * BL, rows_o = noa * BR;
  const int items = rows_o * ns;
  const int q = lane >> 4, c16 = lane & 15;
  const double *ut = usamp + (int64_t)u0 * BL * TP;
  double a[16];
  auto load_u = [&](int mg) {
    const int m = mg + c16;
    if (m < rows_u) {
      const double2 *p = reinterpret_cast<const double2 *>(ut + (int64_t)m * TP + 16 * q);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const double2 v = p[k];
        a[2 * k] = v.x;
        a[2 * k + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) a[k] = 0.0;
    }
  };
  // the first u-row block is requested before the staging loads, so that both are in flight
  load_u(0);
  {
    const double *ot = osamp + (int64_t)o0 * BR * TP;
    const double *vt = V + (int64_t)t * TP * 2;
    const int n_o2 = rows_o * (TP / 2);
    const int n_v2 = t < tl.nt ? ((ns + 1) / 2) * TP : 0;
    for (int i0 = lane; i0 < n_o2 || i0 < n_v2; i0 += 4 * 64) {
      double2 o2[4], v2[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 64 * u;
        if (i < n_o2) o2[u] = reinterpret_cast<const double2 *>(ot)[i];
        if (i < n_v2) {
          const int sp = i / TP, p = i % TP;
          v2[u] = *reinterpret_cast<const double2 *>(vt + (int64_t)sp * pair_stride + 2 * p);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 64 * u;
        if (i < n_o2) *reinterpret_cast<double2 *>(lo + (i / (TP / 2)) * LD + 2 * (i % (TP / 2))) = o2[u];
        if (i < n_v2) {
          const int sp = i / TP, p = i % TP;
          lv[(2 * sp) * LD + p] = v2[u].x;
          if (2 * sp + 1 < ns) lv[(2 * sp + 1) * LD + p] = v2[u].y;
        }
      }
    }
  }
  wave_lds_sync();
  if (t >= tl.nt) return;
  double *dst = partial + tbase[t] * ns;
  for (int mg = 0; mg < rows_u; mg += 16) {
    if (mg > 0) load_u(mg);
    for (int n0 = 0; n0 < items; n0 += 16) {
      const int n = n0 + c16;
      const bool active = n < items;
      const int b = active ? n / ns : 0;
      const int sidx = active ? n - (n / ns) * ns : 0;
      double bf[16];
      {
        const double *orow = lo + b * LD + 16 * q;
        const double *vrow = lv + sidx * LD + 16 * q;
#pragma unroll
        for (int k = 0; k < 16; k += 2) {
          const double2 o2 = *reinterpret_cast<const double2 *>(orow + k);
          const double2 v2 = *reinterpret_cast<const double2 *>(vrow + k);
          bf[k] = active ? o2.x * v2.x : 0.0;
          bf[k + 1] = active ? o2.y * v2.y : 0.0;
        }
      }
      v4d_vint acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 16; ++k) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k], bf[k], acc, 0, 0, 0);
      if (active) {
        // contribution-major: [(u-atom, o-atom)][r][c][state]
        const int jo = b / BR, c = b - (b / BR) * BR;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int m = mg + 4 * j + q;
          if (m < rows_u) {
            const int io = m / BL, r = m - (m / BL) * BL;
            dst[((((int64_t)io * noa + jo) * BL + r) * BR + c) * ns + sidx] = scale * acc[j];
          }
        }
      }
    }
  }
}

// BF16 variant on BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation): the u-row
// fragments are the stored BF16 samples themselves (32 contiguous bytes per lane), and the
// (o-row, state) operand w = o_b V_s is formed in FP32 from the staged o-rows and
// potentials and rounded to BF16 (nearest even) once.  Each MFMA contracts 32 points; lane
// group q supplies points 16 q + 8 t + e (e = 0..7) in call t = 0, 1 for both operands, so
// two calls cover the tile's 64 points.  Everything else as in k_vint_mfma.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int BL, int BR>
__global__ __launch_bounds__(256) void k_vint_mfma_bf16(DevTiles tl, const int64_t *__restrict__ tbase,
                                                        const __hip_bfloat16 *__restrict__ usamp,
                                                        const __hip_bfloat16 *__restrict__ osamp,
                                                        const float *__restrict__ V, int64_t pair_stride,
                                                        int ns, float *__restrict__ partial, float scale) {
  extern __shared__ unsigned char lds_raw[];
  constexpr int LD = TP + 4;
  constexpr int MG = 2;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * (blockDim.x >> 6) + w;
  float *lo = reinterpret_cast<float *>(lds_raw) + (size_t)w * (tl.maxrows_r + ns) * LD;
  float *lv = lo + (size_t)tl.maxrows_r * LD;
  int u0 = 0, nua = 0, o0 = 0, noa = 0;
  if (t < tl.nt) {
    u0 = tl.uptr[t];
    nua = tl.uptr[t + 1] - u0;
    o0 = tl.optr[t];
    noa = tl.optr[t + 1] - o0;
  }
  const int rows_u = nua * BL, rows_o = noa * BR;
  const int items = rows_o * ns;
  const int q = lane >> 4, c16 = lane & 15;
  const __hip_bfloat16 *ut = usamp + (int64_t)u0 * BL * TP;
  v8bf a[MG][2];
  auto load_u = [&](int mg) {
#pragma unroll
    for (int mb = 0; mb < MG; ++mb) {
      const int m = mg + mb * 16 + c16;
      if (m < rows_u) {
        const uint4 *src = reinterpret_cast<const uint4 *>(ut + (int64_t)m * TP + 16 * q);
        a[mb][0] = __builtin_bit_cast(v8bf, src[0]);
        a[mb][1] = __builtin_bit_cast(v8bf, src[1]);
      } else {
        a[mb][0] = __builtin_bit_cast(v8bf, make_uint4(0u, 0u, 0u, 0u));
        a[mb][1] = a[mb][0];
      }
    }
  };
  load_u(0);
  {
    const __hip_bfloat16 *ot = osamp + (int64_t)o0 * BR * TP;
    const float *vt = V + (int64_t)t * TP * 2;
    const int n_o4 = rows_o * (TP / 4);
    const int n_v2 = t < tl.nt ? ((ns + 1) / 2) * TP : 0;
    for (int i0 = lane; i0 < n_o4 || i0 < n_v2; i0 += 4 * 64) {
      float o4[4][4];
      float2 v2[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 64 * u;
        if (i < n_o4) load4<float, __hip_bfloat16>(ot + 4 * i, o4[u]);
        if (i < n_v2) {
          const int sp = i / TP, p = i % TP;
          v2[u] = *reinterpret_cast<const float2 *>(vt + (int64_t)sp * pair_stride + 2 * p);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 64 * u;
        if (i < n_o4) {
          float *d = lo + (i / (TP / 4)) * LD + 4 * (i % (TP / 4));
          *reinterpret_cast<float4 *>(d) = make_float4(o4[u][0], o4[u][1], o4[u][2], o4[u][3]);
        }
        if (i < n_v2) {
          const int sp = i / TP, p = i % TP;
          lv[(2 * sp) * LD + p] = v2[u].x;
          if (2 * sp + 1 < ns) lv[(2 * sp + 1) * LD + p] = v2[u].y;
        }
      }
    }
  }
  wave_lds_sync();
  if (t >= tl.nt) return;
  float *dst = partial + tbase[t] * ns;
  for (int mg = 0; mg < rows_u; mg += 16 * MG) {
    if (mg > 0) load_u(mg);
    for (int n0 = 0; n0 < items; n0 += 16) {
      const int n = n0 + c16;
      const bool active = n < items;
      const int b = active ? n / ns : 0;
      const int sidx = active ? n - (n / ns) * ns : 0;
      v8bf bf[2];
      {
        const float *orow = lo + b * LD + 16 * q;
        const float *vrow = lv + sidx * LD + 16 * q;
#pragma unroll
        for (int k = 0; k < 16; k += 4) {
          const float4 o4 = *reinterpret_cast<const float4 *>(orow + k);
          const float4 v4 = *reinterpret_cast<const float4 *>(vrow + k);
          bf[k >> 3][(k & 7)] = (__bf16)(active ? o4.x * v4.x : 0.0f);
          bf[k >> 3][(k & 7) + 1] = (__bf16)(active ? o4.y * v4.y : 0.0f);
          bf[k >> 3][(k & 7) + 2] = (__bf16)(active ? o4.z * v4.z : 0.0f);
          bf[k >> 3][(k & 7) + 3] = (__bf16)(active ? o4.w * v4.w : 0.0f);
        }
      }
#pragma unroll
      for (int mb = 0; mb < MG; ++mb) {
        if (mg + mb * 16 >= rows_u) break;
        v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mb][0], bf[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mb][1], bf[1], acc, 0, 0, 0);
        if (active) {
          const int jo = b / BR, c = b - (b / BR) * BR;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int m = mg + mb * 16 + 4 * q + j;
            if (m < rows_u) {
              const int io = m / BL, r = m - (m / BL) * BL;
              dst[((((int64_t)io * noa + jo) * BL + r) * BR + c) * ns + sidx] = scale * acc[j];
            }
          }
        }
      }
    }
  }
}

// Vout[ob][ldv][E] (columns 0..ns) = sum over the contributions of block ob.  Each
// contribution is a contiguous run of per = E * ns partial sums, read as per / V vectors
// of V elements.  One wave per overlap block: when a run needs at most 64 lanes, the wave
// splits into G = 64 / (per / V) lane groups that walk the block's contributions G at a
// time (group g takes contributions g, g + G, ...), eight loads in flight per lane; the
// groups' sums are then added into group 0 in group order.  Longer runs are covered in
// chunks of 64 lanes with G = 1.  Contribution indices arrive 64 at a time with one vector
// load and reach the groups by lane shuffles.  Every sum has a fixed order (reproducible).
template <class T, int V>
__global__ __launch_bounds__(256) void k_vint_reduce(int64_t nblk, int ns, int E, int G,
                                                     const int64_t *__restrict__ cptr,
                                                     const int32_t *__restrict__ cidx,
                                                     const T *__restrict__ partial,
                                                     T *__restrict__ Vout, int ldv) {
  using TV = T __attribute__((ext_vector_type(V)));
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // consecutive overlap blocks on one XCD: their contribution runs share 128-byte lines
  // (runs of neighbouring blocks are neighbours in each tile's range), so a line fetched
  // for one block serves its neighbour from that XCD's L2
  const int64_t ob = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + w;
  if (ob >= nblk) return;
  const int per = ns * E;
  const int lpc = per / V;
  const int g = G > 1 ? lane / lpc : 0;
  const int jl = G > 1 ? lane - g * lpc : lane;
  const int64_t q0 = cptr[ob], q1 = cptr[ob + 1];
  for (int j0 = 0; j0 < lpc; j0 += 64) {
    const int j = j0 + jl;
    const bool on = g < G && j < lpc;
    const int64_t off = on ? (int64_t)j * V : 0;
    TV a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = TV(0);
    for (int64_t qb = q0; qb < q1; qb += 64) {
      const int cnt = (int)(q1 - qb < 64 ? q1 - qb : 64);
      const int mine = qb + lane < q1 ? cidx[qb + lane] : 0;
      // rounds of eight steps of G contributions (the last round predicated), so that
      // every round keeps eight independent loads in flight
      for (int k = 0; k * G < cnt; k += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int src = (k + u) * G + g;
          const int c = __shfl(mine, src & 63);
          if (on && src < cnt) a[u] += *reinterpret_cast<const TV *>(partial + (int64_t)c * per + off);
        }
      }
    }
    const TV sum = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    TV tot = sum;
    for (int gg = 1; gg < G; ++gg) {
      TV x;
#pragma unroll
      for (int c = 0; c < V; ++c) x[c] = __shfl(sum[c], gg * lpc + jl);
      tot += x;
    }
    if (g == 0 && j < lpc) {
#pragma unroll
      for (int c = 0; c < V; ++c) {
        const int idx = j * V + c, e = idx / ns, st = idx - (idx / ns) * ns;
        Vout[(ob * ldv + st) * E + e] = tot[c];
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
template <class T>
__global__ void k_alda(int64_t npts, const T *__restrict__ rho, double floor, T *__restrict__ fxc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts) return;
  const double r = (double)rho[2 * i];
  // -(1/3) (3/pi)^{1/3} r^{-2/3}
  const double cx = 0.98474502184269654;   // (3/pi)^{1/3}
  fxc[i] = r >= floor ? (T)(-(cx / 3.0) * pow(r, -2.0 / 3.0)) : T(0);
}

// ---------------------------------------------------------------------------------------
#define TD_GRID_BDIM(BL_, BR_, ...)                                            \
  do {                                                                        \
    if (BL_ == 3 && BR_ == 2) { constexpr int BL = 3, BR = 2; __VA_ARGS__; }   \
    else if (BL_ == 2 && BR_ == 2) { constexpr int BL = 2, BR = 2; __VA_ARGS__; } \
    else if (BL_ == 1 && BR_ == 1) { constexpr int BL = 1, BR = 1; __VA_ARGS__; } \
    else if (BL_ == 3 && BR_ == 3) { constexpr int BL = 3, BR = 3; __VA_ARGS__; } \
    else if (BL_ == 4 && BR_ == 4) { constexpr int BL = 4, BR = 4; __VA_ARGS__; } \
    else if (BL_ == 5 && BR_ == 2) { constexpr int BL = 5, BR = 2; __VA_ARGS__; } \
    else throw Error{TDDFT_E_INVALID, "unsupported padded block shape"};        \
  } while (0)

#define TD_SAMPLE(T_, ST_, ...)                                                       \
  do {                                                                               \
    if (ST_ == SAMPLE_F64) { using S = double; __VA_ARGS__; }                        \
    else if (ST_ == SAMPLE_F32) { using S = float; __VA_ARGS__; }                    \
    else { using S = __hip_bfloat16; __VA_ARGS__; }                                  \
  } while (0)

template <class T>
void density(const DevTiles &tl, int stype, int BL, int BR, const T *X, int ldx, int xc0, int ns,
             T *out, int64_t pair_stride, double scale, hipStream_t s) {
  if (tl.nt == 0 || ns == 0) return;
  const int waves = tl.waves;
  const size_t lds = 0;
  const unsigned grid = (unsigned)((tl.nt + waves - 1) / waves);
#define TD_DENSITY_LAUNCH(NSC_, PB_) \
  TD_SAMPLE(T, stype, TD_GRID_BDIM(BL, BR, hipLaunchKernelGGL((k_density<T, S, BL, BR, NSC_, PB_>), dim3(grid), dim3(64 * waves), lds, s, tl, reinterpret_cast<const S *>(tl.usamp), reinterpret_cast<const S *>(tl.osamp), tl.pidx, X, ldx, xc0, ns, out, pair_stride, (T)scale)))
#define TD_DENSITY_LAUNCH_F64(NSC_) \
  TD_GRID_BDIM(BL, BR, hipLaunchKernelGGL((k_density<T, double, BL, BR, NSC_, true>), dim3(grid), dim3(64 * waves), lds, s, tl, reinterpret_cast<const double *>(tl.usamp), reinterpret_cast<const double *>(tl.osamp), tl.pidx, X, ldx, xc0, ns, out, pair_stride, (T)scale))
  // the broadcast form: FP32 with any samples, FP64 with FP64 samples (the FP64 handles)
  const bool bcast = tl.pbcast != 0 && (std::is_same<T, float>::value || stype == SAMPLE_F64);
  if (bcast) {
    if constexpr (std::is_same<T, float>::value) {
      if (ns <= 2) TD_DENSITY_LAUNCH(2, true);
      else if (ns <= 4) TD_DENSITY_LAUNCH(4, true);
      else TD_DENSITY_LAUNCH(8, true);
    } else {
      if (ns <= 2) TD_DENSITY_LAUNCH_F64(2);
      else if (ns <= 4) TD_DENSITY_LAUNCH_F64(4);
      else TD_DENSITY_LAUNCH_F64(8);
    }
  } else {
    if (ns <= 2) TD_DENSITY_LAUNCH(2, false);
    else if (ns <= 4) TD_DENSITY_LAUNCH(4, false);
    else TD_DENSITY_LAUNCH(8, false);
  }
#undef TD_DENSITY_LAUNCH
#undef TD_DENSITY_LAUNCH_F64
  TD_HIP(hipGetLastError());
}

template <class T>
void potential_integrals(const DevTiles &tl, const DevPartials &pa, int stype, int BL, int BR,
                         const T *V, int64_t pair_stride, int ns, T *partial, T *Vout, int ldv,
                         int64_t nblk_out, double scale, hipStream_t s, Prof *prof) {
  if (tl.nt == 0 || ns == 0) return;
  const int E = BL * BR;
  if (prof) prof->begin(ST_VINT, s);
  const unsigned grid = (unsigned)((tl.nt + 3) / 4);
  if constexpr (std::is_same<T, float>::value) {
    const size_t lds = 4 * (size_t)(tl.maxrows_r + ns) * (TP + 4) * sizeof(float);
    if (lds > tl.lds_limit) throw Error{TDDFT_E_INVALID, "too many functions per grid tile for the LDS budget"};
    if (stype == SAMPLE_BF16)
      TD_GRID_BDIM(BL, BR, hipLaunchKernelGGL((k_vint_mfma_bf16<BL, BR>), dim3(grid), dim3(256), lds, s, tl, pa.tbase, reinterpret_cast<const __hip_bfloat16 *>(tl.usamp), reinterpret_cast<const __hip_bfloat16 *>(tl.osamp), V, pair_stride, ns, partial, (float)scale));
    else
      TD_SAMPLE(T, stype, TD_GRID_BDIM(BL, BR, hipLaunchKernelGGL((k_vint_mfma<S, BL, BR>), dim3(grid), dim3(256), lds, s, tl, pa.tbase, reinterpret_cast<const S *>(tl.usamp), reinterpret_cast<const S *>(tl.osamp), V, pair_stride, ns, partial, (float)scale)));
  } else {
    // FP64 samples on FP64 MFMA when the staged rows fit the LDS; the vector form otherwise.
    // Two tiles (waves) per workgroup: a wave's FP64 rows take twice the LDS of FP32 ones.
    const size_t lds = 2 * (size_t)(tl.maxrows_r + ns) * (TP + 2) * sizeof(double);
    if (stype == SAMPLE_F64 && lds <= tl.lds_limit)
      TD_GRID_BDIM(BL, BR, hipLaunchKernelGGL((k_vint_mfma64<BL, BR>), dim3((unsigned)((tl.nt + 1) / 2)), dim3(128), lds, s, tl, pa.tbase, reinterpret_cast<const double *>(tl.usamp), reinterpret_cast<const double *>(tl.osamp), reinterpret_cast<const double *>(V), pair_stride, ns, reinterpret_cast<double *>(partial), (double)scale));
    else
      TD_SAMPLE(T, stype, TD_GRID_BDIM(BL, BR, hipLaunchKernelGGL((k_vint<T, S, BL, BR>), dim3(grid), dim3(256), 0, s, tl, pa.tbase, reinterpret_cast<const S *>(tl.usamp), reinterpret_cast<const S *>(tl.osamp), V, pair_stride, ns, partial, (T)scale)));
  }
  TD_HIP(hipGetLastError());
  if (prof) prof->end(ST_VINT, s);
  if (nblk_out == 0) return;
  if (prof) prof->begin(ST_VINT_REDUCE, s);
  // widest vector that divides a contribution run (16 bytes at most)
  const int per = ns * E;
  constexpr int VW = 16 / sizeof(T);
  const int vw = per % VW == 0 ? VW : (per % 2 == 0 ? 2 : 1);
  const int lpc = per / vw;
  const int G = lpc <= 64 ? 64 / lpc : 1;
  const dim3 grid_r((unsigned)((nblk_out + 3) / 4));
  if (vw == VW)
    hipLaunchKernelGGL((k_vint_reduce<T, VW>), grid_r, dim3(256), 0, s, nblk_out, ns, E, G, pa.cptr, pa.cidx, partial, Vout, ldv);
  else if (vw == 2)
    hipLaunchKernelGGL((k_vint_reduce<T, 2>), grid_r, dim3(256), 0, s, nblk_out, ns, E, G, pa.cptr, pa.cidx, partial, Vout, ldv);
  else
    hipLaunchKernelGGL((k_vint_reduce<T, 1>), grid_r, dim3(256), 0, s, nblk_out, ns, E, G, pa.cptr, pa.cidx, partial, Vout, ldv);
  TD_HIP(hipGetLastError());
  if (prof) prof->end(ST_VINT_REDUCE, s);
}

template <class T>
void alda_kernel(int64_t npts, const T *rho_pairs, double floor, T *fxc, hipStream_t s) {
  if (npts == 0) return;
  hipLaunchKernelGGL((k_alda<T>), dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s, npts,
                     rho_pairs, floor, fxc);
  TD_HIP(hipGetLastError());
}

template void density<double>(const DevTiles &, int, int, int, const double *, int, int, int,
                              double *, int64_t, double, hipStream_t);
template void density<float>(const DevTiles &, int, int, int, const float *, int, int, int,
                             float *, int64_t, double, hipStream_t);
template void potential_integrals<double>(const DevTiles &, const DevPartials &, int, int, int,
                                          const double *, int64_t, int, double *, double *, int,
                                          int64_t, double, hipStream_t, Prof *);
template void potential_integrals<float>(const DevTiles &, const DevPartials &, int, int, int,
                                         const float *, int64_t, int, float *, float *, int,
                                         int64_t, double, hipStream_t, Prof *);
template void alda_kernel<double>(int64_t, const double *, double, double *, hipStream_t);
template void alda_kernel<float>(int64_t, const float *, double, float *, hipStream_t);

}  // namespace tddft
