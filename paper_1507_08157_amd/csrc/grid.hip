// Real-space grid kernels on 4x4x4 point tiles.
//
// Samples of both function sets are stored tile-major: for every tile, the rows (one per
// function of every atom touching the tile, 64 values each) are contiguous, so each wave
// streams a tile's samples with fully coalesced loads and keeps them in LDS.
//
//  * response density (Sec. III.A):   rho_s(r) = sum_ab u_a(r) P_s,ab o_b(r)
//    per tile: psi_a = sum_b P_ab o_b, then rho = sum_a u_a psi_a, P blocks read with
//    wave-uniform (scalar) loads; also used once for rho0 = 2 sum o K^v o.
//  * potential integrals (Sec. II.C, V_SCF^{chi phi}):  V_s,ab = h^3 sum_r u_a V_s o_b
//    per tile the (u-atom, o-atom) block products are reduced over the 64 points in
//    registers, summed over a brick of tiles in LDS, written per brick to a partial-sum
//    buffer and reduced per block in a fixed order (no global atomics, deterministic).
//  * ALDA exchange kernel f_xc = -(1/3)(3/pi)^{1/3} rho0^{-2/3} (Sec. II.A, xc part).
// Grid fields are tile-major complex pairs: state 2k in the real part, 2k+1 in the
// imaginary part of field k, so the Hartree FFT transforms two states at once.
#include <algorithm>

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

// ---------------------------------------------------------------------------------------
// One wave per tile.  The tile's sample rows are staged in LDS once; for each chunk of NSP
// states the P blocks of every (u-atom, o-atom) pair of the tile are staged too (coalesced
// loads, zero for pairs outside R and states beyond ns), so the FMA loop is branch-free and
// reads P with broadcast LDS loads.
template <class T, class S, int BL, int BR>
__global__ __launch_bounds__(256) void k_density(DevTiles tl, const T *__restrict__ X, int ldx,
                                                 int xc0, int ns, T *__restrict__ out,
                                                 int64_t pair_stride, T scale) {
  extern __shared__ unsigned char lds_raw[];
  constexpr int E = BL * BR;
  constexpr int NSP = 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int p = threadIdx.x & 63;
  const int t = blockIdx.x * (blockDim.x >> 6) + w;
  const size_t per_wave = (size_t)tl.maxrows * TP + (size_t)tl.maxpairs * NSP * E;
  T *lu = reinterpret_cast<T *>(lds_raw) + (size_t)w * per_wave;
  T *lp = lu + (size_t)tl.maxrows * TP;
  int nua = 0, noa = 0, u0 = 0, o0 = 0;
  if (t < tl.nt) {
    u0 = tl.uptr[t];
    nua = tl.uptr[t + 1] - u0;
    o0 = tl.optr[t];
    noa = tl.optr[t + 1] - o0;
  }
  T *lo = lu + (size_t)nua * BL * TP;
  {
    const S *us = reinterpret_cast<const S *>(tl.usamp) + (int64_t)u0 * BL * TP;
    const S *os = reinterpret_cast<const S *>(tl.osamp) + (int64_t)o0 * BR * TP;
    for (int r = 0; r < nua * BL; ++r) lu[r * TP + p] = cvt<T>(us[r * TP + p]);
    for (int r = 0; r < noa * BR; ++r) lo[r * TP + p] = cvt<T>(os[r * TP + p]);
  }
  const int npair = nua * noa;
  const int32_t *pid = tl.pidx + (t < tl.nt ? tl.pptr[t] : 0);
  using T2 = typename Vec2<T>::type;
  for (int s0 = 0; s0 < ns; s0 += NSP) {
    __syncthreads();
    for (int idx = p; idx < npair * NSP * E; idx += 64) {
      const int pr = idx / (NSP * E);
      const int rem = idx - pr * (NSP * E);
      const int sk = rem / E;
      const int pb = pid[pr];
      T v = T(0);
      if (pb >= 0 && s0 + sk < ns) v = X[((int64_t)pb * ldx + xc0 + s0) * E + rem];
      lp[idx] = v;
    }
    __syncthreads();
    if (t >= tl.nt) continue;
    T acc[NSP];
#pragma unroll
    for (int k = 0; k < NSP; ++k) acc[k] = T(0);
    for (int i = 0; i < nua; ++i) {
      T tmp[NSP][BL];
#pragma unroll
      for (int k = 0; k < NSP; ++k)
#pragma unroll
        for (int r = 0; r < BL; ++r) tmp[k][r] = T(0);
      const T *Pi = lp + (size_t)i * noa * NSP * E;
      for (int j = 0; j < noa; ++j) {
        T o[BR];
#pragma unroll
        for (int c = 0; c < BR; ++c) o[c] = lo[(j * BR + c) * TP + p];
        const T *Pj = Pi + (size_t)j * NSP * E;
#pragma unroll
        for (int k = 0; k < NSP; ++k)
#pragma unroll
          for (int r = 0; r < BL; ++r)
#pragma unroll
            for (int c = 0; c < BR; ++c) tmp[k][r] += Pj[k * E + r * BR + c] * o[c];
      }
#pragma unroll
      for (int r = 0; r < BL; ++r) {
        const T u = lu[(i * BL + r) * TP + p];
#pragma unroll
        for (int k = 0; k < NSP; ++k) acc[k] += u * tmp[k][r];
      }
    }
    const int nk = min(NSP, ns - s0);
    T2 v0, v1;
    v0.x = scale * acc[0];
    v0.y = nk > 1 ? scale * acc[1] : T(0);
    *reinterpret_cast<T2 *>(out + (int64_t)(s0 / 2) * pair_stride + ((int64_t)t * TP + p) * 2) = v0;
    if (nk > 2) {
      v1.x = scale * acc[2];
      v1.y = nk > 3 ? scale * acc[3] : T(0);
      *reinterpret_cast<T2 *>(out + (int64_t)(s0 / 2 + 1) * pair_stride + ((int64_t)t * TP + p) * 2) = v1;
    }
  }
}

// ---------------------------------------------------------------------------------------
// One workgroup per brick of tiles.  Per tile the (u-atom, o-atom) block integrals are
// reduced over the 64 points in registers (one pair per lane) and added into the brick's
// LDS accumulator; the accumulator is then written, without atomics, to the brick's slots
// of a partial-sum buffer that k_vint_reduce sums per overlap block in a fixed order.
template <class T, class S, int BL, int BR>
__global__ __launch_bounds__(256) void k_vint(DevTiles tl, DevBricks br, const T *__restrict__ V,
                                              int64_t pair_stride, int ns,
                                              T *__restrict__ partial, T scale) {
  extern __shared__ unsigned char lds_raw[];
  constexpr int E = BL * BR;
  constexpr int LD = TP + 1;   // padded rows: lanes reading different rows hit different banks
  constexpr int SC = 8;        // states per register chunk
  T *acc = reinterpret_cast<T *>(lds_raw);
  const size_t acc_len = ((size_t)br.max_slots * ns * E + 1) & ~(size_t)1;
  T *stage = acc + acc_len;
  const int b = blockIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  T *my = stage + (size_t)w * ((size_t)br.max_rows * LD + (size_t)ns * TP);
  const int bno = br.no[b];
  const int nslots = br.nu[b] * bno;
  for (int i = threadIdx.x; i < nslots * ns * E; i += blockDim.x) acc[i] = T(0);
  const int t0 = br.tptr[b];
  const int ntile = br.tptr[b + 1] - t0;
  const int nw = blockDim.x >> 6;
  for (int round = 0; round < ntile; round += nw) {
    __syncthreads();
    const int k = round + w;
    int t = -1, nua = 0, noa = 0, u0 = 0, o0 = 0;
    if (k < ntile) {
      t = br.tiles[t0 + k];
      u0 = tl.uptr[t];
      nua = tl.uptr[t + 1] - u0;
      o0 = tl.optr[t];
      noa = tl.optr[t + 1] - o0;
    }
    T *lu = my;
    T *lo = lu + (size_t)nua * BL * LD;
    T *lv = lo + (size_t)noa * BR * LD;
    if (t >= 0) {
      const S *us = reinterpret_cast<const S *>(tl.usamp) + (int64_t)u0 * BL * TP;
      const S *os = reinterpret_cast<const S *>(tl.osamp) + (int64_t)o0 * BR * TP;
      for (int r = 0; r < nua * BL; ++r) lu[r * LD + lane] = cvt<T>(us[r * TP + lane]);
      for (int r = 0; r < noa * BR; ++r) lo[r * LD + lane] = cvt<T>(os[r * TP + lane]);
      for (int s = 0; s < ns; ++s)
        lv[s * TP + lane] = V[(int64_t)(s >> 1) * pair_stride + ((int64_t)t * TP + lane) * 2 + (s & 1)];
    }
    __syncthreads();
    if (t >= 0) {
      for (int item = lane; item < nua * noa; item += 64) {
        const int i = item / noa, j = item - (item / noa) * noa;
        const int slot = br.ubl[u0 + i] * bno + br.obl[o0 + j];
        for (int s0 = 0; s0 < ns; s0 += SC) {
          const int nk = min(SC, ns - s0);
          T a[SC][E];
#pragma unroll
          for (int q = 0; q < SC; ++q)
#pragma unroll
            for (int e = 0; e < E; ++e) a[q][e] = T(0);
          for (int pt = 0; pt < TP; ++pt) {
            T uo[E];
#pragma unroll
            for (int r = 0; r < BL; ++r) {
              const T u = lu[(i * BL + r) * LD + pt];
#pragma unroll
              for (int c = 0; c < BR; ++c) uo[r * BR + c] = u * lo[(j * BR + c) * LD + pt];
            }
#pragma unroll
            for (int q = 0; q < SC; ++q) {
              const T v = (q < nk) ? lv[(s0 + q) * TP + pt] : T(0);
#pragma unroll
              for (int e = 0; e < E; ++e) a[q][e] += uo[e] * v;
            }
          }
#pragma unroll
          for (int q = 0; q < SC; ++q)
            if (q < nk)
#pragma unroll
              for (int e = 0; e < E; ++e) atomicAdd(&acc[((size_t)slot * ns + s0 + q) * E + e], a[q][e]);
        }
      }
    }
  }
  __syncthreads();
  T *dst = partial + br.sptr[b] * ns * E;
  for (int idx = threadIdx.x; idx < nslots * ns * E; idx += blockDim.x) dst[idx] = scale * acc[idx];
}

// Vout[ob][ldv][E] (columns 0..ns) = sum over the (brick, slot) contributions of block ob
template <class T>
__global__ __launch_bounds__(256) void k_vint_reduce(int64_t nblk, int ns, int E,
                                                     const int64_t *__restrict__ cptr,
                                                     const int64_t *__restrict__ cslot,
                                                     const T *__restrict__ partial,
                                                     T *__restrict__ Vout, int ldv) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int per = ns * E;
  if (gid >= nblk * per) return;
  const int64_t ob = gid / per;
  const int r = (int)(gid - ob * per);
  T acc = T(0);
  for (int64_t q = cptr[ob]; q < cptr[ob + 1]; ++q) acc += partial[cslot[q] * per + r];
  const int s = r / E, e = r - (r / E) * E;
  Vout[((int64_t)ob * ldv + s) * E + e] = acc;
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
  const size_t per_wave = ((size_t)tl.maxrows * TP + (size_t)tl.maxpairs * 4 * BL * BR) * sizeof(T);
  if (per_wave > tl.lds_limit) throw Error{TDDFT_E_INVALID, "too many functions per grid tile for the LDS budget"};
  const int waves = (int)std::max<size_t>(1, std::min<size_t>(4, tl.lds_limit / per_wave));
  const size_t lds = (size_t)waves * per_wave;
  const unsigned grid = (unsigned)((tl.nt + waves - 1) / waves);
  TD_SAMPLE(T, stype, TD_GRID_BDIM(BL, BR, hipLaunchKernelGGL((k_density<T, S, BL, BR>), dim3(grid), dim3(64 * waves), lds, s, tl, X, ldx, xc0, ns, out, pair_stride, (T)scale)));
  TD_HIP(hipGetLastError());
}

template <class T>
void potential_integrals(const DevTiles &tl, const DevBricks &br, int stype, int BL, int BR,
                         const T *V, int64_t pair_stride, int ns, T *partial, T *Vout, int ldv,
                         int64_t nblk_out, double scale, hipStream_t s, Prof *prof) {
  if (br.nb == 0 || ns == 0) return;
  const int E = BL * BR;
  const size_t acc_len = ((size_t)br.max_slots * ns * E + 1) & ~(size_t)1;
  const size_t per_wave = ((size_t)br.max_rows * (TP + 1) + (size_t)ns * TP) * sizeof(T);
  int waves = 4;
  while (waves > 1 && acc_len * sizeof(T) + waves * per_wave > tl.lds_limit) --waves;
  const size_t lds = acc_len * sizeof(T) + (size_t)waves * per_wave;
  if (lds > tl.lds_limit) throw Error{TDDFT_E_INVALID, "potential-integral accumulator exceeds the LDS budget"};
  if (prof) prof->begin(ST_VINT, s);
  TD_SAMPLE(T, stype, TD_GRID_BDIM(BL, BR, hipLaunchKernelGGL((k_vint<T, S, BL, BR>), dim3(br.nb), dim3(64 * waves), lds, s, tl, br, V, pair_stride, ns, partial, (T)scale)));
  TD_HIP(hipGetLastError());
  if (prof) prof->end(ST_VINT, s);
  const int64_t n = nblk_out * ns * E;
  if (n == 0) return;
  if (prof) prof->begin(ST_VINT_REDUCE, s);
  hipLaunchKernelGGL((k_vint_reduce<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nblk_out, ns, E,
                     br.cptr, br.cslot, partial, Vout, ldv);
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
template void potential_integrals<double>(const DevTiles &, const DevBricks &, int, int, int,
                                          const double *, int64_t, int, double *, double *, int,
                                          int64_t, double, hipStream_t, Prof *);
template void potential_integrals<float>(const DevTiles &, const DevBricks &, int, int, int,
                                         const float *, int64_t, int, float *, float *, int,
                                         int64_t, double, hipStream_t, Prof *);
template void alda_kernel<double>(int64_t, const double *, double, double *, hipStream_t);
template void alda_kernel<float>(int64_t, const float *, double, float *, hipStream_t);

}  // namespace tddft
