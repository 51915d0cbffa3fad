// Periodic Hartree solve plus ALDA term on the real-space grid (Sec. II.A: the Coulomb
// and f_xc parts of the coupling kernel, evaluated as the response potential of
// rho^{q} in Sec. III.A).
//
//   V_s(r) = IFFT[ 4 pi / |G|^2 FFT[rho_s] ](r) + f_xc(r) rho_s(r),   G = 0 term dropped
//
// Two real states share one complex field (real and imaginary part): the Poisson kernel is
// real and even in G, so the transform of the pair yields both potentials exactly.
// Mixed-radix (2, 3, 4, 5, 7, 8) Stockham transforms run on lines held in LDS:
//   pass 1  x-lines, forward   tile-major fields -> natural-order work array
//   pass 2  y-lines, forward   in place
//   pass 3  z-lines, forward, times the Poisson kernel, inverse     in place
//   pass 4  y-lines, inverse   in place
//   pass 5  x-lines, inverse, plus f_xc rho          work array -> tile-major fields
#include <algorithm>

#include "internal.h"
#include "kernels.h"

namespace tddft {

template <class T> struct C2;
template <> struct C2<double> { using type = double2; };
template <> struct C2<float> { using type = float2; };

template <int R>
__host__ __device__ constexpr double root_cos(int k) {
  if constexpr (R == 3) {
    constexpr double c[3] = {1.0, -0.5, -0.5};
    return c[k];
  } else if constexpr (R == 5) {
    constexpr double c[5] = {1.0, 0.309016994374947424102, -0.809016994374947424102,
                             -0.809016994374947424102, 0.309016994374947424102};
    return c[k];
  } else if constexpr (R == 7) {
    constexpr double c[7] = {1.0, 0.623489801858733530525, -0.222520933956314404289,
                             -0.900968867902419126236, -0.900968867902419126236,
                             -0.222520933956314404289, 0.623489801858733530525};
    return c[k];
  } else {  // 8
    constexpr double c[8] = {1.0, 0.707106781186547524401, 0.0, -0.707106781186547524401,
                             -1.0, -0.707106781186547524401, 0.0, 0.707106781186547524401};
    return c[k];
  }
}

template <int R>
__host__ __device__ constexpr double root_sin(int k) {
  if constexpr (R == 3) {
    constexpr double s[3] = {0.0, 0.866025403784438646764, -0.866025403784438646764};
    return s[k];
  } else if constexpr (R == 5) {
    constexpr double s[5] = {0.0, 0.951056516295153572116, 0.587785252292473129169,
                             -0.587785252292473129169, -0.951056516295153572116};
    return s[k];
  } else if constexpr (R == 7) {
    constexpr double s[7] = {0.0, 0.781831482468029808708, 0.974927912181823607018,
                             0.433883739117558120476, -0.433883739117558120476,
                             -0.974927912181823607018, -0.781831482468029808708};
    return s[k];
  } else {
    constexpr double s[8] = {0.0, 0.707106781186547524401, 1.0, 0.707106781186547524401,
                             0.0, -0.707106781186547524401, -1.0, -0.707106781186547524401};
    return s[k];
  }
}

template <class T2>
__device__ __forceinline__ T2 cmul(T2 a, T2 b) {
  T2 r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// small DFT of length R, exponent sign SIGN (-1 forward, +1 inverse)
template <class T, int R, int SIGN>
__device__ __forceinline__ void dft(typename C2<T>::type (&v)[R]) {
  using T2 = typename C2<T>::type;
  if constexpr (R == 2) {
    T2 a = v[0], b = v[1];
    v[0].x = a.x + b.x; v[0].y = a.y + b.y;
    v[1].x = a.x - b.x; v[1].y = a.y - b.y;
  } else if constexpr (R == 4) {
    T2 a0, a1, a2, a3;
    a0.x = v[0].x + v[2].x; a0.y = v[0].y + v[2].y;
    a1.x = v[0].x - v[2].x; a1.y = v[0].y - v[2].y;
    a2.x = v[1].x + v[3].x; a2.y = v[1].y + v[3].y;
    const T dx = v[1].x - v[3].x, dy = v[1].y - v[3].y;
    // (v1 - v3) * (SIGN i)
    a3.x = -SIGN * dy; a3.y = SIGN * dx;
    v[0].x = a0.x + a2.x; v[0].y = a0.y + a2.y;
    v[2].x = a0.x - a2.x; v[2].y = a0.y - a2.y;
    v[1].x = a1.x + a3.x; v[1].y = a1.y + a3.y;
    v[3].x = a1.x - a3.x; v[3].y = a1.y - a3.y;
  } else if constexpr (R == 8) {
    // X[2m] = DFT4(v[k] + v[k+4]),  X[2m+1] = DFT4((v[k] - v[k+4]) w^k),  w = e^{SIGN i pi/4}
    const T h = (T)0.707106781186547524401;
    T2 a[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k].x = v[k].x + v[k + 4].x; a[k].y = v[k].y + v[k + 4].y;
      b[k].x = v[k].x - v[k + 4].x; b[k].y = v[k].y - v[k + 4].y;
    }
    {
      const T x = b[1].x, y = b[1].y;
      b[1].x = (x - SIGN * y) * h; b[1].y = (SIGN * x + y) * h;
    }
    {
      const T x = b[2].x, y = b[2].y;
      b[2].x = -SIGN * y; b[2].y = SIGN * x;
    }
    {
      const T x = b[3].x, y = b[3].y;
      b[3].x = (-x - SIGN * y) * h; b[3].y = (SIGN * x - y) * h;
    }
    dft<T, 4, SIGN>(a);
    dft<T, 4, SIGN>(b);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      v[2 * m] = a[m];
      v[2 * m + 1] = b[m];
    }
  } else {
    T2 o[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
      T2 acc = v[0];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const int k = (r * m) % R;
        const T c = (T)root_cos<R>(k);
        const T s = (T)(SIGN * root_sin<R>(k));
        acc.x += v[r].x * c - v[r].y * s;
        acc.y += v[r].x * s + v[r].y * c;
      }
      o[m] = acc;
    }
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = o[m];
  }
}

// Index divisions by run-time sizes use fdiv (kernels.h): every index divided here is below
// 16 * 4096 = 2^16 and every divisor at most 4096, where the multiply-high is exact.
struct AxisDev {
  int n, npass;
  int radix[12];
  int tw_off[12];
  uint32_t m_nb[12];   // div_magic(n / radix[p])
  uint32_t m_ns[12];   // div_magic(product of the radices before pass p)
};

// one Stockham pass over `nlines` lines (stride ldl) of length N held in LDS
template <class T, int R, int SIGN>
__device__ void fft_pass(const typename C2<T>::type *__restrict__ in,
                         typename C2<T>::type *__restrict__ out, int N, int Ns, int ldl,
                         int nlines, const typename C2<T>::type *__restrict__ tw, uint32_t m_nb,
                         uint32_t m_ns) {
  using T2 = typename C2<T>::type;
  const int nb = N / R;
  const int total = nlines * nb;
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int line = fdiv(q, m_nb);
    const int j = q - line * nb;
    const T2 *src = in + line * ldl;
    T2 *dst = out + line * ldl;
    const int k = j - fdiv(j, m_ns) * Ns;
    T2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * nb];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        T2 w = tw[k * (R - 1) + r - 1];
        if (SIGN > 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    dft<T, R, SIGN>(v);
    const int d = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[d + r * Ns] = v[r];
  }
}

// In-place variant of a pass: each thread first reads the inputs of all its butterflies
// (at most max(1, 8 / R) of them), the workgroup synchronises, and the results then
// overwrite the same buffer.  One LDS buffer instead of two doubles the workgroups a CU can
// hold; the host takes this form when every pass of the axis fits (nlines * N / R <=
// max(1, 8 / R) * blockDim) and the axis has no factor 7 (whose O(R^2) DFT would raise the
// register count of every pass, and with it cost the occupancy gained).
template <class T, int R, int SIGN>
__device__ void fft_pass_inplace(typename C2<T>::type *__restrict__ buf, int N, int Ns, int ldl,
                                 int nlines, const typename C2<T>::type *__restrict__ tw,
                                 uint32_t m_nb, uint32_t m_ns) {
  using T2 = typename C2<T>::type;
  constexpr int NIT = R >= 8 ? 1 : 8 / R;
  const int nb = N / R;
  const int total = nlines * nb;
  T2 v[NIT][R];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int q = threadIdx.x + it * blockDim.x;
    if (q < total) {
      const int line = fdiv(q, m_nb), j = q - line * nb;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = buf[line * ldl + j + r * nb];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int q = threadIdx.x + it * blockDim.x;
    if (q < total) {
      const int line = fdiv(q, m_nb), j = q - line * nb;
      const int k = j - fdiv(j, m_ns) * Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          T2 w = tw[k * (R - 1) + r - 1];
          if (SIGN > 0) w.y = -w.y;
          v[it][r] = cmul(v[it][r], w);
        }
      }
      dft<T, R, SIGN>(v[it]);
      const int d = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[line * ldl + d + r * Ns] = v[it][r];
    }
  }
}

// full transform of the lines in buffer a (scratch b, unused when INPL); returns the
// buffer with the result
template <class T, int SIGN, bool INPL>
__device__ typename C2<T>::type *fft_lines(typename C2<T>::type *a, typename C2<T>::type *b,
                                           int ldl, int nlines, const AxisDev &ax,
                                           const typename C2<T>::type *tw) {
  int Ns = 1;
  for (int p = 0; p < ax.npass; ++p) {
    const int R = ax.radix[p];
    const typename C2<T>::type *t = tw + ax.tw_off[p];
    if constexpr (INPL) {
      switch (R) {
        case 2: fft_pass_inplace<T, 2, SIGN>(a, ax.n, Ns, ldl, nlines, t, ax.m_nb[p], ax.m_ns[p]); break;
        case 3: fft_pass_inplace<T, 3, SIGN>(a, ax.n, Ns, ldl, nlines, t, ax.m_nb[p], ax.m_ns[p]); break;
        case 4: fft_pass_inplace<T, 4, SIGN>(a, ax.n, Ns, ldl, nlines, t, ax.m_nb[p], ax.m_ns[p]); break;
        case 5: fft_pass_inplace<T, 5, SIGN>(a, ax.n, Ns, ldl, nlines, t, ax.m_nb[p], ax.m_ns[p]); break;
        default: fft_pass_inplace<T, 8, SIGN>(a, ax.n, Ns, ldl, nlines, t, ax.m_nb[p], ax.m_ns[p]); break;
      }
      __syncthreads();
    } else {
      switch (R) {
        case 2: fft_pass<T, 2, SIGN>(a, b, ax.n, Ns, ldl, nlines, t, ax.m_nb[p], ax.m_ns[p]); break;
        case 3: fft_pass<T, 3, SIGN>(a, b, ax.n, Ns, ldl, nlines, t, ax.m_nb[p], ax.m_ns[p]); break;
        case 4: fft_pass<T, 4, SIGN>(a, b, ax.n, Ns, ldl, nlines, t, ax.m_nb[p], ax.m_ns[p]); break;
        case 5: fft_pass<T, 5, SIGN>(a, b, ax.n, Ns, ldl, nlines, t, ax.m_nb[p], ax.m_ns[p]); break;
        case 7: fft_pass<T, 7, SIGN>(a, b, ax.n, Ns, ldl, nlines, t, ax.m_nb[p], ax.m_ns[p]); break;
        default: fft_pass<T, 8, SIGN>(a, b, ax.n, Ns, ldl, nlines, t, ax.m_nb[p], ax.m_ns[p]); break;
      }
      __syncthreads();
      typename C2<T>::type *tmp = a;
      a = b;
      b = tmp;
    }
    Ns *= R;
  }
  return a;
}

// global loads each thread keeps in flight when staging lines (one memory round trip per
// batch: a loop with a run-time trip count would otherwise wait on every iteration)
constexpr int kLoadBatch = 8;

struct GeomDev {
  int nx, ny, nz, ntx, nty, ntz;
  int64_t pair_tile;   // elements (complex) per field in tile-major layout
  int64_t pair_work;   // elements per field in natural layout
  uint32_t m_nx, m_nz; // div_magic(nx), div_magic(nz)
};

// ---- pass 1: x forward, tile-major -> natural ---------------------------------------------
// one workgroup per row of tiles (ty, tz): 16 x-lines, contiguous in the tile-major layout
template <class T, bool INPL, int NT>
__global__ __launch_bounds__(NT) void k_fft_x_fwd(GeomDev g, AxisDev ax,
                                                   const typename C2<T>::type *__restrict__ tw,
                                                   const typename C2<T>::type *__restrict__ fields,
                                                   typename C2<T>::type *__restrict__ work) {
  using T2 = typename C2<T>::type;
  extern __shared__ unsigned char lds_raw[];
  T2 *a = reinterpret_cast<T2 *>(lds_raw);
  const int ldl = g.nx + 1;   // odd row length (in complex values): lines start on different banks
  T2 *b = INPL ? a : a + 16 * ldl;
  const int row = blockIdx.x;           // ty + nty * tz
  const int ty = row % g.nty, tz = row / g.nty;
  const int pair = blockIdx.y;
  const T2 *src = fields + pair * g.pair_tile + (int64_t)row * g.ntx * TP;
  const int ntot = g.ntx * TP;
  // loads in batches of kLoadBatch per thread, all in flight before the LDS writes
  for (int b0 = 0; b0 < ntot; b0 += kLoadBatch * NT) {
    T2 v[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = b0 + u * NT + (int)threadIdx.x;
      if (e < ntot) v[u] = src[e];
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = b0 + u * NT + (int)threadIdx.x;
      const int tx = e / TP, p = e - (e / TP) * TP;
      const int px = p & 3, l = p >> 2;
      const int x = tx * 4 + px;
      if (e < ntot && x < g.nx) a[l * ldl + x] = v[u];
    }
  }
  __syncthreads();
  T2 *res = fft_lines<T, -1, INPL>(a, b, ldl, 16, ax, tw);
  for (int e = threadIdx.x; e < 16 * g.nx; e += blockDim.x) {
    const int l = fdiv(e, g.m_nx), x = e - l * g.nx;
    const int y = ty * 4 + (l & 3), z = tz * 4 + (l >> 2);
    if (y < g.ny && z < g.nz)
      work[pair * g.pair_work + ((int64_t)z * g.ny + y) * g.nx + x] = res[l * ldl + x];
  }
}

// ---- pass 2/4: y lines in place ---------------------------------------------------------
constexpr int XB = 16;   // x-columns per workgroup in the strided passes

template <class T, int SIGN, bool INPL, int NT>
__global__ __launch_bounds__(NT) void k_fft_y(GeomDev g, AxisDev ax,
                                               const typename C2<T>::type *__restrict__ tw,
                                               typename C2<T>::type *__restrict__ work, int rev) {
  using T2 = typename C2<T>::type;
  extern __shared__ unsigned char lds_raw[];
  T2 *a = reinterpret_cast<T2 *>(lds_raw);
  const int ldl = g.ny + 1;
  T2 *b = INPL ? a : a + XB * ldl;
  const int nxb = (g.nx + XB - 1) / XB;
  // rev: workgroups in reverse dispatch order.  The forward pass takes it, so that it starts
  // on the lines the x pass wrote last (pair npair - 1, top z-planes), which the memory-side
  // cache still holds (256^3: 0.161 -> 0.143 ms; the other passes gain nothing from order)
  const int bx = rev ? (int)(gridDim.x - 1 - blockIdx.x) : (int)blockIdx.x;
  const int pair = rev ? (int)(gridDim.y - 1 - blockIdx.y) : (int)blockIdx.y;
  const int xb = bx % nxb, z = bx / nxb;
  const int x0 = xb * XB;
  const int nl = min(XB, g.nx - x0);
  T2 *base = work + pair * g.pair_work + (int64_t)z * g.ny * g.nx + x0;
  for (int b0 = 0; b0 < XB * g.ny; b0 += kLoadBatch * NT) {
    T2 v[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = b0 + u * NT + (int)threadIdx.x;
      const int y = e / XB, l = e - y * XB;
      if (e < XB * g.ny && l < nl) v[u] = base[(int64_t)y * g.nx + l];
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = b0 + u * NT + (int)threadIdx.x;
      const int y = e / XB, l = e - y * XB;
      if (e < XB * g.ny && l < nl) a[l * ldl + y] = v[u];
    }
  }
  __syncthreads();
  T2 *res = fft_lines<T, SIGN, INPL>(a, b, ldl, nl, ax, tw);
  for (int e = threadIdx.x; e < XB * g.ny; e += blockDim.x) {
    const int y = e / XB, l = e - y * XB;
    if (l < nl) base[(int64_t)y * g.nx + l] = res[l * ldl + y];
  }
}

// ---- pass 3: z lines, forward, Poisson kernel, inverse -----------------------------------
template <class T, bool INPL, int NT>
__global__ __launch_bounds__(NT) void k_fft_z_poisson(GeomDev g, AxisDev ax,
                                                       const typename C2<T>::type *__restrict__ tw,
                                                       typename C2<T>::type *__restrict__ work,
                                                       double gx, double gy, double gz,
                                                       double scale) {
  using T2 = typename C2<T>::type;
  extern __shared__ unsigned char lds_raw[];
  T2 *a = reinterpret_cast<T2 *>(lds_raw);
  const int ldl = g.nz + 1;
  T2 *b = INPL ? a : a + XB * ldl;
  const int nxb = (g.nx + XB - 1) / XB;
  const int xb = blockIdx.x % nxb, y = blockIdx.x / nxb;
  const int x0 = xb * XB;
  const int nl = min(XB, g.nx - x0);
  const int64_t plane = (int64_t)g.ny * g.nx;
  T2 *base = work + blockIdx.y * g.pair_work + (int64_t)y * g.nx + x0;
  for (int b0 = 0; b0 < XB * g.nz; b0 += kLoadBatch * NT) {
    T2 v[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = b0 + u * NT + (int)threadIdx.x;
      const int z = e / XB, l = e - z * XB;
      if (e < XB * g.nz && l < nl) v[u] = base[(int64_t)z * plane + l];
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = b0 + u * NT + (int)threadIdx.x;
      const int z = e / XB, l = e - z * XB;
      if (e < XB * g.nz && l < nl) a[l * ldl + z] = v[u];
    }
  }
  __syncthreads();
  T2 *res = fft_lines<T, -1, INPL>(a, b, ldl, nl, ax, tw);
  // multiply by 4 pi / |G|^2 (G = 0 -> 0) including the 1/(nx ny nz) normalisation
  const int ky = y <= g.ny / 2 ? y : y - g.ny;
  for (int e = threadIdx.x; e < nl * g.nz; e += blockDim.x) {
    const int l = fdiv(e, g.m_nz), z = e - l * g.nz;
    const int x = x0 + l;
    const int kx = x <= g.nx / 2 ? x : x - g.nx;
    const int kz = z <= g.nz / 2 ? z : z - g.nz;
    // in the field's precision (a double division per value would cost more than the
    // transform's own arithmetic in FP32)
    const T fx = (T)gx * (T)kx, fy = (T)gy * (T)ky, fz = (T)gz * (T)kz;
    const T G2 = fx * fx + fy * fy + fz * fz;
    const T f = G2 > T(0) ? (T)scale / G2 : T(0);
    T2 v = res[l * ldl + z];
    v.x *= f;
    v.y *= f;
    res[l * ldl + z] = v;
  }
  __syncthreads();
  T2 *other = INPL ? res : ((res == a) ? b : a);
  T2 *res2 = fft_lines<T, 1, INPL>(res, other, ldl, nl, ax, tw);
  for (int e = threadIdx.x; e < XB * g.nz; e += blockDim.x) {
    const int z = e / XB, l = e - z * XB;
    if (l < nl) base[(int64_t)z * plane + l] = res2[l * ldl + z];
  }
}

// ---- pass 5: x inverse, natural -> tile-major, plus f_xc rho ---------------------------------
template <class T, bool INPL, int NT>
__global__ __launch_bounds__(NT) void k_fft_x_inv(GeomDev g, AxisDev ax,
                                                   const typename C2<T>::type *__restrict__ tw,
                                                   const typename C2<T>::type *__restrict__ work,
                                                   typename C2<T>::type *__restrict__ fields,
                                                   const T *__restrict__ fxc, int use_fxc) {
  using T2 = typename C2<T>::type;
  extern __shared__ unsigned char lds_raw[];
  T2 *a = reinterpret_cast<T2 *>(lds_raw);
  const int ldl = g.nx + 1;   // odd row length (in complex values): lines start on different banks
  T2 *b = INPL ? a : a + 16 * ldl;
  const int row = blockIdx.x;
  const int ty = row % g.nty, tz = row / g.nty;
  const int pair = blockIdx.y;
  for (int b0 = 0; b0 < 16 * g.nx; b0 += kLoadBatch * NT) {
    T2 v[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = b0 + u * NT + (int)threadIdx.x;
      const int l = fdiv(e, g.m_nx), x = e - l * g.nx;
      const int y = ty * 4 + (l & 3), z = tz * 4 + (l >> 2);
      v[u].x = T(0);
      v[u].y = T(0);
      if (e < 16 * g.nx && y < g.ny && z < g.nz) v[u] = work[pair * g.pair_work + ((int64_t)z * g.ny + y) * g.nx + x];
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = b0 + u * NT + (int)threadIdx.x;
      const int l = fdiv(e, g.m_nx), x = e - l * g.nx;
      if (e < 16 * g.nx) a[l * ldl + x] = v[u];
    }
  }
  __syncthreads();
  T2 *res = fft_lines<T, 1, INPL>(a, b, ldl, 16, ax, tw);
  T2 *dst = fields + pair * g.pair_tile + (int64_t)row * g.ntx * TP;
  const T *fx = fxc + (int64_t)row * g.ntx * TP;
  const int ntot = g.ntx * TP;
  for (int b0 = 0; b0 < ntot; b0 += kLoadBatch * NT) {
    T2 rho[kLoadBatch];
    T f[kLoadBatch];
    if (use_fxc) {
#pragma unroll
      for (int u = 0; u < kLoadBatch; ++u) {
        const int e = b0 + u * NT + (int)threadIdx.x;
        if (e < ntot) {
          rho[u] = dst[e];
          f[u] = fx[e];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = b0 + u * NT + (int)threadIdx.x;
      if (e >= ntot) continue;
      const int tx = e / TP, p = e - (e / TP) * TP;
      const int px = p & 3, l = p >> 2;
      const int x = tx * 4 + px;
      const int y = ty * 4 + (l & 3), z = tz * 4 + (l >> 2);
      T2 v;
      v.x = T(0);
      v.y = T(0);
      if (x < g.nx && y < g.ny && z < g.nz) {
        v = res[l * ldl + x];
        if (use_fxc) {
          v.x += f[u] * rho[u].x;
          v.y += f[u] * rho[u].y;
        }
      }
      dst[e] = v;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Threads per workgroup of an axis pass: the smallest of 256, 512 and 1024 with which every
// radix pass fits the per-thread butterfly budget of fft_pass_inplace for 16 lines, so that
// the pass runs in place in one LDS buffer (a long axis such as 256 needs 512 threads: with
// 256 its radix-8 passes would need two buffers, halving the workgroups a CU holds); 0 when
// none does (a factor 7, or an axis longer than 1024 threads can cover), and then the pass
// takes two buffers on 256 threads.
std::vector<int> fft_inplace_threads(const AxisFFT &a) {
  std::vector<int> out;
  for (int nt : {256, 512, 1024}) {
    bool fits = true;
    for (int R : a.radix)
      if (R == 7 || 16 * (a.n / R) > (R >= 8 ? 1 : 8 / R) * nt) fits = false;
    if (fits) out.push_back(nt);
  }
  return out;
}

// LDS of one workgroup of an axis pass with `nt` threads (0: two buffers; line buffers of
// odd stride n + 1)
static size_t axis_lds_bytes(const AxisFFT &a, int nt, int lines, size_t elem) {
  return (nt > 0 ? 1 : 2) * (size_t)lines * (a.n + 1) * elem;
}

#define TD_COMMA(x) , x
// launch one pass kernel in its in-place form at the axis's thread count, or in the
// two-buffer form on 256 threads
#define TD_FFT_LAUNCH(KERN, TARGS, nt, grid, lds, ...)                                      \
  do {                                                                                    \
    switch (nt) {                                                                         \
      case 256: hipLaunchKernelGGL((KERN<TARGS, true, 256>), grid, dim3(256), lds, __VA_ARGS__); break;   \
      case 512: hipLaunchKernelGGL((KERN<TARGS, true, 512>), grid, dim3(512), lds, __VA_ARGS__); break;   \
      case 1024: hipLaunchKernelGGL((KERN<TARGS, true, 1024>), grid, dim3(1024), lds, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL((KERN<TARGS, false, 256>), grid, dim3(256), lds, __VA_ARGS__); break;  \
    }                                                                                     \
  } while (0)

size_t fft_lds_bytes(const FFTPlan &plan, size_t elem) {
  return std::max({axis_lds_bytes(plan.ax[0], plan.nt[0], 16, elem),
                   axis_lds_bytes(plan.ax[1], plan.nt[1], XB, elem),
                   axis_lds_bytes(plan.ax[2], plan.nt[2], XB, elem)});
}

static AxisDev axis_dev(const AxisFFT &a) {
  AxisDev d{};
  d.n = a.n;
  d.npass = (int)a.radix.size();
  int ns = 1;
  for (int i = 0; i < d.npass; ++i) {
    d.radix[i] = a.radix[i];
    d.tw_off[i] = a.tw_off[i];
    d.m_nb[i] = div_magic(a.n / a.radix[i]);
    d.m_ns[i] = div_magic(ns);
    ns *= a.radix[i];
  }
  return d;
}

template <class T>
void hartree_xc(const GridGeom &gg, const FFTPlan &plan, int npair, T *fields, T *work,
                const T *fxc, bool use_fxc, hipStream_t s, Prof *prof) {
  using T2 = typename C2<T>::type;
  if (npair == 0) return;
  GeomDev g{gg.n[0], gg.n[1], gg.n[2], gg.ntx, gg.nty, gg.ntz,
            (int64_t)gg.ntx * gg.nty * gg.ntz * TP, (int64_t)gg.n[0] * gg.n[1] * gg.n[2],
            div_magic(gg.n[0]), div_magic(gg.n[2])};
  const T2 *tw = reinterpret_cast<const T2 *>(std::is_same<T, double>::value ? (const void *)plan.tw64.p
                                                                             : (const void *)plan.tw32.p);
  int off[3] = {0, plan.ax[0].tw_len, plan.ax[0].tw_len + plan.ax[1].tw_len};
  AxisDev ax = axis_dev(plan.ax[0]), ay = axis_dev(plan.ax[1]), az = axis_dev(plan.ax[2]);
  T2 *F = reinterpret_cast<T2 *>(fields);
  T2 *W = reinterpret_cast<T2 *>(work);
  const double pi = 3.14159265358979323846;
  const double gx = 2.0 * pi / gg.L[0], gy = 2.0 * pi / gg.L[1], gz = 2.0 * pi / gg.L[2];
  const double scale = 4.0 * pi / ((double)gg.n[0] * gg.n[1] * gg.n[2]);
  const unsigned rows = (unsigned)(gg.nty * gg.ntz);
  const unsigned nxb = (unsigned)((gg.n[0] + XB - 1) / XB);
  const size_t lx = axis_lds_bytes(plan.ax[0], plan.nt[0], 16, sizeof(T2));
  const size_t ly = axis_lds_bytes(plan.ax[1], plan.nt[1], XB, sizeof(T2));
  const size_t lz = axis_lds_bytes(plan.ax[2], plan.nt[2], XB, sizeof(T2));
  Prof dummy;
  Prof &pf = prof ? *prof : dummy;
  const int tx = plan.nt[0], ty = plan.nt[1], tz = plan.nt[2];
  pf.begin(ST_FFT_X_FWD, s);
  TD_FFT_LAUNCH(k_fft_x_fwd, T, tx, dim3(rows, npair), lx, s, g, ax, tw + off[0], F, W);
  TD_HIP(hipGetLastError());
  pf.end(ST_FFT_X_FWD, s);
  pf.begin(ST_FFT_Y_FWD, s);
  TD_FFT_LAUNCH(k_fft_y, T TD_COMMA(-1), ty, dim3(nxb * gg.n[2], npair), ly, s, g, ay, tw + off[1], W, 1);
  TD_HIP(hipGetLastError());
  pf.end(ST_FFT_Y_FWD, s);
  pf.begin(ST_FFT_Z_POISSON, s);
  TD_FFT_LAUNCH(k_fft_z_poisson, T, tz, dim3(nxb * gg.n[1], npair), lz, s, g, az, tw + off[2], W, gx, gy, gz,
                scale);
  TD_HIP(hipGetLastError());
  pf.end(ST_FFT_Z_POISSON, s);
  pf.begin(ST_FFT_Y_INV, s);
  TD_FFT_LAUNCH(k_fft_y, T TD_COMMA(1), ty, dim3(nxb * gg.n[2], npair), ly, s, g, ay, tw + off[1], W, 0);
  TD_HIP(hipGetLastError());
  pf.end(ST_FFT_Y_INV, s);
  pf.begin(ST_FFT_X_INV, s);
  TD_FFT_LAUNCH(k_fft_x_inv, T, tx, dim3(rows, npair), lx, s, g, ax, tw + off[0], W, F, fxc, use_fxc ? 1 : 0);
  TD_HIP(hipGetLastError());
  pf.end(ST_FFT_X_INV, s);
}

template void hartree_xc<double>(const GridGeom &, const FFTPlan &, int, double *, double *,
                                 const double *, bool, hipStream_t, Prof *);
template void hartree_xc<float>(const GridGeom &, const FFTPlan &, int, float *, float *,
                                const float *, bool, hipStream_t, Prof *);

}  // namespace tddft
