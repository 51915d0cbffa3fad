// Learned block preconditioner: two-atom features, the network (forward, backward, Adam)
// and the per-block operations the solver needs.
//
// The network is small (inputs ~30, width 128, outputs BU*BO + 1) and is evaluated once per
// solve on one row per block of the response pattern, so its kernels are plain vector
// code: one thread per output element for the layers, fixed-size row chunks with a
// fixed-order reduction for the weight gradients (reproducible sums).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "handle.h"
#include "learned.h"

namespace tddft {

// ---------------------------------------------------------------------------------------
// features (host, once per handle)
int n_features(int bu, int bo) { return bu * (bu + 1) + bo * (bo + 1) + bu + bo + bu * bo + 1; }

// generalised eigenvalues of the leading n x n part of (H, S) (row-major, leading dim B),
// ascending, written to out[0..n); out[n..B) = 0.  Cholesky S = L L^T, C = L^-1 H L^-T,
// cyclic Jacobi rotations on C.
static void small_gen_eig(int n, int B, const double *S, const double *H, double *out) {
  constexpr int LD = 5;   // largest block
  double L[LD * LD] = {0}, C[LD * LD] = {0}, Y[LD * LD] = {0};
  for (int j = 0; j < n; ++j) {
    double d = S[j * B + j];
    for (int k = 0; k < j; ++k) d -= L[j * LD + k] * L[j * LD + k];
    TD_REQUIRE(d > 0.0, "diagonal overlap block is not positive definite");
    L[j * LD + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double v = S[i * B + j];
      for (int k = 0; k < j; ++k) v -= L[i * LD + k] * L[j * LD + k];
      L[i * LD + j] = v / L[j * LD + j];
    }
  }
  // Y = L^-1 H (forward substitution per column), C = Y L^-T
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double v = H[i * B + c];
      for (int k = 0; k < i; ++k) v -= L[i * LD + k] * Y[k * LD + c];
      Y[i * LD + c] = v / L[i * LD + i];
    }
  for (int r = 0; r < n; ++r)
    for (int j = 0; j < n; ++j) {
      double v = Y[r * LD + j];
      for (int k = 0; k < j; ++k) v -= C[r * LD + k] * L[j * LD + k];
      C[r * LD + j] = v / L[j * LD + j];
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) C[i * LD + j] = C[j * LD + i] = 0.5 * (C[i * LD + j] + C[j * LD + i]);
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += C[i * LD + j] * C[i * LD + j];
        if (i != j) off += C[i * LD + j] * C[i * LD + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = C[p * LD + q];
        if (apq == 0.0) continue;
        const double theta = (C[q * LD + q] - C[p * LD + p]) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(tt * tt + 1.0), sn = tt * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double a = C[k * LD + p], b = C[k * LD + q];
          C[k * LD + p] = c * a - sn * b;
          C[k * LD + q] = sn * a + c * b;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double a = C[p * LD + k], b = C[q * LD + k];
          C[p * LD + k] = c * a - sn * b;
          C[q * LD + k] = sn * a + c * b;
        }
      }
  }
  for (int i = 0; i < B; ++i) out[i] = i < n ? C[i * LD + i] : 0.0;
  std::sort(out, out + n);
}

void build_features(Handle &h, const HostBsr &Su, const HostBsr &Hu, const HostBsr &So,
                    const HostBsr &Ho, const tddft_system &sys) {
  const int bu = h.BU, bo = h.BO;
  TD_REQUIRE(bu <= 5 && bo <= 5, "block size");
  const int nf = n_features(bu, bo);
  struct Atom {
    std::vector<double> su, hu, eig;
    double c[3];
  };
  auto atoms = [&](const HostBsr &S, const HostBsr &H, const std::vector<int> &off, int B,
                   const tddft_functions &fs) {
    std::vector<Atom> out(off.size() - 1);
    for (size_t I = 0; I + 1 < off.size(); ++I) {
      const int64_t k = S.pat.find((int)I, (int)I);
      const int64_t kh = H.pat.find((int)I, (int)I);
      TD_REQUIRE(k >= 0 && kh >= 0, "missing diagonal block");
      const double *sb = S.val.data() + k * B * B;
      const double *hb = H.val.data() + kh * B * B;
      Atom &a = out[I];
      for (int r = 0; r < B; ++r)
        for (int c = r; c < B; ++c) {
          a.su.push_back(sb[r * B + c]);
          a.hu.push_back(hb[r * B + c]);
        }
      a.eig.assign(B, 0.0);
      small_gen_eig(off[I + 1] - off[I], B, sb, hb, a.eig.data());
      const int f = off[I];
      for (int d = 0; d < 3; ++d)
        a.c[d] = (fs.origin[3 * f + d] + 0.5 * (fs.extent[3 * f + d] - 1)) * (h.L[d] / h.n[d]);
    }
    return out;
  };
  std::vector<Atom> au = atoms(Su, Hu, h.uoff, bu, sys.vir);
  std::vector<Atom> ao = atoms(So, Ho, h.ooff, bo, sys.occ);
  std::vector<float> F((size_t)h.nR * nf);
  for (int I = 0; I < h.nbu; ++I)
    for (int64_t k = h.R.rowptr[I]; k < h.R.rowptr[I + 1]; ++k) {
      const Atom &u = au[I], &o = ao[h.R.col[k]];
      float *row = F.data() + (size_t)k * nf;
      int q = 0;
      for (double x : u.su) row[q++] = (float)x;
      for (double x : u.hu) row[q++] = (float)x;
      for (double x : o.su) row[q++] = (float)x;
      for (double x : o.hu) row[q++] = (float)x;
      for (double x : u.eig) row[q++] = (float)x;
      for (double x : o.eig) row[q++] = (float)x;
      for (int a = 0; a < bu; ++a)
        for (int b = 0; b < bo; ++b) row[q++] = (float)(u.eig[a] - o.eig[b]);
      double d2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        double x = u.c[d] - o.c[d];
        x -= h.L[d] * std::round(x / h.L[d]);
        d2 += x * x;
      }
      row[q++] = (float)std::sqrt(d2);
    }
  h.nfeat = nf;
  h.features.upload(F, h.stream);
  TD_HIP(hipStreamSynchronize(h.stream));
}

// ---------------------------------------------------------------------------------------
// network kernels
__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
  const float sg = 1.0f / (1.0f + expf(-z));
  return sg * (1.0f + z * (1.0f - sg));
}

// A = act(X^ W + b) (and Z = X^ W + b), X^ = (X - mean) / std when mean is given
__global__ __launch_bounds__(256) void k_dense(int64_t rows, int K, int N, const float *__restrict__ X,
                                               const float *__restrict__ mean,
                                               const float *__restrict__ stdv,
                                               const __hip_bfloat16 *__restrict__ W,
                                               const float *__restrict__ b, float *__restrict__ Z,
                                               float *__restrict__ A, int act) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= rows * N) return;
  const int64_t r = gid / N;
  const int j = (int)(gid - r * N);
  const float *x = X + r * K;
  float acc = b[j];
  for (int k = 0; k < K; ++k) {
    float xv = x[k];
    if (mean) xv = (xv - mean[k]) / stdv[k];
    acc += xv * __bfloat162float(W[(int64_t)k * N + j]);
  }
  if (Z) Z[gid] = acc;
  A[gid] = act ? silu_f(acc) : acc;
}

// loss of the scaling and guess heads; dY; per-block partial losses (fixed-order tree)
__global__ __launch_bounds__(256) void k_loss(int64_t rows, int E, const float *__restrict__ Y,
                                              const float *__restrict__ gr,
                                              const float *__restrict__ gs,
                                              const float *__restrict__ tg, float inv_scale,
                                              float *__restrict__ dY, double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (r < rows) {
    const int no = E + 1;
    for (int e = 0; e < E; ++e) {
      const float g = gr[r * E + e];
      const float res = Y[r * no + e] * g - gs[r * E + e];
      dY[r * no + e] = res * g * inv_scale;
      l += 0.5 * (double)res * res * inv_scale;
    }
    const float lw = Y[r * no + E] - tg[r];
    dY[r * no + E] = lw;
    l += 0.5 * (double)lw * lw;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[r][k] = dsilu(Z[r][k]) * sum_j D[r][j] W[k][j]
__global__ __launch_bounds__(256) void k_backprop(int64_t rows, int N, int K, const float *__restrict__ D,
                                                  const __hip_bfloat16 *__restrict__ W,
                                                  const float *__restrict__ Z, float *__restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= rows * K) return;
  const int64_t r = gid / K;
  const int k = (int)(gid - r * K);
  const float *d = D + r * N;
  const __hip_bfloat16 *w = W + (int64_t)k * N;
  float acc = 0.0f;
  for (int j = 0; j < N; ++j) acc += d[j] * __bfloat162float(w[j]);
  out[gid] = acc * dsilu_f(Z[gid]);
}

// per chunk of rows: [K*N] sums of A[r][k] D[r][j] (A normalised when mean is given), then
// [N] sums of D[r][j]
__global__ __launch_bounds__(256) void k_wgrad(int64_t rows, int K, int N, int64_t chunk,
                                               const float *__restrict__ A,
                                               const float *__restrict__ mean,
                                               const float *__restrict__ stdv,
                                               const float *__restrict__ D, float *__restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = r0 + chunk < rows ? r0 + chunk : rows;
  const int len = K * N + N;
  for (int idx = threadIdx.x; idx < len; idx += blockDim.x) {
    float acc = 0.0f;
    if (idx < K * N) {
      const int k = idx / N, j = idx - (idx / N) * N;
      const float mu = mean ? mean[k] : 0.0f, is = mean ? 1.0f / stdv[k] : 1.0f;
      for (int64_t r = r0; r < r1; ++r) acc += (A[r * K + k] - mu) * is * D[r * N + j];
    } else {
      const int j = idx - K * N;
      for (int64_t r = r0; r < r1; ++r) acc += D[r * N + j];
    }
    part[(int64_t)blockIdx.x * len + idx] = acc;
  }
}

__global__ void k_sum_parts(int nchunk, int len, const float *__restrict__ part, float *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float acc = 0.0f;
  for (int c = 0; c < nchunk; ++c) acc += part[(int64_t)c * len + i];
  out[i] = acc;
}

__global__ void k_adam(int64_t n, float *__restrict__ p, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_to_bf16(int64_t n, const float *__restrict__ src, __hip_bfloat16 *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = __float2bfloat16(src[i]);
}

// per chunk of rows: column sums and sums of squares (FP64)
__global__ __launch_bounds__(256) void k_colstats(int64_t rows, int K, int64_t chunk,
                                                  const float *__restrict__ X, double *__restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = r0 + chunk < rows ? r0 + chunk : rows;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    double s1 = 0.0, s2 = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
      const double x = X[r * K + k];
      s1 += x;
      s2 += x * x;
    }
    part[(int64_t)blockIdx.x * 2 * K + k] = s1;
    part[(int64_t)blockIdx.x * 2 * K + K + k] = s2;
  }
}

static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

// ---------------------------------------------------------------------------------------
// network host logic
void Mlp::init(int n_in_, int width_, int n_out_, hipStream_t st) {
  TD_REQUIRE(n_in_ > 0 && width_ > 0 && n_out_ > 1 && n_in_ <= 4096 && width_ <= 4096 && n_out_ <= 4096,
             "network sizes");
  n_in = n_in_;
  width = width_;
  n_out = n_out_;
  s = st;
  const int64_t sz[6] = {(int64_t)n_in * width, width, (int64_t)width * width, width,
                         (int64_t)width * n_out, n_out};
  int64_t o = 0;
  for (int i = 0; i < 6; ++i) {
    off[i] = o;
    o += sz[i];
  }
  nparams = o;
  p.alloc(nparams);
  g.alloc(nparams);
  m.alloc(nparams);
  v.alloc(nparams);
  wb.alloc(nparams);
  mean.alloc(n_in);
  stdv.alloc(n_in);
  TD_HIP(hipMemsetAsync(m.p, 0, nparams * sizeof(float), s));
  TD_HIP(hipMemsetAsync(v.p, 0, nparams * sizeof(float), s));
  std::vector<float> mu(n_in, 0.0f), sd(n_in, 1.0f);
  mean.upload(mu, s);
  stdv.upload(sd, s);
  t = 0;
  TD_HIP(hipStreamSynchronize(s));
}

void Mlp::randomize(uint64_t seed) {
  std::vector<float> h(nparams, 0.0f);
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 0x2545F4914F6CDD1Dull;
  auto next = [&]() {   // SplitMix64
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const int fan[3] = {n_in, width, width};
  for (int layer = 0; layer < 3; ++layer) {
    const double sd = std::sqrt(2.0 / fan[layer]);
    for (int64_t i = off[2 * layer]; i < off[2 * layer + 1]; i += 2) {   // Box-Muller pairs
      const double u1 = ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
      const double u2 = ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
      const double rr = std::sqrt(-2.0 * std::log(u1));
      h[i] = (float)(sd * rr * std::cos(2.0 * M_PI * u2));
      if (i + 1 < off[2 * layer + 1]) h[i + 1] = (float)(sd * rr * std::sin(2.0 * M_PI * u2));
    }
  }
  p.upload(h, s);
  refresh_bf16();
}

void Mlp::refresh_bf16() {
  hipLaunchKernelGGL(k_to_bf16, dim3(nb256(nparams)), dim3(256), 0, s, nparams, p.p, wb.p);
  TD_HIP(hipGetLastError());
  TD_HIP(hipStreamSynchronize(s));
}

void Mlp::set(const float *params, const float *mu, const float *sd) {
  if (params) {
    p.upload(params, nparams, s);
    TD_HIP(hipMemsetAsync(m.p, 0, nparams * sizeof(float), s));
    TD_HIP(hipMemsetAsync(v.p, 0, nparams * sizeof(float), s));
    t = 0;
  }
  if (mu && sd) {
    for (int k = 0; k < n_in; ++k) TD_REQUIRE(sd[k] > 0.0f && std::isfinite(sd[k]) && std::isfinite(mu[k]), "normalisation");
    mean.upload(mu, n_in, s);
    stdv.upload(sd, n_in, s);
  }
  refresh_bf16();
}

void Mlp::get(float *params, float *mu, float *sd) const {
  if (params) TD_HIP(hipMemcpyAsync(params, p.p, nparams * sizeof(float), hipMemcpyDeviceToHost, s));
  if (mu) TD_HIP(hipMemcpyAsync(mu, mean.p, n_in * sizeof(float), hipMemcpyDeviceToHost, s));
  if (sd) TD_HIP(hipMemcpyAsync(sd, stdv.p, n_in * sizeof(float), hipMemcpyDeviceToHost, s));
  TD_HIP(hipStreamSynchronize(s));
}

static constexpr int64_t kChunk = 512;

void Mlp::fit_normalisation(int64_t rows, const float *X) {
  TD_REQUIRE(rows > 1 && X, "normalisation needs at least two rows");
  const int64_t nchunk = (rows + kChunk - 1) / kChunk;
  DevBuf<double> pt((size_t)nchunk * 2 * n_in);
  hipLaunchKernelGGL(k_colstats, dim3((unsigned)nchunk), dim3(256), 0, s, rows, n_in, kChunk, X, pt.p);
  TD_HIP(hipGetLastError());
  std::vector<double> hpt((size_t)nchunk * 2 * n_in);
  TD_HIP(hipMemcpyAsync(hpt.data(), pt.p, hpt.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  TD_HIP(hipStreamSynchronize(s));
  std::vector<float> mu(n_in), sd(n_in);
  for (int k = 0; k < n_in; ++k) {
    double s1 = 0.0, s2 = 0.0;
    for (int64_t c = 0; c < nchunk; ++c) {
      s1 += hpt[(size_t)c * 2 * n_in + k];
      s2 += hpt[(size_t)c * 2 * n_in + n_in + k];
    }
    const double mval = s1 / rows;
    const double var = std::max(0.0, s2 / rows - mval * mval);
    mu[k] = (float)mval;
    sd[k] = (float)std::max(std::sqrt(var), 1e-6);
  }
  set(nullptr, mu.data(), sd.data());
}

void Mlp::forward(int64_t rows, const float *X, float *Y) {
  TD_REQUIRE(rows >= 0 && (rows == 0 || (X && Y)), "forward arguments");
  if (rows == 0) return;
  if (rows > rows_cap) {
    act.alloc((size_t)rows * 4 * width);
    rows_cap = rows;
  }
  float *Z1 = act.p, *A1 = Z1 + rows * width, *Z2 = A1 + rows * width, *A2 = Z2 + rows * width;
  hipLaunchKernelGGL(k_dense, dim3(nb256(rows * width)), dim3(256), 0, s, rows, n_in, width, X,
                     mean.p, stdv.p, wb.p + off[0], p.p + off[1], Z1, A1, 1);
  hipLaunchKernelGGL(k_dense, dim3(nb256(rows * width)), dim3(256), 0, s, rows, width, width, A1,
                     (const float *)nullptr, (const float *)nullptr, wb.p + off[2], p.p + off[3], Z2, A2, 1);
  hipLaunchKernelGGL(k_dense, dim3(nb256(rows * n_out)), dim3(256), 0, s, rows, width, n_out, A2,
                     (const float *)nullptr, (const float *)nullptr, wb.p + off[4], p.p + off[5],
                     (float *)nullptr, Y, 0);
  TD_HIP(hipGetLastError());
}

double Mlp::train_step(int64_t rows, const float *X, const float *gr, const float *gs,
                       const float *tg, double loss_scale, double lr, float *grad_out) {
  TD_REQUIRE(rows > 0 && X && gr && gs && tg && loss_scale > 0.0 && lr > 0.0, "train_step arguments");
  const int E = n_out - 1;
  DevBuf<float> Y((size_t)rows * n_out), dY((size_t)rows * n_out), D2((size_t)rows * width),
      D1((size_t)rows * width);
  forward(rows, X, Y.p);
  float *Z1 = act.p, *A1 = Z1 + rows * width, *Z2 = A1 + rows * width, *A2 = Z2 + rows * width;
  const unsigned nbl = nb256(rows);
  DevBuf<double> lp(nbl);
  hipLaunchKernelGGL(k_loss, dim3(nbl), dim3(256), 0, s, rows, E, Y.p, gr, gs, tg,
                     (float)(1.0 / loss_scale), dY.p, lp.p);
  // hidden deltas
  hipLaunchKernelGGL(k_backprop, dim3(nb256(rows * width)), dim3(256), 0, s, rows, n_out, width,
                     dY.p, wb.p + off[4], Z2, D2.p);
  hipLaunchKernelGGL(k_backprop, dim3(nb256(rows * width)), dim3(256), 0, s, rows, width, width,
                     D2.p, wb.p + off[2], Z1, D1.p);
  TD_HIP(hipGetLastError());
  // weight and bias gradients: row chunks, then a fixed-order sum
  const int64_t nchunk = (rows + kChunk - 1) / kChunk;
  const int lens[3] = {n_in * width + width, width * width + width, width * n_out + n_out};
  const int maxlen = std::max(lens[0], std::max(lens[1], lens[2]));
  if ((int64_t)part.n < nchunk * maxlen) part.alloc((size_t)nchunk * maxlen);
  struct L { int K, N; const float *A, *mu, *sd, *D; int64_t o; };
  const L layers[3] = {{n_in, width, X, mean.p, stdv.p, D1.p, off[0]},
                       {width, width, A1, nullptr, nullptr, D2.p, off[2]},
                       {width, n_out, A2, nullptr, nullptr, dY.p, off[4]}};
  for (int l = 0; l < 3; ++l) {
    const L &y = layers[l];
    hipLaunchKernelGGL(k_wgrad, dim3((unsigned)nchunk), dim3(256), 0, s, rows, y.K, y.N, kChunk,
                       y.A, y.mu, y.sd, y.D, part.p);
    hipLaunchKernelGGL(k_sum_parts, dim3(nb256(lens[l])), dim3(256), 0, s, (int)nchunk, lens[l],
                       part.p, g.p + y.o);
    TD_HIP(hipGetLastError());
  }
  std::vector<double> hl(nbl);
  TD_HIP(hipMemcpyAsync(hl.data(), lp.p, nbl * sizeof(double), hipMemcpyDeviceToHost, s));
  if (grad_out) TD_HIP(hipMemcpyAsync(grad_out, g.p, nparams * sizeof(float), hipMemcpyDeviceToDevice, s));
  // Adam
  ++t;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - std::pow(b1, (double)t)), c2 = (float)(1.0 - std::pow(b2, (double)t));
  hipLaunchKernelGGL(k_adam, dim3(nb256(nparams)), dim3(256), 0, s, nparams, p.p, g.p, m.p, v.p,
                     (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2);
  TD_HIP(hipGetLastError());
  refresh_bf16();   // synchronises the stream
  double loss = 0.0;
  for (double x : hl) loss += x;
  return loss;
}

namespace {
const char kMagic[8] = {'T', 'D', 'D', 'F', 'T', 'M', 'L', '1'};
}

std::vector<unsigned char> Mlp::blob() const {
  const size_t hdr = 8 + 4 * sizeof(int32_t);
  std::vector<unsigned char> b(hdr + (2 * (size_t)n_in + nparams) * sizeof(float));
  std::memcpy(b.data(), kMagic, 8);
  const int32_t dims[4] = {n_in, width, n_out, 0};
  std::memcpy(b.data() + 8, dims, sizeof(dims));
  float *f = reinterpret_cast<float *>(b.data() + hdr);
  get(f + 2 * n_in, f, f + n_in);
  return b;
}

void Mlp::from_blob(const void *data, int64_t size, hipStream_t st) {
  const size_t hdr = 8 + 4 * sizeof(int32_t);
  TD_REQUIRE(data && size >= (int64_t)hdr && std::memcmp(data, kMagic, 8) == 0, "not a tddft model blob");
  int32_t dims[4];
  std::memcpy(dims, (const unsigned char *)data + 8, sizeof(dims));
  init(dims[0], dims[1], dims[2], st);
  TD_REQUIRE(size == (int64_t)(hdr + (2 * (size_t)n_in + nparams) * sizeof(float)), "model blob size");
  std::vector<float> f(2 * (size_t)n_in + nparams);
  std::memcpy(f.data(), (const unsigned char *)data + hdr, f.size() * sizeof(float));
  for (float x : f) TD_REQUIRE(std::isfinite(x), "model blob holds non-finite values");
  set(f.data() + 2 * n_in, f.data(), f.data() + n_in);
}

// ---------------------------------------------------------------------------------------
// per-block operations of the solver
template <class T>
__global__ void k_block_scale(int64_t n, int ncol, int E, const T *__restrict__ c,
                              const T *__restrict__ X, T *__restrict__ Z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t per = (int64_t)ncol * E;
  const int64_t b = i / per;
  const int e = (int)(i % E);
  Z[i] = c[b * E + e] * X[i];
}

template <class T>
void block_scale(int64_t nblk, int ncol, int E, const T *c, const T *X, T *Z, hipStream_t s) {
  const int64_t n = nblk * ncol * E;
  if (n == 0) return;
  hipLaunchKernelGGL((k_block_scale<T>), dim3(nb256(n)), dim3(256), 0, s, n, ncol, E, c, X, Z);
  TD_HIP(hipGetLastError());
}

template <class T>
__global__ void k_split_outputs(int64_t nblk, int E, const float *__restrict__ Y, T *__restrict__ c,
                                float *__restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nblk * (E + 1)) return;
  const int64_t b = i / (E + 1);
  const int e = (int)(i - b * (E + 1));
  if (e < E) c[b * E + e] = (T)Y[i];
  else t[b] = Y[i];
}

template <class T>
void split_outputs(int64_t nblk, int E, const float *Y, T *c, float *t, hipStream_t s) {
  const int64_t n = nblk * (E + 1);
  if (n == 0) return;
  hipLaunchKernelGGL((k_split_outputs<T>), dim3(nb256(n)), dim3(256), 0, s, nblk, E, Y, c, t);
  TD_HIP(hipGetLastError());
}

__global__ void k_block_sqnorm(int64_t nblk, int n, int64_t nnz, const int64_t *__restrict__ voff,
                               const int32_t *__restrict__ shape, const double *__restrict__ P,
                               double *__restrict__ w) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  const int sz = (shape[b] & 0xff) * (shape[b] >> 8);
  double acc = 0.0;
  for (int i = 0; i < n; ++i)
    for (int e = 0; e < sz; ++e) {
      const double x = P[(int64_t)i * nnz + voff[b] + e];
      acc += x * x;
    }
  w[b] = acc;
}

void block_sqnorm(int64_t nblk, int n, int64_t nnz, const int64_t *voff, const int32_t *shape,
                  const double *Pq, double *w, hipStream_t s) {
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_block_sqnorm, dim3(nb256(nblk)), dim3(256), 0, s, nblk, n, nnz, voff, shape, Pq, w);
  TD_HIP(hipGetLastError());
}

__global__ void k_guess_t(int64_t nblk, const double *__restrict__ w, double inv_total, float *__restrict__ t) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nblk) t[b] = (float)log10(w[b] * inv_total + 1e-8);
}

void guess_from_weights(int64_t nblk, const double *w, double inv_total, float *t, hipStream_t s) {
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_guess_t, dim3(nb256(nblk)), dim3(256), 0, s, nblk, w, inv_total, t);
  TD_HIP(hipGetLastError());
}

template void block_scale<double>(int64_t, int, int, const double *, const double *, double *, hipStream_t);
template void block_scale<float>(int64_t, int, int, const float *, const float *, float *, hipStream_t);
template void split_outputs<double>(int64_t, int, const float *, double *, float *, hipStream_t);
template void split_outputs<float>(int64_t, int, const float *, float *, float *, hipStream_t);

}  // namespace tddft
