// Oscillator strengths in the velocity form (the line strengths of Sec. IV.A, Table
// tab:azo, and of the spectra of Sec. IV.B; the paper prints no formula):
//   f_n = 2 / (3 omega_n) sum_alpha ( sum_ab P^p_n,ab G^alpha_ab )^2,
//   G^alpha_ab = h^3 sum_r u_a(r) (d_alpha o_b)(r),
// with d_alpha the second-order central difference on the periodic grid and P^p = X - Y
// in the mixed function space, Tsiper-normalised (<p_n, q_n> = 1, Sec. III.C).
#include <algorithm>
#include <array>
#include <thread>

#include "handle.h"

namespace tddft {

namespace {

// per axis: pairs (index in box A, index in box B) of the grid points the two periodic
// boxes share
void axis_pairs(int oa, int ea, int ob, int eb, int n, std::vector<std::pair<int, int>> &out) {
  out.clear();
  for (int i = 0; i < ea; ++i) {
    const int g = (oa + i) % n;
    const int j = ((g - ob) % n + n) % n;
    if (j < eb) out.emplace_back(i, j);
  }
}

// Central differences of one function on its box grown by one point on each side: the
// function is zero beyond its box, so its derivative is zero beyond the grown box.  An axis
// on which the grown box would reach round the cell takes the whole axis instead.
// go / ge: origin and extent of the grown box.
void box_gradient(const double *v, const int32_t *o, const int32_t *e, const int n[3],
                  const double h[3], int go[3], int ge[3], std::vector<double> (&d)[3]) {
  for (int a = 0; a < 3; ++a) {
    if (e[a] + 2 > n[a]) {
      go[a] = 0;
      ge[a] = n[a];
    } else {
      go[a] = ((o[a] - 1) % n[a] + n[a]) % n[a];
      ge[a] = e[a] + 2;
    }
  }
  const int64_t np = (int64_t)ge[0] * ge[1] * ge[2];
  for (int a = 0; a < 3; ++a) d[a].assign(np, 0.0);
  // value at global grid coordinates (periodic), zero outside the function's box
  auto at = [&](int gx, int gy, int gz) -> double {
    const int g[3] = {gx, gy, gz};
    int w[3];
    for (int a = 0; a < 3; ++a) {
      w[a] = ((g[a] - o[a]) % n[a] + n[a]) % n[a];
      if (w[a] >= e[a]) return 0.0;
    }
    return v[((int64_t)w[2] * e[1] + w[1]) * e[0] + w[0]];
  };
  for (int k = 0; k < ge[2]; ++k)
    for (int j = 0; j < ge[1]; ++j)
      for (int i = 0; i < ge[0]; ++i) {
        const int x = go[0] + i, y = go[1] + j, z = go[2] + k;   // global (unwrapped)
        const int64_t p = ((int64_t)k * ge[1] + j) * ge[0] + i;
        d[0][p] = (at(x + 1, y, z) - at(x - 1, y, z)) / (2.0 * h[0]);
        d[1][p] = (at(x, y + 1, z) - at(x, y - 1, z)) / (2.0 * h[1]);
        d[2][p] = (at(x, y, z + 1) - at(x, y, z - 1)) / (2.0 * h[2]);
      }
}

}  // namespace

// G^alpha on the blocks of R (C-ABI value layout, alpha-major) from the functions, FP64
void build_gradient_integrals(Handle &h, const tddft_functions &vir, const tddft_functions &occ) {
  std::vector<double> G((size_t)3 * h.nnzR, 0.0);
  const Pattern RT = transpose(h.R);
  double hs[3];
  for (int d = 0; d < 3; ++d) hs[d] = h.L[d] / h.n[d];
  const double dV = h.dV;
  auto work = [&](int J) {
    const int b0 = h.ooff[J], nbj = h.ooff[J + 1] - b0;
    std::vector<std::vector<double>> grads(nbj * 3);
    std::vector<std::array<int, 3>> gorig(nbj), gext(nbj);
    for (int b = 0; b < nbj; ++b) {
      std::vector<double> d[3];
      box_gradient(occ.val + occ.off[b0 + b], occ.origin + 3 * (b0 + b), occ.extent + 3 * (b0 + b),
                   h.n, hs, gorig[b].data(), gext[b].data(), d);
      for (int a = 0; a < 3; ++a) grads[b * 3 + a] = std::move(d[a]);
    }
    std::vector<std::pair<int, int>> px, py, pz;
    for (int64_t q = RT.rowptr[J]; q < RT.rowptr[J + 1]; ++q) {
      const int I = RT.col[q];
      const int64_t k = h.R.find(I, J);
      const int a0 = h.uoff[I], nai = h.uoff[I + 1] - a0;
      for (int ia = 0; ia < nai; ++ia) {
        const int fa = a0 + ia;
        const int *ou = vir.origin + 3 * fa, *eu = vir.extent + 3 * fa;
        for (int b = 0; b < nbj; ++b) {
          const int *oo = gorig[b].data(), *eo = gext[b].data();
          axis_pairs(ou[0], eu[0], oo[0], eo[0], h.n[0], px);
          if (px.empty()) continue;
          axis_pairs(ou[1], eu[1], oo[1], eo[1], h.n[1], py);
          if (py.empty()) continue;
          axis_pairs(ou[2], eu[2], oo[2], eo[2], h.n[2], pz);
          if (pz.empty()) continue;
          const double *u = vir.val + vir.off[fa];
          double s[3] = {0.0, 0.0, 0.0};
          for (const auto &z : pz)
            for (const auto &y : py) {
              const int64_t ru = ((int64_t)z.first * eu[1] + y.first) * eu[0];
              const int64_t rb = ((int64_t)z.second * eo[1] + y.second) * eo[0];
              for (const auto &x : px) {
                const double uv = u[ru + x.first];
                if (uv == 0.0) continue;
                for (int al = 0; al < 3; ++al) s[al] += uv * grads[b * 3 + al][rb + x.second];
              }
            }
          const int cs = nbj;
          for (int al = 0; al < 3; ++al)
            G[(size_t)al * h.nnzR + h.r_voff_host[k] + (size_t)ia * cs + b] = dV * s[al];
        }
      }
    }
  };
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      for (int J = (int)t; J < h.nbo; J += (int)nt) work(J);
    });
  for (auto &x : th) x.join();
  h.grad_uo.upload(G, h.stream);
  TD_HIP(hipStreamSynchronize(h.stream));
}

// partial sums of sum_k Pp[n][k] G[alpha][k]: one workgroup per chunk of k, FP64; the host
// adds the workgroups' partials in index order (reproducible)
__global__ __launch_bounds__(256) void k_moments(int n, int64_t nnz, const double *__restrict__ Pp,
                                                 const double *__restrict__ G, int64_t chunk,
                                                 double *__restrict__ partial) {
  __shared__ double red[256];
  const int64_t k0 = (int64_t)blockIdx.x * chunk, k1 = min(nnz, k0 + chunk);
  for (int s = 0; s < n; ++s)
    for (int al = 0; al < 3; ++al) {
      double acc = 0.0;
      for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x)
        acc += Pp[(int64_t)s * nnz + k] * G[(int64_t)al * nnz + k];
      red[threadIdx.x] = acc;
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
      }
      if (threadIdx.x == 0) partial[((int64_t)blockIdx.x * n + s) * 3 + al] = red[0];
      __syncthreads();
    }
}

void oscillator_strengths(Handle &h, int n, const double *omega, const double *Pp, double *f,
                          double *moments) {
  TD_REQUIRE(h.grad_uo.p != nullptr, "gradient integrals not available on this handle");
  const int64_t nnz = h.nnzR;
  const int64_t chunk = 1 << 16;
  const int nwg = (int)std::max<int64_t>(1, (nnz + chunk - 1) / chunk);
  DevBuf<double> part((size_t)nwg * n * 3);
  hipLaunchKernelGGL(k_moments, dim3(nwg), dim3(256), 0, h.stream, n, nnz, Pp, h.grad_uo.p, chunk, part.p);
  TD_HIP(hipGetLastError());
  std::vector<double> ph((size_t)nwg * n * 3);
  TD_HIP(hipMemcpyAsync(ph.data(), part.p, ph.size() * sizeof(double), hipMemcpyDeviceToHost, h.stream));
  TD_HIP(hipStreamSynchronize(h.stream));
  for (int s = 0; s < n; ++s) {
    double D[3] = {0.0, 0.0, 0.0};
    for (int w = 0; w < nwg; ++w)
      for (int al = 0; al < 3; ++al) D[al] += ph[((size_t)w * n + s) * 3 + al];
    f[s] = 2.0 / (3.0 * omega[s]) * (D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    if (moments)
      for (int al = 0; al < 3; ++al) moments[s * 3 + al] = D[al];
  }
}

}  // namespace tddft
