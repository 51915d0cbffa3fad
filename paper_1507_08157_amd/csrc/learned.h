// The learned block preconditioner: two-atom block features, the small network that maps
// them to an elementwise gradient scaling and a guess weight, and its training.
#pragma once

#include <string>
#include <vector>

#include "internal.h"

namespace tddft {

struct Handle;
struct HostBsr;

// features of every block of R (FP32, [nR][nfeat]) from the host inputs of tddft_create
void build_features(Handle &h, const HostBsr &Su, const HostBsr &Hu, const HostBsr &So,
                    const HostBsr &Ho, const tddft_system &sys);
int n_features(int bu, int bo);

// three affine layers, SiLU between them; FP32 master parameters, BF16 working weights
struct Mlp {
  int n_in = 0, width = 0, n_out = 0;
  hipStream_t s = nullptr;
  int64_t nparams = 0;
  int64_t off[6] = {};          // W1 b1 W2 b2 W3 b3 in the packed parameter vector
  DevBuf<float> p, g, m, v, mean, stdv;
  DevBuf<__hip_bfloat16> wb;    // BF16 copy of the packed parameters (weights used)
  int64_t t = 0;                // Adam steps taken
  DevBuf<float> act;            // activations of the last forward pass
  int64_t rows_cap = 0;
  DevBuf<float> part;           // row-chunk partial sums
  DevBuf<double> part64;
  std::string last_error;

  void init(int n_in, int width, int n_out, hipStream_t s);
  void randomize(uint64_t seed);
  void refresh_bf16();
  void set(const float *params, const float *mean, const float *stdv);
  void get(float *params, float *mean, float *stdv) const;
  void fit_normalisation(int64_t rows, const float *X);
  // Y [rows][n_out]; keeps Z1, A1, Z2, A2 for a following backward pass
  void forward(int64_t rows, const float *X, float *Y);
  double train_step(int64_t rows, const float *X, const float *gr, const float *gs,
                    const float *tg, double loss_scale, double lr, float *grad_out);
  std::vector<unsigned char> blob() const;
  void from_blob(const void *data, int64_t size, hipStream_t s);
};

// Z[blk][col][e] = c[blk][e] * X[blk][col][e]
template <class T>
void block_scale(int64_t nblk, int ncol, int E, const T *c, const T *X, T *Z, hipStream_t s);
// c[blk][e] = Y[blk][e] (e < E) and t[blk] = Y[blk][E] for network outputs Y [nblk][E + 1]
template <class T>
void split_outputs(int64_t nblk, int E, const float *Y, T *c, float *t, hipStream_t s);
// per R block: sum over states of the squared values of Pq (ABI layout)
void block_sqnorm(int64_t nblk, int n, int64_t nnz, const int64_t *voff, const int32_t *shape,
                  const double *Pq, double *w, hipStream_t s);
void guess_from_weights(int64_t nblk, const double *w, double inv_total, float *t, hipStream_t s);

}  // namespace tddft
