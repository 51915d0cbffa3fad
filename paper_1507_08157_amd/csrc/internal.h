// Internal declarations of libtddft: device buffers, host-side patterns and plans, the
// handle, and the launch wrappers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tddft.h"

namespace tddft {

// ---------------------------------------------------------------------------------------
// errors: thrown inside the library, converted to status codes at the C-ABI
struct Error {
  int code;
  std::string msg;
};

#define TD_HIP(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      throw ::tddft::Error{TDDFT_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define TD_REQUIRE(cond, msg)                                                           \
  do {                                                                                  \
    if (!(cond)) throw ::tddft::Error{TDDFT_E_INVALID, (msg)};                          \
  } while (0)

// ---------------------------------------------------------------------------------------
// device buffer (owning, move-only)
template <class T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{TDDFT_E_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed"};
    }
    n = count;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void upload(const T *src, size_t count, hipStream_t s) {
    if (count > n) alloc(count);
    if (count) TD_HIP(hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void upload(const std::vector<T> &v, hipStream_t s) { upload(v.data(), v.size(), s); }
};

// ---------------------------------------------------------------------------------------
// host-side block pattern (CSR over blocks, sorted columns)
struct Pattern {
  int nbr = 0, nbc = 0;
  std::vector<int64_t> rowptr;   // [nbr + 1]
  std::vector<int32_t> col;      // [nnzb]
  int64_t nnzb() const { return rowptr.empty() ? 0 : rowptr.back(); }
  int64_t find(int r, int c) const;  // block index or -1
  static Pattern dense(int nr, int nc);
};

// sparse matrix with blocks padded to br x bc (row-major), FP64 host values
struct HostBsr {
  Pattern pat;
  int br = 0, bc = 0;
  std::vector<double> val;       // [nnzb * br * bc]
};

// product plan: output pattern and, per output block, the (a, b) block pairs to sum
struct Plan {
  Pattern out;
  std::vector<int64_t> ptr;      // [nnzb_out + 1]
  std::vector<int32_t> pa, pb;   // block indices into the two operands
  // when A, B and the output are all complete block patterns: their block counts
  // (A: di x dk, B: dk x dj), else 0; the product is then a plain dense one
  int di = 0, dk = 0, dj = 0;
};

// C = mask_out(A * B), symbolic only: pairs (iA, iB) with A[i,k], B[k,j], (i,j) in out
Plan plan_product(const Pattern &A, const Pattern &B, const Pattern &out);
// exact host product of padded-block matrices onto a given output pattern
HostBsr host_product(const HostBsr &A, const HostBsr &B, const Pattern &out);
// pattern of the full product A * B
Pattern product_pattern(const Pattern &A, const Pattern &B);
// block transpose (pattern and values)
HostBsr host_transpose(const HostBsr &A);

struct DevPlan {
  int64_t nout = 0, npairs = 0;
  int di = 0, dk = 0, dj = 0;    // complete patterns (see Plan)
  int cw = 1;                    // columns per thread of the sparse form (1, 2 or 4; tuned)
  int pb = 4;                    // pairs per batch of the sparse form (1, 2, 4 or 8; tuned)
  int tile = 0;                  // output tile shape of the dense form (0, 1 or 2; tuned)
  DevBuf<int64_t> ptr;
  DevBuf<int2> pairs;
  void upload(const Plan &p, hipStream_t s);
};

// ---------------------------------------------------------------------------------------
// grid tiling
constexpr int TILE = 4;            // tile edge (points)
constexpr int TP = TILE * TILE * TILE;  // points per tile

struct TileSet {
  int ntx = 0, nty = 0, ntz = 0, nt = 0;
  // per tile: atom lists of the left (u) and right (o) sets
  std::vector<int32_t> uptr, optr;     // [nt + 1]
  std::vector<int32_t> uatom, oatom;   // atoms
  // per tile: pair table (u-list x o-list) -> block index in a pattern (or -1)
  std::vector<int64_t> pptr;           // [nt + 1]
};

// ---------------------------------------------------------------------------------------
// FFT plan for one axis: radices and twiddle table offsets
struct AxisFFT {
  int n = 0;
  std::vector<int> radix;          // passes in order
  std::vector<int> tw_off;         // offset of each pass's twiddles
  int tw_len = 0;
};

struct FFTPlan {
  AxisFFT ax[3];                   // x, y, z
  // threads per workgroup of each axis's passes: 256, 512 or 1024 in place (one LDS
  // buffer), 0 for the two-buffer form on 256 threads; set by build_fft_plan to the
  // smallest in-place count that fits, possibly changed by the tuner
  int nt[3] = {0, 0, 0};
  DevBuf<double> tw64;             // [sum tw_len] complex interleaved (re, im)
  DevBuf<float> tw32;
};

// ---------------------------------------------------------------------------------------
// optional per-stage device timing with events on the launching stream
enum Stage {
  ST_KSHIFT_LEFT = 0, ST_KSHIFT_RIGHT, ST_DENSITY, ST_FFT_X_FWD, ST_FFT_Y_FWD, ST_FFT_Z_POISSON,
  ST_FFT_Y_INV, ST_FFT_X_INV, ST_VINT, ST_VINT_REDUCE, ST_SANDWICH_LEFT, ST_SANDWICH_RIGHT,
  ST_PROJECT, ST_COVARIANT, ST_GRAM, ST_LINCOMB, ST_PROJECT_T, ST_GATHER, ST_COUNT
};
extern const char *const kStageNames[ST_COUNT];

struct Prof {
  bool on = false;
  hipEvent_t a[ST_COUNT] = {}, b[ST_COUNT] = {};
  bool pending[ST_COUNT] = {};
  double ms[ST_COUNT] = {};
  int64_t count[ST_COUNT] = {};
  void init();
  void destroy();
  void begin(int k, hipStream_t s);
  void end(int k, hipStream_t s);
  void collect();
  void reset();
};

// ---------------------------------------------------------------------------------------
struct Handle;

}  // namespace tddft
