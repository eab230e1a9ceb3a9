// Argument blocks and launch entry points of the RSKA kernels (host + device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsk {

typedef unsigned long long u64;

// One dense persistent solve (eq. (rska) / Algorithm 1) over K steps.
template <typename T>
struct DenseArgs {
  const T* A;
  int64_t m, n, ld;
  const T* b;
  const T* r2;            // ||a_i||^2
  T lambda, alpha;
  const T* alpha_k;       // nullable, per-step relaxation
  int eta;
  int64_t K;
  const int32_t* idx;     // stream, already advanced by stream_offset
  T* x_star;              // in/out
  T* x;                   // out
  int warm;
  T* y;                   // nullable dual, y[tau_t] -= c_t
  const T* xref;          // nullable monitor target
  int64_t check_every;
  double tol;
  double* err_hist;
  int* status;            // [0] status, [1] steps done
  u64* xP;                // partial dots  [2][G][eta][words] (step parity)
  u64* xC;                // coefficients  [eta][words]
  u64* xM;                // monitor sums  [G][2][2]
  int G;
  int two_hop;            // 1: owners reduce rows, then everyone gathers; 0: everyone reduces everything
  int tile_cache;         // 1: keep the step's row tile in LDS between dot and scatter
  int64_t nchunks;        // ceil(n / VEC)
  int wq_max;             // max chunks per workgroup slice
  int lpr;                // lanes per row in the dot phase (power of two <= 64)
};

// One CSR persistent solve (single workgroup).
constexpr int kCsrMaxEta = 4096;  // rows per step of the CSR kernel
template <typename T>
struct CsrArgs {
  const int64_t* row_ptr;
  const int32_t* col;
  const T* val;
  int64_t m, n;
  const T* b;
  const T* r2;
  T lambda, alpha;
  const T* alpha_k;
  int eta;
  int64_t K;
  const int32_t* idx;
  T* x_star;
  T* x;
  int warm;
  T* y;
  const T* xref;
  int64_t check_every;
  double tol;
  double* err_hist;
  int* status;
  long long* acc;         // n + 1 int64 accumulators (the last a spare), zero on entry and on exit
};

template <typename T>
hipError_t launch_csr(CsrArgs<T>& a, hipStream_t stream);

// Multi-RHS (shared A and stream), float32 MFMA GEMMs per step.
struct MultiRhsArgs {
  const float* A;
  int64_t m, n, ld;
  const float* B;         // m x R row-major
  int R;
  const float* r2;
  float lambda, alpha;
  const float* alpha_k;   // nullable, device
  int eta;
  int64_t K;
  const int32_t* idx;
  float* x_star;          // n x R row-major, in/out
  float* x;               // n x R row-major, out
  int warm;
  int* status;
  float* Y;               // S x eta_pad x R split-K partials
  float* C;               // eta_pad x R coefficients
  int S, eta_pad;
  int64_t kspan;
};
hipError_t launch_multirhs(const MultiRhsArgs& a, hipStream_t stream);

struct DenseLaunch {
  int threads;
  size_t lds_bytes;
  int vec;
};

// Plans and launches; returns a hipError_t.
template <typename T>
hipError_t launch_dense(DenseArgs<T>& a, int vec, hipStream_t stream, int* max_grid_out);

template <typename T>
hipError_t launch_rownorm2_dense(const T* A, int64_t m, int64_t n, int64_t ld, T* r2, hipStream_t stream);

template <typename T>
hipError_t launch_rownorm2_csr(const int64_t* row_ptr, const T* val, int64_t m, T* r2, hipStream_t stream);

hipError_t launch_zero_words(u64* p, size_t nwords, hipStream_t stream);

// float32 register-tile kernel: NT threads, RP row passes of NT/4 rows, CPL float4 chunks per lane
int dense_rt_max_grid(int nt, int rp, int cpl);
hipError_t launch_dense_rt(DenseArgs<float>& a, int nt, int rp, int cpl, hipStream_t stream);
constexpr int kRtMaxEta = 1024, kRtMaxCPL = 5, kRtOwnMax = 4;
hipError_t launch_zero_status(int* status, hipStream_t stream);

// Largest co-resident grid for the dense kernel with these sizes (0 if none).
template <typename T>
int dense_max_grid(int vec, int eta, int wq_max, int tile_cache, size_t* lds_bytes);

}  // namespace rsk
