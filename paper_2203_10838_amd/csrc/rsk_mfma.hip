// Multi-right-hand-side RSKA on the matrix cores (float32 MFMA, float32 accumulate).
//
// R systems A X = B share A and the index stream. In the sketch-and-project
// form of a step (eq. (rska1), start of Sec. 4) the R iterations together are
//     R_tau = A_tau X_k - B_tau                        (eta x R, a GEMM over n)
//     C     = (alpha_k/eta) D_tau^-2 R_tau             (row scaling)
//     X*   -= A_tau^T C                                (n x R, a GEMM over eta)
//     X     = S_lambda(X*)
// Column r of X is exactly the single-RHS iteration on b = B[:, r] with the
// same stream. Both GEMMs read the gathered rows A_tau straight from A (no
// copy of the tile is formed):
//   gemm_at_x   Y_s = A_tau[:, K_s] X[K_s, :]  for split s of the n columns
//   coef        C = (alpha_k/eta)(sum_s Y_s - B_tau) / ||a_tau||^2 (fixed split order)
//   gemm_att_c  W = A_tau^T C with the update of X*, X fused into the epilogue
// Tiles: 64 x 64 outputs per 256-thread workgroup, 4 waves of 32 x 32, each a
// 2 x 2 grid of v_mfma_f32_16x16x4f32 (A fragment: lane l holds row l%16,
// k = l/16; B fragment: column l%16, k = l/16; D: column l%16, rows
// 4*(l/16) + v). K advances 16 at a time through LDS tiles stored k-major.
#include "rsk_device.hpp"
#include "rsk_kernels.hpp"

namespace rsk {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, NTH = 256;

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Inner product of the workgroup's LDS tiles: As[k][m] (BK x BM), Bs[k][n] (BK x BN).
__device__ __forceinline__ void mma_tile(const float (*As)[BM], const float (*Bs)[BN], int wm, int wn, int lane,
                                         f4 (&acc)[2][2]) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < BK; k0 += 4) {
    float a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = As[k0 + lk][wm * 32 + i * 16 + li];
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = Bs[k0 + lk][wn * 32 + j * 16 + li];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
  }
}

}  // namespace

// Y[s][t][r] = sum_{j in split s} A[tau_t, j] X[j, r]. grid = (ceil(eta/64), R/64, S).
__global__ __launch_bounds__(NTH) void gemm_at_x(const float* __restrict__ A, int64_t ld, int64_t n,
                                                  const int32_t* __restrict__ tau, int eta, const float* __restrict__ X,
                                                  int R, float* __restrict__ Y, int eta_pad, int64_t kspan,
                                                  const int* status) {
  if (status[0]) return;
  __shared__ float As[BK][BM];
  __shared__ float Bs[BK][BN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int t0 = blockIdx.x * BM, r0 = blockIdx.y * BN, s = blockIdx.z;
  const int64_t j_begin = (int64_t)s * kspan;
  int64_t j_end = j_begin + kspan;
  if (j_end > n) j_end = n;

  // A tile loader: thread -> row t0 + tid/4, 4 consecutive columns
  const int at = tid >> 2, ac = (tid & 3) * 4;
  const int trow = t0 + at;
  const float* arow = A + (int64_t)(trow < eta ? tau[trow] : 0) * ld;
  // X tile loader: thread -> row k = tid/16, columns r0 + 4*(tid%16)
  const int xk = tid >> 4, xc = (tid & 15) * 4;

  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  for (int64_t j0 = j_begin; j0 < j_end; j0 += BK) {
    float4 av = make_float4(0.f, 0.f, 0.f, 0.f);
    if (trow < eta && j0 + ac < j_end) av = *reinterpret_cast<const float4*>(arow + j0 + ac);
    float4 xv = make_float4(0.f, 0.f, 0.f, 0.f);
    if (j0 + xk < j_end && r0 + xc < R) xv = *reinterpret_cast<const float4*>(X + (j0 + xk) * R + r0 + xc);
    __syncthreads();
    As[ac + 0][at] = av.x;
    As[ac + 1][at] = av.y;
    As[ac + 2][at] = av.z;
    As[ac + 3][at] = av.w;
    *reinterpret_cast<float4*>(&Bs[xk][xc]) = xv;
    __syncthreads();
    mma_tile(As, Bs, wm, wn, lane, acc);
  }
  // D layout: column lane%16, rows 4*(lane/16) + v
  float* Ys = Y + (size_t)s * eta_pad * R;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int t = t0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
        const int r = r0 + wn * 32 + j * 16 + (lane & 15);
        if (r < R) Ys[(size_t)t * R + r] = acc[i][j][v];
      }
}

// C[t][r] = (alpha_k/eta) (sum_s Y[s][t][r] - B[tau_t, r]) / ||a_tau_t||^2; checks the step's
// indices and coefficients, marks the step done. grid-stride over eta_pad x R.
__global__ void coef_kernel(const float* __restrict__ Y, int S, int eta_pad, const int32_t* __restrict__ tau, int eta,
                            const float* __restrict__ B, int R, const float* __restrict__ r2, float alpha,
                            const float* __restrict__ alpha_k, int64_t k, float* __restrict__ C, int* status) {
  if (status[0]) return;
  const float scale = (alpha_k ? alpha_k[k] : alpha) / (float)eta;
  const size_t total = (size_t)eta_pad * R;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int t = (int)(e / R), r = (int)(e % R);
    float c = 0.f;
    if (t < eta) {
      const int i = tau[t];
      float y = 0.f;
      for (int s = 0; s < S; ++s) y += Y[(size_t)s * total + e];
      const float rn = r2[i];
      if (rn == 0.f) set_status(status, ST_ZERO_ROW);
      c = scale * (y - B[(int64_t)i * R + r]) / rn;
      if (!isfinite(c)) set_status(status, ST_NONFINITE);
    }
    C[e] = c;
  }
}

// Step bookkeeping between steps: if the finished steps raised nothing, count
// them, then range-check the next step's indices before any kernel of that
// step reads A.
__global__ void step_check(const int32_t* __restrict__ tau, int eta, int64_t m, int* status, int64_t k_done) {
  if (status[0]) return;
  __syncthreads();
  if (threadIdx.x == 0) status[1] = (int)k_done;
  for (int t = threadIdx.x; t < eta; t += blockDim.x) {
    const int i = tau[t];
    if (i < 0 || (int64_t)i >= m) set_status(status, ST_INDEX);
  }
}

// W = A_tau^T C; epilogue X*[j][r] -= W, X[j][r] = S_lambda(X*). grid = (ceil(n/64), R/64).
__global__ __launch_bounds__(NTH) void gemm_att_c_update(const float* __restrict__ A, int64_t ld, int64_t n,
                                                         const int32_t* __restrict__ tau, int eta,
                                                         const float* __restrict__ C, int R, float* __restrict__ Xs,
                                                         float* __restrict__ X, float lambda, const int* status) {
  if (status[0]) return;
  __shared__ float As[BK][BM];
  __shared__ float Bs[BK][BN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t j0 = (int64_t)blockIdx.x * BM;
  const int r0 = blockIdx.y * BN;
  // A^T tile loader: thread -> sampled row t0 + tid/16, columns j0 + 4*(tid%16)
  const int lt = tid >> 4, lc = (tid & 15) * 4;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  for (int t0 = 0; t0 < eta; t0 += BK) {
    const int t = t0 + lt;
    float4 av = make_float4(0.f, 0.f, 0.f, 0.f);
    if (t < eta && j0 + lc < n) av = *reinterpret_cast<const float4*>(A + (int64_t)tau[t] * ld + j0 + lc);
    float4 cv = make_float4(0.f, 0.f, 0.f, 0.f);
    if (t < eta && r0 + lc < R) cv = *reinterpret_cast<const float4*>(C + (size_t)t * R + r0 + lc);
    __syncthreads();
    *reinterpret_cast<float4*>(&As[lt][lc]) = av;
    *reinterpret_cast<float4*>(&Bs[lt][lc]) = cv;
    __syncthreads();
    mma_tile(As, Bs, wm, wn, lane, acc);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t jj = j0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
        const int r = r0 + wn * 32 + j * 16 + (lane & 15);
        if (jj < n && r < R) {
          const size_t o = (size_t)jj * R + r;
          const float z = Xs[o] - acc[i][j][v];
          Xs[o] = z;
          X[o] = shrink(z, lambda);
        }
      }
}

__global__ void init_multirhs(float* Xs, float* X, size_t total, float lambda, int warm) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const float z = warm ? Xs[e] : 0.f;
    Xs[e] = z;
    X[e] = shrink(z, lambda);
  }
}

hipError_t launch_multirhs(const MultiRhsArgs& a, hipStream_t stream) {
  const size_t total = (size_t)a.n * a.R;
  hipLaunchKernelGGL(init_multirhs, dim3(1024), dim3(256), 0, stream, a.x_star, a.x, total, a.lambda, a.warm);
  if (a.K > 0)
    hipLaunchKernelGGL(step_check, dim3(1), dim3(1024), 0, stream, a.idx, a.eta, a.m, a.status, (int64_t)0);
  const int gt = (a.eta + BM - 1) / BM;
  const int gr = (a.R + BN - 1) / BN;
  const int gn = (int)((a.n + BM - 1) / BM);
  for (int64_t k = 0; k < a.K; ++k) {
    const int32_t* tk = a.idx + k * (int64_t)a.eta;
    hipLaunchKernelGGL(gemm_at_x, dim3(gt, gr, a.S), dim3(NTH), 0, stream, a.A, a.ld, a.n, tk, a.eta, a.x, a.R, a.Y,
                       a.eta_pad, a.kspan, a.status);
    hipLaunchKernelGGL(coef_kernel, dim3(512), dim3(256), 0, stream, a.Y, a.S, a.eta_pad, tk, a.eta, a.B, a.R, a.r2,
                       a.alpha, a.alpha_k, k, a.C, a.status);
    hipLaunchKernelGGL(gemm_att_c_update, dim3(gn, gr), dim3(NTH), 0, stream, a.A, a.ld, a.n, tk, a.eta, a.C, a.R,
                       a.x_star, a.x, a.lambda, a.status);
    const int32_t* tn = (k + 1 < a.K) ? tk + a.eta : tk;
    hipLaunchKernelGGL(step_check, dim3(1), dim3(1024), 0, stream, tn, (k + 1 < a.K) ? a.eta : 0, a.m, a.status,
                       k + 1);
  }
  return hipGetLastError();
}

}  // namespace rsk
