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

constexpr int BM = 64, BN = 64, NTH = 256;

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Pipelined main loop. K advances SK = 64 per stage through LDS tiles stored
// k-major, rows padded to BM + 16 floats: a fragment read (16 consecutive
// floats in each of 4 k rows) then hits 64 distinct banks. Every thread moves
// four float4 of each operand per stage, and the next stage's loads are issued
// before the current stage's MFMAs, so one memory latency overlaps one stage
// of compute. The A_tau X product keeps its A tile row-major (rows padded to
// SK + 4 floats, again 64 distinct banks per fragment read), so that tile is
// stored with float4 writes instead of a transpose.
constexpr int SK = 64, LDP = BM + 16, LDA = SK + 4;
constexpr int kMaxTauLds = 4096;  // sampled rows staged in LDS by the A^T GEMMs

struct Stage {
  float4 a[4], b[4];
};

// A stage loaded without branches: every load reads a valid address, and the positions that lie
// outside the product are zeroed only when the stage is stored to LDS (a select right after the
// load would wait for the load there and then, instead of under the current stage's products).
struct StageM {
  float4 a[4], b[4];
  bool ka[4], kb[4];
};

// v where keep holds, else zeros; element-wise selects (a select of the whole vector would go
// through private memory)
__device__ __forceinline__ float4 keep4(bool keep, float4 v) {
  return make_float4(keep ? v.x : 0.f, keep ? v.y : 0.f, keep ? v.z : 0.f, keep ? v.w : 0.f);
}

template <bool A_ROWS>
__device__ __forceinline__ void mma_stage_t(const float* As, const float (*Bs)[LDP], int wm, int wn, int lane,
                                            f4 (&acc)[2][2]) {
  const int li = lane & 15, lk = lane >> 4;
  // Every fragment of the stage is read before the first product, so the reads' latencies
  // overlap each other and the products instead of stalling each group of four products.
  float a[SK / 4][2], b[SK / 4][2];
#pragma unroll
  for (int s = 0; s < SK / 4; ++s) {
    const int k0 = 4 * s;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int m = wm * 32 + i * 16 + li;
      a[s][i] = A_ROWS ? As[m * LDA + k0 + lk] : As[(k0 + lk) * LDP + m];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) b[s][j] = Bs[k0 + lk][wn * 32 + j * 16 + li];
  }
  __builtin_amdgcn_sched_barrier(0);  // keeps the scheduler from interleaving the reads back in
#pragma unroll
  for (int s = 0; s < SK / 4; ++s)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = mfma16(a[s][i], b[s][j], acc[i][j]);
}

__device__ __forceinline__ void mma_stage(const float (*As)[LDP], const float (*Bs)[LDP], int wm, int wn, int lane,
                                          f4 (&acc)[2][2]) {
  mma_stage_t<false>(&As[0][0], Bs, wm, wn, lane, acc);
}

// acc = A_tau[:, k-range]^T-free product for the A^T GEMMs: acc(m = column j0 + m, n = r0 + n) =
// sum_t A[tau_t, j0 + m] C[t, r0 + n] over t < eta, tau staged in LDS.
__device__ __forceinline__ void att_mainloop(const float* __restrict__ A, int64_t ld, int64_t n,
                                             const int* taus, int eta, const float* __restrict__ C, int R,
                                             int64_t j0, int r0, float (*As)[LDP], float (*Bs)[LDP],
                                             f4 (&acc)[2][2]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = tid >> 4, lc = (tid & 15) * 4;
  const bool colok = j0 + lc < n, rok = r0 + lc < R;
  // Branch-free: every load reads a valid address (out-of-range positions read row taus[0],
  // column 0 or C row 0) and the value is replaced by zero afterwards, so the eight loads of a
  // stage issue back to back.
  const int64_t jc = colok ? j0 + lc : 0;
  const int rc = rok ? r0 + lc : 0;
  auto load = [&](int tb, StageM& st) {
    int rows[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int t = tb + lr + 16 * i;
      rows[i] = taus[t < eta ? t : 0];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int t = tb + lr + 16 * i;
      const bool ok = t < eta;
      st.a[i] = *reinterpret_cast<const float4*>(A + (int64_t)rows[i] * ld + jc);
      st.b[i] = *reinterpret_cast<const float4*>(C + (size_t)(ok ? t : 0) * R + rc);
      st.ka[i] = ok && colok;
      st.kb[i] = ok && rok;
    }
  };
  StageM st;
  if (eta > 0) load(0, st);
  for (int tb = 0; tb < eta; tb += SK) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      *reinterpret_cast<float4*>(&As[lr + 16 * i][lc]) = keep4(st.ka[i], st.a[i]);
      *reinterpret_cast<float4*>(&Bs[lr + 16 * i][lc]) = keep4(st.kb[i], st.b[i]);
    }
    __syncthreads();
    if (tb + SK < eta) load(tb + SK, st);
    mma_stage(As, Bs, wm, wn, lane, acc);
  }
}

// Workgroup-uniform read of the fault word (thread 0 reads, everyone agrees).
__device__ __forceinline__ bool any_fault(const int* status, int* flag) {
  if (threadIdx.x == 0) *flag = __hip_atomic_load(const_cast<int*>(status), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const bool f = *flag != 0;
  __syncthreads();
  return f;
}

__device__ __forceinline__ void stage_tau(const int32_t* __restrict__ tau, int eta, int* taus) {
  for (int t = threadIdx.x; t < eta; t += blockDim.x) taus[t] = tau[t];
}

}  // namespace

// Y[s][t][r] = sum_{j in split s} A[tau_t, j] X[j, r]. One-dimensional grid of gt * gr * S
// workgroups (gt = ceil(eta/64) row tiles, gr = ceil(R/64) column tiles, S splits of n). With S a
// multiple of 8 the gt * gr tiles of one split run on one XCD (workgroup i goes to XCD i % 8), so
// that XCD's L2 fetches A_tau[:, K_s] and X[K_s, :] once and serves their re-reads by the other
// tiles (A_tau by the gr column tiles, X by the gt row tiles).
//
// With m > 0 each workgroup also range-checks the sampled rows it reads (a bad index is read as row
// 0 and faults step k, so no later kernel of the step runs), and workgroup 0 records that the steps
// before k completed (status[1] only grows: a fault at step k records k as well).
__global__ __launch_bounds__(NTH) void gemm_at_x(const float* __restrict__ A, int64_t ld, int64_t n,
                                                  const int32_t* __restrict__ tau, int eta, const float* __restrict__ X,
                                                  int R, float* __restrict__ Y, int eta_pad, int64_t kspan,
                                                  int gt, int gr, int S, int* status, int64_t m, int64_t k) {
  __shared__ __align__(16) float Ar[BM][LDA];
  __shared__ __align__(16) float Bs[SK][LDP];
  // With the index check (m > 0) the fault word is read here and used only where it matters (the
  // index fault and the progress count): its round trip overlaps the index and first operand
  // loads, and after an earlier fault the partials are computed all the same and never used.
  // Without the check the rows may only be read when no fault is recorded.
  __shared__ int flag;
  if (m == 0 && any_fault(status, &flag)) return;
  const int st0 = status[0];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int id = blockIdx.x, T = gt * gr;
  int tile, s;
  if (S % 8 == 0) {
    const int q = id / 8;
    tile = q % T;
    s = id % 8 + 8 * (q / T);
  } else {
    tile = id % T;
    s = id / T;
  }
  const int t0 = (tile % gt) * BM, r0 = (tile / gt) * BN;
  const int64_t j_begin = (int64_t)s * kspan;
  int64_t j_end = j_begin + kspan;
  if (j_end > n) j_end = n;

  // thread -> rows t0 + lr + 16 i of A_tau (4 columns at lc), rows jb + lr + 16 i of X (4 columns at lc)
  const int lr = tid >> 4, lc = (tid & 15) * 4;
  const float* arow[4];
  bool aok[4];
  int bad = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int t = t0 + lr + 16 * i;
    aok[i] = t < eta;
    int row = aok[i] ? tau[t] : 0;
    if (m > 0 && (row < 0 || (int64_t)row >= m)) { bad = 1; row = 0; }
    arow[i] = A + (int64_t)row * ld;
  }
  if (bad && st0 == 0) {
    set_status(status, ST_INDEX);
    atomicMax(status + 1, (int)k);
  }
  // steps before k completed (status[1] only grows; a fault at step k records k as well)
  if (m > 0 && blockIdx.x == 0 && threadIdx.x == 0 && st0 == 0) atomicMax(status + 1, (int)k);
  const bool rok = r0 + lc < R;
  const int rc = rok ? r0 + lc : 0;
  // Branch-free: positions past the split's columns read column 0 (of the same row, or row 0
  // of X) and are replaced by zero, so the eight loads of a stage issue back to back.
  auto load = [&](int64_t jb, StageM& st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t c = jb + lc;
      const int64_t jj = jb + lr + 16 * i;
      st.a[i] = *reinterpret_cast<const float4*>(arow[i] + (c < j_end ? c : 0));
      st.b[i] = *reinterpret_cast<const float4*>(X + (jj < j_end ? jj : 0) * R + rc);
      st.ka[i] = aok[i] && c < j_end;
      st.kb[i] = jj < j_end && rok;
    }
  };

  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  StageM st;
  load(j_begin, st);
  for (int64_t jb = j_begin; jb < j_end; jb += SK) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = lr + 16 * i;
      *reinterpret_cast<float4*>(&Ar[m][lc]) = keep4(st.ka[i], st.a[i]);
      *reinterpret_cast<float4*>(&Bs[m][lc]) = keep4(st.kb[i], st.b[i]);
    }
    __syncthreads();
    if (jb + SK < j_end) load(jb + SK, st);
    mma_stage_t<true>(&Ar[0][0], Bs, wm, wn, lane, acc);
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

// sum_s Y[s * total + e] in ascending s; eight loads are issued before their adds, so the
// partials' latencies overlap instead of adding up (same sum, same order)
__device__ __forceinline__ float split_sum(const float* __restrict__ Y, int S, size_t total, size_t e) {
  float y = 0.f;
  int s = 0;
  for (; s + 8 <= S; s += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = Y[(size_t)(s + u) * total + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) y += v[u];
  }
  for (; s < S; ++s) y += Y[(size_t)s * total + e];
  return y;
}

// C[t][r] = (alpha_k/eta) (sum_s Y[s][t][r] - B[tau_t, r]) / ||a_tau_t||^2; checks the step's
// indices and coefficients, marks the step done. One thread per 4 consecutive r (R % 4 == 0), in
// one pass when the grid covers eta_pad x R / 4, else grid-stride; the S partials load as float4
// before the row index is needed, and sum in split order (as split_sum).
// With Rh non-null the residuals R_tau = sum_s Y_s - B_tau are stored as well (the adjoint's recompute).
__global__ void coef_kernel(const float* __restrict__ Y, int S, int eta_pad, const int32_t* __restrict__ tau, int eta,
                            const float* __restrict__ B, int R, const float* __restrict__ r2,
                            const float* __restrict__ row_w, float alpha, const float* __restrict__ alpha_k,
                            int64_t k, float* __restrict__ C, float* __restrict__ Rh, int* status) {
  const int st0 = status[0];  // read with the first loads, checked before the rows are used
  const float scale = (alpha_k ? alpha_k[k] : alpha) / (float)eta;
  const size_t total = (size_t)eta_pad * R;
  const int R4 = R / 4;
  for (size_t e4 = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e4 < total / 4;
       e4 += (size_t)gridDim.x * blockDim.x) {
    const int t = (int)(e4 / R4), r = (int)(e4 % R4) * 4;
    const size_t e = e4 * 4;
    float c[4] = {0.f, 0.f, 0.f, 0.f}, res[4] = {0.f, 0.f, 0.f, 0.f};
    if (t < eta) {
      const int i = tau[t];
      float y[4] = {0.f, 0.f, 0.f, 0.f};
      int s = 0;
      for (; s + 8 <= S; s += 8) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = *reinterpret_cast<const float4*>(Y + (size_t)(s + u) * total + e);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          y[0] += v[u].x;
          y[1] += v[u].y;
          y[2] += v[u].z;
          y[3] += v[u].w;
        }
      }
      for (; s < S; ++s) {
        const float4 v = *reinterpret_cast<const float4*>(Y + (size_t)s * total + e);
        y[0] += v.x;
        y[1] += v.y;
        y[2] += v.z;
        y[3] += v.w;
      }
      if (st0) return;  // an earlier fault: the step's rows may be out of range
      const float rn = weighted_rn(r2, row_w, i);
      if (rn == 0.f) set_status(status, ST_ZERO_ROW);
      const float* Bi = B + (int64_t)i * R + r;  // B need not be 16-byte aligned
      bool bad = false;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        res[u] = y[u] - Bi[u];
        c[u] = scale * res[u] / rn;
        bad |= !isfinite(c[u]);
      }
      if (bad) set_status(status, ST_NONFINITE);
    }
    if (Rh) {
#pragma unroll
      for (int u = 0; u < 4; ++u) Rh[e + u] = res[u];
    }
    *reinterpret_cast<float4*>(C + e) = make_float4(c[0], c[1], c[2], c[3]);
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

// W = A_tau^T C; epilogue Zout[j][r] = Zin[j][r] - W, X[j][r] = S_lambda(Zout) (Zin may equal Zout:
// every element is read and written by one thread). grid = (ceil(n/64), R/64).
__global__ __launch_bounds__(NTH) void gemm_att_c_update(const float* __restrict__ A, int64_t ld, int64_t n,
                                                         const int32_t* __restrict__ tau, int eta,
                                                         const float* __restrict__ C, int R, const float* Zin,
                                                         float* Zout, float* __restrict__ X, float lambda,
                                                         const int* status) {
  // the fault word travels with the step's indices: the rows are read only when no fault is
  // recorded (an index fault of this step leaves out-of-range indices in tau)
  const int st0 = status[0];
  __shared__ __align__(16) float As[SK][LDP];
  __shared__ __align__(16) float Bs[SK][LDP];
  __shared__ int taus[kMaxTauLds];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t j0 = (int64_t)blockIdx.x * BM;
  const int r0 = blockIdx.y * BN;
  stage_tau(tau, eta, taus);
  __syncthreads();
  if (st0) return;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  att_mainloop(A, ld, n, taus, eta, C, R, j0, r0, As, Bs, acc);
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
          const float z = Zin[o] - acc[i][j][v];
          Zout[o] = z;
          X[o] = shrink(z, lambda);
        }
      }
}

// Row-split A_tau^T C for outputs too small to fill the chip: split s (blockIdx.z) takes the
// sampled rows [s eta / S2, (s + 1) eta / S2) and writes its raw 64 x 64 tile to Wp[s].
// grid = (ceil(n/64), R/64, S2).
__global__ __launch_bounds__(NTH) void gemm_att_partial(const float* __restrict__ A, int64_t ld, int64_t n,
                                                        const int32_t* __restrict__ tau, int eta,
                                                        const float* __restrict__ C, int R, float* __restrict__ Wp,
                                                        const int* status) {
  const int st0 = status[0];  // checked once the indices are staged, as in gemm_att_c_update
  __shared__ __align__(16) float As[SK][LDP];
  __shared__ __align__(16) float Bs[SK][LDP];
  __shared__ int taus[kMaxTauLds];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t j0 = (int64_t)blockIdx.x * BM;
  const int r0 = blockIdx.y * BN;
  const int s = blockIdx.z, S2 = gridDim.z;
  const int t0 = (int)((int64_t)s * eta / S2), t1 = (int)((int64_t)(s + 1) * eta / S2);
  stage_tau(tau + t0, t1 - t0, taus);
  __syncthreads();
  if (st0) return;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  att_mainloop(A, ld, n, taus, t1 - t0, C + (size_t)t0 * R, R, j0, r0, As, Bs, acc);
  float* W = Wp + (size_t)s * n * R;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t jj = j0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
        const int r = r0 + wn * 32 + j * 16 + (lane & 15);
        if (jj < n && r < R) W[(size_t)jj * R + r] = acc[i][j][v];
      }
}

// Epilogue of the row-split update: Zout = Zin - sum_s Wp[s] (s ascending), X = S_lambda(Zout),
// four elements a thread (R % 4 == 0), all S2 partial loads issued before the sum.
template <int S2>
__global__ __launch_bounds__(NTH) void att_reduce_update(const float* __restrict__ Wp, int64_t nr4,
                                                         const float* Zin, float* Zout, float* __restrict__ X,
                                                         float lambda, const int* status) {
  const int st0 = status[0];  // checked before the first write: the loads overlap its round trip
  const float4* W4 = reinterpret_cast<const float4*>(Wp);
  for (int64_t e = blockIdx.x * (int64_t)NTH + threadIdx.x; e < nr4; e += (int64_t)gridDim.x * NTH) {
    float4 w[S2];
#pragma unroll
    for (int q = 0; q < S2; ++q) w[q] = W4[q * nr4 + e];
    float4 z = reinterpret_cast<const float4*>(Zin)[e];
    if (st0) return;
    float4 t = w[0];
#pragma unroll
    for (int q = 1; q < S2; ++q) {
      t.x += w[q].x;
      t.y += w[q].y;
      t.z += w[q].z;
      t.w += w[q].w;
    }
    z.x -= t.x;
    z.y -= t.y;
    z.z -= t.z;
    z.w -= t.w;
    reinterpret_cast<float4*>(Zout)[e] = z;
    reinterpret_cast<float4*>(X)[e] =
        make_float4(shrink(z.x, lambda), shrink(z.y, lambda), shrink(z.z, lambda), shrink(z.w, lambda));
  }
}

__global__ void init_multirhs(float* Xs, float* X, size_t total, float lambda, int warm) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const float z = warm ? Xs[e] : 0.f;
    Xs[e] = z;
    X[e] = shrink(z, lambda);
  }
}

// ---------------------------------------------------------------------------
// Wide-tile products (the plan's tile = 128): TM x TN outputs per 256-thread workgroup
// (TM = 128; TN = 128, or 64 for R <= 64), four waves of (TM/2) x (TN/2), each a grid of
// (TM/32) x (TN/32) v_mfma_f32_16x16x4f32 blocks. K advances 32 per stage. A tile of twice the
// width reads half the bytes per product of the 64 x 64 tiles: those are bound by the rate at
// which a CU pulls its operands through L2 (the same step time whether the sampled rows spread
// over the whole matrix or fit in L2), not by HBM or by the matrix cores.
// Loads are branch-free (every address valid; positions outside the product are zeroed when
// the stage is stored to LDS), and each stage's loads are issued before the previous stage's
// products.
// ---------------------------------------------------------------------------
namespace {

constexpr int SKW = 32;  // K per stage of the wide-tile products
// The wide-tile products run 512 threads: 8 waves in a 4 x 2 grid over the tile, two a SIMD, so
// that one wave's MFMAs cover the other's LDS reads and barriers (with one wave a SIMD they are
// exposed: these grids put about one workgroup on each CU).
constexpr int NTW = 512, WGM = 4, WGN = 2;

template <int TN>
struct WideMap {  // a row of TN floats: TN/4 float4 across consecutive threads
  static constexpr int cpr = TN / 4;           // float4 per row
  static constexpr int rpp = NTW / cpr;        // rows per pass
  static constexpr int passes = SKW / rpp;     // passes over the SKW rows of a stage
};

template <int TM, int TN>
__device__ __forceinline__ void mma_stage_w(const float* As, int a_rows, const float* Bs, int wm, int wn,
                                            int lane, f4 (&acc)[TM / (16 * WGM)][TN / (16 * WGN)]) {
  // a_rows: As is row-major [TM][SKW + 4] (true) or k-major [SKW][TM + 16] (false)
  constexpr int BI = TM / (16 * WGM), BJ = TN / (16 * WGN), PB = TN + 16, PA = TM + 16, LDR = SKW + 4;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < SKW; k0 += 4) {
    float a[BI], b[BJ];
#pragma unroll
    for (int i = 0; i < BI; ++i) {
      const int m = wm * (TM / WGM) + i * 16 + li;
      a[i] = a_rows ? As[m * LDR + k0 + lk] : As[(k0 + lk) * PA + m];
    }
#pragma unroll
    for (int j = 0; j < BJ; ++j) b[j] = Bs[(k0 + lk) * PB + wn * (TN / WGN) + j * 16 + li];
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < BJ; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
  }
}

// acc = A_tau^T C over the sampled rows t < eta (taus in LDS) for output columns j0.. (TM) and
// right-hand sides r0.. (TN): the A operand is k-major in memory (row tau_t, columns j), as is C.
template <int TM, int TN>
__device__ __forceinline__ void att_mainloop_w(const float* __restrict__ A, int64_t ld, int64_t n,
                                               const int* taus, int eta, const float* __restrict__ C, int R,
                                               int64_t j0, int r0, float* As, float* Bs,
                                               f4 (&acc)[TM / (16 * WGM)][TN / (16 * WGN)]) {
  using MA = WideMap<TM>;
  using MB = WideMap<TN>;
  constexpr int PA = TM + 16, PB = TN + 16;
  static_assert(MA::passes >= 1 && MB::passes >= 1 && MA::passes * MA::rpp == SKW && MB::passes * MB::rpp == SKW,
                "a stage's rows split into whole passes");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int ar = tid / MA::cpr, ac = (tid % MA::cpr) * 4;
  const int br = tid / MB::cpr, bc = (tid % MB::cpr) * 4;
  const bool colok = j0 + ac < n, rok = r0 + bc < R;
  const int64_t jc = colok ? j0 + ac : 0;
  const int rc = rok ? r0 + bc : 0;
  struct Buf {
    float4 a[MA::passes], b[MB::passes];
    bool ka[MA::passes], kb[MB::passes];
  };
  auto load = [&](int tb, Buf& st) {
    int rows[MA::passes];
#pragma unroll
    for (int i = 0; i < MA::passes; ++i) {
      const int t = tb + ar + MA::rpp * i;
      rows[i] = taus[t < eta ? t : 0];
    }
#pragma unroll
    for (int i = 0; i < MA::passes; ++i) {
      const int t = tb + ar + MA::rpp * i;
      st.a[i] = *reinterpret_cast<const float4*>(A + (int64_t)rows[i] * ld + jc);
      st.ka[i] = t < eta && colok;
    }
#pragma unroll
    for (int i = 0; i < MB::passes; ++i) {
      const int t = tb + br + MB::rpp * i;
      st.b[i] = *reinterpret_cast<const float4*>(C + (size_t)(t < eta ? t : 0) * R + rc);
      st.kb[i] = t < eta && rok;
    }
  };
  constexpr int ASZ = SKW * PA, BSZ = SKW * PB;  // floats of one LDS buffer of each operand
  auto put = [&](const Buf& st, int buf) {
    // nothing moves across: a select hoisted above this point would wait for the other buffer
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < MA::passes; ++i)
      *reinterpret_cast<float4*>(&As[buf * ASZ + (ar + MA::rpp * i) * PA + ac]) = keep4(st.ka[i], st.a[i]);
#pragma unroll
    for (int i = 0; i < MB::passes; ++i)
      *reinterpret_cast<float4*>(&Bs[buf * BSZ + (br + MB::rpp * i) * PB + bc]) = keep4(st.kb[i], st.b[i]);
  };
  // Two register buffers and two LDS buffers: stage s + 1 is stored to LDS while stage s's
  // products run from the other buffer (one barrier a stage), and the loads of the stage after
  // that are in flight meanwhile (the workgroup is alone on its CU, so no other workgroup covers
  // its load latency). Stage j's loads go to register buffer j % 2, unconditionally (rows past
  // the end are clamped and stored as zeros), so each store waits only for its own buffer.
  const int nst = (eta + SKW - 1) / SKW;
  if (nst == 0) return;
  Buf b0, b1;
  load(0, b0);
  load(SKW, b1);
  put(b0, 0);
  load(2 * SKW, b0);
  __syncthreads();
  for (int q = 0; 2 * q < nst; ++q) {
    mma_stage_w<TM, TN>(As, 0, Bs, wm, wn, lane, acc);  // stage 2q
    if (2 * q + 1 >= nst) break;
    put(b1, 1);                                         // stage 2q + 1
    load((2 * q + 3) * SKW, b1);
    __syncthreads();
    mma_stage_w<TM, TN>(As + ASZ, 0, Bs + BSZ, wm, wn, lane, acc);
    if (2 * q + 2 < nst) {
      put(b0, 0);  // stage 2q + 2
      load((2 * q + 4) * SKW, b0);
    }
    __syncthreads();
  }
}

template <int TM, int TN>
__device__ __forceinline__ void zero_acc(f4 (&acc)[TM / (16 * WGM)][TN / (16 * WGN)]) {
#pragma unroll
  for (int i = 0; i < TM / (16 * WGM); ++i)
#pragma unroll
    for (int j = 0; j < TN / (16 * WGN); ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
}

}  // namespace

// Y[s][t][r] = sum_{j in split s} A[tau_t, j] X[j, r], TM x TN tiles (eta_pad a multiple of TM).
// Grid, XCD order, index check and status as gemm_at_x.
template <int TM, int TN>
__global__ __launch_bounds__(NTW) void gemm_at_x_w(const float* __restrict__ A, int64_t ld, int64_t n,
                                                   const int32_t* __restrict__ tau, int eta,
                                                   const float* __restrict__ X, int R, float* __restrict__ Y,
                                                   int eta_pad, int64_t kspan, int gt, int gr, int S, int* status,
                                                   int64_t m, int64_t k) {
  constexpr int LDR = SKW + 4, PB = TN + 16;
  using MA = WideMap<SKW>;  // a row piece of SKW floats: 8 float4
  using MB = WideMap<TN>;
  __shared__ __align__(16) float Ar[2 * TM * LDR];
  __shared__ __align__(16) float Bs[2 * SKW * PB];
  __shared__ int flag;
  if (m == 0 && any_fault(status, &flag)) return;
  const int st0 = status[0];  // used late, as in gemm_at_x
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int id = blockIdx.x, T = gt * gr;
  int tile, s;
  if (S % 8 == 0) {
    const int q = id / 8;
    tile = q % T;
    s = id % 8 + 8 * (q / T);
  } else {
    tile = id % T;
    s = id / T;
  }
  const int t0 = (tile % gt) * TM, r0 = (tile / gt) * TN;
  const int64_t j_begin = (int64_t)s * kspan;
  int64_t j_end = j_begin + kspan;
  if (j_end > n) j_end = n;

  // A: thread -> row t0 + ar + MA::rpp * i (TM / MA::rpp rows), 4 columns at ac of the stage
  constexpr int AP = TM / MA::rpp;
  static_assert(AP * MA::rpp == TM && MB::passes >= 1 && MB::passes * MB::rpp == SKW, "whole passes");
  const int ar = tid / MA::cpr, ac = (tid % MA::cpr) * 4;
  const float* arow[AP];
  int bad = 0;
#pragma unroll
  for (int i = 0; i < AP; ++i) {
    const int t = t0 + ar + MA::rpp * i;
    int row = t < eta ? tau[t] : 0;
    if (m > 0 && (row < 0 || (int64_t)row >= m)) { bad = 1; row = 0; }
    arow[i] = A + (int64_t)row * ld;
  }
  if (bad && st0 == 0) {
    set_status(status, ST_INDEX);
    atomicMax(status + 1, (int)k);
  }
  // steps before k completed (status[1] only grows; a fault at step k records k as well)
  if (m > 0 && blockIdx.x == 0 && threadIdx.x == 0 && st0 == 0) atomicMax(status + 1, (int)k);
  // X: thread -> rows br + MB::rpp * i of the stage, 4 columns at bc
  const int br = tid / MB::cpr, bc = (tid % MB::cpr) * 4;
  const bool rok = r0 + bc < R;
  const int rc = rok ? r0 + bc : 0;
  struct Buf {
    float4 a[AP], b[MB::passes];
    bool ka[AP], kb[MB::passes];
  };
  auto load = [&](int64_t jb, Buf& st) {
    const int64_t c = jb + ac;
#pragma unroll
    for (int i = 0; i < AP; ++i) {
      st.a[i] = *reinterpret_cast<const float4*>(arow[i] + (c < j_end ? c : 0));
      st.ka[i] = c < j_end;
    }
#pragma unroll
    for (int i = 0; i < MB::passes; ++i) {
      const int64_t jj = jb + br + MB::rpp * i;
      st.b[i] = *reinterpret_cast<const float4*>(X + (jj < j_end ? jj : 0) * R + rc);
      st.kb[i] = jj < j_end && rok;
    }
  };
  constexpr int ASZ = TM * LDR, BSZ = SKW * PB;  // floats of one LDS buffer of each operand
  auto put = [&](const Buf& st, int buf) {
    // nothing moves across: a select hoisted above this point would wait for the other buffer
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < AP; ++i)
      *reinterpret_cast<float4*>(&Ar[buf * ASZ + (ar + MA::rpp * i) * LDR + ac]) = keep4(st.ka[i], st.a[i]);
#pragma unroll
    for (int i = 0; i < MB::passes; ++i)
      *reinterpret_cast<float4*>(&Bs[buf * BSZ + (br + MB::rpp * i) * PB + bc]) = keep4(st.kb[i], st.b[i]);
  };
  f4 acc[TM / (16 * WGM)][TN / (16 * WGN)];
  zero_acc<TM, TN>(acc);
  // two register buffers and two LDS buffers, one barrier a stage (as att_mainloop_w)
  const int nst = j_end > j_begin ? (int)((j_end - j_begin + SKW - 1) / SKW) : 0;
  if (nst > 0) {
    Buf b0, b1;
    load(j_begin, b0);
    load(j_begin + SKW, b1);
    put(b0, 0);
    load(j_begin + 2 * SKW, b0);
    __syncthreads();
    for (int q = 0; 2 * q < nst; ++q) {
      mma_stage_w<TM, TN>(Ar, 1, Bs, wm, wn, lane, acc);  // stage 2q
      if (2 * q + 1 >= nst) break;
      put(b1, 1);                                         // stage 2q + 1
      load(j_begin + (int64_t)(2 * q + 3) * SKW, b1);
      __syncthreads();
      mma_stage_w<TM, TN>(Ar + ASZ, 1, Bs + BSZ, wm, wn, lane, acc);
      if (2 * q + 2 < nst) {
        put(b0, 0);  // stage 2q + 2
        load(j_begin + (int64_t)(2 * q + 4) * SKW, b0);
      }
      __syncthreads();
    }
  }
  // D layout: column lane%16, rows 4*(lane/16) + v
  float* Ys = Y + (size_t)s * eta_pad * R;
#pragma unroll
  for (int i = 0; i < TM / (16 * WGM); ++i)
#pragma unroll
    for (int j = 0; j < TN / (16 * WGN); ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int t = t0 + wm * (TM / WGM) + i * 16 + 4 * (lane >> 4) + v;
        const int r = r0 + wn * (TN / WGN) + j * 16 + (lane & 15);
        if (r < R) Ys[(size_t)t * R + r] = acc[i][j][v];
      }
}

// W = A_tau^T C over the sampled rows [s2 eta / S2, (s2 + 1) eta / S2) (s2 = blockIdx.z).
// UPDATE (S2 = 1): Zout = Zin - W, X = S_lambda(Zout); else W goes to Wp[s2] (summed by
// att_reduce_update / att_reduce_adj). grid = (ceil(n/TM), ceil(R/TN), S2).
template <int TM, int TN, bool UPDATE>
__global__ __launch_bounds__(NTW) void gemm_att_w(const float* __restrict__ A, int64_t ld, int64_t n,
                                                  const int32_t* __restrict__ tau, int eta,
                                                  const float* __restrict__ C, int R, const float* Zin, float* Zout,
                                                  float* __restrict__ X, float lambda, float* __restrict__ Wp,
                                                  const int* status) {
  const int st0 = status[0];  // checked once the indices are staged, as in gemm_att_c_update
  __shared__ __align__(16) float As[2 * SKW * (TM + 16)];
  __shared__ __align__(16) float Bs[2 * SKW * (TN + 16)];
  __shared__ int taus[kMaxTauLds];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t j0 = (int64_t)blockIdx.x * TM;
  const int r0 = blockIdx.y * TN;
  const int s2 = blockIdx.z, S2 = gridDim.z;
  const int tb0 = (int)((int64_t)s2 * eta / S2), tb1 = (int)((int64_t)(s2 + 1) * eta / S2);
  stage_tau(tau + tb0, tb1 - tb0, taus);
  __syncthreads();
  if (st0) return;
  constexpr int BI = TM / (16 * WGM), BJ = TN / (16 * WGN);
  // the update's x* inputs load before the products (in flight under them), not after
  float zin[UPDATE ? BI : 1][UPDATE ? BJ : 1][4];
  if constexpr (UPDATE) {
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < BJ; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t jj = j0 + wm * (TM / WGM) + i * 16 + 4 * (lane >> 4) + v;
          const int r = r0 + wn * (TN / WGN) + j * 16 + (lane & 15);
          zin[i][j][v] = Zin[jj < n && r < R ? (size_t)jj * R + r : 0];
        }
  }
  f4 acc[BI][BJ];
  zero_acc<TM, TN>(acc);
  att_mainloop_w<TM, TN>(A, ld, n, taus, tb1 - tb0, C + (size_t)tb0 * R, R, j0, r0, As, Bs, acc);
  float* W = UPDATE ? nullptr : Wp + (size_t)s2 * n * R;
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t jj = j0 + wm * (TM / WGM) + i * 16 + 4 * (lane >> 4) + v;
        const int r = r0 + wn * (TN / WGN) + j * 16 + (lane & 15);
        if (jj < n && r < R) {
          const size_t o = (size_t)jj * R + r;
          if constexpr (UPDATE) {
            const float z = zin[i][j][v] - acc[i][j][v];
            Zout[o] = z;
            X[o] = shrink(z, lambda);
          } else {
            W[o] = acc[i][j][v];
          }
        }
      }
}

namespace {

constexpr int kCq = 4;  // C items per 64 x 64 tile (16 rows each)

__device__ __forceinline__ float4 ld_dev4(const float* p) {
  const u64 lo = __hip_atomic_load(reinterpret_cast<const u64*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const u64 hi = __hip_atomic_load(reinterpret_cast<const u64*>(p) + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_float4(__uint_as_float((unsigned)lo), __uint_as_float((unsigned)(lo >> 32)),
                     __uint_as_float((unsigned)hi), __uint_as_float((unsigned)(hi >> 32)));
}
__device__ __forceinline__ void st_dev4(float* p, float4 v) {
  __hip_atomic_store(reinterpret_cast<u64*>(p), (u64)__float_as_uint(v.x) | ((u64)__float_as_uint(v.y) << 32),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(reinterpret_cast<u64*>(p) + 1, (u64)__float_as_uint(v.z) | ((u64)__float_as_uint(v.w) << 32),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev1(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The workgroup's stores are complete, then one thread counts the item done.
__device__ __forceinline__ void publish(unsigned* cnt) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 waits until *cnt >= target (bounded), the workgroup learns the outcome: false when a
// fault is recorded or the wait expired (then the fault is ST_ABORTED).
__device__ __forceinline__ bool await(const unsigned* cnt, unsigned target, int* status, int* flag) {
  if (threadIdx.x == 0) {
    int ok = 1;
    unsigned spins = 0;
    for (;;) {
      if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
      if (__hip_atomic_load(const_cast<unsigned*>(cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (++spins > kSpinLimit) { set_status(status, ST_ABORTED); ok = 0; break; }
      __builtin_amdgcn_s_sleep(1);
    }
    *flag = ok;
  }
  __syncthreads();
  const bool ok = *flag != 0;
  __syncthreads();
  return ok;
}

// Whether a fault is recorded, decided once for the whole workgroup (thread 0 reads, all agree).
__device__ __forceinline__ bool faulted(int* status, int* flag) {
  if (threadIdx.x == 0) *flag = __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const bool f = *flag != 0;
  __syncthreads();
  return f;
}

__device__ __forceinline__ void fault(int* status, int code, int64_t k) {
  set_status(status, code);
  atomicMin(status + 1, (int)k);
}

}  // namespace

// status[1] = K after the last step if nothing faulted.
__global__ void steps_done(int* status, int64_t K) {
  if (threadIdx.x == 0 && status[0] == 0) status[1] = (int)K;
}

// A_tau X (split-K partials into Y) for step k with the plan's tile; m > 0: with the index check.
static void launch_at_x(const MultiRhsArgs& a, const int32_t* tk, const float* X, int64_t m, int64_t k,
                        hipStream_t stream) {
  if (a.tile == 128) {
    const int gt = a.eta_pad / 128;
    if (a.R > 64) {
      const int gr = (a.R + 127) / 128;
      hipLaunchKernelGGL((gemm_at_x_w<128, 128>), dim3(gt * gr * a.S), dim3(NTW), 0, stream, a.A, a.ld, a.n, tk,
                         a.eta, X, a.R, a.Y, a.eta_pad, a.kspan, gt, gr, a.S, a.status, m, k);
    } else {
      hipLaunchKernelGGL((gemm_at_x_w<128, 64>), dim3(gt * a.S), dim3(NTW), 0, stream, a.A, a.ld, a.n, tk, a.eta,
                         X, a.R, a.Y, a.eta_pad, a.kspan, gt, 1, a.S, a.status, m, k);
    }
    return;
  }
  const int gt = (a.eta + BM - 1) / BM;
  const int gr = (a.R + BN - 1) / BN;
  hipLaunchKernelGGL(gemm_at_x, dim3(gt * gr * a.S), dim3(NTH), 0, stream, a.A, a.ld, a.n, tk, a.eta, X, a.R, a.Y,
                     a.eta_pad, a.kspan, gt, gr, a.S, a.status, m, k);
}

// W = A_tau^T C with the plan's tile: the S2 = 1 update (Zout = Zin - W, X = S_lambda) when
// update is set, else the S2 row-split partials into Wp.
static void launch_att(const MultiRhsArgs& a, const int32_t* tk, const float* C, const float* zin, float* zout,
                       bool update, hipStream_t stream) {
  const unsigned gn = (unsigned)((a.n + 127) / 128), z = update ? 1u : (unsigned)a.S2;
  if (a.R > 64 && !update) {
    const dim3 g(gn, (unsigned)((a.R + 127) / 128), z);
    hipLaunchKernelGGL((gemm_att_w<128, 128, false>), g, dim3(NTW), 0, stream, a.A, a.ld, a.n, tk, a.eta, C, a.R,
                       zin, zout, a.x, a.lambda, a.Wp, a.status);
    return;
  }
  // The fused update (no row split) takes 128 x 64 tiles at every R: twice the workgroups of
  // 128 x 128 tiles, and no partials to reduce.
  const dim3 g(gn, (unsigned)((a.R + 63) / 64), z);
  if (update)
    hipLaunchKernelGGL((gemm_att_w<128, 64, true>), g, dim3(NTW), 0, stream, a.A, a.ld, a.n, tk, a.eta, C, a.R, zin,
                       zout, a.x, a.lambda, a.Wp, a.status);
  else
    hipLaunchKernelGGL((gemm_att_w<128, 64, false>), g, dim3(NTW), 0, stream, a.A, a.ld, a.n, tk, a.eta, C, a.R, zin,
                       zout, a.x, a.lambda, a.Wp, a.status);
}

// One forward step k: R_tau from x (with the step's index check), C, Zout = Zin - A_tau^T C,
// x = S_lambda(Zout).
static void multirhs_step(const MultiRhsArgs& a, int64_t k, const float* zin, float* zout, float* rh,
                          hipStream_t stream) {
  const int gr = (a.R + BN - 1) / BN;
  const int gn = (int)((a.n + BM - 1) / BM);
  const int32_t* tk = a.idx + k * (int64_t)a.eta;
  launch_at_x(a, tk, a.x, a.m, k, stream);
  hipLaunchKernelGGL(coef_kernel, dim3(512), dim3(256), 0, stream, a.Y, a.S, a.eta_pad, tk, a.eta, a.B, a.R, a.r2,
                     a.row_w, a.alpha, a.alpha_k, k, a.C, rh, a.status);
  if (a.S2 > 1) {
    if (a.tile == 128)
      launch_att(a, tk, a.C, zin, zout, false, stream);
    else
      hipLaunchKernelGGL(gemm_att_partial, dim3(gn, gr, a.S2), dim3(NTH), 0, stream, a.A, a.ld, a.n, tk, a.eta, a.C,
                         a.R, a.Wp, a.status);
    const int64_t nr4 = a.n * a.R / 4;
    const dim3 rg((unsigned)((nr4 + NTH - 1) / NTH < 1024 ? (nr4 + NTH - 1) / NTH : 1024));
    if (a.S2 == 2)
      hipLaunchKernelGGL(att_reduce_update<2>, rg, dim3(NTH), 0, stream, a.Wp, nr4, zin, zout, a.x, a.lambda, a.status);
    else if (a.S2 == 4)
      hipLaunchKernelGGL(att_reduce_update<4>, rg, dim3(NTH), 0, stream, a.Wp, nr4, zin, zout, a.x, a.lambda, a.status);
    else
      hipLaunchKernelGGL(att_reduce_update<8>, rg, dim3(NTH), 0, stream, a.Wp, nr4, zin, zout, a.x, a.lambda, a.status);
  } else if (a.tile == 128) {
    launch_att(a, tk, a.C, zin, zout, true, stream);
  } else {
    hipLaunchKernelGGL(gemm_att_c_update, dim3(gn, gr), dim3(NTH), 0, stream, a.A, a.ld, a.n, tk, a.eta, a.C, a.R,
                       zin, zout, a.x, a.lambda, a.status);
  }
}

hipError_t launch_multirhs(const MultiRhsArgs& a, hipStream_t stream, float* ckpt, int64_t ckpt_every) {
  const size_t total = (size_t)a.n * a.R;
  hipLaunchKernelGGL(init_multirhs, dim3(1024), dim3(256), 0, stream, a.x_star, a.x, total, a.lambda, a.warm);
  for (int64_t k = 0; k < a.K; ++k) {
    if (ckpt && k % ckpt_every == 0) {
      hipError_t e = hipMemcpyAsync(ckpt + (size_t)(k / ckpt_every) * total, a.x_star, total * sizeof(float),
                                    hipMemcpyDeviceToDevice, stream);
      if (e != hipSuccess) return e;
    }
    multirhs_step(a, k, a.x_star, a.x_star, nullptr, stream);
  }
  hipLaunchKernelGGL(steps_done, dim3(1), dim3(64), 0, stream, a.status, a.K);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Persistent multi-RHS forward: all K steps in one cooperative launch.
//
// A step is four phases of work items, the same products as the step kernels above:
//   Y items (row tile t, column tile r, split s):   Y_s[t, r] = A_tau[t, K_s] X[K_s, r]
//   C items (row tile t, column tile r, 16 rows q): C[t, r] = (alpha_k/eta)(sum_s Y_s[t, r] - B_tau) / ||a||^2
//   U items (n tile j, column tile r, row split s2): A_tau^T C over the split's rows; with one
//           split it updates X*[j, r] and X[j, r] = S_lambda(X*) in its epilogue, else it writes
//           its partial and a V item (j, r) adds the S2 partials in order and updates.
// Items depend on earlier items only through cumulative per-tile counters (agent-scope atomics
// that only grow): a Y item of step k waits until every X tile of its split has been updated k
// times, a C item until its tile's S partials of step k are in, a U item until the C tiles of its
// column are, a V item until its S2 partials are. Every workgroup walks its items (item i of a
// phase belongs to workgroup i mod G) in one global order -- the phases of step 0 in turn, then
// those of step 1, ... -- which is also the dependency order, so the earliest unfinished item
// always has its inputs and the grid cannot deadlock (all workgroups are resident: cooperative
// launch). Tiles that cross workgroups (Y partials, C, X, row-split partials) are written with
// device-coherent stores (sc1: through the XCD's own L2) and read with device-coherent loads;
// a producer waits for its stores to complete before it bumps the counter, so a consumer that sees
// the count sees the data, without the L2 write-back a release fence would cost. X* stays with the
// workgroup that owns its tile (the same one every step). Each wait is bounded and ends at once
// when a fault has been recorded; a fault stops every workgroup within the step it occurs in.
// ---------------------------------------------------------------------------


// One item of each phase per call; see the block comment above. grid = G co-resident workgroups.
__global__ __launch_bounds__(NTH) void multirhs_persistent(MultiRhsArgs a, MrpWork w, float* ckpt,
                                                           int64_t ckpt_every) {
  __shared__ __align__(16) float L0[BM * LDP];   // Y phase: A tile (pitch LDA); U phase: A^T tile (pitch LDP)
  __shared__ __align__(16) float L1[SK][LDP];    // B operand tile of either phase
  __shared__ int taus[kMaxTauLds];
  __shared__ int flag;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int G = gridDim.x, me = blockIdx.x;
  const int gt = w.gt, gr = w.gr, gn = w.gn, S = w.S, S2 = a.S2;
  const int64_t kspan = w.kspan;
  const int jpers = (int)(kspan / BM);           // n tiles per split (kspan is a multiple of 64)
  const size_t total = (size_t)a.eta_pad * a.R;
  const int lr = tid >> 4, lc = (tid & 15) * 4;
  int* status = a.status;
  const int nY = gt * gr * S, nC = gt * gr * kCq, nU = gn * gr * S2, nV = S2 > 1 ? gn * gr : 0;

  for (int64_t k = 0; k < a.K; ++k) {
    const int32_t* tk = a.idx + k * (int64_t)a.eta;
    // ---- Y items: partial products of R_tau = A_tau X over the split's columns
    for (int i = me; i < nY; i += G) {
      const int tt = i % gt, rr = (i / gt) % gr, sp = i / (gt * gr);
      const int64_t j_begin = (int64_t)sp * kspan;
      int64_t j_end = j_begin + kspan;
      if (j_end > a.n) j_end = a.n;
      const int njs = (int)((j_end - j_begin + BM - 1) / BM);
      if (!await(&w.xcnt[sp * gr + rr], (unsigned)(k * njs), status, &flag)) return;
      const int t0 = tt * BM, r0 = rr * BN;
      const float* arow[4];
      bool aok[4];
      int bad = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t = t0 + lr + 16 * q;
        aok[q] = t < a.eta;
        int row = aok[q] ? tk[t] : 0;
        if (row < 0 || (int64_t)row >= a.m) { bad = 1; row = 0; }
        arow[q] = a.A + (int64_t)row * a.ld;
      }
      if (bad) fault(status, ST_INDEX, k);
      const bool rok = r0 + lc < a.R;
      auto load = [&](int64_t jb, Stage& st) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t c = jb + lc;
          st.a[q] = (aok[q] && c < j_end) ? *reinterpret_cast<const float4*>(arow[q] + c)
                                          : make_float4(0.f, 0.f, 0.f, 0.f);
          const int64_t jj = jb + lr + 16 * q;
          st.b[q] = (jj < j_end && rok) ? ld_dev4(a.x + jj * a.R + r0 + lc) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      };
      f4 acc[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = f4{0.f, 0.f, 0.f, 0.f};
      Stage st;
      load(j_begin, st);
      for (int64_t jb = j_begin; jb < j_end; jb += SK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int mm = lr + 16 * q;
          *reinterpret_cast<float4*>(&L0[mm * LDA + lc]) = st.a[q];
          *reinterpret_cast<float4*>(&L1[mm][lc]) = st.b[q];
        }
        __syncthreads();
        if (jb + SK < j_end) load(jb + SK, st);
        mma_stage_t<true>(L0, L1, wm, wn, lane, acc);
      }
      float* Ys = a.Y + (size_t)sp * total;
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int t = t0 + wm * 32 + u * 16 + 4 * (lane >> 4) + e;
            const int r = r0 + wn * 32 + v * 16 + (lane & 15);
            if (r < a.R) st_dev1(Ys + (size_t)t * a.R + r, acc[u][v][e]);
          }
      publish(&w.ycnt[tt * gr + rr]);
    }
    // ---- C items: fixed-order sum of the S partials, coefficients
    for (int i = me; i < nC; i += G) {
      const int q = i % kCq, tt = (i / kCq) % gt, rr = i / (kCq * gt);
      if (!await(&w.ycnt[tt * gr + rr], (unsigned)((k + 1) * S), status, &flag)) return;
      const float ak = a.alpha_k ? a.alpha_k[k] : a.alpha;
      const float scale = ak / (float)a.eta;
      const int t = tt * BM + q * 16 + (tid >> 4), r = rr * BN + lc;
      if (r < a.R) {
        const size_t e = (size_t)t * a.R + r;
        // s ascending, eight partial loads issued before their adds (the step kernels' order)
        float4 y = make_float4(0.f, 0.f, 0.f, 0.f);
        int sp = 0;
        for (; sp + 8 <= S; sp += 8) {
          float4 v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = ld_dev4(a.Y + (size_t)(sp + u) * total + e);
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            y.x += v[u].x;
            y.y += v[u].y;
            y.z += v[u].z;
            y.w += v[u].w;
          }
        }
        for (; sp < S; ++sp) {
          const float4 v = ld_dev4(a.Y + (size_t)sp * total + e);
          y.x += v.x;
          y.y += v.y;
          y.z += v.z;
          y.w += v.w;
        }
        float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
        if (t < a.eta) {
          const int row = tk[t];
          if (row >= 0 && (int64_t)row < a.m) {
            const float rn = weighted_rn(a.r2, a.row_w, row);
            if (rn == 0.f) fault(status, ST_ZERO_ROW, k);
            const float4 bb = *reinterpret_cast<const float4*>(a.B + (int64_t)row * a.R + r);
            c = make_float4(scale * (y.x - bb.x) / rn, scale * (y.y - bb.y) / rn, scale * (y.z - bb.z) / rn,
                            scale * (y.w - bb.w) / rn);
            if (!isfinite(c.x) || !isfinite(c.y) || !isfinite(c.z) || !isfinite(c.w)) fault(status, ST_NONFINITE, k);
          }
        }
        st_dev4(a.C + e, c);
      }
      publish(&w.ccnt[rr]);
    }
    // ---- U items: A_tau^T C over a row split; with one split, the update of X*, X
    for (int i = me; i < nU; i += G) {
      const int jt = i % gn, rr = (i / gn) % gr, s2 = i / (gn * gr);
      if (!await(&w.ccnt[rr], (unsigned)((k + 1) * gt * kCq), status, &flag)) return;
      const int64_t j0 = (int64_t)jt * BM;
      const int r0 = rr * BN;
      const int tb0 = (int)((int64_t)s2 * a.eta / S2), tb1 = (int)((int64_t)(s2 + 1) * a.eta / S2);
      stage_tau(tk + tb0, tb1 - tb0, taus);
      __syncthreads();
      const bool colok = j0 + lc < a.n, rok = r0 + lc < a.R;
      const int etaS = tb1 - tb0;
      auto load = [&](int tb, Stage& st) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int t = tb + lr + 16 * q;
          const bool ok = t < etaS;
          const int row = ok ? taus[t] : 0;
          const bool rowok = row >= 0 && (int64_t)row < a.m;
          st.a[q] = (ok && colok && rowok) ? *reinterpret_cast<const float4*>(a.A + (int64_t)row * a.ld + j0 + lc)
                                          : make_float4(0.f, 0.f, 0.f, 0.f);
          st.b[q] = (ok && rok) ? ld_dev4(a.C + (size_t)(tb0 + t) * a.R + r0 + lc) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      };
      f4 acc[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = f4{0.f, 0.f, 0.f, 0.f};
      Stage st;
      load(0, st);
      float(*As)[LDP] = reinterpret_cast<float(*)[LDP]>(L0);
      for (int tb = 0; tb < etaS; tb += SK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          *reinterpret_cast<float4*>(&As[lr + 16 * q][lc]) = st.a[q];
          *reinterpret_cast<float4*>(&L1[lr + 16 * q][lc]) = st.b[q];
        }
        __syncthreads();
        if (tb + SK < etaS) load(tb + SK, st);
        mma_stage(As, L1, wm, wn, lane, acc);
      }
      if (faulted(status, &flag)) return;  // no update from a bad step
      const bool save = ckpt && k % ckpt_every == 0;
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t jj = j0 + wm * 32 + u * 16 + 4 * (lane >> 4) + e;
            const int r = r0 + wn * 32 + v * 16 + (lane & 15);
            if (jj < a.n && r < a.R) {
              const size_t o = (size_t)jj * a.R + r;
              if (S2 == 1) {
                const float zo = a.x_star[o];
                if (save) ckpt[(size_t)(k / ckpt_every) * a.n * a.R + o] = zo;
                const float z = zo - acc[u][v][e];
                a.x_star[o] = z;
                st_dev1(a.x + o, shrink(z, a.lambda));
              } else {
                st_dev1(a.Wp + (size_t)s2 * a.n * a.R + o, acc[u][v][e]);
              }
            }
          }
      if (S2 == 1) {
        publish(&w.xcnt[(int)(j0 / kspan) * gr + rr]);
      } else {
        publish(&w.wcnt[jt * gr + rr]);
      }
    }
    // ---- V items: fixed-order sum of the row-split partials, update of X*, X
    for (int i = me; i < nV; i += G) {
      const int jt = i % gn, rr = i / gn;
      if (!await(&w.wcnt[jt * gr + rr], (unsigned)((k + 1) * S2), status, &flag)) return;
      if (faulted(status, &flag)) return;
      const int64_t j0 = (int64_t)jt * BM;
      const int r0 = rr * BN;
      const bool save = ckpt && k % ckpt_every == 0;
      for (int e4 = tid; e4 < BM * BN / 4; e4 += NTH) {
        const int64_t jj = j0 + e4 / (BN / 4);
        const int r = r0 + (e4 % (BN / 4)) * 4;
        if (jj >= a.n || r >= a.R) continue;
        const size_t o = (size_t)jj * a.R + r;
        float4 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q < S2) v[q] = ld_dev4(a.Wp + (size_t)q * a.n * a.R + o);
        float4 tsum = v[0];
#pragma unroll
        for (int q = 1; q < 8; ++q) {
          if (q < S2) {
            tsum.x += v[q].x;
            tsum.y += v[q].y;
            tsum.z += v[q].z;
            tsum.w += v[q].w;
          }
        }
        float4 z = *reinterpret_cast<const float4*>(a.x_star + o);
        if (save) *reinterpret_cast<float4*>(ckpt + (size_t)(k / ckpt_every) * a.n * a.R + o) = z;
        z.x -= tsum.x;
        z.y -= tsum.y;
        z.z -= tsum.z;
        z.w -= tsum.w;
        *reinterpret_cast<float4*>(a.x_star + o) = z;
        st_dev4(a.x + o, make_float4(shrink(z.x, a.lambda), shrink(z.y, a.lambda), shrink(z.z, a.lambda),
                                     shrink(z.w, a.lambda)));
      }
      publish(&w.xcnt[(int)(j0 / kspan) * gr + rr]);
    }
  }
}

// status[1] = K until a fault lowers it to the step it occurred in
__global__ void mrp_status_init(int* status, int64_t K) {
  if (threadIdx.x == 0) status[1] = (int)K;
}

int multirhs_persistent_grid() {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)&multirhs_persistent, NTH, 0) != hipSuccess)
    return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

hipError_t launch_multirhs_persistent(const MultiRhsArgs& a, const MrpWork& w, int grid, hipStream_t stream,
                                      float* ckpt, int64_t ckpt_every) {
  const size_t total = (size_t)a.n * a.R;
  hipLaunchKernelGGL(init_multirhs, dim3(1024), dim3(256), 0, stream, a.x_star, a.x, total, a.lambda, a.warm);
  hipLaunchKernelGGL(mrp_status_init, dim3(1), dim3(64), 0, stream, a.status, a.K);
  if (a.K == 0) return hipGetLastError();
  MultiRhsArgs aa = a;
  MrpWork ww = w;
  float* ck = ckpt;
  int64_t ce = ckpt_every > 0 ? ckpt_every : 1;
  void* args[] = {&aa, &ww, &ck, &ce};
  return launch_persistent((const void*)&multirhs_persistent, dim3(grid), dim3(NTH), args, 0, stream);
}

// ---------------------------------------------------------------------------
// Adjoint of K unrolled multi-RHS steps (reverse mode, loss gradient dL/dx_K given).
//
// With z = x*, m_k = 1[|z_k| > lambda], A_k = A_tau_k, r_k = A_k x_k - B_tau_k and
// D_k^-2 = diag(1/||a_tau||^2), the step z_{k+1} = z_k - (alpha_k/eta) A_k^T D_k^-2 r_k,
// x_k = S_lambda(z_k) has the reverse step
//   cbar = -A_k zbar_{k+1}                        (GEMM over n, as gemm_at_x)
//   alphabar_k = <cbar, D_k^-2 r_k> / eta           (summed over the R columns)
//   rbar = (alpha_k/eta) D_k^-2 cbar
//   Bbar[tau_t] -= rbar_t                           (repeated rows each time)
//   xbar_k = A_k^T rbar                             (GEMM over eta, as gemm_att)
//   zbar_k = zbar_{k+1} + m_k . xbar_k,   lambdabar -= sum sign(z_k) m_k xbar_k
// seeded with zbar_K = m_K . xbar_K and lambdabar = -sum sign(z_K) m_K xbar_K.
// z_k and r_k of a segment of C steps are recomputed from the segment's x*
// checkpoint with the forward kernels (bitwise the forward's values). All sums
// over workgroups go through per-block partials added in a fixed order.
// ---------------------------------------------------------------------------

// workgroups of adj_coef_bbar: one (t, r) element a thread up to this many, grid-stride beyond
constexpr int kAdjCoefBlocks = 1024;
__host__ __device__ inline int adj_coef_blocks(int eta_pad, int R) {
  const int64_t b = ((int64_t)eta_pad * R + 255) / 256;
  return (int)(b < 1 ? 1 : b > kAdjCoefBlocks ? kAdjCoefBlocks : b);
}

__device__ __forceinline__ double block_sum_d(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < nw; ++w) t += red[w];
  return t;  // valid in thread 0
}

// zbar = m_K . xbar_K; partial of lambdabar per block. grid = kAdjSeedBlocks.
constexpr int kAdjSeedBlocks = 256;
__global__ __launch_bounds__(256) void adj_seed(const float* __restrict__ zK, const float* __restrict__ xbarK,
                                                size_t total, float lambda, float* __restrict__ zbar,
                                                double* __restrict__ lam_part, const int* status) {
  __shared__ double red[4];
  double acc = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const float z = zK[e], xb = xbarK[e];
    const bool on = fabsf(z) > lambda;
    zbar[e] = on ? xb : 0.f;
    if (on) acc -= (z > 0.f ? 1.0 : -1.0) * (double)xb;
  }
  const double t = block_sum_d(acc, red);
  if (threadIdx.x == 0) lam_part[blockIdx.x] = status[0] ? 0.0 : t;
}

// The step's rows in an LDS hash table (first occurrence and count per row, table size H = the
// power of two >= 2 eta) and the positions of the repeated ones: adj_hash_size(eta) slots,
// adj_bbar_lds(eta) bytes.
constexpr int kAdjMaxEta = 4096;
__host__ __device__ inline int adj_hash_size(int eta) {
  int h = 16;
  while (h < 2 * eta) h <<= 1;
  return h;
}
size_t adj_bbar_lds(int eta) { return (size_t)adj_hash_size(eta) * 12 + (size_t)eta * 8 + 16; }

// rbar = (alpha_k/eta) D^-2 cbar and the alphabar partials of step k (grid-stride over eta_pad x R,
// grid = adj_coef_blocks(eta_pad, R)), and Bbar[tau_t][r] -= rbar[t][r] for the same elements: rows repeated
// within the step are summed in ascending t by their first occurrence (no two threads touch one
// element of Bbar), which adds the rbar of the later occurrences, recomputed from the split
// partials with the same operations (the values stored for them, bit for bit), so no element waits
// for another workgroup. Every workgroup builds the step's hash table of rows. Dynamic LDS
// adj_bbar_lds(eta) bytes.
__global__ __launch_bounds__(256) void adj_coef_bbar(const float* __restrict__ Y, int S, int eta_pad,
                                                     const int32_t* __restrict__ tau, int eta,
                                                     const float* __restrict__ Rk, int R, const float* __restrict__ r2,
                                                     const float* __restrict__ alpha_k, int64_t k,
                                                     float* __restrict__ Rbar, double* __restrict__ abar_part,
                                                     float* __restrict__ Bbar, const int* status) {
  extern __shared__ int hsm[];
  __shared__ double red[4];
  const int H = adj_hash_size(eta);
  int* hkey = hsm;
  int* hmin = hsm + H;
  int* hcnt = hsm + 2 * H;
  int* st = hsm + 3 * H;
  int* dup = st + eta;
  int* ndup = dup + eta;
  const size_t total = (size_t)eta_pad * R;
  const float ak = alpha_k[k];
  double acc = 0.0;
  const bool live = status[0] == 0;
  if (live) {
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
      hkey[i] = -1;
      hmin[i] = INT_MAX;
      hcnt[i] = 0;
    }
    if (threadIdx.x == 0) *ndup = 0;
    for (int t = threadIdx.x; t < eta; t += blockDim.x) st[t] = tau[t];
  }
  __syncthreads();
  if (live)
    for (int t = threadIdx.x; t < eta; t += blockDim.x) {
      const int key = st[t];
      int h = (int)(((unsigned)key * 2654435761u) & (unsigned)(H - 1));
      for (;;) {  // at most eta distinct keys in a table of H >= 2 eta slots: a free or matching slot exists
        const int prev = atomicCAS(&hkey[h], -1, key);
        if (prev == -1 || prev == key) break;
        h = (h + 1) & (H - 1);
      }
      atomicMin(&hmin[h], t);
      atomicAdd(&hcnt[h], 1);
    }
  __syncthreads();
  if (live)
    for (int t = threadIdx.x; t < eta; t += blockDim.x) {
      const int key = st[t];
      int h = (int)(((unsigned)key * 2654435761u) & (unsigned)(H - 1));
      while (hkey[h] != key) h = (h + 1) & (H - 1);
      if (hcnt[h] > 1) dup[atomicAdd(ndup, 1)] = t;
    }
  __syncthreads();
  if (live) {
    const int nd = *ndup;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
      const int t = (int)(e / R), r = (int)(e % R);
      float rb = 0.f;
      if (t < eta) {
        const int key = st[t];
        const float cbar = -split_sum(Y, S, total, e);
        const float rn = r2[key];
        rb = (ak / (float)eta) * cbar / rn;
        acc += (double)cbar * (double)Rk[e] / ((double)eta * (double)rn);
        int h = (int)(((unsigned)key * 2654435761u) & (unsigned)(H - 1));
        while (hkey[h] != key) h = (h + 1) & (H - 1);
        if (hmin[h] == t) {
          float sum = rb;
          const int cnt = hcnt[h];
          // the other occurrences of the row, in ascending position
          for (int c = 1, last = t; c < cnt; ++c) {
            int next = INT_MAX;
            for (int i = 0; i < nd; ++i) {
              const int u = dup[i];
              if (u > last && u < next && st[u] == key) next = u;
            }
            if (next == INT_MAX) break;  // cannot happen: every occurrence of a repeated row is listed
            const float cb2 = -split_sum(Y, S, total, (size_t)next * R + r);
            sum += (ak / (float)eta) * cb2 / rn;
            last = next;
          }
          Bbar[(int64_t)key * R + r] -= sum;
        }
      }
      Rbar[e] = rb;
    }
  }
  const double t = block_sum_d(acc, red);
  if (threadIdx.x == 0) abar_part[k * gridDim.x + blockIdx.x] = t;
}

// xbar = A_tau^T Rbar (MFMA as gemm_att_c_update); epilogue zbar += m_k . xbar and the
// lambdabar partial of the block. grid = (ceil(n/64), R/64).
__global__ __launch_bounds__(NTH) void gemm_att_adj(const float* __restrict__ A, int64_t ld, int64_t n,
                                                    const int32_t* __restrict__ tau, int eta,
                                                    const float* __restrict__ Rbar, int R, const float* __restrict__ Zk,
                                                    float* __restrict__ zbar, float lambda,
                                                    double* __restrict__ lam_part, const int* status) {
  __shared__ __align__(16) float As[SK][LDP];
  __shared__ __align__(16) float Bs[SK][LDP];
  __shared__ int taus[kMaxTauLds];
  __shared__ double red[4];
  const int blk = blockIdx.y * gridDim.x + blockIdx.x;
  if (status[0]) {
    if (threadIdx.x == 0) lam_part[blk] = 0.0;
    return;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t j0 = (int64_t)blockIdx.x * BM;
  const int r0 = blockIdx.y * BN;
  stage_tau(tau, eta, taus);
  __syncthreads();
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  att_mainloop(A, ld, n, taus, eta, Rbar, R, j0, r0, As, Bs, acc);
  double lp = 0.0;
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
          const float z = Zk[o];
          if (fabsf(z) > lambda) {
            const float xb = acc[i][j][v];
            zbar[o] += xb;
            lp -= (z > 0.f ? 1.0 : -1.0) * (double)xb;
          }
        }
      }
  const double t = block_sum_d(lp, red);
  if (threadIdx.x == 0) lam_part[blk] = t;
}

// Epilogue of the row-split adjoint product: xbar = sum_s Wp[s] (s ascending), then as in
// gemm_att_adj. grid = (ceil(n/64), R/64), the same blocks (and lambdabar partials) as gemm_att_adj;
// each thread takes four float4 of the block's 64 x 64 tile, all loads issued before use.
template <int S2>
__global__ __launch_bounds__(NTH) void att_reduce_adj(const float* __restrict__ Wp, int64_t n, int R,
                                                      const float* __restrict__ Zk, float* __restrict__ zbar,
                                                      float lambda, double* __restrict__ lam_part, const int* status) {
  __shared__ double red[4];
  const int blk = blockIdx.y * gridDim.x + blockIdx.x;
  if (status[0]) {
    if (threadIdx.x == 0) lam_part[blk] = 0.0;
    return;
  }
  const int64_t j0 = (int64_t)blockIdx.x * BM;
  const int r0 = blockIdx.y * BN;
  const size_t nr = (size_t)n * R;
  constexpr int kPer = BM * BN / (4 * NTH);
  float4 w[kPer][S2], zk[kPer];
  size_t off[kPer];
  bool ok[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = 4 * (threadIdx.x + NTH * u);
    const int64_t jj = j0 + e / BN;
    const int r = r0 + e % BN;
    ok[u] = jj < n && r < R;
    off[u] = ok[u] ? (size_t)jj * R + r : 0;
#pragma unroll
    for (int q = 0; q < S2; ++q) w[u][q] = *reinterpret_cast<const float4*>(Wp + q * nr + off[u]);
    zk[u] = *reinterpret_cast<const float4*>(Zk + off[u]);
  }
  double lp = 0.0;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    if (!ok[u]) continue;
    float4 xb = w[u][0];
#pragma unroll
    for (int q = 1; q < S2; ++q) {
      xb.x += w[u][q].x;
      xb.y += w[u][q].y;
      xb.z += w[u][q].z;
      xb.w += w[u][q].w;
    }
    const float zz[4] = {zk[u].x, zk[u].y, zk[u].z, zk[u].w};
    const float xx[4] = {xb.x, xb.y, xb.z, xb.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (fabsf(zz[c]) > lambda) {
        zbar[off[u] + c] += xx[c];
        lp -= (zz[c] > 0.f ? 1.0 : -1.0) * (double)xx[c];
      }
    }
  }
  const double t = block_sum_d(lp, red);
  if (threadIdx.x == 0) lam_part[blk] = t;
}

// alpha_bar[k] = sum of the step's partials; lambda_bar = seed partials, then steps 0..K-1, each in order.
__global__ __launch_bounds__(256) void adj_finish(const double* __restrict__ abar_part, int nblk_coef,
                                                  const double* __restrict__ lam_part, int64_t K, int nblk_att,
                                                  float* __restrict__ alpha_bar, double* __restrict__ lambda_bar,
                                                  const int* status) {
  __shared__ double red[256];
  for (int64_t k = threadIdx.x; k < K; k += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk_coef; ++b) s += abar_part[k * nblk_coef + b];
    alpha_bar[k] = status[0] ? 0.f : (float)s;
  }
  // lam_part: [kAdjSeedBlocks] seed, then K x nblk_att
  double s = 0.0;
  const int64_t total = kAdjSeedBlocks + K * (int64_t)nblk_att;
  const int64_t per = (total + blockDim.x - 1) / blockDim.x;
  for (int64_t i = threadIdx.x * per; i < (threadIdx.x + 1) * per && i < total; ++i) s += lam_part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)blockDim.x; ++w) t += red[w];
    *lambda_bar = status[0] ? 0.0 : t;
  }
}

__global__ void fill_zero_f32(float* p, size_t total) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x)
    p[e] = 0.f;
}

size_t adjoint_lam_parts(int64_t n, int R, int64_t K) {
  const int gr = (R + BN - 1) / BN;
  const int gn = (int)((n + BM - 1) / BM);
  return kAdjSeedBlocks + (size_t)K * gn * gr;
}
size_t adjoint_abar_parts(int64_t K, int eta_pad, int R) {
  return (size_t)(K > 0 ? K : 1) * adj_coef_blocks(eta_pad, R);
}

hipError_t launch_adjoint(const AdjointArgs& d, hipStream_t stream) {
  const MultiRhsArgs& a = d.f;
  const size_t total = (size_t)a.n * a.R;
  const size_t etot = (size_t)a.eta_pad * a.R;
  const int gt = (a.eta + BM - 1) / BM;
  const int gr = (a.R + BN - 1) / BN;
  const int gn = (int)((a.n + BM - 1) / BM);
  const int nblk_att = gn * gr;
  const int nblk_coef = adj_coef_blocks(a.eta_pad, a.R);
  if (hipFuncSetAttribute((const void*)&adj_coef_bbar, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)adj_bbar_lds(a.eta)) != hipSuccess)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(fill_zero_f32, dim3(1024), dim3(256), 0, stream, d.Bbar, (size_t)a.m * a.R);
  hipLaunchKernelGGL(adj_seed, dim3(kAdjSeedBlocks), dim3(256), 0, stream, d.zK, d.xbarK, total, a.lambda, d.zbar,
                     d.lam_part, a.status);
  const int64_t C = d.ckpt_every;
  const int64_t nseg = (a.K + C - 1) / C;
  MultiRhsArgs f = a;
  for (int64_t s = nseg - 1; s >= 0; --s) {
    const int64_t k0 = s * C, k1 = (k0 + C < a.K) ? k0 + C : a.K;
    // recompute z_k0..z_k1 and r_k0..r_{k1-1} from the checkpoint
    hipError_t e = hipMemcpyAsync(d.Zh, d.ckpt + (size_t)s * total, total * sizeof(float), hipMemcpyDeviceToDevice,
                                  stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(init_multirhs, dim3(1024), dim3(256), 0, stream, d.Zh, a.x, total, a.lambda, 1);
    // the segment's first indices are range-checked before any kernel reads A with them
    hipLaunchKernelGGL(step_check, dim3(1), dim3(1024), 0, stream, a.idx + k0 * (int64_t)a.eta, a.eta, a.m, a.status,
                       k0);
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t j = k - k0;
      f.K = k1;  // the step check after the segment's last step is skipped
      multirhs_step(f, k, d.Zh + (size_t)j * total, d.Zh + (size_t)(j + 1) * total, d.Rh + (size_t)j * etot, stream);
    }
    for (int64_t k = k1 - 1; k >= k0; --k) {
      const int64_t j = k - k0;
      const int32_t* tk = a.idx + k * (int64_t)a.eta;
      launch_at_x(a, tk, d.zbar, 0, k, stream);
      hipLaunchKernelGGL(adj_coef_bbar, dim3(nblk_coef), dim3(256), adj_bbar_lds(a.eta), stream, a.Y, a.S,
                         a.eta_pad, tk, a.eta, d.Rh + (size_t)j * etot, a.R, a.r2, a.alpha_k, k, a.C, d.abar_part,
                         d.Bbar, a.status);
      if (a.S2 > 1) {
        if (a.tile == 128)
          launch_att(a, tk, a.C, nullptr, nullptr, false, stream);
        else
          hipLaunchKernelGGL(gemm_att_partial, dim3(gn, gr, a.S2), dim3(NTH), 0, stream, a.A, a.ld, a.n, tk, a.eta,
                             a.C, a.R, a.Wp, a.status);
        const float* zk = d.Zh + (size_t)j * total;
        double* lp = d.lam_part + kAdjSeedBlocks + (size_t)k * nblk_att;
        if (a.S2 == 2)
          hipLaunchKernelGGL(att_reduce_adj<2>, dim3(gn, gr), dim3(NTH), 0, stream, a.Wp, a.n, a.R, zk, d.zbar,
                             a.lambda, lp, a.status);
        else if (a.S2 == 4)
          hipLaunchKernelGGL(att_reduce_adj<4>, dim3(gn, gr), dim3(NTH), 0, stream, a.Wp, a.n, a.R, zk, d.zbar,
                             a.lambda, lp, a.status);
        else
          hipLaunchKernelGGL(att_reduce_adj<8>, dim3(gn, gr), dim3(NTH), 0, stream, a.Wp, a.n, a.R, zk, d.zbar,
                             a.lambda, lp, a.status);
      } else {
        hipLaunchKernelGGL(gemm_att_adj, dim3(gn, gr), dim3(NTH), 0, stream, a.A, a.ld, a.n, tk, a.eta, a.C, a.R,
                           d.Zh + (size_t)j * total, d.zbar, a.lambda,
                           d.lam_part + kAdjSeedBlocks + (size_t)k * nblk_att, a.status);
      }
    }
  }
  hipLaunchKernelGGL(adj_finish, dim3(1), dim3(256), 0, stream, d.abar_part, nblk_coef, d.lam_part, a.K, nblk_att,
                     d.alpha_bar,
                     d.lambda_bar, a.status);
  return hipGetLastError();
}

}  // namespace rsk
