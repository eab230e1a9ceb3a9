// Linearized Bregman method (the full-batch comparator of RSKA: the remark on
// its convergence rate in Sec. 4, eq. (bsk) with every row in the block):
//   x*_{k+1} = x*_k - s A^T (A x_k - b),  x_{k+1} = S_lambda(x*_{k+1}),
// s = 1/||A||_2^2 in the paper, and sigma_max(A)^2 by power iteration on A^T A.
//
// One iteration reads A once. lb_pass: each persistent workgroup takes a block
// of whole rows; x (n) sits in LDS and the thread's share of the partial
// A^T r (chunks q = tid + NT c) in registers. Per row: the dot from the row
// chunks in registers (the next row's chunks are already in flight), a
// fixed-order block reduction (DPP sums in each wave, then the waves in
// order), r_i = dot - b_i, and the row's contribution r_i a_i to the partial.
// lb_reduce sums the workgroups' partials in a fixed segmented order and applies
// the step with S_lambda fused. All sums have fixed orders: runs are bitwise
// reproducible.
#include "rsk_dense_run.hpp"

namespace rsk {

namespace {

constexpr int kLbWaves = kLbThreads / 64;

}  // namespace

template <typename T, int VEC, int CPT, int NB>
__global__ __launch_bounds__(kLbThreads) void lb_pass(const T* __restrict__ A, int64_t m, int64_t n, int64_t ld,
                                                      const T* __restrict__ x, const T* __restrict__ b,
                                                      T* __restrict__ part, double* __restrict__ rpart,
                                                      const int* status) {
  using V = Vec<T, VEC>;
  extern __shared__ __align__(16) unsigned char lsm[];
  __shared__ T red[2][kLbWaves];
  if (status && status[0]) return;
  V* xs = reinterpret_cast<V*>(lsm);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = blockIdx.x, G = gridDim.x;
  const int64_t nch = (n + VEC - 1) / VEC;
  for (int64_t q = tid; q < nch; q += kLbThreads) {
    V v;
#pragma unroll
    for (int e = 0; e < VEC; ++e) v.v[e] = q * VEC + e < n ? x[q * VEC + e] : T(0);
    xs[q] = v;
  }
  __syncthreads();
  const int64_t i0 = (int64_t)g * m / G, i1 = (int64_t)(g + 1) * m / G;
  V acc[CPT], buf[NB][CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[c].v[e] = T(0);
  // Which loaded elements lie in the row (the rest, past n or past the last chunk, is masked
  // out of the dot; their products in acc land past n and are never read).
  unsigned long long inrow = 0;
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int64_t q = tid + (int64_t)kLbThreads * c;
      if (q < nch && q * VEC + e < n) inrow |= 1ull << (c * VEC + e);
    }
  // Raw 16-byte (or element) loads of row i, the chunk index clamped into the row: no select
  // touches the loaded registers before their use, so the loads stay in flight.
  auto load_row = [&](int64_t i, V (&dst)[CPT]) {
    const T* rowp = A + i * ld;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int64_t q = tid + (int64_t)kLbThreads * c;
      dst[c] = *reinterpret_cast<const V*>(rowp + (q < nch ? q : nch - 1) * VEC);
    }
  };
  double rr = 0.0;
  auto row_step = [&](int64_t i, const V (&cur)[CPT]) {
    const T bi = b ? b[i] : T(0);
    T dot = T(0);
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int64_t q = tid + (int64_t)kLbThreads * c;
      const V xv = xs[q < nch ? q : nch - 1];
#pragma unroll
      for (int e = 0; e < VEC; ++e) dot += ((inrow >> (c * VEC + e)) & 1 ? cur[c].v[e] : T(0)) * xv.v[e];
    }
    dot = lane_sum(dot, 64);
    const int par = (int)(i & 1);
    if (lane == 0) red[par][wave] = dot;
    __syncthreads();  // red[par] is rewritten two rows later, after the next barrier
    T sum = T(0);
#pragma unroll
    for (int w = 0; w < kLbWaves; ++w) sum += red[par][w];
    const T r = sum - bi;
    rr += (double)r * (double)r;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[c].v[e] += r * cur[c].v[e];
  };
  // Rows through NB register buffers used in turn: while row i is reduced, rows i+1 .. i+NB-1
  // are in flight. Past the block's last row the clamped index reloads that row (never used).
  if (i0 < i1) {
#pragma unroll
    for (int u = 0; u < NB - 1; ++u) load_row(i0 + u < i1 ? i0 + u : i1 - 1, buf[u]);
    for (int64_t i = i0; i < i1; i += NB) {
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int64_t ahead = i + u + NB - 1;
        load_row(ahead < i1 ? ahead : i1 - 1, buf[(u + NB - 1) % NB]);
        if (i + u < i1) row_step(i + u, buf[u]);
      }
    }
  }
  T* pg = part + (size_t)g * nch * VEC;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int64_t q = tid + (int64_t)kLbThreads * c;
    if (q < nch) *reinterpret_cast<V*>(pg + q * VEC) = acc[c];
  }
  if (tid == 0) rpart[g] = rr;  // every thread of the block holds the same sum of r_i^2
}

// g_j = sum over the workgroups' partials part[q][j], in a fixed order: kSumSeg segments of
// consecutive workgroups, each summed in order, then the segment sums in order. A block
// covers kSumCols chunks of columns; all of its partial loads are independent.
//   mode 0 (LB): x*_j -= step g_j, x_j = S_lambda(x*_j); residual norm and step count.
//   mode 1 (power iteration): w_j = g_j written over part[0][j] (read by this thread only).
constexpr int kSumSeg = 16, kSumCols = 16;
template <typename T, int VEC>
__global__ __launch_bounds__(kSumSeg * kSumCols) void lb_reduce(T* __restrict__ part, int G, int64_t n,
                                                                int64_t nstride, int mode, T* __restrict__ z,
                                                                T* __restrict__ x, T step, T lambda,
                                                                const double* __restrict__ rpart, double* res_out,
                                                                int* status, int64_t k) {
  using V = Vec<T, VEC>;
  __shared__ V red[kSumSeg][kSumCols];
  if (status && status[0]) return;
  const int col = threadIdx.x % kSumCols, seg = threadIdx.x / kSumCols;
  const int64_t nch = (n + VEC - 1) / VEC;
  const int64_t qc = blockIdx.x * (int64_t)kSumCols + col;
  const int g0 = seg * G / kSumSeg, g1 = (seg + 1) * G / kSumSeg;
  V acc;
#pragma unroll
  for (int e = 0; e < VEC; ++e) acc.v[e] = T(0);
  if (qc < nch) {
    const T* p = part + qc * VEC;
#pragma unroll 8
    for (int q = g0; q < g1; ++q) {
      const V t = *reinterpret_cast<const V*>(p + (size_t)q * nstride);
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc.v[e] += t.v[e];
    }
  }
  red[seg][col] = acc;
  __syncthreads();
  int bad = 0;
  if (seg == 0 && qc < nch) {
    V t = red[0][col];
#pragma unroll
    for (int sg = 1; sg < kSumSeg; ++sg)
#pragma unroll
      for (int e = 0; e < VEC; ++e) t.v[e] += red[sg][col].v[e];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int64_t j = qc * VEC + e;
      if (j >= n) break;
      if (mode == 0) {
        const T zj = z[j] - step * t.v[e];
        z[j] = zj;
        x[j] = shrink(zj, lambda);
        bad |= !isfinite(zj);
      } else {
        part[j] = t.v[e];
      }
    }
  }
  if (mode == 0) {
    if (bad) set_status(status, ST_NONFINITE);
    if (blockIdx.x == 0 && threadIdx.x < 64) {
      double r2 = 0.0;
      for (int q = threadIdx.x; q < G; q += 64) r2 += rpart[q];
      r2 = wave_sum(r2);
      if (threadIdx.x == 0) {
        status[1] = (int)(k + 1);  // iterations started; the nonfinite check marks a failed one
        if (res_out) *res_out = sqrt(r2);
      }
    }
  }
}

// Start: x* = 0 and x = 0, or (warm) x = S_lambda(x*) from the given x*.
template <typename T>
__global__ void lb_init(T* z, T* x, int64_t n, T lambda, int warm) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    if (warm) {
      x[j] = shrink(z[j], lambda);
    } else {
      z[j] = T(0);
      x[j] = T(0);
    }
  }
}

// One workgroup: ||x - xref|| / ||xref|| into err (fixed order).
template <typename T>
__global__ __launch_bounds__(1024) void lb_err(const T* __restrict__ x, const T* __restrict__ xref, int64_t n,
                                               double* err, const int* status) {
  __shared__ double red[2][16];
  if (status[0]) return;
  double e2 = 0.0, r2 = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    const double rf = (double)xref[j], d = (double)x[j] - rf;
    e2 += d * d;
    r2 += rf * rf;
  }
  e2 = wave_sum(e2);
  r2 = wave_sum(r2);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = e2; red[1][threadIdx.x >> 6] = r2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double se = 0.0, sr = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { se += red[0][w]; sr += red[1][w]; }
    *err = sr > 0.0 ? sqrt(se / sr) : sqrt(se);
  }
}

// est = <v, w> (||v|| = 1), then v = w / ||w||.
template <typename T>
__global__ __launch_bounds__(1024) void pw_finish(const T* __restrict__ w, int64_t n, T* __restrict__ v,
                                                  double* est) {
  __shared__ double red[2][16];
  __shared__ double scale;
  double vw = 0.0, ww = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    const double wj = (double)w[j];
    vw += (double)v[j] * wj;
    ww += wj * wj;
  }
  vw = wave_sum(vw);
  ww = wave_sum(ww);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = vw; red[1][threadIdx.x >> 6] = ww; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { a += red[0][k]; c += red[1][k]; }
    *est = a;
    scale = c > 0.0 ? 1.0 / sqrt(c) : 0.0;
  }
  __syncthreads();
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) v[j] = (T)((double)w[j] * scale);
}

// v_j = (1 + (j mod 7)/7) / ||.||
template <typename T>
__global__ __launch_bounds__(1024) void pw_start(T* v, int64_t n) {
  __shared__ double red[16];
  __shared__ double sc;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    const double a = 1.0 + (double)(j % 7) / 7.0;
    s += a * a;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    sc = 1.0 / sqrt(t);
  }
  __syncthreads();
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) v[j] = (T)((1.0 + (double)(j % 7) / 7.0) * sc);
}

// ---------------------------------------------------------------------------
// Block sparse Kaczmarz, eq. (bsk) of Sec. 1.1 (eta <= kBskMaxEta rows a step):
//   x*_{k+1} = x*_k - w A_tau^T (A_tau x_k - b_tau) / ||A_tau||_2^2,  x_{k+1} = S_lambda(x*_{k+1}).
// ||A_tau_k||_2^2 depends on the step's rows only, not on x, so bsk_norms computes it for
// every step up front (persistent workgroups, one step at a time): the Gram matrix
// A_tau A_tau^T over LDS tiles of the rows, then its largest eigenvalue to rounding
// (Householder tridiagonalisation in double, Sturm-count multisection). It writes the
// per-step relaxation alpha_k = eta w / ||A_tau_k||_2^2, with which the RSKA step with unit
// row norms, (alpha_k / eta) sum_t (<a_t, x> - b_t) a_t, is the block step of eq. (bsk);
// the iteration itself then runs in the persistent RSKA kernels.
// ---------------------------------------------------------------------------

constexpr int kBskTile = 64;  // columns per LDS tile
constexpr int kBskQ = kBskMaxEta / (kBskThreads / 64);  // columns of the Gram matrix a lane updates

struct BskEig {
  double Gm[kBskMaxEta][kBskMaxEta + 1];
  double vs[kBskMaxEta], ws[kBskMaxEta], dd[kBskMaxEta], ee[kBskMaxEta];
  double pr[kBskThreads / 64][kBskMaxEta];
  double bnd[2][kBskThreads / 64];
};

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Largest eigenvalue of the symmetric eta x eta matrix in L.Gm (destroyed), by the whole
// workgroup. Lane i of wave q owns row i and columns kBskQ q .. kBskQ q + kBskQ - 1; the
// scalars every wave needs are computed by every wave alike from the same data.
__device__ double gram_lambda_max(BskEig& L, int eta) {
  const int tid = threadIdx.x, i = tid & 63, q = tid >> 6, j0 = q * kBskQ;
  if (tid < kBskMaxEta) { L.vs[tid] = 0.0; L.ws[tid] = 0.0; L.ee[tid] = 0.0; L.dd[tid] = 0.0; }
  __syncthreads();
  // Householder reduction to tridiagonal form: H = I - beta v v^T on rows/columns k+1..
  for (int k = 0; k + 2 < eta; ++k) {
    const bool own = i > k && i < eta;
    const double xi = own ? L.Gm[i][k] : 0.0;
    const double nx2 = lane_sum(xi * xi, 64);
    double alpha = 0.0;
    if (nx2 > 0.0) {
      const double x0 = L.Gm[k + 1][k];
      alpha = x0 > 0.0 ? -sqrt(nx2) : sqrt(nx2);
      const double vi = own ? (i == k + 1 ? xi - alpha : xi) : 0.0;
      const double beta = 2.0 / lane_sum(vi * vi, 64);
      if (q == 0) L.vs[i] = vi;
      __syncthreads();
      double pp = 0.0;
#pragma unroll 4
      for (int c = 0; c < kBskQ; ++c) {
        const int j = j0 + c;
        pp += (own && j > k && j < eta) ? L.Gm[i][j] * L.vs[j] : 0.0;
      }
      L.pr[q][i] = pp;
      __syncthreads();
      double pi = 0.0;
#pragma unroll
      for (int r = 0; r < kBskThreads / 64; ++r) pi += L.pr[r][i];
      pi *= beta;
      const double pv = lane_sum(own ? pi * vi : 0.0, 64);
      const double wi = pi - 0.5 * beta * pv * vi;
      if (q == 0) L.ws[i] = wi;
      __syncthreads();
#pragma unroll 4
      for (int c = 0; c < kBskQ; ++c) {
        const int j = j0 + c;
        if (own && j > k && j < eta) L.Gm[i][j] -= vi * L.ws[j] + wi * L.vs[j];
      }
      __syncthreads();
    }
    if (tid == 0) {
      L.dd[k] = L.Gm[k][k];
      L.ee[k] = alpha;
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (eta >= 2) {
      L.dd[eta - 2] = L.Gm[eta - 2][eta - 2];
      L.ee[eta - 2] = L.Gm[eta - 1][eta - 2];
    }
    L.dd[eta - 1] = L.Gm[eta - 1][eta - 1];
  }
  __syncthreads();
  // count(s) = #eigenvalues < s = #negative pivots of T - s I; thread l tests shift s_l.
  const double di = i < eta ? L.dd[i] : -INFINITY;
  const double ri = i < eta ? fabs(i > 0 ? L.ee[i - 1] : 0.0) + fabs(i + 1 < eta ? L.ee[i] : 0.0) : 0.0;
  double lo = wave_max_d(di), hi = wave_max_d(i < eta ? di + ri : -INFINITY);
  const double e2max = wave_max_d(i < eta ? L.ee[i] * L.ee[i] : 0.0);
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, e2max);
  constexpr double kParts = kBskThreads + 1;
  for (int round = 0; round < 10 && hi > lo; ++round) {
    const double width = hi - lo;
    const double sg = lo + width * (double)(tid + 1) / kParts;
    int cnt = 0;
    double qv = L.dd[0] - sg;
    if (fabs(qv) < pivmin) qv = -pivmin;
    cnt += qv < 0.0;
    for (int t = 1; t < eta; ++t) {
      qv = (L.dd[t] - sg) - L.ee[t - 1] * L.ee[t - 1] / qv;
      if (fabs(qv) < pivmin) qv = -pivmin;
      cnt += qv < 0.0;
    }
    // shifts at or below lambda_max have cnt < eta; they are a prefix of the threads
    const unsigned long long below = __ballot(cnt < eta);
    if (i == 0) L.bnd[round & 1][q] = (double)__popcll(below);
    __syncthreads();
    int nb = 0;
#pragma unroll
    for (int r = 0; r < kBskThreads / 64; ++r) nb += (int)L.bnd[round & 1][r];
    if (nb == 0) {
      hi = lo + width / kParts;
    } else {
      const double nlo = lo + width * (double)nb / kParts;
      hi = nb == kBskThreads ? hi : lo + width * (double)(nb + 1) / kParts;
      lo = nlo;
    }
  }
  return 0.5 * (lo + hi);
}

template <typename T>
__global__ __launch_bounds__(kBskThreads) void bsk_norms(const T* __restrict__ A, int64_t m, int64_t n, int64_t ld,
                                                         const int* __restrict__ tau0, int eta, int64_t K, double w,
                                                         T* __restrict__ alpha_k, double* __restrict__ norm2,
                                                         int* status) {
  __shared__ T tile[kBskMaxEta][kBskTile + 1];
  __shared__ int rows[kBskMaxEta];
  __shared__ BskEig L;
  const int tid = threadIdx.x;
  const int eta4 = (eta + 3) & ~3;
  const int bi = tid / 16, bj = tid % 16;  // this thread's 4x4 block of the Gram matrix
  const bool gb = 4 * bi < eta && 4 * bj < eta;
  constexpr int kLoads = kBskMaxEta * kBskTile / kBskThreads;  // tile elements a thread loads
  for (int64_t k = blockIdx.x; k < K; k += gridDim.x) {
    if (tid < kBskMaxEta) {
      int r = -1;
      if (tid < eta) {
        r = tau0[k * eta + tid];
        if (r < 0 || r >= m) {
          set_status(status, ST_INDEX);
          r = -1;
        }
      }
      rows[tid] = r;
    }
    __syncthreads();
    T acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = T(0);
    for (int64_t cb = 0; cb < n; cb += kBskTile) {
      const int cw = (int)(n - cb < kBskTile ? n - cb : kBskTile);
      T v[kLoads];
#pragma unroll
      for (int u = 0; u < kLoads; ++u) {  // all loads issued before any LDS store
        const int e = tid + u * kBskThreads, t = e / kBskTile, j = e % kBskTile;
        const int r = rows[t];
        v[u] = (t < eta4 && j < cw && r >= 0) ? A[(int64_t)r * ld + cb + j] : T(0);
      }
      __syncthreads();  // the previous tile's reads are done
#pragma unroll
      for (int u = 0; u < kLoads; ++u) {
        const int e = tid + u * kBskThreads;
        tile[e / kBskTile][e % kBskTile] = v[u];
      }
      __syncthreads();
      if (gb) {
#pragma unroll 4
        for (int j = 0; j < kBskTile; ++j) {
          T a[4], c[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            a[u] = tile[4 * bi + u][j];
            c[u] = tile[4 * bj + u][j];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) acc[u][vv] += a[u] * c[vv];
        }
      }
    }
    if (gb) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv)
          if (4 * bi + u < eta && 4 * bj + vv < eta) L.Gm[4 * bi + u][4 * bj + vv] = (double)acc[u][vv];
    }
    __syncthreads();
    const double s2 = gram_lambda_max(L, eta);
    if (tid == 0) {
      if (s2 > 0.0 && isfinite(s2)) {
        alpha_k[k] = (T)((double)eta * w / s2);
      } else {
        alpha_k[k] = T(0);
        set_status(status, ST_ZERO_ROW);
      }
      if (norm2) norm2[k] = s2;
    }
    __syncthreads();  // rows, tile and L are reused by the next step
  }
}

template <typename T>
__global__ void fill_value(T* p, int64_t count, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// Three row buffers where they fit in the registers of two waves per SIMD, else two.
template <typename T, int V, int CPT>
constexpr int kLbBuffers = CPT * V * (int)sizeof(T) <= 160 ? 3 : 2;

template <typename T, int V>
static void* lb_pass_fn_v(int cpt) {
  switch (cpt) {
    case 1: return (void*)&lb_pass<T, V, 1, kLbBuffers<T, V, 1>>;
    case 2: return (void*)&lb_pass<T, V, 2, kLbBuffers<T, V, 2>>;
    case 4: return (void*)&lb_pass<T, V, 4, kLbBuffers<T, V, 4>>;
    case 6: return (void*)&lb_pass<T, V, 6, kLbBuffers<T, V, 6>>;
    case 8: return (void*)&lb_pass<T, V, 8, kLbBuffers<T, V, 8>>;
    case 10: return (void*)&lb_pass<T, V, 10, kLbBuffers<T, V, 10>>;
    case 12: return (void*)&lb_pass<T, V, 12, kLbBuffers<T, V, 12>>;
    default: return nullptr;
  }
}

template <typename T>
static void* lb_pass_fn(int vec, int cpt) {
  return vec == 1 ? lb_pass_fn_v<T, 1>(cpt) : lb_pass_fn_v<T, kLbVec<T>>(cpt);
}

// vec: kLbVec<T> (A 16-byte aligned, ld a multiple of kLbVec) or 1.
// Returns 1 when planned, 0 when the shape is not supported, -1 when a HIP query failed.
template <typename T>
int lb_plan(int64_t n, int vec, int* cpt, size_t* lds, int* grid, int64_t* nstride) {
  const int64_t nch = (n + vec - 1) / vec;
  const int64_t need = (nch + kLbThreads - 1) / kLbThreads;
  *cpt = 0;
  for (int c : {1, 2, 4, 6, 8, 10, 12})
    if (need <= c) { *cpt = c; break; }
  if (n < 1 || !*cpt || (vec != 1 && vec != kLbVec<T>)) return 0;
  *nstride = nch * vec;
  *lds = (size_t)nch * vec * sizeof(T);
  void* fn = lb_pass_fn<T>(vec, *cpt);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)*lds) != hipSuccess) return -1;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kLbThreads, *lds) != hipSuccess) return -1;
  if (per_cu < 1) return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  *grid = per_cu * cus;
  return 1;
}

template <typename T>
static hipError_t lb_pass_launch(const LbArgs<T>& a, const T* x, const T* b, hipStream_t s) {
  void* fn = lb_pass_fn<T>(a.vec, a.cpt);
  if (!fn) return hipErrorInvalidValue;
  const T* Ap = a.A;
  int64_t m = a.m, n = a.n, ld = a.ld;
  T* part = a.part;
  double* rpart = a.rpart;
  const int* status = a.status;
  void* args[] = {&Ap, &m, &n, &ld, &x, &b, &part, &rpart, &status};
  return hipLaunchKernel(fn, dim3(a.G), dim3(kLbThreads), args, a.lds, s);
}

template <typename T>
static void lb_reduce_launch(const LbArgs<T>& a, int mode, int64_t k, hipStream_t s) {
  const int64_t nch = (a.n + a.vec - 1) / a.vec;
  const dim3 grid((unsigned)((nch + kSumCols - 1) / kSumCols)), block(kSumSeg * kSumCols);
  T* z = mode == 0 ? a.z : nullptr;
  T* x = mode == 0 ? a.x : nullptr;
  int* st = mode == 0 ? a.status : nullptr;
  double* res = mode == 0 && a.res_hist ? a.res_hist + k : nullptr;
  if (a.vec == 1)
    hipLaunchKernelGGL((lb_reduce<T, 1>), grid, block, 0, s, a.part, a.G, a.n, a.nstride, mode, z, x, a.step,
                       a.lambda, a.rpart, res, st, k);
  else
    hipLaunchKernelGGL((lb_reduce<T, kLbVec<T>>), grid, block, 0, s, a.part, a.G, a.n, a.nstride, mode, z, x,
                       a.step, a.lambda, a.rpart, res, st, k);
}

template <typename T>
hipError_t launch_lb(const LbArgs<T>& a, hipStream_t s) {
  const int64_t ib = (a.n + 255) / 256;
  const int ub = (int)(ib < 1024 ? ib : 1024);
  hipLaunchKernelGGL(lb_init<T>, dim3(ub), dim3(256), 0, s, a.z, a.x, a.n, a.lambda, a.warm);
  for (int64_t k = 0; k < a.K; ++k) {
    hipError_t e = lb_pass_launch(a, a.x, a.b, s);
    if (e != hipSuccess) return e;
    lb_reduce_launch(a, 0, k, s);
    if (a.xref && a.check_every > 0 && a.err_hist && (k + 1) % a.check_every == 0)
      hipLaunchKernelGGL(lb_err<T>, dim3(1), dim3(1024), 0, s, a.x, a.xref, a.n,
                         a.err_hist + (k + 1) / a.check_every - 1, a.status);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_power(const LbArgs<T>& a, int64_t iters, T* v, double* est, hipStream_t s) {
  hipLaunchKernelGGL(pw_start<T>, dim3(1), dim3(1024), 0, s, v, a.n);
  for (int64_t it = 0; it < iters; ++it) {
    hipError_t e = lb_pass_launch(a, v, (const T*)nullptr, s);
    if (e != hipSuccess) return e;
    lb_reduce_launch(a, 1, it, s);
    hipLaunchKernelGGL(pw_finish<T>, dim3(1), dim3(1024), 0, s, a.part, a.n, v, est);
  }
  return hipGetLastError();
}

// Resident workgroups of bsk_norms (at most K).
template <typename T>
int bsk_grid(int64_t K) {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)&bsk_norms<T>, kBskThreads, 0) != hipSuccess ||
      per_cu < 1)
    return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const int64_t g = (int64_t)per_cu * cus;
  return (int)(K < g ? (K > 0 ? K : 1) : g);
}

template <typename T>
hipError_t launch_bsk_norms(const BskArgs<T>& a, hipStream_t s) {
  const int64_t ib = (a.m + 255) / 256;
  hipLaunchKernelGGL(fill_value<T>, dim3((unsigned)(ib < 1024 ? ib : 1024)), dim3(256), 0, s, a.ones, a.m, T(1));
  if (a.K > 0) {
    const int G = bsk_grid<T>(a.K);
    if (G < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bsk_norms<T>, dim3(G), dim3(kBskThreads), 0, s, a.A, a.m, a.n, a.ld, a.tau, a.eta, a.K, a.w,
                       a.alpha_k, a.norm2_hist, a.status);
  }
  return hipGetLastError();
}

template hipError_t launch_bsk_norms<float>(const BskArgs<float>&, hipStream_t);
template hipError_t launch_bsk_norms<double>(const BskArgs<double>&, hipStream_t);

template int lb_plan<float>(int64_t, int, int*, size_t*, int*, int64_t*);
template int lb_plan<double>(int64_t, int, int*, size_t*, int*, int64_t*);
template hipError_t launch_lb<float>(const LbArgs<float>&, hipStream_t);
template hipError_t launch_lb<double>(const LbArgs<double>&, hipStream_t);
template hipError_t launch_power<float>(const LbArgs<float>&, int64_t, float*, double*, hipStream_t);
template hipError_t launch_power<double>(const LbArgs<double>&, int64_t, double*, double*, hipStream_t);

}  // namespace rsk
