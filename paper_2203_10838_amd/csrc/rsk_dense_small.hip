// Dense RSKA for small systems: one workgroup runs the whole iteration (eq. (rska), Algorithm 1)
// with no exchange between workgroups.
//
// Thread tid owns the columns tid + 256 c, c < CPT (n <= 256 CPT), and keeps their x* and x in
// registers; the step's row tile (eta rows of the thread's columns) is in registers too. A step:
//   1. partial dots of the eta rows over the own columns, summed over each wave's lanes, then over
//      the four waves in a fixed order by thread t (row t): r_t = <a_tau_t, x_k>;
//   2. c_t = (alpha_k/eta)(r_t - b_tau_t)/||a_tau_t||^2, shared through LDS;
//   3. x*_j -= sum_t c_t A[tau_t, j] over t ascending for the own columns, x_j = S_lambda(x*_j).
// Two barriers a step. The rows, b and ||a||^2 of the step after next are loaded during a step (the
// index stream three steps ahead), so a step waits for no memory round trip once the pipeline is full:
// the path for the latency-bound small systems of the paper's experiments (Sec. 5), where a
// multi-workgroup exchange costs more than the step's arithmetic.
//
// Limits: n <= 2048 (CPT = 1, 2, 4, 8) and eta <= 32 / CPT rows a step (the tiles of three steps stay
// in registers; the indices of the next three steps wait in LDS). Any leading dimension and alignment (one element a
// load, consecutive threads on consecutive columns). Summation orders are fixed: x*, x and y are
// bitwise reproducible.
#include "rsk_device.hpp"
#include "rsk_kernels.hpp"

namespace rsk {

namespace {

constexpr int kSmallThreads = 256;
constexpr int kSmallWaves = kSmallThreads / 64;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sums of N values over the 64 lanes of a wave, every lane getting every sum: within each DPP row
// of 16 lanes by rotations of 8, 4, 2, 1, then across rows by xor 16 and 32. One level for all N
// values before the next, so their latencies overlap. A fixed order: the same bits on every run.
template <typename T, int N>
__device__ __forceinline__ void lane_rows_sum(T (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x128>(v[i]);  // row_ror:8
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x124>(v[i]);  // row_ror:4
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x122>(v[i]);  // row_ror:2
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x121>(v[i]);  // row_ror:1
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], 16);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], 32);
}

template <int CPT>
struct SmallShape {
  static constexpr int emax = 32 / CPT;  // rows a step: the tile is at most 32 elements a thread
};

}  // namespace

template <typename T, int CPT>
__global__ __launch_bounds__(kSmallThreads) void rska_dense_small(DenseArgs<T> a) {
  constexpr int EMAX = SmallShape<CPT>::emax;
  __shared__ T part[kSmallWaves][EMAX];
  __shared__ T cs[EMAX];
  __shared__ int rows_sh[3][EMAX];  // indices of step q in slot q % 3 (steps k + 1 .. k + 3)
  __shared__ int badw[3];           // an index of that step is out of range
  __shared__ int rows_y[EMAX];
  __shared__ double mon[kSmallWaves][2];
  __shared__ double err_sh;
  __shared__ int flags[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int eta = a.eta;
  const int64_t K = a.K;

  int64_t col[CPT];
  bool cok[CPT];
  T z[CPT], xv[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    col[c] = tid + (int64_t)kSmallThreads * c;
    cok[c] = col[c] < a.n;
    z[c] = (a.warm && cok[c]) ? a.x_star[col[c]] : T(0);
    xv[c] = shrink(z[c], a.lambda);
  }

  // Every load below is issued unconditionally (addresses clamped into range, unused values
  // discarded later) and nothing branches on a loaded value before it is needed: the memory
  // counter then counts the same loads on every path, and each wait is for one step's loads only.
  //
  // Thread t < eta loads index t of step q; checked when it is stored to LDS (slot q % 3), where an
  // out-of-range index becomes row 0 and flags the step.
  const int tix = tid < eta ? tid : 0;
  auto fetch_index = [&](int64_t q) -> int { return a.idx[(q < K ? q : K - 1) * (int64_t)eta + tix]; };
  auto store_index = [&](int64_t q, int i) {
    if (q < K && tid < eta) {
      const bool bad = i < 0 || (int64_t)i >= a.m;
      rows_sh[q % 3][tid] = bad ? 0 : i;
      if (bad) atomicOr(&badw[q % 3], 1);
    }
  };
  // The tile of a step from its indices in LDS (rows past eta read row 0 and columns past n column
  // 0: they meet c = 0 and x = 0) and, for thread t < eta, b, ||a||^2 and the weight of row t
  // (combined where they are used).
  const T* wsrc = a.row_w ? a.row_w : a.r2;
  auto load_tile = [&](const int* rows, T (&tl)[EMAX][CPT], T& bt, T& rnt, T& wt) {
#pragma unroll
    for (int t = 0; t < EMAX; ++t) {
      const T* rp = a.A + (int64_t)(t < eta ? rows[t] : 0) * a.ld;
#pragma unroll
      for (int c = 0; c < CPT; ++c) tl[t][c] = rp[cok[c] ? col[c] : 0];
    }
    const int r = rows[tix];
    bt = a.b[r];
    rnt = a.r2[r];
    wt = wsrc[r];
  };

  // Three tiles in registers: a step runs on one while the next two load, so each tile's loads have
  // two steps to land.
  T t0[EMAX][CPT], t1[EMAX][CPT], t2[EMAX][CPT];
  T b0 = T(0), b1 = T(0), b2 = T(0), n0 = T(1), n1 = T(1), n2 = T(1), w0 = T(1), w1 = T(1), w2 = T(1);
#pragma unroll
  for (int t = 0; t < EMAX; ++t)
#pragma unroll
    for (int c = 0; c < CPT; ++c) t0[t][c] = t1[t][c] = t2[t][c] = T(0);

  int64_t k_done = 0;
  int stop_code = 0;
  int64_t kend = K;  // the first step whose indices are out of range, else K
  bool converged = false, zero_row = false;
  if (tid < 3) badw[tid] = 0;
  if (tid < 2) flags[tid] = 0;
  __syncthreads();
  if (K > 0) {
    for (int q = 0; q < 3; ++q) store_index(q, fetch_index(q));
    __syncthreads();
    if (badw[0]) kend = 0;
    else if (K > 1 && badw[1]) kend = 1;
    // rows_sh slots of steps past K hold no indices yet: row 0 stands in
    if (tid < EMAX) {
      if (K < 2) rows_sh[1][tid] = 0;
      if (K < 3) rows_sh[2][tid] = 0;
    }
    __syncthreads();
    load_tile(rows_sh[0], t0, b0, n0, w0);
    load_tile(rows_sh[1], t1, b1, n1, w1);
  }

  // One step k on tile `cur` (b, ||a||^2, w of row tid in cb, cn, cw); the tile of step k + 2 loads
  // into `fill` (with fb, fn, fw). Returns false when the run stops.
  auto step = [&](int64_t k, T (&cur)[EMAX][CPT], T cb, T cn, T cw, T (&fill)[EMAX][CPT], T& fb, T& fn,
                  T& fw) -> bool {
    const T akv = (a.alpha_k ? a.alpha_k : a.b)[a.alpha_k ? k : 0];
    const int i3 = fetch_index(k + 3);
    __builtin_amdgcn_sched_barrier(0);  // these two stay older than the tile loads
    const int par = (int)(k & 1);
    const int s0 = (int)(k % 3), s2 = (int)((k + 2) % 3);
    // the tile of step k + 2 (slots of steps past K or past a bad index hold in-range rows)
    if (k + 2 < kend && badw[s2]) kend = k + 2;  // uniform: every thread read the same word
    load_tile(rows_sh[s2], fill, fb, fn, fw);
    if (tid == 0) badw[s0] = 0;  // its last reader was step k - 2, before that step's first barrier

    // partial dots over the own columns, summed over the wave level by level across the rows, so
    // that the rows' exchange latencies overlap (rows past eta are summed too and never read)
    T p[EMAX];
#pragma unroll
    for (int t = 0; t < EMAX; ++t) {
      p[t] = T(0);
#pragma unroll
      for (int c = 0; c < CPT; ++c) p[t] += cur[t][c] * xv[c];
    }
    lane_rows_sum<T, EMAX>(p);
    if (lane == 0)
#pragma unroll
      for (int t = 0; t < EMAX; ++t) part[wave][t] = p[t];
    __syncthreads();
    store_index(k + 3, i3);
    int flag = 0;
    if (tid < eta) {
      T r = T(0);
#pragma unroll
      for (int w = 0; w < kSmallWaves; ++w) r += part[w][tid];
      T c;
      if (cn == T(0)) {
        c = T(NAN);
        flag |= 8;  // a referenced zero row (reported after the loop: no global store in a step)
      } else {
        // ||a||^2 / w: the row's weight folded into its norm (w = 0: no update from the row)
        const T rn = a.row_w ? cn / cw : cn;
        const T ak = a.alpha_k ? akv : a.alpha;
        c = (ak / (T)eta) * (r - cb) / rn;
      }
      if (!isfinite(c)) flag |= 2;
      cs[tid] = c;
    }
    if (flag) atomicOr(&flags[par], flag);
    __syncthreads();
    const int fl = flags[par];
    if (tid == 0) flags[par ^ 1] = 0;
    if (fl & 2) {
      if (fl & 8) zero_row = true;
      stop_code = ST_NONFINITE;
      return false;
    }

    // transposed update of the own columns, t ascending, and S_lambda
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      T d = T(0);
#pragma unroll
      for (int t = 0; t < EMAX; ++t)
        if (t < eta) d += cs[t] * cur[t][c];
      // a column past n keeps x* = x = 0, so the copies of column 0 its tile holds add nothing
      if (cok[c]) {
        z[c] -= d;
        xv[c] = shrink(z[c], a.lambda);
      }
    }
    if (a.y) {
      // y_i -= c_t for every slot t of row i, in ascending t, applied by the row's first slot
      if (tid < eta) rows_y[tid] = a.idx[k * (int64_t)eta + tid];
      __syncthreads();
      if (tid < eta) {
        const int i = rows_y[tid];
        bool first = true;
        for (int t = 0; t < tid; ++t) first = first && rows_y[t] != i;
        if (first) {
          T v = a.y[i];
          for (int t = tid; t < eta; ++t)
            if (rows_y[t] == i) v -= cs[t];
          a.y[i] = v;
        }
      }
      __builtin_amdgcn_s_waitcnt(0);  // the stores are done here, so no later wait of the step counts them
      __syncthreads();
    }
    k_done = k + 1;

    if (a.xref && a.check_every > 0 && (k + 1) % a.check_every == 0) {
      double e2 = 0.0, r2s = 0.0;
#pragma unroll
      for (int c = 0; c < CPT; ++c)
        if (cok[c]) {
          const double rf = (double)a.xref[col[c]];
          const double d = (double)xv[c] - rf;
          e2 += d * d;
          r2s += rf * rf;
        }
      e2 = wave_sum(e2);
      r2s = wave_sum(r2s);
      if (lane == 0) { mon[wave][0] = e2; mon[wave][1] = r2s; }
      __syncthreads();
      if (tid == 0) {
        double se = 0.0, sr = 0.0;
        for (int w = 0; w < kSmallWaves; ++w) { se += mon[w][0]; sr += mon[w][1]; }
        const double err = sr > 0.0 ? sqrt(se / sr) : sqrt(se);
        if (a.err_hist) a.err_hist[(k + 1) / a.check_every - 1] = err;
        err_sh = err;
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (a.tol > 0.0 && err_sh <= a.tol) {
        converged = true;
        return false;
      }
    }
    return true;
  };

  for (int64_t k = 0; k < kend; k += 3) {
    if (!step(k, t0, b0, n0, w0, t2, b2, n2, w2) || k + 1 >= kend) break;
    if (!step(k + 1, t1, b1, n1, w1, t0, b0, n0, w0) || k + 2 >= kend) break;
    if (!step(k + 2, t2, b2, n2, w2, t1, b1, n1, w1)) break;
  }
  __builtin_amdgcn_s_waitcnt(0);  // no load of a step that will not run stays in flight
  if (!stop_code && !converged && k_done == kend && kend < K) stop_code = ST_INDEX;
  if (zero_row && tid == 0) set_status(a.status, ST_ZERO_ROW);
  if (stop_code && tid == 0) set_status(a.status, stop_code);
#pragma unroll
  for (int c = 0; c < CPT; ++c)
    if (cok[c]) { a.x_star[col[c]] = z[c]; a.x[col[c]] = xv[c]; }
  if (tid == 0) a.status[1] = (int)k_done;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int dense_small_cpt(int64_t n, int eta) {
  if (n <= 0 || eta < 1) return 0;
  const int64_t need = (n + kSmallThreads - 1) / kSmallThreads;
  const int cpt = need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 0;
  if (!cpt) return 0;
  return eta <= 32 / cpt ? cpt : 0;
}

template <typename T>
hipError_t launch_dense_small(DenseArgs<T>& a, hipStream_t stream) {
  const int cpt = dense_small_cpt(a.n, a.eta);
  const dim3 grid(1), block(kSmallThreads);
  switch (cpt) {
    case 1: hipLaunchKernelGGL((rska_dense_small<T, 1>), grid, block, 0, stream, a); break;
    case 2: hipLaunchKernelGGL((rska_dense_small<T, 2>), grid, block, 0, stream, a); break;
    case 4: hipLaunchKernelGGL((rska_dense_small<T, 4>), grid, block, 0, stream, a); break;
    case 8: hipLaunchKernelGGL((rska_dense_small<T, 8>), grid, block, 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_dense_small<float>(DenseArgs<float>&, hipStream_t);
template hipError_t launch_dense_small<double>(DenseArgs<double>&, hipStream_t);

}  // namespace rsk
