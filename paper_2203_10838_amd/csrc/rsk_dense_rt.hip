// Dense RSKA, float32, register-tile persistent kernel for one system: the step body is
// rt_run (rsk_dense_rt.hpp); each workgroup is one column slice (and row group).
#include "rsk_dense_rt.hpp"

namespace rsk {

template <int NT, int RP, int CPL, int RG>
__global__ __launch_bounds__(NT) void rska_dense_rt(DenseArgs<float> a) {
  rt_run<NT, RP, CPL, RG, false>(a, blockIdx.x, CPL);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <int NT, int RP, int CPL, int RG>
static void* rt_ptr() {
  return reinterpret_cast<void*>(&rska_dense_rt<NT, RP, CPL, RG>);
}

// 1024 threads for eta <= 768 (RP <= 3), 512 threads (256 VGPRs a lane) for 768 < eta <= 1024.
static void* rt_kernel(int nt, int rp, int cpl, int rg) {
#define RT_CASE(N, R, C, H) if (nt == N && rp == R && cpl == C && rg == H) return rt_ptr<N, R, C, H>();
#define RT_CPL(N, R, H) RT_CASE(N, R, 1, H) RT_CASE(N, R, 2, H) RT_CASE(N, R, 3, H) RT_CASE(N, R, 4, H) RT_CASE(N, R, 5, H)
  RT_CPL(1024, 1, 1) RT_CPL(1024, 2, 1) RT_CPL(1024, 3, 1)
  RT_CPL(512, 7, 1) RT_CPL(512, 8, 1)
  RT_CPL(1024, 1, 2) RT_CPL(1024, 2, 2) RT_CPL(1024, 3, 2)
  RT_CPL(512, 7, 2) RT_CPL(512, 8, 2)
#undef RT_CPL
#undef RT_CASE
  return nullptr;
}

int dense_rt_max_grid(int nt, int rp, int cpl, int rg) {
  void* fn = rt_kernel(nt, rp, cpl, rg);
  if (!fn) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nt, 0) != hipSuccess) return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

hipError_t launch_dense_rt(DenseArgs<float>& a, int nt, int rp, int cpl, int rg, hipStream_t stream) {
  void* fn = rt_kernel(nt, rp, cpl, rg);
  if (!fn) return hipErrorInvalidValue;
  if (a.G % rg != 0 || (rg > 1 && !a.xU)) return hipErrorInvalidValue;
  if (a.G > kMaxG || dense_rt_max_grid(nt, rp, cpl, rg) < a.G) return hipErrorCooperativeLaunchTooLarge;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(fn, dim3(a.G), dim3(nt), args, 0, stream);
}

}  // namespace rsk
