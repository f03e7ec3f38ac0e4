// VALU issue-rate microbenchmark for gfx950: the rates the RBE kernels' roofline uses.
// Each kernel runs 8 independent dependency chains per lane of one instruction kind
// (inline VALU asm where the compiler would otherwise rewrite the operation) on 32 waves
// per CU, and reports lane-ops per second as a fraction of one op per lane per clock.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                         \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) {                                                              \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);        \
      std::exit(1);                                                                      \
    }                                                                                    \
  } while (0)

constexpr int kIter = 512;

template <int OP>
__global__ __launch_bounds__(256) void rate_kernel(float* outf, double* outd, int* outi, float a, float b, int ia,
                                                   int ib, double da, double db) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  float x[8];
  int y[8];
  double z[8];
  for (int j = 0; j < 8; ++j) {
    x[j] = 0.001f * (tid % 7 + j);
    y[j] = tid + j;
    z[j] = 0.001 * (tid % 5 + j);
  }
  for (int it = 0; it < kIter; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (OP == 0) x[j] = __builtin_amdgcn_sinf(x[j]);
      if (OP == 1) x[j] = __builtin_amdgcn_cosf(x[j]);
      if (OP == 2) x[j] = fmaf(x[j], a, b);
      if (OP == 3) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(y[j]) : "v"(ia));
      if (OP == 4) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(y[j]) : "v"(ia), "v"(ib));
      if (OP == 5) asm volatile("v_alignbit_b32 %0, %1, %0, 9" : "+v"(y[j]) : "v"(ib));
      if (OP == 6) z[j] = fma(z[j], da, db);
      if (OP == 7) asm volatile("v_rndne_f64 %0, %0" : "+v"(z[j]));
      if (OP == 8) {   // one sin next to four full-rate integer ops: co-issue check
        x[j] = __builtin_amdgcn_sinf(x[j]);
        asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(y[j]) : "v"(ia));
        asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(y[j]) : "v"(ib));
        asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(y[j]) : "v"(ia));
        asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(y[j]) : "v"(ib));
      }
    }
  }
  float sx = 0;
  int sy = 0;
  double sz = 0;
  for (int j = 0; j < 8; ++j) {
    sx += x[j];
    sy += y[j];
    sz += z[j];
  }
  if (sx == 1234.5f) outf[tid] = sx;
  if (sy == 123457) outi[tid] = sy;
  if (sz == 1234.5) outd[tid] = sz;
}

template <int OP>
float time_op(int blocks, float* f, double* d, int* i) {
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(256), 0, 0, f, d, i, 1.0001f, 0.0001f, 3, 5, 1.0000001, 1e-7);
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0));
  for (int r = 0; r < 5; ++r)
    hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(256), 0, 0, f, d, i, 1.0001f, 0.0001f, 3, 5, 1.0000001, 1e-7);
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
  return ms / 5;
}

int main() {
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  std::printf("device %s, %d CUs, %d kHz\n", prop.gcnArchName, prop.multiProcessorCount, prop.clockRate);
  const int blocks = prop.multiProcessorCount * 32;
  const size_t nt = (size_t)blocks * 256;
  float* f;
  double* d;
  int* ii;
  CHECK(hipMalloc(&f, nt * 4));
  CHECK(hipMalloc(&d, nt * 8));
  CHECK(hipMalloc(&ii, nt * 4));
  const double lane_iters = (double)nt * kIter * 8;
  const double peak = (double)prop.multiProcessorCount * 64 * (prop.clockRate * 1e3);
  const char* names[] = {"v_sin_f32", "v_cos_f32", "v_fma_f32", "v_mul_lo_u32", "v_add3_u32",
                         "v_alignbit_b32", "v_fma_f64", "v_rndne_f64", "v_sin_f32 + 4 v_mul_lo_u32"};
  float t[9];
  t[0] = time_op<0>(blocks, f, d, ii);
  t[1] = time_op<1>(blocks, f, d, ii);
  t[2] = time_op<2>(blocks, f, d, ii);
  t[3] = time_op<3>(blocks, f, d, ii);
  t[4] = time_op<4>(blocks, f, d, ii);
  t[5] = time_op<5>(blocks, f, d, ii);
  t[6] = time_op<6>(blocks, f, d, ii);
  t[7] = time_op<7>(blocks, f, d, ii);
  t[8] = time_op<8>(blocks, f, d, ii);
  std::printf("%-28s %10s %16s %12s\n", "instruction", "ms", "lane-iters/s", "of 1/lane/clk");
  for (int k = 0; k < 9; ++k)
    std::printf("%-28s %10.3f %16.4e %12.3f\n", names[k], t[k], lane_iters / (t[k] * 1e-3),
                lane_iters / (t[k] * 1e-3) / peak);
  CHECK(hipFree(f));
  CHECK(hipFree(d));
  CHECK(hipFree(ii));
  return 0;
}
