// VALU issue-rate microbenchmark for gfx950: the per-instruction costs the RBE kernels'
// roofline uses.  Each kernel runs 16 independent streams per lane of one instruction
// (inline VALU asm with VGPR operands, so the compiler cannot rewrite it) on 8 waves per
// SIMD, long enough (several ms) for event timing.  It reports lane-ops per CU per clock
// at the 2.4 GHz peak clock and at the clock the waves themselves measured
// (s_memtime against the 100 MHz s_memrealtime over each wave's loop).
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

constexpr int kIter = 2048;
constexpr int kStreams = 16;
constexpr int kOps = 28;

// ops per stream step and their names
const char* kNames[kOps] = {"v_fma_f32", "v_fmac_f32", "v_add_f32", "v_mul_f32", "v_mul_lo_u32",
                            "v_add3_u32", "v_alignbit_b32", "v_cvt_f32_i32", "v_sin_f32", "v_cos_f32",
                            "v_fma_f64", "v_rndne_f64", "v_sin_f32 + 4 dependent v_fma_f32", "v_sin_f32 + 4 dependent v_mul_lo_u32",
                            "v_sin_f32 + v_cos_f32 + 2 x 4 dependent v_fma_f32", "v_mul_u32_u24", "v_mad_u32_u24",
                            "v_rndne_f32", "v_fract_f32", "v_cvt_f32_u32", "v_xad_u32",
                            "v_sin_f32 + 4 independent v_fma_f32", "4 v_mul_lo_u32 then 4 v_fma_f32",
                            "v_sin_f32 + 4 v_mul_lo_u32 + 4 v_fma_f32", "force term: sin cos 5 int 5 fma",
                            "rho term: sin cos 5 int 2 fma", "v_mad_u64_u32",
                            "rho term, mad_u64 phase: sin cos 4 int 2 fma"};
const int kInstr[kOps] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 5, 5, 10, 1, 1, 1, 1, 1, 1, 5, 8, 9, 12, 9, 1, 8};

template <int OP>
__global__ __launch_bounds__(256) void rate_kernel(float* out, unsigned long long* clk, int n_out) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  float x[kStreams], a = 1.0001f, b = 1e-4f;
  uint32_t y[kStreams], ia = 3, ib = 5;
  double z[kStreams], da = 1.0000001, db = 1e-7;
  for (int j = 0; j < kStreams; ++j) {
    x[j] = 1e-3f * (tid % 7 + j);
    y[j] = tid + j;
    z[j] = 1e-3 * (tid % 5 + j);
  }
  const unsigned long long t0 = __builtin_readcyclecounter();
  const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
  for (int it = 0; it < kIter; ++it) {
#pragma unroll
    for (int j = 0; j < kStreams; ++j) {
      if (OP == 0) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(x[j]) : "v"(a), "v"(b));
      if (OP == 1) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(x[j]) : "v"(a), "v"(b));
      if (OP == 2) asm volatile("v_add_f32 %0, %0, %1" : "+v"(x[j]) : "v"(b));
      if (OP == 3) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x[j]) : "v"(a));
      if (OP == 4) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(y[j]) : "v"(ia));
      if (OP == 5) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(y[j]) : "v"(ia), "v"(ib));
      if (OP == 6) asm volatile("v_alignbit_b32 %0, %1, %0, 9" : "+v"(y[j]) : "v"(ib));
      if (OP == 7) asm volatile("v_cvt_f32_i32 %0, %1" : "=v"(x[j]) : "v"(y[j]));
      if (OP == 8) asm volatile("v_sin_f32 %0, %0" : "+v"(x[j]));
      if (OP == 9) asm volatile("v_cos_f32 %0, %0" : "+v"(x[j]));
      if (OP == 10) asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(z[j]) : "v"(da), "v"(db));
      if (OP == 11) asm volatile("v_rndne_f64 %0, %0" : "+v"(z[j]));
      if (OP == 12) {
        asm volatile("v_sin_f32 %0, %0" : "+v"(x[j]));
        asm volatile("v_fma_f32 %0, %0, %1, %2\n v_fma_f32 %0, %0, %1, %2\n v_fma_f32 %0, %0, %1, %2\n v_fma_f32 %0, %0, %1, %2"
                     : "+v"(x[(j + 8) % kStreams]) : "v"(a), "v"(b));
      }
      if (OP == 13) {
        asm volatile("v_sin_f32 %0, %0" : "+v"(x[j]));
        asm volatile("v_mul_lo_u32 %0, %0, %1\n v_mul_lo_u32 %0, %0, %1\n v_mul_lo_u32 %0, %0, %1\n v_mul_lo_u32 %0, %0, %1"
                     : "+v"(y[j]) : "v"(ia));
      }
      if (OP == 15) asm volatile("v_mul_u32_u24 %0, %0, %1" : "+v"(y[j]) : "v"(ia));
      if (OP == 16) asm volatile("v_mad_u32_u24 %0, %0, %1, %2" : "+v"(y[j]) : "v"(ia), "v"(ib));
      if (OP == 17) asm volatile("v_rndne_f32 %0, %0" : "+v"(x[j]));
      if (OP == 18) asm volatile("v_fract_f32 %0, %0" : "+v"(x[j]));
      if (OP == 19) asm volatile("v_cvt_f32_u32 %0, %1" : "=v"(x[j]) : "v"(y[j]));
      if (OP == 20) asm volatile("v_xad_u32 %0, %0, %1, %2" : "+v"(y[j]) : "v"(ia), "v"(ib));
      // mixes with independent FP32 operands: f[] streams 4 apart, so no FMA waits on another
      float& f0 = x[(j + 4) % kStreams];
      float& f1 = x[(j + 8) % kStreams];
      float& f2 = x[(j + 12) % kStreams];
      float& f3 = x[(j + 2) % kStreams];
      float& f4 = x[(j + 6) % kStreams];
      uint32_t& y0 = y[j];
      uint32_t& y1 = y[(j + 4) % kStreams];
      uint32_t& y2 = y[(j + 8) % kStreams];
      uint32_t& y3 = y[(j + 12) % kStreams];
      if (OP == 21) {
        asm volatile("v_sin_f32 %0, %0" : "+v"(x[j]));
        asm volatile("v_fma_f32 %0, %0, %4, %5\n v_fma_f32 %1, %1, %4, %5\n v_fma_f32 %2, %2, %4, %5\n v_fma_f32 %3, %3, %4, %5"
                     : "+v"(f0), "+v"(f1), "+v"(f2), "+v"(f3) : "v"(a), "v"(b));
      }
      if (OP == 22) {
        asm volatile("v_mul_lo_u32 %0, %0, %4\n v_mul_lo_u32 %1, %1, %4\n v_mul_lo_u32 %2, %2, %4\n v_mul_lo_u32 %3, %3, %4"
                     : "+v"(y0), "+v"(y1), "+v"(y2), "+v"(y3) : "v"(ia));
        asm volatile("v_fma_f32 %0, %0, %4, %5\n v_fma_f32 %1, %1, %4, %5\n v_fma_f32 %2, %2, %4, %5\n v_fma_f32 %3, %3, %4, %5"
                     : "+v"(f0), "+v"(f1), "+v"(f2), "+v"(f3) : "v"(a), "v"(b));
      }
      if (OP == 23) {
        asm volatile("v_sin_f32 %0, %0" : "+v"(x[j]));
        asm volatile("v_mul_lo_u32 %0, %0, %4\n v_mul_lo_u32 %1, %1, %4\n v_mul_lo_u32 %2, %2, %4\n v_mul_lo_u32 %3, %3, %4"
                     : "+v"(y0), "+v"(y1), "+v"(y2), "+v"(y3) : "v"(ia));
        asm volatile("v_fma_f32 %0, %0, %4, %5\n v_fma_f32 %1, %1, %4, %5\n v_fma_f32 %2, %2, %4, %5\n v_fma_f32 %3, %3, %4, %5"
                     : "+v"(f0), "+v"(f1), "+v"(f2), "+v"(f3) : "v"(a), "v"(b));
      }
      if (OP == 24 || OP == 25) {
        // one (particle, wave vector) term: phase (3 mul_lo, add3, alignbit), sin, cos, then
        // the force pass's 5 FP32 ops or the rho pass's 2
        asm volatile("v_sin_f32 %0, %0" : "+v"(x[j]));
        asm volatile("v_cos_f32 %0, %0" : "+v"(x[(j + 1) % kStreams]));
        asm volatile("v_mul_lo_u32 %0, %0, %4\n v_mul_lo_u32 %1, %1, %4\n v_mul_lo_u32 %2, %2, %4\n v_add3_u32 %3, %3, %4, %5\n v_alignbit_b32 %0, %5, %0, 9"
                     : "+v"(y0), "+v"(y1), "+v"(y2), "+v"(y3) : "v"(ia), "v"(ib));
        if (OP == 24)
          asm volatile("v_fma_f32 %0, %0, %5, %6\n v_fma_f32 %1, %1, %5, %6\n v_fma_f32 %2, %2, %5, %6\n v_fma_f32 %3, %3, %5, %6\n v_fma_f32 %4, %4, %5, %6"
                       : "+v"(f0), "+v"(f1), "+v"(f2), "+v"(f3), "+v"(f4) : "v"(a), "v"(b));
        else
          asm volatile("v_fma_f32 %0, %0, %2, %3\n v_fma_f32 %1, %1, %2, %3" : "+v"(f0), "+v"(f1) : "v"(a), "v"(b));
      }
      if (OP == 26) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(z[j]) : "v"(ia), "v"(ib) : "vcc");
      if (OP == 27) {
        // the rho term with the phase as mul_lo and two 64-bit-accumulating multiply-adds
        // (the low word of a u32 x u32 + u64 product is the phase mod 2^32)
        asm volatile("v_sin_f32 %0, %0" : "+v"(x[j]));
        asm volatile("v_cos_f32 %0, %0" : "+v"(x[(j + 1) % kStreams]));
        asm volatile("v_mul_lo_u32 %0, %0, %3\n v_mad_u64_u32 %1, vcc, %3, %4, %1\n v_mad_u64_u32 %2, vcc, %3, %4, %2\n v_alignbit_b32 %0, %4, %0, 9"
                     : "+v"(y0), "+v"(z[j]), "+v"(z[(j + 8) % kStreams]) : "v"(ia), "v"(ib) : "vcc");
        asm volatile("v_fma_f32 %0, %0, %2, %3\n v_fma_f32 %1, %1, %2, %3" : "+v"(f0), "+v"(f1) : "v"(a), "v"(b));
      }
      if (OP == 14) {
        asm volatile("v_sin_f32 %0, %0" : "+v"(x[j]));
        asm volatile("v_cos_f32 %0, %0" : "+v"(x[(j + 4) % kStreams]));
        asm volatile("v_fma_f32 %0, %0, %1, %2\n v_fma_f32 %0, %0, %1, %2\n v_fma_f32 %0, %0, %1, %2\n v_fma_f32 %0, %0, %1, %2"
                     : "+v"(x[(j + 8) % kStreams]) : "v"(a), "v"(b));
        asm volatile("v_fma_f32 %0, %0, %1, %2\n v_fma_f32 %0, %0, %1, %2\n v_fma_f32 %0, %0, %1, %2\n v_fma_f32 %0, %0, %1, %2"
                     : "+v"(x[(j + 12) % kStreams]) : "v"(a), "v"(b));
      }
    }
  }
  const unsigned long long t1 = __builtin_readcyclecounter();
  const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
  float sx = 0;
  uint32_t sy = 0;
  double sz = 0;
  for (int j = 0; j < kStreams; ++j) {
    sx += x[j];
    sy += y[j];
    sz += z[j];
  }
  if ((sx == 1234.5f || sy == 123457u || sz == 1234.5) && tid < n_out) out[tid] = sx;
  // one (cycles, realtime ticks) pair per wave
  const int wave = tid >> 6;
  if ((threadIdx.x & 63) == 0 && 2 * wave + 1 < n_out) {
    clk[2 * wave] = t1 - t0;
    clk[2 * wave + 1] = r1 - r0;
  }
}

template <int OP>
void time_op(int blocks, int lds, float* f, unsigned long long* clk, int n_out, unsigned long long* h, float* ms,
             double* ghz) {
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(256), lds, 0, f, clk, n_out);
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0));
  for (int r = 0; r < 3; ++r) hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(256), lds, 0, f, clk, n_out);
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  CHECK(hipEventElapsedTime(ms, e0, e1));
  *ms /= 3;
  const int waves = blocks * 4;
  CHECK(hipMemcpy(h, clk, sizeof(unsigned long long) * 2 * waves, hipMemcpyDeviceToHost));
  double c = 0, r = 0;
  for (int i = 0; i < waves; ++i) {
    c += (double)h[2 * i];
    r += (double)h[2 * i + 1];
  }
  *ghz = c / (r * 10.0);   // cycles per 10 ns tick of the 100 MHz real-time counter
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
}

int main() {
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  const int cus = prop.multiProcessorCount;
  std::printf("device %s, %d CUs, %d kHz\n", prop.gcnArchName, cus, prop.clockRate);
  const int wps = 8;                       // waves per SIMD
  const int blocks = cus * wps;            // 256-thread blocks: one wave per SIMD each
  const int lds = 160 * 1024 / wps - 1024; // caps the blocks per CU at wps
  const int n_out = blocks * 256;
  float* f;
  unsigned long long* clk;
  CHECK(hipMalloc(&f, sizeof(float) * (size_t)n_out));
  CHECK(hipMalloc(&clk, sizeof(unsigned long long) * (size_t)n_out));
  unsigned long long* h = (unsigned long long*)std::malloc(sizeof(unsigned long long) * (size_t)n_out);
  float ms[kOps];
  double ghz[kOps];
  time_op<0>(blocks, lds, f, clk, n_out, h, &ms[0], &ghz[0]);
  time_op<1>(blocks, lds, f, clk, n_out, h, &ms[1], &ghz[1]);
  time_op<2>(blocks, lds, f, clk, n_out, h, &ms[2], &ghz[2]);
  time_op<3>(blocks, lds, f, clk, n_out, h, &ms[3], &ghz[3]);
  time_op<4>(blocks, lds, f, clk, n_out, h, &ms[4], &ghz[4]);
  time_op<5>(blocks, lds, f, clk, n_out, h, &ms[5], &ghz[5]);
  time_op<6>(blocks, lds, f, clk, n_out, h, &ms[6], &ghz[6]);
  time_op<7>(blocks, lds, f, clk, n_out, h, &ms[7], &ghz[7]);
  time_op<8>(blocks, lds, f, clk, n_out, h, &ms[8], &ghz[8]);
  time_op<9>(blocks, lds, f, clk, n_out, h, &ms[9], &ghz[9]);
  time_op<10>(blocks, lds, f, clk, n_out, h, &ms[10], &ghz[10]);
  time_op<11>(blocks, lds, f, clk, n_out, h, &ms[11], &ghz[11]);
  time_op<12>(blocks, lds, f, clk, n_out, h, &ms[12], &ghz[12]);
  time_op<13>(blocks, lds, f, clk, n_out, h, &ms[13], &ghz[13]);
  time_op<14>(blocks, lds, f, clk, n_out, h, &ms[14], &ghz[14]);
  time_op<15>(blocks, lds, f, clk, n_out, h, &ms[15], &ghz[15]);
  time_op<16>(blocks, lds, f, clk, n_out, h, &ms[16], &ghz[16]);
  time_op<17>(blocks, lds, f, clk, n_out, h, &ms[17], &ghz[17]);
  time_op<18>(blocks, lds, f, clk, n_out, h, &ms[18], &ghz[18]);
  time_op<19>(blocks, lds, f, clk, n_out, h, &ms[19], &ghz[19]);
  time_op<20>(blocks, lds, f, clk, n_out, h, &ms[20], &ghz[20]);
  time_op<21>(blocks, lds, f, clk, n_out, h, &ms[21], &ghz[21]);
  time_op<22>(blocks, lds, f, clk, n_out, h, &ms[22], &ghz[22]);
  time_op<23>(blocks, lds, f, clk, n_out, h, &ms[23], &ghz[23]);
  time_op<24>(blocks, lds, f, clk, n_out, h, &ms[24], &ghz[24]);
  time_op<25>(blocks, lds, f, clk, n_out, h, &ms[25], &ghz[25]);
  time_op<26>(blocks, lds, f, clk, n_out, h, &ms[26], &ghz[26]);
  time_op<27>(blocks, lds, f, clk, n_out, h, &ms[27], &ghz[27]);
  std::printf("%d waves per SIMD, %d independent streams per lane, %d steps\n", wps, kStreams, kIter);
  std::printf("%-36s %8s %8s %14s %14s %12s\n", "instruction (per step)", "ms", "GHz", "ops/CU/clk@2.4", "ops/CU/clk@own",
              "cyc/wave64");
  for (int k = 0; k < kOps; ++k) {
    const double ops = (double)n_out * kIter * kStreams * kInstr[k];
    const double per_cu_clk_peak = ops / (ms[k] * 1e-3) / cus / 2.4e9;
    const double per_cu_clk_own = ops / (ms[k] * 1e-3) / cus / (ghz[k] * 1e9);
    std::printf("%-36s %8.3f %8.3f %14.1f %14.1f %12.2f\n", kNames[k], ms[k], ghz[k], per_cu_clk_peak, per_cu_clk_own,
                4.0 * 64.0 / per_cu_clk_own);
  }
  std::free(h);
  CHECK(hipFree(f));
  CHECK(hipFree(clk));
  return 0;
}
