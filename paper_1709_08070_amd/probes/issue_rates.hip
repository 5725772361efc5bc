// Sustained VALU issue rates of single-instruction streams on one GPU: the yardstick against
// which the pair kernels' executed instruction counts are read.
//
// Each stream kernel runs 8 independent dependency chains per lane for kIters iterations with
// every wave resident from the start (256·W blocks of 4 waves: W waves per SIMD on 256 CUs),
// timed with events; the FP32 streams take their operands from vector registers except the
// ones named "sgpr", which read a kernel argument (a scalar register). The shader clock during
// each stream is read from the wave's cycle counter against the constant 100 MHz counter.
// Output: wave instructions per second, lane operations per second, and cycles per wave
// instruction per SIMD at the measured clock.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kIters = 16384;
constexpr int kChains = 8;

enum Op { kFmac, kFmaVop3, kMul, kAdd, kFmacSgpr, kExp, kRsq, kFma64 };

template <int OP>
__global__ void __launch_bounds__(256) k_stream(double* out, long long* clk, float b) {
  float a[kChains], x[kChains];
  double d[kChains];
  for (int i = 0; i < kChains; ++i) {
    a[i] = threadIdx.x * 1e-4f + i * 1e-2f + 0.5f;
    x[i] = 0.25f + 1e-3f * i + threadIdx.x * 1e-6f;
    d[i] = a[i];
  }
  const long long c0 = clock64(), r0 = wall_clock64();
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
      if (OP == kFmac) a[i] = __fmaf_rn(x[i], x[(i + 1) % kChains], a[i]);
      if (OP == kFmaVop3) a[i] = __fmaf_rn(a[i], x[i], x[(i + 1) % kChains]);
      if (OP == kMul) a[i] = a[i] * x[i];
      if (OP == kAdd) a[i] = a[i] + x[i];
      if (OP == kFmacSgpr) a[i] = __fmaf_rn(b, x[i], a[i]);
      if (OP == kExp) a[i] = __builtin_amdgcn_exp2f(a[i]);
      if (OP == kRsq) a[i] = __builtin_amdgcn_rsqf(a[i]);
      if (OP == kFma64) d[i] = fma(d[i], (double)x[i], (double)x[(i + 1) % kChains]);
    }
  }
  const long long c1 = clock64(), r1 = wall_clock64();
  double s = 0.0;
  for (int i = 0; i < kChains; ++i) s += (double)a[i] + d[i];
  const int g = blockIdx.x * 256 + threadIdx.x;
  out[g] = s;
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = c1 - c0;
    clk[2 * blockIdx.x + 1] = r1 - r0;
  }
}

#define CK(x)                                                                           \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                                     \
    }                                                                                   \
  } while (0)

template <int OP>
void run(const char* name, int lane_ops_per_inst, int W, double* out, long long* clk, int wall_mhz) {
  const int blocks = 256 * W;
  hipEvent_t t0, t1;
  CK(hipEventCreate(&t0));
  CK(hipEventCreate(&t1));
  k_stream<OP><<<blocks, 256>>>(out, clk, 1.0001f);  // warm-up
  CK(hipEventRecord(t0));
  k_stream<OP><<<blocks, 256>>>(out, clk, 1.0001f);
  CK(hipEventRecord(t1));
  CK(hipEventSynchronize(t1));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, t0, t1));
  long long* h = (long long*)std::malloc(sizeof(long long) * 2 * blocks);
  CK(hipMemcpy(h, clk, sizeof(long long) * 2 * blocks, hipMemcpyDeviceToHost));
  double cyc = 0.0, wall = 0.0;
  for (int i = 0; i < blocks; ++i) cyc += (double)h[2 * i], wall += (double)h[2 * i + 1];
  std::free(h);
  const double ghz = cyc / (wall / (wall_mhz * 1e-3)) ;  // cycles per ns
  const double winst = (double)blocks * 4 * kIters * kChains;
  const double rate = winst / (ms * 1e-3);
  std::printf("%-10s W=%d  %.3e wave-inst/s  %.1f T lane-ops/s  clock %.2f GHz  %.2f cycles per wave-inst per SIMD\n",
              name, W, rate, rate * 64 * lane_ops_per_inst / 1e12, ghz, 1024.0 * ghz * 1e9 / rate);
  CK(hipEventDestroy(t0));
  CK(hipEventDestroy(t1));
}

}  // namespace

int main() {
  const int wmax = 8;
  double* out;
  long long* clk;
  CK(hipMalloc(&out, sizeof(double) * 256 * wmax * 256));
  CK(hipMalloc(&clk, sizeof(long long) * 2 * 256 * wmax));
  int wall_khz = 0;
  CK(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, 0));
  const int wall_mhz = wall_khz / 1000;
  std::printf("streams of %d x %d independent instructions per lane; constant clock %d MHz\n", kIters, kChains,
              wall_mhz);
  for (int W : {4, 8}) {
    run<kFmac>("fmac_f32", 2, W, out, clk, wall_mhz);
    run<kFmaVop3>("fma_f32", 2, W, out, clk, wall_mhz);
    run<kMul>("mul_f32", 1, W, out, clk, wall_mhz);
    run<kAdd>("add_f32", 1, W, out, clk, wall_mhz);
    run<kFmacSgpr>("fmac_sgpr", 2, W, out, clk, wall_mhz);
    run<kExp>("exp_f32", 1, W, out, clk, wall_mhz);
    run<kRsq>("rsq_f32", 1, W, out, clk, wall_mhz);
    run<kFma64>("fma_f64", 2, W, out, clk, wall_mhz);
  }
  CK(hipFree(out));
  CK(hipFree(clk));
  return 0;
}
