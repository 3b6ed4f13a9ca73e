// bench_valu_issue.hip -- measures the FP32 VALU issue rate of gfx950 that
// bench.py's roofline uses as its peak.
//
// Each kernel runs independent chains of FP32 VALU instructions and reports
// lane-instructions per second against the single-issue rate (CUs x 64 lanes
// x 2.4 GHz).  Kernels:
//   sgpr  adds whose second operand is a scalar register;
//   vgpr  adds on vector registers only;
//   cell  the DP cell of the sDTW kernels (t = a - r; c = t*t;
//         d = min3(d, x, y) + c), vector registers only, at 1, 2, 4 and 8
//         wavefronts per SIMD;
//   fma   fused multiply-adds on vector registers only;
//   code  the cell of the uint8-code forward (t = a - r;
//         d = fma(t, t, min3(d, x, y))), at 1, 2, 4 and 8 wavefronts per SIMD.
// Run under rocprofv3 with SQ_INSTS_VALU and SQ_ACTIVE_INST_VALU2 to see the
// share of instructions issued two per SIMD per quad-cycle.
#include <hip/hip_runtime.h>

#include <cstdio>

#define CHK(x)                                                                  \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                                 \
    }                                                                           \
  } while (0)

constexpr int kIters = 4096;
constexpr int kChains = 8;

// mode 0: add with an SGPR operand; 1: add, VGPRs only; 2: DP cell, VGPRs only;
// 3: fma, VGPRs only; 4: code cell (sub, min3, fma), VGPRs only
template <int MODE>
__global__ __launch_bounds__(256) void issue_kernel(float* out, const float* in, float s) {
  const int l = threadIdx.x & 31;
  float d[kChains], a[kChains], x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    d[c] = in[(l + c) & 31];
    a[c] = in[32 + ((l + 3 * c) & 31)];
    x[c] = in[64 + ((l + 5 * c) & 31)];
  }
  float r = in[96 + l], y = in[128 + l];
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (MODE == 0) {
        d[c] = d[c] + s;
      } else if constexpr (MODE == 1) {
        d[c] = d[c] + a[c];
      } else if constexpr (MODE == 3) {
        d[c] = __builtin_fmaf(a[c], x[c], d[c]);
      } else if constexpr (MODE == 4) {
        const float t = a[c] - r;
        d[c] = __builtin_fmaf(t, t, __builtin_fminf(__builtin_fminf(d[c], x[c]), y));
      } else {
        const float t = a[c] - r;
        const float cc = t * t;
        d[c] = __builtin_fminf(__builtin_fminf(d[c], x[c]), y) + cc;
      }
    }
    if constexpr (MODE == 2 || MODE == 4) r = r + y;
  }
  float acc = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc += d[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

template <int MODE>
int run(const char* name, int cus, int waves_per_simd, float* out, const float* in) {
  hipEvent_t a, b;
  CHK(hipEventCreate(&a));
  CHK(hipEventCreate(&b));
  const int blocks = cus * waves_per_simd;     // 256 threads: one wave per SIMD
  float best = 1e30f;
  for (int rep = 0; rep < 3; ++rep) {
    CHK(hipEventRecord(a));
    hipLaunchKernelGGL(issue_kernel<MODE>, dim3(blocks), dim3(256), 0, 0, out, in, 1.0001f);
    CHK(hipGetLastError());
    CHK(hipEventRecord(b));
    CHK(hipEventSynchronize(b));
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, a, b));
    if (ms < best) best = ms;
  }
  const double per_iter = MODE == 2 ? kChains * 4 + 1 : (MODE == 4 ? kChains * 3 + 1 : kChains);
  const double ops = (double)blocks * 256 * kIters * per_iter;
  const double rate = ops / (best * 1e-3);
  std::printf("{\"kernel\": \"%s\", \"waves_per_simd\": %d, \"ms\": %.4f, "
              "\"lane_instr_per_s\": %.4e, \"x_single_issue_2p4GHz\": %.3f}\n",
              name, waves_per_simd, best, rate, rate / (cus * 64.0 * 2.4e9));
  CHK(hipEventDestroy(a));
  CHK(hipEventDestroy(b));
  return 0;
}

int main() {
  int cus = 0;
  CHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
  float *out = nullptr, *in = nullptr;
  CHK(hipMalloc(&out, sizeof(float) * cus * 8 * 256));
  CHK(hipMalloc(&in, sizeof(float) * 256));
  CHK(hipMemset(in, 0, sizeof(float) * 256));
  if (run<0>("add_sgpr_operand", cus, 8, out, in)) return 1;
  if (run<1>("add_vgpr_only", cus, 8, out, in)) return 1;
  for (int w : {1, 2, 4, 8})
    if (run<2>("dp_cell_vgpr_only", cus, w, out, in)) return 1;
  if (run<3>("fma_vgpr_only", cus, 8, out, in)) return 1;
  for (int w : {1, 2, 4, 8})
    if (run<4>("code_cell_vgpr_only", cus, w, out, in)) return 1;
  CHK(hipFree(out));
  CHK(hipFree(in));
  return 0;
}
