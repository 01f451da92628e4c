// valu_rates.hip -- issue cost of single-precision VALU instructions on one gfx950 SIMD.
//
// Each kernel runs 8 wavefronts per SIMD (2048 workgroups of 256 lanes on 256
// CUs), every lane carrying 8 independent dependency chains of one
// instruction for 4096 iterations, so issue rate rather than latency sets the
// time.  Cycles per wavefront instruction per SIMD = kernel time x 2.4 GHz /
// (8 waves x 4096 x 8).  The kernel durations come from
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o /tmp/valu_rates paper_2411_03418_amd/probes/valu_rates.hip
//   rocprofv3 --kernel-trace --stats -d <dir> -o rates -- /tmp/valu_rates
// (the program also prints its own estimate from HIP events).  Used to read
// the level kernels' instruction counts against the chip's issue rates.
#include <hip/hip_runtime.h>
#include <cstdio>

namespace {

constexpr int kChains = 8;
constexpr int kIters = 4096;
constexpr int kBlocks = 2048;

template <int OP>
__global__ void __launch_bounds__(256) k_rate(float* out) {
  float v[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) v[c] = 0.25f + 0.01f * c + 1e-6f * threadIdx.x;
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (OP == 0) v[c] = fmaf(v[c], 0.999f, 0.001f);          // v_fma_f32
      else if constexpr (OP == 1) v[c] = v[c] * 1.0001f;                 // v_mul_f32
      else if constexpr (OP == 2) v[c] = v[c] + 0.0001f;                 // v_add_f32
      else if constexpr (OP == 3) v[c] = __builtin_amdgcn_exp2f(-v[c]);  // v_exp_f32
      else if constexpr (OP == 4) v[c] = __builtin_amdgcn_rcpf(v[c]);    // v_rcp_f32
      else v[c] = __builtin_amdgcn_sqrtf(v[c]);                          // v_sqrt_f32
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += v[c];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int OP>
bool run(float* out, const char* name) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return false;
  float ms = 0.0f;
  for (int rep = 0; rep < 3; ++rep) {
    if (hipEventRecord(a) != hipSuccess) return false;
    k_rate<OP><<<kBlocks, 256>>>(out);
    if (hipEventRecord(b) != hipSuccess || hipEventSynchronize(b) != hipSuccess) return false;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return false;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  const double insts = (double)kBlocks * 4 / 1024 * kIters * kChains;   // per SIMD
  std::printf("%-5s %8.3f ms  %5.2f cycles per wavefront instruction per SIMD\n", name, ms,
              ms * 1e-3 * 2.4e9 / insts);
  return true;
}

}  // namespace

int main() {
  float* out = nullptr;
  if (hipMalloc(&out, (size_t)kBlocks * 256 * sizeof(float)) != hipSuccess) return 1;
  const bool ok = run<0>(out, "fma") && run<1>(out, "mul") && run<2>(out, "add") && run<3>(out, "exp2") &&
                  run<4>(out, "rcp") && run<5>(out, "sqrt");
  return ok && hipDeviceSynchronize() == hipSuccess ? 0 : 2;
}
