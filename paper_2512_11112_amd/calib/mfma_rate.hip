// Sustained int8 MFMA rate of this GPU for the exact-GEMM accumulation pattern:
// 4 waves per block, each wave issuing 128 v_mfma_i32_32x32x32_i8 per step into
// 15 shift-class accumulators (8 x 8 digit pairs, two 32-deep halves), operands held
// in registers (no memory traffic at all).  Run once with random operand bytes (the
// digits of uniformly random residues look like this) and once with small structured
// operands: the gap between the two is the clock the chip can hold at its power limit
// when the matrix cores switch random data, i.e. the practical ceiling for the GEMM.
//
//   mfma_rate [blocks] [steps]      prints one JSON line
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));          \
      exit(1);                                                                \
    }                                                                         \
  } while (0)

template <bool RANDOM>
__global__ __launch_bounds__(256, 1) void k_rate(int steps, int *out) {
  const int t = threadIdx.x, lane = t & 63;
  v16i acc[15];
#pragma unroll
  for (int s = 0; s < 15; s++) acc[s] = (v16i){0};
  v4i a[2][8], b[2][8];
  uint32_t h = (uint32_t)(t * 131 + blockIdx.x * 15485863u) | 1u;
  auto mix = [&]() {  // xorshift32
    h ^= h << 13;
    h ^= h >> 17;
    h ^= h << 5;
    return (int)h;
  };
#pragma unroll
  for (int kk = 0; kk < 2; kk++)
#pragma unroll
    for (int d = 0; d < 8; d++) {
      if (RANDOM) {
        a[kk][d] = (v4i){mix(), mix(), mix(), mix()};
        b[kk][d] = (v4i){mix(), mix(), mix(), mix()};
      } else {
        a[kk][d] = (v4i){t + d, kk, lane, d};
        b[kk][d] = (v4i){t - d, kk + 1, lane, 3 * d};
      }
    }
  for (int st = 0; st < steps; st++) {
#pragma unroll
    for (int kk = 0; kk < 2; kk++)
#pragma unroll
      for (int dk = 0; dk < 8; dk++)
#pragma unroll
        for (int dl = 0; dl < 8; dl++)
          acc[dk + dl] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[kk][dk], b[kk][dl], acc[dk + dl], 0, 0, 0);
  }
  int s = 0;
#pragma unroll
  for (int c = 0; c < 15; c++)
#pragma unroll
    for (int r = 0; r < 16; r++) s += acc[c][r];
  out[(size_t)blockIdx.x * 256 + t] = s;
}

int main(int argc, char **argv) {
  const int blocks = argc > 1 ? atoi(argv[1]) : 4096;
  const int steps = argc > 2 ? atoi(argv[2]) : 400;
  if (blocks < 1 || blocks > 65536 || steps < 1 || steps > 100000) {
    fprintf(stderr, "blocks in [1, 65536], steps in [1, 100000]\n");
    return 2;
  }
  int *out;
  CHECK(hipMalloc(&out, (size_t)blocks * 256 * sizeof(int)));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  double tops[2];
  for (int mode = 0; mode < 2; mode++) {
    float best = 1e30f;
    for (int rep = 0; rep < 4; rep++) {  // the first is a warm-up
      CHECK(hipEventRecord(e0));
      if (mode == 0)
        hipLaunchKernelGGL((k_rate<true>), dim3(blocks), dim3(256), 0, 0, steps, out);
      else
        hipLaunchKernelGGL((k_rate<false>), dim3(blocks), dim3(256), 0, 0, steps, out);
      CHECK(hipGetLastError());
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      float ms;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0 && ms < best) best = ms;
    }
    const double ops = (double)blocks * 4 * steps * 128 * 32.0 * 32 * 32 * 2;
    tops[mode] = ops / (best * 1e-3) / 1e12;
  }
  printf("{\"int8_mfma_register_tops_random\": %.1f, \"int8_mfma_register_tops_structured\": %.1f, "
         "\"blocks\": %d, \"steps\": %d}\n",
         tops[0], tops[1], blocks, steps);
  CHECK(hipFree(out));
  return 0;
}
