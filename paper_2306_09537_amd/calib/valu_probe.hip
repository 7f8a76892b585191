// VALU issue-cost probe for the ALU roofline of the stepper kernels.
//
// Each kernel runs eight independent chains of one instruction kind over
// 32 waves per SIMD (8192 workgroups of 256 lanes), so the SIMD issue rate,
// not the chains' latency, sets the time.  Printed per kind: the event time
// and the cycles per wave64 VALU instruction at 2.4 GHz, counting the
// probed instructions of the loop (per-kind count below; the compiler keeps
// each chain as written, which rocprofv3's SQ_INSTS_VALU confirms).  The
// integer ring compiles to a mix of xor and add, and the 64-bit multiply-add
// ring to one move per multiply-add: for those two the cost per instruction
// is the time over SQ_INSTS_VALU.  Every
// lane writes one float to out[gid]; out holds one float per lane.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                  \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                               \
    }                                                                             \
  } while (0)

enum Kind { ADD_F32, FMA_F32, MUL_F32, MAX_F32, CNDMASK, CVT_F32_U32, EXP_F32, SQRT_F32,
            RCP_F32, ADD_U32, XOR_B32, MAD_U64_U32 };

template <int K>
__global__ __launch_bounds__(256) void probe(float* out, int iters, float x, float y) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  float a[8];
  unsigned u[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = gid * 1e-7f + j;
    u[j] = gid + j;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if constexpr (K == ADD_F32) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] += x;
      } else if constexpr (K == FMA_F32) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = __builtin_fmaf(a[j], x, y);
      } else if constexpr (K == MUL_F32) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] *= x;
      } else if constexpr (K == MAX_F32) {  // ring: not foldable
        const float t0 = a[0];
#pragma unroll
        for (int j = 0; j < 7; ++j) a[j] = __builtin_fmaxf(a[j], a[j + 1]);
        a[7] = __builtin_fmaxf(a[7], t0);
      } else if constexpr (K == CNDMASK) {  // one lane mask per unrolled position
        const bool c = ((gid >> (r & 7)) & 1) != 0;
        const float t0 = a[0], t1 = a[1];
#pragma unroll
        for (int j = 0; j < 6; ++j) a[j] = c ? a[j + 1] : a[j + 2];
        a[6] = c ? a[7] : t0;
        a[7] = c ? t0 : t1;
      } else if constexpr (K == CVT_F32_U32) {
        const unsigned t0 = u[0];
#pragma unroll
        for (int j = 0; j < 7; ++j) u[j] = __float_as_uint((float)u[j + 1]);
        u[7] = __float_as_uint((float)t0);
      } else if constexpr (K == EXP_F32) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = __builtin_amdgcn_exp2f(a[j]);
      } else if constexpr (K == SQRT_F32) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = __builtin_amdgcn_sqrtf(a[j]);
      } else if constexpr (K == RCP_F32) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = __builtin_amdgcn_rcpf(a[j]);
      } else if constexpr (K == ADD_U32) {
        const unsigned t0 = u[0];
#pragma unroll
        for (int j = 0; j < 7; ++j) u[j] += u[j + 1];
        u[7] += t0;
      } else if constexpr (K == XOR_B32) {
        const unsigned t0 = u[0];
#pragma unroll
        for (int j = 0; j < 7; ++j) u[j] ^= u[j + 1] + (unsigned)r;
        u[7] ^= t0;
      } else if constexpr (K == MAD_U64_U32) {  // 32 x 32 + 64 -> 64, halves cross over
        unsigned long long p[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          p[j] = (unsigned long long)u[2 * j] * (j & 1 ? 0xCD9E8D57u : 0xD2511F53u) + u[2 * j + 1];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          u[2 * j] = (unsigned)(p[(j + 1) & 3] >> 32);
          u[2 * j + 1] = (unsigned)p[(j + 2) & 3];
        }
      }
    }
  }
  float s = 0.f;
  unsigned v = 0u;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    s += a[j];
    v ^= u[j];
  }
  out[gid] = s + __uint_as_float(v & 0x3fffffffu);
}

template <int K>
void run(const char* name, float* d, int blocks, int iters, double per_iter) {
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  probe<K><<<blocks, 256>>>(d, iters, 1.0000001f, 1e-7f);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  float best = 1e30f;
  for (int rep = 0; rep < 5; ++rep) {
    CHECK(hipEventRecord(e0));
    probe<K><<<blocks, 256>>>(d, iters, 1.0000001f, 1e-7f);
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) best = ms;
  }
  const double waves_per_simd = blocks * 256.0 / 64.0 / 1024.0;
  const double insts = waves_per_simd * iters * per_iter;  // probed instructions per SIMD
  if (per_iter > 0)
    std::printf("%-14s %8.3f ms  %6.2f cycles per wave64 instruction\n", name, best,
                best * 1e-3 * 2.4e9 / insts);
  else  // a mix of kinds: the cost per instruction comes from SQ_INSTS_VALU
    std::printf("%-14s %8.3f ms  (mixed kinds)\n", name, best);
  std::fflush(stdout);
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
}

int main() {
  const int blocks = 8192;  // 32 waves per SIMD on 256 CUs x 4 SIMDs
  float* d;
  CHECK(hipMalloc(&d, sizeof(float) * blocks * 256));
  std::printf("kind           time (best of 5)  cost\n");
  run<ADD_F32>("v_add_f32", d, blocks, 256, 128);
  run<FMA_F32>("v_fma_f32", d, blocks, 256, 128);
  run<MUL_F32>("v_mul_f32", d, blocks, 256, 128);
  run<MAX_F32>("v_max_f32", d, blocks, 256, 128);
  run<CNDMASK>("v_cndmask_b32", d, blocks, 256, 128);
  run<CVT_F32_U32>("v_cvt_f32_u32", d, blocks, 256, 128);
  run<EXP_F32>("v_exp_f32", d, blocks, 64, 128);
  run<SQRT_F32>("v_sqrt_f32", d, blocks, 64, 128);
  run<RCP_F32>("v_rcp_f32", d, blocks, 64, 128);
  run<ADD_U32>("v_add_u32", d, blocks, 256, 128);
  run<XOR_B32>("xor/add_u32", d, blocks, 256, 0);
  run<MAD_U64_U32>("mad_u64+mov", d, blocks, 64, 0);
  CHECK(hipFree(d));
  return 0;
}
