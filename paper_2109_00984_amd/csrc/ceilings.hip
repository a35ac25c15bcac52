// ceilings.hip -- sustained arithmetic ceilings of the two ring GEMM forms on
// this GPU, with no memory traffic in the timed loops (a standalone program;
// prints one JSON line).
//
//  * INT8 matrix cores: v_mfma_i32_16x16x64_i8 over register-resident,
//    uniformly random operand fragments (the matrix cores' power draw, and so
//    the clock they sustain, depends on the data; random bytes are what limb
//    planes of secret shares are), 8 diagonal accumulators per 16x16 block and
//    4 blocks per wave, as in the limb GEMM's 64x64 tile.
//  * Vector ALUs: the plain GEMM's ring multiply-accumulate on 32-bit halves
//    (a 64-bit lo*lo multiply-add and two 32-bit cross products) over 8x4
//    register blocks.
//
// and two streaming rates of HBM, with buffers far larger than the caches
// (the 256 MB Infinity Cache included), each the best over a few loop forms
// (grid size, pairs of elements per thread and iteration):
//
//  * ten input streams and two output streams per element with trivial
//    arithmetic (a sum and an exclusive or): the access pattern of the fused
//    Beaver product, 96 bytes per element, at 2^24 elements per stream (the
//    size the Beaver product is measured at) and at 2^28;
//  * one input and one output stream (a copy), 16 bytes per element.
#include <hip/hip_runtime.h>
#include <cstdint>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>

typedef uint64_t u64;
typedef uint32_t u32;
typedef int v4i __attribute__((ext_vector_type(4)));

#define CK(x)                                                                          \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) {                                                            \
      std::fprintf(stderr, "ceilings: %s: %s\n", #x, hipGetErrorString(e_));           \
      return 1;                                                                        \
    }                                                                                  \
  } while (0)

__device__ __forceinline__ void mfma16(v4i& acc, const v4i& a, const v4i& b) {
  asm volatile("v_mfma_i32_16x16x64_i8 %0, %1, %2, %0" : "+a"(acc) : "v"(a), "v"(b));
}
__device__ __forceinline__ void mfma16_first(v4i& acc, const v4i& a, const v4i& b) {
  asm volatile("v_mfma_i32_16x16x64_i8 %0, %1, %2, 0" : "=a"(acc) : "v"(a), "v"(b));
}

// One wave: 4 blocks of 16x16 outputs x 8 diagonals; per step the 36 limb
// pairs of every block (144 MFMAs).  Consecutive MFMAs go to the 4 blocks in
// turn, so an MFMA's accumulator was last written 4 MFMAs earlier, as in the
// limb GEMM's tiles.
constexpr int RB = 4;
__global__ void __launch_bounds__(256, 1) k_mfma_ceiling(int steps, const v4i* __restrict__ rnd, int* out) {
  const int lane = threadIdx.x & 63;
  v4i a[RB][8], b[8], acc[RB][8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
#pragma unroll
    for (int r = 0; r < RB; ++r) a[r][i] = rnd[(i * (RB + 1) + r) * 64 + lane];
    b[i] = rnd[(i * (RB + 1) + RB) * 64 + lane];
  }
#pragma unroll
  for (int l = 0; l < 8; ++l)
#pragma unroll
    for (int s = l; s < 8; ++s)
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (l == 0) mfma16_first(acc[r][s], a[r][l], b[s - l]);
        else mfma16(acc[r][s], a[r][l], b[s - l]);
      }
  for (int k = 1; k < steps; ++k) {
#pragma unroll
    for (int l = 0; l < 8; ++l)
#pragma unroll
      for (int s = l; s < 8; ++s)
#pragma unroll
        for (int r = 0; r < RB; ++r) mfma16(acc[r][s], a[r][l], b[s - l]);
  }
  int sum = 0;
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int r = 0; r < RB; ++r) asm volatile("s_nop 3" : "+a"(acc[r][s]));
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int r = 0; r < RB; ++r) sum += acc[r][s][0] ^ acc[r][s][3];
  out[blockIdx.x * 256 + threadIdx.x] = sum;
}

constexpr int TM = 8, TN = 4;
__global__ void __launch_bounds__(256) k_valu_ceiling(int iters, u64 seed, u64* out) {
  u64 lo[TM][TN], a[TM], b[TN];
  u32 cr[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i) a[i] = seed * (i + 3) + threadIdx.x;
#pragma unroll
  for (int j = 0; j < TN; ++j) b[j] = (seed * (j + 7)) ^ threadIdx.x;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      lo[i][j] = 0;
      cr[i][j] = 0;
    }
  for (int it = 0; it < iters; ++it) {
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const u32 al = (u32)a[i], ah = (u32)(a[i] >> 32);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const u32 bl = (u32)b[j], bh = (u32)(b[j] >> 32);
          lo[i][j] += (u64)al * (u64)bl;
          cr[i][j] += al * bh + ah * bl;
        }
      }
      // new operands every k, so nothing is loop-invariant
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] += 0x9e3779b97f4a7c15ULL;
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] ^= (u64)kk << 17;
    }
  }
  u64 s = 0;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) s += lo[i][j] + ((u64)cr[i][j] << 32);
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

// Streaming kernels: 16-byte non-temporal loads and stores, grid-stride over
// pairs of 64-bit elements; each thread takes U pairs 256 apart per iteration
// and issues all their loads before any store.
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u64x2 ld(const u64x2* p, size_t i) { return __builtin_nontemporal_load(p + i); }
__device__ __forceinline__ void st(u64x2* p, size_t i, u64x2 v) { __builtin_nontemporal_store(v, p + i); }

struct Ins10 {
  const u64x2* p[10];
};

template <int U>
__global__ void __launch_bounds__(256) k_stream_10r2w(size_t n2, Ins10 in, u64x2* __restrict__ o0, u64x2* __restrict__ o1) {
  const size_t step = (size_t)gridDim.x * 256 * U;
  for (size_t i = (size_t)blockIdx.x * 256 * U + threadIdx.x; i < n2; i += step) {
    u64x2 sum[U], x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t j = i + (size_t)u * 256;
      sum[u] = x[u] = u64x2{0, 0};
      if (j < n2) {
#pragma unroll
        for (int a = 0; a < 10; ++a) {
          const u64x2 v = ld(in.p[a], j);
          sum[u] += v;
          x[u] ^= v;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t j = i + (size_t)u * 256;
      if (j < n2) {
        st(o0, j, sum[u]);
        st(o1, j, x[u]);
      }
    }
  }
}

template <int U>
__global__ void __launch_bounds__(256) k_copy(size_t n2, const u64x2* __restrict__ in, u64x2* __restrict__ out) {
  const size_t step = (size_t)gridDim.x * 256 * U;
  for (size_t i = (size_t)blockIdx.x * 256 * U + threadIdx.x; i < n2; i += step) {
    u64x2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = i + (size_t)u * 256 < n2 ? ld(in, i + (size_t)u * 256) : u64x2{0, 0};
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + (size_t)u * 256 < n2) st(out, i + (size_t)u * 256, v[u]);
  }
}

// SplitMix64 bytes for the operand fragments (Steele, Lea and Flood, 2014).
__global__ void k_fill(u64* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  u64 z = (u64)(i + 1) * 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  p[i] = z ^ (z >> 31);
}

// Times `reps` launches after `warm` untimed ones: the engine clock ramps up
// over the first few milliseconds of sustained load.
template <class F>
static int time_ms(F launch, int warm, int reps, float* ms) {
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  for (int w = 0; w < warm; ++w) launch();
  CK(hipDeviceSynchronize());
  CK(hipEventRecord(e0, 0));
  for (int r = 0; r < reps; ++r) launch();
  CK(hipEventRecord(e1, 0));
  CK(hipEventSynchronize(e1));
  CK(hipEventElapsedTime(ms, e0, e1));
  *ms /= reps;
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
  return 0;
}

// `ceilings mfma <seconds>`: only the INT8 MFMA loop, launched back to back
// for that long (for power readings under sustained matrix-core load);
// prints its mean rate.
static int mfma_only(double secs) {
  const int blocks = 2048, steps = 128;
  v4i* rnd = nullptr;
  int* iout = nullptr;
  constexpr int kFrags = 8 * (RB + 1) * 64;
  CK(hipMalloc(&rnd, kFrags * sizeof(v4i)));
  CK(hipMalloc(&iout, (size_t)blocks * 256 * sizeof(int)));
  hipLaunchKernelGGL(k_fill, dim3((kFrags * 2 + 255) / 256), dim3(256), 0, 0, (u64*)rnd, kFrags * 2);
  CK(hipGetLastError());
  double total_ms = 0;
  long launches = 0;
  while (total_ms < secs * 1e3) {
    float ms = 0.f;
    if (time_ms([&] { hipLaunchKernelGGL(k_mfma_ceiling, dim3(blocks), dim3(256), 0, 0, steps, rnd, iout); }, 0, 50,
                &ms))
      return 1;
    total_ms += 50.0 * ms;
    launches += 50;
  }
  const double ops = 2.0 * 16 * 16 * 64 * (36.0 * RB) * steps * 4.0 * blocks * launches;
  std::printf("{\"mfma_i8_random_tops\": %.1f, \"seconds\": %.2f}\n", ops / (total_ms * 1e-3) / 1e12, total_ms * 1e-3);
  CK(hipFree(rnd));
  CK(hipFree(iout));
  return 0;
}

int main(int argc, char** argv) {
  if (argc == 3 && std::string(argv[1]) == "mfma") return mfma_only(std::atof(argv[2]));
  const int blocks = 2048;
  v4i* rnd = nullptr;
  int* iout = nullptr;
  u64* uout = nullptr;
  constexpr int kFrags = 8 * (RB + 1) * 64;  // operand fragments of all lanes
  CK(hipMalloc(&rnd, kFrags * sizeof(v4i)));
  CK(hipMalloc(&iout, (size_t)blocks * 256 * sizeof(int)));
  CK(hipMalloc(&uout, (size_t)blocks * 256 * sizeof(u64)));
  hipLaunchKernelGGL(k_fill, dim3((kFrags * 2 + 255) / 256), dim3(256), 0, 0, (u64*)rnd, kFrags * 2);
  CK(hipGetLastError());
  const int steps = 128;
  float mfma_ms = 0.f, valu_ms = 0.f;
  if (time_ms([&] { hipLaunchKernelGGL(k_mfma_ceiling, dim3(blocks), dim3(256), 0, 0, steps, rnd, iout); }, 40, 10,
              &mfma_ms))
    return 1;
  const int iters = 64;
  if (time_ms([&] { hipLaunchKernelGGL(k_valu_ceiling, dim3(blocks), dim3(256), 0, 0, iters, 12345ULL, uout); }, 10, 5,
              &valu_ms))
    return 1;
  const double mfma_ops = 2.0 * 16 * 16 * 64 * (36.0 * RB) * steps * 4.0 * blocks;
  const double valu_macs = (double)blocks * 256 * iters * 16 * TM * TN;

  // streams: 12 buffers of 2^28 elements (24 GiB in all) for the Beaver
  // pattern, measured over their first 2^24 and over all 2^28 elements; the
  // copy over 2^28 elements (4 GiB of traffic); best of grids of 16384..65536
  // workgroups and 1, 2 or 4 pairs per thread and iteration
  const size_t n_big = (size_t)1 << 28, n_bv = (size_t)1 << 24;
  u64x2* bufs[12];
  for (auto& b : bufs) {
    CK(hipMalloc(&b, n_big * sizeof(u64)));
    CK(hipMemset(b, 0x5a, n_big * sizeof(u64)));
  }
  Ins10 ins;
  for (int a = 0; a < 10; ++a) ins.p[a] = bufs[a];
  const unsigned grids[] = {16384, 32768, 65536};
  auto best_rate = [&](auto launch_u1, auto launch_u2, auto launch_u4, double bytes, int reps, double* gbs) {
    *gbs = 0;
    for (unsigned g : grids)
      for (int u : {1, 2, 4}) {
        float ms = 0.f;
        const int r = time_ms([&] { u == 1 ? launch_u1(g) : u == 2 ? launch_u2(g) : launch_u4(g); }, 2, reps, &ms);
        if (r) return r;
        *gbs = std::max(*gbs, bytes / (ms * 1e-3) / 1e9);
      }
    return 0;
  };
  auto bv = [&](size_t n, int u, unsigned g) {
    const size_t n2 = n / 2, need = (n2 + 256 * (size_t)u - 1) / (256 * (size_t)u);
    return dim3((unsigned)std::min<size_t>(g, need));
  };
  double bv_gbs = 0, bv28_gbs = 0, cp_gbs = 0;
#define MPC_BV_LAUNCH(U, N)                                                                                        \
  [&](unsigned g) {                                                                                              \
    hipLaunchKernelGGL(k_stream_10r2w<U>, bv(N, U, g), dim3(256), 0, 0, (N) / 2, ins, bufs[10], bufs[11]); \
  }
#define MPC_CP_LAUNCH(U)                                                                                        \
  [&](unsigned g) {                                                                                           \
    hipLaunchKernelGGL(k_copy<U>, bv(n_big, U, g), dim3(256), 0, 0, n_big / 2, bufs[0], bufs[11]); \
  }
  if (best_rate(MPC_BV_LAUNCH(1, n_bv), MPC_BV_LAUNCH(2, n_bv), MPC_BV_LAUNCH(4, n_bv), 96.0 * n_bv, 20, &bv_gbs))
    return 1;
  if (best_rate(MPC_BV_LAUNCH(1, n_big), MPC_BV_LAUNCH(2, n_big), MPC_BV_LAUNCH(4, n_big), 96.0 * n_big, 3,
                &bv28_gbs))
    return 1;
  if (best_rate(MPC_CP_LAUNCH(1), MPC_CP_LAUNCH(2), MPC_CP_LAUNCH(4), 16.0 * n_big, 10, &cp_gbs)) return 1;
#undef MPC_BV_LAUNCH
#undef MPC_CP_LAUNCH

  std::printf("{\"mfma_i8_random_tops\": %.1f, \"valu_ring_tmacs\": %.3f, \"hbm_stream_10r2w_gbs\": %.1f, "
              "\"hbm_stream_10r2w_2e28_gbs\": %.1f, \"hbm_copy_gbs\": %.1f}\n",
              mfma_ops / (mfma_ms * 1e-3) / 1e12, valu_macs / (valu_ms * 1e-3) / 1e12, bv_gbs, bv28_gbs, cp_gbs);
  for (auto b : bufs) CK(hipFree(b));
  CK(hipFree(rnd));
  CK(hipFree(iout));
  CK(hipFree(uout));
  return 0;
}
