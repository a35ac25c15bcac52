// elementwise.hip -- HBM-bound element-wise kernels of the secret-sharing path:
// PRG fills, sharing, reveal, truncation, dealer triples, the fused Beaver
// element-wise product and square, the matmul open step and im2col.
//
// Each kernel is a grid-stride loop over 64-bit elements with 256-thread
// workgroups; consecutive lanes touch consecutive elements, so every wavefront
// load or store is one contiguous 512-byte access.
#include <initializer_list>

#include "internal.h"

namespace mpc {
namespace {

constexpr int kThreads = 256;

// Up to 65536 workgroups (16M threads): with many streams per element (the
// Beaver product reads ten), HBM throughput keeps rising with the number of
// loads in flight well past the point where the chip is "full".
inline int grid_for(size_t n) {
  size_t g = (n + kThreads - 1) / kThreads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

__device__ __forceinline__ u64 prg_at(u64 key, u64 i) { return sm_out(key, i); }

// floor(s64(v) / 2^bits): arithmetic shift of the signed share.
__device__ __forceinline__ u64 trunc_share(u64 v, int bits) {
  return bits ? (u64)((i64)v >> bits) : v;
}

#define GRID_STRIDE(i, n) \
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)

__global__ void __launch_bounds__(kThreads) k_prg_fill(u64 key, u64* __restrict__ out, size_t n) {
  GRID_STRIDE(i, n) out[i] = prg_at(key, i);
}

// Pseudorandom zero-share (-m, m); the source party adds its value.
__global__ void __launch_bounds__(kThreads)
    k_share(const u64* __restrict__ x, size_t n, int src, u64 key, u64* __restrict__ s0,
            u64* __restrict__ s1) {
  GRID_STRIDE(i, n) {
    const u64 m = prg_at(key, i);
    const u64 mine = x[i] - m;
    if (src == 0) {
      s0[i] = mine;
      s1[i] = m;
    } else {
      s0[i] = m;
      s1[i] = mine;
    }
  }
}

__global__ void __launch_bounds__(kThreads)
    k_reveal(const u64* s0, const u64* s1, size_t n, u64* out) {
  GRID_STRIDE(i, n) out[i] = s0[i] + s1[i];
}

__global__ void __launch_bounds__(kThreads) k_add(const u64* x, const u64* y, size_t n, u64* out) {
  GRID_STRIDE(i, n) out[i] = x[i] + y[i];
}

__global__ void __launch_bounds__(kThreads) k_truncate(u64* __restrict__ v, size_t n, int bits) {
  GRID_STRIDE(i, n) v[i] = trunc_share(v[i], bits);
}

struct Keys6 {
  u64 k[6];
};

__global__ void __launch_bounds__(kThreads)
    k_dealer_mul(Keys6 key, size_t n, u64* __restrict__ a0, u64* __restrict__ a1,
                 u64* __restrict__ b0, u64* __restrict__ b1, u64* __restrict__ c0,
                 u64* __restrict__ c1) {
  GRID_STRIDE(i, n) {
    const u64 va0 = prg_at(key.k[kSlotA0], i), va1 = prg_at(key.k[kSlotA1], i);
    const u64 vb0 = prg_at(key.k[kSlotB0], i), vb1 = prg_at(key.k[kSlotB1], i);
    const u64 vc0 = prg_at(key.k[kSlotC0], i);
    a0[i] = va0;
    a1[i] = va1;
    b0[i] = vb0;
    b1[i] = vb1;
    c0[i] = vc0;
    c1[i] = (va0 + va1) * (vb0 + vb1) - vc0;
  }
}

__global__ void __launch_bounds__(kThreads)
    k_dealer_square(Keys6 key, size_t n, u64* __restrict__ a0, u64* __restrict__ a1,
                    u64* __restrict__ b0, u64* __restrict__ b1) {
  GRID_STRIDE(i, n) {
    const u64 va0 = prg_at(key.k[kSlotA0], i), va1 = prg_at(key.k[kSlotA1], i);
    const u64 vb0 = prg_at(key.k[kSlotB0], i);
    const u64 a = va0 + va1;
    a0[i] = va0;
    a1[i] = va1;
    b0[i] = vb0;
    b1[i] = a * a - vb0;
  }
}

// Fused Beaver product for both parties: mask, open (device-local sum),
// finish and truncation in one pass; 10 shares in, 2 shares out per element.
__global__ void __launch_bounds__(kThreads)
    k_beaver_mul(size_t n, const u64* __restrict__ x0, const u64* __restrict__ x1,
                 const u64* __restrict__ y0, const u64* __restrict__ y1,
                 const u64* __restrict__ a0, const u64* __restrict__ a1,
                 const u64* __restrict__ b0, const u64* __restrict__ b1,
                 const u64* __restrict__ c0, const u64* __restrict__ c1, int trunc,
                 u64* __restrict__ z0, u64* __restrict__ z1) {
  GRID_STRIDE(i, n) {
    const u64 va0 = a0[i], va1 = a1[i], vb0 = b0[i], vb1 = b1[i];
    const u64 eps = (x0[i] - va0) + (x1[i] - va1);
    const u64 del = (y0[i] - vb0) + (y1[i] - vb1);
    const u64 r0 = c0[i] + eps * vb0 + va0 * del + eps * del;
    const u64 r1 = c1[i] + eps * vb1 + va1 * del;
    z0[i] = trunc_share(r0, trunc);
    z1[i] = trunc_share(r1, trunc);
  }
}

// Square with a Beaver pair (a, b = a^2): 6 shares in, 2 out.
__global__ void __launch_bounds__(kThreads)
    k_beaver_square(size_t n, const u64* __restrict__ x0, const u64* __restrict__ x1,
                    const u64* __restrict__ a0, const u64* __restrict__ a1,
                    const u64* __restrict__ b0, const u64* __restrict__ b1, int trunc,
                    u64* __restrict__ z0, u64* __restrict__ z1) {
  GRID_STRIDE(i, n) {
    const u64 va0 = a0[i], va1 = a1[i];
    const u64 eps = (x0[i] - va0) + (x1[i] - va1);
    const u64 r0 = b0[i] + 2 * eps * va0 + eps * eps;
    const u64 r1 = b1[i] + 2 * eps * va1;
    z0[i] = trunc_share(r0, trunc);
    z1[i] = trunc_share(r1, trunc);
  }
}

// Two-element variants for 16-byte aligned arrays: one 16-byte load per
// array per lane (half as many memory instructions), streamed with
// non-temporal hints since no element is touched twice.
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u64x2 ld2(const u64* p, size_t i) {
  return __builtin_nontemporal_load((const u64x2*)p + i);
}
__device__ __forceinline__ void st2(u64* p, size_t i, u64x2 v) {
  __builtin_nontemporal_store(v, (u64x2*)p + i);
}

__global__ void __launch_bounds__(kThreads)
    k_beaver_mul2(size_t n2, const u64* __restrict__ x0, const u64* __restrict__ x1,
                  const u64* __restrict__ y0, const u64* __restrict__ y1,
                  const u64* __restrict__ a0, const u64* __restrict__ a1,
                  const u64* __restrict__ b0, const u64* __restrict__ b1,
                  const u64* __restrict__ c0, const u64* __restrict__ c1, int trunc,
                  u64* __restrict__ z0, u64* __restrict__ z1) {
  GRID_STRIDE(i, n2) {
    const u64x2 va0 = ld2(a0, i), va1 = ld2(a1, i), vb0 = ld2(b0, i), vb1 = ld2(b1, i);
    const u64x2 eps = (ld2(x0, i) - va0) + (ld2(x1, i) - va1);
    const u64x2 del = (ld2(y0, i) - vb0) + (ld2(y1, i) - vb1);
    const u64x2 r0 = ld2(c0, i) + eps * vb0 + va0 * del + eps * del;
    const u64x2 r1 = ld2(c1, i) + eps * vb1 + va1 * del;
    st2(z0, i, u64x2{trunc_share(r0.x, trunc), trunc_share(r0.y, trunc)});
    st2(z1, i, u64x2{trunc_share(r1.x, trunc), trunc_share(r1.y, trunc)});
  }
}

__global__ void __launch_bounds__(kThreads)
    k_beaver_square2(size_t n2, const u64* __restrict__ x0, const u64* __restrict__ x1,
                     const u64* __restrict__ a0, const u64* __restrict__ a1,
                     const u64* __restrict__ b0, const u64* __restrict__ b1, int trunc,
                     u64* __restrict__ z0, u64* __restrict__ z1) {
  GRID_STRIDE(i, n2) {
    const u64x2 va0 = ld2(a0, i), va1 = ld2(a1, i);
    const u64x2 eps = (ld2(x0, i) - va0) + (ld2(x1, i) - va1);
    const u64x2 r0 = ld2(b0, i) + 2 * eps * va0 + eps * eps;
    const u64x2 r1 = ld2(b1, i) + 2 * eps * va1;
    st2(z0, i, u64x2{trunc_share(r0.x, trunc), trunc_share(r0.y, trunc)});
    st2(z1, i, u64x2{trunc_share(r1.x, trunc), trunc_share(r1.y, trunc)});
  }
}

bool aligned16(std::initializer_list<const void*> ps) {
  for (const void* p : ps)
    if (((uintptr_t)p & 15) != 0) return false;
  return true;
}

// Open step of Beaver bilinear products: one workgroup per chunk of
// kOpenChunk elements of one job (the job is found once per workgroup).
__global__ void __launch_bounds__(kThreads)
    k_open(const OpenJob* __restrict__ jobs, const i64* __restrict__ chunk_start, int njobs) {
  const i64 c = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (chunk_start[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  const OpenJob jb = jobs[lo];
  const i64 base = (c - chunk_start[lo]) * kOpenChunk;
  const i64 end = min(base + kOpenChunk, jb.n);
  for (i64 i = base + threadIdx.x; i < end; i += kThreads) {
    const u64 va0 = jb.a0[i];
    const u64 e = (jb.x0[i] - va0) + (jb.x1[i] - jb.a1[i]);
    jb.out0[i] = e;
    if (jb.kind == kOpenLeft) jb.out1[i] = va0 + e;
  }
}

// Beaver product (or square) of element i of one job: both parties' shares.
__device__ __forceinline__ void mul_one(const MulJob& jb, i64 i, int trunc) {
  const u64 va0 = jb.a0[i], va1 = jb.a1[i], vb0 = jb.b0[i], vb1 = jb.b1[i];
  const u64 eps = (jb.x0[i] - va0) + (jb.x1[i] - va1);
  u64 r0, r1;
  if (jb.y0) {
    const u64 del = (jb.y0[i] - vb0) + (jb.y1[i] - vb1);
    r0 = jb.c0[i] + eps * vb0 + va0 * del + eps * del;
    r1 = jb.c1[i] + eps * vb1 + va1 * del;
  } else {
    r0 = vb0 + 2 * eps * va0 + eps * eps;
    r1 = vb1 + 2 * eps * va1;
  }
  jb.z0[i] = trunc_share(r0, trunc);
  jb.z1[i] = trunc_share(r1, trunc);
}

// Many Beaver products in one launch: workgroup = one chunk of one job (the
// job is found once per workgroup by binary search over the chunk table).
// Aligned jobs move two elements per 16-byte load, as k_beaver_mul2 does;
// each thread takes kMulPairs pairs kThreads apart and issues all their loads
// before any store (the arrays of one job never overlap its outputs).
constexpr int kMulPairs = (int)(kMulChunk / 2 / kThreads);
static_assert(kMulPairs * 2 * kThreads == kMulChunk, "a chunk is whole rounds of pairs");

__global__ void __launch_bounds__(kThreads)
    k_beaver_mul_grouped(const MulJob* __restrict__ jobs, const i64* __restrict__ chunk_start, int njobs,
                         int trunc) {
  const i64 c = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (chunk_start[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  const MulJob jb = jobs[lo];
  const i64 base = (c - chunk_start[lo]) * kMulChunk;
  const i64 end = min(base + kMulChunk, jb.n);
  if (!jb.vec2) {
    for (i64 i = base + threadIdx.x; i < end; i += kThreads) mul_one(jb, i, trunc);
    return;
  }
  const u64 *__restrict__ x0 = jb.x0, *__restrict__ x1 = jb.x1, *__restrict__ y0 = jb.y0,
                          *__restrict__ y1 = jb.y1, *__restrict__ a0 = jb.a0, *__restrict__ a1 = jb.a1,
                          *__restrict__ b0 = jb.b0, *__restrict__ b1 = jb.b1, *__restrict__ c0 = jb.c0,
                          *__restrict__ c1 = jb.c1;
  u64* __restrict__ z0 = jb.z0;
  u64* __restrict__ z1 = jb.z1;
  const bool sq = y0 == nullptr;
  const i64 p_end = base / 2 + (end - base) / 2;  // whole pairs of the chunk
  u64x2 v[kMulPairs][10];
#pragma unroll
  for (int u = 0; u < kMulPairs; ++u) {
    const i64 p = base / 2 + threadIdx.x + (i64)u * kThreads;
    if (p < p_end) {
      v[u][0] = ld2(x0, p);
      v[u][1] = ld2(x1, p);
      v[u][2] = ld2(a0, p);
      v[u][3] = ld2(a1, p);
      v[u][4] = ld2(b0, p);
      v[u][5] = ld2(b1, p);
      if (!sq) {
        v[u][6] = ld2(y0, p);
        v[u][7] = ld2(y1, p);
        v[u][8] = ld2(c0, p);
        v[u][9] = ld2(c1, p);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kMulPairs; ++u) {
    const i64 p = base / 2 + threadIdx.x + (i64)u * kThreads;
    if (p < p_end) {
      const u64x2 eps = (v[u][0] - v[u][2]) + (v[u][1] - v[u][3]);
      u64x2 r0, r1;
      if (!sq) {
        const u64x2 del = (v[u][6] - v[u][4]) + (v[u][7] - v[u][5]);
        r0 = v[u][8] + eps * v[u][4] + v[u][2] * del + eps * del;
        r1 = v[u][9] + eps * v[u][5] + v[u][3] * del;
      } else {
        r0 = v[u][4] + 2 * eps * v[u][2] + eps * eps;
        r1 = v[u][5] + 2 * eps * v[u][3];
      }
      st2(z0, p, u64x2{trunc_share(r0.x, trunc), trunc_share(r0.y, trunc)});
      st2(z1, p, u64x2{trunc_share(r1.x, trunc), trunc_share(r1.y, trunc)});
    }
  }
  if ((end - base) % 2 && threadIdx.x == 0) mul_one(jb, end - 1, trunc);  // odd last element
}

__global__ void __launch_bounds__(kThreads)
    k_im2col(const u64* __restrict__ x, const u64* __restrict__ add, i64 cin, i64 len, i64 ksz,
             i64 stride, i64 lout, i64 ncols, size_t total, u64* __restrict__ col) {
  GRID_STRIDE(i, total) {
    const i64 k = (i64)(i / (size_t)ncols), n = (i64)(i % (size_t)ncols);
    const i64 c = k / ksz, j = k % ksz;
    const i64 b = n / lout, l = n % lout;
    const size_t src = (size_t)((b * cin + c) * len + l * stride + j);
    u64 v = x[src];
    if (add) v += add[src];
    col[i] = v;
  }
}

}  // namespace

hipError_t launch_beaver_mul_grouped(hipStream_t s, const MulJob* jobs, const i64* chunk_start, int njobs,
                                     i64 total_chunks, int trunc) {
  if (total_chunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_beaver_mul_grouped, dim3((unsigned)total_chunks), dim3(kThreads), 0, s, jobs, chunk_start,
                     njobs, trunc);
  return hipGetLastError();
}

hipError_t launch_prg_fill(hipStream_t s, u64 key, u64* out, size_t n) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_prg_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, key, out, n);
  return hipGetLastError();
}

hipError_t launch_share(hipStream_t s, const u64* x, size_t n, int src, u64 key, u64* s0,
                        u64* s1) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_share, dim3(grid_for(n)), dim3(kThreads), 0, s, x, n, src, key, s0, s1);
  return hipGetLastError();
}

hipError_t launch_reveal(hipStream_t s, const u64* s0, const u64* s1, size_t n, u64* out) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_reveal, dim3(grid_for(n)), dim3(kThreads), 0, s, s0, s1, n, out);
  return hipGetLastError();
}

hipError_t launch_add(hipStream_t s, const u64* x, const u64* y, size_t n, u64* out) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_add, dim3(grid_for(n)), dim3(kThreads), 0, s, x, y, n, out);
  return hipGetLastError();
}

hipError_t launch_truncate(hipStream_t s, u64* v, size_t n, int bits) {
  if (!n || !bits) return hipSuccess;
  hipLaunchKernelGGL(k_truncate, dim3(grid_for(n)), dim3(kThreads), 0, s, v, n, bits);
  return hipGetLastError();
}

hipError_t launch_dealer_mul(hipStream_t s, const u64 key[6], size_t n, u64* a0, u64* a1, u64* b0,
                             u64* b1, u64* c0, u64* c1) {
  if (!n) return hipSuccess;
  Keys6 k;
  for (int i = 0; i < 6; ++i) k.k[i] = key[i];
  hipLaunchKernelGGL(k_dealer_mul, dim3(grid_for(n)), dim3(kThreads), 0, s, k, n, a0, a1, b0, b1,
                     c0, c1);
  return hipGetLastError();
}

hipError_t launch_dealer_square(hipStream_t s, const u64 key[6], size_t n, u64* a0, u64* a1,
                                u64* b0, u64* b1) {
  if (!n) return hipSuccess;
  Keys6 k;
  for (int i = 0; i < 6; ++i) k.k[i] = key[i];
  hipLaunchKernelGGL(k_dealer_square, dim3(grid_for(n)), dim3(kThreads), 0, s, k, n, a0, a1, b0,
                     b1);
  return hipGetLastError();
}

hipError_t launch_beaver_mul(hipStream_t s, size_t n, const u64* x0, const u64* x1, const u64* y0,
                             const u64* y1, const u64* a0, const u64* a1, const u64* b0,
                             const u64* b1, const u64* c0, const u64* c1, int trunc, u64* z0,
                             u64* z1) {
  if (!n) return hipSuccess;
  if (n % 2 == 0 && aligned16({x0, x1, y0, y1, a0, a1, b0, b1, c0, c1, z0, z1})) {
    hipLaunchKernelGGL(k_beaver_mul2, dim3(grid_for(n / 2)), dim3(kThreads), 0, s, n / 2, x0, x1, y0, y1,
                       a0, a1, b0, b1, c0, c1, trunc, z0, z1);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_beaver_mul, dim3(grid_for(n)), dim3(kThreads), 0, s, n, x0, x1, y0, y1, a0,
                     a1, b0, b1, c0, c1, trunc, z0, z1);
  return hipGetLastError();
}

hipError_t launch_beaver_square(hipStream_t s, size_t n, const u64* x0, const u64* x1,
                                const u64* a0, const u64* a1, const u64* b0, const u64* b1,
                                int trunc, u64* z0, u64* z1) {
  if (!n) return hipSuccess;
  if (n % 2 == 0 && aligned16({x0, x1, a0, a1, b0, b1, z0, z1})) {
    hipLaunchKernelGGL(k_beaver_square2, dim3(grid_for(n / 2)), dim3(kThreads), 0, s, n / 2, x0, x1, a0,
                       a1, b0, b1, trunc, z0, z1);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_beaver_square, dim3(grid_for(n)), dim3(kThreads), 0, s, n, x0, x1, a0, a1,
                     b0, b1, trunc, z0, z1);
  return hipGetLastError();
}

hipError_t launch_open(hipStream_t s, const OpenJob* jobs, const i64* chunk_start, int njobs,
                       i64 total_chunks) {
  if (total_chunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_open, dim3((unsigned)total_chunks), dim3(kThreads), 0, s, jobs, chunk_start,
                     njobs);
  return hipGetLastError();
}

hipError_t launch_im2col(hipStream_t s, const u64* x, const u64* add, i64 B, i64 cin, i64 len,
                         i64 ksz, i64 stride, i64 lout, u64* col) {
  const i64 ncols = B * lout;
  const size_t total = (size_t)(cin * ksz) * (size_t)ncols;
  if (!total) return hipSuccess;
  hipLaunchKernelGGL(k_im2col, dim3(grid_for(total)), dim3(kThreads), 0, s, x, add, cin, len, ksz,
                     stride, lout, ncols, total, col);
  return hipGetLastError();
}

}  // namespace mpc
