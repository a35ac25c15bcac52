// gemm_fp64.hip -- the ring GEMM in the paper's own GPU form: fp64 limbs.
//
// Section 5.3 (off-loading computations to the GPU) computes an int64 ring
// product with floating-point library GEMMs: each 64-bit operand is split
// into four 16-bit components (ten pairwise products), or into three 22-bit
// components (six products) when the sums stay small enough, and every
// pairwise product is exact in float64.  This file holds the element-wise
// parts of that form -- splitting operands into fp64 limb planes and
// combining the exact per-diagonal sums into the ring result -- while the
// pairwise products themselves run as fp64 GEMMs of the vendor BLAS (one call
// per diagonal, over concatenated k).  It exists to measure the paper's
// method on this GPU next to the INT8 limb form; both are bit-exact.
//
// Limbs.  With L limbs of w bits and u = v + bias (mod 2^64), where bias adds
// 2^(w-1) at every limb position that lies inside 64 bits,
//   d_i = field_i(u) - 2^(w-1)   (limbs that are whole w-bit fields)
//   d_i = field_i(u)             (a top limb cut short by the 64-bit width)
// gives v = sum_i d_i 2^(w i) (mod 2^64).  L = 4, w = 16: all four fields are
// whole, |d_i| <= 2^15.  L = 3, w = 22: the top field has 20 bits and is
// unsigned, |d_0|, |d_1| <= 2^21, 0 <= d_2 < 2^20.
#include "internal.h"

namespace mpc {
namespace {

constexpr int kFpThreads = 256;

struct Split {
  int L, w;
  u64 bias, mask;
};

__host__ __device__ inline Split fp64_split(int L) {
  Split s;
  s.L = L;
  s.w = L == 4 ? 16 : 22;
  s.mask = (1ull << s.w) - 1;
  s.bias = 0;
  for (int i = 0; i < L; ++i)
    if (s.w * (i + 1) <= 64) s.bias += (1ull << (s.w - 1)) << (s.w * i);
  return s;
}

__device__ __forceinline__ double limb(const Split& s, u64 u, int i) {
  const u64 f = (u >> (s.w * i)) & s.mask;
  const i64 d = s.w * (i + 1) <= 64 ? (i64)f - ((i64)1 << (s.w - 1)) : (i64)f;
  return (double)d;
}

// LA[m][i*Kt + k] = d_i(A[m][k]),  A = [A0 (M x K0, lda0) | A1 (M x K1, lda1)]
__global__ void __launch_bounds__(kFpThreads)
    k_fp64_pack_left(i64 M, i64 K0, i64 K1, const u64* __restrict__ A0, i64 lda0,
                     const u64* __restrict__ A1, i64 lda1, int L, double* __restrict__ LA) {
  const Split sp = fp64_split(L);
  const i64 Kt = K0 + K1, total = M * Kt;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    const i64 m = e / Kt, k = e % Kt;
    const u64 v = k < K0 ? A0[m * lda0 + k] : A1[m * lda1 + (k - K0)];
    const u64 u = v + sp.bias;
    double* row = LA + m * (L * Kt) + k;
    for (int i = 0; i < L; ++i) row[i * Kt] = limb(sp, u, i);
  }
}

// RB[(L-1-j)*Kt + k][n] = d_j(B[k][n]),  B = [B0 (K0 x N, ldb0) ; B1 (K1 x N, ldb1)]
// (limb planes in reverse order, so diagonal s reads one contiguous row range)
__global__ void __launch_bounds__(kFpThreads)
    k_fp64_pack_right(i64 N, i64 K0, i64 K1, const u64* __restrict__ B0, i64 ldb0,
                      const u64* __restrict__ B1, i64 ldb1, int L, double* __restrict__ RB) {
  const Split sp = fp64_split(L);
  const i64 Kt = K0 + K1, total = Kt * N;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    const i64 k = e / N, n = e % N;
    const u64 v = k < K0 ? B0[k * ldb0 + n] : B1[(k - K0) * ldb1 + n];
    const u64 u = v + sp.bias;
    for (int j = 0; j < L; ++j) RB[((i64)(L - 1 - j) * Kt + k) * N + n] = limb(sp, u, j);
  }
}

// out = sum_s 2^(w s) X_s (mod 2^64), X_s exact integers in float64, then the
// shared epilogue (accumulate, add or subtract a share, truncate, store).
__global__ void __launch_bounds__(kFpThreads)
    k_fp64_combine(i64 M, i64 N, int L, const double* __restrict__ X, Epilogue ep) {
  const Split sp = fp64_split(L);
  const i64 total = M * N;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    const i64 m = e / N, n = e % N;
    u64 v = 0;
    for (int s = 0; s < L; ++s) v += (u64)(i64)X[(i64)s * total + e] << (sp.w * s);
    const i64 off = m * ep.view.ld_m + (n / ep.view.n_div) * ep.view.ld_q + (n % ep.view.n_div);
    if (ep.accumulate) v += ep.Out[off];
    if (ep.Cadd) v += (ep.csign < 0) ? (u64)0 - ep.Cadd[off] : ep.Cadd[off];
    if (ep.trunc_bits) v = (u64)((i64)v >> ep.trunc_bits);
    ep.Out[off] = v;
  }
}

unsigned grid_of(i64 n) {
  const i64 b = (n + kFpThreads - 1) / kFpThreads;
  return (unsigned)(b < 1 ? 1 : b > 16384 ? 16384 : b);
}

}  // namespace

int fp64_limbs(i64 Kt) { return Kt < kFp64Limb22MaxK ? 3 : 4; }

hipError_t launch_fp64_pack_left(hipStream_t s, i64 M, i64 K0, i64 K1, const u64* A0, i64 lda0,
                                 const u64* A1, i64 lda1, int L, double* LA) {
  if (M * (K0 + K1) <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fp64_pack_left, dim3(grid_of(M * (K0 + K1))), dim3(kFpThreads), 0, s, M, K0, K1,
                     A0, lda0, A1, lda1, L, LA);
  return hipGetLastError();
}

hipError_t launch_fp64_pack_right(hipStream_t s, i64 N, i64 K0, i64 K1, const u64* B0, i64 ldb0,
                                  const u64* B1, i64 ldb1, int L, double* RB) {
  if (N * (K0 + K1) <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fp64_pack_right, dim3(grid_of(N * (K0 + K1))), dim3(kFpThreads), 0, s, N, K0, K1,
                     B0, ldb0, B1, ldb1, L, RB);
  return hipGetLastError();
}

hipError_t launch_fp64_combine(hipStream_t s, i64 M, i64 N, int L, const double* X, const Epilogue& ep) {
  if (M * N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fp64_combine, dim3(grid_of(M * N)), dim3(kFpThreads), 0, s, M, N, L, X, ep);
  return hipGetLastError();
}

}  // namespace mpc
