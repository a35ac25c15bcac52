// gemm_plain.hip -- ring GEMM over Z/2^64 on the vector ALUs (the "plain" form).
//
// C = [A0 (+A0add) | A1] @ [B0 (+B0add) ; B1] mod 2^64 for a list of problems
// in one launch.  A 256-thread workgroup computes a 128x64 tile; each thread
// owns an 8x4 register block.  Operand tiles of 16 k are staged through LDS
// (the left tile stored k-major) with the next tile prefetched into registers;
// the LDS tiles are double-buffered, so one barrier per step hands them over.
//
// One ring multiply-accumulate a*b on 32-bit halves a = aL + 2^32 aH,
// b = bL + 2^32 bH:  a*b = aL*bL + 2^32 (aL*bH + aH*bL)  (mod 2^64).  The full
// aL*bL goes into a 64-bit accumulator (v_mad_u64_u32); the cross terms only
// matter modulo 2^32 and go into a 32-bit accumulator that is shifted in once
// at the end.
#include "internal.h"

namespace mpc {
namespace {

constexpr int BM = 128, BN = 64, BK = kPlainBK;
constexpr int TM = 8, TN = 4;
constexpr int kThreads = 256;

__device__ __forceinline__ int find_problem(const int* __restrict__ start, int nprob, int t) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ u64 load_a(const PlainProblem& p, i64 m, i64 k) {
  if (m >= p.M) return 0;
  if (k < p.K0) {
    u64 v = p.A0[m * p.lda0 + k];
    if (p.A0add) v += p.A0add[m * p.lda0 + k];
    return v;
  }
  if (k < p.K0 + p.K1) return p.A1[m * p.lda1 + (k - p.K0)];
  return 0;
}

__device__ __forceinline__ u64 load_b(const PlainProblem& p, i64 k, i64 n) {
  if (n >= p.N) return 0;
  if (k < p.K0) {
    u64 v = p.B0[k * p.ldb0 + n];
    if (p.B0add) v += p.B0add[k * p.ldb0 + n];
    return v;
  }
  if (k < p.K0 + p.K1) return p.B1[(k - p.K0) * p.ldb1 + n];
  return 0;
}

__global__ void __launch_bounds__(kThreads, 2)
    k_plain_gemm(const PlainProblem* __restrict__ probs, TileMap map) {
  // two buffers: a step computes from one while the next step's tiles are
  // stored into the other, so one barrier per step hands them over
  __shared__ u64 As[2][BK][BM];
  __shared__ u64 Bs[2][BK][BN];

  const int t = blockIdx.x;
  const int pi = find_problem(map.tile_start, map.nprob, t);
  const PlainProblem p = probs[pi];
  const int local = t - map.tile_start[pi];
  const int ntn = (int)((p.N + BN - 1) / BN);
  const int tiles_mn = (int)((p.M + BM - 1) / BM) * ntn;
  const int slice = local / tiles_mn, lt = local % tiles_mn;
  const i64 m0 = (i64)(lt / ntn) * BM, n0 = (i64)(lt % ntn) * BN;
  // this workgroup's k range: one slice of a split problem, else all of k
  const i64 kbeg = (i64)slice * p.kslice;
  const i64 Ktot = min(p.K0 + p.K1, kbeg + p.kslice);

  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  // loader coordinates
  const int la_row = tid >> 1, la_k = (tid & 1) * 8;  // 8 consecutive k of one row
  const int lb_k = tid >> 4, lb_n = (tid & 15) * 4;   // 4 consecutive n of one k

  u64 ra[8], rb[4];
  auto fetch = [&](i64 k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) ra[q] = load_a(p, m0 + la_row, k0 + la_k + q);
#pragma unroll
    for (int q = 0; q < 4; ++q) rb[q] = load_b(p, k0 + lb_k, n0 + lb_n + q);
  };

  u64 lo[TM][TN];
  u32 cr[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      lo[i][j] = 0;
      cr[i][j] = 0;
    }

  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 8; ++q) As[buf][la_k + q][la_row] = ra[q];
#pragma unroll
    for (int q = 0; q < 4; ++q) Bs[buf][lb_k][lb_n + q] = rb[q];
  };
  if (kbeg < Ktot) {
    fetch(kbeg);
    store(0);
  }
  __syncthreads();
  int cur = 0;
  for (i64 k0 = kbeg; k0 < Ktot; k0 += BK) {
    // the next step's loads go out first and land during this step's
    // multiply-adds; they are then stored into the other buffer, which every
    // thread finished reading before the previous barrier
    const bool more = k0 + BK < Ktot;
    if (more) fetch(k0 + BK);
#pragma unroll 4
    for (int kk = 0; kk < BK; ++kk) {
      u64 a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[cur][kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[cur][kk][tx + 16 * j];
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
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  if (p.ksplit > 1) {
    // raw slice sum; the reduction adds the slices and applies the epilogue
    u64* part = p.partial + (i64)slice * p.M * p.N;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const i64 m = m0 + ty + 16 * i;
      if (m >= p.M) continue;
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const i64 n = n0 + tx + 16 * j;
        if (n < p.N) part[m * p.N + n] = lo[i][j] + ((u64)cr[i][j] << 32);
      }
    }
    return;
  }
  const Epilogue& ep = p.ep;
  i64 coff[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const i64 n = n0 + tx + 16 * j;
    coff[j] = (n / ep.view.n_div) * ep.view.ld_q + (n % ep.view.n_div);
  }
  // Every added term is loaded before any store, unconditionally (a thread
  // past the product's edge reads its first element, and stores nothing): with
  // a store between two loads, each load would wait for the store before it,
  // since the compiler cannot tell the output from the added terms.  Four
  // rows (16 outputs) at a time, to stay within the registers of two
  // workgroups per compute unit.
  auto ok = [&](int i, int j) { return m0 + ty + 16 * i < p.M && n0 + tx + 16 * j < p.N; };
  auto at = [&](int i, int j) { return ok(i, j) ? (m0 + ty + 16 * i) * ep.view.ld_m + coff[j] : (i64)0; };
  const u64 neg = ep.csign < 0 ? ~(u64)0 : 0;  // -c as (c ^ ~0) + 1
  constexpr int kRows = 4;
#pragma unroll
  for (int i0 = 0; i0 < TM; i0 += kRows) {
    u64 v[kRows][TN];
#pragma unroll
    for (int i = 0; i < kRows; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) v[i][j] = lo[i0 + i][j] + ((u64)cr[i0 + i][j] << 32);
    if (ep.accumulate) {
#pragma unroll
      for (int i = 0; i < kRows; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) v[i][j] += ep.Out[at(i0 + i, j)];
    }
    if (ep.Cadd) {
#pragma unroll
      for (int i = 0; i < kRows; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          v[i][j] += (ep.Cadd[at(i0 + i, j)] ^ neg) + (neg & 1);
    }
#pragma unroll
    for (int i = 0; i < kRows; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        if (ok(i0 + i, j))
          ep.Out[at(i0 + i, j)] = ep.trunc_bits ? (u64)((i64)v[i][j] >> ep.trunc_bits) : v[i][j];
  }
}

__device__ __forceinline__ void reduce_one(const u64* __restrict__ partial, int ks, i64 total, i64 N,
                                           const Epilogue& ep, i64 e) {
  // four independent sums keep several loads in flight (the ring sum does
  // not depend on the order)
  u64 v0 = 0, v1 = 0, v2 = 0, v3 = 0;
  int s = 0;
  for (; s + 4 <= ks; s += 4) {
    v0 += partial[(i64)s * total + e];
    v1 += partial[(i64)(s + 1) * total + e];
    v2 += partial[(i64)(s + 2) * total + e];
    v3 += partial[(i64)(s + 3) * total + e];
  }
  for (; s < ks; ++s) v0 += partial[(i64)s * total + e];
  u64 v = (v0 + v1) + (v2 + v3);
  const i64 m = e / N, n = e % N;
  const i64 off = m * ep.view.ld_m + (n / ep.view.n_div) * ep.view.ld_q + (n % ep.view.n_div);
  if (ep.accumulate) v += ep.Out[off];
  if (ep.Cadd) v += (ep.csign < 0) ? (u64)0 - ep.Cadd[off] : ep.Cadd[off];
  if (ep.trunc_bits) v = (u64)((i64)v >> ep.trunc_bits);
  ep.Out[off] = v;
}

__global__ void __launch_bounds__(kThreads)
    k_splitk_reduce_grouped(const ReduceJob* __restrict__ jobs, const i64* __restrict__ chunk_start, int njobs) {
  const i64 c = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (chunk_start[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  const ReduceJob& jb = jobs[lo];
  const i64 total = jb.M * jb.N;
  const i64 base = (c - chunk_start[lo]) * kReduceChunk;
  const i64 end = min(base + kReduceChunk, total);
  for (i64 e = base + threadIdx.x; e < end; e += kThreads) reduce_one(jb.partial, jb.ks, total, jb.N, jb.ep, e);
}

}  // namespace

hipError_t launch_splitk_reduce_grouped(hipStream_t s, const ReduceJob* jobs, const i64* chunk_start, int njobs,
                                        i64 total_chunks) {
  if (total_chunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_splitk_reduce_grouped, dim3((unsigned)total_chunks), dim3(kThreads), 0, s, jobs,
                     chunk_start, njobs);
  return hipGetLastError();
}

// Whole Beaver matmul of a small product in one launch.  A workgroup owns a
// 4x4 block of outputs of both parties' shares; its 256 threads are those 16
// outputs times 16 lanes of k (k = lane, lane + 16, ...).  Each thread forms
// the opened eps = x - a and delta = y - b of the elements it reads from the
// shares themselves (an open pass and its workspace would cost more than the
// product at this size), accumulates
//   z_0 = eps b_0 + (a_0 + eps) delta,  z_1 = eps b_1 + a_1 delta
// over its k, and the 16 partial sums of an output are added through LDS
// before c_p and the truncation.  Ring sums do not depend on their order.
constexpr int kSmallSide = 4, kSmallOut = kSmallSide * kSmallSide, kSmallKl = kThreads / kSmallOut;

__global__ void __launch_bounds__(kThreads) k_beaver_matmul_small(SmallMatmul s) {
  __shared__ u64 part[2][kSmallKl][kSmallOut];
  const int o = threadIdx.x % kSmallOut, kl = threadIdx.x / kSmallOut;
  const i64 ntn = (s.N + kSmallSide - 1) / kSmallSide;
  const i64 m = (blockIdx.x / ntn) * kSmallSide + o / kSmallSide;
  const i64 n = (blockIdx.x % ntn) * kSmallSide + o % kSmallSide;
  const bool ok = m < s.M && n < s.N;
  u64 z0 = 0, z1 = 0;
  if (ok) {
#pragma unroll 8
    for (i64 k = kl; k < s.K; k += kSmallKl) {
      const i64 ia = m * s.K + k, ib = k * s.N + n;
      const u64 a0 = s.a0[ia], a1 = s.a1[ia], b0 = s.b0[ib], b1 = s.b1[ib];
      const u64 eps = (s.x0[ia] - a0) + (s.x1[ia] - a1);
      const u64 del = (s.y0[ib] - b0) + (s.y1[ib] - b1);
      z0 += eps * b0 + (a0 + eps) * del;
      z1 += eps * b1 + a1 * del;
    }
  }
  part[0][kl][o] = z0;
  part[1][kl][o] = z1;
  __syncthreads();
  if (kl == 0 && ok) {
    u64 v0 = 0, v1 = 0;
#pragma unroll
    for (int q = 0; q < kSmallKl; ++q) {
      v0 += part[0][q][o];
      v1 += part[1][q][o];
    }
    const i64 off = m * s.N + n;
    v0 += s.c0[off];
    v1 += s.c1[off];
    if (s.trunc) {
      v0 = (u64)((i64)v0 >> s.trunc);
      v1 = (u64)((i64)v1 >> s.trunc);
    }
    s.z0[off] = v0;
    s.z1[off] = v1;
  }
}

int plain_tiles(i64 M, i64 N) { return (int)(((M + BM - 1) / BM) * ((N + BN - 1) / BN)); }

hipError_t launch_beaver_matmul_small(hipStream_t s, const SmallMatmul& m) {
  const i64 tiles = ((m.M + kSmallSide - 1) / kSmallSide) * ((m.N + kSmallSide - 1) / kSmallSide);
  if (tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_beaver_matmul_small, dim3((unsigned)tiles), dim3(kThreads), 0, s, m);
  return hipGetLastError();
}

hipError_t launch_plain_gemm(hipStream_t s, const PlainProblem* probs, TileMap map,
                             int total_tiles) {
  if (total_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plain_gemm, dim3(total_tiles), dim3(kThreads), 0, s, probs, map);
  return hipGetLastError();
}

}  // namespace mpc
