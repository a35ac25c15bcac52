// gemm_limb.hip -- bit-exact ring GEMM over Z/2^64 on INT8 matrix cores.
//
// Limbs.  For v in Z/2^64 let u = v + 0x8080808080808080 (mod 2^64) and
// d_i = byte_i(u) - 128 in [-128, 127].  Then v = sum_i d_i 2^(8i) (mod 2^64),
// and the byte pattern of d_i is byte_i(u) ^ 0x80, i.e. the bytes of
// u ^ 0x8080808080808080 read as int8.  For C = A @ B:
//   C = sum_{s=0..7} 2^(8s) X_s (mod 2^64),  X_s = sum_{i+j=s} D_i @ E_j,
// because pairs with i + j >= 8 vanish modulo 2^64: 36 int8 GEMMs per ring
// GEMM.  Each X_s is accumulated exactly in int32 by v_mfma_i32_32x32x32_i8:
// a diagonal has at most 8 pairs of products bounded by 2^14, so K <= 16320
// per launch keeps |X_s| < 2^31 (longer K is split into launches that add
// into the output).  No floating point is involved anywhere.
//
// Packing.  pack kernels turn uint64 operands into the blocked limb layout
// described in internal.h (one 8 KiB block = eight 1 KiB planes of a 32x32
// tile, each plane stored as the 64 lanes' 16-byte MFMA fragments in lane
// order), padding with zeros.  The GEMM then streams whole blocks from global
// memory into LDS with 16-byte loads and reads fragments with conflict-free
// 16-byte LDS reads: no conversion work is left in the GEMM's inner loop.
//
// GEMM.  A 256-thread workgroup (four waves, one per SIMD) owns a 128x64
// output tile; each wave a 64x32 sub-tile held as 2 (row halves) x 8
// (diagonals) 32x32 int32 accumulators (256 accumulation registers).  Per
// 32-wide k step the workgroup stages 4 left and 2 right blocks (48 KiB)
// through a double-buffered LDS ring with one barrier per step, and each wave
// issues 72 MFMAs.  The launch is persistent (one workgroup per CU) and maps
// consecutive tiles of a round to the same XCD so they share its L2.
#include "internal.h"

namespace mpc {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr u64 kLimbBias = 0x8080808080808080ULL;

typedef __attribute__((address_space(1))) const v4i gv4i;

// 16-byte load through the global (not flat) address space, so the wait
// counters of LDS traffic and global traffic stay separate.
__device__ __forceinline__ v4i ld_global16(const uint8_t* p) { return *(gv4i*)p; }

// ------------------------------------------------------------------ packing
constexpr int kPackThreads = 256;  // 4 waves, one 32x32 block each

__device__ __forceinline__ int find_job(const i64* __restrict__ start, int njobs, i64 blk) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ u64 pack_fetch(const PackJob& jb, i64 r, i64 k) {
  if (r >= jb.rows || k >= jb.K) return 0;
  size_t off;
  if (jb.kind == kPackRow) {
    off = (size_t)(r * jb.ld + k);
  } else if (jb.kind == kPackCol) {
    off = (size_t)(k * jb.ld + r);
  } else {
    const i64 b = r / jb.lout, l = r % jb.lout;
    const i64 c = k / jb.ksz, j = k % jb.ksz;
    off = (size_t)((b * jb.cin + c) * jb.len + l * jb.stride + j);
  }
  u64 v = jb.src[off];
  if (jb.add) v += jb.add[off];
  return v;
}

__global__ void __launch_bounds__(kPackThreads)
    k_pack(const PackJob* __restrict__ jobs, const i64* __restrict__ block_start, int njobs) {
  const i64 blk = (i64)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (blk >= block_start[njobs]) return;
  const int lane = threadIdx.x & 63;
  const int ji = find_job(block_start, njobs, blk);
  const PackJob jb = jobs[ji];
  const i64 local = blk - block_start[ji];
  const i64 rb = local / jb.kblocks, kb = local % jb.kblocks;
  const i64 r = rb * 32 + (lane & 31);
  const i64 k0 = kb * 32 + (lane >> 5) * 16;

  u64 d[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) d[q] = (pack_fetch(jb, r, k0 + q) + kLimbBias) ^ kLimbBias;

  uint8_t* out = jb.dst + ((size_t)local << 13) + lane * 16;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    v4i w;
#pragma unroll
    for (int word = 0; word < 4; ++word) {
      u32 x = 0;
#pragma unroll
      for (int by = 0; by < 4; ++by) x |= (u32)((d[word * 4 + by] >> (8 * i)) & 0xff) << (8 * by);
      w[word] = (int)x;
    }
    *(v4i*)(out + i * 1024) = w;
  }
}

// ------------------------------------------------------------------ GEMM
constexpr int kThreads = 256;
constexpr int LBM = 128, LBN = 64;  // output tile
constexpr int kABlocks = LBM / 32, kBBlocks = LBN / 32;
constexpr int kStageBytes = (kABlocks + kBBlocks) * kLimbBlockBytes;  // 48 KiB
constexpr int kLoadsPerThread = kStageBytes / (kThreads * 16);       // 12
constexpr int kGroupM = 8;

__device__ __forceinline__ int find_problem(const int* __restrict__ start, int nprob, int t) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Address of the 16 bytes thread `tid` copies for load q of k-block kg.
__device__ __forceinline__ const uint8_t* stage_src(const LimbProblem& p, i64 tm, i64 tn, int kg,
                                                    int q, int tid) {
  const int bi = q >> 1;                         // block within the stage
  const int within = ((q & 1) << 12) + tid * 16;  // byte within the block
  const bool seg0 = kg < p.kb0;
  const i64 kb = seg0 ? kg : kg - p.kb0;
  const i64 kbs = seg0 ? p.kb0 : p.kb1;
  if (bi < kABlocks) {
    const i64 mb = tm * kABlocks + bi;
    const uint8_t* base = seg0 ? p.PA0 : p.PA1;
    return base + ((size_t)(mb * kbs + kb) << 13) + within;
  }
  const i64 nb = tn * kBBlocks + (bi - kABlocks);
  const uint8_t* base = seg0 ? p.PB0 : p.PB1;
  return base + ((size_t)(nb * kbs + kb) << 13) + within;
}

__global__ void __launch_bounds__(kThreads, 1)
    k_limb_gemm(const LimbProblem* __restrict__ probs, TileMap map, int total_tiles) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];  // 2 stages
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int G = gridDim.x;

  for (int it = 0;; ++it) {
    const int t0 = it * G + blockIdx.x;
    if (t0 >= total_tiles) break;
    // Consecutive tiles of a full round go to the same XCD (blocks are
    // dispatched to XCDs round-robin), so they share that XCD's L2.
    int t = t0;
    if ((it + 1) * G <= total_tiles && (G & 7) == 0) t = it * G + (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);

    const int pi = find_problem(map.tile_start, map.nprob, t);
    const LimbProblem& p = probs[pi];
    const int local = t - map.tile_start[pi];
    const int ntm = (int)((p.M + LBM - 1) / LBM), ntn = (int)((p.N + LBN - 1) / LBN);
    const int per_group = kGroupM * ntn;
    const int group = local / per_group;
    const int first_m = group * kGroupM;
    const int gsize = min(ntm - first_m, kGroupM);
    const int in_group = local % per_group;
    const i64 tm = first_m + in_group % gsize, tn = in_group / gsize;

    v16i acc[2][8];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[r][s][e] = 0;

    const int kbeg = p.kb_begin, nk = p.kb_end - p.kb_begin;
    v4i pre[kLoadsPerThread];
    if (nk > 0) {
#pragma unroll
      for (int q = 0; q < kLoadsPerThread; ++q)
        pre[q] = ld_global16(stage_src(p, tm, tn, kbeg, q, tid));
#pragma unroll
      for (int q = 0; q < kLoadsPerThread; ++q) *(v4i*)(lds + q * 4096 + tid * 16) = pre[q];
      if (nk > 1) {
#pragma unroll
        for (int q = 0; q < kLoadsPerThread; ++q)
          pre[q] = ld_global16(stage_src(p, tm, tn, kbeg + 1, q, tid));
      }
    }
    __syncthreads();

    for (int kk = 0; kk < nk; ++kk) {
      const uint8_t* st = lds + (kk & 1) * kStageBytes;
      v4i bf[8];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        bf[i] = *(const v4i*)(st + (kABlocks + wc) * kLimbBlockBytes + i * 1024 + lane * 16);
      // level l: pairs (i = l, j = s - l) for every diagonal s >= l
#pragma unroll
      for (int l = 0; l < 8; ++l) {
        v4i af[2];
#pragma unroll
        for (int r = 0; r < 2; ++r)
          af[r] = *(const v4i*)(st + (2 * wr + r) * kLimbBlockBytes + l * 1024 + lane * 16);
#pragma unroll
        for (int s = l; s < 8; ++s)
#pragma unroll
          for (int r = 0; r < 2; ++r)
            acc[r][s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[r], bf[s - l], acc[r][s], 0, 0, 0);
      }

      if (kk + 1 < nk) {
        uint8_t* nx = lds + ((kk + 1) & 1) * kStageBytes;
#pragma unroll
        for (int q = 0; q < kLoadsPerThread; ++q) *(v4i*)(nx + q * 4096 + tid * 16) = pre[q];
        if (kk + 2 < nk) {
#pragma unroll
          for (int q = 0; q < kLoadsPerThread; ++q)
            pre[q] = ld_global16(stage_src(p, tm, tn, kbeg + kk + 2, q, tid));
        }
      }
      __syncthreads();
    }

    // Epilogue: C = sum_s 2^(8s) X_s (mod 2^64), then the shared epilogue.
    // 32x32 accumulator layout: lane l, register e holds row
    // 8*(e/4) + 4*(l/32) + e%4 and column l%32 of the 32x32 block.
    const Epilogue& ep = p.ep;
    const i64 n = tn * LBN + wc * 32 + (lane & 31);
    const bool n_ok = n < p.N;
    const i64 coff = (n / ep.view.n_div) * ep.view.ld_q + (n % ep.view.n_div);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const i64 m = tm * LBM + wr * 64 + r * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        u64 v = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) v += (u64)(i64)acc[r][s][e] << (8 * s);
        if (n_ok && m < p.M) {
          const i64 off = m * ep.view.ld_m + coff;
          if (ep.accumulate) v += ep.Out[off];
          if (ep.Cadd) v += (ep.csign < 0) ? (u64)0 - ep.Cadd[off] : ep.Cadd[off];
          if (ep.trunc_bits) v = (u64)((i64)v >> ep.trunc_bits);
          ep.Out[off] = v;
        }
      }
    }
  }
}

bool g_attr_set = false;

}  // namespace

i64 limb_rblocks(i64 rows) {
  const i64 b = (rows + 31) / 32;
  return (b + kLimbRowPad - 1) / kLimbRowPad * kLimbRowPad;
}
i64 limb_kblocks(i64 K) { return (K + 31) / 32; }
int limb_tiles(i64 M, i64 N) { return (int)(((M + LBM - 1) / LBM) * ((N + LBN - 1) / LBN)); }

hipError_t launch_pack(hipStream_t s, const PackJob* jobs, const i64* block_start, int njobs,
                       i64 total_blocks) {
  if (total_blocks <= 0) return hipSuccess;
  const i64 grid = (total_blocks + 3) / 4;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)grid), dim3(kPackThreads), 0, s, jobs, block_start,
                     njobs);
  return hipGetLastError();
}

hipError_t launch_limb_gemm(hipStream_t s, const LimbProblem* probs, TileMap map, int total_tiles,
                            int grid) {
  if (total_tiles <= 0) return hipSuccess;
  if (!g_attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_limb_gemm,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 2 * kStageBytes);
    if (e != hipSuccess) return e;
    g_attr_set = true;
  }
  if (grid > total_tiles) grid = total_tiles;
  hipLaunchKernelGGL(k_limb_gemm, dim3(grid), dim3(kThreads), 2 * kStageBytes, s, probs, map,
                     total_tiles);
  return hipGetLastError();
}

}  // namespace mpc
