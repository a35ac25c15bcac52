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
// (diagonals) 32x32 int32 accumulators (256 accumulation registers).  Each
// wave streams its own fragments from global memory through buffer loads
// (every wave load is one contiguous KiB), with one k step of loads in flight
// behind the 72 MFMAs of the current step: no LDS and no barrier.  One
// workgroup per tile; tiles are remapped so each XCD works on a contiguous
// run of them and shares operand blocks in its L2.
#include "internal.h"

namespace mpc {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr u64 kLimbBias = 0x8080808080808080ULL;


// ------------------------------------------------------------------ packing
constexpr int kPackThreads = 256;  // 4 waves, one 32x32 block each
constexpr int kTPad = 33;          // LDS row stride (elements) of the transpose tile

__device__ __forceinline__ int find_job(const i64* __restrict__ start, int njobs, i64 blk) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// acc[o][q] += coef[o][i] * v
__device__ __forceinline__ void accumulate(u64 (&acc)[kPackMaxOut][16], const PackJob& jb, int i,
                                           int q, u64 v) {
#pragma unroll
  for (int o = 0; o < kPackMaxOut; ++o) {
    const int c = jb.coef[o][i];
    acc[o][q] += c > 0 ? v : (c < 0 ? (u64)0 - v : (u64)0);
  }
}

// Writes one lane's 16 elements (row or col l % 32, k = (l / 32) * 16 + q) of a
// block as signed 8-bit limbs: plane i gets byte i of (v + 0x80..80) ^ 0x80..80.
__device__ __forceinline__ void write_limbs(uint8_t* blockp, int lane, const u64 (&v)[16]) {
  u64 d[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) d[q] = (v[q] + kLimbBias) ^ kLimbBias;
  uint8_t* out = blockp + lane * 16;
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

// One wave packs one 32x32 block of every output of a job.  Right operands
// (COL, IM2COL) are read in the packed lane order directly: for each k the
// 32 lanes of a half-wave read 32 consecutive columns.  Left operands (ROW)
// are read with 32 lanes along a row (coalesced) and transposed through a
// padded LDS tile.
__global__ void __launch_bounds__(kPackThreads)
    k_pack(const PackJob* __restrict__ jobs, const i64* __restrict__ block_start, int njobs) {
  __shared__ u64 tile[4][32 * kTPad];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const i64 blk = (i64)blockIdx.x * 4 + wave;
  if (blk >= block_start[njobs]) return;  // whole wave leaves; only wave-level sync below
  const PackJob& jb = jobs[find_job(block_start, njobs, blk)];
  const i64 local = blk - block_start[find_job(block_start, njobs, blk)];
  const i64 rb = local / jb.kblocks, kb = local % jb.kblocks;
  const size_t boff = (size_t)local << 13;

  u64 acc[kPackMaxOut][16];
#pragma unroll
  for (int o = 0; o < kPackMaxOut; ++o)
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[o][q] = 0;

  if (jb.kind == kPackRow) {
    // load layout: step q covers rows 2q and 2q+1 of the block, k = lane % 32
    const i64 k = kb * 32 + (lane & 31);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const i64 r = rb * 32 + 2 * q + (lane >> 5);
      const bool ok = r < jb.rows && k < jb.K;
      for (int i = 0; i < jb.nin; ++i) {
        const u64 v = ok ? jb.in[i][r * jb.ld + k] : 0;
        accumulate(acc, jb, i, q, v);
      }
    }
    u64* t = tile[wave];
#pragma unroll
    for (int o = 0; o < kPackMaxOut; ++o) {
      if (o >= jb.nout) break;
#pragma unroll
      for (int q = 0; q < 16; ++q) t[(2 * q + (lane >> 5)) * kTPad + (lane & 31)] = acc[o][q];
      __builtin_amdgcn_wave_barrier();
      u64 v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = t[(lane & 31) * kTPad + (lane >> 5) * 16 + q];
      __builtin_amdgcn_wave_barrier();
      write_limbs(jb.dst[o] + boff, lane, v);
    }
    return;
  }

  // right operands: lane covers column n = rb*32 + lane%32, k = kb*32 + (lane/32)*16 + q
  const i64 n = rb * 32 + (lane & 31);
  const i64 k0 = kb * 32 + (lane >> 5) * 16;
  i64 col_base = 0;
  if (jb.kind == kPackIm2col && n < jb.rows) {
    const i64 b = n / jb.lout, l = n % jb.lout;
    col_base = b * jb.cin * jb.len + l * jb.stride;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const i64 k = k0 + q;
    const bool ok = n < jb.rows && k < jb.K;
    i64 off = 0;
    if (ok) off = jb.kind == kPackCol ? k * jb.ld + n : col_base + (k / jb.ksz) * jb.len + k % jb.ksz;
    for (int i = 0; i < jb.nin; ++i) {
      const u64 v = ok ? jb.in[i][off] : 0;
      accumulate(acc, jb, i, q, v);
    }
  }
#pragma unroll
  for (int o = 0; o < kPackMaxOut; ++o)
    if (o < jb.nout) write_limbs(jb.dst[o] + boff, lane, acc[o]);
}

// ------------------------------------------------------------------ GEMM
constexpr int kThreads = 256;
constexpr int LBM = 128, LBN = 64;  // output tile of a workgroup
constexpr int kABlocks = LBM / 32, kBBlocks = LBN / 32;
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

// Buffer resource over `bytes` bytes at `base` (raw, no stride).  Loads go
// through the scalar descriptor with a per-lane byte offset in one VGPR, a
// per-step scalar offset and the plane offset in the instruction's immediate.
constexpr int kBufferWord3 = 0x00020000;  // 32-bit raw data format, gfx9 family

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const uint8_t* base, i64 bytes) {
  const int n = bytes > 0x7fffffff ? 0x7fffffff : (int)bytes;
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, 0, n, kBufferWord3);
}

__device__ __forceinline__ v4i ld_buf(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, soff, 0);
}

// The blocks one wave reads in one problem segment: the strip of its two
// 32-row left blocks (consecutive row blocks, so one descriptor covers both)
// and the strip of its 32-col right block, each kbs blocks of 8 KiB long.
struct SegSrc {
  __amdgpu_buffer_rsrc_t a, b;
  int kbs;
};

__device__ __forceinline__ SegSrc seg_src(const uint8_t* PA, const uint8_t* PB, int kbs, i64 mb0,
                                          i64 nb) {
  SegSrc q;
  const i64 strip = (i64)kbs << 13;
  q.a = make_rsrc(PA + mb0 * strip, 2 * strip);
  q.b = make_rsrc(PB + nb * strip, strip);
  q.kbs = kbs;
  return q;
}

// Scalar offsets of one k step: block kb of the left strip (row half r at
// +r*kbs blocks) and of the right strip.
struct StepOff {
  __amdgpu_buffer_rsrc_t a, b;
  int a0, a1, bo;
};

__device__ __forceinline__ StepOff step_off(const SegSrc& s0, const SegSrc& s1, int kb0, int kg) {
  const bool seg0 = kg < kb0;
  const SegSrc& q = seg0 ? s0 : s1;
  const int kb = seg0 ? kg : kg - kb0;
  StepOff o;
  o.a = q.a;
  o.b = q.b;
  o.a0 = kb << 13;
  o.a1 = (kb + q.kbs) << 13;
  o.bo = kb << 13;
  return o;
}

__device__ __forceinline__ void load_b(v4i (&b)[8], const StepOff& o, unsigned lo) {
#pragma unroll
  for (int i = 0; i < 8; ++i) b[i] = ld_buf(o.b, lo + i * 1024, o.bo);
}

// One 32-wide k step: 72 MFMAs.  Level l multiplies left plane l with right
// planes 0..7-l into diagonals l..7 (for both 32-row halves); consecutive
// MFMAs write different accumulators.  Left plane l is dead after level l, so
// it is reloaded in place for the next step right away (a whole step of
// latency to hide); right plane 0 is used by every level, so the right planes
// are double-buffered by the caller.
__device__ __forceinline__ void mfma_step(v16i (&acc)[2][8], v4i (&a)[2][8], const v4i (&b)[8],
                                          const StepOff& next, unsigned lo) {
#pragma unroll
  for (int l = 0; l < 8; ++l) {
#pragma unroll
    for (int s = l; s < 8; ++s)
#pragma unroll
      for (int r = 0; r < 2; ++r)
        acc[r][s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[r][l], b[s - l], acc[r][s], 0, 0, 0);
    a[0][l] = ld_buf(next.a, lo + l * 1024, next.a0);
    a[1][l] = ld_buf(next.a, lo + l * 1024, next.a1);
    // keep this order: reordering across levels lengthens the fragments'
    // live ranges past the register file
    __builtin_amdgcn_sched_barrier(0);
  }
}

// GEMM over a tile list.  A 256-thread workgroup (one wave per
// SIMD) owns a 128x64 output tile and each wave a 64x32 quarter of it, held
// as 2 (row halves) x 8 (diagonals) 32x32 int32 accumulators.  Each wave
// streams its fragments straight from global memory into two register sets:
// while the MFMAs consume one k step, the loads of the step two ahead are in
// flight, so no LDS traffic and no barrier sit between MFMAs.  The four waves
// of a workgroup read overlapping blocks at about the same time, which the
// CU's L1 and the XCD's L2 serve.
__global__ void __launch_bounds__(kThreads, 1)
    k_limb_gemm(const LimbProblem* __restrict__ probs, TileMap map) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // the wave index is uniform across the wave: keep it (and every address
  // derived from it) in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  // One workgroup per tile.  Workgroups are dispatched to the 8 XCDs
  // round-robin in index order, so index b runs on XCD b % 8; remapping
  // b -> (b % 8) * (G / 8) + b / 8 gives each XCD a contiguous run of tiles,
  // which then share that XCD's L2.
  const int G = gridDim.x, b = blockIdx.x;
  const int G8 = G & ~7;
  {
    const int t = b < G8 ? (b & 7) * (G8 >> 3) + (b >> 3) : b;
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
    const i64 mb0 = tm * kABlocks + 2 * wr;  // this wave's first left block
    const i64 nb = tn * kBBlocks + wc;       // this wave's right block

    v16i acc[2][8];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[r][s][e] = 0;

    const int kbeg = p.kb_begin, nk = p.kb_end - p.kb_begin;
    const unsigned lo = (unsigned)lane * 16u;
    const SegSrc s0 = seg_src(p.PA0, p.PB0, p.kb0, mb0, nb);
    const SegSrc s1 = seg_src(p.PA1 ? p.PA1 : p.PA0, p.PB1 ? p.PB1 : p.PB0, p.kb1, mb0, nb);
    v4i a[2][8], b0[8], b1[8];
    if (nk > 0) {
      const StepOff o = step_off(s0, s1, p.kb0, kbeg);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        a[0][i] = ld_buf(o.a, lo + i * 1024, o.a0);
        a[1][i] = ld_buf(o.a, lo + i * 1024, o.a1);
      }
      load_b(b0, o, lo);
      load_b(b1, step_off(s0, s1, p.kb0, kbeg + min(1, nk - 1)), lo);
    }
    // Steps alternate between the two right-operand buffers; an odd last step
    // runs after the loop so the loop body has no branch.  Loads past the last
    // step re-read the last step's blocks (valid memory, results unused).
    const int klast = kbeg + nk - 1;
    int kk = 0;
    for (; kk + 1 < nk; kk += 2) {
      mfma_step(acc, a, b0, step_off(s0, s1, p.kb0, min(kbeg + kk + 1, klast)), lo);
      load_b(b0, step_off(s0, s1, p.kb0, min(kbeg + kk + 2, klast)), lo);
      mfma_step(acc, a, b1, step_off(s0, s1, p.kb0, min(kbeg + kk + 2, klast)), lo);
      load_b(b1, step_off(s0, s1, p.kb0, min(kbeg + kk + 3, klast)), lo);
    }
    if (kk < nk) mfma_step(acc, a, b0, step_off(s0, s1, p.kb0, klast), lo);

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
                            int /*num_cu*/) {
  if (total_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_limb_gemm, dim3(total_tiles), dim3(kThreads), 0, s, probs, map);
  return hipGetLastError();
}

}  // namespace mpc
