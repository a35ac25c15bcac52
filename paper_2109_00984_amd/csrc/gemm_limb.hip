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

// Pointers into device global memory (global, not flat, instructions).
typedef __attribute__((address_space(1))) const u64 gcu64;
typedef __attribute__((address_space(1))) v4i gv4i;
__device__ __forceinline__ gcu64* gptr(const u64* p) { return (gcu64*)p; }


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

// Writes one lane's 16 elements (row or col l % 32, k = (l / 32) * 16 + q) of a
// block as signed 8-bit limbs: plane i gets byte i of (v + 0x80..80) ^ 0x80..80.
__device__ __forceinline__ void write_limbs(uint8_t* blockp, int lane, const u64 (&v)[16]) {
  u64 d[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) d[q] = (v[q] + kLimbBias) ^ kLimbBias;
  gv4i* out = (gv4i*)(blockp + lane * 16);
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
    out[i * 64] = w;  // plane i starts 1 KiB further
  }
}

template <int MODE> struct Mode;
template <> struct Mode<kModeCopy> {
  static constexpr int nin = 1, nout = 1;
  __device__ static u64 out(int, const u64* v) { return v[0]; }
};
template <> struct Mode<kModeSum2> {
  static constexpr int nin = 2, nout = 1;
  __device__ static u64 out(int, const u64* v) { return v[0] + v[1]; }
};
template <> struct Mode<kModeOpenLeft> {  // x0, x1, a0, a1 -> eps, g0 = a0 + eps, a1
  static constexpr int nin = 4, nout = 3;
  __device__ static u64 out(int o, const u64* v) {
    return o == 0 ? v[0] + v[1] - v[2] - v[3] : o == 1 ? v[0] + v[1] - v[3] : v[3];
  }
};
template <> struct Mode<kModeOpenRight> {  // y0, y1, b0, b1 -> delta, b0, b1
  static constexpr int nin = 4, nout = 3;
  __device__ static u64 out(int o, const u64* v) {
    return o == 0 ? v[0] + v[1] - v[2] - v[3] : o == 1 ? v[2] : v[3];
  }
};

// Element offsets of a lane's 16 loads and whether each is inside the operand.
template <int KIND>
__device__ __forceinline__ void pack_offsets(const PackJob& jb, i64 rb, i64 kb, int lane,
                                             i64 (&off)[16], bool (&ok)[16]) {
  if (KIND == kPackRow) {
    // load layout: step q covers rows 2q and 2q+1 of the block, k = lane % 32
    const i64 k = kb * 32 + (lane & 31);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const i64 r = rb * 32 + 2 * q + (lane >> 5);
      ok[q] = r < jb.rows && k < jb.K;
      off[q] = r * jb.ld + k;
    }
  } else if (KIND == kPackCol) {
    // lane covers column n = rb*32 + lane%32, k = kb*32 + (lane/32)*16 + q
    const i64 n = rb * 32 + (lane & 31);
    const i64 k0 = kb * 32 + (lane >> 5) * 16;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      ok[q] = n < jb.rows && k0 + q < jb.K;
      off[q] = (k0 + q) * jb.ld + n;
    }
  } else {
    // im2col: column n = (b, l), k = (c, j); (c, j) advances incrementally
    const i64 n = rb * 32 + (lane & 31);
    const i64 k0 = kb * 32 + (lane >> 5) * 16;
    const bool n_ok = n < jb.rows;
    const i64 nn = n_ok ? n : 0;
    const i64 b = nn / jb.lout, l = nn % jb.lout;
    i64 c = k0 / jb.ksz, j = k0 % jb.ksz;
    const i64 base = b * jb.cin * jb.len + l * jb.stride;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      ok[q] = n_ok && k0 + q < jb.K;
      off[q] = base + c * jb.len + j;
      if (++j == jb.ksz) {
        j = 0;
        ++c;
      }
    }
  }
}

// One wave packs one 32x32 block of every output of a job; all loads of a
// lane are issued before any is used.  Right operands (COL, IM2COL) are read
// in the packed lane order directly: for each k the 32 lanes of a half-wave
// read 32 consecutive columns.  Left operands (ROW) are read with 32 lanes
// along a row (coalesced) and transposed through a padded LDS tile.
template <int KIND, int MODE>
__global__ void __launch_bounds__(kPackThreads)
    k_pack(const PackJob* __restrict__ jobs, const i64* __restrict__ block_start, int njobs) {
  using Md = Mode<MODE>;
  __shared__ u64 tile[4][32 * kTPad];
  // the wave index is uniform across the wave: everything derived from the
  // block index (job, block coordinates, the interior test) stays scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const i64 blk = (i64)blockIdx.x * 4 + wave;
  if (blk >= block_start[njobs]) return;  // whole wave leaves; only wave-level sync below
  const int ji = find_job(block_start, njobs, blk);
  const PackJob& jb = jobs[ji];
  const i64 local = blk - block_start[ji];
  const i64 rb = local / jb.kblocks, kb = local % jb.kblocks;
  const size_t boff = (size_t)local << 13;

  i64 off[16];
  bool ok[16];
  pack_offsets<KIND>(jb, rb, kb, lane, off, ok);
  gcu64* in[Md::nin];
#pragma unroll
  for (int i = 0; i < Md::nin; ++i) in[i] = gptr(jb.in[i]);
  const bool interior = (rb + 1) * 32 <= jb.rows && (kb + 1) * 32 <= jb.K;
  u64 v[16][Md::nin];
  if (interior) {
#pragma unroll
    for (int q = 0; q < 16; ++q)
#pragma unroll
      for (int i = 0; i < Md::nin; ++i) v[q][i] = in[i][off[q]];
  } else {
#pragma unroll
    for (int q = 0; q < 16; ++q)
#pragma unroll
      for (int i = 0; i < Md::nin; ++i) v[q][i] = ok[q] ? in[i][off[q]] : 0;
  }

#pragma unroll
  for (int o = 0; o < Md::nout; ++o) {
    u64 w[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) w[q] = Md::out(o, v[q]);
    if (KIND == kPackRow) {
      u64* t = tile[wave];
#pragma unroll
      for (int q = 0; q < 16; ++q) t[(2 * q + (lane >> 5)) * kTPad + (lane & 31)] = w[q];
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int q = 0; q < 16; ++q) w[q] = t[(lane & 31) * kTPad + (lane >> 5) * 16 + q];
      __builtin_amdgcn_wave_barrier();
    }
    write_limbs(jb.dst[o] + boff, lane, w);
  }
}

// ------------------------------------------------------------------ GEMM
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

// Wave tile of SA left x SB right 32-blocks (SA, SB in {1, 2}, SA*SB <= 2);
// the workgroup's four waves form a 2x2 grid, so its output tile is
// (64*SA) x (64*SB).  The operand with more blocks per wave ("outer") is
// iterated by level and reloaded in place; the other ("inner") is
// double-buffered, because its plane 0 is used by every level.
template <int SA, int SB>
struct Shape {
  static constexpr int BM = 64 * SA, BN = 64 * SB;
  static constexpr bool kOuterA = SA >= SB;
  static constexpr int SO = kOuterA ? SA : SB, SI = kOuterA ? SB : SA;
  static constexpr int kOcc = SA * SB == 1 ? 2 : 1;  // workgroups per CU the registers allow
};

// The blocks one wave reads in one problem segment: its strips of left and
// right blocks, each block kbs k-blocks of 8 KiB long; consecutive row (col)
// blocks are consecutive strips, so one descriptor covers a wave's strips.
struct SegSrc {
  __amdgpu_buffer_rsrc_t a, b;
  int kbs;
};

__device__ __forceinline__ SegSrc seg_src(const uint8_t* PA, const uint8_t* PB, int kbs, i64 mb0,
                                          i64 nb0, int sa, int sb) {
  SegSrc q;
  const i64 strip = (i64)kbs << 13;
  q.a = make_rsrc(PA + mb0 * strip, sa * strip);
  q.b = make_rsrc(PB + nb0 * strip, sb * strip);
  q.kbs = kbs;
  return q;
}

// Descriptors and scalar byte offsets of k-block kg (block r of a strip at
// +r*kbs blocks).
struct StepOff {
  __amdgpu_buffer_rsrc_t a, b;
  int kb, kbs;
  __device__ int off(int r) const { return (kb + r * kbs) << 13; }
};

__device__ __forceinline__ StepOff step_off(const SegSrc& s0, const SegSrc& s1, int kb0, int kg) {
  const bool seg0 = kg < kb0;
  const SegSrc& q = seg0 ? s0 : s1;
  StepOff o;
  o.a = q.a;
  o.b = q.b;
  o.kb = seg0 ? kg : kg - kb0;
  o.kbs = q.kbs;
  return o;
}

template <int S>
__device__ __forceinline__ void load_blocks(v4i (&f)[S][8], __amdgpu_buffer_rsrc_t r, const StepOff& o,
                                            unsigned lo) {
#pragma unroll
  for (int x = 0; x < S; ++x)
#pragma unroll
    for (int i = 0; i < 8; ++i) f[x][i] = ld_buf(r, lo + i * 1024, o.off(x));
}

// One 32-wide k step: 36 MFMAs per (left block, right block) pair.  Level l
// multiplies outer plane l with inner planes 0..7-l into diagonals l..7;
// consecutive MFMAs write different accumulators.  Outer plane l is dead after
// level l and is reloaded in place for the next step right away.
template <int SA, int SB, int SO, int SI>
__device__ __forceinline__ void mfma_step(v16i (&acc)[SA][SB][8], v4i (&outer)[SO][8],
                                          const v4i (&inner)[SI][8], const StepOff& next,
                                          unsigned lo) {
  using S = Shape<SA, SB>;
#pragma unroll
  for (int l = 0; l < 8; ++l) {
#pragma unroll
    for (int s = l; s < 8; ++s)
#pragma unroll
      for (int o = 0; o < S::SO; ++o)
#pragma unroll
        for (int i = 0; i < S::SI; ++i) {
          if (S::kOuterA)
            acc[o][i][s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(outer[o][l], inner[i][s - l], acc[o][i][s], 0, 0, 0);
          else
            acc[i][o][s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(inner[i][s - l], outer[o][l], acc[i][o][s], 0, 0, 0);
        }
#pragma unroll
    for (int o = 0; o < S::SO; ++o)
      outer[o][l] = ld_buf(S::kOuterA ? next.a : next.b, lo + l * 1024, next.off(o));
    // keep this order: reordering across levels lengthens the fragments'
    // live ranges past the register file
    __builtin_amdgcn_sched_barrier(0);
  }
}

// GEMM over a tile list.  Each wave streams its fragments straight from
// global memory (buffer loads, each wave load one contiguous KiB): the outer
// planes are reloaded one step ahead right after their last use, the inner
// planes are double-buffered, so no LDS traffic and no barrier sit between
// MFMAs.  The four waves of a workgroup read overlapping blocks at about the
// same time, which the CU's L1 and the XCD's L2 serve.
template <int SA, int SB>
__global__ void __launch_bounds__(kThreads, (Shape<SA, SB>::kOcc))
    k_limb_gemm(const LimbProblem* __restrict__ probs, TileMap map, TileSched sched) {
  using S = Shape<SA, SB>;
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
  const int t = (sched.xcd_remap && b < G8) ? (b & 7) * (G8 >> 3) + (b >> 3) : b;
  const int pi = find_problem(map.tile_start, map.nprob, t);
  const LimbProblem& p = probs[pi];
  const int local = t - map.tile_start[pi];
  // grouped raster: runs of group_m tile rows, column by column
  const int ntm = (int)((p.M + S::BM - 1) / S::BM), ntn = (int)((p.N + S::BN - 1) / S::BN);
  const int gm = sched.group_m;
  const int per_group = gm * ntn;
  const int first_m = (local / per_group) * gm;
  const int gsize = min(ntm - first_m, gm);
  const int in_group = local % per_group;
  const i64 tm = first_m + in_group % gsize, tn = in_group / gsize;
  const i64 mb0 = tm * 2 * SA + wr * SA;  // this wave's first left block
  const i64 nb0 = tn * 2 * SB + wc * SB;  // this wave's first right block

  v16i acc[SA][SB][8];
#pragma unroll
  for (int x = 0; x < SA; ++x)
#pragma unroll
    for (int y = 0; y < SB; ++y)
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[x][y][s][e] = 0;

  const int kbeg = p.kb_begin, nk = p.kb_end - p.kb_begin;
  const unsigned lo = (unsigned)lane * 16u;
  const SegSrc s0 = seg_src(p.PA0, p.PB0, p.kb0, mb0, nb0, SA, SB);
  const SegSrc s1 = seg_src(p.PA1 ? p.PA1 : p.PA0, p.PB1 ? p.PB1 : p.PB0, p.kb1, mb0, nb0, SA, SB);
  v4i outer[S::SO][8], in0[S::SI][8], in1[S::SI][8];
  if (nk > 0) {
    const StepOff o = step_off(s0, s1, p.kb0, kbeg);
    const StepOff o1 = step_off(s0, s1, p.kb0, kbeg + min(1, nk - 1));
    load_blocks<S::SO>(outer, S::kOuterA ? o.a : o.b, o, lo);
    load_blocks<S::SI>(in0, S::kOuterA ? o.b : o.a, o, lo);
    load_blocks<S::SI>(in1, S::kOuterA ? o1.b : o1.a, o1, lo);
  }
  // Steps alternate between the two inner buffers; an odd last step runs
  // after the loop so the loop body has no branch.  Loads past the last step
  // re-read the last step's blocks (valid memory, results unused).
  const int klast = kbeg + nk - 1;
  int kk = 0;
  for (; kk + 1 < nk; kk += 2) {
    mfma_step<SA, SB, S::SO, S::SI>(acc, outer, in0, step_off(s0, s1, p.kb0, min(kbeg + kk + 1, klast)), lo);
    {
      const StepOff o = step_off(s0, s1, p.kb0, min(kbeg + kk + 2, klast));
      load_blocks<S::SI>(in0, S::kOuterA ? o.b : o.a, o, lo);
    }
    mfma_step<SA, SB, S::SO, S::SI>(acc, outer, in1, step_off(s0, s1, p.kb0, min(kbeg + kk + 2, klast)), lo);
    {
      const StepOff o = step_off(s0, s1, p.kb0, min(kbeg + kk + 3, klast));
      load_blocks<S::SI>(in1, S::kOuterA ? o.b : o.a, o, lo);
    }
  }
  if (kk < nk) mfma_step<SA, SB, S::SO, S::SI>(acc, outer, in0, step_off(s0, s1, p.kb0, klast), lo);

  // Epilogue: C = sum_s 2^(8s) X_s (mod 2^64), then the shared epilogue.
  // 32x32 accumulator layout: lane l, register e holds row
  // 8*(e/4) + 4*(l/32) + e%4 and column l%32 of the 32x32 block.
  const Epilogue& ep = p.ep;
#pragma unroll
  for (int y = 0; y < SB; ++y) {
    const i64 n = tn * S::BN + (wc * SB + y) * 32 + (lane & 31);
    const bool n_ok = n < p.N;
    const i64 coff = (n / ep.view.n_div) * ep.view.ld_q + (n % ep.view.n_div);
#pragma unroll
    for (int x = 0; x < SA; ++x) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const i64 m = tm * S::BM + (wr * SA + x) * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        u64 v = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) v += (u64)(i64)acc[x][y][s][e] << (8 * s);
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
int limb_tiles(i64 M, i64 N, int variant) {
  const i64 bm = 64 * limb_variant_sa(variant), bn = 64 * limb_variant_sb(variant);
  return (int)(((M + bm - 1) / bm) * ((N + bn - 1) / bn));
}
int limb_variant_sa(int variant) { return variant == kLimb128x64 ? 2 : 1; }
int limb_variant_sb(int variant) { return variant == kLimb64x128 ? 2 : 1; }

hipError_t launch_pack(hipStream_t s, const PackJob* jobs, const i64* block_start, int njobs,
                       i64 total_blocks, int kind, int mode) {
  if (total_blocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)((total_blocks + 3) / 4)), block(kPackThreads);
#define MPC_PACK_CASE(K, MO)                                                            \
  if (kind == K && mode == MO) {                                                         \
    hipLaunchKernelGGL((k_pack<K, MO>), grid, block, 0, s, jobs, block_start, njobs);   \
    return hipGetLastError();                                                            \
  }
  MPC_PACK_CASE(kPackRow, kModeCopy)
  MPC_PACK_CASE(kPackRow, kModeSum2)
  MPC_PACK_CASE(kPackRow, kModeOpenLeft)
  MPC_PACK_CASE(kPackRow, kModeOpenRight)
  MPC_PACK_CASE(kPackCol, kModeCopy)
  MPC_PACK_CASE(kPackCol, kModeSum2)
  MPC_PACK_CASE(kPackCol, kModeOpenRight)
  MPC_PACK_CASE(kPackIm2col, kModeSum2)
  MPC_PACK_CASE(kPackIm2col, kModeOpenLeft)
#undef MPC_PACK_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_limb_gemm(hipStream_t s, const LimbProblem* probs, TileMap map, int total_tiles,
                            TileSched sched) {
  if (total_tiles <= 0) return hipSuccess;
  if (sched.group_m < 1) sched.group_m = 1;
  const dim3 grid(total_tiles), block(kThreads);
  switch (sched.variant) {
    case kLimb128x64: hipLaunchKernelGGL((k_limb_gemm<2, 1>), grid, block, 0, s, probs, map, sched); break;
    case kLimb64x128: hipLaunchKernelGGL((k_limb_gemm<1, 2>), grid, block, 0, s, probs, map, sched); break;
    case kLimb64x64: hipLaunchKernelGGL((k_limb_gemm<1, 1>), grid, block, 0, s, probs, map, sched); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mpc
