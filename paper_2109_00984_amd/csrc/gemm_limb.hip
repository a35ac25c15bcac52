// gemm_limb.hip -- bit-exact ring GEMM over Z/2^64 on INT8 matrix cores.
//
// Limbs.  For v in Z/2^64 let u = v + 0x8080808080808080 (mod 2^64) and
// d_i = byte_i(u) - 128 in [-128, 127].  Then v = sum_i d_i 2^(8i) (mod 2^64),
// and the byte pattern of d_i is byte_i(u) ^ 0x80, i.e. the bytes of
// u ^ 0x8080808080808080 read as int8.  For C = A @ B:
//   C = sum_{s=0..7} 2^(8s) X_s (mod 2^64),  X_s = sum_{i+j=s} D_i @ E_j,
// because pairs with i + j >= 8 vanish modulo 2^64: 36 int8 GEMMs per ring
// GEMM.  Each X_s is accumulated exactly in int32 by v_mfma_i32_16x16x64_i8:
// a diagonal has at most 8 pairs of products bounded by 2^14, so K <= 16320
// per launch keeps |X_s| < 2^31 (longer K is split into launches that add
// into the output).  No floating point is involved anywhere.
//
// Packing.  pack kernels turn uint64 operands into the blocked limb layout
// described in internal.h (one 8 KiB block = eight 1 KiB planes of a 32x32
// tile, each plane stored as 64 lanes' 16-byte runs in lane order), with
// zeros past K, so no conversion work is left in the GEMM's inner loop.
//
// GEMM.  A workgroup of four waves (one per SIMD; eight for two of the LDS
// shapes) owns one output tile of 64x64, 64x128 or 128x64; each wave a
// sub-tile held as 16x16 blocks with 8 diagonal int32 accumulators each (256
// accumulation registers for a 32x64 or 64x32 sub-tile, 128 for 32x32).
// Operand blocks are read through buffer descriptors, whose 32-bit range
// bounds one k segment to 65534 k-blocks (the host refuses longer ones).
// Two forms:
// k_limb_gemm, where each wave streams its own fragments from global memory
// through buffer loads, one k step of loads in flight behind the MFMAs of the
// current step, with no LDS and no barrier; and k_limb_gemm_lds, where the
// operand with more fragments per wave is copied once per workgroup into LDS
// (its 64x64 tile runs two workgroups per CU).  One workgroup per tile; tiles
// are remapped so the tiles an XCD holds at a time are neighbours sharing
// operand blocks in its L2.  The 16x16x64 instruction sustains a higher rate
// than 32x32x32 on this chip, with uniformly random operands as well as
// constant ones.
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


// Constant-memory views of a launch's descriptor tables (PackTables,
// GemmTables): inline entries are read from the kernel-argument segment,
// uploaded ones through the same constant address space, so that every
// access is a scalar load.  Each kernel takes its table struct as its only
// argument, so the struct starts the segment.  (The host compilation pass
// only parses the kernels; it gets plain pointers, which it can copy through.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using cptr = __attribute__((address_space(4))) const T*;
#define MPC_KERNARG_PTR() __builtin_amdgcn_kernarg_segment_ptr()
#else
template <class T>
using cptr = const T*;
#define MPC_KERNARG_PTR() nullptr
#endif

struct PackView {
  cptr<PackJob> jobs;
  cptr<i64> bstart;
  int njobs;
};
__device__ __forceinline__ PackView pack_view() {
  const cptr<PackTables> t = (cptr<PackTables>)MPC_KERNARG_PTR();
  PackView v;
  v.njobs = t->njobs;
  v.jobs = t->jobs ? (cptr<PackJob>)(uintptr_t)t->jobs : t->ijobs;
  v.bstart = t->jobs ? (cptr<i64>)(uintptr_t)t->block_start : t->ibstart;
  return v;
}

struct GemmView {
  cptr<LimbProblem> probs;
  cptr<int> tile_start;
  int nprob;
  TileSched sched;
  unsigned* queue;
};
__device__ __forceinline__ GemmView gemm_view() {
  const cptr<GemmTables> t = (cptr<GemmTables>)MPC_KERNARG_PTR();
  GemmView v;
  v.nprob = t->map.nprob;
  v.sched = t->sched;
  v.queue = t->queue;
  v.probs = t->probs ? (cptr<LimbProblem>)(uintptr_t)t->probs : t->iprobs;
  v.tile_start = t->probs ? (cptr<int>)(uintptr_t)t->map.tile_start : t->itile_start;
  return v;
}

// ------------------------------------------------------------------ packing
constexpr int kPackThreads = 256;  // 4 waves, one 32x32 block each
constexpr int kTPad = 33;          // LDS row stride (elements) of the transpose tile

__device__ __forceinline__ int find_job(cptr<i64> start, int njobs, i64 blk) {
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
template <> struct Mode<kModePrgSum2> {  // v0, v1 drawn from the PRG -> v0 + v1
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
template <> struct Mode<kModePrgSum2A> {  // PRG v0, v1 -> v0 + v1, v1
  static constexpr int nin = 2, nout = 2;
  __device__ static u64 out(int o, const u64* v) { return o == 0 ? v[0] + v[1] : v[1]; }
};
template <> struct Mode<kModePrgSum2B> {  // PRG v0, v1 -> v0 + v1, v0, v1
  static constexpr int nin = 2, nout = 3;
  __device__ static u64 out(int o, const u64* v) { return o == 0 ? v[0] + v[1] : o == 1 ? v[0] : v[1]; }
};
template <> struct Mode<kModeOpenLeft2> {  // x0, x1, a0, a1 -> eps, g0 = a0 + eps
  static constexpr int nin = 4, nout = 2;
  __device__ static u64 out(int o, const u64* v) { return o == 0 ? v[0] + v[1] - v[2] - v[3] : v[0] + v[1] - v[3]; }
};
template <> struct Mode<kModeOpenRight1> {  // y0, y1, b0, b1 -> delta
  static constexpr int nin = 4, nout = 1;
  __device__ static u64 out(int, const u64* v) { return v[0] + v[1] - v[2] - v[3]; }
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
__global__ void __launch_bounds__(kPackThreads) k_pack(PackTables) {
  using Md = Mode<MODE>;
  const PackView tv = pack_view();
  const cptr<i64> block_start = tv.bstart;
  const int njobs = tv.njobs;
  __shared__ u64 tile[4][32 * kTPad];
  // the wave index is uniform across the wave: everything derived from the
  // block index (job, block coordinates, the interior test) stays scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const i64 blk = (i64)blockIdx.x * 4 + wave;
  if (blk >= block_start[njobs]) return;  // whole wave leaves; only wave-level sync below
  const int ji = find_job(block_start, njobs, blk);
  const PackJob jb = tv.jobs[ji];
  const i64 local = blk - block_start[ji];
  // Traversal order: the waves of a workgroup take neighbouring blocks along
  // the operand's rows in memory, so that together they read contiguous runs
  // of each row: k-blocks for a left operand (rows are m, contiguous in k),
  // row blocks for a right one (rows are k, contiguous in n).  The packed
  // layout is the same either way: block (rb, kb) at rb * kblocks + kb.
  const i64 rb = KIND == kPackRow ? local / jb.kblocks : local % jb.rreal;
  const i64 kb = KIND == kPackRow ? local % jb.kblocks : local / jb.rreal;
  const size_t boff = (size_t)(rb * jb.kblocks + kb) << 13;

  i64 off[16];
  bool ok[16];
  pack_offsets<KIND>(jb, rb, kb, lane, off, ok);
  gcu64* in[Md::nin];
#pragma unroll
  for (int i = 0; i < Md::nin; ++i) in[i] = gptr(jb.in[i]);
  const bool interior = (rb + 1) * 32 <= jb.rows && (kb + 1) * 32 <= jb.K;
  u64 v[16][Md::nin];
  if constexpr (MODE == kModePrgSum2 || MODE == kModePrgSum2A || MODE == kModePrgSum2B) {
    // the shares are the PRG at each element's row-major offset; write them
    // out in this (coalesced) load layout
#pragma unroll
    for (int q = 0; q < 16; ++q)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        v[q][i] = ok[q] ? sm_out(jb.key[i], (u64)off[q]) : 0;
        if (ok[q]) jb.share[i][off[q]] = v[q][i];
      }
  } else if (interior) {
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

__device__ __forceinline__ int find_problem(cptr<int> start, int nprob, int t) {
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
// (64*SA) x (64*SB).  The MFMA unit is v_mfma_i32_16x16x64_i8, so a wave
// holds HA = 2*SA by HB = 2*SB blocks of 16x16 outputs, each with 8 diagonal
// accumulators of 4 registers.  The operand with more 16-halves per wave
// ("outer") is iterated by level and each of its planes is reloaded in place
// right after its last use; the other ("inner") keeps planes 3..7 the same
// way, while its planes 0..2, used by the last levels of a step, are
// double-buffered.
template <int SA, int SB>
struct Shape {
  static constexpr int BM = 64 * SA, BN = 64 * SB;
  static constexpr int HA = 2 * SA, HB = 2 * SB;
  static constexpr bool kOuterA = SA >= SB;
  static constexpr int HO = kOuterA ? HA : HB, HI = kOuterA ? HB : HA;
  static constexpr int kDbl = 3;  // inner planes 0..kDbl-1 are double-buffered
};

// The blocks one wave reads in one problem segment: its strips of left and
// right 32-blocks, each strip kbs k-blocks of 8 KiB long; consecutive row
// (col) blocks are consecutive strips, so one descriptor covers a wave's
// strips.
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

// Descriptors and scalar byte offsets of the k step starting at k-block kg
// (32-block x of a strip sits at +x*kbs blocks).
struct StepOff {
  __amdgpu_buffer_rsrc_t a, b;
  int kb, kbs;
  __device__ int off(int x) const { return (kb + x * kbs) << 13; }
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

// A 16x16x64 fragment is gathered from two consecutive 32x32 planes (k-blocks
// kb and kb+1): lane l takes rows (or cols) 16*h + l%16 and 16 k values of
// group g = l/16, i.e. k-block kb + g/2, plane lane 16*h + l%16 + 32*(g%2).
// The k order inside a step is the same for both operands, which is all the
// product needs.  lane_off = (g/2)*8192 + (g%2)*512 + (l%16)*16; half h and
// plane i add h*256 + i*1024, which go into the scalar offset so that every
// load of a wave shares the one lane-offset register.
struct LaneOff {
  unsigned lo;
  __device__ static int sub(int h, int i) { return (h & 1) * 256 + i * 1024; }
};

__device__ __forceinline__ v4i ld_frag(__amdgpu_buffer_rsrc_t r, const LaneOff& lo, const StepOff& o,
                                       int h, int i) {
  return ld_buf(r, lo.lo, o.off(h >> 1) + LaneOff::sub(h, i));
}

// acc += A @ B on one 16x16x64 int8 tile, accumulating in place.  Written as
// inline assembly so that the accumulator stays in the same four AGPRs from
// one MFMA to the next (the compiler's own form of this instruction takes a
// fresh destination and then copies it back).  Ordering: the operands come
// from buffer loads, which the compiler's wait-count pass covers; two MFMAs
// into the same accumulator are at least HO*HI MFMAs apart in the step below,
// and the first MFMA of every accumulator takes the literal 0 as its input, so
// no VALU write precedes an MFMA read.
__device__ __forceinline__ void mfma16(v4i& acc, const v4i& a, const v4i& b) {
  asm volatile("v_mfma_i32_16x16x64_i8 %0, %1, %2, %0" : "+a"(acc) : "v"(a), "v"(b));
}
__device__ __forceinline__ void mfma16_first(v4i& acc, const v4i& a, const v4i& b) {
  asm volatile("v_mfma_i32_16x16x64_i8 %0, %1, %2, 0" : "=a"(acc) : "v"(a), "v"(b));
}

// One 64-wide k step: 36 MFMAs per (left half, right half) pair.  Level l
// multiplies outer plane l with inner planes 0..7-l into diagonals l..7.
//
// Loads are spread evenly over the MFMAs rather than issued in bursts: the
// four waves of a CU share one vector-memory pipeline, and a burst stalls
// every wave's in-order issue (MFMAs included) until the pipeline accepts it.
// Level L reloads the registers freed by level L-1: outer plane L-1 and inner
// plane 8-L (for the next step); level 0 reloads outer plane 7 for this step
// (freed by the previous step's level 7) and fills the next step's
// double-buffered inner planes.
// (HO, HI, ND repeat Shape<SA, SB>'s HO, HI, kDbl: array bounds in a
// parameter list cannot depend on the template's own members.)
// Registers of one wave's k loop, bundled so the compile-time-indexed helpers
// below take one reference.
template <int SA, int SB>
struct StepRegs {
  using S = Shape<SA, SB>;
  v4i (&acc)[2 * SA][2 * SB][8];
  v4i (&outer)[S::HO][8];
  v4i (&inner)[S::HI][8];
  const v4i (&dcur)[S::HI][S::kDbl];
  v4i (&dnext)[S::HI][S::kDbl];
};

// Load number Q of level L (see mfma_step).
template <int SA, int SB, bool FIRST, int L, int Q>
__device__ __forceinline__ void level_load(StepRegs<SA, SB>& r, const StepOff& cur, const StepOff& next,
                                           const LaneOff& lo) {
  using S = Shape<SA, SB>;
  constexpr int HO = S::HO, ND = S::kDbl;
  if constexpr (L == 0) {
    constexpr int NO = FIRST ? 0 : HO;  // the first step's planes come from the prologue
    if constexpr (Q < NO) {
      r.outer[Q][7] = ld_frag(S::kOuterA ? cur.a : cur.b, lo, cur, Q, 7);
    } else {
      constexpr int D = Q - NO;
      r.dnext[D / ND][D % ND] = ld_frag(S::kOuterA ? next.b : next.a, lo, next, D / ND, D % ND);
    }
  } else if constexpr (Q < HO) {
    r.outer[Q][L - 1] = ld_frag(S::kOuterA ? next.a : next.b, lo, next, Q, L - 1);
  } else {
    r.inner[Q - HO][8 - L] = ld_frag(S::kOuterA ? next.b : next.a, lo, next, Q - HO, 8 - L);
  }
}

// MFMA number M (0-based) of level L, then the load that falls after it, then
// the rest of the level.  MFMA M multiplies outer plane L of half o with inner
// plane s - L of half i into diagonal s; the level's NL loads sit at the ends
// of NL + 1 equal fractions of its NM MFMAs (NL < NM: at most one per MFMA).
template <int SA, int SB, bool FIRST, int L, int M>
__device__ __forceinline__ void mfma_level(StepRegs<SA, SB>& r, const StepOff& cur, const StepOff& next,
                                           const LaneOff& lo) {
  using S = Shape<SA, SB>;
  constexpr int HO = S::HO, HI = S::HI, ND = S::kDbl;
  constexpr int NM = (8 - L) * HO * HI;
  if constexpr (M < NM) {
    constexpr int s = L + M / (HO * HI), o = (M / HI) % HO, i = M % HI;
    const v4i& in = (s - L) < ND ? r.dcur[i][(s - L) % ND] : r.inner[i][s - L];
    v4i& c = S::kOuterA ? r.acc[o][i][s] : r.acc[i][o][s];
    const v4i& a = S::kOuterA ? r.outer[o][L] : in;
    const v4i& b = S::kOuterA ? in : r.outer[o][L];
    if constexpr (FIRST && L == 0) mfma16_first(c, a, b);
    else mfma16(c, a, b);
    constexpr int NL = L == 0 ? (FIRST ? 0 : HO) + HI * ND : HO + (8 - L >= ND ? HI : 0);
    constexpr int Q = (M + 1) * (NL + 1) / NM - 1, QPREV = M * (NL + 1) / NM - 1;
    if constexpr (Q >= 0 && Q < NL && Q != QPREV) {
      __builtin_amdgcn_sched_barrier(0);
      level_load<SA, SB, FIRST, L, Q>(r, cur, next, lo);
      __builtin_amdgcn_sched_barrier(0);
    }
    mfma_level<SA, SB, FIRST, L, M + 1>(r, cur, next, lo);
  }
}

template <int SA, int SB, bool FIRST, int L>
__device__ __forceinline__ void mfma_levels(StepRegs<SA, SB>& r, const StepOff& cur, const StepOff& next,
                                            const LaneOff& lo) {
  if constexpr (L < 8) {
    mfma_level<SA, SB, FIRST, L, 0>(r, cur, next, lo);
    // keep this order: reordering across levels lengthens the fragments'
    // live ranges past the register file
    __builtin_amdgcn_sched_barrier(0);
    mfma_levels<SA, SB, FIRST, L + 1>(r, cur, next, lo);
  }
}

// One 64-wide k step: 36 MFMAs per (left half, right half) pair.  Level l
// multiplies outer plane l with inner planes 0..7-l into diagonals l..7.
//
// Loads are spread evenly over the MFMAs rather than issued in bursts: the
// four waves of a CU share one vector-memory pipeline, and a burst stalls
// every wave's in-order issue (MFMAs included) until the pipeline accepts it.
// Level L reloads the registers freed by level L-1: outer plane L-1 and inner
// plane 8-L (for the next step); level 0 reloads outer plane 7 for this step
// (freed by the previous step's level 7) and fills the next step's
// double-buffered inner planes.
template <int SA, int SB, bool FIRST>
__device__ __forceinline__ void mfma_step(StepRegs<SA, SB> r, const StepOff& cur, const StepOff& next,
                                          const LaneOff& lo) {
  mfma_levels<SA, SB, FIRST, 0>(r, cur, next, lo);
}

// Output tile of this workgroup.  One workgroup per tile.  Workgroups are
// dispatched to the 8 XCDs round-robin in index order, so index b runs on XCD
// b % 8 as that XCD's (b / 8)-th workgroup.  With the remap, each XCD takes
// runs of `run` consecutive tiles, the tiles it holds at one time (its 32
// compute units times the workgroups per unit), the runs going round the XCDs
// in turn: the tiles an XCD runs together are neighbours that share operand
// blocks in its L2, and when tiles differ in cost (a grouped launch lists its
// longest problems first) every XCD gets its share of each kind.  Inside a
// problem the tiles follow a grouped raster: runs of group_m tile rows, column
// by column.
constexpr int kXcds = 8, kXcdCUs = 32;

__device__ __forceinline__ int remap_tile(int b, int G, int run) {
  const int span = kXcds * run;
  if (b >= G / span * span) return b;  // the last partial round keeps dispatch order
  const int x = b % kXcds, j = b / kXcds;
  return ((j / run) * kXcds + x) * run + j % run;
}

struct TilePos {
  int pi;
  i64 tm, tn;
};

// This workgroup's problem and its tile index inside that problem.
template <int PER_CU>
__device__ __forceinline__ void tile_of(const GemmView& v, int& pi, i64& local) {
  const int b = blockIdx.x;
  const int t = v.sched.xcd_remap ? remap_tile(b, gridDim.x, kXcdCUs * PER_CU) : b;
  pi = find_problem(v.tile_start, v.nprob, t);
  local = t - v.tile_start[pi];
}

// Tile coordinates of tile `local` of problem pi for a BM x BN tile.
template <int BM, int BN>
__device__ __forceinline__ TilePos tile_coords(const GemmView& v, int pi, i64 local) {
  TilePos q;
  q.pi = pi;
  const i64 M = v.probs[pi].M, N = v.probs[pi].N;
  const i64 ntm = (M + BM - 1) / BM, ntn = (N + BN - 1) / BN;
  const i64 gm = v.sched.group_m;  // 1..64, checked by the host
  const i64 per_group = gm * ntn;
  const i64 first_m = (local / per_group) * gm;
  const i64 gsize = min(ntm - first_m, gm);
  const i64 in_group = local % per_group;
  q.tm = first_m + in_group % gsize;
  q.tn = in_group / gsize;
  return q;
}

template <int BM, int BN, int PER_CU>
__device__ __forceinline__ TilePos tile_pos(const GemmView& v) {
  int pi;
  i64 local;
  tile_of<PER_CU>(v, pi, local);
  return tile_coords<BM, BN>(v, pi, local);
}

// Wait states between the last MFMAs and the reads of their results: every
// accumulator passes through a short s_nop in diagonal order, and diagonal
// s = 7 (written by the last MFMAs of a step) comes last.  Then
// C = sum_s 2^(8s) X_s (mod 2^64) and the shared epilogue.  16x16 accumulator
// layout: lane l, register e holds row 4*(l/16) + e and column l%16 of the
// 16x16 block.
template <int HA, int HB, int BM, int BN>
__device__ __forceinline__ void store_tile(v4i (&acc)[HA][HB][8], cptr<LimbProblem> pp, i64 tm, i64 tn, int wr,
                                           int wc, int lane) {
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int x = 0; x < HA; ++x)
#pragma unroll
      for (int y = 0; y < HB; ++y) asm volatile("s_nop 3" : "+a"(acc[x][y][s]));
  const Epilogue ep = pp->ep;
  // Three passes over this lane's outputs: combine the limb diagonals, load
  // every added term (the triple share, the previous K chunk's sum), then add,
  // truncate and store.  With no store between them the loads are in flight
  // together; interleaved with the stores, each would wait for the one before
  // (the compiler cannot tell the output from the added terms).
  u64 v[HB][HA][4];
  i64 off[HB][HA][4];
  bool ok[HB][HA][4];
#pragma unroll
  for (int y = 0; y < HB; ++y) {
    const i64 n = tn * BN + wc * 16 * HB + y * 16 + (lane & 15);
    const bool n_ok = n < pp->N;
    const i64 coff = (n / ep.view.n_div) * ep.view.ld_q + (n % ep.view.n_div);
#pragma unroll
    for (int x = 0; x < HA; ++x)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const i64 m = tm * BM + wr * 16 * HA + x * 16 + 4 * (lane >> 4) + e;
        u64 s8 = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) s8 += (u64)(i64)acc[x][y][s][e] << (8 * s);
        v[y][x][e] = s8;
        ok[y][x][e] = n_ok && m < pp->M;
        off[y][x][e] = m * ep.view.ld_m + coff;
      }
  }
  // The loads are unconditional (no branch around each one): a lane whose
  // output lies past the product's edge reads the product's first element,
  // which exists, and masks it to nothing.
  if (ep.accumulate) {
#pragma unroll
    for (int y = 0; y < HB; ++y)
#pragma unroll
      for (int x = 0; x < HA; ++x)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const u64 o = ep.Out[ok[y][x][e] ? off[y][x][e] : 0];
          v[y][x][e] += o & (u64)0 - (u64)ok[y][x][e];
        }
  }
  if (ep.Cadd) {
    const u64 neg = ep.csign < 0 ? ~(u64)0 : 0;  // -c as (c ^ ~0) + 1
#pragma unroll
    for (int y = 0; y < HB; ++y)
#pragma unroll
      for (int x = 0; x < HA; ++x)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const u64 c = ep.Cadd[ok[y][x][e] ? off[y][x][e] : 0];
          v[y][x][e] += ((c ^ neg) + (neg & 1)) & (u64)0 - (u64)ok[y][x][e];
        }
  }
#pragma unroll
  for (int y = 0; y < HB; ++y)
#pragma unroll
    for (int x = 0; x < HA; ++x)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (ok[y][x][e]) ep.Out[off[y][x][e]] = ep.trunc_bits ? (u64)((i64)v[y][x][e] >> ep.trunc_bits) : v[y][x][e];
}

// GEMM over a tile list.  Each wave streams its fragments straight from
// global memory (buffer loads; every wave load reads four contiguous 256-byte
// runs), one k step ahead of the MFMAs, so no LDS traffic and no barrier sit
// between MFMAs.  The four waves of a workgroup read overlapping blocks at
// about the same time, which the CU's L1 and the XCD's L2 serve.
template <int SA, int SB>
__global__ void __launch_bounds__(kThreads, 1) k_limb_gemm(GemmTables) {
  using S = Shape<SA, SB>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // the wave index is uniform across the wave: keep it (and every address
  // derived from it) in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const GemmView tv = gemm_view();
  const TilePos tp = tile_pos<S::BM, S::BN, 1>(tv);
  const cptr<LimbProblem> pp = tv.probs + tp.pi;
  const i64 tm = tp.tm, tn = tp.tn;
  const i64 mb0 = tm * 2 * SA + wr * SA;  // this wave's first left 32-block
  const i64 nb0 = tn * 2 * SB + wc * SB;  // this wave's first right 32-block

  v4i acc[S::HA][S::HB][8];

  // k runs in steps of two 32-blocks; every segment holds an even number of
  // blocks, so a step never straddles two segments
  const int kbeg = pp->kb_begin, nsteps = (pp->kb_end - pp->kb_begin) >> 1;
  const int g = lane >> 4;
  const LaneOff lo{(unsigned)((g >> 1) * 8192 + (g & 1) * 512 + (lane & 15) * 16)};
  const SegSrc s0 = seg_src(pp->PA0, pp->PB0, pp->kb0, mb0, nb0, SA, SB);
  const SegSrc s1 = seg_src(pp->PA1 ? pp->PA1 : pp->PA0, pp->PB1 ? pp->PB1 : pp->PB0, pp->kb1, mb0, nb0, SA, SB);
  v4i outer[S::HO][8], inner[S::HI][8], d0[S::HI][S::kDbl], d1[S::HI][S::kDbl];
  if (nsteps > 0) {
    const StepOff o = step_off(s0, s1, pp->kb0, kbeg);
    const __amdgpu_buffer_rsrc_t ro = S::kOuterA ? o.a : o.b, ri = S::kOuterA ? o.b : o.a;
#pragma unroll
    for (int h = 0; h < S::HO; ++h)
#pragma unroll
      for (int i = 0; i < 8; ++i) outer[h][i] = ld_frag(ro, lo, o, h, i);
#pragma unroll
    for (int h = 0; h < S::HI; ++h) {
#pragma unroll
      for (int i = 0; i < S::kDbl; ++i) d0[h][i] = ld_frag(ri, lo, o, h, i);
#pragma unroll
      for (int i = S::kDbl; i < 8; ++i) inner[h][i] = ld_frag(ri, lo, o, h, i);
    }
  }
  // Steps alternate between the two buffers of inner planes 0..kDbl-1; the
  // first step starts every accumulator, and the loop body holds two steps so
  // it has no branch.  Loads past the last step re-read the last step's
  // blocks (valid memory, results unused).
  const int klast = kbeg + 2 * (nsteps - 1);
  if (nsteps > 0) {
    using R = StepRegs<SA, SB>;
    auto off = [&](int st) { return step_off(s0, s1, pp->kb0, min(kbeg + 2 * st, klast)); };
    mfma_step<SA, SB, true>(R{acc, outer, inner, d0, d1}, off(0), off(1), lo);
    int st = 1;
    for (; st + 1 < nsteps; st += 2) {
      mfma_step<SA, SB, false>(R{acc, outer, inner, d1, d0}, off(st), off(st + 1), lo);
      mfma_step<SA, SB, false>(R{acc, outer, inner, d0, d1}, off(st + 1), off(st + 2), lo);
    }
    if (st < nsteps) mfma_step<SA, SB, false>(R{acc, outer, inner, d1, d0}, off(st), off(st + 1), lo);
  } else {
#pragma unroll
    for (int x = 0; x < S::HA; ++x)
#pragma unroll
      for (int y = 0; y < S::HB; ++y)
#pragma unroll
        for (int s = 0; s < 8; ++s) acc[x][y][s] = v4i{0, 0, 0, 0};
  }
  store_tile<S::HA, S::HB, S::BM, S::BN>(acc, pp, tm, tn, wr, wc, lane);
}


// ------------------------------------------------------------------ LDS-staged GEMM
// The same product with the outer operand staged through LDS.  In k_limb_gemm
// the waves that share an outer strip each fetch it from global memory.  Here
// each k step's outer blocks of the whole workgroup (one 16 KiB run of two
// k-blocks per strip) are copied once into LDS by buffer loads that write LDS
// directly, an equal share by each wave, and every wave reads its fragments
// back with 16-byte LDS reads (64 lanes reading four 256-byte runs: no bank
// conflicts).  The inner operand still goes from global memory straight into
// registers.
//
// Geometry LGeo<HA, HB, WR, WC>: a WR x WC grid of waves, each owning HA x HB
// blocks of 16x16 outputs (8 diagonal accumulators each).  Four waves (one per
// SIMD) with 2x2.. 4x2 blocks, or eight waves (two per SIMD) with 1x4 or 4x1
// blocks and 128 accumulator registers each, so that a second wave on every
// SIMD covers the first one's stalls without shrinking the tile.
//
// Two LDS buffers alternate between steps: a step computes from one while its
// copies for the next step land in the other.  One barrier per step hands
// them over; it sits in level 6, after the last read of the step's buffer
// (outer limb 7) has returned and after the wave's copies have landed, so
// that the next step's limb 0 can be read during levels 6 and 7.

typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(3))) v4i lds_v4i;

template <int HA_, int HB_, int WR_, int WC_>
struct LGeo {
  static constexpr int HA = HA_, HB = HB_, WR = WR_, WC = WC_;
  static constexpr int kWaves = WR * WC, kThreads = 64 * kWaves;
  static constexpr int BM = 16 * HA * WR, BN = 16 * HB * WC;
  // the operand with more halves per wave, or when equal the one more waves
  // share (A is shared along a row of WC waves, B along a column of WR)
  static constexpr bool kOuterA = HA != HB ? HA > HB : WC >= WR;
  static constexpr int HO = kOuterA ? HA : HB, HI = kOuterA ? HB : HA;
  static constexpr int kStrips = (kOuterA ? BM : BN) / 32;  // outer strips per workgroup
  static constexpr int kBufBytes = kStrips << 14;           // two 8 KiB k-blocks per strip
  static constexpr int kCopies = kStrips * 16 / kWaves;     // 1 KiB copies per wave and step
  // Workgroups per CU: two for the four-wave 64x64 tile (128 accumulator
  // registers) and the thin 32x64 / 64x32 ones (64), whose prologue,
  // epilogue and stalls then overlap the other workgroup's MFMAs.  Both
  // that and the eight-wave shapes leave 128 other registers per lane.
  static constexpr int kMinBlocks = (HA * HB <= 4 && kWaves == 4) ? 2 : 1;
  static constexpr bool kTight = kMinBlocks == 2 || kWaves == 8;
  // Inner planes 0..kDbl-1 are double-buffered; planes kDbl..7 are reloaded
  // in place for the next step at level 8 - p, after their last use.  With
  // 256 registers per lane every plane is double-buffered (the registers the
  // outer operand no longer needs pay for it).
  static constexpr int kDbl = kTight ? 3 : 8;
  // Levels 0..kLoadLevels-1 issue every global load of a step: the copies
  // first, then the double-buffered planes, then the in-place planes 7, 6,
  // ..., kDbl, each load in the level of its position in proportion to the
  // levels' MFMAs.  The hand-over in level 6 finds them long done.
  static constexpr int kLoadLevels = kDbl == 8 ? 3 : 9 - kDbl;
  static constexpr int kInner = HI * 8;
  static constexpr int kLoads = kCopies + kInner;
  static constexpr int mfmas_upto(int L) {
    int c = 0;
    for (int l = 0; l <= L; ++l) c += (8 - l) * HO * HI;
    return c;
  }
  static constexpr int loads_upto(int L) {
    if (L < 0) return 0;
    if (L >= kLoadLevels - 1) return kLoads;
    const int last = mfmas_upto(kLoadLevels - 1);
    return (kLoads * mfmas_upto(L) + last / 2) / last;
  }
  static constexpr int loads_at(int L) { return loads_upto(L) - loads_upto(L - 1); }
  static constexpr int level_of(int q) {
    int L = 0;
    while (loads_upto(L) <= q) ++L;
    return L;
  }
  // Load q >= kCopies + HI*kDbl reloads plane p = 7 - (q - kCopies - HI*kDbl)/HI.
  static constexpr bool schedule_ok() {
    for (int L = 0; L < 8; ++L)
      if (loads_at(L) >= (8 - L) * HO * HI) return false;  // at most one load per MFMA
    for (int q = kCopies + HI * kDbl; q < kLoads; ++q)
      if (level_of(q) < 8 - (7 - (q - kCopies - HI * kDbl) / HI)) return false;  // after last use
    return true;
  }
  static_assert(schedule_ok(), "load schedule");
  static_assert(2 * kBufBytes * kMinBlocks <= 160 * 1024, "step buffers must fit in LDS");
  static_assert(HO % 2 == 0, "a wave's outer halves cover whole strips");
  static_assert(HI == 1 || HI % 2 == 0, "a wave's inner halves start on a strip unless there is one");
  static_assert(kCopies * kWaves == kStrips * 16 && (16 % kCopies == 0 || kCopies % 16 == 0),
                "copies split evenly over the waves");
  // Vector-memory loads complete in issue order, and a step issues its copies
  // before its inner loads, so the hand-over need not wait for the last
  // kPending loads (inner planes for the next step, still in flight); half of
  // the inner loads keeps a margin.
  static constexpr int kPending = kInner / 2;
  static_assert(kPending < 64, "vmcnt holds the pending inner loads");
};

// Descriptors and offsets of one k step: the wave's inner strips and the
// workgroup's outer strips (strip x of either at +x*kbs k-blocks).
struct LStep {
  __amdgpu_buffer_rsrc_t inner, outer;
  int kb, kbs;
  __device__ int off(int x) const { return (kb + x * kbs) << 13; }
};

template <bool OUTER_A>
__device__ __forceinline__ LStep lstep(const SegSrc& s0, const SegSrc& s1, const SegSrc& w0,
                                       const SegSrc& w1, int kb0, int kg) {
  const bool seg0 = kg < kb0;
  LStep o;
  o.inner = OUTER_A ? (seg0 ? s0.b : s1.b) : (seg0 ? s0.a : s1.a);
  o.outer = OUTER_A ? (seg0 ? w0.a : w1.a) : (seg0 ? w0.b : w1.b);
  o.kb = seg0 ? kg : kg - kb0;
  o.kbs = seg0 ? s0.kbs : s1.kbs;
  return o;
}

// Per-wave constants of the LDS path.
struct LCtx {
  unsigned rd;    // LDS byte offset of this lane's fragment in the wave's first outer strip
  unsigned lane;  // lane * 16: a copy's per-lane source offset (LDS takes lane * 16 itself)
  int cx, cu0;    // strip and first 1 KiB unit of this wave's copies
};

// Copy j of this wave: 1 KiB of the next step's outer run into LDS.
__device__ __forceinline__ void copy_unit(const LCtx& c, const LStep& o, lds_u8* buf, int j) {
  const int u = c.cu0 + j;
  __builtin_amdgcn_raw_ptr_buffer_load_lds(o.outer, (__attribute__((address_space(3))) void*)(buf + (c.cx << 14) + (u << 10)),
                                           16, c.lane, o.off(c.cx) + (u << 10), 0, 0);
}

// Outer fragment (half h, limb i) of this wave from an LDS buffer.
__device__ __forceinline__ v4i lds_frag(const lds_u8* buf, const LCtx& c, int h, int i) {
  return *(const lds_v4i*)(buf + c.rd + (h >> 1) * 16384 + (h & 1) * 256 + i * 1024);
}

// Wait until at most PENDING of this wave's vector-memory loads are in flight
// and its LDS reads have returned, then for the other waves.
template <int PENDING>
__device__ __forceinline__ void lds_handover() {
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(PENDING) : "memory");
}

template <class G>
struct LRegs {
  v4i (&acc)[G::HA][G::HB][8];
  v4i (&z)[G::HO];      // outer limb 0
  v4i (&ob)[2][G::HO];  // outer limbs 1..7: limb l in ob[l & 1]
  v4i (&inner)[G::HI][8];  // inner planes kDbl..7 (reloaded in place)
  const v4i (&dcur)[G::HI][G::kDbl];  // inner planes 0..kDbl-1 of this step
  v4i (&dnext)[G::HI][G::kDbl];       // and of the next
  const lds_u8* cur;  // this step's outer blocks
  lds_u8* next;       // the next step's
};

// Global load number Q of level L: the step's copies come first, then the
// next step's double-buffered inner planes, then its in-place planes.
template <class G, int L, int Q>
__device__ __forceinline__ void lds_level_load(LRegs<G>& r, const LCtx& c, const LStep& next, const LaneOff& lo) {
  constexpr int q = G::loads_upto(L - 1) + Q, ND = G::kDbl;
  if constexpr (q < G::kCopies) {
    copy_unit(c, next, r.next, q);
  } else if constexpr (q < G::kCopies + G::HI * ND) {
    constexpr int h = (q - G::kCopies) / ND, i = (q - G::kCopies) % ND;
    r.dnext[h][i] = ld_buf(next.inner, lo.lo, next.off(h >> 1) + LaneOff::sub(h, i));
  } else {
    constexpr int u = q - G::kCopies - G::HI * ND, h = u % G::HI, i = 7 - u / G::HI;
    r.inner[h][i] = ld_buf(next.inner, lo.lo, next.off(h >> 1) + LaneOff::sub(h, i));
  }
}

// MFMA number M of level L and what follows it: at M = 0 the reads of outer
// limb L + 1 (this step's buffer); in level 6, half way, the hand-over and the
// reads of the next step's limb 0; and the level's global loads, evenly spread.
// A tile's odd last step issues no loads, copies or hand-over.
template <class G, bool FIRST, bool LAST, int L, int M>
__device__ __forceinline__ void lds_level(LRegs<G>& r, const LCtx& c, const LStep& next, const LaneOff& lo) {
  constexpr int HO = G::HO, HI = G::HI;
  constexpr int NM = (8 - L) * HO * HI;
  if constexpr (M < NM) {
    constexpr int s = L + M / (HO * HI), o = (M / HI) % HO, i = M % HI;
    const v4i& in = (s - L) < G::kDbl ? r.dcur[i][(s - L) % G::kDbl] : r.inner[i][s - L];
    const v4i& out = L == 0 ? r.z[o] : r.ob[L & 1][o];
    v4i& acc = G::kOuterA ? r.acc[o][i][s] : r.acc[i][o][s];
    const v4i& a = G::kOuterA ? out : in;
    const v4i& b = G::kOuterA ? in : out;
    if constexpr (FIRST && L == 0) mfma16_first(acc, a, b);
    else mfma16(acc, a, b);
    if constexpr (M == 0 && L < 7) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int h = 0; h < HO; ++h) r.ob[(L + 1) & 1][h] = lds_frag(r.cur, c, h, L + 1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (!LAST && L == 6 && M == NM / 2 - 1) {
      __builtin_amdgcn_sched_barrier(0);
      lds_handover<G::kPending>();
#pragma unroll
      for (int h = 0; h < HO; ++h) r.z[h] = lds_frag(r.next, c, h, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    constexpr int NL = LAST ? 0 : G::loads_at(L);
    constexpr int Q = (M + 1) * (NL + 1) / NM - 1, QPREV = M * (NL + 1) / NM - 1;
    if constexpr (Q >= 0 && Q < NL && Q != QPREV) {
      __builtin_amdgcn_sched_barrier(0);
      lds_level_load<G, L, Q>(r, c, next, lo);
      __builtin_amdgcn_sched_barrier(0);
    }
    lds_level<G, FIRST, LAST, L, M + 1>(r, c, next, lo);
  }
}

template <class G, bool FIRST, bool LAST, int L>
__device__ __forceinline__ void lds_levels(LRegs<G>& r, const LCtx& c, const LStep& next, const LaneOff& lo) {
  if constexpr (L < 8) {
    lds_level<G, FIRST, LAST, L, 0>(r, c, next, lo);
    __builtin_amdgcn_sched_barrier(0);
    lds_levels<G, FIRST, LAST, L + 1>(r, c, next, lo);
  }
}

template <class G, bool FIRST, bool LAST>
__device__ __forceinline__ void lds_step(LRegs<G> r, const LCtx& c, const LStep& next, const LaneOff& lo) {
  // Re-define the LDS read base in every step: otherwise each (buffer, half,
  // limb) address is hoisted out of the loop into a register of its own,
  // instead of one base register and the read's immediate offset.
  LCtx cs = c;
  asm volatile("" : "+v"(cs.rd));
  lds_levels<G, FIRST, LAST, 0>(r, cs, next, lo);
}

// One output tile of geometry G over its two LDS step buffers.
template <class G>
__device__ __forceinline__ void lds_tile(lds_u8* b0, lds_u8* b1, const GemmView& tv, const TilePos& tp) {
  constexpr int HA = G::HA, HB = G::HB, WC = G::WC;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave / WC, wc = wave % WC;
  const cptr<LimbProblem> pp = tv.probs + tp.pi;
  const i64 tm = tp.tm, tn = tp.tn;
  const i64 mw = tm * (G::BM / 32), nw = tn * (G::BN / 32);  // the workgroup's first left / right 32-block
  // the wave's first outer and inner 16-half inside the workgroup tile
  const int ho0 = (G::kOuterA ? wr : wc) * G::HO, hi0 = (G::kOuterA ? wc : wr) * G::HI;

  v4i acc[HA][HB][8];
  const int kbeg = pp->kb_begin, nsteps = (pp->kb_end - pp->kb_begin) >> 1;
  const int g = lane >> 4;
  const unsigned lane_off = (unsigned)((g >> 1) * 8192 + (g & 1) * 512 + (lane & 15) * 16);
  // inner loads: the wave's descriptor starts at the strip of its first half;
  // a single inner half may be the second half of that strip
  const LaneOff lo{lane_off + (unsigned)((hi0 & 1) << 8)};
  const uint8_t* PA1 = pp->PA1 ? pp->PA1 : pp->PA0;
  const uint8_t* PB1 = pp->PB1 ? pp->PB1 : pp->PB0;
  constexpr int kInStrips = (G::HI + 1) / 2;
  const i64 mi = G::kOuterA ? mw : mw + (hi0 >> 1), ni = G::kOuterA ? nw + (hi0 >> 1) : nw;
  const SegSrc s0 = seg_src(pp->PA0, pp->PB0, pp->kb0, mi, ni, G::kOuterA ? 1 : kInStrips, G::kOuterA ? kInStrips : 1);
  const SegSrc s1 = seg_src(PA1, PB1, pp->kb1, mi, ni, G::kOuterA ? 1 : kInStrips, G::kOuterA ? kInStrips : 1);
  const SegSrc w0 = seg_src(pp->PA0, pp->PB0, pp->kb0, mw, nw, G::BM / 32, G::BN / 32);
  const SegSrc w1 = seg_src(PA1, PB1, pp->kb1, mw, nw, G::BM / 32, G::BN / 32);
  const int c0 = wave * G::kCopies;
  const LCtx c{(unsigned)((ho0 >> 1) << 14) + lane_off, (unsigned)lane * 16u, c0 >> 4, c0 & 15};

  v4i z[G::HO], ob[2][G::HO], inner[G::HI][8], d0[G::HI][G::kDbl], d1[G::HI][G::kDbl];
  const int klast = kbeg + 2 * (nsteps - 1);
  if (nsteps > 0) {
    auto off = [&](int st) {
      return lstep<G::kOuterA>(s0, s1, w0, w1, pp->kb0, min(kbeg + 2 * st, klast));
    };
    // prologue: step 0's outer run into buffer 0, its inner planes into registers
    {
      const LStep o = off(0);
#pragma unroll
      for (int j = 0; j < G::kCopies; ++j) copy_unit(c, o, b0, j);
#pragma unroll
      for (int h = 0; h < G::HI; ++h) {
#pragma unroll
        for (int i = 0; i < G::kDbl; ++i) d0[h][i] = ld_buf(o.inner, lo.lo, o.off(h >> 1) + LaneOff::sub(h, i));
#pragma unroll
        for (int i = G::kDbl; i < 8; ++i) inner[h][i] = ld_buf(o.inner, lo.lo, o.off(h >> 1) + LaneOff::sub(h, i));
      }
      lds_handover<0>();
#pragma unroll
      for (int h = 0; h < G::HO; ++h) z[h] = lds_frag(b0, c, h, 0);
    }
    // Steps alternate between the two LDS buffers and the two sets of inner
    // planes; the loop body holds two steps.  An odd last step (the tail)
    // issues no loads; otherwise loads past the last step re-read its blocks
    // (valid memory, results unused) and complete at its hand-over.
    using R = LRegs<G>;
    lds_step<G, true, false>(R{acc, z, ob, inner, d0, d1, b0, b1}, c, off(1), lo);
    int st = 1;
    for (; st + 1 < nsteps; st += 2) {
      lds_step<G, false, false>(R{acc, z, ob, inner, d1, d0, b1, b0}, c, off(st + 1), lo);
      lds_step<G, false, false>(R{acc, z, ob, inner, d0, d1, b0, b1}, c, off(st + 2), lo);
    }
    if (st < nsteps) lds_step<G, false, true>(R{acc, z, ob, inner, d1, d0, b1, b0}, c, off(st + 1), lo);
  } else {
#pragma unroll
    for (int x = 0; x < HA; ++x)
#pragma unroll
      for (int y = 0; y < HB; ++y)
#pragma unroll
        for (int s = 0; s < 8; ++s) acc[x][y][s] = v4i{0, 0, 0, 0};
  }
  store_tile<HA, HB, G::BM, G::BN>(acc, pp, tm, tn, wr, wc, lane);
}

template <int HA, int HB, int WR, int WC>
__global__ void __launch_bounds__(64 * WR * WC, (HA * HB <= 4 && WR * WC == 4) ? 2 : 1)  // LGeo::kMinBlocks
    k_limb_gemm_lds(GemmTables) {
  using G = LGeo<HA, HB, WR, WC>;
  __shared__ v4i stage[2][G::kBufBytes / 16];
  const GemmView tv = gemm_view();
  lds_tile<G>((lds_u8*)&stage[0][0], (lds_u8*)&stage[1][0], tv, tile_pos<G::BM, G::BN, G::kMinBlocks>(tv));
}

// Tile classes in one launch: every problem carries its class (LimbProblem::
// cls), and each workgroup runs its problem's tile shape, all three with four
// waves of 32x32 outputs (the 64x64 tile's per-wave register reuse) and two
// workgroups per CU: 64x64, 32x128 (1x4 waves, for products of at most 32
// rows) and 128x32 (4x1 waves, at most 32 columns).
using GClass0 = LGeo<2, 2, 2, 2>;
using GClass1 = LGeo<2, 2, 1, 4>;
using GClass2 = LGeo<2, 2, 4, 1>;
constexpr int kClassBuf = GClass0::kBufBytes > GClass1::kBufBytes
                              ? (GClass0::kBufBytes > GClass2::kBufBytes ? GClass0::kBufBytes : GClass2::kBufBytes)
                              : (GClass1::kBufBytes > GClass2::kBufBytes ? GClass1::kBufBytes : GClass2::kBufBytes);
static_assert(GClass0::kMinBlocks == 2 && GClass1::kMinBlocks == 2 && GClass2::kMinBlocks == 2,
              "every class runs two workgroups per CU");
static_assert(2 * 2 * kClassBuf <= 160 * 1024, "two workgroups' step buffers fit in LDS");

__global__ void __launch_bounds__(256, 2) k_limb_gemm_classes(GemmTables) {
  __shared__ v4i stage[2][kClassBuf / 16];
  const GemmView tv = gemm_view();
  int pi;
  i64 local;
  tile_of<2>(tv, pi, local);
  lds_u8* b0 = (lds_u8*)&stage[0][0];
  lds_u8* b1 = (lds_u8*)&stage[1][0];
  const int cls = tv.probs[pi].cls;
  if (cls == 1)
    lds_tile<GClass1>(b0, b1, tv, tile_coords<GClass1::BM, GClass1::BN>(tv, pi, local));
  else if (cls == 2)
    lds_tile<GClass2>(b0, b1, tv, tile_coords<GClass2::BM, GClass2::BN>(tv, pi, local));
  else
    lds_tile<GClass0>(b0, b1, tv, tile_coords<GClass0::BM, GClass0::BN>(tv, pi, local));
}

// ------------------------------------------------------------------ persistent grouped GEMM
// The classes launch as a persistent kernel (kLimbPersist): the grid is the
// workgroups the chip holds at once (two per CU, a multiple of the XCD
// count), and each workgroup runs tiles one after another, taken from queues
// of tiles per XCD.  XCD x's queue lists the tiles the dispatch-order remap
// above gives the workgroups the dispatcher would hand to XCD x (it deals
// workgroups round the XCDs in index order), in the order it would hand them
// out: runs of neighbouring tiles, then the tail of the list in dispatch
// order.  So the tiles an XCD holds at a time still share operand blocks in
// its L2, and the longest tiles (listed first) still start first.  A
// workgroup reads which XCD it runs on from the hardware, takes from that
// XCD's queue until it runs dry, then from the other XCDs' queues in turn
// (evening out the XCDs' last tiles), and leaves when all eight are dry: so
// every tile runs exactly once wherever the workgroups land.  A queue's head
// is a device-wide counter, taken by one vector atomic per tile (after the
// tile: an atomic still in flight when the next tile's prologue waits for
// its loads would stall it) and broadcast through LDS; the last workgroup
// to leave sets the counters back to zero for the next launch.

// Tile j of XCD x's queue, or -1 past its end (T tiles in the launch).
__device__ __forceinline__ int xcd_queue_tile(int x, int j, int T, bool remap, int run) {
  if (remap) {
    const int span = kXcds * run, full = T / span;
    if (j < full * run) return ((j / run) * kXcds + x) * run + j % run;
    const int t = full * span + (j - full * run) * kXcds + x;
    return t < T ? t : -1;
  }
  const int t = j * kXcds + x;
  return t < T ? t : -1;
}

__device__ __forceinline__ unsigned queue_take(unsigned* q) {
  return __hip_atomic_fetch_add(q, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The XCD this wave runs on (hardware register XCC_ID).
__device__ __forceinline__ int xcd_id() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(v));
  return (int)(v & (kXcds - 1));
}

__global__ void __launch_bounds__(256, 2) k_limb_gemm_persist(GemmTables) {
  __shared__ v4i stage[2][kClassBuf / 16];
  __shared__ int head[2];
  const GemmView tv = gemm_view();
  lds_u8* b0 = (lds_u8*)&stage[0][0];
  lds_u8* b1 = (lds_u8*)&stage[1][0];
  const int tid = threadIdx.x;
  const int x = xcd_id();
  const int T = tv.tile_start[tv.nprob];
  unsigned* const q = tv.queue;
  // head[] is double-buffered: a slot is written only after the barrier
  // that follows every wave's read of its previous value
  if (tid == 0) head[0] = (int)queue_take(q + x);
  __syncthreads();
  int j = __builtin_amdgcn_readfirstlane(head[0]);
  int qi = 0;  // queue (x + qi) mod 8: the own XCD's first
  for (int it = 1;; ++it) {
    const int xq = (x + qi) & (kXcds - 1);
    const int t = xcd_queue_tile(xq, j, T, tv.sched.xcd_remap != 0, kXcdCUs * 2);
    if (t < 0) {
      if (++qi == kXcds) break;
      if (tid == 0) head[it & 1] = (int)queue_take(q + ((x + qi) & (kXcds - 1)));
      __syncthreads();
      j = __builtin_amdgcn_readfirstlane(head[it & 1]);
      continue;
    }
    const int pi = find_problem(tv.tile_start, tv.nprob, t);
    const i64 local = t - tv.tile_start[pi];
    const int cls = tv.probs[pi].cls;
    if (cls == 1)
      lds_tile<GClass1>(b0, b1, tv, tile_coords<GClass1::BM, GClass1::BN>(tv, pi, local));
    else if (cls == 2)
      lds_tile<GClass2>(b0, b1, tv, tile_coords<GClass2::BM, GClass2::BN>(tv, pi, local));
    else
      lds_tile<GClass0>(b0, b1, tv, tile_coords<GClass0::BM, GClass0::BN>(tv, pi, local));
    if (tid == 0) head[it & 1] = (int)queue_take(q + xq);
    // every wave is past its last LDS read of this tile before the next
    // tile's copies overwrite the step buffers
    __syncthreads();
    j = __builtin_amdgcn_readfirstlane(head[it & 1]);
  }
  // every workgroup found all eight queues dry above; the last to get here
  // clears the counters
  if (tid == 0 && queue_take(q + kXcds) == gridDim.x - 1) {
    for (int i = 0; i <= kXcds; ++i) __hip_atomic_store(q + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------------------ GEMM with both operands in LDS
// k_limb_gemm_lds still streams the inner operand from global memory into
// every wave's registers, so each inner strip crosses the vector-memory path
// once per wave that uses it; that traffic, not the matrix cores, is what
// holds the LDS kernel back (with operands resident in L2, leaving out the
// inner loads alone speeds it up by a tenth).  Here both operands of a k step
// are copied once per workgroup into LDS, and every fragment is read from
// there.  LDS holds exactly one k step of both operands (64 KiB for a 64x64
// tile, 96 KiB for 64x128), not two: a step's limb planes die at different
// levels, so each plane is refilled as soon as every wave is past its last
// read.  Level l reads outer limb l + 1 (limb 0 of the next step at level 7),
// and inner limb j of the next step is read into registers right after its
// last use, at level 8 - j (limbs 0..2, used up to the last level, into a
// second register set at level 3).  Two barriers per step certify which planes
// are dead and which copies have landed:
//   B2, before level 0 of step t: copy outer 4..7 of step t, outer 0 and
//       inner 0..5 of step t + 1;
//   B1, before level 3 of step t: copy outer 1..3 of step t + 1 and inner 6, 7
//       of step t + 2.
// Every copy issued after one barrier lands before the next (each waits for
// its own copies, then the barrier), and every plane it overwrites was read
// before the barrier it follows:
//   outer 1..3 read at levels 0..2, outer 4..7 at levels 3..6 (after B1),
//   outer 0 of the next step at level 7; inner 7 and 6 (next step) at levels 1
//   and 2, inner 5 and 0..2 at level 3 (after B1), inner 4 at level 4, inner 3
//   at level 5.
// Geometry SGeo<WR, WC>: WR x WC waves of 32x32 outputs (2x2 blocks of 16x16,
// 8 diagonal accumulators each): 64x64 with four waves, two workgroups per CU
// (one's barrier is covered by the other's matrix-core work), or 64x128 and
// 128x64 with eight waves, which hold both halves of the tile at the same k
// (neighbouring tiles share operand blocks in L2 for longer).
template <int WR_, int WC_>
struct SGeo {
  static constexpr int WR = WR_, WC = WC_;
  static constexpr int kWaves = WR * WC, kThreads = 64 * kWaves;
  static constexpr int BM = 32 * WR, BN = 32 * WC;
  static constexpr bool kOuterA = WR > WC;  // the operand with more strips is outer
  static constexpr int SO = kOuterA ? WR : WC, SI = kOuterA ? WC : WR;  // strips per workgroup
  static constexpr int kOPlane = SO * 2048, kIPlane = SI * 2048;       // one limb plane of a step
  static constexpr int kIBase = 8 * kOPlane;
  static constexpr int kBytes = 8 * (kOPlane + kIPlane);
  static constexpr int kMinBlocks = kWaves == 4 ? 2 : 1;
  // 1 KiB copy units per plane (strips x 2 k-blocks)
  static constexpr int kOU = 2 * SO, kIU = 2 * SI;
  static constexpr int kB1 = 3 * kOU + 2 * kIU, kB2 = 5 * kOU + 6 * kIU;
  static constexpr int kC1 = kB1 / kWaves, kC2 = kB2 / kWaves;  // copies per wave
  // a tile's last step still copies its own outer limbs 4..7 (the head of
  // the level-0 batch), but nothing for later steps
  static constexpr int kC2Last = 4 * kOU / kWaves;
  static_assert(kB1 % kWaves == 0 && kB2 % kWaves == 0, "copies split evenly over the waves");
  // every group of a batch starts at a multiple of kWaves, so a copy's group
  // is a compile-time property of its position in the wave's list
  static_assert((3 * kOU) % kWaves == 0 && (4 * kOU) % kWaves == 0 && (5 * kOU) % kWaves == 0,
                "batch groups aligned to the waves");
  static_assert(kC1 < 5 * 4 && kC2 < 8 * 4, "at most one copy per MFMA");
  static_assert(kBytes * kMinBlocks <= 160 * 1024, "one step of both operands per workgroup fits in LDS");
};

// Descriptors and k-block of one k step (both operands, the workgroup's strips).
struct SStep {
  __amdgpu_buffer_rsrc_t a, b;
  int kb, kbs;
  __device__ int off(int x) const { return (kb + x * kbs) << 13; }
};

__device__ __forceinline__ SStep sstep(const SegSrc& w0, const SegSrc& w1, int kb0, int kg) {
  const bool seg0 = kg < kb0;
  SStep o;
  o.a = seg0 ? w0.a : w1.a;
  o.b = seg0 ? w0.b : w1.b;
  o.kb = seg0 ? kg : kg - kb0;
  o.kbs = seg0 ? w0.kbs : w1.kbs;
  return o;
}

// The k steps a step's copies draw from: this one, the next, the one after.
struct SSteps {
  SStep t0, t1, t2;
};

struct SCtx {
  unsigned rdo, rdi;  // LDS byte offsets of this lane's fragment in its outer / inner strip
  unsigned lane16;    // lane * 16: a copy's per-lane source offset
  int wave;
};

// Fragment (half h, limb i) of the outer / inner operand from LDS.
template <class G>
__device__ __forceinline__ v4i sh_frag_o(const lds_u8* lds, const SCtx& c, int h, int i) {
  return *(const lds_v4i*)(lds + c.rdo + h * 256 + i * G::kOPlane);
}
template <class G>
__device__ __forceinline__ v4i sh_frag_i(const lds_u8* lds, const SCtx& c, int h, int i) {
  return *(const lds_v4i*)(lds + c.rdi + h * 256 + i * G::kIPlane);
}

// Copy number J of this wave in batch B (1: before level 3, 2: before level 0;
// 1 is also the prologue's, with the steps shifted back by one).  Unit
// u = J * waves + wave of the batch's list of (plane, strip, k-block) units.
template <class G, int B, int J>
__device__ __forceinline__ void sh_copy(const SCtx& c, lds_u8* lds, const SSteps& st) {
  constexpr int u0 = J * G::kWaves;
  // group: outer planes [p0, p0 + n) or inner planes, from step `sel`
  constexpr bool outer = B == 1 ? u0 < 3 * G::kOU : u0 < 5 * G::kOU;
  constexpr int start = B == 1 ? (outer ? 0 : 3 * G::kOU)
                               : (u0 < 4 * G::kOU ? 0 : outer ? 4 * G::kOU : 5 * G::kOU);
  constexpr int p0 = B == 1 ? (outer ? 1 : 6) : (u0 < 4 * G::kOU ? 4 : outer ? 0 : 0);
  constexpr int sel = B == 1 ? (outer ? 1 : 2) : (u0 < 4 * G::kOU ? 0 : 1);
  constexpr int upp = outer ? G::kOU : G::kIU;
  const SStep& s = sel == 0 ? st.t0 : sel == 1 ? st.t1 : st.t2;
  const int v = u0 - start + c.wave;
  const int plane = p0 + v / upp, x = (v % upp) >> 1, kk = v & 1;
  const bool is_a = outer == G::kOuterA;
  const unsigned dst = (outer ? 0u : (unsigned)G::kIBase) + plane * (outer ? G::kOPlane : G::kIPlane) + x * 2048 + kk * 1024;
  __builtin_amdgcn_raw_ptr_buffer_load_lds(is_a ? s.a : s.b, (__attribute__((address_space(3))) void*)(lds + dst), 16,
                                           c.lane16, s.off(x) + kk * 8192 + plane * 1024, 0, 0);
}

// All of this wave's copies of batch B from number J on, back to back.
template <class G, int B, int J>
__device__ __forceinline__ void sh_copies(const SCtx& c, lds_u8* lds, const SSteps& st) {
  if constexpr (J < (B == 1 ? G::kC1 : G::kC2)) {
    sh_copy<G, B, J>(c, lds, st);
    sh_copies<G, B, J + 1>(c, lds, st);
  }
}

template <class G>
struct SRegs {
  v4i (&acc)[2][2][8];
  v4i (&z)[2];             // outer limb 0
  v4i (&ob)[2][2];         // outer limbs 1..7: limb l in ob[l & 1]
  v4i (&inner)[2][8];      // inner limbs 3..7, reloaded in place with the next step's
  const v4i (&dcur)[2][3]; // inner limbs 0..2 of this step
  v4i (&dnext)[2][3];      // and of the next
};

// Waits for this wave's copies and LDS reads, then for the other waves.
__device__ __forceinline__ void sh_barrier() {
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// MFMA number M of level L and what follows it.  A tile's odd last step
// copies and reads nothing for a next step.
template <class G, bool FIRST, bool LAST, int L, int M>
__device__ __forceinline__ void sh_level(SRegs<G>& r, const SCtx& c, lds_u8* lds, const SSteps& st) {
  constexpr int NM = (8 - L) * 4;
  if constexpr (M < NM) {
    if constexpr (M == 0 && (L == 0 || L == 3)) {
      __builtin_amdgcn_sched_barrier(0);
      sh_barrier();  // B2 (level 0) or B1 (level 3)
      __builtin_amdgcn_sched_barrier(0);
    }
    constexpr int s = L + M / 4, o = (M / 2) % 2, i = M % 2;
    const v4i& in = (s - L) < 3 ? r.dcur[i][s - L] : r.inner[i][s - L];
    const v4i& out = L == 0 ? r.z[o] : r.ob[L & 1][o];
    v4i& acc = G::kOuterA ? r.acc[o][i][s] : r.acc[i][o][s];
    const v4i& a = G::kOuterA ? out : in;
    const v4i& b = G::kOuterA ? in : out;
    if constexpr (FIRST && L == 0) mfma16_first(acc, a, b);
    else mfma16(acc, a, b);
    if constexpr (M == 0) {
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (L < 7) {
#pragma unroll
        for (int h = 0; h < 2; ++h) r.ob[(L + 1) & 1][h] = sh_frag_o<G>(lds, c, h, L + 1);
      } else if constexpr (!LAST) {
#pragma unroll
        for (int h = 0; h < 2; ++h) r.z[h] = sh_frag_o<G>(lds, c, h, 0);
      }
      if constexpr (!LAST && L >= 1 && L <= 5) {
#pragma unroll
        for (int h = 0; h < 2; ++h) r.inner[h][8 - L] = sh_frag_i<G>(lds, c, h, 8 - L);
      }
      if constexpr (!LAST && L == 3) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int j = 0; j < 3; ++j) r.dnext[h][j] = sh_frag_i<G>(lds, c, h, j);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    constexpr int NL = L == 0 ? (LAST ? G::kC2Last : G::kC2) : (L == 3 && !LAST) ? G::kC1 : 0;
    constexpr int Q = (M + 1) * (NL + 1) / NM - 1, QPREV = M * (NL + 1) / NM - 1;
    if constexpr (Q >= 0 && Q < NL && Q != QPREV) {
      __builtin_amdgcn_sched_barrier(0);
      sh_copy<G, L == 0 ? 2 : 1, Q>(c, lds, st);
      __builtin_amdgcn_sched_barrier(0);
    }
    sh_level<G, FIRST, LAST, L, M + 1>(r, c, lds, st);
  }
}

template <class G, bool FIRST, bool LAST, int L>
__device__ __forceinline__ void sh_levels(SRegs<G>& r, const SCtx& c, lds_u8* lds, const SSteps& st) {
  if constexpr (L < 8) {
    sh_level<G, FIRST, LAST, L, 0>(r, c, lds, st);
    __builtin_amdgcn_sched_barrier(0);
    sh_levels<G, FIRST, LAST, L + 1>(r, c, lds, st);
  }
}

template <class G, bool FIRST, bool LAST>
__device__ __forceinline__ void sh_step(SRegs<G> r, const SCtx& c, lds_u8* lds, const SSteps& st) {
  // one base register per operand, the plane and half in each read's offset
  SCtx cs = c;
  asm volatile("" : "+v"(cs.rdo), "+v"(cs.rdi));
  sh_levels<G, FIRST, LAST, 0>(r, cs, lds, st);
}

template <int WR, int WC>
__global__ void __launch_bounds__(64 * WR * WC, WR * WC == 4 ? 2 : 1)  // SGeo::kMinBlocks
    k_limb_gemm_sh(GemmTables) {
  using G = SGeo<WR, WC>;
  __shared__ v4i lds_words[G::kBytes / 16];
  lds_u8* lds = (lds_u8*)&lds_words[0];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave / WC, wc = wave % WC;
  const GemmView tv = gemm_view();
  const TilePos tp = tile_pos<G::BM, G::BN, G::kMinBlocks>(tv);
  const cptr<LimbProblem> pp = tv.probs + tp.pi;
  const i64 tm = tp.tm, tn = tp.tn;
  const i64 mw = tm * WR, nw = tn * WC;  // the workgroup's first left / right 32-block
  const int xo = G::kOuterA ? wr : wc, xi = G::kOuterA ? wc : wr;  // the wave's outer / inner strip

  v4i acc[2][2][8];
  const int kbeg = pp->kb_begin, nsteps = (pp->kb_end - pp->kb_begin) >> 1;
  const int g = lane >> 4;
  const unsigned lane_lds = (unsigned)((g >> 1) * 1024 + (g & 1) * 512 + (lane & 15) * 16);
  const SCtx c{(unsigned)(xo * 2048) + lane_lds, (unsigned)(G::kIBase + xi * 2048) + lane_lds,
               (unsigned)lane * 16u, wave};
  const uint8_t* PA1 = pp->PA1 ? pp->PA1 : pp->PA0;
  const uint8_t* PB1 = pp->PB1 ? pp->PB1 : pp->PB0;
  const SegSrc w0 = seg_src(pp->PA0, pp->PB0, pp->kb0, mw, nw, WR, WC);
  const SegSrc w1 = seg_src(PA1, PB1, pp->kb1, mw, nw, WR, WC);

  v4i z[2], ob[2][2], inner[2][8], d0[2][3], d1[2][3];
  const int klast = kbeg + 2 * (nsteps - 1);
  if (nsteps > 0) {
    // steps past the last re-read the last step's blocks (valid memory, unused)
    auto off = [&](int t) { return sstep(w0, w1, pp->kb0, min(kbeg + 2 * max(t, 0), klast)); };
    // prologue: step 0's outer limb 0 and inner limbs straight into registers
    // (global fragment offsets: k-block g/2 of the step is 8 KiB further);
    // then the copies a B1 barrier of step -1 would have issued
    {
      const SStep s0 = off(0);
      const unsigned lane_g = (unsigned)((g >> 1) * 8192 + (g & 1) * 512 + (lane & 15) * 16);
      const __amdgpu_buffer_rsrc_t ro = G::kOuterA ? s0.a : s0.b, ri = G::kOuterA ? s0.b : s0.a;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        z[h] = ld_buf(ro, lane_g, s0.off(xo) + h * 256);
#pragma unroll
        for (int j = 0; j < 3; ++j) d0[h][j] = ld_buf(ri, lane_g, s0.off(xi) + h * 256 + j * 1024);
#pragma unroll
        for (int j = 3; j < 8; ++j) inner[h][j] = ld_buf(ri, lane_g, s0.off(xi) + h * 256 + j * 1024);
      }
      const SSteps pro{s0, s0, off(1)};
      sh_copies<G, 1, 0>(c, lds, pro);
    }
    using R = SRegs<G>;
    auto steps = [&](int t) { return SSteps{off(t), off(t + 1), off(t + 2)}; };
    sh_step<G, true, false>(R{acc, z, ob, inner, d0, d1}, c, lds, steps(0));
    int t = 1;
    for (; t + 1 < nsteps; t += 2) {
      sh_step<G, false, false>(R{acc, z, ob, inner, d1, d0}, c, lds, steps(t));
      sh_step<G, false, false>(R{acc, z, ob, inner, d0, d1}, c, lds, steps(t + 1));
    }
    if (t < nsteps) sh_step<G, false, true>(R{acc, z, ob, inner, d1, d0}, c, lds, steps(t));
    // no copy may still be writing this workgroup's LDS when it ends
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  } else {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int s = 0; s < 8; ++s) acc[x][y][s] = v4i{0, 0, 0, 0};
  }
  store_tile<2, 2, G::BM, G::BN>(acc, pp, tm, tn, wr, wc, lane);
}

}  // namespace

i64 limb_rblocks(i64 rows) {
  const i64 b = (rows + 31) / 32;
  return (b + kLimbRowPad - 1) / kLimbRowPad * kLimbRowPad;
}
i64 limb_kblocks(i64 K) { return (K + 63) / 64 * 2; }
int limb_tiles(i64 M, i64 N, int variant) {
  const i64 bm = limb_variant_bm(variant), bn = limb_variant_bn(variant);
  return (int)(((M + bm - 1) / bm) * ((N + bn - 1) / bn));
}
// output rows and columns of one workgroup tile, per variant
// (the classes variants: their class-0 tile; limb_class_tiles gives every class's)
static const int kVariantBM[kLimbVariants] = {128, 64, 64, 128, 64, 64, 64, 128, 64, 64, 64, 128, 32, 128, 64, 64};
static const int kVariantBN[kLimbVariants] = {64, 128, 64, 64, 128, 64, 128, 64, 128, 64, 128, 64, 128, 32, 64, 64};
int limb_variant_bm(int variant) { return kVariantBM[variant]; }
int limb_variant_bn(int variant) { return kVariantBN[variant]; }
void limb_class_shape(int cls, int* bm, int* bn) {
  *bm = cls == 1 ? GClass1::BM : cls == 2 ? GClass2::BM : GClass0::BM;
  *bn = cls == 1 ? GClass1::BN : cls == 2 ? GClass2::BN : GClass0::BN;
}
int limb_class_tiles(i64 M, i64 N, int cls) {
  const i64 bm = cls == 1 ? GClass1::BM : cls == 2 ? GClass2::BM : GClass0::BM;
  const i64 bn = cls == 1 ? GClass1::BN : cls == 2 ? GClass2::BN : GClass0::BN;
  return (int)(((M + bm - 1) / bm) * ((N + bn - 1) / bn));
}

hipError_t launch_pack(hipStream_t s, const PackTables& t, i64 total_blocks, int kind, int mode) {
  if (total_blocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)((total_blocks + 3) / 4)), block(kPackThreads);
#define MPC_PACK_CASE(K, MO)                                                            \
  if (kind == K && mode == MO) {                                                         \
    hipLaunchKernelGGL((k_pack<K, MO>), grid, block, 0, s, t);                          \
    return hipGetLastError();                                                            \
  }
  MPC_PACK_CASE(kPackRow, kModeCopy)
  MPC_PACK_CASE(kPackRow, kModeSum2)
  MPC_PACK_CASE(kPackRow, kModeOpenLeft)
  MPC_PACK_CASE(kPackRow, kModeOpenRight)
  MPC_PACK_CASE(kPackRow, kModePrgSum2)
  MPC_PACK_CASE(kPackRow, kModePrgSum2A)
  MPC_PACK_CASE(kPackRow, kModeOpenLeft2)
  MPC_PACK_CASE(kPackCol, kModeCopy)
  MPC_PACK_CASE(kPackCol, kModeSum2)
  MPC_PACK_CASE(kPackCol, kModeOpenRight)
  MPC_PACK_CASE(kPackCol, kModePrgSum2)
  MPC_PACK_CASE(kPackCol, kModePrgSum2B)
  MPC_PACK_CASE(kPackCol, kModeOpenRight1)
  MPC_PACK_CASE(kPackIm2col, kModeSum2)
  MPC_PACK_CASE(kPackIm2col, kModeOpenLeft)
#undef MPC_PACK_CASE
  return hipErrorInvalidValue;
}

int limb_persist_grid(int total_tiles, int num_cu) {
  const int cap = std::max(kXcds, 2 * num_cu / kXcds * kXcds);
  return std::min(cap, (total_tiles + kXcds - 1) / kXcds * kXcds);
}

hipError_t launch_limb_gemm(hipStream_t s, const GemmTables& t, int total_tiles) {
  if (total_tiles <= 0) return hipSuccess;
  const TileSched& sched = t.sched;
  if (sched.group_m < 1 || sched.group_m > 64) return hipErrorInvalidValue;
  if (sched.variant == kLimbPersist) {
    // a multiple of the XCD count, so that every queue has workgroups
    if (!t.queue || t.persist_grid < kXcds || t.persist_grid % kXcds) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_limb_gemm_persist, dim3(t.persist_grid), dim3(256), 0, s, t);
    return hipGetLastError();
  }
  const dim3 grid(total_tiles);
#define MPC_LDS_CASE(V, HA, HB, WR, WC)                                                                    \
  case V:                                                                                                 \
    hipLaunchKernelGGL((k_limb_gemm_lds<HA, HB, WR, WC>), grid, dim3(64 * WR * WC), 0, s, t); \
    break;
#define MPC_SH_CASE(V, WR, WC)                                                                        \
  case V:                                                                                         \
    hipLaunchKernelGGL((k_limb_gemm_sh<WR, WC>), grid, dim3(64 * WR * WC), 0, s, t); \
    break;
  switch (sched.variant) {
    case kLimb128x64: hipLaunchKernelGGL((k_limb_gemm<2, 1>), grid, dim3(kThreads), 0, s, t); break;
    case kLimb64x128: hipLaunchKernelGGL((k_limb_gemm<1, 2>), grid, dim3(kThreads), 0, s, t); break;
    case kLimb64x64: hipLaunchKernelGGL((k_limb_gemm<1, 1>), grid, dim3(kThreads), 0, s, t); break;
    MPC_LDS_CASE(kLimbLds128x64, 4, 2, 2, 2)
    MPC_LDS_CASE(kLimbLds64x128, 2, 4, 2, 2)
    MPC_LDS_CASE(kLimbLds64x64, 2, 2, 2, 2)
    MPC_LDS_CASE(kLimbLds64x128w8, 1, 4, 4, 2)
    MPC_LDS_CASE(kLimbLds128x64w8, 4, 1, 2, 4)
    MPC_LDS_CASE(kLimbLds64x128w8s, 2, 2, 2, 4)
    MPC_LDS_CASE(kLimbThin32x128, 2, 2, 1, 4)
    MPC_LDS_CASE(kLimbThin128x32, 2, 2, 4, 1)
    case kLimbClasses: hipLaunchKernelGGL(k_limb_gemm_classes, grid, dim3(256), 0, s, t); break;
    MPC_SH_CASE(kLimbSh64x64, 2, 2)
    MPC_SH_CASE(kLimbSh64x128, 2, 4)
    MPC_SH_CASE(kLimbSh128x64, 4, 2)
    default: return hipErrorInvalidValue;
  }
#undef MPC_LDS_CASE
#undef MPC_SH_CASE
  return hipGetLastError();
}

}  // namespace mpc
