// internal.h -- shared declarations of libmpc's HIP sources (not installed).
//
// Ring elements are uint64; every kernel is integer-only.  The launchers
// declared here are defined in the .hip files and called by api.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mpc {

using u64 = uint64_t;
using i64 = int64_t;
using u32 = uint32_t;

// ---------------------------------------------------------------- PRG
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).  A stream with state s
// returns mix(s + (i+1)*gamma) as its i-th output.  Domains nest: the key of
// (seed, tag, slot) is out_slot(out_tag(seed)) and element i is out_i(key).
constexpr u64 kGamma = 0x9e3779b97f4a7c15ULL;

__host__ __device__ __forceinline__ u64 sm_mix(u64 z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ u64 sm_out(u64 s, u64 i) { return sm_mix(s + (i + 1) * kGamma); }
inline u64 stream_key(u64 seed, u64 tag, u64 slot) { return sm_out(sm_out(seed, tag), slot); }

enum Slot : u64 { kSlotShare = 0, kSlotA0 = 1, kSlotA1 = 2, kSlotB0 = 3, kSlotB1 = 4, kSlotC0 = 5 };
// Slots of sharings among P > 2 parties: base + party index.
enum MpSlot : u64 { kMpShare = 0x100, kMpA = 0x200, kMpB = 0x300, kMpC = 0x400, kMpR = 0x500, kMpT = 0x600 };

// ---------------------------------------------------------------- views
// Element (m, n) of a GEMM output (and of its additive term) lives at
//   m * ld_m + (n / n_div) * ld_q + (n % n_div).
// A row-major MxN matrix is {N, N, 0} (or any ld); the transposed conv1d output
// [B][Cout][Lout] with m = cout and n = b*Lout + l is {Lout, Lout, Cout*Lout}.
struct OutView {
  i64 ld_m, n_div, ld_q;
};

// Epilogue shared by both GEMM forms:
//   v = acc (+ Out if accumulate) (+ csign * Cadd);  if (trunc) v = s64(v) >> trunc
struct Epilogue {
  const u64* Cadd;  // may be null
  int csign;        // +1 or -1
  int trunc_bits;   // 0 = none
  int accumulate;   // add the current contents of Out (continuation of a K chunk)
  u64* Out;
  OutView view;
};

// Plain-form problem: C = [A0 (+A0add) | A1] @ [B0 (+B0add) ; B1], row-major
// segments.  K1 may be 0 (then A1/B1 are unused).
struct PlainProblem {
  i64 M, N, K0, K1;
  const u64* A0;
  const u64* A0add;
  i64 lda0;
  const u64* A1;
  i64 lda1;
  const u64* B0;
  const u64* B0add;
  i64 ldb0;
  const u64* B1;
  i64 ldb1;
  Epilogue ep;
  // Split-K: the k range is cut into ksplit slices of kslice values (a
  // multiple of the kernel's k tile); with ksplit > 1 each slice writes its raw
  // sum to partial[slice][M][N] and a reduction applies the epilogue.
  int ksplit;
  i64 kslice;
  u64* partial;
};

// ---------------------------------------------------------------- limb packing
// A packed operand holds, for every 32x32 block of a matrix (32 rows x 32 k
// for a left operand, 32 k x 32 cols for a right operand), eight 1 KiB planes
// of signed 8-bit limbs.  Inside a plane the 64 lanes of a wavefront each own
// 16 bytes: lane l covers row (or col) l % 32 and k = (l / 32) * 16 + [0, 16).
// Block (rb, kb) starts at byte ((rb * kblocks + kb) << 13).  Rows, cols and k
// are padded with zeros (the limbs of 0 are all 0) to whole blocks; row and
// col block counts are further padded to a multiple of kLimbRowPad blocks and
// k block counts to an even number (the GEMM steps over 64 k at a time).
constexpr int kLimbBlockBytes = 8192;
constexpr int kLimbRowPad = 4;

// A pack job reads one to four uint64 operands of one shape, elementwise, and
// writes one to three packed outputs (mode):
//   COPY       in0                                  -> out0
//   SUM2       in0 + in1                            -> out0
//   OPEN_LEFT  (x0, x1, a0, a1): eps = x0+x1-a0-a1  -> out0,
//              g0 = a0 + eps = x0+x1-a1 -> out1,  a1 -> out2
//   OPEN_RIGHT (y0, y1, b0, b1): delta = y0+y1-b0-b1 -> out0,  b0 -> out1,  b1 -> out2
// so one pass opens a masked value and packs it with the triple's shares.
// Element (r, k) of the logical operand (zero outside rows x K) is
//   kind ROW:    left operand MxK, in[r*ld + k]
//   kind COL:    right operand KxN, in[k*ld + r]  (r is the column)
//   kind IM2COL: right operand, k = c*ksz + j, n = b*Lout + l, element
//                in[b][c][l*stride + j] of a [B][Cin][L] activation
enum PackKind : int { kPackRow = 0, kPackCol = 1, kPackIm2col = 2 };
// kModePrgSum2 draws the two inputs from the PRG instead of reading them:
// element e (its row-major offset) gets v_i = G(key[i], e), which is also
// written to share[i][e]; the packed output is v_0 + v_1.  Used by the
// dealer for matrix operands, where every element is visited exactly once.
// The offline-packed matrix triple: kModePrgSum2A also packs the second
// share (a_1) and kModePrgSum2B both (b_0, b_1) for the finish, and the
// online open then packs only what it must: kModeOpenLeft2 eps and
// g0 = a0 + eps, kModeOpenRight1 delta.
enum PackMode : int {
  kModeCopy = 0, kModeSum2 = 1, kModeOpenLeft = 2, kModeOpenRight = 3, kModePrgSum2 = 4,
  kModePrgSum2A = 5, kModePrgSum2B = 6, kModeOpenLeft2 = 7, kModeOpenRight1 = 8
};
inline bool pack_prg(int mode) { return mode == kModePrgSum2 || mode == kModePrgSum2A || mode == kModePrgSum2B; }
constexpr int kPackMaxIn = 4, kPackMaxOut = 3;

struct PackJob {
  int kind;
  int mode;
  i64 rows;  // M for ROW, N for COL/IM2COL (the non-k dimension)
  i64 K;
  const u64* in[kPackMaxIn];
  i64 ld;
  i64 cin, len, ksz, stride, lout;  // im2col geometry
  uint8_t* dst[kPackMaxOut];
  i64 rblocks;  // padded block counts of every output
  i64 kblocks;
  // Row blocks that hold data, ceil(rows / 32).  Only these are written: the
  // padding row blocks beyond them (up to rblocks) are read by the GEMM's edge
  // tiles but only reach outputs past the last row or column, which are never
  // stored.  (All kblocks are written: zeros past K enter every output.)
  i64 rreal;
  u64 key[2];    // kModePrgSum2: PRG stream keys of the two shares
  u64* share[2];  // kModePrgSum2: where the two shares are written
};

inline int pack_nin(int mode) { return mode == kModeCopy ? 1 : (mode == kModeSum2 || pack_prg(mode)) ? 2 : 4; }
inline int pack_nout(int mode) {
  return (mode <= kModeSum2 || mode == kModePrgSum2 || mode == kModeOpenRight1)
             ? 1
             : (mode == kModePrgSum2A || mode == kModeOpenLeft2) ? 2 : 3;
}

// Limb-form problem over packed segments; k-blocks [kb_begin, kb_end) of the
// concatenation [segment 0 | segment 1] are processed (K chunking).
struct LimbProblem {
  i64 M, N;
  int kb0, kb1;  // k-blocks of segment 0 and 1
  int kb_begin, kb_end;
  const uint8_t* PA0;
  const uint8_t* PA1;
  const uint8_t* PB0;
  const uint8_t* PB1;
  i64 mblocks;  // padded row blocks of the left operand
  i64 nblocks;  // padded col blocks of the right operand
  Epilogue ep;
  int cls;      // tile class, read by the classes variant only
};

// Largest number of concatenated k values one limb launch may cover: with all
// limbs -128 a diagonal of 8 pairs adds 8 * 2^14 per k, so 16320 * 2^17 < 2^31.
// (Even, so chunk boundaries fall between the GEMM's 64-wide k steps.)
constexpr int kLimbMaxKBlocks = 510;  // 510 * 32 = 16320
// Smallest split-K slice of the limb GEMM, in 64-wide k steps.
constexpr int kLimbMinSliceSteps = 4;
static_assert(kLimbMaxKBlocks % 2 == 0, "chunks must hold whole k steps");
// Longest k segment the limb GEMM addresses.  A wave reads up to 4 strips of
// 32 rows of one packed segment through one buffer descriptor, whose byte
// range and offsets are 32-bit: 4 strips * 65534 k-blocks * 8 KiB stays below
// 2^31.  Longer segments take the plain form.
constexpr i64 kLimbMaxSegK = 65534 * 32;  // 2,097,088

// Tile-to-problem table for grouped launches.
struct TileMap {
  int nprob;
  const int* tile_start;  // device, nprob+1 entries
};

// ---------------------------------------------------------------- launchers
// Element-wise kernels (elementwise.hip).  All take the stream to launch on.
hipError_t launch_prg_fill(hipStream_t s, u64 key, u64* out, size_t n);
hipError_t launch_share(hipStream_t s, const u64* x, size_t n, int src, u64 key, u64* s0, u64* s1);
hipError_t launch_reveal(hipStream_t s, const u64* s0, const u64* s1, size_t n, u64* out);
hipError_t launch_truncate(hipStream_t s, u64* v, size_t n, int bits);
hipError_t launch_dealer_mul(hipStream_t s, const u64 key[6], size_t n, u64* a0, u64* a1, u64* b0,
                             u64* b1, u64* c0, u64* c1);
hipError_t launch_dealer_square(hipStream_t s, const u64 key[6], size_t n, u64* a0, u64* a1,
                                u64* b0, u64* b1);
hipError_t launch_beaver_mul(hipStream_t s, size_t n, const u64* x0, const u64* x1, const u64* y0,
                             const u64* y1, const u64* a0, const u64* a1, const u64* b0,
                             const u64* b1, const u64* c0, const u64* c1, int trunc, u64* z0,
                             u64* z1);
hipError_t launch_beaver_square(hipStream_t s, size_t n, const u64* x0, const u64* x1,
                                const u64* a0, const u64* a1, const u64* b0, const u64* b1,
                                int trunc, u64* z0, u64* z1);
// Open step of Beaver bilinear products, many operands per launch.  A job of
// kind kOpenLeft writes eps = (x0-a0)+(x1-a1) to out0 and g = a0 + eps to
// out1; kind kOpenRight writes delta = (x0-a0)+(x1-a1) to out0 only.  Jobs
// are split into chunks of kOpenChunk elements; chunk_start (njobs+1 prefix
// sums of per-job chunk counts) and jobs are device arrays.
enum OpenKind : int { kOpenLeft = 0, kOpenRight = 1 };
struct OpenJob {
  int kind;
  i64 n;
  const u64* x0;
  const u64* x1;
  const u64* a0;
  const u64* a1;
  u64* out0;
  u64* out1;
};
constexpr i64 kOpenChunk = 4096;
hipError_t launch_open(hipStream_t s, const OpenJob* jobs, const i64* chunk_start, int njobs,
                       i64 total_chunks);
// Grouped element-wise Beaver products: job j multiplies (or, with y0 null,
// squares with the pair a, b = a^2) n shared elements, then truncates; one
// workgroup per chunk of kMulChunk elements of one job.  chunk_start
// (njobs+1 prefix sums of per-job chunk counts) and jobs are device arrays.
struct MulJob {
  i64 n;
  int vec2;  // every array 16-byte aligned: two elements per load
  const u64 *x0, *x1, *y0, *y1, *a0, *a1, *b0, *b1, *c0, *c1;
  u64 *z0, *z1;
};
constexpr i64 kMulChunk = 1024;  // even, so a chunk's first element keeps the pairs aligned
hipError_t launch_beaver_mul_grouped(hipStream_t s, const MulJob* jobs, const i64* chunk_start, int njobs,
                                     i64 total_chunks, int trunc);
// col[k][n] = x[b][c][l*stride + j] (+ add) with k = c*ksz + j, n = b*Lout + l
hipError_t launch_im2col(hipStream_t s, const u64* x, const u64* add, i64 B, i64 cin, i64 len,
                         i64 ksz, i64 stride, i64 lout, u64* col);
// out = x + y
hipError_t launch_add(hipStream_t s, const u64* x, const u64* y, size_t n, u64* out);

// Plain ring GEMM (gemm_plain.hip): one launch over all problems of `probs`
// (a device array), tiles listed by `map`.
// A whole two-party Beaver matmul of a small product (plain arithmetic) in
// one launch: operands, triple shares and outputs as in mpc_beaver_matmul.
struct SmallMatmul {
  i64 M, N, K;
  const u64 *x0, *x1, *y0, *y1, *a0, *a1, *b0, *b1, *c0, *c1;
  u64 *z0, *z1;
  int trunc;
};
// Products of at most kSmallMatmulMacs ring multiply-accumulates per party
// with k at most kSmallMatmulK (each thread then runs at most 64 steps of k)
// take it.
constexpr i64 kSmallMatmulMacs = (i64)1 << 18, kSmallMatmulK = 1024;
hipError_t launch_beaver_matmul_small(hipStream_t s, const SmallMatmul& m);
hipError_t launch_plain_gemm(hipStream_t s, const PlainProblem* probs, TileMap map,
                             int total_tiles);
int plain_tiles(i64 M, i64 N);
constexpr int kPlainBK = 16;  // k tile of the plain GEMM (split-K slices are multiples)
// Split-K reduction shared by both GEMM forms, for every split problem of a
// call at once: v = sum of a job's ks partial M x N results
// (partial[slice][M][N]), then its epilogue.  One workgroup per chunk of
// kReduceChunk outputs of one job (chunk_start: njobs+1 prefix sums of per-job
// chunk counts; jobs and chunk_start are device arrays).
struct ReduceJob {
  const u64* partial;
  int ks;
  i64 M, N;
  Epilogue ep;
};
constexpr i64 kReduceChunk = 256;  // one output per thread
hipError_t launch_splitk_reduce_grouped(hipStream_t s, const ReduceJob* jobs, const i64* chunk_start, int njobs,
                                        i64 total_chunks);

// Limb form (gemm_limb.hip).
// The descriptor tables of one pack or GEMM launch travel either as device
// arrays (uploaded by the host) or, when they are short, inside the kernel's
// arguments: then no upload (no copy on the stream, no host staging) precedes
// the launch.  The kernels read whichever the host filled through the
// kernel-argument segment, as constant memory.
constexpr int kInlineJobs = 4, kInlineProbs = 4;
// Jobs of one pack launch: `jobs`/`block_start` (device; njobs+1 prefix sums
// of rreal*kblocks), or when `jobs` is null the first njobs entries of
// ijobs/ibstart.  Every job of one launch has the launch's kind and mode.
struct PackTables {
  const PackJob* jobs;
  const i64* block_start;
  int njobs;
  PackJob ijobs[kInlineJobs];
  i64 ibstart[kInlineJobs + 1];
};
hipError_t launch_pack(hipStream_t s, const PackTables& t, i64 total_blocks, int kind, int mode);
// Tile shapes of the limb GEMM (workgroup output tile) and the tile order.
// Variants 3..8 stage the outer operand through LDS (k_limb_gemm_lds); 6, 7
// and 8 run eight waves per workgroup (two per SIMD): 6 and 7 with 16x64 and
// 64x16 wave sub-tiles, 8 with 32x32 ones, as in the four-wave 64x64 tile.
// Variants 9..11 stage both operands through LDS (k_limb_gemm_sh), every wave
// owning 32x32 outputs: 9 with four waves (two workgroups per CU), 10 and 11
// with eight.  Variants 12 and 13 are thin tiles for products of at most 32
// rows or columns: 32x128 and 128x32 in the LDS form, four waves of 32x32
// outputs in a row or a column, two workgroups per CU.  Variant 14 takes
// each problem's tile class from LimbProblem::cls (0: 64x64, 1: 32x128,
// 2: 128x32), all in one launch.  Variant 15 is variant 14 as a persistent
// kernel: as many workgroups as the chip holds at once, each taking tiles
// from its XCD's queue until the queue is empty.
enum LimbVariant : int {
  kLimb128x64 = 0, kLimb64x128 = 1, kLimb64x64 = 2,
  kLimbLds128x64 = 3, kLimbLds64x128 = 4, kLimbLds64x64 = 5,
  kLimbLds64x128w8 = 6, kLimbLds128x64w8 = 7, kLimbLds64x128w8s = 8,
  kLimbSh64x64 = 9, kLimbSh64x128 = 10, kLimbSh128x64 = 11,
  kLimbThin32x128 = 12, kLimbThin128x32 = 13, kLimbClasses = 14, kLimbPersist = 15
};
constexpr int kLimbVariants = 16;
inline bool limb_per_class(int variant) { return variant == kLimbClasses || variant == kLimbPersist; }
struct TileSched {
  int variant;    // LimbVariant
  int group_m;    // tile rows per raster group
  int xcd_remap;  // hand tiles to the XCDs in runs of neighbouring tiles
};
// ---------------------------------------------------------------- binary sharing (two parties)
// Slots: 0x700 share, 0x701..0x705 AND triple a0, a1, b0, b1, c0, 0x706/0x707
// the parties' re-sharing in A2B, 0x708..0x70a Algorithm 2's bit r, <r>_0, [r]_0.
enum BinSlot : u64 {
  kBinShare = 0x700, kBinA0 = 0x701, kBinA1 = 0x702, kBinB0 = 0x703, kBinB1 = 0x704, kBinC0 = 0x705,
  kA2bY0 = 0x706, kA2bY1 = 0x707, kB2aR = 0x708, kB2aRb0 = 0x709, kB2aRa0 = 0x70a
};
constexpr int kA2bTriples = 12;  // AND triples per word of one A2B conversion
struct TriplePtrs {
  const u64 *a0, *a1, *b0, *b1, *c0, *c1;
};
struct BinKeys {
  u64 a0, a1, b0, b1, c0;
};
hipError_t launch_bin_share(hipStream_t s, const u64* x, size_t n, int src, u64 key, u64* s0, u64* s1);
hipError_t launch_bin_reveal(hipStream_t s, const u64* s0, const u64* s1, size_t n, u64* out);
hipError_t launch_dealer_and(hipStream_t s, const BinKeys& k, size_t n, u64* a0, u64* a1, u64* b0, u64* b1,
                             u64* c0, u64* c1);
hipError_t launch_bin_and(hipStream_t s, size_t n, const u64* x0, const u64* x1, const u64* y0, const u64* y1,
                          const TriplePtrs& t, u64* z0, u64* z1);
// t: kA2bTriples AND triples per element, triple j of element i at j * n + i
hipError_t launch_a2b(hipStream_t s, size_t n, const u64* x0, const u64* x1, u64 ky0, u64 ky1,
                      const TriplePtrs& t, u64* z0, u64* z1);
hipError_t launch_dealer_b2a(hipStream_t s, size_t n, u64 kr, u64 krb, u64 kra, u64* rb0, u64* rb1, u64* ra0,
                             u64* ra1);
hipError_t launch_b2a_bit(hipStream_t s, size_t n, int bit, const u64* b0, const u64* b1, const u64* rb0,
                          const u64* rb1, const u64* ra0, const u64* ra1, u64* z0, u64* z1);
// m: an arithmetic MUL triple
hipError_t launch_relu(hipStream_t s, size_t n, const u64* x0, const u64* x1, u64 ky0, u64 ky1,
                       const TriplePtrs& t, const u64* rb0, const u64* rb1, const u64* ra0, const u64* ra1,
                       const TriplePtrs& m, u64* z0, u64* z1);

// ---------------------------------------------------------------- more than two parties
constexpr int kMaxParties = 16;
struct MpOut {
  u64* p[kMaxParties];
};
struct MpIn {
  const u64* p[kMaxParties];
};
struct MpKeys {
  u64 k[kMaxParties];
};
hipError_t launch_mp_share(hipStream_t s, const u64* x, size_t n, int P, int src, const MpKeys& keys,
                           const MpOut& out);
hipError_t launch_mp_reveal(hipStream_t s, const MpIn& in, int P, size_t n, u64* out);
hipError_t launch_mp_fill_sum(hipStream_t s, const MpKeys& keys, int cnt, size_t n, const MpOut& out,
                              u64* sum);
hipError_t launch_mp_dealer_mul(hipStream_t s, const MpKeys& ka, const MpKeys& kb, const MpKeys& ks, int P,
                                size_t n, int square, const MpOut& a, const MpOut& b, const MpOut& c);
hipError_t launch_mp_open(hipStream_t s, const MpIn& x, const MpIn& a, int P, size_t n, u64* eps);
hipError_t launch_mp_beaver_mul(hipStream_t s, const MpIn& x, const MpIn& y, const MpIn& a, const MpIn& b,
                                const MpIn& c, int P, size_t n, int square, const MpOut& z);
hipError_t launch_mp_dealer_trunc(hipStream_t s, const MpKeys& kr, const MpKeys& kt, int P, size_t n,
                                  const MpOut& r, const MpOut& t);
hipError_t launch_mp_truncate(hipStream_t s, const MpOut& x, const MpIn& r, const MpIn& t, int P, size_t n,
                              int bits);

// ---------------------------------------------------------------- fp64 limb form
// The paper's GPU form of the ring GEMM: L fp64 limb planes per operand (L = 3
// of 22 bits when the concatenated k is below kFp64Limb22MaxK, else L = 4 of
// 16 bits), one fp64 GEMM per diagonal, exact combine.  Per-k diagonal sums
// are bounded by 2^43 (L = 3) and 2^32 (L = 4), so every partial sum of up to
// kFp64Limb22MaxK (resp. kFp64MaxK) terms stays an integer below 2^53.
constexpr i64 kFp64Limb22MaxK = 1024;     // L = 3 needs Kt < 2^10
constexpr i64 kFp64MaxK = (i64)1 << 21;   // L = 4 needs Kt < 2^21
int fp64_limbs(i64 Kt);
// LA: M x (L*Kt) row-major, limb i in columns [i*Kt, (i+1)*Kt)
hipError_t launch_fp64_pack_left(hipStream_t s, i64 M, i64 K0, i64 K1, const u64* A0, i64 lda0,
                                 const u64* A1, i64 lda1, int L, double* LA);
// RB: (L*Kt) x N row-major, limb j in rows [(L-1-j)*Kt, (L-j)*Kt)
hipError_t launch_fp64_pack_right(hipStream_t s, i64 N, i64 K0, i64 K1, const u64* B0, i64 ldb0,
                                  const u64* B1, i64 ldb1, int L, double* RB);
// X: L x M x N row-major diagonal sums -> epilogue
hipError_t launch_fp64_combine(hipStream_t s, i64 M, i64 N, int L, const double* X, const Epilogue& ep);

// Problems of one GEMM launch: `probs` with `map.tile_start` (device), or when
// `probs` is null the first map.nprob entries of iprobs/itile_start.  The
// persistent variant also takes `queue` (kLimbQueueWords zeroed words of
// device memory, left zeroed when the launch ends; launches that share them
// must not overlap in time) and runs `persist_grid` workgroups.
constexpr int kLimbQueueWords = 16;
struct GemmTables {
  const LimbProblem* probs;
  TileMap map;
  TileSched sched;
  unsigned* queue;
  int persist_grid;
  LimbProblem iprobs[kInlineProbs];
  int itile_start[kInlineProbs + 1];
};
hipError_t launch_limb_gemm(hipStream_t s, const GemmTables& t, int total_tiles);
// Workgroups of a persistent launch over `total_tiles` tiles on `num_cu` CUs.
int limb_persist_grid(int total_tiles, int num_cu);
int limb_tiles(i64 M, i64 N, int variant);
int limb_variant_bm(int variant);  // output rows of a workgroup tile
int limb_variant_bn(int variant);  // and columns
int limb_class_tiles(i64 M, i64 N, int cls);  // tiles of an M x N product in tile class cls
void limb_class_shape(int cls, int* bm, int* bn);  // workgroup tile of tile class cls
i64 limb_rblocks(i64 rows);  // padded 32-row block count
i64 limb_kblocks(i64 K);

}  // namespace mpc
