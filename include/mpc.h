/*
 * mpc.h -- C ABI of libmpc: two-party arithmetic secret sharing over the ring
 * Z/2^64 on one AMD MI355X (gfx950).
 *
 * The operations are those of CrypTen (Knott et al., NeurIPS 2021): additive
 * sharing of fixed-point values (section 5.1), Beaver multiplication of shared
 * values and its bilinear variants (section 5.2 and App. C.1.1), the square
 * with a Beaver pair (App. C.1.1, Square), local share truncation (App. C.1.1,
 * Truncation; zero rounds for two parties per Table 1) and reveal.
 *
 * Conventions for every call below.
 *   - Ring elements are uint64_t; arithmetic wraps modulo 2^64.  A fixed-point
 *     value with f fractional bits is the ring element whose signed 64-bit
 *     reading is round(x * 2^f).
 *   - Unless a parameter says "host", every pointer is a DEVICE pointer on the
 *     context's device, 8-byte aligned, to a dense row-major array owned by the
 *     caller.  The library owns only the context and its workspace.
 *   - Both parties' shares live on the one GPU as separate buffers ("party 0"
 *     and "party 1"), and the context holds one HIP stream per party.  Every
 *     call is issued on party 0's stream: it sees all work the caller ordered
 *     before it on that stream, and work the caller orders after it on that
 *     stream sees its results.  Work local to party 1 (its truncation) is
 *     forked onto party 1's stream with an event and joined back before the
 *     call returns.  Steps that need both parties (opening a masked value,
 *     reveal, the dealer) are device-local sums on party 0's stream; nothing
 *     crosses a network or a second GPU.
 *   - Every call is asynchronous with respect to the host.  Argument errors are
 *     reported synchronously; faults in kernels are reported by mpc_sync().
 *   - No call throws, aborts or prints.  Outputs must not alias inputs unless a
 *     call says so (MPC_E_ALIAS).
 *   - A context is used by one host thread at a time (its workspace, upload
 *     buffers and counters are not locked); different contexts may be used
 *     from different threads at once.
 *   - Sizes are element counts.  n = 0 (or an empty matrix) is valid and does
 *     nothing.
 *   - Randomness: G(seed, tag, slot, i) is a counter-based SplitMix64 value
 *     (Steele, Lea and Flood, OOPSLA 2014): with out_i(s) = mix(s + (i+1)γ),
 *     T = out_tag(seed), S = out_slot(T), G = out_i(S).  Slots: 0 share mask,
 *     1 a_0, 2 a_1, 3 b_0, 4 b_1, 5 c_0.  Equal (seed, tag) always regenerate
 *     identical shares and triples; reusing a triple is the caller's bug.
 */
#ifndef MPC_H
#define MPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPC_OK = 0,
  MPC_E_INVAL = -1,       /* null pointer, misalignment, bad enum or bit count */
  MPC_E_SHAPE = -2,       /* negative or inconsistent sizes */
  MPC_E_ALIAS = -3,       /* an output overlaps an input */
  MPC_E_NOMEM = -4,       /* workspace allocation failed */
  MPC_E_HIP = -5,         /* a HIP runtime call failed (see mpc_last_hip_error) */
  MPC_E_UNSUPPORTED = -6, /* valid request the library does not support */
  MPC_E_RANGE = -7        /* a real value does not fit the fixed-point range */
} mpc_status;

/* Form of the ring matrix product.
 *   PLAIN: uint64 wraparound multiply-accumulate on the vector ALUs.
 *   LIMB8: each operand split into eight signed 8-bit limbs; the 36 limb
 *          pairs (i, j) with i + j <= 7 are multiplied on INT8 matrix cores
 *          with exact int32 accumulation (K split so no sum can overflow) and
 *          combined as sum 2^(8(i+j)) D_i E_j mod 2^64.  Bit-identical to PLAIN.
 *          Each operand's k range (K of a product; each of the two halves of
 *          a Beaver finish, whose summed k is 2K) is at most 2,097,088 long;
 *          longer ones return MPC_E_UNSUPPORTED.
 *   AUTO:  the library's choice (LIMB8 unless the problem is tiny or its k
 *          is longer than LIMB8 takes; then PLAIN).
 *   FP64LIMB: the paper's own GPU method (Section 5.3, off-loading to the
 *          GPU): operands split into four 16-bit limbs (ten pairwise products)
 *          or, when the summed k is below 1024, three 22-bit limbs (six), each
 *          pairwise product an exact float64 GEMM of the vendor BLAS, combined
 *          mod 2^64.  Bit-identical to PLAIN; kept for comparison.  Supported
 *          by mpc_ring_gemm, mpc_beaver_matmul, mpc_beaver_matmul_grouped and
 *          mpc_beaver_conv1d (over im2col matrices written to the workspace)
 *          for summed k below 2^21; otherwise MPC_E_UNSUPPORTED.  The vendor
 *          BLAS handle is made on the context's first fp64 call, which must
 *          not be under graph capture (MPC_E_UNSUPPORTED, nothing recorded);
 *          after that, fp64 calls are captured like any other. */
typedef enum {
  MPC_FORM_PLAIN = 0,
  MPC_FORM_LIMB8 = 1,
  MPC_FORM_AUTO = 2,
  MPC_FORM_FP64LIMB = 3
} mpc_form;

typedef enum {
  MPC_TRIPLE_MUL = 0,    /* element-wise: a, b, c = a*b, all of length n          */
  MPC_TRIPLE_SQUARE = 1, /* Beaver pair: a and b = a*a of length n; c unused      */
  MPC_TRIPLE_MATMUL = 2, /* a: MxK, b: KxN, c = a@b: MxN                          */
  MPC_TRIPLE_CONV1D = 3  /* a: activation [B][Cin][L], b: weight [Cout][Cin][k],
                            c = conv1d(a, b): [B][Cout][Lout]                     */
} mpc_triple_kind;

/* Additive shares of a Beaver triple: party p holds a_p, b_p, c_p. */
typedef struct {
  uint64_t *a0, *a1, *b0, *b1, *c0, *c1;
} mpc_triple;

/* 1-D convolution with valid padding: Lout = (length - ksize) / stride + 1. */
typedef struct {
  int64_t batch, cin, length, cout, ksize, stride;
} mpc_conv1d_shape;

typedef struct mpc_ctx mpc_ctx;

/* Counters kept by a context: opens (communication rounds: one per Beaver
 * product, AND gate, B2A conversion and reveal, seven per A2B conversion, one
 * per truncation among more than two parties, none for a two-party
 * truncation), bytes a two-GPU deployment would send per party in those
 * rounds, truncations, kernel launches and GEMM problems issued. */
typedef struct {
  uint64_t opens, open_bytes_per_party, truncations, launches, gemm_problems;
} mpc_stats;

const char *mpc_status_str(mpc_status s);
/* Last HIP error code seen by the library in this process (0 if none). */
int mpc_last_hip_error(void);

/* ---- host-only fixed-point codec (section 5.1) ------------------------- */
/* out[i] = round-half-even(x[i] * 2^frac_bits) as int64.  x and out are HOST
 * pointers.  MPC_E_RANGE if a value (or NaN) does not fit; out is then
 * partially written.  frac_bits in [0, 62]. */
mpc_status mpc_encode(const double *x, size_t n, int frac_bits, int64_t *out);
/* out[i] = (double)v[i] / 2^frac_bits.  HOST pointers. */
mpc_status mpc_decode(const int64_t *v, size_t n, int frac_bits, double *out);

/* ---- context ------------------------------------------------------------ */
/* Binds `device` and the two party streams (hipStream_t values).  stream0 may
 * be NULL, the device's null stream; stream1 NULL makes the library create and
 * own a stream for party 1.  `seed` is the parties' synchronised PRG seed used
 * for sharing. */
mpc_status mpc_ctx_create(int device, void *stream0, void *stream1, uint64_t seed,
                          mpc_ctx **out);
/* Waits for both party streams and frees the context and its buffers;
 * MPC_E_INVAL (nothing freed) while a graph it captured still exists. */
mpc_status mpc_ctx_destroy(mpc_ctx *ctx);
/* Waits for both party streams; reports kernel faults. */
mpc_status mpc_sync(mpc_ctx *ctx);
mpc_status mpc_ctx_stats(const mpc_ctx *ctx, mpc_stats *out);
/* Pre-sizes the library-owned workspace to at least `bytes` (optional; calls
 * grow it on demand, synchronising both streams when they do). */
mpc_status mpc_reserve(mpc_ctx *ctx, size_t bytes);

/* ---- sharing (section 5.1) --------------------------------------------- */
/* Party `src` (0 or 1) secret-shares the ring elements x[0..n):
 *   m_i = G(seed, tag, 0, i);  s_src = x - m;  s_other = m.
 * x, s0, s1: device arrays of n.  s0/s1 must not overlap x or each other. */
mpc_status mpc_share(mpc_ctx *ctx, const uint64_t *x, size_t n, int src, uint64_t tag,
                     uint64_t *s0, uint64_t *s1);
/* out = s0 + s1 mod 2^64 (read it as int64 for the signed value).  out may
 * be s0 or s1 itself (in place); any other overlap returns MPC_E_ALIAS. */
mpc_status mpc_reveal(mpc_ctx *ctx, const uint64_t *s0, const uint64_t *s1, size_t n,
                      uint64_t *out);
/* Local truncation, in place: each party replaces its share s by
 * floor(s64(s) / 2^bits) on its own stream.  bits in [0, 63]. */
mpc_status mpc_truncate(mpc_ctx *ctx, uint64_t *s0, uint64_t *s1, size_t n, int bits);

/* ---- trusted third party (section 4; App. C.1.1) ------------------------ */
/* Draws a fresh triple from the dealer's own seed:
 *   a_p = G(dseed, tag, 1+p, i), b_p = G(dseed, tag, 3+p, i),
 *   c_0 = G(dseed, tag, 5, i),   c_1 = f(a_0 + a_1, b_0 + b_1) - c_0,
 * f being *, @ or conv1d per `kind`; for SQUARE b_1 = (a_0 + a_1)^2 - b_0.
 * dims: MUL/SQUARE {n}; MATMUL {M, N, K}; CONV1D the six fields of
 * mpc_conv1d_shape in order.  `out` is a HOST struct of device pointers sized
 * for the kind (c0/c1 ignored for SQUARE). */
mpc_status mpc_dealer_triples(mpc_ctx *ctx, mpc_triple_kind kind, uint64_t dseed, uint64_t tag,
                              const int64_t *dims, const mpc_triple *out);

/* ---- Beaver products (section 5.2; App. C.1.1) -------------------------- */
/* Element-wise product of shared x and y with an element-wise triple:
 *   eps = sum_p (x_p - a_p), delta = sum_p (y_p - b_p)   (the one open)
 *   z_p = c_p + eps*b_p + a_p*delta (+ eps*delta for party 0)
 * With y0 == y1 == NULL it is the square with a Beaver pair (a, b = a^2):
 *   z_p = b_p + 2*eps*a_p (+ eps^2 for party 0).
 * Then each party truncates by trunc_bits (0 = none, else 1..63).  All arrays
 * have n elements; `t` is a HOST struct of device pointers.  z may not
 * overlap any input. */
mpc_status mpc_beaver_mul(mpc_ctx *ctx, size_t n, const uint64_t *x0, const uint64_t *x1,
                          const uint64_t *y0, const uint64_t *y1, const mpc_triple *t,
                          int trunc_bits, uint64_t *z0, uint64_t *z1);

/* Matrix product of shared X (MxK) and Y (KxN) with a matrix triple:
 *   z_p = c_p + eps @ b_p + (a_p + [p = 0] eps) @ delta,  then truncation.
 * Each party's finish is one ring GEMM of M x N x 2K over the concatenations
 * [eps | a_p + [p=0] eps] and [b_p ; delta]; both parties' GEMMs are issued as
 * one launch on party 0's stream.  z_p: MxN. */
mpc_status mpc_beaver_matmul(mpc_ctx *ctx, int64_t M, int64_t N, int64_t K, const uint64_t *x0,
                             const uint64_t *x1, const uint64_t *y0, const uint64_t *y1,
                             const mpc_triple *t, int trunc_bits, mpc_form form, uint64_t *z0,
                             uint64_t *z1);

/* mpc_beaver_matmul for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same product, bit for bit, with no hipMalloc, hipFree or host pinned
 * allocation in the call.  Its workspace is one 64 MiB array per device,
 * part of the library's code object (resident from the first context on that
 * device until the process ends), that every such call on that device shares:
 * calls that overlap in time on one device (any context, any stream) race and
 * must be ordered by the caller.  The packed operands must fit it:
 * 24*(M*K + K*N) bytes up to padding (e.g. M = N = K = 1024), else
 * MPC_E_SHAPE.  form: MPC_FORM_LIMB8, or MPC_FORM_AUTO, which also takes the
 * one-launch plain product for products of at most 2^18 multiply-accumulates
 * (no workspace); other forms return MPC_E_UNSUPPORTED.  The limb GEMM runs
 * without split-K and its descriptor tables travel in the kernel arguments.
 * MPC_E_HIP if the array's address could not be found when the context was
 * created.  GEMM launches of this call are not timed by mpc_profile_*. */
mpc_status mpc_beaver_matmul_noalloc(mpc_ctx *ctx, int64_t M, int64_t N, int64_t K, const uint64_t *x0,
                                     const uint64_t *x1, const uint64_t *y0, const uint64_t *y1,
                                     const mpc_triple *t, int trunc_bits, mpc_form form, uint64_t *z0,
                                     uint64_t *z1);

/* Convolution of a shared activation x [B][Cin][L] with a shared weight
 * w [Cout][Cin][k] (valid padding) with a CONV1D triple, lowered onto the ring
 * GEMM (weights as the left operand, im2col of the activation as the right):
 *   z_p = c_p + conv(eps, b_p) + conv(a_p + [p=0] eps, delta), then truncation.
 * z_p: [B][Cout][Lout]. */
mpc_status mpc_beaver_conv1d(mpc_ctx *ctx, const mpc_conv1d_shape *shape, const uint64_t *x0,
                             const uint64_t *x1, const uint64_t *w0, const uint64_t *w1,
                             const mpc_triple *t, int trunc_bits, mpc_form form, uint64_t *z0,
                             uint64_t *z1);

/* Public ring GEMM C = A @ B mod 2^64 (A: MxK, B: KxN, C: MxN), on party 0's
 * stream: the kernel the Beaver forms use, exposed for comparison. */
mpc_status mpc_ring_gemm(mpc_ctx *ctx, int64_t M, int64_t N, int64_t K, const uint64_t *A,
                         const uint64_t *B, uint64_t *C, mpc_form form);

/* ---- measurement -------------------------------------------------------- */
/* While enabled, every ring GEMM launch the context issues is bracketed by two
 * HIP events on the stream it is launched on (party 0's).  mpc_profile_read
 * waits for both party streams, then returns per form the number of GEMM
 * launches since the last read, their summed event-measured duration and
 * their algorithmic work (ring multiply-accumulates M*N*K over true, unpadded
 * sizes; the limb form also performs 36 int8 multiply-accumulates per ring
 * one, the fp64 limb form 6 or 10 float64 ones), and clears the record.  In
 * the fp64 limb form the bracket covers its vendor-BLAS GEMM calls (one per
 * limb diagonal) as one launch.  Any output pointer may be NULL. */
typedef struct {
  uint64_t launches;
  double total_ms;
  double ring_macs;
} mpc_gemm_timing;
mpc_status mpc_profile_enable(mpc_ctx *ctx, int on);
mpc_status mpc_profile_read(mpc_ctx *ctx, mpc_gemm_timing *limb8, mpc_gemm_timing *plain,
                            mpc_gemm_timing *fp64limb);

/* ---- batching form ------------------------------------------------------ */
/* One Beaver matmul of a group (all pointers device, as in mpc_beaver_matmul). */
typedef struct {
  int64_t M, N, K;
  const uint64_t *x0, *x1, *y0, *y1;
  mpc_triple t;
  uint64_t *z0, *z1;
} mpc_matmul_desc;

/* Many independent Beaver matmuls of uneven shapes (batching amortises the
 * rounds, Section 6.1): in the limb form one fused open+pack launch per
 * operand kind and one grouped GEMM launch over the tiles of all problems and
 * both parties (a tile-to-problem table; one workgroup per tile, handed out
 * by the hardware dispatcher); the plain form likewise with one open launch.
 * Each problem follows mpc_beaver_matmul's rules, and since the problems run
 * concurrently no output may overlap another problem's inputs or outputs
 * (MPC_E_ALIAS).  `descs` is a HOST array of `count` descriptors. */
mpc_status mpc_beaver_matmul_grouped(mpc_ctx *ctx, size_t count, const mpc_matmul_desc *descs,
                                     int trunc_bits, mpc_form form);

/* ---- offline-packed matrix triples (limb form) --------------------------- */
/* Triples are made offline by the dealer (section 4, the trusted third
 * party; App. C.1.1).  Three of a matrix triple's shares enter the finish
 * unchanged, a_1 (party 1's left operand) and b_0, b_1 (the right ones), so
 * the dealer can also store them in the limb form's packed layout; the online
 * Beaver matmul then packs only eps, a_0 + eps and delta (the open step's
 * writes fall from 6 to 3 packed operands).  `packed` is a caller-owned
 * device buffer of mpc_packed_triple_bytes(M, N, K) bytes, 256-byte aligned,
 * holding the three packed operands; it belongs to the triple and is read by
 * the online call, never written.
 *
 * mpc_packed_triple_bytes: that size (0 for shapes mpc_beaver_matmul would
 * refuse).  mpc_dealer_triples_packed: exactly the MATMUL triple of
 * mpc_dealer_triples with the same (dseed, tag), plus `packed` (left
 * unwritten when M, N or K is 0; MPC_E_UNSUPPORTED for K beyond the limb
 * form's segment).  mpc_beaver_matmul_prepacked and its grouped form: the
 * limb-form mpc_beaver_matmul / mpc_beaver_matmul_grouped (same shares, bit
 * for bit) with the triples' packed operands; `packed` must not overlap an
 * output (MPC_E_ALIAS); null or misaligned: MPC_E_INVAL. */
size_t mpc_packed_triple_bytes(int64_t M, int64_t N, int64_t K);
mpc_status mpc_dealer_triples_packed(mpc_ctx *ctx, uint64_t dseed, uint64_t tag, int64_t M, int64_t N, int64_t K,
                                     const mpc_triple *out, void *packed);
mpc_status mpc_beaver_matmul_prepacked(mpc_ctx *ctx, int64_t M, int64_t N, int64_t K, const uint64_t *x0,
                                       const uint64_t *x1, const uint64_t *y0, const uint64_t *y1,
                                       const mpc_triple *t, const void *packed, int trunc_bits, uint64_t *z0,
                                       uint64_t *z1);
/* `packed`: HOST array of `count` device pointers, one per descriptor. */
mpc_status mpc_beaver_matmul_grouped_prepacked(mpc_ctx *ctx, size_t count, const mpc_matmul_desc *descs,
                                               const void *const *packed, int trunc_bits);

/* Many independent element-wise Beaver products (or squares) of uneven
 * lengths in ONE launch (section 5.2; batching amortises the rounds, Section
 * 6.1): each descriptor is what mpc_beaver_mul takes (y0 == y1 == NULL for a
 * square with the pair a, b = a^2; c unused then), all truncated by
 * trunc_bits.  One workgroup per chunk of 1024 elements of one product, found
 * through a chunk table uploaded with the call (a permanent buffer made
 * before capture when the call is captured in a graph).  Validation and
 * aliasing rules are those of mpc_beaver_mul, and since the products run
 * concurrently no output may overlap another product's inputs or outputs
 * (MPC_E_ALIAS).  `descs` is a HOST array of `count` descriptors. */
typedef struct {
  size_t n;
  const uint64_t *x0, *x1, *y0, *y1;
  mpc_triple t;
  uint64_t *z0, *z1;
} mpc_mul_desc;
mpc_status mpc_beaver_mul_grouped(mpc_ctx *ctx, size_t count, const mpc_mul_desc *descs, int trunc_bits);

/* ---- autotuning of the limb GEMM ---------------------------------------- */
/* A tile schedule: the workgroup tile shape (0: 128x64, 1: 64x128, 2: 64x64
 * outputs, every wave fetching its operand fragments from global memory;
 * 3, 4, 5: the same shapes with the operand that has more fragments per wave
 * copied once per workgroup into LDS and read from there; 6: 64x128 and
 * 7: 128x64 in that LDS form with eight waves, two per SIMD, each wave 16x64
 * or 64x16 outputs; 8: 64x128 with eight waves of 32x32 outputs; 9, 10, 11:
 * 64x64 (two workgroups per compute unit), 64x128 and 128x64 (eight waves)
 * with both operands copied once per workgroup into LDS and every wave
 * owning 32x32 outputs; 12: 32x128 and 13: 128x32 thin tiles in the LDS
 * form, four waves of 32x32 outputs in a row or a column, two workgroups per
 * compute unit; 14: every product in its own tile class, 64x64, 32x128 or
 * 128x32, in one launch; 15: schedule 14 as a persistent launch, two
 * workgroups per compute unit taking tiles from per-XCD queues in the order
 * that schedule 14 dispatches them, its queue heads in a 64-byte buffer of
 * the context), the number of tile
 * rows per raster group, and whether tiles are handed to the 8 XCDs in runs
 * of 32 neighbouring tiles (one per compute unit, so that the tiles an XCD
 * runs together share operand blocks in its L2) instead of one by one.
 * group_m is 1..64: schedules outside that range (from mpc_set_default_tile_config
 * or a cache file) are refused or, when loaded, skipped. */
typedef struct {
  int variant, group_m, xcd_remap;
  double ms; /* measured time of the tuned launch(es), filled by the tuner */
} mpc_tile_config;

/* Tile classes: a limb-form Beaver matmul (single or grouped) gives each
 * product a class by its shape: "thin in M" (at most 32 rows) or "thin in N"
 * (at most 32 columns) when the 32x128 or 128x32 tile leaves at most nine
 * tenths of the 64x64 tile's padded work, else "regular"; a grouped call
 * issues one GEMM launch per schedule in use.  Under schedules 14 and 15 a
 * regular product's last rows (columns), when they fill at most half of a
 * 64-row (64-column) tile, run as a strip of 32x128 (128x32) tiles beside its
 * 64x64 tiles, wherever that issues fewer outputs than the 64x64 tiles
 * alone.  Untuned, every product takes
 * the default schedule (schedule 14 or 15 as the default: each product in its
 * own class), unless some product is thin and no default was set
 * with mpc_set_default_tile_config: then all of them run in one launch of
 * schedule 14, each in its own class (with the default's group_m and
 * remap).
 *
 * mpc_autotune_matmul times every tile schedule, class by class, on the
 * exact GEMM problems that a Beaver matmul (count = 1) or a grouped call of
 * these `count` shapes issues in the limb form (dims: HOST array of M, N, K
 * per problem), on random operands, and remembers each class's fastest for
 * later calls with the same shapes, unless one launch of all of them is
 * faster than the classes' separate launches (each single schedule, and
 * schedules 14 and 15 with every product in its own class, are timed that way).  `best` (may be NULL) receives the
 * schedule of the class that takes longest and, in `ms`, the summed time of
 * all classes.  Uses the context's workspace and party 0's stream;
 * synchronises it. */
mpc_status mpc_autotune_matmul(mpc_ctx *ctx, size_t count, const int64_t *dims, mpc_tile_config *best);
/* Writes / reads the tuned schedules (a text file, one line per shape list:
 * its hash, then variant, group_m and remap of the regular, thin-in-M and
 * thin-in-N classes). */
mpc_status mpc_autotune_save(const mpc_ctx *ctx, const char *path);
mpc_status mpc_autotune_load(mpc_ctx *ctx, const char *path);
/* Schedule used when no tuned entry matches (default: shape 5, the 64x64
 * LDS tile at two workgroups per compute unit, group_m 8, remap on): set it,
 * or read it back (`ms` reads 0). */
mpc_status mpc_set_default_tile_config(mpc_ctx *ctx, const mpc_tile_config *cfg);
mpc_status mpc_get_default_tile_config(const mpc_ctx *ctx, mpc_tile_config *cfg);

/* Host-only planning query (no context, no device work): how the limb GEMM
 * tiles one product's M x N row-major output under tile schedule `variant`
 * (0..15, as above).  *cls receives the product's tile class (0 regular,
 * 1 thin in M, 2 thin in N; the rule above).  `regions` (HOST, room for 4
 * entries of 6 int64) receives the output rectangles that run as GEMM
 * problems of their own, each as first row, first column, rows, columns,
 * tile rows, tile columns, and *count their number: the whole output in the
 * variant's tile (under 14 and 15 the class's tile), except that under 14
 * and 15 a regular product with edge strips gives its 64x64 interior, the
 * strips and their corner.  Every rectangle starts at a multiple of 32 rows
 * and columns, and its tiles stay inside the packed operands' padded extent
 * (rows and columns rounded up to a multiple of 128).  `tiles` (may be NULL)
 * receives the tile count over all regions.  Column-strided outputs (the
 * convolution's) always run whole.  MPC_E_INVAL for a null output or a
 * variant outside 0..15, MPC_E_SHAPE for M or N below 1 or M * N beyond the
 * element limit. */
mpc_status mpc_limb_plan(int64_t M, int64_t N, int variant, int *cls, int64_t *regions, int *count,
                         int64_t *tiles);

/* Stream capture of the context's work into a HIP graph: begin, issue calls,
 * end.  Party 0's stream must not be the null stream (MPC_E_INVAL).  The workspace must
 * already be large enough (issue the same calls once eagerly first, or call
 * mpc_reserve).  mpc_graph_launch replays the graph on party 0's stream of
 * the context that captured it (MPC_E_INVAL for another context);
 * mpc_graph_destroy frees it.  A graph refers to the context's workspace by
 * address, so while any graph of a context exists the workspace cannot move:
 * a call that would need a larger one returns MPC_E_NOMEM (reserve enough
 * before capturing).  A graph owns the descriptor buffers made while it was
 * captured and frees them in mpc_graph_destroy, which first waits for party
 * 0's stream.  Destroy a context's graphs before the context:
 * mpc_ctx_destroy returns MPC_E_INVAL and frees nothing while any exists. */
mpc_status mpc_graph_begin(mpc_ctx *ctx);
mpc_status mpc_graph_end(mpc_ctx *ctx, void **graph_exec);
mpc_status mpc_graph_launch(mpc_ctx *ctx, void *graph_exec);
mpc_status mpc_graph_destroy(void *graph_exec);

/* ---- binary sharing, two parties (App. C.1.1) -----------------------------
 * A binary sharing holds 64 independent shared bits per word:
 * x = <x>_0 XOR <x>_1.  Bitwise AND uses triples (a, b, c = a AND b) from the
 * dealer, one per word.  All calls run on party 0's stream; every opening is
 * a device-local XOR, and each counts as one opening (one round) in the
 * statistics.  Outputs must not alias inputs (MPC_E_ALIAS).  PRG domains:
 * slot 0x700 of (seed, tag) for sharing, 0x706/0x707 for the parties'
 * re-sharing inside A2B; slots 0x701-0x705 and 0x708-0x70a of (dseed, tag)
 * for the dealer. */

/* Binary sharing (XOR zero-share (m, m); party src XORs in x) and reveal. */
mpc_status mpc_bin_share(mpc_ctx *ctx, const uint64_t *x, size_t n, int src, uint64_t tag, uint64_t *s0,
                         uint64_t *s1);
mpc_status mpc_bin_reveal(mpc_ctx *ctx, const uint64_t *s0, const uint64_t *s1, size_t n, uint64_t *out);
/* n bitwise AND triples (words): a_p, b_p uniform, c = a AND b XOR-shared. */
mpc_status mpc_dealer_and_triples(mpc_ctx *ctx, uint64_t dseed, uint64_t tag, size_t n, const mpc_triple *out);
/* Bitwise AND (App. C.1.1, Bitwise AND): eps = x ^ a, delta = y ^ b opened;
 * z_p = c_p ^ (eps & b_p) ^ (a_p & delta) (^ eps & delta for party 0). */
mpc_status mpc_bin_and(mpc_ctx *ctx, size_t n, const uint64_t *x0, const uint64_t *x1, const uint64_t *y0,
                       const uint64_t *y1, const mpc_triple *t, uint64_t *z0, uint64_t *z1);
/* Arithmetic to binary sharing (App. C.1.1, From [x] to <x>): each party
 * binary-shares its arithmetic share, and a carry-lookahead adder over binary
 * shares adds them: 7 rounds, 12 AND triples per word (t holds 12*n triples,
 * triple j of word i at j*n + i, e.g. from mpc_dealer_and_triples with 12*n). */
mpc_status mpc_a2b(mpc_ctx *ctx, size_t n, const uint64_t *x0, const uint64_t *x1, uint64_t tag,
                   const mpc_triple *t, uint64_t *z0, uint64_t *z1);
/* The dealer of Algorithm 2's random bits: r in {0, 1} per word, shared as
 * <r> = (rb0, rb1) (bit 0) and [r] = (ra0, ra1). */
mpc_status mpc_dealer_b2a(mpc_ctx *ctx, uint64_t dseed, uint64_t tag, size_t n, uint64_t *rb0, uint64_t *rb1,
                          uint64_t *ra0, uint64_t *ra1);
/* Binary to arithmetic for bit `bit` (0..63) of each word (Algorithm 2):
 * z = that bit of <b> XOR <r> is opened, [b] = [r] + z - 2 z [r]. */
mpc_status mpc_b2a_bit(mpc_ctx *ctx, size_t n, int bit, const uint64_t *b0, const uint64_t *b1,
                       const uint64_t *rb0, const uint64_t *rb1, const uint64_t *ra0, const uint64_t *ra1,
                       uint64_t *z0, uint64_t *z1);
/* ReLU (App. C.1.1, Sign, absolute value, and ReLU) of a fixed-point sharing:
 * [x < 0] is the sign bit of A2B([x]) converted by Algorithm 2, and
 * z = [x] * (1 - [x < 0]) by one Beaver product with the MUL triple m (no
 * truncation).  9 rounds; t: 12*n AND triples; (rb, ra): n B2A bits; m: n. */
mpc_status mpc_relu(mpc_ctx *ctx, size_t n, const uint64_t *x0, const uint64_t *x1, uint64_t tag,
                    const mpc_triple *t, const uint64_t *rb0, const uint64_t *rb1, const uint64_t *ra0,
                    const uint64_t *ra1, const mpc_triple *m, uint64_t *z0, uint64_t *z1);

/* ---- more than two parties (App. C.1.1; Algorithm 1) --------------------
 * A sharing among P parties (2 <= P <= MPC_MAX_PARTIES) is a HOST array of P
 * device pointers, one buffer per party, all of the same length.  Every call
 * runs all parties' work on party 0's stream, as one pass per step (the
 * opening of a masked value is a device-local sum over the P buffers); each
 * Beaver product and each truncation counts one opening.  Outputs must not
 * alias inputs (MPC_E_ALIAS), except mpc_mp_truncate, which works in place.
 * PRG domains: party p's zero-share stream is slot 0x100+p of (seed, tag);
 * the dealer's a, b, c, r, theta_r streams are slots 0x200+p ... 0x600+p of
 * (dseed, tag). */
#define MPC_MAX_PARTIES 16

/* Sharing (section 5.1): a pseudorandom zero-share of P numbers summing to 0,
 * z_p = m_p - m_{(p+1) mod P} with m_p party p's stream; party src adds x. */
mpc_status mpc_mp_share(mpc_ctx *ctx, int P, const uint64_t *x, size_t n, int src, uint64_t tag,
                        uint64_t *const *s);
/* x = sum_p s_p (mod 2^64). */
mpc_status mpc_mp_reveal(mpc_ctx *ctx, int P, const uint64_t *const *s, size_t n, uint64_t *out);

/* Shares of a triple among P parties (arrays indexed by party). */
typedef struct {
  uint64_t *a[MPC_MAX_PARTIES], *b[MPC_MAX_PARTIES], *c[MPC_MAX_PARTIES];
} mpc_mp_triple;
/* The dealer (TTP): a_p, b_p uniform; c = a*b (MUL), b = a*a (SQUARE, c
 * unused) or c = a@b (MATMUL) split as c_p = G(p) for p < P-1 and the rest
 * for the last party.  dims: {n} for MUL/SQUARE, {M, N, K} for MATMUL. */
mpc_status mpc_mp_dealer_triples(mpc_ctx *ctx, int P, mpc_triple_kind kind, uint64_t dseed, uint64_t tag,
                                 const int64_t *dims, const mpc_mp_triple *out);
/* The dealer of Algorithm 1's inputs: shares r_p of a uniform r and shares
 * t_p of r's wrap count theta_r (sum_p s64(r_p) = s64(r) + theta_r 2^64). */
mpc_status mpc_mp_dealer_trunc(mpc_ctx *ctx, int P, uint64_t dseed, uint64_t tag, size_t n,
                               uint64_t *const *r, uint64_t *const *theta_r);

/* Beaver product among P parties: eps = sum_p (x_p - a_p), delta likewise;
 * z_p = c_p + eps b_p + a_p delta (+ eps delta for party 0).  y == NULL: the
 * square with the pair (a, b = a^2), z_p = b_p + 2 eps a_p (+ eps^2). */
mpc_status mpc_mp_beaver_mul(mpc_ctx *ctx, int P, size_t n, const uint64_t *const *x,
                             const uint64_t *const *y, const mpc_mp_triple *t, uint64_t *const *z);
/* Beaver matmul among P parties (X: MxK, Y: KxN, z_p: MxN):
 * z_p = c_p + (a_p + [p=0] eps) @ delta + eps @ b_p, one ring GEMM of
 * M x N x 2K per party, all P in one launch (PLAIN, LIMB8 or AUTO). */
mpc_status mpc_mp_beaver_matmul(mpc_ctx *ctx, int P, int64_t M, int64_t N, int64_t K,
                                const uint64_t *const *x, const uint64_t *const *y, const mpc_mp_triple *t,
                                mpc_form form, uint64_t *const *z);
/* Truncation by 2^bits (1 <= bits <= 63) of a P-party sharing, in place, by
 * Algorithm 1 with eta = 0: z = x + r is opened with its wrap count, each
 * party's share of theta_x = theta_z + beta - theta_r is formed locally, and
 * x_p <- floor(s64(x_p) / 2^bits) - [theta_x]_p 2^(64 - bits).  The result is
 * within P-1 below floor(x / 2^bits) unless x + r leaves the signed range
 * (probability about |x| / 2^64).  r, theta_r from mpc_mp_dealer_trunc, one
 * fresh pair per truncation. */
mpc_status mpc_mp_truncate(mpc_ctx *ctx, int P, size_t n, int bits, uint64_t *const *x,
                           const uint64_t *const *r, const uint64_t *const *theta_r);

#ifdef __cplusplus
}
#endif

#endif /* MPC_H */
