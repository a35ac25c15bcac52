/*
 * oracle.c -- plain, slow, obviously correct CPU reference for two-party
 * arithmetic secret sharing over the ring Z/2^64 (CrypTen, Knott et al.,
 * NeurIPS 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library) shares no code, header, table or helper with this file and must
 * never call it.
 *
 * Every ring element is a uint64_t; C unsigned arithmetic wraps modulo 2^64,
 * which is exactly the ring of the paper (section 5.1, App. C.1.1: Q = 2^64).
 * The signed view of an element v is the two's-complement int64 with the same
 * bits.  Loops are the textbook definitions, with no blocking or fusion.  The
 * only liberty taken is OpenMP over independent output rows in the GEMM and
 * convolution loops; each output element is still the plain sum over k taken
 * in increasing k.
 *
 * Parity status: every function here is pinned by the CPU test-suite against
 * facts fixed outside this file (published PRG outputs, the paper's worked
 * example, Python arbitrary-precision products, numpy's uint64 matmul, the
 * truncation error law and closed forms).  See the test files for the pins.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef uint64_t u64;
typedef int64_t i64;

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets the number of threads later calls use (n < 1 is ignored). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Counter-based PRG.                                                        */
/*                                                                           */
/* The paper fixes no generator; it asks only that the parties draw          */
/* pseudorandom zero-shares from synchronised seeds (section 5.1) and that   */
/* the trusted third party draws uniform triples (section 5.2).  We use the  */
/* SplitMix64 generator (Steele, Lea and Flood, "Fast splittable             */
/* pseudorandom number generators", OOPSLA 2014): a stream with state s      */
/* returns, as its i-th output (i = 0, 1, ...), mix(s + (i+1)*GAMMA).         */
/* Domains are nested streams:                                               */
/*   T = output number `tag`  of the stream with state `seed`                */
/*   S = output number `slot` of the stream with state T                     */
/*   G(seed, tag, slot, idx) = output number `idx` of the stream with state S */
/* ------------------------------------------------------------------------ */
#define SM_GAMMA 0x9e3779b97f4a7c15ULL

u64 orc_sm64_mix(u64 z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* i-th output (0-based) of the SplitMix64 stream whose state starts at s */
u64 orc_sm64_at(u64 s, u64 i) { return orc_sm64_mix(s + (i + 1) * SM_GAMMA); }

u64 orc_prg(u64 seed, u64 tag, u64 slot, u64 idx) {
  u64 t = orc_sm64_at(seed, tag);
  u64 s = orc_sm64_at(t, slot);
  return orc_sm64_at(s, idx);
}

void orc_prg_fill(u64 seed, u64 tag, u64 slot, size_t n, u64 *out) {
  for (size_t i = 0; i < n; ++i) out[i] = orc_prg(seed, tag, slot, (u64)i);
}

void orc_prg_at(u64 seed, u64 tag, u64 slot, const u64 *idx, size_t n, u64 *out) {
  for (size_t t = 0; t < n; ++t) out[t] = orc_prg(seed, tag, slot, idx[t]);
}

/* PRG slots (domains inside one tag). */
enum { SLOT_SHARE = 0, SLOT_A0 = 1, SLOT_A1 = 2, SLOT_B0 = 3, SLOT_B1 = 4, SLOT_C0 = 5 };

/* ------------------------------------------------------------------------ */
/* Fixed-point encoding (section 5.1, App. C.1.1): x = round(B * x_R) with    */
/* B = 2^L; decoding is x / B.  Rounding is to nearest with ties to even      */
/* (C rint() in the default rounding mode).  Values whose encoding does not  */
/* fit a signed 64-bit integer are rejected: returns the index+1 of the      */
/* first offending element, 0 on success.                                    */
/* ------------------------------------------------------------------------ */
size_t orc_encode(const double *x, size_t n, int frac_bits, i64 *out) {
  const double scale = ldexp(1.0, frac_bits);
  for (size_t i = 0; i < n; ++i) {
    double r = rint(x[i] * scale);
    if (!(r >= -9223372036854775808.0 && r < 9223372036854775808.0)) return i + 1;
    out[i] = (i64)r;
  }
  return 0;
}

void orc_decode(const u64 *v, size_t n, int frac_bits, double *out) {
  const double scale = ldexp(1.0, frac_bits);
  for (size_t i = 0; i < n; ++i) out[i] = (double)(i64)v[i] / scale;
}

/* ------------------------------------------------------------------------ */
/* Sharing and reveal (section 5.1).                                          */
/* Two parties: the zero-share is (-m, m) with m = G(seed, tag, SHARE, i);    */
/* the source party adds its value, so s_src = x - m and s_other = m.         */
/* ------------------------------------------------------------------------ */
/* Element i of the vector, whose value there is x. */
static void share_elem(u64 x, u64 i, int src, u64 seed, u64 tag, u64 *s0, u64 *s1) {
  u64 m = orc_prg(seed, tag, SLOT_SHARE, i);
  u64 zs_src = (u64)0 - m; /* the two zero-share entries sum to 0 mod Q */
  u64 zs_other = m;
  if (src == 0) {
    *s0 = x + zs_src;
    *s1 = zs_other;
  } else {
    *s0 = zs_other;
    *s1 = x + zs_src;
  }
}

void orc_share(const u64 *x, size_t n, int src, u64 seed, u64 tag, u64 *s0, u64 *s1) {
  for (size_t i = 0; i < n; ++i) share_elem(x[i], (u64)i, src, seed, tag, &s0[i], &s1[i]);
}

/* Selected elements only: x[t] is the value of element idx[t]. */
void orc_share_at(const u64 *x, const u64 *idx, size_t n, int src, u64 seed, u64 tag, u64 *s0,
                  u64 *s1) {
  for (size_t t = 0; t < n; ++t) share_elem(x[t], idx[t], src, seed, tag, &s0[t], &s1[t]);
}

/* x = sum_p [x]_p mod Q */
void orc_reveal(const u64 *s0, const u64 *s1, size_t n, u64 *out) {
  for (size_t i = 0; i < n; ++i) out[i] = s0[i] + s1[i];
}

/* Private addition (App. C.1.1, Addition): each party adds its own shares. */
void orc_add(const u64 *x, const u64 *y, size_t n, u64 *out) {
  for (size_t i = 0; i < n; ++i) out[i] = x[i] + y[i];
}

/* ------------------------------------------------------------------------ */
/* Truncation (App. C.1.1, Truncation; Table 1: zero rounds for two parties).  */
/* Each party divides its own share, read as a signed integer, by 2^bits,    */
/* rounding toward minus infinity.  Written as an explicit floor division.   */
/* ------------------------------------------------------------------------ */
static i64 floor_div_pow2(i64 v, int bits) {
  if (bits == 0) return v;
  if (bits == 63) return v < 0 ? -1 : 0; /* 2^63 itself is not an int64 */
  const i64 d = (i64)1 << bits;
  i64 q = v / d; /* C division truncates toward zero */
  i64 r = v % d;
  if (r != 0 && v < 0) q -= 1;
  return q;
}

void orc_truncate(u64 *s, size_t n, int bits) {
  for (size_t i = 0; i < n; ++i) s[i] = (u64)floor_div_pow2((i64)s[i], bits);
}

/* ------------------------------------------------------------------------ */
/* Plain ring products.                                                      */
/* ------------------------------------------------------------------------ */
/* C[i][j] = sum_k A[i][k] * B[k][j] mod 2^64; A is MxK, B is KxN, row-major. */
void orc_ring_gemm(i64 M, i64 N, i64 K, const u64 *A, const u64 *B, u64 *C) {
#pragma omp parallel for schedule(static)
  for (i64 i = 0; i < M; ++i) {
    u64 *c = C + i * N;
    for (i64 j = 0; j < N; ++j) c[j] = 0;
    for (i64 k = 0; k < K; ++k) {
      const u64 a = A[i * K + k];
      const u64 *b = B + k * N;
      for (i64 j = 0; j < N; ++j) c[j] += a * b[j];
    }
  }
}

/* The same definition evaluated only at the listed (row, col) positions. */
void orc_ring_gemm_at(i64 M, i64 N, i64 K, const u64 *A, const u64 *B, i64 npts,
                      const i64 *rows, const i64 *cols, u64 *out) {
  (void)M;
#pragma omp parallel for schedule(static)
  for (i64 t = 0; t < npts; ++t) {
    u64 acc = 0;
    for (i64 k = 0; k < K; ++k) acc += A[rows[t] * K + k] * B[k * N + cols[t]];
    out[t] = acc;
  }
}

/* 1-D convolution, valid padding:
 *   y[b][o][l] = sum_{c,j} w[o][c][j] * x[b][c][l*stride + j]
 * x is [Bt][Cin][L], w is [Cout][Cin][ksz], y is [Bt][Cout][Lout] with
 * Lout = (L - ksz)/stride + 1. */
i64 orc_conv1d_lout(i64 L, i64 ksz, i64 stride) { return L < ksz ? 0 : (L - ksz) / stride + 1; }

void orc_conv1d(i64 Bt, i64 Cin, i64 L, i64 Cout, i64 ksz, i64 stride, const u64 *x,
                const u64 *w, u64 *y) {
  const i64 Lout = orc_conv1d_lout(L, ksz, stride);
#pragma omp parallel for collapse(2) schedule(static)
  for (i64 b = 0; b < Bt; ++b)
    for (i64 o = 0; o < Cout; ++o)
      for (i64 l = 0; l < Lout; ++l) {
        u64 acc = 0;
        for (i64 c = 0; c < Cin; ++c)
          for (i64 j = 0; j < ksz; ++j)
            acc += w[(o * Cin + c) * ksz + j] * x[(b * Cin + c) * L + l * stride + j];
        y[(b * Cout + o) * Lout + l] = acc;
      }
}

/* The same definition at listed output positions (b, o, l). */
void orc_conv1d_at(i64 Bt, i64 Cin, i64 L, i64 Cout, i64 ksz, i64 stride, const u64 *x,
                   const u64 *w, i64 npts, const i64 *bs, const i64 *os, const i64 *ls,
                   u64 *out) {
  (void)Bt;
  (void)Cout;
#pragma omp parallel for schedule(static)
  for (i64 t = 0; t < npts; ++t) {
    u64 acc = 0;
    for (i64 c = 0; c < Cin; ++c)
      for (i64 j = 0; j < ksz; ++j)
        acc += w[(os[t] * Cin + c) * ksz + j] * x[(bs[t] * Cin + c) * L + ls[t] * stride + j];
    out[t] = acc;
  }
}

/* ------------------------------------------------------------------------ */
/* Trusted third party (section 4 and App. C.1.1, Multiplication): draws      */
/* a and b uniformly, sets c = f(a, b), and hands each party additive shares. */
/*   a_p = G(dseed, tag, A_p, i),  b_p = G(dseed, tag, B_p, i),               */
/*   c_0 = G(dseed, tag, C_0, i),  c_1 = c - c_0.                             */
/* For the square pair (App. C.1.1, Square) b = a^2, so b_1 = a^2 - b_0.     */
/* ------------------------------------------------------------------------ */
/* Element i of a product triple and of a square pair. */
static void dealer_mul_elem(u64 dseed, u64 tag, u64 i, u64 *a0, u64 *a1, u64 *b0, u64 *b1, u64 *c0,
                            u64 *c1) {
  *a0 = orc_prg(dseed, tag, SLOT_A0, i);
  *a1 = orc_prg(dseed, tag, SLOT_A1, i);
  *b0 = orc_prg(dseed, tag, SLOT_B0, i);
  *b1 = orc_prg(dseed, tag, SLOT_B1, i);
  u64 a = *a0 + *a1, b = *b0 + *b1;
  u64 c = a * b;
  *c0 = orc_prg(dseed, tag, SLOT_C0, i);
  *c1 = c - *c0;
}

static void dealer_square_elem(u64 dseed, u64 tag, u64 i, u64 *a0, u64 *a1, u64 *b0, u64 *b1) {
  *a0 = orc_prg(dseed, tag, SLOT_A0, i);
  *a1 = orc_prg(dseed, tag, SLOT_A1, i);
  u64 a = *a0 + *a1;
  *b0 = orc_prg(dseed, tag, SLOT_B0, i);
  *b1 = a * a - *b0;
}

void orc_dealer_mul(u64 dseed, u64 tag, size_t n, u64 *a0, u64 *a1, u64 *b0, u64 *b1,
                    u64 *c0, u64 *c1) {
  for (size_t i = 0; i < n; ++i)
    dealer_mul_elem(dseed, tag, (u64)i, &a0[i], &a1[i], &b0[i], &b1[i], &c0[i], &c1[i]);
}

void orc_dealer_square(u64 dseed, u64 tag, size_t n, u64 *a0, u64 *a1, u64 *b0, u64 *b1) {
  for (size_t i = 0; i < n; ++i) dealer_square_elem(dseed, tag, (u64)i, &a0[i], &a1[i], &b0[i], &b1[i]);
}

/* Selected elements idx[0..n) of a triple (pair) of any length. */
void orc_dealer_mul_at(u64 dseed, u64 tag, const u64 *idx, size_t n, u64 *a0, u64 *a1, u64 *b0,
                       u64 *b1, u64 *c0, u64 *c1) {
  for (size_t t = 0; t < n; ++t)
    dealer_mul_elem(dseed, tag, idx[t], &a0[t], &a1[t], &b0[t], &b1[t], &c0[t], &c1[t]);
}

void orc_dealer_square_at(u64 dseed, u64 tag, const u64 *idx, size_t n, u64 *a0, u64 *a1, u64 *b0,
                          u64 *b1) {
  for (size_t t = 0; t < n; ++t) dealer_square_elem(dseed, tag, idx[t], &a0[t], &a1[t], &b0[t], &b1[t]);
}

/* Matrix triple: a is MxK, b is KxN, c = a @ b is MxN. */
void orc_dealer_matmul(u64 dseed, u64 tag, i64 M, i64 N, i64 K, u64 *a0, u64 *a1, u64 *b0,
                       u64 *b1, u64 *c0, u64 *c1) {
  orc_prg_fill(dseed, tag, SLOT_A0, (size_t)(M * K), a0);
  orc_prg_fill(dseed, tag, SLOT_A1, (size_t)(M * K), a1);
  orc_prg_fill(dseed, tag, SLOT_B0, (size_t)(K * N), b0);
  orc_prg_fill(dseed, tag, SLOT_B1, (size_t)(K * N), b1);
  u64 *a = (u64 *)malloc(sizeof(u64) * (size_t)(M * K));
  u64 *b = (u64 *)malloc(sizeof(u64) * (size_t)(K * N));
  u64 *c = (u64 *)malloc(sizeof(u64) * (size_t)(M * N));
  orc_add(a0, a1, (size_t)(M * K), a);
  orc_add(b0, b1, (size_t)(K * N), b);
  orc_ring_gemm(M, N, K, a, b, c);
  orc_prg_fill(dseed, tag, SLOT_C0, (size_t)(M * N), c0);
  for (i64 i = 0; i < M * N; ++i) c1[i] = c[i] - c0[i];
  free(a);
  free(b);
  free(c);
}

/* Matrix triple evaluated at listed output positions only: fills c0, c1 at
 * (rows[t], cols[t]).  a_p and b_p are the full PRG fills (cheap). */
void orc_dealer_matmul_c_at(u64 dseed, u64 tag, i64 M, i64 N, i64 K, const u64 *a0,
                            const u64 *a1, const u64 *b0, const u64 *b1, i64 npts,
                            const i64 *rows, const i64 *cols, u64 *c0, u64 *c1) {
  (void)M;
#pragma omp parallel for schedule(static)
  for (i64 t = 0; t < npts; ++t) {
    u64 c = 0;
    for (i64 k = 0; k < K; ++k) {
      u64 a = a0[rows[t] * K + k] + a1[rows[t] * K + k];
      u64 b = b0[k * N + cols[t]] + b1[k * N + cols[t]];
      c += a * b;
    }
    c0[t] = orc_prg(dseed, tag, SLOT_C0, (u64)(rows[t] * N + cols[t]));
    c1[t] = c - c0[t];
  }
}

/* Rows rows[0..R) of a matrix triple with k = K and N columns, for matrices
 * of any height: a_p and c_p of those rows (R x K and R x N) and all of b_p. */
void orc_dealer_matmul_rows(u64 dseed, u64 tag, i64 N, i64 K, i64 R, const i64 *rows, u64 *a0,
                            u64 *a1, u64 *b0, u64 *b1, u64 *c0, u64 *c1) {
  for (i64 r = 0; r < R; ++r)
    for (i64 k = 0; k < K; ++k) {
      a0[r * K + k] = orc_prg(dseed, tag, SLOT_A0, (u64)(rows[r] * K + k));
      a1[r * K + k] = orc_prg(dseed, tag, SLOT_A1, (u64)(rows[r] * K + k));
    }
  orc_prg_fill(dseed, tag, SLOT_B0, (size_t)(K * N), b0);
  orc_prg_fill(dseed, tag, SLOT_B1, (size_t)(K * N), b1);
  u64 *a = (u64 *)malloc(sizeof(u64) * (size_t)(R * K));
  u64 *b = (u64 *)malloc(sizeof(u64) * (size_t)(K * N));
  u64 *c = (u64 *)malloc(sizeof(u64) * (size_t)(R * N));
  orc_add(a0, a1, (size_t)(R * K), a);
  orc_add(b0, b1, (size_t)(K * N), b);
  orc_ring_gemm(R, N, K, a, b, c);
  for (i64 r = 0; r < R; ++r)
    for (i64 j = 0; j < N; ++j) {
      c0[r * N + j] = orc_prg(dseed, tag, SLOT_C0, (u64)(rows[r] * N + j));
      c1[r * N + j] = c[r * N + j] - c0[r * N + j];
    }
  free(a);
  free(b);
  free(c);
}

/* Convolution triple: a has activation shape [Bt][Cin][L], b has weight
 * shape [Cout][Cin][ksz], c = conv1d(a, b) has shape [Bt][Cout][Lout]. */
void orc_dealer_conv1d(u64 dseed, u64 tag, i64 Bt, i64 Cin, i64 L, i64 Cout, i64 ksz,
                       i64 stride, u64 *a0, u64 *a1, u64 *b0, u64 *b1, u64 *c0, u64 *c1) {
  const i64 nx = Bt * Cin * L, nw = Cout * Cin * ksz;
  const i64 ny = Bt * Cout * orc_conv1d_lout(L, ksz, stride);
  orc_prg_fill(dseed, tag, SLOT_A0, (size_t)nx, a0);
  orc_prg_fill(dseed, tag, SLOT_A1, (size_t)nx, a1);
  orc_prg_fill(dseed, tag, SLOT_B0, (size_t)nw, b0);
  orc_prg_fill(dseed, tag, SLOT_B1, (size_t)nw, b1);
  u64 *a = (u64 *)malloc(sizeof(u64) * (size_t)nx);
  u64 *b = (u64 *)malloc(sizeof(u64) * (size_t)nw);
  u64 *c = (u64 *)malloc(sizeof(u64) * (size_t)(ny > 0 ? ny : 1));
  orc_add(a0, a1, (size_t)nx, a);
  orc_add(b0, b1, (size_t)nw, b);
  orc_conv1d(Bt, Cin, L, Cout, ksz, stride, a, b, c);
  orc_prg_fill(dseed, tag, SLOT_C0, (size_t)ny, c0);
  for (i64 i = 0; i < ny; ++i) c1[i] = c[i] - c0[i];
  free(a);
  free(b);
  free(c);
}

/* ------------------------------------------------------------------------ */
/* Beaver multiplication (section 5.2 and App. C.1.1, Multiplication):        */
/*   [eps] = [x] - [a],  [delta] = [y] - [b]    (each party, locally)          */
/*   eps, delta revealed                         (one round)                   */
/*   [z]_p = [c]_p + eps [b]_p + [a]_p delta  (+ eps delta for party 0 only)  */
/* then each party truncates its share by 2^trunc_bits (0 = no truncation).   */
/* ------------------------------------------------------------------------ */
void orc_beaver_mul(size_t n, const u64 *x0, const u64 *x1, const u64 *y0, const u64 *y1,
                    const u64 *a0, const u64 *a1, const u64 *b0, const u64 *b1, const u64 *c0,
                    const u64 *c1, int trunc_bits, u64 *z0, u64 *z1) {
  for (size_t i = 0; i < n; ++i) {
    u64 e0 = x0[i] - a0[i], e1 = x1[i] - a1[i]; /* [eps]_p   */
    u64 d0 = y0[i] - b0[i], d1 = y1[i] - b1[i]; /* [delta]_p */
    u64 eps = e0 + e1, delta = d0 + d1;         /* open      */
    z0[i] = c0[i] + eps * b0[i] + a0[i] * delta + eps * delta;
    z1[i] = c1[i] + eps * b1[i] + a1[i] * delta;
  }
  orc_truncate(z0, n, trunc_bits);
  orc_truncate(z1, n, trunc_bits);
}

/* Square with a Beaver pair (a, b = a^2) (App. C.1.1, Square):
 *   [eps] = [x] - [a];  eps revealed;  [x^2] = [b] + 2 eps [a] + eps^2
 * with the public eps^2 added by party 0 only. */
void orc_beaver_square(size_t n, const u64 *x0, const u64 *x1, const u64 *a0, const u64 *a1,
                       const u64 *b0, const u64 *b1, int trunc_bits, u64 *z0, u64 *z1) {
  for (size_t i = 0; i < n; ++i) {
    u64 eps = (x0[i] - a0[i]) + (x1[i] - a1[i]);
    z0[i] = b0[i] + 2 * eps * a0[i] + eps * eps;
    z1[i] = b1[i] + 2 * eps * a1[i];
  }
  orc_truncate(z0, n, trunc_bits);
  orc_truncate(z1, n, trunc_bits);
}

/* Beaver matrix product (App. C.1.1: the same identity for any bilinear f).
 * Keeps the factor order of the matrix product:
 *   [z]_p = [c]_p + eps @ [b]_p + [a]_p @ delta (+ eps @ delta for party 0).
 * x_p: MxK, y_p: KxN, a_p: MxK, b_p: KxN, c_p and z_p: MxN. */
void orc_beaver_matmul(i64 M, i64 N, i64 K, const u64 *x0, const u64 *x1, const u64 *y0,
                       const u64 *y1, const u64 *a0, const u64 *a1, const u64 *b0,
                       const u64 *b1, const u64 *c0, const u64 *c1, int trunc_bits, u64 *z0,
                       u64 *z1) {
  const size_t nA = (size_t)(M * K), nB = (size_t)(K * N), nC = (size_t)(M * N);
  u64 *eps = (u64 *)malloc(sizeof(u64) * (nA ? nA : 1));
  u64 *delta = (u64 *)malloc(sizeof(u64) * (nB ? nB : 1));
  u64 *t = (u64 *)malloc(sizeof(u64) * (nC ? nC : 1));
  for (size_t i = 0; i < nA; ++i) eps[i] = (x0[i] - a0[i]) + (x1[i] - a1[i]);
  for (size_t i = 0; i < nB; ++i) delta[i] = (y0[i] - b0[i]) + (y1[i] - b1[i]);
  /* party 0 */
  for (size_t i = 0; i < nC; ++i) z0[i] = c0[i];
  orc_ring_gemm(M, N, K, eps, b0, t);
  for (size_t i = 0; i < nC; ++i) z0[i] += t[i];
  orc_ring_gemm(M, N, K, a0, delta, t);
  for (size_t i = 0; i < nC; ++i) z0[i] += t[i];
  orc_ring_gemm(M, N, K, eps, delta, t);
  for (size_t i = 0; i < nC; ++i) z0[i] += t[i];
  /* party 1 */
  for (size_t i = 0; i < nC; ++i) z1[i] = c1[i];
  orc_ring_gemm(M, N, K, eps, b1, t);
  for (size_t i = 0; i < nC; ++i) z1[i] += t[i];
  orc_ring_gemm(M, N, K, a1, delta, t);
  for (size_t i = 0; i < nC; ++i) z1[i] += t[i];
  orc_truncate(z0, nC, trunc_bits);
  orc_truncate(z1, nC, trunc_bits);
  free(eps);
  free(delta);
  free(t);
}

/* The same protocol evaluated at listed output positions.  c0/c1 are the
 * triple's c shares AT THOSE POSITIONS (length npts). */
void orc_beaver_matmul_at(i64 M, i64 N, i64 K, const u64 *x0, const u64 *x1, const u64 *y0,
                          const u64 *y1, const u64 *a0, const u64 *a1, const u64 *b0,
                          const u64 *b1, const u64 *c0_at, const u64 *c1_at, int trunc_bits,
                          i64 npts, const i64 *rows, const i64 *cols, u64 *z0, u64 *z1) {
  (void)M;
#pragma omp parallel for schedule(static)
  for (i64 t = 0; t < npts; ++t) {
    const i64 i = rows[t], j = cols[t];
    u64 s_eb0 = 0, s_eb1 = 0, s_ad0 = 0, s_ad1 = 0, s_ed = 0;
    for (i64 k = 0; k < K; ++k) {
      u64 eps = (x0[i * K + k] - a0[i * K + k]) + (x1[i * K + k] - a1[i * K + k]);
      u64 delta = (y0[k * N + j] - b0[k * N + j]) + (y1[k * N + j] - b1[k * N + j]);
      s_eb0 += eps * b0[k * N + j];
      s_eb1 += eps * b1[k * N + j];
      s_ad0 += a0[i * K + k] * delta;
      s_ad1 += a1[i * K + k] * delta;
      s_ed += eps * delta;
    }
    z0[t] = c0_at[t] + s_eb0 + s_ad0 + s_ed;
    z1[t] = c1_at[t] + s_eb1 + s_ad1;
  }
  orc_truncate(z0, (size_t)npts, trunc_bits);
  orc_truncate(z1, (size_t)npts, trunc_bits);
}

/* Beaver convolution: the bilinear f is conv1d(activation, weight).
 * x_p, a_p: [Bt][Cin][L];  y_p, b_p: [Cout][Cin][ksz];  c_p, z_p: [Bt][Cout][Lout].
 *   [z]_p = [c]_p + conv(eps, [b]_p) + conv([a]_p, delta) (+ conv(eps, delta), p = 0) */
void orc_beaver_conv1d(i64 Bt, i64 Cin, i64 L, i64 Cout, i64 ksz, i64 stride, const u64 *x0,
                       const u64 *x1, const u64 *y0, const u64 *y1, const u64 *a0,
                       const u64 *a1, const u64 *b0, const u64 *b1, const u64 *c0,
                       const u64 *c1, int trunc_bits, u64 *z0, u64 *z1) {
  const i64 Lout = orc_conv1d_lout(L, ksz, stride);
  const size_t nx = (size_t)(Bt * Cin * L), nw = (size_t)(Cout * Cin * ksz);
  const size_t ny = (size_t)(Bt * Cout * Lout);
  u64 *eps = (u64 *)malloc(sizeof(u64) * (nx ? nx : 1));
  u64 *delta = (u64 *)malloc(sizeof(u64) * (nw ? nw : 1));
  u64 *t = (u64 *)malloc(sizeof(u64) * (ny ? ny : 1));
  for (size_t i = 0; i < nx; ++i) eps[i] = (x0[i] - a0[i]) + (x1[i] - a1[i]);
  for (size_t i = 0; i < nw; ++i) delta[i] = (y0[i] - b0[i]) + (y1[i] - b1[i]);
  for (size_t i = 0; i < ny; ++i) z0[i] = c0[i];
  orc_conv1d(Bt, Cin, L, Cout, ksz, stride, eps, b0, t);
  for (size_t i = 0; i < ny; ++i) z0[i] += t[i];
  orc_conv1d(Bt, Cin, L, Cout, ksz, stride, a0, delta, t);
  for (size_t i = 0; i < ny; ++i) z0[i] += t[i];
  orc_conv1d(Bt, Cin, L, Cout, ksz, stride, eps, delta, t);
  for (size_t i = 0; i < ny; ++i) z0[i] += t[i];
  for (size_t i = 0; i < ny; ++i) z1[i] = c1[i];
  orc_conv1d(Bt, Cin, L, Cout, ksz, stride, eps, b1, t);
  for (size_t i = 0; i < ny; ++i) z1[i] += t[i];
  orc_conv1d(Bt, Cin, L, Cout, ksz, stride, a1, delta, t);
  for (size_t i = 0; i < ny; ++i) z1[i] += t[i];
  orc_truncate(z0, ny, trunc_bits);
  orc_truncate(z1, ny, trunc_bits);
  free(eps);
  free(delta);
  free(t);
}

/* Convolution triple's c shares at listed output positions (b, o, l):
 * c = conv1d(a_0 + a_1, b_0 + b_1) there, c_0 from the PRG at the flat output
 * index, c_1 = c - c_0. */
void orc_dealer_conv1d_c_at(u64 dseed, u64 tag, i64 Bt, i64 Cin, i64 L, i64 Cout, i64 ksz,
                            i64 stride, const u64 *a0, const u64 *a1, const u64 *b0,
                            const u64 *b1, i64 npts, const i64 *bs, const i64 *os,
                            const i64 *ls, u64 *c0, u64 *c1) {
  (void)Bt;
  const i64 Lout = orc_conv1d_lout(L, ksz, stride);
#pragma omp parallel for schedule(static)
  for (i64 t = 0; t < npts; ++t) {
    u64 c = 0;
    for (i64 ci = 0; ci < Cin; ++ci)
      for (i64 j = 0; j < ksz; ++j) {
        const i64 xi = (bs[t] * Cin + ci) * L + ls[t] * stride + j;
        const i64 wi = (os[t] * Cin + ci) * ksz + j;
        c += (a0[xi] + a1[xi]) * (b0[wi] + b1[wi]);
      }
    c0[t] = orc_prg(dseed, tag, SLOT_C0, (u64)((bs[t] * Cout + os[t]) * Lout + ls[t]));
    c1[t] = c - c0[t];
  }
}

/* Beaver convolution at listed output positions; c0_at/c1_at are the
 * triple's c shares at those positions. */
void orc_beaver_conv1d_at(i64 Bt, i64 Cin, i64 L, i64 Cout, i64 ksz, i64 stride, const u64 *x0,
                          const u64 *x1, const u64 *y0, const u64 *y1, const u64 *a0,
                          const u64 *a1, const u64 *b0, const u64 *b1, const u64 *c0_at,
                          const u64 *c1_at, int trunc_bits, i64 npts, const i64 *bs,
                          const i64 *os, const i64 *ls, u64 *z0, u64 *z1) {
  (void)Bt;
  (void)Cout;
#pragma omp parallel for schedule(static)
  for (i64 t = 0; t < npts; ++t) {
    u64 s_eb0 = 0, s_eb1 = 0, s_ad0 = 0, s_ad1 = 0, s_ed = 0;
    for (i64 ci = 0; ci < Cin; ++ci)
      for (i64 j = 0; j < ksz; ++j) {
        const i64 xi = (bs[t] * Cin + ci) * L + ls[t] * stride + j;
        const i64 wi = (os[t] * Cin + ci) * ksz + j;
        const u64 eps = (x0[xi] - a0[xi]) + (x1[xi] - a1[xi]);
        const u64 delta = (y0[wi] - b0[wi]) + (y1[wi] - b1[wi]);
        s_eb0 += eps * b0[wi];
        s_eb1 += eps * b1[wi];
        s_ad0 += a0[xi] * delta;
        s_ad1 += a1[xi] * delta;
        s_ed += eps * delta;
      }
    z0[t] = c0_at[t] + s_eb0 + s_ad0 + s_ed;
    z1[t] = c1_at[t] + s_eb1 + s_ad1;
  }
  orc_truncate(z0, (size_t)npts, trunc_bits);
  orc_truncate(z1, (size_t)npts, trunc_bits);
}

/* ------------------------------------------------------------------------ */
/* Signed 8-bit limb decomposition (a test helper for the limb GEMM form;     */
/* not a step of the protocol).  For v in Z/2^64:                            */
/*   u = v + 0x8080808080808080 (mod 2^64),  d_i = byte_i(u) - 128,          */
/* so d_i is in [-128, 127] and sum_i d_i 2^(8i) = v (mod 2^64).              */
/* ------------------------------------------------------------------------ */
void orc_limbs(const u64 *v, size_t n, int8_t *d /* n x 8 */) {
  for (size_t t = 0; t < n; ++t) {
    u64 u = v[t] + 0x8080808080808080ULL;
    for (int i = 0; i < 8; ++i) d[t * 8 + i] = (int8_t)((int)((u >> (8 * i)) & 0xff) - 128);
  }
}

/* Ring GEMM through limbs: C = sum_{i+j<=7} 2^(8(i+j)) (D_i @ E_j) mod 2^64,
 * where each D_i @ E_j is an exact integer matrix product accumulated in
 * int32 over chunks of at most kchunk terms (each chunk's partial sum is then
 * sign-extended to 64 bits).  Returns -1 if some chunk sum would leave int32. */
int orc_limb_gemm(i64 M, i64 N, i64 K, const u64 *A, const u64 *B, i64 kchunk, u64 *C) {
  int8_t *dA = (int8_t *)malloc((size_t)(M * K * 8 > 0 ? M * K * 8 : 1));
  int8_t *dB = (int8_t *)malloc((size_t)(K * N * 8 > 0 ? K * N * 8 : 1));
  orc_limbs(A, (size_t)(M * K), dA);
  orc_limbs(B, (size_t)(K * N), dB);
  int bad = 0;
  for (i64 r = 0; r < M; ++r)
    for (i64 c = 0; c < N; ++c) {
      u64 acc = 0;
      for (int i = 0; i < 8; ++i)
        for (int j = 0; i + j < 8; ++j)
          for (i64 k0 = 0; k0 < K; k0 += kchunk) {
            i64 part = 0; /* exact */
            for (i64 k = k0; k < K && k < k0 + kchunk; ++k)
              part += (i64)dA[(r * K + k) * 8 + i] * (i64)dB[(k * N + c) * 8 + j];
            if (part > INT32_MAX || part < INT32_MIN) bad = 1;
            acc += (u64)(i64)(int32_t)part << (8 * (i + j));
          }
      C[r * N + c] = acc;
    }
  free(dA);
  free(dB);
  return bad ? -1 : 0;
}

/* ======================================================================== */
/* More than two parties (App. C.1.1, arithmetic secret sharing for any      */
/* number of parties |P|; Algorithm 1 for the truncation).  A sharing among  */
/* P parties is an array of P share buffers.  PRG domains of these functions */
/* are separate slots: 0x100+p share, 0x200+p a, 0x300+p b, 0x400+p c,       */
/* 0x500+p r, 0x600+p theta_r, for party p.                                  */
/* ======================================================================== */
enum { MP_SHARE = 0x100, MP_A = 0x200, MP_B = 0x300, MP_C = 0x400, MP_R = 0x500, MP_T = 0x600 };

/* signed view and exact integer helpers */
static inline i64 s64(u64 v) { return (i64)v; }

/* Sharing (section 5.1): a pseudorandom zero-share of P numbers summing to 0,
 * z_p = m_p - m_{(p+1) mod P} with m_p = G(seed, tag, 0x100+p, i); the source
 * party adds its value. */
void orc_mp_share(const u64 *x, size_t n, int P, int src, u64 seed, u64 tag, u64 *const *s) {
  for (size_t i = 0; i < n; ++i)
    for (int p = 0; p < P; ++p) {
      const u64 mp = orc_prg(seed, tag, MP_SHARE + (u64)p, (u64)i);
      const u64 mq = orc_prg(seed, tag, MP_SHARE + (u64)((p + 1) % P), (u64)i);
      s[p][i] = (mp - mq) + (p == src ? x[i] : 0);
    }
}

/* x = sum_p [x]_p mod Q */
void orc_mp_reveal(int P, const u64 *const *s, size_t n, u64 *out) {
  for (size_t i = 0; i < n; ++i) {
    u64 acc = 0;
    for (int p = 0; p < P; ++p) acc += s[p][i];
    out[i] = acc;
  }
}

/* The last party's share of a value v whose other P-1 shares are drawn from
 * the PRG: v - sum_{p<P-1} G(slot+p). */
static void mp_split(u64 dseed, u64 tag, u64 slot, int P, size_t n, const u64 *v, u64 *const *out) {
  for (size_t i = 0; i < n; ++i) {
    u64 rest = v[i];
    for (int p = 0; p < P - 1; ++p) {
      out[p][i] = orc_prg(dseed, tag, slot + (u64)p, (u64)i);
      rest -= out[p][i];
    }
    out[P - 1][i] = rest;
  }
}

/* Dealer (the TTP), element-wise: a_p, b_p uniform from the PRG; c = a*b
 * shared as c_p = G(0x400+p) for p < P-1 and the rest for the last party.
 * square != 0: the Beaver pair (a, b = a^2), b shared the same way, c unused. */
void orc_mp_dealer_mul(u64 dseed, u64 tag, int P, size_t n, int square, u64 *const *a, u64 *const *b,
                       u64 *const *c) {
  u64 *prod = (u64 *)malloc((n ? n : 1) * sizeof(u64));
  for (int p = 0; p < P; ++p) orc_prg_fill(dseed, tag, MP_A + (u64)p, n, a[p]);
  if (!square)
    for (int p = 0; p < P; ++p) orc_prg_fill(dseed, tag, MP_B + (u64)p, n, b[p]);
  for (size_t i = 0; i < n; ++i) {
    u64 av = 0, bv = 0;
    for (int p = 0; p < P; ++p) av += a[p][i];
    if (!square)
      for (int p = 0; p < P; ++p) bv += b[p][i];
    prod[i] = square ? av * av : av * bv;
  }
  if (square) mp_split(dseed, tag, MP_B, P, n, prod, b);
  else mp_split(dseed, tag, MP_C, P, n, prod, c);
  free(prod);
}

/* Dealer, matrix triple: a_p (MxK), b_p (KxN) uniform; c = a @ b (MxN). */
void orc_mp_dealer_matmul(u64 dseed, u64 tag, int P, i64 M, i64 N, i64 K, u64 *const *a, u64 *const *b,
                          u64 *const *c) {
  const size_t na = (size_t)(M * K), nb = (size_t)(K * N), nc = (size_t)(M * N);
  u64 *as = (u64 *)calloc(na ? na : 1, sizeof(u64));
  u64 *bs = (u64 *)calloc(nb ? nb : 1, sizeof(u64));
  u64 *cs = (u64 *)malloc((nc ? nc : 1) * sizeof(u64));
  for (int p = 0; p < P; ++p) {
    orc_prg_fill(dseed, tag, MP_A + (u64)p, na, a[p]);
    orc_prg_fill(dseed, tag, MP_B + (u64)p, nb, b[p]);
    for (size_t i = 0; i < na; ++i) as[i] += a[p][i];
    for (size_t i = 0; i < nb; ++i) bs[i] += b[p][i];
  }
  orc_ring_gemm(M, N, K, as, bs, cs);
  mp_split(dseed, tag, MP_C, P, nc, cs, c);
  free(as);
  free(bs);
  free(cs);
}

/* Beaver product among P parties (App. C.1.1, Multiplication and Square):
 * eps = sum_p ([x]_p - [a]_p), delta = sum_p ([y]_p - [b]_p) are opened, and
 * [z]_p = [c]_p + eps [b]_p + [a]_p delta (+ eps delta for party 0).
 * y == NULL: the square with the pair (a, b = a^2):
 * [z]_p = [b]_p + 2 eps [a]_p (+ eps^2 for party 0). */
void orc_mp_beaver_mul(int P, size_t n, const u64 *const *x, const u64 *const *y, const u64 *const *a,
                       const u64 *const *b, const u64 *const *c, u64 *const *z) {
  for (size_t i = 0; i < n; ++i) {
    u64 eps = 0, delta = 0;
    for (int p = 0; p < P; ++p) eps += x[p][i] - a[p][i];
    if (y)
      for (int p = 0; p < P; ++p) delta += y[p][i] - b[p][i];
    for (int p = 0; p < P; ++p) {
      if (y) z[p][i] = c[p][i] + eps * b[p][i] + a[p][i] * delta + (p == 0 ? eps * delta : 0);
      else z[p][i] = b[p][i] + 2 * eps * a[p][i] + (p == 0 ? eps * eps : 0);
    }
  }
}

/* Beaver matmul among P parties, the three products kept separate and in
 * order: [z]_p = [c]_p + eps @ [b]_p + [a]_p @ delta (+ eps @ delta, party 0). */
void orc_mp_beaver_matmul(int P, i64 M, i64 N, i64 K, const u64 *const *x, const u64 *const *y,
                          const u64 *const *a, const u64 *const *b, const u64 *const *c, u64 *const *z) {
  const size_t na = (size_t)(M * K), nb = (size_t)(K * N), nc = (size_t)(M * N);
  u64 *eps = (u64 *)calloc(na ? na : 1, sizeof(u64));
  u64 *del = (u64 *)calloc(nb ? nb : 1, sizeof(u64));
  u64 *t1 = (u64 *)malloc((nc ? nc : 1) * sizeof(u64));
  u64 *t2 = (u64 *)malloc((nc ? nc : 1) * sizeof(u64));
  u64 *t3 = (u64 *)malloc((nc ? nc : 1) * sizeof(u64));
  for (int p = 0; p < P; ++p) {
    for (size_t i = 0; i < na; ++i) eps[i] += x[p][i] - a[p][i];
    for (size_t i = 0; i < nb; ++i) del[i] += y[p][i] - b[p][i];
  }
  orc_ring_gemm(M, N, K, eps, del, t3);
  for (int p = 0; p < P; ++p) {
    orc_ring_gemm(M, N, K, eps, b[p], t1);
    orc_ring_gemm(M, N, K, a[p], del, t2);
    for (size_t i = 0; i < nc; ++i) z[p][i] = c[p][i] + t1[i] + t2[i] + (p == 0 ? t3[i] : 0);
  }
  free(eps);
  free(del);
  free(t1);
  free(t2);
  free(t3);
}

/* The wrap count theta_v of shares v_0..v_{P-1} (App. C.1.1, Truncation): the
 * integer with sum_p s64(v_p) = s64(v) + theta_v Q, v = sum_p v_p mod Q. */
static i64 mp_wraps(int P, const u64 *const *v, size_t i) {
  __int128 sum = 0;
  u64 ring = 0;
  for (int p = 0; p < P; ++p) {
    sum += (__int128)s64(v[p][i]);
    ring += v[p][i];
  }
  return (i64)((sum - (__int128)s64(ring)) / ((__int128)1 << 64));
}

/* Dealer of the truncation randomness (Algorithm 1's inputs): r_p uniform
 * from the PRG, and a sharing of the wrap count theta_r of r's shares
 * (t_p = G(0x600+p) for p < P-1, the last share the rest). */
void orc_mp_dealer_trunc(u64 dseed, u64 tag, int P, size_t n, u64 *const *r, u64 *const *t) {
  u64 *th = (u64 *)malloc((n ? n : 1) * sizeof(u64));
  for (int p = 0; p < P; ++p) orc_prg_fill(dseed, tag, MP_R + (u64)p, n, r[p]);
  for (size_t i = 0; i < n; ++i) th[i] = (u64)mp_wraps(P, (const u64 *const *)r, i);
  mp_split(dseed, tag, MP_T, P, n, th, t);
  free(th);
}

/* Truncation by 2^bits among P parties (App. C.1.1, Truncation, Algorithm 1
 * with eta set to 0 as the paper does), in place:
 *   [z] = [x] + [r];  beta_p = (s64(x_p) + s64(r_p) - s64(z_p)) / Q;
 *   z = reveal([z]), theta_z = the wrap count of z's shares;
 *   [theta_x] = theta_z (added by party 0) + [beta] - [theta_r];
 *   [x / 2^bits]_p = floor(s64(x_p) / 2^bits) - [theta_x]_p * 2^(64 - bits). */
void orc_mp_truncate(int P, size_t n, int bits, u64 *const *x, const u64 *const *r, const u64 *const *t) {
  if (bits <= 0 || P < 1 || P > 64) return; /* nothing to divide by / out of this oracle's range */
  u64 *zs[64];
  for (int p = 0; p < P; ++p) zs[p] = (u64 *)malloc((n ? n : 1) * sizeof(u64));
  for (size_t i = 0; i < n; ++i)
    for (int p = 0; p < P; ++p) zs[p][i] = x[p][i] + r[p][i];
  for (size_t i = 0; i < n; ++i) {
    const i64 theta_z = mp_wraps(P, (const u64 *const *)zs, i);
    for (int p = 0; p < P; ++p) {
      const __int128 beta = ((__int128)s64(x[p][i]) + s64(r[p][i]) - s64(zs[p][i])) / ((__int128)1 << 64);
      const u64 theta_x = (p == 0 ? (u64)theta_z : 0) + (u64)(i64)beta - t[p][i];
      x[p][i] = (u64)floor_div_pow2(s64(x[p][i]), bits) - theta_x * ((u64)1 << (64 - bits));
    }
  }
  for (int p = 0; p < P; ++p) free(zs[p]);
}

/* ======================================================================== */
/* Binary sharing (App. C.1.1, Binary Secret Sharing; Converting Between     */
/* Secret-Sharing Types; Logic-based Operations), two parties.  A binary     */
/* sharing holds 64 independent bits per word: x = <x>_0 XOR <x>_1.          */
/* PRG slots: 0x700 share, 0x701-0x705 AND triple (a0, a1, b0, b1, c0),      */
/* 0x706/0x707 the parties' re-sharing in A2B, 0x708-0x70a the B2A bit.      */
/* ======================================================================== */
enum {
  BIN_SHARE = 0x700, BIN_A0 = 0x701, BIN_A1 = 0x702, BIN_B0 = 0x703, BIN_B1 = 0x704, BIN_C0 = 0x705,
  A2B_Y0 = 0x706, A2B_Y1 = 0x707, B2A_R = 0x708, B2A_RB0 = 0x709, B2A_RA0 = 0x70a
};
#define A2B_TRIPLES 12

/* Sharing: XOR zero-share (m, m); the source party XORs its value in. */
void orc_bin_share(const u64 *x, size_t n, int src, u64 seed, u64 tag, u64 *s0, u64 *s1) {
  for (size_t i = 0; i < n; ++i) {
    const u64 m = orc_prg(seed, tag, BIN_SHARE, (u64)i);
    s0[i] = src == 0 ? x[i] ^ m : m;
    s1[i] = src == 1 ? x[i] ^ m : m;
  }
}

void orc_bin_reveal(const u64 *s0, const u64 *s1, size_t n, u64 *out) {
  for (size_t i = 0; i < n; ++i) out[i] = s0[i] ^ s1[i];
}

/* Dealer of bitwise AND triples: a_p, b_p random words, c = a AND b shared as
 * c0 = G, c1 = c XOR c0. */
void orc_dealer_and(u64 dseed, u64 tag, size_t n, u64 *a0, u64 *a1, u64 *b0, u64 *b1, u64 *c0, u64 *c1) {
  for (size_t i = 0; i < n; ++i) {
    a0[i] = orc_prg(dseed, tag, BIN_A0, (u64)i);
    a1[i] = orc_prg(dseed, tag, BIN_A1, (u64)i);
    b0[i] = orc_prg(dseed, tag, BIN_B0, (u64)i);
    b1[i] = orc_prg(dseed, tag, BIN_B1, (u64)i);
    c0[i] = orc_prg(dseed, tag, BIN_C0, (u64)i);
    c1[i] = ((a0[i] ^ a1[i]) & (b0[i] ^ b1[i])) ^ c0[i];
  }
}

/* Bitwise AND (App. C.1.1, Bitwise AND): eps = x XOR a, delta = y XOR b are
 * opened; <z>_p = <c>_p ^ (eps & <b>_p) ^ (<a>_p & delta) (^ eps & delta for
 * party 0). */
void orc_bin_and(size_t n, const u64 *x0, const u64 *x1, const u64 *y0, const u64 *y1, const u64 *a0,
                 const u64 *a1, const u64 *b0, const u64 *b1, const u64 *c0, const u64 *c1, u64 *z0,
                 u64 *z1) {
  for (size_t i = 0; i < n; ++i) {
    const u64 eps = (x0[i] ^ a0[i]) ^ (x1[i] ^ a1[i]);
    const u64 del = (y0[i] ^ b0[i]) ^ (y1[i] ^ b1[i]);
    z0[i] = c0[i] ^ (eps & b0[i]) ^ (a0[i] & del) ^ (eps & del);
    z1[i] = c1[i] ^ (eps & b1[i]) ^ (a1[i] & del);
  }
}

/* One AND of two binary sharings held in local arrays, with triple t of a
 * [A2B_TRIPLES][n] triple buffer. */
static void a2b_and(size_t n, size_t t, const u64 *x0, const u64 *x1, const u64 *y0, const u64 *y1,
                    const u64 *const *tr, u64 *z0, u64 *z1) {
  const size_t o = t * n;
  orc_bin_and(n, x0, x1, y0, y1, tr[0] + o, tr[1] + o, tr[2] + o, tr[3] + o, tr[4] + o, tr[5] + o, z0, z1);
}

/* Arithmetic to binary (App. C.1.1, From [x] to <x>): each party binary-shares
 * its arithmetic share (party p is the source of <y_p>), and the parties add
 * <y_0> + <y_1> with a carry-lookahead (Kogge-Stone) adder over binary shares:
 *   G = y0 AND y1, P = y0 XOR y1 (the per-bit generate and propagate);
 *   for k = 1, 2, 4, ..., 32:  G <- G XOR (P AND (G << k)),  P <- P AND (P << k)
 *   (the two terms of the group-generate OR never both hold, so XOR is OR;
 *   the last level's P is not needed), then x = (y0 XOR y1) XOR (G << 1).
 * tr: six pointers (a0, a1, b0, b1, c0, c1), each [A2B_TRIPLES][n] words. */
void orc_a2b(size_t n, const u64 *x0, const u64 *x1, u64 seed, u64 tag, const u64 *const *tr, u64 *z0, u64 *z1) {
  const size_t cnt = n ? n : 1;
  u64 *y00 = calloc(cnt, sizeof(u64)), *y01 = calloc(cnt, sizeof(u64)), *y10 = calloc(cnt, sizeof(u64)), *y11 = calloc(cnt, sizeof(u64));
  u64 *g0 = calloc(cnt, sizeof(u64)), *g1 = calloc(cnt, sizeof(u64)), *p0 = calloc(cnt, sizeof(u64)), *p1 = calloc(cnt, sizeof(u64));
  u64 *s0 = calloc(cnt, sizeof(u64)), *s1 = calloc(cnt, sizeof(u64)), *t0 = calloc(cnt, sizeof(u64)), *t1 = calloc(cnt, sizeof(u64));
  u64 *q0 = calloc(cnt, sizeof(u64)), *q1 = calloc(cnt, sizeof(u64));
  /* <y_0> = (x0 ^ m0, m0), <y_1> = (m1, x1 ^ m1) */
  for (size_t i = 0; i < n; ++i) {
    const u64 m0 = orc_prg(seed, tag, A2B_Y0, (u64)i), m1 = orc_prg(seed, tag, A2B_Y1, (u64)i);
    y00[i] = x0[i] ^ m0;
    y01[i] = m0;
    y10[i] = m1;
    y11[i] = x1[i] ^ m1;
  }
  size_t t = 0;
  a2b_and(n, t++, y00, y01, y10, y11, tr, g0, g1);
  for (size_t i = 0; i < n; ++i) {
    p0[i] = y00[i] ^ y10[i];
    p1[i] = y01[i] ^ y11[i];
  }
  for (int k = 1; k < 64; k <<= 1) {
    for (size_t i = 0; i < n; ++i) {
      s0[i] = g0[i] << k;
      s1[i] = g1[i] << k;
    }
    a2b_and(n, t++, p0, p1, s0, s1, tr, t0, t1); /* P AND (G << k) */
    if (k < 32) {
      for (size_t i = 0; i < n; ++i) {
        s0[i] = p0[i] << k;
        s1[i] = p1[i] << k;
      }
      a2b_and(n, t++, p0, p1, s0, s1, tr, q0, q1); /* P AND (P << k) */
    }
    for (size_t i = 0; i < n; ++i) {
      g0[i] ^= t0[i];
      g1[i] ^= t1[i];
      if (k < 32) {
        p0[i] = q0[i];
        p1[i] = q1[i];
      }
    }
  }
  for (size_t i = 0; i < n; ++i) {
    z0[i] = (y00[i] ^ y10[i]) ^ (g0[i] << 1);
    z1[i] = (y01[i] ^ y11[i]) ^ (g1[i] << 1);
  }
  free(y00); free(y01); free(y10); free(y11); free(g0); free(g1); free(p0); free(p1);
  free(s0); free(s1); free(t0); free(t1); free(q0); free(q1);
}

/* Dealer of Algorithm 2's random bit: r in {0, 1} shared both ways,
 * <r> = (w, w XOR r) and [r] = (v, r - v). */
void orc_dealer_b2a(u64 dseed, u64 tag, size_t n, u64 *rb0, u64 *rb1, u64 *ra0, u64 *ra1) {
  for (size_t i = 0; i < n; ++i) {
    const u64 r = orc_prg(dseed, tag, B2A_R, (u64)i) & 1;
    rb0[i] = orc_prg(dseed, tag, B2A_RB0, (u64)i);
    rb1[i] = rb0[i] ^ r;
    ra0[i] = orc_prg(dseed, tag, B2A_RA0, (u64)i);
    ra1[i] = r - ra0[i];
  }
}

/* Binary to arithmetic for bit `bit` of <b> (Algorithm 2): <z> = <b> XOR <r>
 * on that bit, z = reveal(<z>), [b] = [r] + z - 2 [r] z (z added by party 0). */
void orc_b2a_bit(size_t n, int bit, const u64 *b0, const u64 *b1, const u64 *rb0, const u64 *rb1,
                 const u64 *ra0, const u64 *ra1, u64 *z0, u64 *z1) {
  for (size_t i = 0; i < n; ++i) {
    const u64 zb = ((((b0[i] >> bit) ^ rb0[i]) ^ ((b1[i] >> bit) ^ rb1[i])) & 1);
    z0[i] = ra0[i] + zb - 2 * ra0[i] * zb;
    z1[i] = ra1[i] - 2 * ra1[i] * zb;
  }
}

/* ReLU (App. C.1.1, Sign, absolute value, and ReLU): [x < 0] is the sign bit
 * of <x> = A2B([x]) converted by Algorithm 2; ReLU([x]) = [x] * (1 - [x < 0])
 * with one Beaver product (no truncation: the factor is an integer 0/1).
 * tr: the A2B triples; (rb, ra): the B2A bit; (ma..mc): a MUL triple. */
void orc_relu(size_t n, const u64 *x0, const u64 *x1, u64 seed, u64 tag, const u64 *const *tr,
              const u64 *rb0, const u64 *rb1, const u64 *ra0, const u64 *ra1, const u64 *ma0,
              const u64 *ma1, const u64 *mb0, const u64 *mb1, const u64 *mc0, const u64 *mc1, u64 *z0,
              u64 *z1) {
  const size_t cnt = n ? n : 1;
  u64 *w0 = calloc(cnt, sizeof(u64)), *w1 = calloc(cnt, sizeof(u64)), *l0 = calloc(cnt, sizeof(u64)), *l1 = calloc(cnt, sizeof(u64));
  orc_a2b(n, x0, x1, seed, tag, tr, w0, w1);
  orc_b2a_bit(n, 63, w0, w1, rb0, rb1, ra0, ra1, l0, l1); /* [x < 0] */
  for (size_t i = 0; i < n; ++i) {                        /* [x >= 0] = 1 - [x < 0] */
    l0[i] = 1 - l0[i];
    l1[i] = (u64)0 - l1[i];
  }
  orc_beaver_mul(n, x0, x1, l0, l1, ma0, ma1, mb0, mb1, mc0, mc1, 0, z0, z1);
  free(w0); free(w1); free(l0); free(l1);
}
