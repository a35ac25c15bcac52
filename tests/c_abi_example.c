/* The library driven from plain C through include/mpc.h: a two-party Beaver
 * matrix product in the limb and plain forms, an element-wise Beaver product
 * and a grouped call of two products (section 5.2), each revealed and checked
 * against the product computed here with uint64 wraparound (no truncation, so
 * every check is exact).  Device memory comes from the HIP runtime; the
 * library receives plain device pointers.  Exit status 0 when every check
 * passes. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mpc.h"

#define M 37
#define N 29
#define K 101
#define NE 5000

static int failures = 0;

#define CHECK(cond, what)                                  \
  do {                                                     \
    if (!(cond)) {                                         \
      fprintf(stderr, "c_abi_example: FAILED %s\n", what); \
      ++failures;                                          \
    }                                                      \
  } while (0)

#define MPC(call)                                                                          \
  do {                                                                                     \
    mpc_status st_ = (call);                                                               \
    if (st_ != MPC_OK) {                                                                   \
      fprintf(stderr, "c_abi_example: %s -> %s\n", #call, mpc_status_str(st_));            \
      exit(2);                                                                             \
    }                                                                                      \
  } while (0)

#define HIP(call)                                                       \
  do {                                                                  \
    if ((call) != hipSuccess) {                                         \
      fprintf(stderr, "c_abi_example: %s failed\n", #call);             \
      exit(3);                                                          \
    }                                                                   \
  } while (0)

/* host test data: SplitMix64 (Steele, Lea and Flood, 2014) over a counter */
static uint64_t mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
static void fill(uint64_t* v, size_t n, uint64_t seed) {
  for (size_t i = 0; i < n; ++i) v[i] = mix(seed + (i + 1) * 0x9e3779b97f4a7c15ULL);
}

static uint64_t* dalloc(size_t n) {
  void* p = NULL;
  HIP(hipMalloc(&p, (n ? n : 1) * sizeof(uint64_t)));
  return (uint64_t*)p;
}
static uint64_t* upload(const uint64_t* h, size_t n) {
  uint64_t* d = dalloc(n);
  HIP(hipMemcpy(d, h, n * sizeof(uint64_t), hipMemcpyHostToDevice));
  return d;
}
static void download(uint64_t* h, const uint64_t* d, size_t n) {
  HIP(hipMemcpy(h, d, n * sizeof(uint64_t), hipMemcpyDeviceToHost));
}

static mpc_triple triple(size_t na, size_t nb, size_t nc) {
  mpc_triple t;
  t.a0 = dalloc(na);
  t.a1 = dalloc(na);
  t.b0 = dalloc(nb);
  t.b1 = dalloc(nb);
  t.c0 = dalloc(nc);
  t.c1 = dalloc(nc);
  return t;
}

int main(void) {
  mpc_ctx* ctx = NULL;
  MPC(mpc_ctx_create(0, NULL, NULL, 20240901ULL, &ctx));

  /* ---- matrix product: reveal(Beaver(X, W)) == X @ W (mod 2^64) ---- */
  uint64_t* hx = malloc(sizeof(uint64_t) * M * K);
  uint64_t* hw = malloc(sizeof(uint64_t) * K * N);
  uint64_t* want = calloc((size_t)M * N, sizeof(uint64_t));
  uint64_t* got = malloc(sizeof(uint64_t) * M * N);
  fill(hx, (size_t)M * K, 1);
  fill(hw, (size_t)K * N, 2);
  for (int i = 0; i < M; ++i)
    for (int k = 0; k < K; ++k)
      for (int j = 0; j < N; ++j) want[i * N + j] += hx[i * K + k] * hw[k * N + j];
  uint64_t *x = upload(hx, (size_t)M * K), *w = upload(hw, (size_t)K * N);
  uint64_t *x0 = dalloc((size_t)M * K), *x1 = dalloc((size_t)M * K);
  uint64_t *w0 = dalloc((size_t)K * N), *w1 = dalloc((size_t)K * N);
  uint64_t *z0 = dalloc((size_t)M * N), *z1 = dalloc((size_t)M * N), *out = dalloc((size_t)M * N);
  MPC(mpc_share(ctx, x, (size_t)M * K, 0, 11, x0, x1));
  MPC(mpc_share(ctx, w, (size_t)K * N, 1, 12, w0, w1));
  const int64_t dims[3] = {M, N, K};
  mpc_triple tm = triple((size_t)M * K, (size_t)K * N, (size_t)M * N);
  MPC(mpc_dealer_triples(ctx, MPC_TRIPLE_MATMUL, 7, 13, dims, &tm));
  const mpc_form forms[2] = {MPC_FORM_LIMB8, MPC_FORM_PLAIN};
  for (int f = 0; f < 2; ++f) {
    MPC(mpc_beaver_matmul(ctx, M, N, K, x0, x1, w0, w1, &tm, 0, forms[f], z0, z1));
    MPC(mpc_reveal(ctx, z0, z1, (size_t)M * N, out));
    MPC(mpc_sync(ctx));
    download(got, out, (size_t)M * N);
    CHECK(memcmp(got, want, sizeof(uint64_t) * M * N) == 0, f == 0 ? "matmul, limb form" : "matmul, plain form");
  }

  /* ---- element-wise products, single and grouped ---- */
  uint64_t *ha = malloc(sizeof(uint64_t) * NE), *hb = malloc(sizeof(uint64_t) * NE);
  uint64_t *hp = malloc(sizeof(uint64_t) * NE), *hg = malloc(sizeof(uint64_t) * NE);
  fill(ha, NE, 3);
  fill(hb, NE, 4);
  for (int i = 0; i < NE; ++i) hp[i] = ha[i] * hb[i];
  uint64_t *ea = upload(ha, NE), *eb = upload(hb, NE);
  uint64_t *a0 = dalloc(NE), *a1 = dalloc(NE), *b0 = dalloc(NE), *b1 = dalloc(NE);
  uint64_t *p0 = dalloc(NE), *p1 = dalloc(NE), *q0 = dalloc(NE), *q1 = dalloc(NE), *pe = dalloc(NE);
  MPC(mpc_share(ctx, ea, NE, 0, 21, a0, a1));
  MPC(mpc_share(ctx, eb, NE, 1, 22, b0, b1));
  const int64_t ne[1] = {NE};
  mpc_triple te = triple(NE, NE, NE), te2 = triple(NE, NE, NE);
  MPC(mpc_dealer_triples(ctx, MPC_TRIPLE_MUL, 7, 23, ne, &te));
  MPC(mpc_dealer_triples(ctx, MPC_TRIPLE_MUL, 7, 24, ne, &te2));
  MPC(mpc_beaver_mul(ctx, NE, a0, a1, b0, b1, &te, 0, p0, p1));
  MPC(mpc_reveal(ctx, p0, p1, NE, pe));
  MPC(mpc_sync(ctx));
  download(hg, pe, NE);
  CHECK(memcmp(hg, hp, sizeof(uint64_t) * NE) == 0, "element-wise product");

  mpc_mul_desc d[2];
  memset(d, 0, sizeof d);
  d[0].n = NE;
  d[0].x0 = a0; d[0].x1 = a1; d[0].y0 = b0; d[0].y1 = b1; d[0].t = te; d[0].z0 = p0; d[0].z1 = p1;
  d[1] = d[0];
  d[1].n = NE - 1;  /* a shorter second product with its own triple and outputs */
  d[1].t = te2; d[1].z0 = q0; d[1].z1 = q1;
  MPC(mpc_beaver_mul_grouped(ctx, 2, d, 0));
  MPC(mpc_reveal(ctx, p0, p1, NE, pe));
  MPC(mpc_sync(ctx));
  download(hg, pe, NE);
  CHECK(memcmp(hg, hp, sizeof(uint64_t) * NE) == 0, "grouped product 0");
  MPC(mpc_reveal(ctx, q0, q1, NE - 1, pe));
  MPC(mpc_sync(ctx));
  download(hg, pe, NE - 1);
  CHECK(memcmp(hg, hp, sizeof(uint64_t) * (NE - 1)) == 0, "grouped product 1");

  /* ---- errors are status codes ---- */
  CHECK(mpc_share(ctx, ea, NE, 2, 25, a0, a1) == MPC_E_INVAL, "bad party index is MPC_E_INVAL");
  CHECK(mpc_beaver_mul(ctx, NE, a0, a1, b0, b1, &te, 0, a0, p1) == MPC_E_ALIAS, "aliased output is MPC_E_ALIAS");
  CHECK(mpc_status_str(MPC_E_ALIAS) != NULL, "status string");

  MPC(mpc_ctx_destroy(ctx));
  if (failures) return 1;
  printf("c_abi_example: all checks passed\n");
  return 0;
}
