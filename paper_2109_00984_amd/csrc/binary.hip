// binary.hip -- binary (XOR) sharing between two parties and the conversions
// to and from arithmetic sharing (App. C.1.1: binary secret sharing, bitwise
// AND, converting between secret-sharing types, logic-based operations).
//
// A binary sharing holds 64 independent shared bits per word, so one 64-bit
// XOR / AND per lane processes 64 bits; bitwise AND is the Beaver product
// over Z/2 with triples from the dealer.  Both parties' shares sit on the one
// GPU, so every opening inside a circuit is a device-local XOR: the whole
// arithmetic-to-binary adder (one AND round to start, six carry-lookahead
// levels) runs as one pass that reads the operand shares and the 12 AND
// triples of each word and writes the binary shares.  ReLU fuses that adder,
// the sign-bit conversion of Algorithm 2 and the final Beaver product.
#include "internal.h"

namespace mpc {
namespace {

constexpr int kBinThreads = 256;

#define BIN_LOOP(i, n) \
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)

// x = <x>_0 ^ <x>_1 with the zero-share (m, m); the source XORs its value in.
__global__ void __launch_bounds__(kBinThreads)
    k_bin_share(const u64* __restrict__ x, size_t n, int src, u64 key, u64* __restrict__ s0,
                u64* __restrict__ s1) {
  BIN_LOOP(i, n) {
    const u64 m = sm_out(key, i);
    s0[i] = src == 0 ? x[i] ^ m : m;
    s1[i] = src == 1 ? x[i] ^ m : m;
  }
}

__global__ void __launch_bounds__(kBinThreads)
    k_bin_reveal(const u64* __restrict__ s0, const u64* __restrict__ s1, size_t n, u64* __restrict__ out) {
  BIN_LOOP(i, n) out[i] = s0[i] ^ s1[i];
}

// AND triples: a_p, b_p, c_0 from the dealer's streams, c_1 = (a & b) ^ c_0.
__global__ void __launch_bounds__(kBinThreads)
    k_dealer_and(BinKeys k, size_t n, u64* __restrict__ a0, u64* __restrict__ a1, u64* __restrict__ b0,
                 u64* __restrict__ b1, u64* __restrict__ c0, u64* __restrict__ c1) {
  BIN_LOOP(i, n) {
    const u64 va0 = sm_out(k.a0, i), va1 = sm_out(k.a1, i), vb0 = sm_out(k.b0, i), vb1 = sm_out(k.b1, i);
    const u64 vc0 = sm_out(k.c0, i);
    a0[i] = va0;
    a1[i] = va1;
    b0[i] = vb0;
    b1[i] = vb1;
    c0[i] = vc0;
    c1[i] = ((va0 ^ va1) & (vb0 ^ vb1)) ^ vc0;
  }
}

// One Beaver AND on register values: both parties' shares in, both out.
struct Pair {
  u64 s0, s1;
};
__device__ __forceinline__ Pair and_gate(Pair x, Pair y, const TriplePtrs& t, size_t idx) {
  const u64 a0 = t.a0[idx], a1 = t.a1[idx], b0 = t.b0[idx], b1 = t.b1[idx];
  const u64 eps = (x.s0 ^ a0) ^ (x.s1 ^ a1);  // opened
  const u64 del = (y.s0 ^ b0) ^ (y.s1 ^ b1);  // opened
  return Pair{t.c0[idx] ^ (eps & b0) ^ (a0 & del) ^ (eps & del), t.c1[idx] ^ (eps & b1) ^ (a1 & del)};
}
__device__ __forceinline__ Pair shl(Pair v, int k) { return Pair{v.s0 << k, v.s1 << k}; }
__device__ __forceinline__ Pair xr(Pair a, Pair b) { return Pair{a.s0 ^ b.s0, a.s1 ^ b.s1}; }

__global__ void __launch_bounds__(kBinThreads)
    k_bin_and(size_t n, const u64* __restrict__ x0, const u64* __restrict__ x1, const u64* __restrict__ y0,
              const u64* __restrict__ y1, TriplePtrs t, u64* __restrict__ z0, u64* __restrict__ z1) {
  BIN_LOOP(i, n) {
    const Pair z = and_gate(Pair{x0[i], x1[i]}, Pair{y0[i], y1[i]}, t, i);
    z0[i] = z.s0;
    z1[i] = z.s1;
  }
}

// Arithmetic to binary for element i: each party binary-shares its share
// (<y_0> = (x0 ^ m0, m0), <y_1> = (m1, x1 ^ m1)), then the carry-lookahead
// adder: G = y0 & y1, P = y0 ^ y1; for k = 1..32 (doubling) G ^= P & (G << k)
// and (except at k = 32) P &= P << k, each level's two ANDs using the values
// from before it; sum = (y0 ^ y1) ^ (G << 1).  AND triple j of element i is
// entry j * n + i of the triple buffers.
__device__ __forceinline__ Pair a2b_one(u64 x0, u64 x1, u64 ky0, u64 ky1, const TriplePtrs& t, size_t i,
                                        size_t n) {
  const u64 m0 = sm_out(ky0, i), m1 = sm_out(ky1, i);
  const Pair y0{x0 ^ m0, m0}, y1{m1, x1 ^ m1};
  const Pair p0 = xr(y0, y1);
  size_t j = 0;
  Pair g = and_gate(y0, y1, t, (j++) * n + i);
  Pair p = p0;
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) {
    const Pair gk = and_gate(p, shl(g, k), t, (j++) * n + i);
    if (k < 32) p = and_gate(p, shl(p, k), t, (j++) * n + i);
    g = xr(g, gk);
  }
  return xr(p0, shl(g, 1));
}

__global__ void __launch_bounds__(kBinThreads)
    k_a2b(size_t n, const u64* __restrict__ x0, const u64* __restrict__ x1, u64 ky0, u64 ky1, TriplePtrs t,
          u64* __restrict__ z0, u64* __restrict__ z1) {
  BIN_LOOP(i, n) {
    const Pair z = a2b_one(x0[i], x1[i], ky0, ky1, t, i, n);
    z0[i] = z.s0;
    z1[i] = z.s1;
  }
}

// Algorithm 2's random bit r in {0, 1}: <r> = (w, w ^ r), [r] = (v, r - v).
__global__ void __launch_bounds__(kBinThreads)
    k_dealer_b2a(size_t n, u64 kr, u64 krb, u64 kra, u64* __restrict__ rb0, u64* __restrict__ rb1,
                 u64* __restrict__ ra0, u64* __restrict__ ra1) {
  BIN_LOOP(i, n) {
    const u64 r = sm_out(kr, i) & 1, w = sm_out(krb, i), v = sm_out(kra, i);
    rb0[i] = w;
    rb1[i] = w ^ r;
    ra0[i] = v;
    ra1[i] = r - v;
  }
}

// Algorithm 2 on one bit: z = bit of <b> ^ <r> (opened), [b] = [r] + z - 2 z [r].
__device__ __forceinline__ Pair b2a_one(Pair b, int bit, u64 rb0, u64 rb1, u64 ra0, u64 ra1) {
  const u64 z = (((b.s0 >> bit) ^ rb0) ^ ((b.s1 >> bit) ^ rb1)) & 1;
  return Pair{ra0 + z - 2 * z * ra0, ra1 - 2 * z * ra1};
}

__global__ void __launch_bounds__(kBinThreads)
    k_b2a_bit(size_t n, int bit, const u64* __restrict__ b0, const u64* __restrict__ b1,
              const u64* __restrict__ rb0, const u64* __restrict__ rb1, const u64* __restrict__ ra0,
              const u64* __restrict__ ra1, u64* __restrict__ z0, u64* __restrict__ z1) {
  BIN_LOOP(i, n) {
    const Pair z = b2a_one(Pair{b0[i], b1[i]}, bit, rb0[i], rb1[i], ra0[i], ra1[i]);
    z0[i] = z.s0;
    z1[i] = z.s1;
  }
}

// ReLU: s = [x < 0] = B2A(sign bit of A2B(x)), then x * (1 - s) by one Beaver
// product with the MUL triple m (no truncation: the factor is 0 or 1).
__global__ void __launch_bounds__(kBinThreads)
    k_relu(size_t n, const u64* __restrict__ x0, const u64* __restrict__ x1, u64 ky0, u64 ky1, TriplePtrs t,
           const u64* __restrict__ rb0, const u64* __restrict__ rb1, const u64* __restrict__ ra0,
           const u64* __restrict__ ra1, TriplePtrs m, u64* __restrict__ z0, u64* __restrict__ z1) {
  BIN_LOOP(i, n) {
    const u64 v0 = x0[i], v1 = x1[i];
    const Pair bx = a2b_one(v0, v1, ky0, ky1, t, i, n);
    const Pair neg = b2a_one(bx, 63, rb0[i], rb1[i], ra0[i], ra1[i]);
    const u64 f0 = 1 - neg.s0, f1 = (u64)0 - neg.s1;  // [x >= 0]
    const u64 a0 = m.a0[i], a1 = m.a1[i], b0 = m.b0[i], b1 = m.b1[i];
    const u64 eps = (v0 - a0) + (v1 - a1);
    const u64 del = (f0 - b0) + (f1 - b1);
    z0[i] = m.c0[i] + eps * b0 + a0 * del + eps * del;
    z1[i] = m.c1[i] + eps * b1 + a1 * del;
  }
}

unsigned grid_of(size_t n) {
  const size_t b = (n + kBinThreads - 1) / kBinThreads;
  return (unsigned)(b < 1 ? 1 : b > 65536 ? 65536 : b);
}

}  // namespace

#define BIN_LAUNCH(kernel, n, ...)                                                             \
  do {                                                                                         \
    if (!(n)) return hipSuccess;                                                               \
    hipLaunchKernelGGL(kernel, dim3(grid_of(n)), dim3(kBinThreads), 0, s, __VA_ARGS__);       \
    return hipGetLastError();                                                                  \
  } while (0)

hipError_t launch_bin_share(hipStream_t s, const u64* x, size_t n, int src, u64 key, u64* s0, u64* s1) {
  BIN_LAUNCH(k_bin_share, n, x, n, src, key, s0, s1);
}
hipError_t launch_bin_reveal(hipStream_t s, const u64* s0, const u64* s1, size_t n, u64* out) {
  BIN_LAUNCH(k_bin_reveal, n, s0, s1, n, out);
}
hipError_t launch_dealer_and(hipStream_t s, const BinKeys& k, size_t n, u64* a0, u64* a1, u64* b0, u64* b1,
                             u64* c0, u64* c1) {
  BIN_LAUNCH(k_dealer_and, n, k, n, a0, a1, b0, b1, c0, c1);
}
hipError_t launch_bin_and(hipStream_t s, size_t n, const u64* x0, const u64* x1, const u64* y0, const u64* y1,
                          const TriplePtrs& t, u64* z0, u64* z1) {
  BIN_LAUNCH(k_bin_and, n, n, x0, x1, y0, y1, t, z0, z1);
}
hipError_t launch_a2b(hipStream_t s, size_t n, const u64* x0, const u64* x1, u64 ky0, u64 ky1,
                      const TriplePtrs& t, u64* z0, u64* z1) {
  BIN_LAUNCH(k_a2b, n, n, x0, x1, ky0, ky1, t, z0, z1);
}
hipError_t launch_dealer_b2a(hipStream_t s, size_t n, u64 kr, u64 krb, u64 kra, u64* rb0, u64* rb1, u64* ra0,
                             u64* ra1) {
  BIN_LAUNCH(k_dealer_b2a, n, n, kr, krb, kra, rb0, rb1, ra0, ra1);
}
hipError_t launch_b2a_bit(hipStream_t s, size_t n, int bit, const u64* b0, const u64* b1, const u64* rb0,
                          const u64* rb1, const u64* ra0, const u64* ra1, u64* z0, u64* z1) {
  BIN_LAUNCH(k_b2a_bit, n, n, bit, b0, b1, rb0, rb1, ra0, ra1, z0, z1);
}
hipError_t launch_relu(hipStream_t s, size_t n, const u64* x0, const u64* x1, u64 ky0, u64 ky1,
                       const TriplePtrs& t, const u64* rb0, const u64* rb1, const u64* ra0, const u64* ra1,
                       const TriplePtrs& m, u64* z0, u64* z1) {
  BIN_LAUNCH(k_relu, n, n, x0, x1, ky0, ky1, t, rb0, rb1, ra0, ra1, m, z0, z1);
}

}  // namespace mpc
