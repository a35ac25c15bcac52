// multiparty.hip -- element-wise kernels for sharing among P > 2 parties.
//
// App. C.1.1 describes arithmetic sharing for any number of parties |P|:
// sharing by a pseudorandom zero-share (section 5.1), the Beaver product and
// square with one opening, and a truncation that corrects for the number of
// times the parties' shares wrap around the ring (Algorithm 1, where the
// plaintext wrap eta is taken as 0).  All P parties' shares live on the one
// GPU as P buffers; each kernel here takes them as arrays of pointers, so one
// pass over HBM serves every party, and the opened values never leave the
// device.  The matrix product reuses the ring GEMM forms (see api.cpp).
//
// Wrap counts are kept exactly with signed-overflow tests: adding v to an
// accumulator a wraps upwards when a and v are both >= 0 and the sum is < 0
// (the exact sum is the signed result plus Q), downwards when both are < 0
// and the sum is >= 0 (minus Q).
#include "internal.h"

namespace mpc {
namespace {

constexpr int kMpThreads = 256;

__device__ __forceinline__ int add_wrap(u64 a, u64 v, u64 s) {
  const i64 sa = (i64)a, sv = (i64)v, ss = (i64)s;
  return (sa >= 0 && sv >= 0 && ss < 0) ? 1 : (sa < 0 && sv < 0 && ss >= 0) ? -1 : 0;
}

__device__ __forceinline__ size_t first_index() { return (size_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ size_t grid_stride() { return (size_t)gridDim.x * blockDim.x; }

// s_p = (m_p - m_{(p+1) mod P}) + [p = src] x,  m_p = G(key_p, i)
__global__ void __launch_bounds__(kMpThreads)
    k_mp_share(const u64* __restrict__ x, size_t n, int P, int src, MpKeys keys, MpOut s) {
  for (size_t i = first_index(); i < n; i += grid_stride()) {
    const u64 first = sm_out(keys.k[0], i);
    u64 cur = first;
    for (int p = 0; p < P; ++p) {
      const u64 next = p + 1 < P ? sm_out(keys.k[p + 1], i) : first;
      s.p[p][i] = (cur - next) + (p == src ? x[i] : 0);
      cur = next;
    }
  }
}

__global__ void __launch_bounds__(kMpThreads) k_mp_reveal(MpIn s, int P, size_t n, u64* __restrict__ out) {
  for (size_t i = first_index(); i < n; i += grid_stride()) {
    u64 v = 0;
    for (int p = 0; p < P; ++p) v += s.p[p][i];
    out[i] = v;
  }
}

// out_p = G(key_p, i) for p < cnt, and sum = sum of them (sum may be null)
__global__ void __launch_bounds__(kMpThreads)
    k_mp_fill_sum(MpKeys keys, int cnt, size_t n, MpOut out, u64* __restrict__ sum) {
  for (size_t i = first_index(); i < n; i += grid_stride()) {
    u64 v = 0;
    for (int p = 0; p < cnt; ++p) {
      const u64 g = sm_out(keys.k[p], i);
      out.p[p][i] = g;
      v += g;
    }
    if (sum) sum[i] = v;
  }
}

// Element-wise dealer: a_p, b_p from the PRG; the product (a*b, or a*a for
// the square pair, then into b) is split with keys ks: G for the first P-1
// parties, the rest for the last.
__global__ void __launch_bounds__(kMpThreads)
    k_mp_dealer_mul(MpKeys ka, MpKeys kb, MpKeys ks, int P, size_t n, int square, MpOut a, MpOut b,
                    MpOut c) {
  for (size_t i = first_index(); i < n; i += grid_stride()) {
    u64 av = 0, bv = 0;
    for (int p = 0; p < P; ++p) {
      const u64 g = sm_out(ka.k[p], i);
      a.p[p][i] = g;
      av += g;
    }
    if (!square)
      for (int p = 0; p < P; ++p) {
        const u64 g = sm_out(kb.k[p], i);
        b.p[p][i] = g;
        bv += g;
      }
    u64 rest = square ? av * av : av * bv;
    MpOut& dst = square ? b : c;
    for (int p = 0; p < P - 1; ++p) {
      const u64 g = sm_out(ks.k[p], i);
      dst.p[p][i] = g;
      rest -= g;
    }
    dst.p[P - 1][i] = rest;
  }
}

// eps = sum_p (x_p - a_p)
__global__ void __launch_bounds__(kMpThreads)
    k_mp_open(MpIn x, MpIn a, int P, size_t n, u64* __restrict__ eps) {
  for (size_t i = first_index(); i < n; i += grid_stride()) {
    u64 v = 0;
    for (int p = 0; p < P; ++p) v += x.p[p][i] - a.p[p][i];
    eps[i] = v;
  }
}

// Beaver product / square among P parties, mask, open and finish in one pass.
// The loops run over PMAX >= P parties (the smallest of 2, 4, 8, 16) with a
// test of p against P, so that every index is known when compiling: a_p and
// b_p, read for the open, stay in registers for the finish (each share is
// read from memory once), and the register arrays stay small for the usual
// party counts.
template <int PMAX>
__global__ void __launch_bounds__(kMpThreads)
    k_mp_beaver_mul(MpIn x, MpIn y, MpIn a, MpIn b, MpIn c, int P, size_t n, int square, MpOut z) {
  for (size_t i = first_index(); i < n; i += grid_stride()) {
    u64 av[PMAX], bv[PMAX];
    u64 eps = 0, del = 0;
#pragma unroll
    for (int p = 0; p < PMAX; ++p)
      if (p < P) {
        av[p] = a.p[p][i];
        eps += x.p[p][i] - av[p];
      }
    if (!square) {
#pragma unroll
      for (int p = 0; p < PMAX; ++p)
        if (p < P) {
          bv[p] = b.p[p][i];
          del += y.p[p][i] - bv[p];
        }
    }
#pragma unroll
    for (int p = 0; p < PMAX; ++p)
      if (p < P) {
        u64 v;
        if (square) v = b.p[p][i] + 2 * eps * av[p] + (p == 0 ? eps * eps : 0);
        else v = c.p[p][i] + eps * bv[p] + av[p] * del + (p == 0 ? eps * del : 0);
        z.p[p][i] = v;
      }
  }
}

// Dealer of Algorithm 1's inputs: r_p = G(kr_p); the wrap count theta_r of
// r's shares, shared as t_p = G(kt_p) for p < P-1 and the rest for the last.
__global__ void __launch_bounds__(kMpThreads)
    k_mp_dealer_trunc(MpKeys kr, MpKeys kt, int P, size_t n, MpOut r, MpOut t) {
  for (size_t i = first_index(); i < n; i += grid_stride()) {
    u64 acc = 0;
    i64 theta = 0;
    for (int p = 0; p < P; ++p) {
      const u64 g = sm_out(kr.k[p], i);
      r.p[p][i] = g;
      const u64 s = acc + g;
      theta += add_wrap(acc, g, s);
      acc = s;
    }
    u64 rest = (u64)theta;
    for (int p = 0; p < P - 1; ++p) {
      const u64 g = sm_out(kt.k[p], i);
      t.p[p][i] = g;
      rest -= g;
    }
    t.p[P - 1][i] = rest;
  }
}

// Algorithm 1 and the division, in place (eta = 0):
//   z_p = x_p + r_p with beta_p its wrap;  theta_z = the wrap count of the z_p;
//   [theta_x]_p = [p = 0] theta_z + beta_p - t_p;
//   x_p <- floor(s64(x_p) / 2^bits) - [theta_x]_p * 2^(64 - bits).
__global__ void __launch_bounds__(kMpThreads)
    k_mp_truncate(MpOut x, MpIn r, MpIn t, int P, size_t n, int bits) {
  for (size_t i = first_index(); i < n; i += grid_stride()) {
    u64 xv[kMaxParties];
    int beta[kMaxParties];
    u64 acc = 0;
    i64 theta_z = 0;
    for (int p = 0; p < P; ++p) {
      xv[p] = x.p[p][i];
      const u64 rv = r.p[p][i];
      const u64 z = xv[p] + rv;
      beta[p] = add_wrap(xv[p], rv, z);
      const u64 s = acc + z;
      theta_z += add_wrap(acc, z, s);
      acc = s;
    }
    const u64 scale = (u64)1 << (64 - bits);
    for (int p = 0; p < P; ++p) {
      const u64 th = (p == 0 ? (u64)theta_z : 0) + (u64)(i64)beta[p] - t.p[p][i];
      x.p[p][i] = (u64)((i64)xv[p] >> bits) - th * scale;
    }
  }
}

unsigned grid_for(size_t n) {
  const size_t b = (n + kMpThreads - 1) / kMpThreads;
  return (unsigned)(b < 1 ? 1 : b > 65536 ? 65536 : b);
}

}  // namespace

hipError_t launch_mp_share(hipStream_t s, const u64* x, size_t n, int P, int src, const MpKeys& keys,
                           const MpOut& out) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_mp_share, dim3(grid_for(n)), dim3(kMpThreads), 0, s, x, n, P, src, keys, out);
  return hipGetLastError();
}

hipError_t launch_mp_reveal(hipStream_t s, const MpIn& in, int P, size_t n, u64* out) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_mp_reveal, dim3(grid_for(n)), dim3(kMpThreads), 0, s, in, P, n, out);
  return hipGetLastError();
}

hipError_t launch_mp_fill_sum(hipStream_t s, const MpKeys& keys, int cnt, size_t n, const MpOut& out,
                              u64* sum) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_mp_fill_sum, dim3(grid_for(n)), dim3(kMpThreads), 0, s, keys, cnt, n, out, sum);
  return hipGetLastError();
}

hipError_t launch_mp_dealer_mul(hipStream_t s, const MpKeys& ka, const MpKeys& kb, const MpKeys& ks, int P,
                                size_t n, int square, const MpOut& a, const MpOut& b, const MpOut& c) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_mp_dealer_mul, dim3(grid_for(n)), dim3(kMpThreads), 0, s, ka, kb, ks, P, n, square, a,
                     b, c);
  return hipGetLastError();
}

hipError_t launch_mp_open(hipStream_t s, const MpIn& x, const MpIn& a, int P, size_t n, u64* eps) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_mp_open, dim3(grid_for(n)), dim3(kMpThreads), 0, s, x, a, P, n, eps);
  return hipGetLastError();
}

hipError_t launch_mp_beaver_mul(hipStream_t s, const MpIn& x, const MpIn& y, const MpIn& a, const MpIn& b,
                                const MpIn& c, int P, size_t n, int square, const MpOut& z) {
  if (!n) return hipSuccess;
  const dim3 grid(grid_for(n)), block(kMpThreads);
  if (P <= 2) hipLaunchKernelGGL(k_mp_beaver_mul<2>, grid, block, 0, s, x, y, a, b, c, P, n, square, z);
  else if (P <= 4) hipLaunchKernelGGL(k_mp_beaver_mul<4>, grid, block, 0, s, x, y, a, b, c, P, n, square, z);
  else if (P <= 8) hipLaunchKernelGGL(k_mp_beaver_mul<8>, grid, block, 0, s, x, y, a, b, c, P, n, square, z);
  else hipLaunchKernelGGL(k_mp_beaver_mul<kMaxParties>, grid, block, 0, s, x, y, a, b, c, P, n, square, z);
  return hipGetLastError();
}

hipError_t launch_mp_dealer_trunc(hipStream_t s, const MpKeys& kr, const MpKeys& kt, int P, size_t n,
                                  const MpOut& r, const MpOut& t) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_mp_dealer_trunc, dim3(grid_for(n)), dim3(kMpThreads), 0, s, kr, kt, P, n, r, t);
  return hipGetLastError();
}

hipError_t launch_mp_truncate(hipStream_t s, const MpOut& x, const MpIn& r, const MpIn& t, int P, size_t n,
                              int bits) {
  if (!n || bits <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mp_truncate, dim3(grid_for(n)), dim3(kMpThreads), 0, s, x, r, t, P, n, bits);
  return hipGetLastError();
}

}  // namespace mpc
