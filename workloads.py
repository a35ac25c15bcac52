"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module only draws inputs (numpy ``Generator(PCG64)``) and describes
shapes; it contains none of the method's arithmetic (no encoding, sharing,
products or truncation).  Real-valued inputs are returned as float64 and are
encoded by whichever side consumes them; raw ring operands are uniform uint64.

Workloads (the paper's private-inference setting of section 6: a secret-shared
model applied to secret-shared data, two parties, Z/2^64, 16 fractional bits):
  * small:   X[64x128] @ W[128x32] and an element-wise product over 4096
             elements, values uniform in [-4, 4];
  * mlp:     3-layer perceptron 784-1024-1024-10, batch 128, values in [-1, 1],
             square activations between layers;
  * gemm4k:  one ring GEMM / Beaver matmul at M = N = K = 4096 on uniform
             uint64 operands;
  * conv:    a 10-layer 1-D convolution stack with Wav2Letter's shapes
             (section 6.2), batch 8, 40 channels x 1600 samples, values in
             [-2, 2], square activations after every layer but the last;
  * grouped: 256 independent Beaver matmuls with log-uniform M in [16, 2048],
             N in [16, 1024], K in [32, 4096].
No dataset is used: synthetic values of the paper's shapes stand in for its
text, speech and image data.
"""
import math

import numpy as np

FRAC_BITS = 16


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform(seed, shape, lo, hi):
    """float64 values uniform in [lo, hi)."""
    return rng(seed).uniform(lo, hi, size=shape)


def uniform_u64(seed, shape):
    """Ring elements uniform over all 2^64 values."""
    return rng(seed).integers(0, 2**64, size=shape, dtype=np.uint64, endpoint=False)


def loguniform_dims(seed, count, lo, hi):
    """dim = clamp(round(exp(U(ln lo, ln hi))), lo, hi)."""
    u = rng(seed).uniform(math.log(lo), math.log(hi), size=count)
    return np.clip(np.rint(np.exp(u)), lo, hi).astype(np.int64)


# Seeds: workload c uses data seed 1000 + c, party (PRZS) seed 2000 + c and
# dealer seed 3000 + c.
def seeds(c):
    return 1000 + c, 2000 + c, 3000 + c


SMALL = dict(M=64, K=128, N=32, n_elem=4096, lo=-4.0, hi=4.0)
MLP = dict(batch=128, dims=(784, 1024, 1024, 10), lo=-1.0, hi=1.0)
GEMM4K = dict(M=4096, N=4096, K=4096)
GROUPED = dict(count=256, M=(16, 2048), N=(16, 1024), K=(32, 4096))

# (Cin, Cout, kernel, stride) per layer; activations after all but the last.
CONV_STACK = [(40, 250, 48, 2)] + [(250, 250, 7, 1)] * 7 + [(250, 2000, 32, 1), (2000, 40, 1, 1)]
CONV = dict(batch=8, channels=40, length=1600, lo=-2.0, hi=2.0, layers=CONV_STACK)


def conv_shapes(batch, length, layers=CONV_STACK):
    """[(Bt, Cin, L, Cout, ksz, stride, Lout)] for a valid-padding stack."""
    out = []
    L = length
    for cin, cout, k, s in layers:
        lout = (L - k) // s + 1
        out.append((batch, cin, L, cout, k, s, lout))
        L = lout
    return out


def grouped_shapes(seed, count=256, M=(16, 2048), N=(16, 1024), K=(32, 4096)):
    ms = loguniform_dims(seed, count, *M)
    ns = loguniform_dims(seed + 1, count, *N)
    ks = loguniform_dims(seed + 2, count, *K)
    return [(int(m), int(n), int(k)) for m, n, k in zip(ms, ns, ks)]
