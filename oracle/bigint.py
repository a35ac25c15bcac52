"""Arbitrary-precision twin of the oracle for tiny shapes (TEST INFRASTRUCTURE ONLY).

Python integers never overflow, so every ring result here is formed exactly
over the integers and only then reduced with an explicit ``% 2**64``.  This is
the plain definition of arithmetic in Z/2^64 (section 5.1 of the paper).
"""
Q = 1 << 64


def s64(v):
    """Signed (two's-complement) reading of a ring element."""
    v %= Q
    return v - Q if v >= Q // 2 else v


def matmul(A, B):
    """Exact integer product of two nested lists, reduced mod 2^64."""
    K = len(B)
    N = len(B[0]) if K else 0
    return [[sum(int(A[i][k]) * int(B[k][j]) for k in range(K)) % Q for j in range(N)]
            for i in range(len(A))]


def floor_div_pow2(v, bits):
    """floor(s64(v) / 2^bits) as a ring element (Python // floors)."""
    return (s64(v) // (1 << bits)) % Q


def splitmix64_stream(state, count):
    """First `count` outputs of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
    from the given state, stepping the state by the golden gamma each draw."""
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) % Q
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) % Q
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) % Q
        out.append(z ^ (z >> 31))
    return out
