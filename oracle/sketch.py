"""Sketch operator Omega of the randomized SVD (Alg. 4, first step).

The paper draws the sketch uniformly from [-1, 1].  To let two independent
implementations draw the *same* sketch, element ``i`` (row-major linear index
over (column multi-index of the implicit operator, sketch column j), j
fastest) is produced by a counter-based generator built from the SplitMix64
output function (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014):

    mix(z):  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
             z ^= z >> 27; z *= 0x94D049BB133111EB;
             z ^= z >> 31
    base   = mix(mix(seed) + stream_id)
    h_i    = mix(base + (i + 1) * 0x9E3779B97F4A7C15)
    Omega_i = 2 * (h_i >> 11) * 2^-53 - 1          (uniform in [-1, 1))

All integer arithmetic is modulo 2^64.  The float result is exact (no
rounding), so any correct implementation reproduces it bitwise.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z):
    """SplitMix64 output function on uint64 (array or scalar), wrapping mod 2^64."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z ^ (z >> np.uint64(30))
        z = z * _M1
        z = z ^ (z >> np.uint64(27))
        z = z * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def stream_base(seed, stream_id):
    with np.errstate(over="ignore"):
        return mix64(mix64(np.uint64(seed)) + np.uint64(stream_id))


def sketch(seed, stream_id, n_cols, k):
    """Omega of shape (n_cols, k), float64, uniform in [-1, 1)."""
    base = stream_base(seed, stream_id)
    i = np.arange(n_cols * k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        h = mix64(base + (i + np.uint64(1)) * _GOLDEN)
    mant = (h >> np.uint64(11)).astype(np.float64)
    return (2.0 * mant * 2.0 ** -53 - 1.0).reshape(n_cols, k)


def stream_id(pass_, nrow, ncol, row, col):
    """Sketch stream of the einsumsvd that absorbs lattice column ``col`` of row
    ``row`` during contraction pass ``pass_`` (0 top-down, 1 bottom-up)."""
    return 1 + ((pass_ * nrow + row) * ncol + col)
