"""Low-precision number formats used by the sketch in reduced precision
(test infrastructure: only tests/, the smoke check and the benchmark's CPU
baseline use this package; nothing here runs on the GPU path).

The method itself (the paper) is stated in real arithmetic; the sketch C, D
may be stored in a narrower format before the product (the precision
variants of Alg. 1 step 2 / Alg. 2 step 4). Two formats are defined here from
their published specifications:

* bfloat16: 8 exponent bits, 7 stored mantissa bits; round to nearest, ties
  to even (applied to the float32 value).
* OCP 8-bit floating point E4M3 ("FN" variant: bias 7, no infinities, the
  all-ones code is NaN, largest finite magnitude 448 = 1.75 * 2^8, smallest
  normal 2^-6, subnormals in steps of 2^-9), used in the OCP microscaling
  ("MX") block format: each run of 32 consecutive elements shares one
  power-of-two scale 2^X with X = floor(log2(amax)) - 8 (8 being the largest
  E4M3 exponent; at least -127, the smallest E8M0 scale), and each element is
  the E4M3 value nearest to x / 2^X, clamped to +-448.

All arithmetic is exact: the power-of-two divisions are exact in float64 and
the rounding uses numpy.rint (round half to even) on values scaled so that
the retained digits are integers.
"""
import numpy as np

E4M3_MAX = 448.0
E4M3_EMAX = 8          # exponent of the largest binade (448 = 1.75 * 2^8)
E4M3_EMIN = -6         # smallest normal exponent
E4M3_MBITS = 3
MX_BLOCK = 32


def f32(x):
    """float64 values rounded once to float32 (returned as float64)."""
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def bf16(x):
    """float64 values rounded to float32, then to bfloat16 (nearest, ties to
    even), returned as float64."""
    u = np.asarray(x, np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def e4m3(x):
    """Nearest E4M3 value of each float64 in x (ties to even mantissa),
    saturating at +-448; zero keeps its sign."""
    x = np.asarray(x, np.float64)
    a = np.abs(x)
    # binade exponent of |x| (frexp: a = f 2^e with 0.5 <= f < 1), held at the
    # subnormal exponent below the normal range
    _, e = np.frexp(np.where(a > 0, a, 1.0))
    e = np.maximum(e - 1, E4M3_EMIN)
    quantum = np.ldexp(1.0, e - E4M3_MBITS)
    q = np.rint(a / quantum) * quantum
    q = np.minimum(q, E4M3_MAX)
    return np.copysign(q, x)


def e4m3_values():
    """The finite E4M3 magnitudes, ascending (0, the 7 subnormals, the
    normals up to 448), from the encoding: code = exponent field * 8 +
    mantissa field, exponent field 0 subnormal."""
    vals = []
    for code in range(0x7F):            # 0x7f is NaN
        ef, mf = code >> 3, code & 7
        vals.append(mf * 2.0 ** -9 if ef == 0 else (1 + mf / 8.0) * 2.0 ** (ef - 7))
    return np.array(vals)


def mx_scale_exponents(X, block=MX_BLOCK):
    """Shared exponents of the MX blocks of each row of X (r x K, K a
    multiple of `block`): floor(log2(amax)) - 8, and 0 for an all-zero
    block."""
    X = np.asarray(X, np.float64)
    r, K = X.shape
    amax = np.abs(X).reshape(r, K // block, block).max(axis=2)
    _, e = np.frexp(np.where(amax > 0, amax, 1.0))
    # the E8M0 scale byte holds 2^-127 .. 2^127
    return np.where(amax > 0, np.maximum((e - 1) - E4M3_EMAX, -127), 0).astype(np.int64)


def mx_quantize(X, block=MX_BLOCK):
    """MX E4M3 quantization of the rows of X: returns (values, exponents)
    with values[i, k] = e4m3(X[i, k] / 2^E[i, k // block]) * 2^E[i, k //
    block] (the value the block format represents) and the exponents E."""
    X = np.asarray(X, np.float64)
    r, K = X.shape
    E = mx_scale_exponents(X, block)
    Eb = np.repeat(E, block, axis=1)
    return np.ldexp(e4m3(np.ldexp(X, -Eb)), Eb), E
