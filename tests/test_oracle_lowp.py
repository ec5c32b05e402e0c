"""Pins of the oracle's low-precision formats (CPU only): E4M3 rounding
against a brute-force nearest-value search over the format's code table,
the code table against the format's defining constants, bfloat16 against
torch's conversion, and the MX block quantization against its definition."""
import numpy as np
import pytest

from oracle import lowp


def test_e4m3_code_table():
    v = lowp.e4m3_values()
    assert len(v) == 127 and v[0] == 0.0
    assert v[-1] == 448.0                      # largest finite: S.1111.110
    assert v[1] == 2.0 ** -9 and v[7] == 7 * 2.0 ** -9 and v[8] == 2.0 ** -6
    assert np.all(np.diff(v) > 0)
    # every binade from 2^-6 up holds 8 equally spaced values
    for e in range(-6, 9):
        b = v[(v >= 2.0 ** e) & (v < 2.0 ** (e + 1))]
        assert len(b) == (8 if e < 8 else 7)
        assert np.allclose(np.diff(b), 2.0 ** (e - 3))


def _brute(x):
    """Nearest finite E4M3 magnitude by search, ties to the even mantissa
    (code with an even last bit), saturating; sign restored."""
    v = lowp.e4m3_values()
    out = np.empty_like(x)
    for i, xi in enumerate(x):
        a = abs(xi)
        if a >= 448.0:
            m = 448.0
        else:
            d = np.abs(v - a)
            best = np.flatnonzero(d == d.min())
            m = v[best[0]] if len(best) == 1 else v[[b for b in best if b % 2 == 0][0]]
        out[i] = np.copysign(m, xi)
    return out


def test_e4m3_matches_brute_force():
    g = np.random.Generator(np.random.PCG64(3))
    x = np.concatenate([
        g.standard_normal(3000) * 10.0 ** g.uniform(-4, 3, 3000),
        lowp.e4m3_values(), -lowp.e4m3_values(),
        # every midpoint between neighbouring codes (exact ties)
        (lowp.e4m3_values()[1:] + lowp.e4m3_values()[:-1]) / 2,
        [448.0, 460.0, 480.0, 1e6, -1e6, 2.0 ** -10, 3 * 2.0 ** -11, 2.0 ** -12],
    ])
    assert np.array_equal(lowp.e4m3(x), _brute(x))


def test_e4m3_is_idempotent_and_saturates():
    v = lowp.e4m3_values()
    assert np.array_equal(lowp.e4m3(v), v)
    assert lowp.e4m3(np.array([1e30]))[0] == 448.0
    assert lowp.e4m3(np.array([-464.0]))[0] == -448.0   # the midpoint to the missing 480 saturates


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    g = np.random.Generator(np.random.PCG64(4))
    x = g.standard_normal(20000) * 10.0 ** g.uniform(-30, 30, 20000)
    ref = torch.from_numpy(x).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lowp.bf16(x), ref)


def test_mx_quantize_definition():
    g = np.random.Generator(np.random.PCG64(5))
    X = g.standard_normal((7, 96)) * np.exp(g.normal(0, 3, (7, 96)))
    X[2, 32:64] = 0.0                           # an all-zero block
    Q, E = lowp.mx_quantize(X)
    assert E.shape == (7, 3) and E[2, 1] == 0 and np.all(Q[2, 32:64] == 0)
    for i in range(7):
        for b in range(3):
            blk = X[i, 32 * b:32 * b + 32]
            amax = np.abs(blk).max()
            if amax == 0:
                continue
            e = int(np.floor(np.log2(amax)))
            assert E[i, b] == e - 8
            # the largest element lands in [256, 512) before clamping to 448
            assert 256 <= amax / 2.0 ** E[i, b] < 512
            assert np.array_equal(Q[i, 32 * b:32 * b + 32],
                                  _brute(blk / 2.0 ** E[i, b]) * 2.0 ** E[i, b])


def test_mx_quantize_power_of_two_invariance():
    g = np.random.Generator(np.random.PCG64(6))
    X = g.standard_normal((4, 64))
    Q, E = lowp.mx_quantize(X)
    Q2, E2 = lowp.mx_quantize(X * 2.0 ** 37)
    assert np.array_equal(Q2, Q * 2.0 ** 37) and np.array_equal(E2, E + 37)
