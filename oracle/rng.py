"""Oracle random factors: Philox4x64-10 words and the Gaussian transform.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Parity: pinned.
The Philox words are pinned against ``numpy.random.Philox`` (a third-party
Philox4x64-10); the transform is pinned against numpy's ``log``/``cos``/
``sqrt`` composition to a few ulp and by its moments.

The paper only asks for independent mean-zero, unit-variance sub-Gaussian
entries in every factor of a KRP (Definition 2.1; Gaussian entries in all its
experiments).  Both implementations of this project draw the same Gaussians,
entry by entry, from this counter-based definition (the "RNG spec"):

Generator
    Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): round
    multipliers 0xD2E7470EE14C6C93 and 0xCA5A826395121157, key increments
    0x9E3779B97F4A7C15 and 0xBB67AE8584CAA73B.
Key
    (seed, 0).
Counter of the entries (row a, columns 4j .. 4j+3) of factor ``f`` drawn for sketch ``k``
    (a, j, draw * 2**32 + k * 2**16 + f, instance).
    ``k`` is the sketched mode (0-based) in the Tucker algorithms, 0xFFFF for
    a factor set shared by all modes; ``f`` is the factor's mode; for the
    block-Hankel sketch f = 0, 1, 2, 3 name Omega1, Omega2, Psi1, Psi2 and
    ``instance`` is the Hankel instance (0 for tensors).
Transform of the output words (w0, w1, w2, w3)
    Pair p = 0 uses (w0, w1), pair p = 1 uses (w2, w3); for pair p with words
    (wu, wv):
    u1 = ((wu >> 11) + 1) * 2**-53  in (0, 1]
    k2 = wv >> 11                   (u2 = k2 * 2**-53 in [0, 1))
    r  = sqrt(-2 ln u1)
    column 4j + 2p     gets  r * cos(2 pi u2),
    column 4j + 2p + 1 gets  r * sin(2 pi u2),
    the two Box-Muller outputs of one (u1, u2), which are independent
    standard normals.  sin(2 pi u2) is defined as cos(2 pi u2 - pi/2), i.e.
    ``cos_two_pi((k2 - 2**51) mod 2**53)``, a shift that is exact in integers.
    ``ln`` and ``cos`` are this module's own FMA-free polynomial evaluations
    (below), so that any IEEE-754 binary64 implementation that performs the
    same correctly rounded +, -, *, / and sqrt in the same order reproduces
    every entry bit for bit.
Working-precision copies
    fp32: RNE to binary32.  bf16: RNE of the fp32 value to bfloat16.
    split bf16 pair: hi = bf16(fp32(g)), lo = bf16(fp32(g) - hi), the
    difference being exact in binary32.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_M32 = np.uint64(0xFFFFFFFF)
_PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
_PHILOX_M1 = np.uint64(0xCA5A826395121157)
_PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
_PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)
ROUNDS = 10

# ---------------------------------------------------------------------------
# Philox4x64-10
# ---------------------------------------------------------------------------


def _mulhilo64(a: np.ndarray, m: np.uint64):
    """Full 128-bit product of uint64 arrays ``a`` and the constant ``m``."""
    a = a.astype(np.uint64)
    a_lo, a_hi = a & _M32, a >> np.uint64(32)
    m_lo, m_hi = m & _M32, m >> np.uint64(32)
    with np.errstate(over="ignore"):
        lo = a * m  # wraps modulo 2**64
        ll = a_lo * m_lo
        lh = a_lo * m_hi
        hl = a_hi * m_lo
        hh = a_hi * m_hi
        mid = (ll >> np.uint64(32)) + (lh & _M32) + (hl & _M32)
        hi = hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1):
    """Philox4x64-10 of counter (c0..c3) under key (k0, k1); arrays broadcast.

    Returns the four output words as uint64 arrays.
    """
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.broadcast_to(np.asarray(k0, dtype=np.uint64), c0.shape)
    k1 = np.broadcast_to(np.asarray(k1, dtype=np.uint64), c0.shape)
    for r in range(ROUNDS):
        hi0, lo0 = _mulhilo64(c0, _PHILOX_M0)
        hi1, lo1 = _mulhilo64(c2, _PHILOX_M1)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if r != ROUNDS - 1:
            with np.errstate(over="ignore"):
                k0 = k0 + _PHILOX_W0
                k1 = k1 + _PHILOX_W1
    return c0, c1, c2, c3


# ---------------------------------------------------------------------------
# Constants of the transform, each the correctly rounded double of an exact
# rational or of a 60-digit value.
# ---------------------------------------------------------------------------
mpmath.mp.dps = 60
_LN2 = mpmath.log(2)
TWO_PI = float(2 * mpmath.pi)
SQRT2 = float(mpmath.sqrt(2))
# ln 2 split so that e * LN2_HI is exact for |e| < 2**21.
LN2_HI = float(np.frombuffer(
    (np.frombuffer(np.float64(float(_LN2)).tobytes(), dtype=np.uint64)
     & np.uint64(0xFFFFFFFFFFE00000)).tobytes(), dtype=np.float64)[0])
LN2_LO = float(_LN2 - mpmath.mpf(LN2_HI))
# ln m = 2 s (1 + s^2/3 + s^4/5 + ...), |s| <= 0.1716 -> 12 terms.
LOG_COEF = [1.0 / (2 * j + 1) for j in range(12)]
# cos t = sum (-1)^k t^(2k)/(2k)!  (11 terms), sin t = t sum (-1)^k t^(2k)/(2k+1)!
# (10 terms) on |t| <= pi/4.
COS_COEF = [(-1) ** k / math.factorial(2 * k) for k in range(11)]
SIN_COEF = [(-1) ** k / math.factorial(2 * k + 1) for k in range(10)]


def _horner(z: np.ndarray, coef) -> np.ndarray:
    """sum_j coef[j] z^j by Horner's rule with separate multiply and add."""
    p = np.full_like(z, coef[-1])
    for cj in reversed(coef[:-1]):
        p = p * z
        p = p + cj
    return p


def log_unit(u1: np.ndarray) -> np.ndarray:
    """ln(u1) for u1 in (0, 1], FMA-free, reproducible bit for bit."""
    u1 = np.asarray(u1, dtype=np.float64)
    bits = u1.view(np.uint64)
    e = ((bits >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64) - 1023
    mbits = (bits & np.uint64(0x000FFFFFFFFFFFFF)) | np.uint64(0x3FF0000000000000)
    m = mbits.view(np.float64).copy()  # m in [1, 2), u1 = m 2^e exactly
    big = m > SQRT2
    m = np.where(big, m * 0.5, m)
    e = np.where(big, e + 1, e)
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    p = _horner(z, LOG_COEF)
    ln_m = (s + s) * p
    ef = e.astype(np.float64)
    return ef * LN2_HI + (ef * LN2_LO + ln_m)


def cos_two_pi(k2: np.ndarray) -> np.ndarray:
    """cos(2 pi k2 2^-53) for integers 0 <= k2 < 2^53, FMA-free.

    Reduction by the nearest quarter turn q is exact in integers:
    f = (k2 - q 2^51) 2^-53 lies in [-1/8, 1/8]; theta = 2 pi f.
    """
    k2 = np.asarray(k2, dtype=np.uint64)
    q = (k2 + np.uint64(1 << 50)) >> np.uint64(51)
    rem = k2.astype(np.int64) - (q.astype(np.int64) << 51)
    f = rem.astype(np.float64) * 2.0 ** -53
    theta = TWO_PI * f
    z = theta * theta
    c = _horner(z, COS_COEF)
    s = theta * _horner(z, SIN_COEF)
    qm = (q & np.uint64(3)).astype(np.int64)
    return np.select([qm == 0, qm == 1, qm == 2], [c, -s, -c], s)


def sin_two_pi(k2: np.ndarray) -> np.ndarray:
    """sin(2 pi k2 2^-53) = cos(2 pi (k2 - 2^51) 2^-53), the shift taken mod 2^53."""
    k2 = np.asarray(k2, dtype=np.uint64)
    return cos_two_pi((k2 - np.uint64(1 << 51)) & np.uint64((1 << 53) - 1))


def _radius_and_angle(wu, wv):
    wu = np.asarray(wu, dtype=np.uint64)
    wv = np.asarray(wv, dtype=np.uint64)
    u1 = ((wu >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * log_unit(u1)), wv >> np.uint64(11)


def gaussian_from_words(w0, w1) -> np.ndarray:
    """The cosine output of the Box-Muller transform of one word pair."""
    r, k2 = _radius_and_angle(w0, w1)
    return r * cos_two_pi(k2)


def gaussian_sin_from_words(w0, w1) -> np.ndarray:
    """The sine output of the Box-Muller transform of one word pair."""
    r, k2 = _radius_and_angle(w0, w1)
    return r * sin_two_pi(k2)


def counter_word2(draw: int, sketch: int, f: int) -> int:
    return (int(draw) << 32) | (int(sketch) << 16) | int(f)


def factor(seed: int, draw: int, sketch: int, f: int, rows: int, cols: int,
           instance: int = 0) -> np.ndarray:
    """Gaussian factor matrix (rows x cols, float64) of the RNG spec."""
    a = np.arange(rows, dtype=np.uint64)[:, None]
    c = np.arange(cols, dtype=np.uint64)[None, :]
    w = philox4x64(a, c >> np.uint64(2), np.uint64(counter_word2(draw, sketch, f)),
                   np.uint64(instance), np.uint64(seed), np.uint64(0))
    w = [np.broadcast_to(x, (rows, cols)) for x in w]
    second = ((c >> np.uint64(1)) & np.uint64(1)) == 1   # pair p = 1: words (w2, w3)
    wu = np.where(second, w[2], w[0])
    wv = np.where(second, w[3], w[1])
    odd = (c & np.uint64(1)) == 1                        # sine output of the pair
    g = np.where(odd, gaussian_sin_from_words(wu, wv), gaussian_from_words(wu, wv))
    return g.reshape(rows, cols)


# ---------------------------------------------------------------------------
# Working-precision copies
# ---------------------------------------------------------------------------


def to_bf16_bits(x32: np.ndarray) -> np.ndarray:
    """Round binary32 values to bfloat16 (nearest, ties to even); uint16 bits."""
    b = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = (b + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return (r & np.uint64(0xFFFF)).astype(np.uint16)


def bf16_bits_to_f32(h: np.ndarray) -> np.ndarray:
    return (np.asarray(h, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def round_fp32(g: np.ndarray) -> np.ndarray:
    return np.asarray(g, dtype=np.float64).astype(np.float32)


def round_bf16(g: np.ndarray) -> np.ndarray:
    """bf16(fp32(g)) as float32 values."""
    return bf16_bits_to_f32(to_bf16_bits(round_fp32(g)))


def split_bf16(g: np.ndarray):
    """(hi, lo) bfloat16 pair of fp32(g), returned as float32 values."""
    x = round_fp32(g)
    hi = bf16_bits_to_f32(to_bf16_bits(x))
    lo = bf16_bits_to_f32(to_bf16_bits((x - hi).astype(np.float32)))
    return hi, lo
