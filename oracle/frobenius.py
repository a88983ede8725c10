"""Stage oracle for the Frobenius-partition variant -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module; it shares no code with the GPU library.
It follows App. C of Chen, Cheng, Kuo, Li, Yang, "Faster Multiplication for
Long Binary Polynomials" (arXiv:1708.09746): a polynomial of GF(2)[x] with
fewer than 128 n coefficients (n = 2^m) is represented, with no Kronecker
segmentation, by its values at the n points beta_{m+64} + V_m of GF(2^128),
where V_m = span(beta_0 .. beta_{m-1}) for the Cantor basis of the simple
variant (the field and basis of ``oracle.simple``).

Steps (App. C, the partition of points, the truncated FFT, the encoding):
* BasisCvt (Alg. 3) of the 2^(m+7) coefficients, each a bit;
* the "encoding": the first seven layers of FFT_LCH at alpha = beta_{m+64}
  over 2^(m+7) points, keeping only the branch of the first 2^m outputs: the
  element i < n is sum over j < 128 of g_{j n + i} times the product of the
  multipliers s_{m+t}(alpha) over the set bits t of j;
* FFT_LCH at alpha over the remaining n points.
A product c = a b with deg c < 128 n is recovered from the pointwise products
of the two value vectors: iFFT_LCH, then the inverse of the encoding (one
128 x 128 GF(2) system per point), then iBasisCvt.

Readings (also in the design notes): s_{m+t}(beta_{m+64}) = beta_{64-t} by the
Cantor shift rule (Sec. 3.3), so the encoding multiplier of bit t of j is
beta_{64-t}; n is the least power of two with 128 n at least the product's
length (at least 1).
"""
from __future__ import annotations

from functools import lru_cache

from . import simple as S
from . import tower as T


def alpha_coord(m: int) -> int:
    """Cantor coordinates of alpha = beta_{m+64}."""
    return 1 << (m + 64)


def point(m: int, j: int) -> int:
    """The evaluation point beta_{m+64} + phi(j), j < 2^m."""
    return S.phi(alpha_coord(m) ^ j)


@lru_cache(maxsize=None)
def encoding_products(m: int) -> tuple[int, ...]:
    """P_j = prod over set bits t of j of s_{m+t}(alpha), j < 128: the weight of
    coefficient j n + i in element i after the first seven layers."""
    lam = [S.s_cantor(m + t, alpha_coord(m)) for t in range(7)]
    out = []
    for j in range(128):
        p = 1
        for t in range(7):
            if (j >> t) & 1:
                p = S.mul(p, lam[t])
        out.append(p)
    return tuple(out)


def encode(bits: list[int], m: int) -> list[int]:
    """The encoding of App. C: element i = sum_j bits[j n + i] P_j."""
    n = 1 << m
    P = encoding_products(m)
    out = []
    for i in range(n):
        e = 0
        for j in range(128):
            if bits[j * n + i]:
                e ^= P[j]
        out.append(e)
    return out


@lru_cache(maxsize=None)
def _decoder(m: int):
    """Rows (pivot, vector, combination) that invert e = sum_j b_j P_j."""
    rows = []
    for j, p in enumerate(encoding_products(m)):
        v, comb = p, 1 << j
        for piv, rv, rc in rows:
            if (v >> piv) & 1:
                v ^= rv
                comb ^= rc
        if v == 0:
            raise RuntimeError("the encoding products are linearly dependent")
        piv = v.bit_length() - 1
        rows = [(q, rv ^ v, rc ^ comb) if (rv >> piv) & 1 else (q, rv, rc) for q, rv, rc in rows]
        rows.append((piv, v, comb))
    return tuple(rows)


def decode(elems: list[int], m: int) -> list[int]:
    """The inverse of encode: the 128 n bits back from n elements."""
    n = 1 << m
    rows = _decoder(m)
    bits = [0] * (128 * n)
    for i, e in enumerate(elems):
        comb = 0
        for piv, rv, rc in rows:
            if (e >> piv) & 1:
                e ^= rv
                comb ^= rc
        if e:
            raise ValueError("element outside the span of the encoding products")
        for j in range(128):
            bits[j * n + i] = (comb >> j) & 1
    return bits


def bits_of(a: int, nbits: int, total: int) -> list[int]:
    return [(a >> k) & 1 if k < nbits else 0 for k in range(total)]


def evaluate(a: int, nbits: int, m: int) -> list[int]:
    """E(a): the values of a at beta_{m+64} + V_m via BasisCvt of the bits,
    the encoding and FFT_LCH at alpha (requires nbits <= 128 * 2^m)."""
    total = 128 << m
    if nbits > total:
        raise ValueError("polynomial too long for 2^m points")
    g = T.basis_cvt(bits_of(a, nbits, total))
    return S.fft_lch(encode(g, m), alpha_coord(m))


def interpolate(vals: list[int], m: int, nbits: int) -> int:
    """The inverse of evaluate: iFFT_LCH at alpha, decode, iBasisCvt."""
    bits = T.from_novel(decode(S.ifft_lch(vals, alpha_coord(m)), m))
    r = 0
    for k in range(min(nbits, len(bits))):
        if bits[k]:
            r |= 1 << k
    return r


def points_log(na_bits: int, nb_bits: int) -> int:
    """m with 128 * 2^m the least such length holding the product."""
    nc = na_bits + nb_bits - 1
    m = 0
    while (128 << m) < nc:
        m += 1
    return m


def binpolymul_frobenius(a: int, na_bits: int, b: int, nb_bits: int) -> int:
    """c = a b through the Frobenius partition (App. C), small inputs only."""
    if na_bits == 0 or nb_bits == 0:
        return 0
    m = points_log(na_bits, nb_bits)
    fa = evaluate(a, na_bits, m)
    fb = evaluate(b, nb_bits, m)
    return interpolate([S.mul(x, y) for x, y in zip(fa, fb)], m, na_bits + nb_bits - 1)
