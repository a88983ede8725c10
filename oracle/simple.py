"""Stage oracle for the simple variant of the multiplier -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It shares no code with the GPU library.  It follows Alg. 4 of
Chen, Cheng, Kuo, Li, Yang, "Faster Multiplication for Long Binary
Polynomials" (arXiv:1708.09746): the working field stays in the polynomial
basis, the LCH FFT evaluates at points of a Cantor basis, and each field
product is a full GF(2^128) product.

Conventions
-----------
* GF(2^128) = GF(2)[x]/(x^128 + x^7 + x^2 + x + 1), the field of Sec. 3.1
  (the irreducible-polynomial construction, the same field as AES-GCM).  An
  element is a Python int below 2^128: bit e is the coefficient of x^e.  A
  64-bit word of the input is the element of degree < 64 with the same bits,
  so Split needs no change of representation.
* The Cantor basis (Sec. 3.3): beta_0 = 1 and beta_i^2 + beta_i = beta_{i-1}.
  phi(k) = sum of beta_j over the set bits j of k (Sec. 3.3, the element
  represented by k).  The FFT output index j holds the value at phi(j).

Readings of the paper taken here (each also listed in the design notes):
* Of the two roots y, y + 1 of y^2 + y = beta_{i-1}, beta_i is the one whose
  coefficient of x^0 is zero (the paper does not fix the choice; any choice
  gives a Cantor basis, and the product does not depend on it).
* FFT size and operand conversion as in Alg. 5 with w = 64: N = max(2,
  2^ceil(log2(n_a + n_b - 1))) points for n_a and n_b words, each operand
  converted at its own power-of-two length.
* The subspace polynomials s_i of the Cantor basis are the ones the tower
  variant uses (the paper states that both bases share them), so BasisCvt
  (Alg. 3) is taken from the tower oracle; a pin checks that the s_i vanish
  on the spans of this Cantor basis.
"""
from __future__ import annotations

from functools import lru_cache

from . import tower

MODULUS = (1 << 128) | 0x87  # x^128 + x^7 + x^2 + x + 1


# --------------------------------------------------------------------------
# The field (Sec. 3.1, the irreducible-polynomial construction)
# --------------------------------------------------------------------------


def clmul(a: int, b: int) -> int:
    """Carry-less product of two GF(2)[x] polynomials held as ints."""
    r = 0
    i = 0
    while b >> i:
        if (b >> i) & 1:
            r ^= a << i
        i += 1
    return r


def reduce(p: int) -> int:
    """p mod x^128 + x^7 + x^2 + x + 1, by long division from the top bit."""
    for e in range(p.bit_length() - 1, 127, -1):
        if (p >> e) & 1:
            p ^= MODULUS << (e - 128)
    return p


def mul(a: int, b: int) -> int:
    """Product in GF(2^128): the polynomial product, then its remainder."""
    return reduce(clmul(a, b))


def power(a: int, e: int) -> int:
    r = 1
    while e:
        if e & 1:
            r = mul(r, a)
        a = mul(a, a)
        e >>= 1
    return r


# --------------------------------------------------------------------------
# The Cantor basis (Sec. 3.3) and the subspace polynomials in it
# --------------------------------------------------------------------------


@lru_cache(maxsize=None)
def _artin_schreier_solver():
    """Row-reduced columns of L(y) = y^2 + y, a GF(2)-linear map on the field.

    L(x^i) for i = 1..127 are independent (the kernel of L is {0, 1}, and
    L(1) = 0), so each reachable c has exactly one preimage with no x^0 term.
    Returns a list of (pivot_bit, image, preimage) with distinct pivots.
    """
    rows = []
    for i in range(1, 128):
        img, pre = mul(1 << i, 1 << i) ^ (1 << i), 1 << i
        for piv, v, p in rows:
            if (img >> piv) & 1:
                img ^= v
                pre ^= p
        if img == 0:
            raise RuntimeError("y^2 + y has a kernel beyond {0, 1}")
        piv = img.bit_length() - 1
        # keep the rows fully reduced on their pivots
        new = []
        for q, v, p in rows:
            if (v >> piv) & 1:
                v ^= img
                p ^= pre
            new.append((q, v, p))
        rows = new + [(piv, img, pre)]
    return tuple(rows)


def solve_artin_schreier(c: int) -> int:
    """The root y of y^2 + y = c whose coefficient of x^0 is zero."""
    y = 0
    for piv, v, p in _artin_schreier_solver():
        if (c >> piv) & 1:
            c ^= v
            y ^= p
    if c:
        raise ValueError("y^2 + y = c has no root in GF(2^128) (trace of c is 1)")
    return y


@lru_cache(maxsize=None)
def cantor_basis(count: int = 64) -> tuple[int, ...]:
    """beta_0 = 1, beta_i^2 + beta_i = beta_{i-1} (Sec. 3.3)."""
    b = [1]
    while len(b) < count:
        b.append(solve_artin_schreier(b[-1]))
    return tuple(b)


def phi(k: int) -> int:
    """phi(k) = sum of beta_j over the set bits j of k (Sec. 3.3)."""
    B = cantor_basis(max(64, k.bit_length()))
    r = 0
    j = 0
    while k >> j:
        if (k >> j) & 1:
            r ^= B[j]
        j += 1
    return r


def s_eval_def(i: int, x: int) -> int:
    """s_i(x) = prod over a in V_i = span(beta_0 .. beta_{i-1}) of (x - a),
    by the definition (Sec. 3.3, Def. of the subspace polynomials)."""
    r = 1
    for k in range(1 << i):
        r = mul(r, x ^ phi(k))
    return r


def s_eval(i: int, x: int) -> int:
    """s_i(x) from its GF(2) coefficients (the same s_i as the tower variant)."""
    r = 0
    for e in tower.s_exponent_set(i):
        r ^= power(x, e)
    return r


def s_cantor(i: int, k: int) -> int:
    """s_i(phi(k)) = phi(k >> i): a multiplier computed in Cantor coordinates
    and mapped into the field (Sec. 3.3, evaluating s_i in the Cantor basis)."""
    return phi(k >> i)


# --------------------------------------------------------------------------
# Alg. 1 with Cantor points, and its inverse
# --------------------------------------------------------------------------


def fft_lch(g: list[int], a: int = 0) -> list[int]:
    """FFT_LCH(g, alpha) with alpha = phi(a): the values of sum g_k X_k at
    alpha + V_m, output j holding the value at phi(a) + phi(j).

    g = p0 + s_k p1 (X_{2^k} = s_k); h0 = p0 + s_k(alpha) p1 and, since
    s_k(beta_k) = 1 in the Cantor basis, h1 = h0 + p1.
    """
    n = len(g)
    if n == 1:
        return [g[0]]
    k = n.bit_length() - 2
    half = n // 2
    p0, p1 = g[:half], g[half:]
    lam = s_cantor(k, a)
    h0 = [p0[t] ^ mul(lam, p1[t]) for t in range(half)]
    h1 = [h0[t] ^ p1[t] for t in range(half)]
    return fft_lch(h0, a) + fft_lch(h1, a ^ (1 << k))


def ifft_lch(vals: list[int], a: int = 0) -> list[int]:
    """The inverse of fft_lch: the butterflies in reverse order."""
    n = len(vals)
    if n == 1:
        return [vals[0]]
    k = n.bit_length() - 2
    half = n // 2
    h0 = ifft_lch(vals[:half], a)
    h1 = ifft_lch(vals[half:], a ^ (1 << k))
    lam = s_cantor(k, a)
    p1 = [h0[t] ^ h1[t] for t in range(half)]
    p0 = [h0[t] ^ mul(lam, p1[t]) for t in range(half)]
    return p0 + p1


def horner(coeffs: list[int], x: int) -> int:
    acc = 0
    for c in reversed(coeffs):
        acc = mul(acc, x) ^ c
    return acc


# --------------------------------------------------------------------------
# Alg. 4 end to end (small inputs only)
# --------------------------------------------------------------------------


def forward_spectrum(a: int, na_bits: int, npoints: int) -> list[int]:
    """Split into 64-bit words, BasisCvt at the operand's own power-of-two
    length, then FFT_LCH at 0 over npoints Cantor points."""
    words = tower.words_of(a, na_bits, 64)
    n1 = tower.next_pow2(len(words))
    g = tower.basis_cvt(words + [0] * (n1 - len(words)))
    return fft_lch(g + [0] * (npoints - n1))


def inverse_to_product(spec: list[int], nc_bits: int) -> int:
    """iFFT_LCH, iBasisCvt, InterleavedCombine: coefficient k (degree < 127)
    is added in at bit 64 k."""
    fc = tower.from_novel(ifft_lch(spec))
    r = 0
    for k, e in enumerate(fc):
        r ^= e << (64 * k)
    return r & ((1 << nc_bits) - 1)


def binpolymul_simple(a: int, na_bits: int, b: int, nb_bits: int) -> int:
    """Alg. 4 binPolyMul for small operands."""
    if na_bits == 0 or nb_bits == 0:
        return 0
    N = tower.fft_size(na_bits, nb_bits, 64)
    fa = forward_spectrum(a, na_bits, N)
    fb = forward_spectrum(b, nb_bits, N)
    return inverse_to_product([mul(x, y) for x, y in zip(fa, fb)], na_bits + nb_bits - 1)


def spectrum_point(words: list[int], j: int) -> int:
    """f(phi(j)) with f(y) = sum_k a_k y^k: one point of the forward
    spectrum, by Horner's rule."""
    return horner(list(words), phi(j))
