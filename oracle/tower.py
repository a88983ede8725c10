"""Stage oracle for the tower-field additive-FFT multiplier -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It shares no code with the GPU library: every function here is
written from the paper's definitions and algorithms (Chen, Cheng, Kuo, Li, Yang,
"Faster Multiplication for Long Binary Polynomials", arXiv:1708.09746), plainly
and slowly, for small inputs.

Conventions
-----------
* Field elements are Python ints.  Bit k of an element is the coefficient of the
  tower basis element v_k (Sec. 3.2, Definition of (v_k)): v_k is the product of
  the generators x_{j+1} over the set bits j of k.  So 0x2 = x_1, 0x4 = x_2,
  0x10 = x_3, 1 << 64 = x_7, and "ī" is simply the integer i.
* TGF(2^W) for W a power of two is the set of ints below 2^W (Sec. 3.2, tower
  construction): TGF(2^W) = TGF(2^{W/2})[X]/(X^2 + X + c_W), X = x_{log2 W},
  c_W = x_1 x_2 ... x_{log2 W - 1}.  An element a = a0 + a1 X keeps a0 in the low
  W/2 bits and a1 in the high W/2 bits.
* Polynomials over a field (or over 64-bit words) are lists of coefficients,
  lowest degree first.  Polynomials over GF(2) are Python ints (bit e is the
  coefficient of x^e).

Readings of the paper taken here (each also listed in the design notes):
* The Kronecker embedding uses theta = x_7 (the element 1 << 64): any element of
  TGF(2^128) outside TGF(2^64) generates the field (Sec. 2.1 allows any
  irreducible polynomial of degree 2w; Sec. 4.3 leaves the isomorphism matrix
  unprinted), and the product does not depend on the choice.
* Word width w = 128 (the TGF(2^256) variant of Alg. 5): theta = x_8 (the
  element 1 << 128), which lies outside TGF(2^128), the only maximal subfield
  of TGF(2^256), and so generates it.
* FFT size: N = max(2, 2^ceil(log2(n_a + n_b - 1))) points for operands of
  n_a and n_b words; each operand is converted at its own power-of-two size.
"""
from __future__ import annotations

from functools import lru_cache

# --------------------------------------------------------------------------
# Tower field arithmetic (Sec. 3.2, the tower construction and Def. of (v_k))
# --------------------------------------------------------------------------


def tower_c(width: int) -> int:
    """c_W = x_1 ... x_{log2 W - 1}, the constant term of X^2 + X + c_W.

    As an element of the half field it is v_{2^{k-1}-1} for W = 2^k (product of
    all generators below X), i.e. the int with only bit W/2 - 1 set.
    """
    k = width.bit_length() - 1
    idx = (1 << (k - 1)) - 1 if k >= 1 else 0
    return 1 << idx


def gf_mul_plain(a: int, b: int, width: int) -> int:
    """Product in TGF(2^width) straight from the defining relations.

    (a0 + a1 X)(b0 + b1 X) = a0 b0 + a1 b1 X^2 + (a0 b1 + a1 b0) X and
    X^2 = X + c_W give  lo = a0 b0 + c_W a1 b1,  hi = a0 b1 + a1 b0 + a1 b1.
    Four sub-products, no Karatsuba: the plain form of the tower product.
    """
    if width == 1:
        return a & b
    h = width // 2
    m = (1 << h) - 1
    a0, a1 = a & m, a >> h
    b0, b1 = b & m, b >> h
    t = gf_mul_plain(a1, b1, h)
    lo = gf_mul_plain(a0, b0, h) ^ gf_mul_plain(tower_c(width), t, h)
    hi = gf_mul_plain(a0, b1, h) ^ gf_mul_plain(a1, b0, h) ^ t
    return lo | (hi << h)


@lru_cache(maxsize=None)
def _gf256_table() -> bytes:
    """Full product table of GF(256) = TGF(2^8): entry 256*a + b = a*b.

    Built with the plain recursion, whose TGF(2^4) level is itself tabulated
    first (both tables are pinned in the tests against gf_mul_plain).
    """
    t16 = [[gf_mul_plain(a, b, 4) for b in range(16)] for a in range(16)]
    out = bytearray(65536)
    c8 = tower_c(8)
    for a in range(256):
        a0, a1 = a & 15, a >> 4
        for b in range(256):
            b0, b1 = b & 15, b >> 4
            t = t16[a1][b1]
            lo = t16[a0][b0] ^ t16[c8][t]
            hi = t16[a0][b1] ^ t16[a1][b0] ^ t
            out[256 * a + b] = lo | (hi << 4)
    return bytes(out)


def gf256_mul(a: int, b: int) -> int:
    return _gf256_table()[256 * a + b]


def _gf16_mul_via256(a: int, b: int) -> int:
    """TGF(2^16) product by the plain relation over the GF(256) table."""
    a0, a1 = a & 255, a >> 8
    b0, b1 = b & 255, b >> 8
    t = gf256_mul(a1, b1)
    lo = gf256_mul(a0, b0) ^ gf256_mul(tower_c(16), t)
    hi = gf256_mul(a0, b1) ^ gf256_mul(a1, b0) ^ t
    return lo | (hi << 8)


@lru_cache(maxsize=None)
def _gf16_tables():
    """log/exp tables of TGF(2^16), built from the plain product.

    Used only to make the plain product fast enough for tests; the tables are
    themselves pinned (tests check that products through the tables equal
    gf_mul_plain on random pairs).
    """
    order = (1 << 16) - 1
    # find a primitive element: its powers must hit all 65535 nonzero values
    for g in range(2, 1 << 16):
        exp = [0] * (2 * order)
        x = 1
        ok = True
        seen = bytearray(1 << 16)
        for e in range(order):
            if seen[x]:
                ok = False
                break
            seen[x] = 1
            exp[e] = x
            x = _gf16_mul_via256(x, g)
        if ok and x == 1:
            for e in range(order, 2 * order):
                exp[e] = exp[e - order]
            log = [0] * (1 << 16)
            for e in range(order):
                log[exp[e]] = e
            return g, exp, log
    raise RuntimeError("no primitive element found")


def gf16_mul(a: int, b: int) -> int:
    if a == 0 or b == 0:
        return 0
    _, exp, log = _gf16_tables()
    return exp[log[a] + log[b]]


def gf_mul(a: int, b: int, width: int = 128) -> int:
    """Product in TGF(2^width): the plain recursion, ending at TGF(2^16)."""
    if width <= 16:
        if width == 16:
            return gf16_mul(a, b)
        return gf_mul_plain(a, b, width)
    h = width // 2
    m = (1 << h) - 1
    a0, a1 = a & m, a >> h
    b0, b1 = b & m, b >> h
    if a1 == 0 and b1 == 0:
        return gf_mul(a0, b0, h)
    if b1 == 0:
        # b in the subfield: Prop. 2, the product is taken component-wise
        return gf_mul(a0, b0, h) | (gf_mul(a1, b0, h) << h)
    if a1 == 0:
        return gf_mul(a0, b0, h) | (gf_mul(a0, b1, h) << h)
    t = gf_mul(a1, b1, h)
    lo = gf_mul(a0, b0, h) ^ gf_mul(tower_c(width), t, h)
    hi = gf_mul(a0, b1, h) ^ gf_mul(a1, b0, h) ^ t
    return lo | (hi << h)


def gf_pow(a: int, e: int, width: int = 128) -> int:
    r = 1
    while e:
        if e & 1:
            r = gf_mul(r, a, width)
        a = gf_mul(a, a, width)
        e >>= 1
    return r


def gf_inv(a: int, width: int) -> int:
    """a^(2^W - 2), the inverse of a nonzero element."""
    return gf_pow(a, (1 << width) - 2, width)


# --------------------------------------------------------------------------
# Subspace vanishing polynomials (Sec. 2.2 Def. of s_i; Sec. 3.2.1, Claim 1)
# --------------------------------------------------------------------------


def span(i: int) -> range:
    """V_i = span(v_0, ..., v_{i-1}): in the tower representation these are
    exactly the ints below 2^i (Sec. 3.2.1)."""
    return range(1 << i)


def s_eval_def(i: int, x: int, width: int = 32) -> int:
    """s_i(x) = prod_{c in V_i} (x - c), by the definition (2^i products)."""
    r = 1
    for c in span(i):
        r = gf_mul(r, x ^ c, width)
        if r == 0:
            return 0
    return r


@lru_cache(maxsize=None)
def s_exponent_set(i: int) -> frozenset:
    """Exponents of s_i as a polynomial over GF(2), kept sparse.

    By the recursivity corollary of Sec. 3.2.1, s_{i+1}(x) = s_i(x)^2 + s_i(x)
    (this uses s_i(v_i) = 1, Prop. 1); s_0(x) = x.  Squaring over GF(2) doubles
    every exponent (Frobenius) and the sum cancels equal terms in pairs.
    """
    if i == 0:
        return frozenset([1])
    prev = s_exponent_set(i - 1)
    return frozenset({2 * e for e in prev} ^ set(prev))


def s_exponents(i: int) -> list[int]:
    """Exponents present in s_i (all powers of two, linearity)."""
    return sorted(s_exponent_set(i))


@lru_cache(maxsize=None)
def s_poly(i: int) -> int:
    """s_i as a dense GF(2)[x] int (bit e = coefficient of x^e); small i only."""
    if i > 24:
        raise ValueError("s_poly is dense; use s_exponent_set for large i")
    r = 0
    for e in s_exponent_set(i):
        r |= 1 << e
    return r


def s_eval(i: int, x: int, width: int = 32) -> int:
    """s_i(x) by the recursivity property s_i = s_1(s_{i-1}): apply
    s_1: y -> y^2 + y to x, i times (Sec. 2.2 properties, Sec. 3.2.1)."""
    for _ in range(i):
        x = gf_mul(x, x, width) ^ x
    return x


# --------------------------------------------------------------------------
# Novel polynomial basis (Sec. 2.3.1, Def. of X_k) and basis conversion
# --------------------------------------------------------------------------


def gf2_polymul(a: int, b: int) -> int:
    """Carry-less product of two GF(2)[x] polynomials held as ints."""
    r = 0
    while b:
        low = b & -b
        r ^= a * low  # a shifted left by the position of the lowest set bit
        b ^= low
    return r


@lru_cache(maxsize=None)
def novel_X(k: int) -> int:
    """X_k(x) = prod over set bits i of k of s_i(x), a GF(2)[x] polynomial."""
    r = 1
    i = 0
    while k >> i:
        if (k >> i) & 1:
            r = gf2_polymul(r, s_poly(i))
        i += 1
    return r


def to_novel_solve(f: list[int]) -> list[int]:
    """BasisCvt by its definition: the unique g with sum_k g_k X_k = f.

    X_k has degree k and leading coefficient 1, so the system is triangular:
    peel off the top coefficient and subtract g_k X_k, from the top down.
    Coefficients are combined with XOR, so this works for field elements and
    for 64-bit words alike (the conversion is GF(2)-linear, coefficient-wise).
    """
    f = list(f)
    n = len(f)
    g = [0] * n
    for k in range(n - 1, -1, -1):
        gk = f[k]
        g[k] = gk
        if gk:
            xk = novel_X(k)
            e = 0
            while xk >> e:
                if (xk >> e) & 1:
                    f[e] ^= gk
                e += 1
    return g


def from_novel(g: list[int]) -> list[int]:
    """Inverse conversion by definition: f = sum_k g_k X_k(x)."""
    n = len(g)
    f = [0] * n
    for k, gk in enumerate(g):
        if gk:
            xk = novel_X(k)
            e = 0
            while xk >> e:
                if (xk >> e) & 1:
                    f[e] ^= gk
                e += 1
    return f


def _deg_bound(f: list[int]) -> int:
    """deg f taken as len(f) - 1 (padded bound; zero top coefficients allowed)."""
    return len(f) - 1


def var_subs(f: list[int], K: int, trace=None, unit: int = 1) -> list[list[int]]:
    """Alg. 2 VarSubs(f, y) with y = x^(2^K) + x.

    Returns h_0, h_1, ... (each a coefficient list of length 2^K) with
    f(x) = sum_t h_t(x) y^t.  Follows the algorithm: if deg f < 2^K return f;
    otherwise take the largest k = 2^j with deg(y^k) = k 2^K <= deg f, divide f
    by y^k = x^(k 2^K) + x^k to get f = f0 + y^k f1, and recurse on both.
    Degrees are the padded bounds len - 1 of power-of-two lengths.
    If `trace` is a list, every division appends (D, k, unit, xor_count), where
    `unit` is the width of the coefficient vectors the caller works on.
    """
    bk = 1 << K
    if _deg_bound(f) < bk:
        return [list(f) + [0] * (bk - len(f))]
    k = 1
    while 2 * k * bk <= _deg_bound(f):
        k *= 2
    D = k * bk  # y^k = x^D + x^k
    # division by x^D + x^k through repeated subtraction, from the top down
    rem = list(f)
    q = [0] * (len(f) - D)
    for t in range(len(f) - 1, D - 1, -1):
        c = rem[t]
        q[t - D] = c
        rem[t] ^= c
        rem[t - D + k] ^= c
    if trace is not None:
        trace.append((D, k, unit, len(f) - D))
    f0 = rem[:D]
    f1 = q
    return var_subs(f0, K, trace, unit) + var_subs(f1, K, trace, unit)


def basis_cvt(f: list[int], trace=None, unit: int = 1) -> list[int]:
    """Alg. 3 BasisCvt: monomial coefficients -> novel-basis coefficients.

    len(f) must be a power of two; deg f is read as len(f) - 1.
    If deg f <= 1 the polynomial is already g_0 + g_1 X_1.  Otherwise pick the
    largest K = 2^i with deg s_K = 2^K <= deg f, substitute y = s_K(x)
    (VarSubs), convert the series in y (its coefficients are polynomials in x of
    degree < 2^K, handled as vectors), then convert every coefficient.
    """
    n = len(f)
    if n <= 2:
        return list(f)
    K = 1
    while (1 << (2 * K)) <= n - 1:
        K *= 2
    h = var_subs(f, K, trace, unit)  # h_t(x), t < n / 2^K
    bk = 1 << K
    # BasisCvt of h(y): coefficients are vectors of 2^K words; the conversion
    # only XORs coefficients, so convert each column of the vectors.
    cols = []
    for r in range(bk):
        cols.append(basis_cvt([h[t][r] for t in range(len(h))], trace, unit * bk))
    q = [[cols[r][t] for r in range(bk)] for t in range(len(h))]
    out = []
    for t in range(len(h)):
        out.extend(basis_cvt(q[t], trace, unit))
    return out


# --------------------------------------------------------------------------
# Evaluation and the LCH FFT (Sec. 2.3.2, Alg. 1)
# --------------------------------------------------------------------------


def horner(coeffs: list[int], x: int, width: int = 128) -> int:
    """f(x) = sum_k c_k x^k in TGF(2^width), by Horner's rule."""
    acc = 0
    for c in reversed(coeffs):
        acc = gf_mul(acc, x, width) ^ c
    return acc


def fft_lch(g: list[int], alpha: int, width: int = 128, trace=None) -> list[int]:
    """Alg. 1 FFT_LCH(g, alpha): the values of f = sum g_k X_k at alpha + V_m.

    Output index j holds f(alpha + j̄).  g = p0 + X_{2^k} p1 with X_{2^k} = s_k;
    h0 = p0 + s_k(alpha) p1, and h1 = h0 + s_k(v_k) p1 = h0 + p1 (Prop. 1).
    If `trace` is a list, each butterfly stage appends (k, alpha, s_k(alpha)).
    """
    n = len(g)
    if n == 1:
        return [g[0]]
    k = n.bit_length() - 2  # largest i with 2^i <= n - 1
    half = n // 2
    p0, p1 = g[:half], g[half:]
    lam = s_eval(k, alpha, width)
    if trace is not None:
        trace.append((k, alpha, lam))
    h0 = [p0[t] ^ gf_mul(lam, p1[t], width) for t in range(half)]
    h1 = [h0[t] ^ p1[t] for t in range(half)]
    vk = 1 << k
    return fft_lch(h0, alpha, width, trace) + fft_lch(h1, alpha ^ vk, width, trace)


def ifft_lch(vals: list[int], alpha: int, width: int = 128) -> list[int]:
    """The inverse of Alg. 1: the butterflies of FFT_LCH run in reverse.

    From the values on alpha + V_{k+1} recover h0 and h1 recursively, then
    p1 = h0 + h1 and p0 = h0 + s_k(alpha) p1.
    """
    n = len(vals)
    if n == 1:
        return [vals[0]]
    k = n.bit_length() - 2
    half = n // 2
    h0 = ifft_lch(vals[:half], alpha, width)
    h1 = ifft_lch(vals[half:], alpha ^ (1 << k), width)
    lam = s_eval(k, alpha, width)
    p1 = [h0[t] ^ h1[t] for t in range(half)]
    p0 = [h0[t] ^ gf_mul(lam, p1[t], width) for t in range(half)]
    return p0 + p1


# --------------------------------------------------------------------------
# Change of representation (Sec. 2.1 Kronecker segmentation; Sec. 4.3)
# --------------------------------------------------------------------------

def theta_of(width: int) -> int:
    """The Kronecker point of TGF(2^width): its top generator x_{log2 width},
    the element 1 << (width / 2) (x_7 for w = 64, x_8 for w = 128)."""
    return 1 << (width // 2)


@lru_cache(maxsize=None)
def theta_powers(width: int = 128) -> tuple[int, ...]:
    th = theta_of(width)
    pw = [1]
    for _ in range(width - 1):
        pw.append(gf_mul(pw[-1], th, width))
    return tuple(pw)


def phi(u: int, width: int = 128) -> int:
    """changeRepr into the tower: the polynomial u(z) (deg < width) at z = theta."""
    pw = theta_powers(width)
    r = 0
    j = 0
    while u >> j:
        if (u >> j) & 1:
            r ^= pw[j]
        j += 1
    return r


@lru_cache(maxsize=None)
def _psi_basis(width: int = 128):
    """Row-reduce the width x width matrix whose column j is theta^j.

    Returns a list of (pivot_bit, element, combination) with echelon elements,
    so that any tower element can be written as a combination of theta^j.
    """
    pw = theta_powers(width)
    basis = []  # (pivot, vector, combo)
    for j, v in enumerate(pw):
        combo = 1 << j
        for piv, bv, bc in basis:
            if (v >> piv) & 1:
                v ^= bv
                combo ^= bc
        if v == 0:
            raise ValueError("theta powers are linearly dependent")
        piv = v.bit_length() - 1
        # keep the basis fully reduced on its pivots
        new = []
        for p2, bv, bc in basis:
            if (bv >> piv) & 1:
                bv ^= v
                bc ^= combo
            new.append((p2, bv, bc))
        new.append((piv, v, combo))
        basis = new
    return basis


def psi(e: int, width: int = 128) -> int:
    """changeRepr back: the polynomial u (deg < width) with u(theta) = e."""
    u = 0
    for piv, bv, bc in _psi_basis(width):
        if (e >> piv) & 1:
            e ^= bv
            u ^= bc
    if e:
        raise ValueError("element not in the span (cannot happen for a basis)")
    return u


# --------------------------------------------------------------------------
# Alg. 5: the tower-field multiplier, end to end (small inputs only)
# --------------------------------------------------------------------------


def words_of(x: int, nbits: int, w: int = 64) -> list[int]:
    """The w-bit words (Split, Alg. 5) of a polynomial of nbits bits."""
    nw = (nbits + w - 1) // w
    x &= (1 << nbits) - 1
    return [(x >> (w * k)) & ((1 << w) - 1) for k in range(nw)]


def int_of(words: list[int], w: int = 64) -> int:
    r = 0
    for k, x in enumerate(words):
        r |= x << (w * k)
    return r


def next_pow2(n: int) -> int:
    p = 1
    while p < n:
        p *= 2
    return p


def fft_size(na_bits: int, nb_bits: int, w: int = 64) -> int:
    na = (na_bits + w - 1) // w
    nb = (nb_bits + w - 1) // w
    return max(2, next_pow2(na + nb - 1))


def forward_spectrum(a: int, na_bits: int, npoints: int, w: int = 64) -> list[int]:
    """Split, BasisCvt (w-bit words), changeRepr, FFT_LCH at 0, per Alg. 5,
    over TGF(2^(2w)).

    The operand is converted at its own power-of-two length n'; the FFT over
    npoints >= n' points is FFT_LCH of the converted polynomial, whose
    coefficients beyond n' are zero.
    """
    words = words_of(a, na_bits, w)
    n1 = next_pow2(len(words))
    words = words + [0] * (n1 - len(words))
    g = basis_cvt(words)
    gt = [phi(x, 2 * w) for x in g] + [0] * (npoints - n1)
    return fft_lch(gt, 0, 2 * w)


def inverse_to_product(spec: list[int], nc_bits: int, w: int = 64) -> int:
    """iFFT_LCH, iBasisCvt, changeRepr back, InterleavedCombine (Alg. 5):
    the preimage of coefficient k (a polynomial of degree < 2w - 1) is added
    in at bit w k."""
    gc = ifft_lch(spec, 0, 2 * w)
    fc = from_novel(gc)
    r = 0
    for k, e in enumerate(fc):
        r ^= psi(e, 2 * w) << (w * k)
    return r & ((1 << nc_bits) - 1)


def binpolymul_tower(a: int, na_bits: int, b: int, nb_bits: int, w: int = 64) -> int:
    """Alg. 5 binPolyMul with w-bit words over TGF(2^(2w)) (w = 64 or 128),
    for small operands."""
    if na_bits == 0 or nb_bits == 0:
        return 0
    N = fft_size(na_bits, nb_bits, w)
    fa = forward_spectrum(a, na_bits, N, w)
    fb = forward_spectrum(b, nb_bits, N, w)
    fc = [gf_mul(x, y, 2 * w) for x, y in zip(fa, fb)]
    return inverse_to_product(fc, na_bits + nb_bits - 1, w)


def spectrum_point(words: list[int], nbits: int, j: int, w: int = 64) -> int:
    """f(j̄) with f(x) = sum_k Φ(a_k) x^k: one point of the forward spectrum,
    by Horner's rule (the definition of the evaluation the FFT computes)."""
    ws = list(words_of(int_of(words, w), nbits, w))
    return horner([phi(x, 2 * w) for x in ws], j, 2 * w)


# --------------------------------------------------------------------------
# Brute force over GF(2)[x]
# --------------------------------------------------------------------------


def clmul_int(a: int, b: int) -> int:
    """Carry-less product of two GF(2)[x] polynomials held as ints (bit loop)."""
    r = 0
    i = 0
    while b >> i:
        if (b >> i) & 1:
            r ^= a << i
        i += 1
    return r
