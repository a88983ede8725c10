"""Pins for the simple-variant oracle (oracle/simple.py, Alg. 4) against what
the paper and the mathematics fix: the modulus is irreducible (Rabin's test),
field axioms and closed-form products, the defining relation of the Cantor
basis and the subfields its prefixes span, the subspace polynomials by their
definition and the shift rule s_i(phi(k)) = phi(k >> i), the FFT against
Horner evaluation at the Cantor points, and Alg. 4 against the bitwise product.

Each check is a plain function so that the planted-mistake test at the end can
re-run them against deliberately broken copies of the oracle."""
import random

import pytest

import oracle.simple as S
import oracle.tower as T

# ---------------------------------------------------------- GF(2)[x] helpers


def _polymod(a: int, m: int) -> int:
    dm = m.bit_length() - 1
    while a and a.bit_length() - 1 >= dm:
        a ^= m << (a.bit_length() - 1 - dm)
    return a


def _polygcd(a: int, b: int) -> int:
    while b:
        a, b = b, _polymod(a, b)
    return a


def _rank(vectors) -> int:
    rows = []
    for v in vectors:
        for r in rows:
            v = min(v, v ^ r)
        if v:
            rows.append(v)
    return len(rows)


# ----------------------------------------------------------------- checks


def check_modulus_irreducible():
    """Rabin's test for degree 128 = 2^7: x^(2^128) = x mod P, and
    gcd(x^(2^64) - x, P) = 1 (64 is the only maximal proper divisor)."""
    x = 2
    y = x
    frob = {}
    for k in range(1, 129):
        y = S.mul(y, y)
        frob[k] = y
    assert frob[128] == x
    assert _polygcd(S.MODULUS, frob[64] ^ x) == 1
    # the degree of the modulus and its terms
    assert S.MODULUS == (1 << 128) | (1 << 7) | (1 << 2) | (1 << 1) | 1


def check_field_axioms_and_closed_forms():
    rng = random.Random(4)
    for _ in range(40):
        a, b, c = (rng.getrandbits(128) for _ in range(3))
        assert S.mul(a, b) == S.mul(b, a)
        assert S.mul(S.mul(a, b), c) == S.mul(a, S.mul(b, c))
        assert S.mul(a, b ^ c) == S.mul(a, b) ^ S.mul(a, c)
        assert S.mul(a, 1) == a
    for _ in range(3):
        a = rng.getrandbits(128) | 1
        assert S.mul(a, S.power(a, (1 << 128) - 2)) == 1  # Fermat inverse
    # x^64 x^64 = x^128 = x^7 + x^2 + x + 1; x^127 x = x^128
    assert S.mul(1 << 64, 1 << 64) == 0x87
    assert S.mul(1 << 127, 2) == 0x87
    # x^254 = x^126 (x^7 + x^2 + x + 1), folded once more by hand
    want = (1 << 127) | (1 << 126) | (1 << 12) | (1 << 6) | (1 << 5) | (1 << 2) | (1 << 1) | 1
    assert S.mul(1 << 127, 1 << 127) == want
    # two words of degree < 64 multiply with no reduction (Split needs none)
    for _ in range(20):
        u, v = rng.getrandbits(64), rng.getrandbits(64)
        assert S.mul(u, v) == T.clmul_int(u, v)


def check_cantor_basis():
    B = S.cantor_basis(128)
    assert B[0] == 1
    for i in range(1, 128):
        assert S.mul(B[i], B[i]) ^ B[i] == B[i - 1], i
        assert B[i] & 1 == 0, i  # the reading: the root with no x^0 term
    assert _rank(B) == 128
    # beta_0 .. beta_{2^k - 1} span GF(2^(2^k)); beta_{2^k} lies outside it
    for k in range(7):
        q = 1 << k
        for j in list(range(q)) + ([q] if q < 128 else []):
            z = B[j]
            for _ in range(q):
                z = S.mul(z, z)
            assert (z == B[j]) == (j < q), (k, j)


def check_subspace_polynomials():
    rng = random.Random(5)
    for i in range(5):
        for _ in range(3):
            x = rng.getrandbits(128)
            assert S.s_eval_def(i, x) == S.s_eval(i, x), i
        for j in range(40):
            assert S.s_eval_def(i, S.phi(j)) == S.phi(j >> i), (i, j)
    # s_i vanishes on V_i and takes the value 1 at beta_i
    for i in range(1, 5):
        for j in range(1 << i):
            assert S.s_eval_def(i, S.phi(j)) == 0
    for i in range(12):
        assert S.s_eval(i, S.cantor_basis(64)[i]) == 1, i
        for _ in range(3):
            k = rng.getrandbits(24)
            assert S.s_eval(i, S.phi(k)) == S.phi(k >> i) == S.s_cantor(i, k), (i, k)


def check_fft_is_evaluation():
    rng = random.Random(6)
    for n, npts in ((16, 16), (8, 32), (32, 32)):
        f = [rng.getrandbits(64) for _ in range(n)]
        g = T.basis_cvt(f)
        vals = S.fft_lch(g + [0] * (npts - n))
        for j in range(npts):
            assert vals[j] == S.horner(f, S.phi(j)), (n, npts, j)
    # a shifted coset alpha + V_m, alpha = phi(a)
    f = [rng.getrandbits(128) for _ in range(16)]
    g = T.basis_cvt(f)
    a = 0x5A30
    vals = S.fft_lch(g, a)
    for j in (0, 1, 7, 15):
        assert vals[j] == S.horner(f, S.phi(a ^ j))


def check_ifft_inverts():
    rng = random.Random(7)
    for n in (2, 4, 32):
        g = [rng.getrandbits(128) for _ in range(n)]
        assert S.ifft_lch(S.fft_lch(g)) == g
        assert S.ifft_lch(S.fft_lch(g, 0x340), 0x340) == g


def check_alg4_end_to_end():
    rng = random.Random(8)
    sizes = [(1, 1), (1, 64), (64, 1), (64, 64), (65, 64), (63, 129), (128, 128), (129, 500), (300, 7), (500, 500),
             (1000, 1)]
    for na, nb in sizes:
        a = rng.getrandbits(na) | (1 << (na - 1))
        b = rng.getrandbits(nb) | (1 << (nb - 1))
        assert S.binpolymul_simple(a, na, b, nb) == T.clmul_int(a, b), (na, nb)
    na = 700
    a = rng.getrandbits(na)
    words = T.words_of(a, na)
    spec = S.forward_spectrum(a, na, 32)
    for j in (0, 1, 9, 31):
        assert spec[j] == S.spectrum_point(words, j)


CHECKS = [
    check_modulus_irreducible,
    check_field_axioms_and_closed_forms,
    check_cantor_basis,
    check_subspace_polynomials,
    check_fft_is_evaluation,
    check_ifft_inverts,
    check_alg4_end_to_end,
]


@pytest.mark.parametrize("check", CHECKS, ids=[c.__name__ for c in CHECKS])
def test_pin(check):
    check()


# ---------------------------------------------------- planted mistakes


def _clear_caches():
    S._artin_schreier_solver.cache_clear()
    S.cantor_basis.cache_clear()
    T.s_exponent_set.cache_clear()


def _mut_fft_h1(g, a=0):
    # h1 = h0: the s_k(beta_k) p1 term dropped
    n = len(g)
    if n == 1:
        return [g[0]]
    k = n.bit_length() - 2
    half = n // 2
    lam = S.s_cantor(k, a)
    h0 = [g[t] ^ S.mul(lam, g[half + t]) for t in range(half)]
    return _mut_fft_h1(h0, a) + _mut_fft_h1(list(h0), a ^ (1 << k))


def _mut_cantor_sqrt(count=64):
    # beta_i^2 = beta_{i-1} (the "+ beta_i" of the relation dropped)
    b = [1, 1 << 64]
    while len(b) < count:
        b.append(S.power(b[-1], 1 << 127))
    return tuple(b)


MUTATIONS = {
    "modulus_term": ("MODULUS", (1 << 128) | 0x83),
    "multiplier_shift": ("s_cantor", lambda i, k: S.phi(k >> (i + 1))),
    "fft_h1": ("fft_lch", _mut_fft_h1),
    "cantor_relation": ("cantor_basis", _mut_cantor_sqrt),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, value = MUTATIONS[name]
    _clear_caches()
    monkeypatch.setattr(S, attr, value)
    try:
        caught = False
        for c in CHECKS:
            try:
                c()
            except (AssertionError, ValueError, IndexError, RuntimeError):
                caught = True
                break
        assert caught, name
    finally:
        monkeypatch.undo()
        _clear_caches()
