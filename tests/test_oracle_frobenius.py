"""Pins for the Frobenius-partition oracle (oracle/frobenius.py, App. C)
against what the paper and the mathematics fix: the values are the
polynomial's values at beta_{m+64} + V_m by Horner's rule over its bits; the
encoding equals the first seven layers of the full FFT_LCH over 128 n points
(the truncated transform of App. C); the map is a bijection (the Frobenius
orbits of the n points are disjoint, of size 128 each, and the encoding
products are independent); interpolation inverts evaluation; products equal
the bitwise product; BasisCvt over bits factors through 64-bit words.
Planted mistakes in the oracle are caught."""
import random

import pytest

import oracle.frobenius as F
import oracle.simple as S
import oracle.tower as T


def _horner_bits(a: int, nbits: int, p: int) -> int:
    acc = 0
    for k in reversed(range(nbits)):
        acc = S.mul(acc, p) ^ ((a >> k) & 1)
    return acc


def check_values_are_evaluations():
    rng = random.Random(11)
    for m in (0, 1, 2):
        nbits = 128 << m
        a = rng.getrandbits(nbits)
        vals = F.evaluate(a, nbits, m)
        for j in range(1 << m):
            assert vals[j] == _horner_bits(a, nbits, F.point(m, j)), (m, j)


def check_encoding_is_the_truncated_fft():
    rng = random.Random(12)
    for m in (0, 1):
        n = 1 << m
        a = rng.getrandbits(128 * n)
        g = T.basis_cvt(F.bits_of(a, 128 * n, 128 * n))
        full = S.fft_lch(g, F.alpha_coord(m))  # all 128 n points of alpha + V_{m+7}
        assert full[:n] == S.fft_lch(F.encode(g, m), F.alpha_coord(m)), m


def check_bijection():
    # the encoding products span GF(2^128) for every m used
    for m in range(0, 25):
        F._decoder(m)
    # the Frobenius orbits of the points are disjoint and of size 128
    for m in (0, 1, 2):
        seen = set()
        for j in range(1 << m):
            p = F.point(m, j)
            orbit = []
            x = p
            for _ in range(128):
                orbit.append(x)
                x = S.mul(x, x)
            assert x == p
            assert len(set(orbit)) == 128, (m, j)
            assert seen.isdisjoint(orbit), (m, j)
            seen.update(orbit)


def check_interpolation_inverts_evaluation():
    rng = random.Random(13)
    for m in (0, 1, 2):
        nbits = 128 << m
        a = rng.getrandbits(nbits)
        assert F.interpolate(F.evaluate(a, nbits, m), m, nbits) == a, m


def check_products():
    rng = random.Random(14)
    for na, nb in [(1, 1), (64, 64), (100, 29), (128, 1), (65, 64), (129, 128), (300, 300), (1000, 37), (700, 800)]:
        a = rng.getrandbits(na) | (1 << (na - 1))
        b = rng.getrandbits(nb) | (1 << (nb - 1))
        assert F.binpolymul_frobenius(a, na, b, nb) == T.clmul_int(a, b), (na, nb)


def _polydivmod(a: int, b: int):
    q = 0
    db = b.bit_length() - 1
    while a and a.bit_length() - 1 >= db:
        sh = a.bit_length() - 1 - db
        q ^= 1 << sh
        a ^= b << sh
    return q, a


def check_bit_basiscvt_factors_through_words():
    """BasisCvt over GF(2) coefficients factors through 64-bit words: with
    z = s_6(x), X_{64q+r}(x) = X_r(x) X_q(z) (s_{6+j} = s_j o s_6), so the
    bit-level conversion is the z-adic expansion a = sum_q H_q(x) z^q
    (deg H_q < 64), then BasisCvt of the word sequence H_q, then the 64-bit
    conversion inside each word."""
    z = T.s_poly(6)
    assert z == (1 << 64) | (1 << 16) | (1 << 4) | (1 << 1)
    rng = random.Random(15)
    for M in (7, 8, 10):
        n = 1 << M
        a = rng.getrandbits(n)
        direct = T.basis_cvt([(a >> k) & 1 for k in range(n)])
        digits, r = [], a
        for _ in range(n // 64):
            r, h = _polydivmod(r, z)
            digits.append(h)
        assert r == 0
        out = []
        for gq in T.basis_cvt(digits):
            out.extend(T.basis_cvt([(gq >> i) & 1 for i in range(64)]))
        assert out == direct, M


CHECKS = [
    check_bit_basiscvt_factors_through_words,
    check_values_are_evaluations,
    check_encoding_is_the_truncated_fft,
    check_bijection,
    check_interpolation_inverts_evaluation,
    check_products,
]


@pytest.mark.parametrize("check", CHECKS, ids=[c.__name__ for c in CHECKS])
def test_pin(check):
    check()


# ---------------------------------------------------- planted mistakes


def _clear():
    F.encoding_products.cache_clear()
    F._decoder.cache_clear()


def _mut_products_reversed(m):
    lam = [S.s_cantor(m + 6 - t, F.alpha_coord(m)) for t in range(7)]  # layers in the wrong order
    out = []
    for j in range(128):
        p = 1
        for t in range(7):
            if (j >> t) & 1:
                p = S.mul(p, lam[t])
        out.append(p)
    return tuple(out)


MUTATIONS = {
    # alpha = beta_{m+63}: for m = 0 it lies in GF(2^64), orbits of size 64
    "alpha_index": ("alpha_coord", lambda m: 1 << (m + 63)),
    "encoding_order": ("encoding_products", _mut_products_reversed),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, value = MUTATIONS[name]
    _clear()
    monkeypatch.setattr(F, attr, value)
    try:
        caught = False
        for c in CHECKS:
            try:
                c()
            except (AssertionError, ValueError, RuntimeError):
                caught = True
                break
        assert caught, name
    finally:
        monkeypatch.undo()
        _clear()
