"""Pins for the product oracle (oracle/gf2x_oracle.c) against facts that do not
come from the oracle itself: bitwise brute force on tiny inputs, closed forms
(a*1, a*x^k, a*(1+x^k), a*a), ring invariants, and the two clmul variants."""
import random

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from oracle.tower import clmul_int
from paper_1708_09746_amd import inputs


def to_int(words) -> int:
    return int.from_bytes(np.ascontiguousarray(words, dtype=np.uint64).tobytes(), "little")


def to_words(x: int, nbits: int) -> np.ndarray:
    nw = (nbits + 63) // 64
    return np.frombuffer(x.to_bytes(8 * nw, "little"), dtype=np.uint64).copy()


def brute_bits(a: int, b: int) -> int:
    """c_k = XOR over i + j = k of a_i AND b_j, coefficient by coefficient."""
    la, lb = a.bit_length(), b.bit_length()
    c = 0
    for k in range(la + lb):
        bit = 0
        for i in range(max(0, k - lb + 1), min(k, la - 1) + 1):
            bit ^= ((a >> i) & 1) & ((b >> (k - i)) & 1)
        c |= bit << k
    return c


def spread(x: int) -> int:
    """Bit i of x moved to bit 2i: the square of x over GF(2)."""
    r = 0
    i = 0
    while x:
        if x & 1:
            r |= 1 << (2 * i)
        x >>= 1
        i += 1
    return r


def test_clmul64_variants_agree_and_match_brute_force():
    rng = random.Random(7)
    edge = [0, 1, 2, 3, (1 << 64) - 1, 1 << 63, 0x8000000000000001, 0x5555555555555555]
    pairs = [(x, y) for x in edge for y in edge] + [(rng.getrandbits(64), rng.getrandbits(64)) for _ in range(300)]
    for x, y in pairs:
        bl = oracle.clmul64(x, y, "bitloop")
        wn = oracle.clmul64(x, y, "window")
        assert bl == wn
        assert bl == clmul_int(x, y)
    for x, y in pairs[:60]:
        assert oracle.clmul64(x, y) == brute_bits(x, y)


def test_clmul_int_is_the_bitwise_definition():
    rng = random.Random(8)
    for _ in range(50):
        a = rng.getrandbits(rng.randint(1, 120))
        b = rng.getrandbits(rng.randint(1, 120))
        assert clmul_int(a, b) == brute_bits(a, b)


@pytest.mark.parametrize("na,nb", [(1, 1), (1, 64), (64, 1), (63, 65), (64, 64), (65, 64), (100, 300),
                                   (511, 512), (512, 512), (129, 1), (200, 7)])
def test_tiny_products_against_bitwise_brute_force(na, nb):
    a = inputs.random_poly(1000 + na, na)
    b = inputs.random_poly(2000 + nb, nb)
    c = oracle.mul(a, na, b, nb)
    assert len(c) == (na + nb - 1 + 63) // 64
    assert to_int(c) == brute_bits(to_int(a), to_int(b))


def test_high_garbage_bits_are_ignored():
    na, nb = 70, 33
    a = inputs.random_poly(5, na)
    b = inputs.random_poly(6, nb)
    ag = a.copy()
    bg = b.copy()
    ag[-1] |= np.uint64(0xFFFFFFFFFFFFFFC0)  # bits >= 70 set
    bg[-1] |= np.uint64(0xFFFFFFFE00000000)  # bits >= 33 set
    assert np.array_equal(oracle.mul(ag, na, bg, nb), oracle.mul(a, na, b, nb))


def test_empty_operands_give_empty_product():
    a = inputs.random_poly(1, 100)
    assert oracle.out_words(0, 100) == 0
    assert oracle.mul(a, 0, a, 100).size == 0
    assert oracle.mul(a, 100, a, 0).size == 0


@pytest.mark.parametrize("n", [1, 7, 12, 13, 25, 40, 97, 300, 1000])
def test_karatsuba_against_schoolbook(n):
    rng = np.random.default_rng(n)
    a = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    b = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    s = oracle.mul_schoolbook(a, b)
    k = oracle.mul(a, 64 * n, b, 64 * n)
    assert np.array_equal(s[: len(k)], k)
    assert not s[len(k):].any()


@pytest.mark.parametrize("na,nb", [(3000, 17), (17, 3000), (2000, 1999), (64 * 123, 64 * 7 + 5)])
def test_unbalanced_products_against_python(na, nb):
    a = inputs.random_poly(11, na)
    b = inputs.random_poly(12, nb)
    assert to_int(oracle.mul(a, na, b, nb)) == clmul_int(to_int(a), to_int(b))


def test_threads_do_not_change_the_result():
    n = 64 * 5000 + 3
    a = inputs.random_poly(21, n)
    b = inputs.random_poly(22, n)
    c1 = oracle.mul(a, n, b, n, threads=1)
    c8 = oracle.mul(a, n, b, n, threads=8)
    assert np.array_equal(c1, c8)


def test_closed_forms_at_2_16_bits():
    n = 1 << 16
    a = inputs.random_poly(0x16A, n)
    ai = to_int(a)
    one = np.array([1], dtype=np.uint64)
    # a * 1 = a
    assert to_int(oracle.mul(a, n, one, 1)) == ai
    # a * x^k = a << k
    for k in (1, 63, 64, 65, 1000):
        xk = to_words(1 << k, k + 1)
        assert to_int(oracle.mul(a, n, xk, k + 1)) == ai << k
        # a * (1 + x^k) = a + (a << k)
        xk1 = to_words((1 << k) | 1, k + 1)
        assert to_int(oracle.mul(a, n, xk1, k + 1)) == ai ^ (ai << k)
    # a * a = bit-spread(a) (the Frobenius map)
    assert to_int(oracle.mul(a, n, a, n)) == spread(ai)


def test_sparse_operand_gives_xor_of_shifts():
    n = 5000
    a = inputs.random_poly(3, n)
    ai = to_int(a)
    ks = [0, 5, 64, 200, 777]
    b = 0
    for k in ks:
        b |= 1 << k
    c = oracle.mul(a, n, to_words(b, 778), 778)
    expect = 0
    for k in ks:
        expect ^= ai << k
    assert to_int(c) == expect


@settings(max_examples=40, deadline=None)
@given(st.integers(1, 700), st.integers(1, 700), st.integers(1, 700), st.integers(0, 2**32))
def test_ring_invariants(na, nb, nc, seed):
    a = inputs.random_poly(seed, na)
    b = inputs.random_poly(seed + 1, nb)
    c = inputs.random_poly(seed + 2, nc)
    ab = to_int(oracle.mul(a, na, b, nb))
    # deg(ab) = deg a + deg b  (top bits forced to 1)
    assert ab.bit_length() - 1 == (na - 1) + (nb - 1)
    # commutativity
    assert to_int(oracle.mul(b, nb, a, na)) == ab
    # distributivity: a(b + c) = ab + ac
    m = max(nb, nc)
    bc = to_words(to_int(b) ^ to_int(c), m)
    lhs = to_int(oracle.mul(a, na, bc, m))
    rhs = ab ^ to_int(oracle.mul(a, na, c, nc))
    assert lhs == rhs
    # Frobenius: (a + b)^2 = a^2 + b^2
    m2 = max(na, nb)
    s = to_words(to_int(a) ^ to_int(b), m2)
    assert to_int(oracle.mul(s, m2, s, m2)) == to_int(oracle.mul(a, na, a, na)) ^ to_int(oracle.mul(b, nb, b, nb))


@pytest.mark.parametrize("na,nb", [(1, 1), (64, 64), (100, 1000), (4096, 4096), (3001, 77)])
def test_single_output_words_match_full_product(na, nb):
    a = inputs.random_poly(31, na)
    b = inputs.random_poly(32, nb)
    c = oracle.mul(a, na, b, nb)
    for k in range(len(c)):
        assert oracle.word(a, na, b, nb, k) == int(c[k])
    assert oracle.word(a, na, b, nb, len(c)) == 0


def test_residues_mod_x64_plus_q():
    rng = random.Random(41)
    for _ in range(20):
        q = rng.getrandbits(64)
        nbits = rng.randint(1, 3000)
        x = rng.getrandbits(nbits)
        Q = (1 << 64) | q
        # Python long division over GF(2)
        r = x
        while r.bit_length() > 64:
            r ^= Q << (r.bit_length() - 65)
        assert oracle.mod(to_words(x, nbits), nbits, q) == r
    # (a mod Q)(b mod Q) = ab mod Q
    na = nb = 5000
    a = inputs.random_poly(51, na)
    b = inputs.random_poly(52, nb)
    c = oracle.mul(a, na, b, nb)
    for _ in range(5):
        q = rng.getrandbits(64)
        lhs = oracle.mulmod(oracle.mod(a, na, q), oracle.mod(b, nb, q), q)
        assert lhs == oracle.mod(c, na + nb - 1, q)
