"""Pins for the stage oracle (oracle/tower.py) against what the paper and the
mathematics fix: field axioms by brute force, the defining relations of the
tower, Props. 1 and 3, Claim 1 (through an explicitly built Cantor basis),
Tab. 1, the multipliers of the Fig. 2 example, the App. B division layers, the
Kronecker property of changeRepr, and Alg. 5 against the bitwise product.

Every check is a plain function so that the planted-mistake test at the end can
re-run them against deliberately broken copies of the oracle."""
import random
from collections import Counter

import pytest

import oracle.tower as T
from conftest import golden_lines

# ----------------------------------------------------------------- checks


def check_small_fields_are_fields():
    for width in (2, 4, 8):
        q = 1 << width
        elems = range(q)
        # GF(256) through its table (the table is pinned to the plain product)
        mul = (lambda a, b: T.gf256_mul(a, b)) if width == 8 else (lambda a, b: T.gf_mul_plain(a, b, width))
        for a in elems:
            # a^(2^W) = a
            x = a
            for _ in range(width):
                x = mul(x, x)
            assert x == a
            if a:
                assert any(mul(a, b) == 1 for b in elems), (width, a)
    # GF(16): commutativity, associativity, distributivity over all triples
    for a in range(16):
        for b in range(16):
            ab = T.gf_mul_plain(a, b, 4)
            assert ab == T.gf_mul_plain(b, a, 4)
            for c in range(16):
                assert T.gf_mul_plain(ab, c, 4) == T.gf_mul_plain(a, T.gf_mul_plain(b, c, 4), 4)
                assert T.gf_mul_plain(a, b ^ c, 4) == ab ^ T.gf_mul_plain(a, c, 4)


def check_large_fields_random_axioms():
    rng = random.Random(3)
    for width in (16, 32, 64, 128):
        for _ in range(30):
            a, b, c = (rng.getrandbits(width) for _ in range(3))
            ab = T.gf_mul(a, b, width)
            assert ab == T.gf_mul(b, a, width)
            assert T.gf_mul(ab, c, width) == T.gf_mul(a, T.gf_mul(b, c, width), width)
            assert T.gf_mul(a, b ^ c, width) == ab ^ T.gf_mul(a, c, width)
            assert T.gf_mul(a, 1, width) == a
        x = rng.getrandbits(width) | 1
        assert T.gf_mul(x, T.gf_inv(x, width), width) == 1


def check_fast_paths_equal_plain():
    rng = random.Random(4)
    tab = T._gf256_table()
    for _ in range(3000):
        a, b = rng.getrandbits(8), rng.getrandbits(8)
        assert tab[256 * a + b] == T.gf_mul_plain(a, b, 8)
    for _ in range(300):
        a, b = rng.getrandbits(16), rng.getrandbits(16)
        assert T.gf16_mul(a, b) == T.gf_mul_plain(a, b, 16)
    for width in (32, 64, 128):
        for _ in range(6):
            a, b = rng.getrandbits(width), rng.getrandbits(width)
            assert T.gf_mul(a, b, width) == T.gf_mul_plain(a, b, width)
            s = rng.getrandbits(width // 4)  # subfield operand (Prop. 2 path)
            assert T.gf_mul(a, s, width) == T.gf_mul_plain(a, s, width)


def check_defining_relations():
    # x_k^2 = x_k + x_1 ... x_{k-1} in TGF(2^{2^k}); x_k is the int 1 << 2^{k-1}
    for k in range(1, 8):
        width = 1 << k
        xk = 1 << (1 << (k - 1))
        prod = 1
        for j in range(1, k):
            prod = T.gf_mul(prod, 1 << (1 << (j - 1)), width)
        assert T.gf_mul(xk, xk, width) == xk ^ prod, k


def check_basis_fixture():
    def gen(j):  # x_j as an int
        return 1 << (1 << (j - 1))

    # v_k = product of x_{j+1} over the set bits j of k, and it is the int 1 << k
    for k in range(128):
        v = 1
        for j in range(7):
            if (k >> j) & 1:
                v = T.gf_mul(v, gen(j + 1), 128)
        assert v == 1 << k, k
    for line in golden_lines("tower_basis.txt"):
        parts = line.split()
        if parts[0] == "element":
            val = int(parts[1], 16)
            assert val == sum(1 << int(p[1:]) for p in parts[3:])
        elif parts[0] == "basis":
            k = int(parts[1][1:])
            v = 1
            for p in parts[3:]:
                v = T.gf_mul(v, gen(int(p[1:])), 128)
            assert v == 1 << k
        elif parts[0] == "subfield":
            small, big = int(parts[1]), int(parts[3])
            wb = big.bit_length() - 1
            for a in range(small):
                for b in range(small):
                    assert T.gf_mul(a, b, wb) < small
        elif parts[0] == "not_cantor":
            i, j = int(parts[1][1:]), int(parts[2][1:])
            vi = 1 << i
            assert T.gf_mul(vi, vi, 128) ^ vi != 1 << j
        else:
            raise AssertionError(line)


def check_prop1_and_prop3():
    # Prop. 1: s_k(v_k) = 1, by the definition for small k and by s_i for more
    for k in range(0, 11):
        assert T.s_eval_def(k, 1 << k, 32) == 1, k
    for k in range(0, 64):
        assert T.s_eval(k, 1 << k, 128) == 1, k
    # Prop. 3: v_i^2 + v_i lies in V_i; base case v_{2^k}^2 + v_{2^k} = v_{2^k - 1}
    for i in range(128):
        vi = 1 << i
        assert (T.gf_mul(vi, vi, 128) ^ vi) < vi or i == 0
    for k in range(7):
        v = 1 << (1 << k)
        assert T.gf_mul(v, v, 128) ^ v == 1 << ((1 << k) - 1)


def check_tab1():
    rng = random.Random(5)
    for line in golden_lines("tab1_si.txt"):
        parts = line.split()
        if parts[0].startswith("s"):
            i = int(parts[0][1:])
            assert sorted(T.s_exponents(i)) == sorted(int(e) for e in parts[1:]), i
        elif parts[0] == "compose":
            ab = int(parts[1][1:])
            a, b = int(parts[3][1:]), int(parts[5][1:])
            assert a + b == ab
            for _ in range(10):
                x = rng.getrandbits(32)
                assert T.s_eval(ab, x, 32) == T.s_eval(a, T.s_eval(b, x, 32), 32)
    # the polynomial form agrees with the product over V_i
    for i in range(0, 9):
        for _ in range(8):
            x = rng.getrandbits(32)
            assert T.s_eval(i, x, 32) == T.s_eval_def(i, x, 32)
    # the sparse exponent form gives the same values as iterating s_1
    for i in range(0, 40):
        x = rng.getrandbits(64)
        val = 0
        for e in T.s_exponents(i):
            val ^= T.gf_pow(x, e, 64)
        assert val == T.s_eval(i, x, 64), i
    # two terms exactly when i is a power of two (Sec. 2.2 properties)
    for i in range(1, 33):
        assert (len(T.s_exponents(i)) == 2) == ((i & (i - 1)) == 0)


def _solve_s1(gamma: int, width: int) -> int:
    """A root x of x^2 + x = gamma in TGF(2^width) by Gaussian elimination
    (s_1 is GF(2)-linear)."""
    cols = [T.gf_mul(1 << j, 1 << j, width) ^ (1 << j) for j in range(width)]
    rows = []  # (pivot, vec, combo)
    for j, v in enumerate(cols):
        combo = 1 << j
        for piv, bv, bc in rows:
            if (v >> piv) & 1:
                v ^= bv
                combo ^= bc
        if v:
            piv = v.bit_length() - 1
            rows = [(p2, bv ^ v if (bv >> piv) & 1 else bv, bc ^ combo if (bv >> piv) & 1 else bc) for p2, bv, bc in rows]
            rows.append((piv, v, combo))
    x = 0
    for piv, bv, bc in rows:
        if (gamma >> piv) & 1:
            gamma ^= bv
            x ^= bc
    assert gamma == 0, "no root"
    return x


def check_claim1_cantor_compatible():
    # Build a Cantor basis beta_0 = 1, beta_i^2 + beta_i = beta_{i-1} in TGF(2^32)
    # and check span(beta_0..beta_{k-1}) = V_k, i.e. beta_i has bit length i + 1.
    width = 32
    beta = [1]
    for i in range(1, width):
        b = _solve_s1(beta[-1], width)
        assert T.gf_mul(b, b, width) ^ b == beta[-1]
        beta.append(b)
    for i, b in enumerate(beta):
        assert b.bit_length() == i + 1, i
    # the vanishing polynomials agree: s_k vanishes on span(beta_0..beta_{k-1})
    rng = random.Random(6)
    for k in range(1, 12):
        for _ in range(5):
            x = 0
            for j in range(k):
                if rng.getrandbits(1):
                    x ^= beta[j]
            assert T.s_eval(k, x, width) == 0


def check_fig2_multipliers():
    # The 16-point FFT of a degree-7 polynomial: record the oracle's butterfly
    # multipliers and compare them, layer by layer, with the example.
    rng = random.Random(9)
    g = [rng.getrandbits(128) for _ in range(8)] + [0] * 8
    trace = []
    T.fft_lch(g, 0, 128, trace)
    by_k = {}
    for k, alpha, lam in trace:
        by_k.setdefault(k, {})[alpha] = lam
    assert set(by_k[3]) == {0}  # layer 1: one block, and p1 = 0: a fan-out
    for line in golden_lines("fig2_multipliers.txt"):
        left, right = line.split(":")
        _, layer, i = left.split()
        alphas_s, mults_s = right.split("->")
        alphas = [int(x, 16) for x in alphas_s.split()]
        mults = [int(x, 16) for x in mults_s.split()]
        i = int(i)
        assert sorted(by_k[i]) == sorted(alphas), layer
        assert [by_k[i][a] for a in alphas] == mults, layer
        assert [T.s_eval(i, a, 32) for a in alphas] == mults


def check_novel_basis_and_basiscvt():
    rng = random.Random(10)
    for k in range(64):
        xk = T.novel_X(k)
        assert xk.bit_length() - 1 == k  # deg X_k = k, monic
    # X_{i 2^K}(x) = X_i(s_K(x)) (the substitution behind Alg. 3)
    for K in (1, 2):
        sK = T.s_poly(K)
        for i in range(1, 8):
            comp = 0
            xi = T.novel_X(i)
            power = 1
            e = 0
            while xi >> e:
                if (xi >> e) & 1:
                    comp ^= power
                power = T.gf2_polymul(power, sK)
                e += 1
            assert comp == T.novel_X(i << K)
    for m in range(0, 9):
        n = 1 << m
        f = [rng.getrandbits(64) for _ in range(n)]
        g = T.basis_cvt(f)
        assert g == T.to_novel_solve(f), m
        assert T.from_novel(g) == f
    trace = []
    T.basis_cvt([rng.getrandbits(64) for _ in range(16)], trace)
    groups = Counter()
    for D, k, unit, nx in trace:
        groups[(D, k, unit)] += nx
    spec = {}
    for line in golden_lines("appB_basiscvt.txt"):
        parts = line.split()
        if parts[0] == "layers":
            assert len(groups) == int(parts[1])
        elif parts[0] == "divisor":
            unit = int(parts[5]) if len(parts) > 4 else 1
            spec[(int(parts[2]), int(parts[3]), unit)] = True
    assert set(groups) == set(spec)
    assert len(set(groups.values())) == 1  # equal XOR counts in every layer


def check_fft_is_evaluation():
    rng = random.Random(11)
    for m in range(0, 6):
        n = 1 << m
        g = [rng.getrandbits(128) for _ in range(n)]
        f = T.from_novel(g)
        for alpha in (0, n, 3 * n, rng.getrandbits(20) << m):
            vals = T.fft_lch(g, alpha)
            assert vals == [T.horner(f, alpha ^ j) for j in range(n)]
            assert T.ifft_lch(vals, alpha) == g


def check_change_of_representation():
    rng = random.Random(12)
    for _ in range(40):
        u = rng.getrandbits(128)
        assert T.psi(T.phi(u)) == u
    for _ in range(60):
        u, v = rng.getrandbits(64), rng.getrandbits(64)
        assert T.psi(T.gf_mul(T.phi(u), T.phi(v), 128)) == T.clmul_int(u, v)
    # additivity
    u, v = rng.getrandbits(128), rng.getrandbits(128)
    assert T.phi(u ^ v) == T.phi(u) ^ T.phi(v)


def check_change_of_representation_w128():
    """w = 128: theta = x_8 in TGF(2^256); the images of two 128-bit blocks
    multiply to the image of their carry-less product (degree < 255)."""
    rng = random.Random(14)
    for _ in range(12):
        u = rng.getrandbits(256)
        assert T.psi(T.phi(u, 256), 256) == u
    for _ in range(12):
        u, v = rng.getrandbits(128), rng.getrandbits(128)
        assert T.psi(T.gf_mul(T.phi(u, 256), T.phi(v, 256), 256), 256) == T.clmul_int(u, v)
    u, v = rng.getrandbits(256), rng.getrandbits(256)
    assert T.phi(u ^ v, 256) == T.phi(u, 256) ^ T.phi(v, 256)
    # the fast product at width 256 (Karatsuba with the subfield shortcuts)
    # against the plain defining relations
    for _ in range(4):
        x, y = rng.getrandbits(256), rng.getrandbits(256)
        assert T.gf_mul(x, y, 256) == T.gf_mul_plain(x, y, 256)
    # a subfield scalar (Prop. 2: component-wise) against the plain relations
    x, y = rng.getrandbits(256), rng.getrandbits(20)
    assert T.gf_mul(x, y, 256) == T.gf_mul_plain(x, y, 256)


def check_alg5_end_to_end_w128():
    """Alg. 5 with 128-bit words over TGF(2^256) against the schoolbook
    carry-less product, at sizes around the word and power-of-two edges."""
    rng = random.Random(15)
    sizes = [(1, 1), (1, 128), (128, 1), (128, 128), (129, 128), (127, 257), (256, 256), (257, 600),
             (600, 9), (1000, 1000)]
    for na, nb in sizes:
        a = rng.getrandbits(na) | (1 << (na - 1))
        b = rng.getrandbits(nb) | (1 << (nb - 1))
        assert T.binpolymul_tower(a, na, b, nb, 128) == T.clmul_int(a, b), (na, nb)
    # the spectrum is the evaluation of sum_k phi(a_k) x^k over TGF(2^256)
    na = 700
    a = rng.getrandbits(na)
    words = T.words_of(a, na, 128)
    spec = T.forward_spectrum(a, na, 16, 128)
    for j in (0, 1, 6, 15):
        assert spec[j] == T.spectrum_point(words, na, j, 128)


def check_alg5_end_to_end():
    rng = random.Random(13)
    sizes = [(1, 1), (1, 64), (64, 1), (64, 64), (65, 64), (63, 129), (128, 128), (129, 500), (300, 7), (500, 500)]
    for na, nb in sizes:
        a = rng.getrandbits(na) | (1 << (na - 1))
        b = rng.getrandbits(nb) | (1 << (nb - 1))
        assert T.binpolymul_tower(a, na, b, nb) == T.clmul_int(a, b), (na, nb)
    # the spectrum is the evaluation of sum_k phi(a_k) x^k
    na = 300
    a = rng.getrandbits(na)
    words = T.words_of(a, na)
    spec = T.forward_spectrum(a, na, 16)
    for j in (0, 1, 5, 15):
        assert spec[j] == T.spectrum_point(words, na, j)


CHECKS = [
    check_small_fields_are_fields,
    check_large_fields_random_axioms,
    check_fast_paths_equal_plain,
    check_defining_relations,
    check_basis_fixture,
    check_prop1_and_prop3,
    check_tab1,
    check_claim1_cantor_compatible,
    check_fig2_multipliers,
    check_novel_basis_and_basiscvt,
    check_fft_is_evaluation,
    check_change_of_representation,
    check_alg5_end_to_end,
    check_change_of_representation_w128,
    check_alg5_end_to_end_w128,
]


@pytest.mark.parametrize("check", CHECKS, ids=[c.__name__ for c in CHECKS])
def test_pin(check):
    check()


# ---------------------------------------------------- planted mistakes

_CACHED = ["s_exponent_set", "s_poly", "novel_X", "_gf256_table", "_gf16_tables", "theta_powers", "_psi_basis"]


def _clear_caches():
    for name in _CACHED:
        getattr(T, name).cache_clear()


def _some_check_fails(checks):
    for c in checks:
        try:
            c()
        except (AssertionError, ValueError, IndexError, KeyError, RuntimeError):
            return True
    return False


def _mut_tower_constant(width):
    return 1  # dropped the x_1 ... x_{k-1} factor


def _mut_gf_mul_plain_hi(a, b, width):
    if width == 1:
        return a & b
    h = width // 2
    m = (1 << h) - 1
    a0, a1, b0, b1 = a & m, a >> h, b & m, b >> h
    t = _mut_gf_mul_plain_hi(a1, b1, h)
    lo = _mut_gf_mul_plain_hi(a0, b0, h) ^ _mut_gf_mul_plain_hi(T.tower_c(width), t, h)
    hi = _mut_gf_mul_plain_hi(a0, b1, h) ^ _mut_gf_mul_plain_hi(a1, b0, h)  # dropped a1 b1
    return lo | (hi << h)


def _mut_s_eval(i, x, width=32):
    # s_i applied as i squarings (dropped the "+ y" of s_1: y -> y^2 + y)
    for _ in range(i):
        x = T.gf_mul(x, x, width)
    return x


MUTATIONS = {
    "tower_constant": ("tower_c", _mut_tower_constant),
    "dropped_hi_term": ("gf_mul_plain", _mut_gf_mul_plain_hi),
    "s_recursion": ("s_eval", _mut_s_eval),
    "theta_in_subfield": ("theta_of", lambda width: 1 << (width // 2 - 1)),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, value = MUTATIONS[name]
    fast = [check_defining_relations, check_basis_fixture, check_tab1, check_fig2_multipliers,
            check_prop1_and_prop3, check_change_of_representation, check_fast_paths_equal_plain,
            check_change_of_representation_w128]
    _clear_caches()
    monkeypatch.setattr(T, attr, value)
    try:
        assert _some_check_fails(fast), name
    finally:
        monkeypatch.undo()
        _clear_caches()
