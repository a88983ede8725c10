"""The simple variant (Alg. 4: polynomial-basis GF(2^128), Cantor points) on
the GPU: spectra against the simple-variant oracle element by element,
products at ragged sizes against the product oracle, the headline size
against its recorded SHA-256, sampled words and the tower method's product,
and the entry points' error paths."""
import hashlib
import os
import random
import sys

import numpy as np
import pytest

import oracle
import oracle.simple as OS
import oracle.tower as OT
import paper_1708_09746_amd as P
from helpers import dev, host
from paper_1708_09746_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "product_sha256.txt")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _int_of(words: np.ndarray, nbits: int) -> int:
    return OT.int_of([int(x) for x in words], 64) & ((1 << nbits) - 1)


def _spec_ints(spec) -> list:
    h = host(spec.reshape(-1)).reshape(-1, 2)
    return [int(lo) | (int(hi) << 64) for lo, hi in h]


# no layers (one-word operands), the bottom pass only (on groups of 8 for an
# 8-word operand), one strided pass above it, and two (N = 2^11; groups of 8
# for the 1024-word operands, whose strided layers fit one pass only then)
@pytest.mark.parametrize("na,log2n", [(1, 0), (1, 1), (64, 3), (64 * 8, 3), (64 * 8, 6), (700, 5), (64 * 16, 4),
                                      (2000, 9), (3000, 10), (64 * 1024, 10), (64 * 1024, 11)])
def test_simple_spectrum_equals_oracle(ctx, na, log2n):
    a = inputs.random_poly(0x5A + na, na)
    say(f"case simple spectrum {na} bits at 2^{log2n} points")
    got = _spec_ints(ctx.simple_forward(dev(a), na, log2n))
    torch.cuda.synchronize()
    if (1 << log2n) <= 512 and na <= 3000:
        want = OS.forward_spectrum(_int_of(a, na), na, 1 << log2n)
        assert got == want
    else:
        words = OT.words_of(_int_of(a, na), na, 64)
        rng = random.Random(na)
        for j in [0, 1, (1 << log2n) - 1] + [rng.randrange(1 << log2n) for _ in range(3)]:
            assert got[j] == OS.spectrum_point(words, j), j


SIZES = [(1, 1), (1, 64), (64, 1), (64, 64), (65, 64), (63, 129), (1000, 999), (64 * 31, 64 * 33), (5000, 70),
         (70, 5000), (4095, 4097), (1, 100000), (64 * 256, 64 * 256 + 1), (100000, 3), (64 * 2047 + 5, 64 * 2049 + 11),
         (320007, 192001), (1 << 20, (1 << 20) - 1)]


@pytest.mark.parametrize("na,nb", SIZES)
def test_simple_products(ctx, na, nb):
    a = inputs.random_poly(0x51A + na % 97, na)
    b = inputs.random_poly(0x51B + nb % 89, nb)
    say(f"case simple product {na}x{nb}")
    got = host(ctx.simple_mul(dev(a), na, dev(b), nb))
    assert np.array_equal(got, oracle.mul(a, na, b, nb)), (na, nb)


def test_simple_equals_tower_random_lengths(ctx):
    rng = random.Random(4)
    for _ in range(12):
        na, nb = rng.randrange(1, 1 << 21), rng.randrange(1, 1 << 21)
        a, b = inputs.random_poly(rng.getrandbits(32), na), inputs.random_poly(rng.getrandbits(32), nb)
        say(f"case simple vs tower {na}x{nb}")
        da, db = dev(a), dev(b)
        x = host(ctx.simple_mul(da, na, db, nb))
        y = host(ctx.mul(da, na, db, nb))
        torch.cuda.synchronize()
        assert np.array_equal(x, y), (na, nb)


def test_simple_squaring_aliases(ctx):
    n = 123457
    a = inputs.random_poly(77, n)
    da = dev(a)
    say("case simple squaring")
    got = host(ctx.simple_mul(da, n, da, n))
    assert np.array_equal(got, oracle.mul(a, n, a, n))


def _golden(name):
    if not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith(name + " "):
                return line.split()
    return None


def test_simple_headline_product(ctx):
    n = 1 << 28
    sa, sb = inputs.SEEDS["c3a"]
    a = inputs.random_poly(sa, n)
    b = inputs.random_poly(sb, n)
    say(f"case simple headline product {n}x{n}")
    got = host(ctx.simple_mul(dev(a), n, dev(b), n))
    torch.cuda.synchronize()
    assert got.size == P.out_words(n, n)
    rng = random.Random(n + 4)
    for k in [0, 1, got.size // 2, got.size - 1] + [rng.randrange(got.size) for _ in range(6)]:
        assert int(got[k]) == oracle.word(a, n, b, n, k), k
    g = _golden("c3a")
    assert g is not None, f"tests/golden/product_sha256.txt has no line for c3a"
    assert hashlib.sha256(got.tobytes()).hexdigest() == g[6]


def test_simple_error_paths(ctx):
    a = dev(inputs.random_poly(1, 640))
    with pytest.raises(P.Gf2xError):
        ctx.simple_mul_into(a, 640, a, 640, a)  # product overlaps an operand
    with pytest.raises(P.Gf2xError):
        ctx.simple_forward(a, 640, 3)  # 10 words need 16 points
    with pytest.raises(P.Gf2xError):
        ctx.simple_forward(a, 640, 33)
    c = torch.zeros(4, dtype=torch.int64, device="cuda")
    ctx.simple_mul_into(a, 0, a, 640, c)  # empty product: nothing written
    torch.cuda.synchronize()
    assert not c.any()
