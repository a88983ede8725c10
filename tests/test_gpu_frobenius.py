"""The Frobenius-partition variant (App. C) on the GPU: value vectors
against the Frobenius oracle element by element (and against Horner's rule
over the bits at sampled points of larger vectors), the inverse against the
oracle's interpolation, products at ragged and configured sizes against the
product oracle, the headline sizes against their recorded SHA-256 and
sampled words, and the entry points' error paths."""
import hashlib
import os
import random
import sys

import numpy as np
import pytest

import oracle
import oracle.frobenius as OF
import oracle.simple as OS
import oracle.tower as OT
import paper_1708_09746_amd as P
from helpers import dev, host, spread_words
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


def _spec_tensor(vals) -> "torch.Tensor":
    raw = np.zeros(2 * len(vals), dtype=np.uint64)
    for j, v in enumerate(vals):
        raw[2 * j] = v & ((1 << 64) - 1)
        raw[2 * j + 1] = v >> 64
    return torch.from_numpy(raw.view(np.int64).copy()).cuda().reshape(-1, 2)


def _value_at(words: np.ndarray, p: int) -> int:
    """a(p) by the definition, word by word: a = sum_k w_k(x) x^(64 k), each
    w_k(p) the sum of p^e over its set bits e, then Horner's rule in p^64."""
    pw = [1]
    for _ in range(64):
        pw.append(OS.mul(pw[-1], p))
    q = pw[64]
    acc = 0
    for w in reversed([int(x) for x in words]):
        v = 0
        e = 0
        while w >> e:
            if (w >> e) & 1:
                v ^= pw[e]
            e += 1
        acc = OS.mul(acc, q) ^ v
    return acc


# n < 64 (the small encoding path), one encoding tile (n = 64 .. 512), the
# operand much shorter than 128 n, and exactly 128 n bits
@pytest.mark.parametrize("na,log2n", [(1, 0), (64, 0), (128, 0), (100, 1), (256, 1), (500, 2), (1024, 3), (700, 4),
                                      (2048, 4), (4096, 5), (8192, 6), (3000, 6), (64 * 200, 7)])
def test_frobenius_values_equal_oracle(ctx, na, log2n):
    a = inputs.random_poly(0xF0 + na, na)
    say(f"case Frobenius values {na} bits at 2^{log2n} points")
    got = _spec_ints(ctx.frobenius_forward(dev(a), na, log2n))
    torch.cuda.synchronize()
    assert got == OF.evaluate(_int_of(a, na), na, log2n)


# several encoding tiles and z-adic passes: sampled points by Horner's rule
@pytest.mark.parametrize("na,log2n", [(9000, 10), (64 * 1024, 10), (70000, 13), ((1 << 20) + 3, 14)])
def test_frobenius_values_sampled(ctx, na, log2n):
    a = inputs.random_poly(0xF1 + na, na)
    say(f"case Frobenius values {na} bits at 2^{log2n} points, sampled")
    got = _spec_ints(ctx.frobenius_forward(dev(a), na, log2n))
    torch.cuda.synchronize()
    rng = random.Random(na)
    for j in [0, 1, (1 << log2n) - 1] + [rng.randrange(1 << log2n) for _ in range(2)]:
        assert got[j] == _value_at(a, OF.point(log2n, j)), j


@pytest.mark.parametrize("nbits,log2n", [(1, 0), (128, 0), (200, 1), (512, 2), (1000, 3), (2048, 4), (8192, 6),
                                         (9000, 7)])
def test_frobenius_inverse_equals_oracle(ctx, nbits, log2n):
    rng = random.Random(nbits * 7 + log2n)
    vals = [rng.getrandbits(128) for _ in range(1 << log2n)]
    total = 128 << log2n
    say(f"case Frobenius inverse of 2^{log2n} random values, {nbits} bits")
    got = host(ctx.frobenius_inverse(_spec_tensor(vals), log2n, nbits))
    torch.cuda.synchronize()
    want = OF.interpolate(vals, log2n, total) & ((1 << nbits) - 1)
    assert _int_of(got, nbits) == want


@pytest.mark.parametrize("na,log2n", [(64 * 4096, 11), ((1 << 20) - 3, 14), (1 << 22, 15)])
def test_frobenius_round_trip(ctx, na, log2n):
    a = inputs.random_poly(0xF2 + na, na)
    say(f"case Frobenius round trip {na} bits at 2^{log2n} points")
    spec = ctx.frobenius_forward(dev(a), na, log2n)
    got = host(ctx.frobenius_inverse(spec, log2n, na))
    torch.cuda.synchronize()
    assert np.array_equal(got, a)  # random_poly clears the bits above na


SIZES = [(1, 1), (1, 64), (64, 1), (64, 64), (65, 64), (63, 129), (128, 1), (129, 1), (100, 29), (1000, 999),
         (64 * 31, 64 * 33), (5000, 70), (70, 5000), (4095, 4097), (4096, 4097), (1, 100000), (64 * 256, 64 * 256 + 1),
         (100000, 3), (64 * 2047 + 5, 64 * 2049 + 11), (320007, 192001), (1 << 20, (1 << 20) - 1),
         ((1 << 21) + 7, 1 << 19)]


@pytest.mark.parametrize("na,nb", SIZES)
def test_frobenius_products(ctx, na, nb):
    a = inputs.random_poly(0xF1A + na % 97, na)
    b = inputs.random_poly(0xF1B + nb % 89, nb)
    say(f"case Frobenius product {na}x{nb}")
    got = host(ctx.frobenius_mul(dev(a), na, dev(b), nb))
    assert np.array_equal(got, oracle.mul(a, na, b, nb, threads=8)), (na, nb)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_frobenius_configured_sizes(ctx, name):
    n = {"c1": 1 << 16, "c2": 1 << 20}[name]
    sa, sb = inputs.SEEDS[name]
    a, b = inputs.random_poly(sa, n), inputs.random_poly(sb, n)
    say(f"case Frobenius {name} {n}x{n}")
    got = host(ctx.frobenius_mul(dev(a), n, dev(b), n))
    assert np.array_equal(got, oracle.mul(a, n, b, n, threads=8))
    g = _golden(name)
    assert g is not None and hashlib.sha256(got.tobytes()).hexdigest() == g[6]


def test_frobenius_equals_tower_random_lengths(ctx):
    rng = random.Random(5)
    for _ in range(12):
        na, nb = rng.randrange(1, 1 << 23), rng.randrange(1, 1 << 23)
        a, b = inputs.random_poly(rng.getrandbits(32), na), inputs.random_poly(rng.getrandbits(32), nb)
        say(f"case Frobenius vs tower {na}x{nb}")
        da, db = dev(a), dev(b)
        x = host(ctx.frobenius_mul(da, na, db, nb))
        y = host(ctx.mul(da, na, db, nb))
        torch.cuda.synchronize()
        assert np.array_equal(x, y), (na, nb)


def test_frobenius_squaring_aliases(ctx):
    n = (1 << 24) + 12345
    a = inputs.random_poly(78, n)
    da = dev(a)
    say("case Frobenius squaring")
    got = host(ctx.frobenius_mul(da, n, da, n))
    assert np.array_equal(got, spread_words(a, n))


def _golden(name):
    if not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith(name + " "):
                return line.split()
    return None


@pytest.mark.parametrize("name", ["c3a", "c3b"])
def test_frobenius_headline_product(ctx, name):
    n = {"c3a": 1 << 28, "c3b": 1 << 29}[name]
    sa, sb = inputs.SEEDS[name]
    a = inputs.random_poly(sa, n)
    b = inputs.random_poly(sb, n)
    say(f"case Frobenius headline product {n}x{n}")
    got = host(ctx.frobenius_mul(dev(a), n, dev(b), n))
    torch.cuda.synchronize()
    assert got.size == P.out_words(n, n)
    rng = random.Random(n + 5)
    for k in [0, 1, got.size // 2, got.size - 1] + [rng.randrange(got.size) for _ in range(6)]:
        assert int(got[k]) == oracle.word(a, n, b, n, k), k
    g = _golden(name)
    assert g is not None, f"tests/golden/product_sha256.txt has no line for {name}"
    assert hashlib.sha256(got.tobytes()).hexdigest() == g[6]


def test_frobenius_error_paths(ctx):
    L = P.lib()
    a = dev(inputs.random_poly(1, 640))
    with pytest.raises(P.Gf2xError):
        ctx.frobenius_mul_into(a, 640, a, 640, a)  # product overlaps an operand
    with pytest.raises(P.Gf2xError):
        ctx.frobenius_forward(a, 640, 2)  # 640 bits need 2^3 points (128 bits each)
    with pytest.raises(P.Gf2xError):
        ctx.frobenius_forward(a, 640, 33)
    spec = torch.zeros((4, 2), dtype=torch.int64, device="cuda")
    with pytest.raises(P.Gf2xError):
        ctx.frobenius_inverse(spec, 2, 513)  # 4 points hold 512 bits
    c = torch.zeros(4, dtype=torch.int64, device="cuda")
    ctx.frobenius_mul_into(a, 0, a, 640, c)  # empty product: nothing written
    torch.cuda.synchronize()
    assert not c.any()
    assert P.frobenius_log2n(1, 1) == 0 and P.frobenius_log2n(128, 1) == 0 and P.frobenius_log2n(129, 1) == 1
    assert P.frobenius_log2n(1 << 28, 1 << 28) == 22 and P.frobenius_log2n(0, 5) == -1
    assert L.gf2x_frobenius_workspace_bytes(1 << 28, 1 << 28) == 2 * (32 << 20) + 2 * (64 << 20)
