"""BasisCvt sub-conversions run inside FFT passes (gf2x_set_fusion): for every
mask (0: none, also for the small products the default fuses) at every
size, products at ragged sizes of one and several FFT passes bit-exact
against the oracle, with 128-bit words too, a batch staged and persistent
against the oracle job by job, the 2^28-bit product against its recorded
SHA-256, and the setting's error paths."""
import hashlib
import os
import random
import sys

import numpy as np
import pytest

import oracle
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


# one pass (2^1 .. 2^12 points), a bottom pass and one or two strided passes,
# unbalanced operands
SIZES = [(1, 1), (65, 64), (1000, 999), (64 * 33, 64 * 31), (5000, 70), (1 << 16, 1 << 16), (100000, 3),
         (64 * 2047 + 5, 64 * 2049 + 11), (1 << 20, 1 << 20), ((1 << 21) + 7, 1 << 19), ((1 << 22) - 9, 1 << 22)]


@pytest.mark.parametrize("mask", [0, 1, 2, 4, 6, 7])
def test_fused_products(ctx, mask):
    ctx.set_fusion(mask, 32, 32)
    try:
        for na, nb in SIZES:
            a = inputs.random_poly(0xF5 + na % 97, na)
            b = inputs.random_poly(0xF6 + nb % 89, nb)
            say(f"case fusion mask {mask}: product {na}x{nb}")
            c = torch.full((P.out_words(na, nb),), -1, dtype=torch.int64, device="cuda")
            ctx.mul_into(dev(a), na, dev(b), nb, c)
            assert np.array_equal(host(c), oracle.mul(a, na, b, nb, threads=8)), (mask, na, nb)
    finally:
        ctx.set_fusion(7, 13, 11)  # the default


@pytest.mark.parametrize("mask", [3, 7])
def test_fused_products_128(ctx, mask):
    ctx.set_fusion(mask, 32, 32)
    ctx.set_word_bits(128)
    try:
        for na, nb in [(129, 128), (1000, 999), (1 << 16, 1 << 16), (100000, 3), ((1 << 20) + 3, 1 << 19)]:
            a = inputs.random_poly(0xF7 + na % 97, na)
            b = inputs.random_poly(0xF8 + nb % 89, nb)
            say(f"case fusion mask {mask}, 128-bit words: product {na}x{nb}")
            c = torch.full((P.out_words(na, nb),), -1, dtype=torch.int64, device="cuda")
            ctx.mul_into(dev(a), na, dev(b), nb, c)
            assert np.array_equal(host(c), oracle.mul(a, na, b, nb, threads=8)), (mask, na, nb)
    finally:
        ctx.set_word_bits(64)
        ctx.set_fusion(7, 13, 11)  # the default


@pytest.mark.parametrize("persistent", [False, True])
def test_fused_batch(ctx, persistent):
    ctx.set_fusion(7, 32, 32)
    try:
        rng = random.Random(77)
        jobs, want = [], []
        for _ in range(48):
            na, nb = rng.randrange(1, 1 << 18), rng.randrange(1, 1 << 18)
            a = inputs.random_poly(rng.getrandbits(32), na)
            b = inputs.random_poly(rng.getrandbits(32), nb)
            jobs.append((dev(a), na, dev(b), nb,
                         torch.full((P.out_words(na, nb),), -1, dtype=torch.int64, device="cuda")))
            want.append(oracle.mul(a, na, b, nb, threads=8))
        say(f"case fusion batch of 48 jobs, persistent={persistent}")
        B = ctx.batch(jobs, persistent=persistent)
        try:
            B.run()
            B.check()
            torch.cuda.synchronize()
        finally:
            B.close()
        for k, (j, w) in enumerate(zip(jobs, want)):
            assert np.array_equal(host(j[4]), w), k
    finally:
        ctx.set_fusion(7, 13, 11)  # the default


def test_fused_headline_product(ctx):
    n = 1 << 28
    sa, sb = inputs.SEEDS["c3a"]
    a, b = inputs.random_poly(sa, n), inputs.random_poly(sb, n)
    with open(GOLDEN) as f:
        g = [line.split() for line in f if line.startswith("c3a ")]
    assert g, "tests/golden/product_sha256.txt has no line for c3a"
    ctx.set_fusion(7, 32, 32)
    try:
        say("case fusion mask 7: 2^28 x 2^28-bit product")
        c = torch.empty(P.out_words(n, n), dtype=torch.int64, device="cuda")
        ctx.mul_into(dev(a), n, dev(b), n, c)
        got = host(c)
    finally:
        ctx.set_fusion(7, 13, 11)  # the default
    assert hashlib.sha256(got.tobytes()).hexdigest() == g[0][6]


def test_fusion_setting_errors(ctx):
    with pytest.raises(P.Gf2xError):
        ctx.set_fusion(8, 20, 20)
    with pytest.raises(P.Gf2xError):
        ctx.set_fusion(-1, 20, 20)
    with pytest.raises(P.Gf2xError):
        ctx.set_fusion(1, 33, 11)
    with pytest.raises(P.Gf2xError):
        ctx.set_fusion(1, 13, 33)
    ctx.set_fusion(7, 13, 11)  # the default
