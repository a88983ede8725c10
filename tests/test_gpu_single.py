"""Products of at most 2^12 points in one launch when the context asks for it
(a single block runs every stage of Alg. 5 in order): bit-exact against the oracle at ragged sizes up
to the bound, equal to the op-by-op launches, one dispatch per product (the
library's trace), with 128-bit words and with truncated transforms."""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    c.set_single_launch(12)
    yield c
    torch.cuda.synchronize()
    c.close()


# 2^1 .. 2^12 points, ragged tails, unbalanced pairs, the bound itself
SIZES = [(1, 1), (64, 64), (65, 64), (127, 129), (1000, 999), (64 * 31, 64 * 33), (5000, 70), (70, 5000),
         (4095, 4097), (1 << 16, 1 << 16), (1 << 16, (1 << 16) - 3), (64 * 1023 + 5, 64 * 1025 + 11),
         ((1 << 17) - 64, 1 << 17), (1 << 17, 1 << 17), (100000, 3), (3, 100000), (200000, 61000)]


@pytest.mark.parametrize("na,nb", SIZES)
def test_single_launch_products(ctx, na, nb):
    assert P.fft_log2(na, nb) <= 12
    a = inputs.random_poly(0x51C + na % 101, na)
    b = inputs.random_poly(0x51D + nb % 103, nb)
    da, db = dev(a), dev(b)
    say(f"case single launch {na}x{nb}")
    ctx.trace_begin(0x3FF)
    c = torch.full((P.out_words(na, nb),), -1, dtype=torch.int64, device="cuda")
    ctx.mul_into(da, na, db, nb, c)
    recs = ctx.trace_end()
    got = host(c)
    assert [r["kernel"] for r in recs] == ["k_single"], recs
    assert np.array_equal(got, oracle.mul(a, na, b, nb, threads=8)), (na, nb)
    # the same product op by op
    ctx.set_single_launch(-1)
    try:
        c2 = torch.full_like(c, -1)
        ctx.mul_into(da, na, db, nb, c2)
        assert np.array_equal(host(c2), got), (na, nb)
    finally:
        ctx.set_single_launch(12)


def test_single_launch_boundary(ctx):
    """2^12 points take one launch, 2^13 the op-by-op path."""
    for na, m, single in [((1 << 17) + 64, 13, False), (1 << 17, 12, True)]:
        a = inputs.random_poly(0x51E, na)
        da = dev(a)
        assert P.fft_log2(na, na) == m
        ctx.trace_begin(0x3FF)
        c = ctx.mul(da, na, da, na)
        recs = ctx.trace_end()
        assert (["k_single"] == [r["kernel"] for r in recs]) == single, recs
        assert np.array_equal(host(c), oracle.mul(a, na, a, na, threads=8))


def test_single_launch_w128_and_truncated():
    c_ = P.Context(0)
    c_.set_single_launch(12)
    try:
        for setup in ("w128", "trunc"):
            if setup == "w128":
                c_.set_word_bits(128)
            else:
                c_.set_word_bits(64)
                c_.set_truncation(3, 4)
            for na, nb in [(1, 1), (1000, 999), (64 * 31, 64 * 33 + 7), (1 << 16, (1 << 16) - 5), (70000, 9000)]:
                a = inputs.random_poly(0x51F + na, na)
                b = inputs.random_poly(0x520 + nb, nb)
                say(f"case single launch {setup} {na}x{nb}")
                got = host(c_.mul(dev(a), na, dev(b), nb))
                assert np.array_equal(got, oracle.mul(a, na, b, nb, threads=8)), (setup, na, nb)
    finally:
        torch.cuda.synchronize()
        c_.close()


def test_single_launch_setting_errors(ctx):
    with pytest.raises(P.Gf2xError):
        ctx.set_single_launch(13)
    with pytest.raises(P.Gf2xError):
        ctx.set_single_launch(-2)
    ctx.set_single_launch(12)
