"""Split into 128-bit words (Alg. 5 with w = 128, TGF(2^256)) on the GPU:
products at ragged sizes against the oracle, the headline size against its
recorded SHA-256 and sampled words, products equal to the w = 64 path's,
batches (staged and persistent) and the serving engine in w = 128, and the
word-width setting's error paths."""
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
    c.set_word_bits(128)
    yield c
    torch.cuda.synchronize()
    c.close()


def words128(bits):
    return (bits + 127) // 128


# around the 128-bit word and power-of-two edges, one-word and unbalanced
SIZES = [(1, 1), (1, 128), (128, 1), (64, 64), (127, 129), (128, 128), (129, 128), (256, 256), (257, 255),
         (300, 7), (1000, 999), (128 * 31, 128 * 33), (5000, 70), (70, 5000), (4095, 4097),
         (128 * 1024, 128 * 1024 + 1), (100000, 3), (128 * 2047 + 5, 128 * 2049 + 11), (320007, 192001)]


@pytest.mark.parametrize("na,nb", SIZES)
def test_w128_products(ctx, na, nb):
    a = inputs.random_poly(0x128A + na % 97, na)
    b = inputs.random_poly(0x128B + nb % 89, nb)
    say(f"case w128 product {na}x{nb}")
    got = host(ctx.mul(dev(a), na, dev(b), nb))
    assert np.array_equal(got, oracle.mul(a, na, b, nb)), (na, nb)


def test_w128_sizes_and_setting(ctx):
    assert ctx.word_bits() == 128
    for na, nb in [(1, 1), (128, 128), (129, 128), (128 * 1024, 128 * 1000)]:
        N = max(2, 1 << (words128(na) + words128(nb) - 2).bit_length())
        assert ctx.eval_points(na, nb) == N  # never truncated
    other = P.Context(0)
    try:
        assert other.word_bits() == 64
        for w in (0, 32, 96, 256):
            with pytest.raises(P.Gf2xError):
                other.set_word_bits(w)
        assert other.word_bits() == 64
    finally:
        other.close()


def test_w128_equals_w64_random_lengths(ctx):
    """Both widths give the same product bits (different fields, spectra and
    transform lengths)."""
    c64 = P.Context(0)
    rng = random.Random(128)
    try:
        for _ in range(12):
            na, nb = rng.randrange(1, 1 << 19), rng.randrange(1, 1 << 19)
            a, b = inputs.random_poly(rng.getrandbits(32), na), inputs.random_poly(rng.getrandbits(32), nb)
            say(f"case w128 vs w64 {na}x{nb}")
            da, db = dev(a), dev(b)
            x = host(ctx.mul(da, na, db, nb))
            y = host(c64.mul(da, na, db, nb))
            torch.cuda.synchronize()
            assert np.array_equal(x, y), (na, nb)
            if na + nb < 40000:
                assert np.array_equal(x, oracle.mul(a, na, b, nb))
    finally:
        torch.cuda.synchronize()
        c64.close()


def _golden(name):
    if not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith(name + " "):
                return line.split()
    return None


def test_w128_headline_product(ctx):
    n = 1 << 28
    sa, sb = inputs.SEEDS["c3a"]
    a = inputs.random_poly(sa, n)
    b = inputs.random_poly(sb, n)
    say(f"case w128 headline product {n}x{n}")
    got = host(ctx.mul(dev(a), n, dev(b), n))
    torch.cuda.synchronize()
    assert got.size == P.out_words(n, n)
    rng = random.Random(n + 128)
    for k in [0, 1, got.size // 2, got.size - 1] + [rng.randrange(got.size) for _ in range(6)]:
        assert int(got[k]) == oracle.word(a, n, b, n, k), k
    g = _golden("c3a")
    assert g is not None, f"tests/golden/product_sha256.txt has no line for c3a"
    assert hashlib.sha256(got.tobytes()).hexdigest() == g[6]


def _jobs(spec):
    jobs, ref = [], []
    for na, nb, sa, sb in spec:
        a, b = inputs.random_poly(sa, na), inputs.random_poly(sb, nb)
        c = torch.zeros(max(P.out_words(na, nb), 1), dtype=torch.int64, device="cuda")
        jobs.append((dev(a), na, dev(b), nb, c))
        ref.append((a, b))
    return jobs, ref


@pytest.mark.parametrize("persistent", [False, True], ids=["staged", "persistent"])
def test_w128_batch(ctx, persistent):
    spec = inputs.batch_workload(48, 6, 17)
    jobs, ref = _jobs(spec)
    say(f"case w128 batch (48 jobs, persistent={persistent})")
    B = ctx.batch(jobs, persistent=persistent)
    for rep in range(2):
        for j in jobs:
            j[4].zero_()
        torch.cuda.synchronize()
        B.run()
        torch.cuda.synchronize()
        B.check()
        for (da, na, db, nb, c), (a, b) in zip(jobs, ref):
            assert np.array_equal(host(c)[: P.out_words(na, nb)], oracle.mul(a, na, b, nb)), (rep, na, nb)
    B.close()


@pytest.mark.parametrize("persistent", [False, True], ids=["staged", "persistent"])
def test_w128_server_mix_equals_oracle(ctx, persistent):
    reqs = []
    for na, nb, sa, sb, _u in inputs.serve_workload(24, 0, 10, 18):
        a, b = inputs.random_poly(sa, na), inputs.random_poly(sb, nb)
        c = torch.full((max(P.out_words(na, nb), 1),), -1, dtype=torch.int64, device="cuda")
        reqs.append((a, na, b, nb, dev(a), dev(b), c))
    say(f"case w128 server (24 requests, persistent={persistent})")
    srv = ctx.server(1 << 30, max_active=32, levels_per_iter=2, persistent=persistent)
    for i, (a, na, b, nb, da, db, c) in enumerate(reqs):
        srv.submit(da, na, db, nb, c, i)
        if i % 8 == 7:
            srv.step(P.now_ns() + 100_000)
    done = srv.drain()
    srv.close()
    assert sorted(d["tag"] for d in done) == list(range(len(reqs)))
    assert all(d["status"] == 0 for d in done)
    for a, na, b, nb, da, db, c in reqs:
        assert np.array_equal(host(c)[: P.out_words(na, nb)], oracle.mul(a, na, b, nb)), (na, nb)
