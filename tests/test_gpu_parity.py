"""GPU parity: the HIP path (through the C ABI) against the oracle, bit for bit.

* products at ragged and configured sizes against oracle.mul (full compare);
* the headline sizes 2^28 and 2^29 against the oracle's recorded SHA-256, plus
  sampled output words (oracle.word), residues mod x^64 + q, and closed forms
  (a*a, a*(1 + x^k)) that hold at any size;
* stage entry points against the paper's definitions in oracle/tower.py
  (BasisCvt, the spectrum as an evaluation, the tower product);
* error paths of the ABI.
"""
import hashlib
import os
import random
import sys

import numpy as np
import pytest

import oracle
import oracle.tower as T
import paper_1708_09746_amd as P
from helpers import dev, host, spectrum_ints, spread_words, to_int, to_words
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


def gpu_mul(ctx, a, na, b, nb):
    da, db = dev(a), dev(b)
    c = ctx.mul(da, na, db, nb)
    torch.cuda.synchronize()
    return host(c)


SMALL = [(1, 1), (1, 64), (64, 1), (63, 65), (64, 64), (65, 64), (65, 65), (127, 129), (128, 128),
         (200, 7), (7, 200), (300, 300), (511, 512), (1000, 999), (64 * 31, 64 * 33), (5000, 70),
         (70, 5000), (4095, 4097), (64 * 1024, 64 * 1024 + 1), (100000, 3), (3, 100000),
         (64 * 2047 + 5, 64 * 2049 + 11), (320007, 192001)]


@pytest.mark.parametrize("na,nb", SMALL)
def test_product_small_sizes(ctx, na, nb):
    say(f"case product {na}x{nb}")
    a = inputs.random_poly(0x1000 + na, na)
    b = inputs.random_poly(0x2000 + nb, nb)
    got = gpu_mul(ctx, a, na, b, nb)
    ref = oracle.mul(a, na, b, nb)
    assert got.size == ref.size == P.out_words(na, nb)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_product_configured_sizes_full(ctx, name):
    n = {"c1": 1 << 16, "c2": 1 << 20}[name]
    sa, sb = inputs.SEEDS[name]
    say(f"case product {name} {n}x{n}")
    a = inputs.random_poly(sa, n)
    b = inputs.random_poly(sb, n)
    got = gpu_mul(ctx, a, n, b, n)
    assert np.array_equal(got, oracle.mul(a, n, b, n, threads=8))


def test_random_length_products(ctx):
    rng = random.Random(2024)
    for it in range(40):
        na = rng.randint(1, 1 << rng.randint(1, 18))
        nb = rng.randint(1, 1 << rng.randint(1, 18))
        say(f"case random product {it}: {na}x{nb}")
        a = inputs.random_poly(0x3000 + it, na)
        b = inputs.random_poly(0x4000 + it, nb)
        assert np.array_equal(gpu_mul(ctx, a, na, b, nb), oracle.mul(a, na, b, nb))


def test_garbage_bits_ignored_and_squaring_alias(ctx):
    na, nb = 6400 + 17, 3 * 64 + 1
    a = inputs.random_poly(5, na)
    b = inputs.random_poly(6, nb)
    ag, bg = a.copy(), b.copy()
    ag[-1] |= np.uint64(~((1 << (na % 64)) - 1) & 0xFFFFFFFFFFFFFFFF)
    bg[-1] |= np.uint64(~((1 << (nb % 64)) - 1) & 0xFFFFFFFFFFFFFFFF)
    say("case garbage high bits")
    assert np.array_equal(gpu_mul(ctx, ag, na, bg, nb), oracle.mul(a, na, b, nb))
    say("case squaring with aliased operands")
    da = dev(a)
    c = ctx.mul(da, na, da, na)
    torch.cuda.synchronize()
    assert np.array_equal(host(c), spread_words(a, na))


def test_empty_operand_writes_nothing(ctx):
    a = dev(inputs.random_poly(1, 100))
    c = torch.full((4,), 7, dtype=torch.int64, device="cuda")
    say("case empty operand")
    ctx.mul_into(a, 0, a, 100, c)
    ctx.mul_into(a, 100, a, 0, c)
    torch.cuda.synchronize()
    assert (c.cpu() == 7).all()


def test_host_pointer_entry_point():
    na, nb = 70000, 12345
    a = inputs.random_poly(71, na)
    b = inputs.random_poly(72, nb)
    say("case gf2x_mul host pointers")
    assert np.array_equal(P.mul_host(a, na, b, nb), oracle.mul(a, na, b, nb))


def test_results_do_not_depend_on_the_stream(ctx):
    na = nb = 1 << 18
    a = inputs.random_poly(81, na)
    b = inputs.random_poly(82, nb)
    da, db = dev(a), dev(b)
    s = torch.cuda.Stream()
    say("case side stream")
    with torch.cuda.stream(s):
        c1 = ctx.mul(da, na, db, nb, stream=s)
    s.synchronize()
    c2 = ctx.mul(da, na, db, nb)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2)
    assert np.array_equal(host(c2), oracle.mul(a, na, b, nb))


def test_back_to_back_products_across_the_fork_sizes(ctx):
    """Products enqueued on one stream with no synchronisation in between,
    sizes ascending (the workspace grows between them) and on both sides of
    the range whose forward transforms run on a second stream: each result
    is checked after a single synchronisation."""
    cases = [((1 << 16) - 9, 1 << 16, False), (1 << 19, (1 << 17) + 3, False), ((1 << 20) + 5, 0, True),
             ((1 << 20) + 64, 1 << 12, False), (1 << 25, 0, True)]
    ops = []
    for i, (na, nb, square) in enumerate(cases):
        a = inputs.random_poly(0x900 + i, na)
        b = None if square else inputs.random_poly(0x950 + i, nb)
        da = dev(a)
        ops.append((a, na, b, na if square else nb, da, da if square else dev(b)))
    torch.cuda.synchronize()
    say("case back-to-back products across the fork sizes")
    jobs = [(a, na, b, nb, ctx.mul(da, na, db, nb)) for a, na, b, nb, da, db in ops]
    torch.cuda.synchronize()
    for a, na, b, nb, c in jobs:
        want = spread_words(a, na) if b is None else oracle.mul(a, na, b, nb)
        assert np.array_equal(host(c), want), (na, nb)


def test_calls_on_mixed_streams_are_serialised(ctx):
    """Products on two streams in turn, with no synchronisation and no event
    from the caller between them, sizes ascending so the shared workspace
    grows: each call on a stream other than the previous call's waits for
    that call's work (the header's stream rule), so every result is exact."""
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    sizes = [(1 << 14, 1 << 14), (1 << 18, (1 << 18) - 7), (1 << 16, 1 << 16), ((1 << 21) + 3, 1 << 20),
             (1 << 12, 999), ((1 << 22) + 64, (1 << 22) - 1)]
    ops = []
    for i, (na, nb) in enumerate(sizes):
        a = inputs.random_poly(0xA00 + i, na)
        b = inputs.random_poly(0xA50 + i, nb)
        ops.append((a, na, b, nb, dev(a), dev(b)))
    cs = [torch.full((P.out_words(na, nb),), -1, dtype=torch.int64, device="cuda") for _, na, _, nb, _, _ in ops]
    torch.cuda.synchronize()
    say("case products on alternating streams")
    outs = []
    for i, (a, na, b, nb, da, db) in enumerate(ops):
        st = s1 if i % 2 == 0 else s2
        outs.append((a, na, b, nb, ctx.mul_into(da, na, db, nb, cs[i], stream=st)))
    s1.synchronize()
    s2.synchronize()
    for a, na, b, nb, c in outs:
        assert np.array_equal(host(c), oracle.mul(a, na, b, nb, threads=8)), (na, nb)


# ------------------------------------------------------------- stages


@pytest.mark.parametrize("m", [0, 1, 2, 3, 4, 5, 7, 9, 10])
def test_basiscvt_matches_definition(ctx, m):
    n = 1 << m
    w = inputs.splitmix64(0x500 + m, n)
    say(f"case basiscvt m={m}")
    d = dev(w)
    ctx.basiscvt(d, m)
    torch.cuda.synchronize()
    got = [int(x) for x in host(d)]
    assert got == T.to_novel_solve([int(x) for x in w])
    ctx.basiscvt(d, m, inverse=True)
    torch.cuda.synchronize()
    assert np.array_equal(host(d), w)


@pytest.mark.parametrize("m", [13, 14, 16])
def test_basiscvt_mixed_schedule_matches_alg3(ctx, m):
    """Sizes whose schedule mixes LDS tile runs and global layers, against the
    oracle's Alg. 3 on the whole array."""
    n = 1 << m
    w = inputs.splitmix64(0x600 + m, n)
    say(f"case basiscvt vs Alg. 3 m={m}")
    d = dev(w)
    ctx.basiscvt(d, m)
    torch.cuda.synchronize()
    assert [int(x) for x in host(d)] == T.basis_cvt([int(x) for x in w])


def test_basiscvt_global_layers_roundtrip(ctx):
    """2^29 words (4 GiB): the top VarSubs layers fit no class tile and run as
    global layer ops; iBasisCvt must undo BasisCvt (it once ran the two parts
    of such a layer in the forward order)."""
    m = 29
    g = torch.Generator(device="cuda")
    g.manual_seed(0x29)
    x = torch.empty(1 << m, dtype=torch.int64, device="cuda").random_(generator=g)
    y = x.clone()
    say(f"case basiscvt roundtrip with global layers m={m}")
    ctx.basiscvt(y, m)
    torch.cuda.synchronize()
    assert not torch.equal(x, y)
    ctx.basiscvt(y, m, inverse=True)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    del x, y
    torch.cuda.empty_cache()


@pytest.mark.parametrize("m", [20, 22, 23])
def test_basiscvt_large_roundtrip_and_linearity(ctx, m):
    """iBasisCvt undoes BasisCvt and the map is GF(2)-linear; a single nonzero
    word converts to the oracle's novel-basis coefficients of a monomial."""
    n = 1 << m
    w = inputs.splitmix64(0x600 + m, n)
    say(f"case basiscvt roundtrip m={m}")
    d = dev(w)
    ctx.basiscvt(d, m)
    fw = host(d).copy()
    ctx.basiscvt(d, m, inverse=True)
    torch.cuda.synchronize()
    assert np.array_equal(host(d), w)
    w2 = inputs.splitmix64(0x700 + m, n)
    d2 = dev(w2)
    ctx.basiscvt(d2, m)
    d3 = dev(w ^ w2)
    ctx.basiscvt(d3, m)
    torch.cuda.synchronize()
    assert np.array_equal(host(d3), fw ^ host(d2))
    for e in (0, 1, 255, 256, 1000):
        one = np.zeros(n, dtype=np.uint64)
        one[e] = np.uint64(1)
        do = dev(one)
        ctx.basiscvt(do, m)
        torch.cuda.synchronize()
        got = host(do)
        pre = 1
        while pre < e + 1:
            pre *= 2
        ref = T.to_novel_solve([1 if k == e else 0 for k in range(pre)])
        assert [int(x) for x in got[:pre]] == ref
        assert not got[pre:].any()


@pytest.mark.parametrize("na,log2n", [(1, 0), (1, 3), (64, 1), (130, 2), (64 * 8, 4), (64 * 16 - 5, 5), (700, 6)])
def test_forward_spectrum_is_evaluation(ctx, na, log2n):
    words = inputs.random_poly(0x800 + na, na)
    say(f"case forward spectrum na={na} log2n={log2n}")
    spec = ctx.forward(dev(words), na, log2n)
    torch.cuda.synchronize()
    got = spectrum_ints(spec)
    ws = [int(x) for x in words]
    for j in range(1 << log2n):
        assert got[j] == T.spectrum_point(ws, na, j), j


@pytest.mark.parametrize("na,log2n", [(1 << 14, 9), (1 << 16, 12), (1 << 20, 15), ((1 << 20) + 77, 17)])
def test_forward_spectrum_sampled_points(ctx, na, log2n):
    words = inputs.random_poly(0x900 + log2n, na)
    say(f"case forward spectrum sampled na={na} log2n={log2n}")
    spec = ctx.forward(dev(words), na, log2n)
    torch.cuda.synchronize()
    raw = host(spec)
    ws = [int(x) for x in words]
    rng = random.Random(log2n)
    pts = [0, 1, (1 << log2n) - 1] + [rng.randrange(1 << log2n) for _ in range(2)]
    for j in pts:
        got = int(raw[2 * j]) | (int(raw[2 * j + 1]) << 64)
        assert got == T.spectrum_point(ws, na, j), j


def test_pointmul_is_tower_product(ctx):
    n = 3000
    rng = np.random.default_rng(9)
    xa = rng.integers(0, 2**63, size=(n, 2), dtype=np.int64)
    xb = rng.integers(0, 2**63, size=(n, 2), dtype=np.int64)
    # include subfield and boundary values
    xa[0] = [0, 0]
    xa[1] = [1, 0]
    xb[2] = [0, 1 << 62]
    say("case pointmul")
    sa, sb = torch.from_numpy(xa).cuda(), torch.from_numpy(xb).cuda()
    sc = ctx.pointmul(sa, sb)
    torch.cuda.synchronize()
    A, B, C = spectrum_ints(sa), spectrum_ints(sb), spectrum_ints(sc)
    for j in range(0, n, 7):
        assert C[j] == T.gf_mul(A[j], B[j], 128), j
    assert C[1] == B[1]


@pytest.mark.parametrize("na,log2n", [(1, 1), (64 * 5, 3), (64 * 1000 + 3, 11), ((1 << 20) - 1, 15), (1 << 22, 16)])
def test_inverse_undoes_forward(ctx, na, log2n):
    """iFFT and iBasisCvt undo the forward transform, and changeRepr back
    undoes changeRepr, so inverse(forward(a)) returns a."""
    a = inputs.random_poly(0xA00 + log2n, na)
    say(f"case inverse(forward) na={na} log2n={log2n}")
    spec = ctx.forward(dev(a), na, log2n)
    c = ctx.inverse(spec, log2n, na)
    torch.cuda.synchronize()
    assert np.array_equal(host(c), a)


def test_inverse_of_oracle_spectrum(ctx):
    """Values of F(x) = sum_k Phi128(P_k) x^k at all 16 points, computed by the
    oracle, map back to the Kronecker combination of the 127-bit P_k."""
    rng = random.Random(77)
    N = 16
    Pk = [rng.getrandbits(127) for _ in range(N)]
    F = [T.phi(p) for p in Pk]
    vals = [T.horner(F, j) for j in range(N)]
    raw = np.zeros(2 * N, dtype=np.uint64)
    for j, v in enumerate(vals):
        raw[2 * j] = np.uint64(v & ((1 << 64) - 1))
        raw[2 * j + 1] = np.uint64(v >> 64)
    spec = torch.from_numpy(raw.view(np.int64).reshape(N, 2).copy()).cuda()
    nbits = 64 * N + 64
    say("case inverse of oracle spectrum")
    c = ctx.inverse(spec, 4, nbits)
    torch.cuda.synchronize()
    expect = 0
    for k, p in enumerate(Pk):
        expect ^= p << (64 * k)
    assert to_int(host(c)) == expect & ((1 << nbits) - 1)


def test_staged_product_equals_mul(ctx):
    na, nb = 123457, 98765
    a = inputs.random_poly(91, na)
    b = inputs.random_poly(92, nb)
    m = P.fft_log2(na, nb)
    say("case staged forward/pointmul/inverse")
    sa = ctx.forward(dev(a), na, m)
    sb = ctx.forward(dev(b), nb, m)
    ctx.pointmul(sa, sb, sb)
    c = ctx.inverse(sb, m, na + nb - 1)
    torch.cuda.synchronize()
    assert np.array_equal(host(c), oracle.mul(a, na, b, nb))


# ---------------------------------------------------------- batch


def test_batch_matches_oracle_and_single_calls(ctx):
    jobs_spec = inputs.batch_workload(64, 6, 16)
    jobs, ops = [], []
    for na, nb, sa, sb in jobs_spec:
        a, b = inputs.random_poly(sa, na), inputs.random_poly(sb, nb)
        da, db = dev(a), dev(b)
        c = torch.zeros(P.out_words(na, nb), dtype=torch.int64, device="cuda")
        jobs.append((da, na, db, nb, c))
        ops.append((a, na, b, nb))
    say("case batch of 64 uneven products")
    ctx.mul_batch(jobs)
    torch.cuda.synchronize()
    for (da, na, db, nb, c), (a, _, b, _) in zip(jobs, ops):
        assert np.array_equal(host(c), oracle.mul(a, na, b, nb))
        single = ctx.mul(da, na, db, nb)
        torch.cuda.synchronize()
        assert torch.equal(single, c)


# ------------------------------------------------------ headline sizes


def _golden(name):
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith(name + " "):
                return line.split()
    return None


@pytest.mark.parametrize("name", ["c3a", "c3b"])
def test_headline_product(ctx, name):
    n = {"c3a": 1 << 28, "c3b": 1 << 29}[name]
    sa, sb = inputs.SEEDS[name]
    a = inputs.random_poly(sa, n)
    b = inputs.random_poly(sb, n)
    say(f"case headline product {name}: {n}x{n}")
    c = ctx.mul(dev(a), n, dev(b), n)
    torch.cuda.synchronize()
    got = host(c)
    assert got.size == P.out_words(n, n)
    # sampled words straight from the convolution sum
    rng = random.Random(n)
    for k in [0, 1, got.size // 2, got.size - 1] + [rng.randrange(got.size) for _ in range(8)]:
        assert int(got[k]) == oracle.word(a, n, b, n, k), k
    # (a mod Q)(b mod Q) = c mod Q for random Q = x^64 + q
    for _ in range(3):
        q = rng.getrandbits(64)
        assert oracle.mulmod(oracle.mod(a, n, q), oracle.mod(b, n, q), q) == oracle.mod(got, 2 * n - 1, q)
    g = _golden(name)
    assert g is not None, f"tests/golden/product_sha256.txt has no line for {name}"
    assert hashlib.sha256(got.tobytes()).hexdigest() == g[6]


def test_product_2p30_widest_multipliers(ctx):
    """2^30-bit operands: 2^25 points, so the multipliers of the lowest layers
    have up to 25 bits (the general TGF(2^32) case of the butterflies, whose
    high TGF(2^16) half is not a byte); sampled words, and the square in full
    against its closed form."""
    n = 1 << 30
    assert P.fft_log2(n, n) == 25
    a = inputs.random_poly(0x30A, n)
    b = inputs.random_poly(0x30B, n)
    da = dev(a)
    say(f"case product {n}x{n} (2^25 points)")
    got = host(ctx.mul(da, n, dev(b), n))
    torch.cuda.synchronize()
    assert got.size == P.out_words(n, n)
    rng = random.Random(30)
    for k in [0, 1, 2, got.size - 2, got.size - 1] + [rng.randrange(got.size) for _ in range(2)]:
        assert int(got[k]) == oracle.word(a, n, b, n, k), k
    del got
    say(f"case squaring {n} (2^25 points)")
    sq = host(ctx.mul(da, n, da, n))
    torch.cuda.synchronize()
    assert np.array_equal(sq, spread_words(a, n))


@pytest.mark.parametrize("n", [1 << 28])
def test_headline_closed_forms(ctx, n):
    a = inputs.random_poly(0x28C, n)
    da = dev(a)
    say(f"case headline squaring {n}")
    c = ctx.mul(da, n, da, n)
    torch.cuda.synchronize()
    assert np.array_equal(host(c), spread_words(a, n))
    # a * (1 + x^k) = a + (a << k)
    k = 64 * 1000 + 13
    bk = np.zeros((k + 64) // 64, dtype=np.uint64)
    bk[0] = np.uint64(1)
    bk[k // 64] |= np.uint64(1 << (k % 64))
    say(f"case headline a*(1+x^k) {n}")
    c = ctx.mul(da, n, dev(bk), k + 1)
    torch.cuda.synchronize()
    got = host(c)
    ai = np.concatenate([a, np.zeros(got.size - a.size, dtype=np.uint64)])
    sh = np.zeros_like(ai)
    w, r = divmod(k, 64)
    sh[w:] = ai[: ai.size - w]
    shifted = (sh << np.uint64(r)) | np.concatenate([[np.uint64(0)], sh[:-1] >> np.uint64(64 - r)])
    assert np.array_equal(got, ai ^ shifted)


# ------------------------------------------------------------ errors


def test_error_paths(ctx):
    L = P.lib()
    import ctypes

    nul = ctypes.c_void_p(0)
    a = dev(inputs.random_poly(1, 640))
    say("case error paths")
    assert L.gf2x_mul_dev(ctx.handle, nul, 640, P._ptr(a), 640, P._ptr(a), nul) == P.GF2X_EINVAL
    # product overlapping an operand
    assert L.gf2x_mul_dev(ctx.handle, P._ptr(a), 640, P._ptr(a), 640, P._ptr(a), nul) == P.GF2X_EINVAL
    spec = torch.zeros((4, 2), dtype=torch.int64, device="cuda")
    assert L.gf2x_forward_dev(ctx.handle, P._ptr(a), 640, 33, P._ptr(spec), nul) == P.GF2X_ERANGE
    assert L.gf2x_forward_dev(ctx.handle, P._ptr(a), 640, 2, P._ptr(spec), nul) == P.GF2X_EINVAL
    assert L.gf2x_ctx_create(ctypes.byref(ctypes.c_void_p()), 1 << 20) == P.GF2X_EDEVICE
    assert L.gf2x_mul_batch(ctx.handle, None, 3, nul) == P.GF2X_EINVAL
    assert L.gf2x_last_error(ctx.handle).decode() == "NULL job array"
    # the message names the failing call's cause, and a later success clears it
    assert L.gf2x_mul_dev(ctx.handle, P._ptr(a), 640, P._ptr(a), 640, P._ptr(a), nul) == P.GF2X_EINVAL
    assert L.gf2x_last_error(ctx.handle).decode() == "product overlaps an operand"
    c = torch.zeros(P.out_words(640, 640), dtype=torch.int64, device="cuda")
    assert L.gf2x_mul_dev(ctx.handle, P._ptr(a), 640, P._ptr(a), 640, P._ptr(c), nul) == P.GF2X_OK
    assert L.gf2x_last_error(ctx.handle).decode() == ""
    torch.cuda.synchronize()
