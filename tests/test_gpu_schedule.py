"""FFT pass schedules on the GPU: every schedule in range gives the oracle's
product bits, the autotuner keeps a schedule per size and products planned
with it stay exact, and out-of-range schedules are refused."""
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
    yield c
    torch.cuda.synchronize()
    c.close()


# (na_bits, nb_bits): N = 2^12 (unbalanced, ragged), 2^15, 2^17 (a coset fan-out)
SIZES = [(64 * 700 + 3, 64 * 900 + 1), (1 << 20, 1 << 20), (1 << 22, 1 << 20)]
CASES = {}


def case(na, nb):
    if (na, nb) not in CASES:
        a = inputs.random_poly(0x5C0 + na % 97, na)
        b = inputs.random_poly(0x5C1 + nb % 89, nb)
        CASES[(na, nb)] = (a, b, oracle.mul(a, na, b, nb))
    return CASES[(na, nb)]


@pytest.mark.parametrize("sched", [(12, 6), (12, 12), (11, 8), (10, 5), (9, 3), (7, 11), (3, 2), (1, 1)])
def test_every_schedule_is_exact(ctx, sched):
    b, r = sched
    for m in range(1, 33):
        ctx.set_schedule(m, b, r)
    try:
        for na, nb in SIZES:
            a, bb, ref = case(na, nb)
            say(f"case schedule ({b}, {r}) {na} x {nb}")
            got = host(ctx.mul(dev(a), na, dev(bb), nb))
            assert np.array_equal(got, ref), (sched, na, nb)
    finally:
        for m in range(1, 33):
            ctx.set_schedule(m, 12, 6)


def test_autotune_then_products(ctx):
    say("case autotune m = 6..18")
    recs = ctx.autotune(6, 18, reps=3)
    assert [r["m"] for r in recs] == list(range(6, 19))
    for r in recs:
        assert ctx.get_schedule(r["m"]) == (r["bottom_log"], r["col_rows_log"])
        assert 1 <= r["bottom_log"] <= 12 and 1 <= r["col_rows_log"] <= 12
        assert r["candidates"] >= 1 and r["us_best"] <= r["us_default"]
    for na, nb in SIZES:
        a, bb, ref = case(na, nb)
        assert np.array_equal(host(ctx.mul(dev(a), na, dev(bb), nb)), ref)
    # a batch planned with the tuned schedules
    spec = inputs.batch_workload(64, 10, 18)
    jobs, refs = [], []
    for na, nb, sa, sb in spec:
        a, bb = inputs.random_poly(sa, na), inputs.random_poly(sb, nb)
        jobs.append((dev(a), na, dev(bb), nb, torch.zeros(P.out_words(na, nb), dtype=torch.int64, device="cuda")))
        refs.append(oracle.mul(a, na, bb, nb))
    ctx.mul_batch(jobs)
    torch.cuda.synchronize()
    for (da, na, db, nb, c), ref in zip(jobs, refs):
        assert np.array_equal(host(c), ref), (na, nb)
    for m in range(1, 33):
        ctx.set_schedule(m, 12, 6)


def test_schedule_range_checks(ctx):
    for bad in [(0, 11, 8), (33, 11, 8), (10, 0, 8), (10, 13, 8), (10, 11, 0), (10, 11, 13)]:
        with pytest.raises(P.Gf2xError) as e:
            ctx.set_schedule(*bad)
        assert e.value.code == P.GF2X_EINVAL
    with pytest.raises(P.Gf2xError):
        ctx.autotune(0, 5)
    with pytest.raises(P.Gf2xError):
        ctx.autotune(10, 27)
