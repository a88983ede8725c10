"""The serving engine on the GPU: continuous batching keeps every result
bit-identical to the same product computed alone, under staggered arrivals,
admission limited by arena space and slots, both execution modes and several
iteration lengths; errors are reported per request without stopping the rest."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

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


def make_requests(nreq, lo, hi, rate_index=0):
    reqs = []
    for na, nb, sa, sb, _u in inputs.serve_workload(nreq, rate_index, lo, hi):
        a, b = inputs.random_poly(sa, na), inputs.random_poly(sb, nb)
        c = torch.full((max(P.out_words(na, nb), 1),), -1, dtype=torch.int64, device="cuda")
        reqs.append(dict(na=na, nb=nb, a=a, b=b, da=dev(a), db=dev(b), c=c))
    return reqs


def alone(ctx, reqs):
    """Each product computed by itself through gf2x_mul_dev."""
    out = []
    for r in reqs:
        out.append(host(ctx.mul(r["da"], r["na"], r["db"], r["nb"])))
    torch.cuda.synchronize()
    return out


def run_staggered(srv, reqs, waves=4):
    """Submit in waves; between waves the engine runs a little, so later
    requests join while earlier ones are still on the device."""
    done = []
    per = (len(reqs) + waves - 1) // waves
    for w in range(waves):
        for i in range(w * per, min(len(reqs), (w + 1) * per)):
            r = reqs[i]
            srv.submit(r["da"], r["na"], r["db"], r["nb"], r["c"], i)
        srv.step(P.now_ns() + 200_000)
        done.extend(srv.poll())
    done.extend(srv.drain())
    return done


@pytest.fixture(scope="module")
def workload(ctx):
    reqs = make_requests(48, 10, 18)
    ref = alone(ctx, reqs)
    # the single-call path itself against the oracle on a few requests
    for i in (0, 1, 2):
        r = reqs[i]
        assert np.array_equal(ref[i], oracle.mul(r["a"], r["na"], r["b"], r["nb"]))
    return reqs, ref


@pytest.mark.parametrize("persistent", [False, True], ids=["staged", "persistent"])
@pytest.mark.parametrize("levels", [1, 3, 1000])
def test_mix_equals_alone(ctx, workload, persistent, levels):
    reqs, ref = workload
    for r in reqs:
        r["c"].fill_(-1)
    say(f"case serve mix: 48 requests, levels_per_iter={levels}, persistent={persistent}")
    srv = ctx.server(1 << 30, max_active=64, levels_per_iter=levels, persistent=persistent)
    done = run_staggered(srv, reqs)
    st = srv.stats()
    srv.close()
    assert sorted(d["tag"] for d in done) == list(range(len(reqs)))
    assert all(d["status"] == 0 for d in done)
    for d in done:
        assert d["t_submit_ns"] <= d["t_admit_ns"] <= d["t_done_ns"]
    for i, r in enumerate(reqs):
        assert np.array_equal(host(r["c"])[: P.out_words(r["na"], r["nb"])], ref[i]), (i, r["na"], r["nb"])
    assert st["completed"] == st["submitted"] == len(reqs)
    assert st["iterations"] >= 1 and st["arena_used"] == 0


def test_admission_by_footprint(ctx, workload):
    """An arena that holds only about two of the largest requests, and few
    slots: requests wait in the queue, memory is reused, results stay exact."""
    reqs, ref = workload
    for r in reqs:
        r["c"].fill_(-1)
    big = max(P.workspace_bytes(r["na"], r["nb"]) for r in reqs)
    arena = 2 * big + (1 << 16)
    say(f"case serve admission: arena {arena} bytes, 5 slots")
    srv = ctx.server(arena, max_active=5, levels_per_iter=2)
    done = run_staggered(srv, reqs, waves=2)
    st = srv.stats()
    srv.close()
    assert all(d["status"] == 0 for d in done) and len(done) == len(reqs)
    assert st["active_peak"] <= 5
    assert 0 < st["arena_peak"] <= arena
    # waiting happened: some request was admitted well after it was submitted
    assert any(d["t_admit_ns"] > d["t_submit_ns"] for d in done)
    for i, r in enumerate(reqs):
        assert np.array_equal(host(r["c"])[: P.out_words(r["na"], r["nb"])], ref[i]), i


def test_rejections_and_empty(ctx):
    """A request larger than the whole arena and a bad one are refused at
    submit; an empty product completes at once; the rest still completes."""
    na = nb = 1 << 14
    a, b = inputs.random_poly(0x77, na), inputs.random_poly(0x78, nb)
    da, db = dev(a), dev(b)
    c = torch.zeros(P.out_words(na, nb), dtype=torch.int64, device="cuda")
    ws = P.workspace_bytes(na, nb)
    srv = ctx.server(ws + 4096, max_active=4)
    big = 1 << 16
    ba = dev(inputs.random_poly(0x79, big))
    cb = torch.zeros(P.out_words(big, big), dtype=torch.int64, device="cuda")
    with pytest.raises(P.Gf2xError) as e:
        srv.submit(ba, big, ba, big, cb, 1)
    assert e.value.code == P.GF2X_ENOMEM
    with pytest.raises(P.Gf2xError) as e:
        srv.submit(da, na, db, nb, da, 2)  # product overlaps an operand
    assert e.value.code == P.GF2X_EINVAL
    srv.submit(da, 0, db, nb, c, 3)
    srv.submit(da, na, db, nb, c, 4)
    done = srv.drain()
    srv.close()
    assert sorted(d["tag"] for d in done) == [3, 4]
    assert all(d["status"] == 0 for d in done)
    assert np.array_equal(host(c), oracle.mul(a, na, b, nb))


def test_serving_workload_sizes(ctx):
    """Requests with operands up to 2^22 bits (the serving length range cut
    to keep the test short); sampled results against the oracle."""
    reqs = make_requests(24, 10, 22, rate_index=1)
    say("case serve sizes 2^10..2^22, 24 requests")
    srv = ctx.server(1 << 31, max_active=32, levels_per_iter=4)
    done = run_staggered(srv, reqs, waves=3)
    srv.close()
    assert all(d["status"] == 0 for d in done) and len(done) == len(reqs)
    for i in sorted(range(len(reqs)), key=lambda i: reqs[i]["na"] + reqs[i]["nb"])[:8]:
        r = reqs[i]
        assert np.array_equal(host(r["c"])[: P.out_words(r["na"], r["nb"])],
                              oracle.mul(r["a"], r["na"], r["b"], r["nb"])), i
    ref = alone(ctx, reqs)
    for i, r in enumerate(reqs):
        assert np.array_equal(host(r["c"])[: P.out_words(r["na"], r["nb"])], ref[i]), i


def test_serving_full_length_range_against_oracle(ctx):
    """Requests over the whole configured length range 2^10..2^24 bits per
    operand (24 drawn by the serving workload's generator, plus two with both
    operands of 2^24 bits), submitted in waves to the adaptive engine; every
    result compared with the oracle."""
    reqs = make_requests(24, 10, 24, rate_index=3)
    for k in range(2):
        n = 1 << 24
        a, b = inputs.random_poly(0x5F00 + 2 * k, n), inputs.random_poly(0x5F01 + 2 * k, n)
        c = torch.full((P.out_words(n, n),), -1, dtype=torch.int64, device="cuda")
        reqs.append(dict(na=n, nb=n, a=a, b=b, da=dev(a), db=dev(b), c=c))
    assert max(max(r["na"], r["nb"]) for r in reqs) == 1 << 24
    say("case serve 2^10..2^24 bits, 26 requests, adaptive engine")
    srv = ctx.server(1 << 31, max_active=32, levels_per_iter=2, persistent="adaptive")
    done = run_staggered(srv, reqs, waves=3)
    srv.close()
    assert sorted(d["tag"] for d in done) == list(range(len(reqs)))
    assert all(d["status"] == 0 for d in done)
    torch.cuda.synchronize()
    say("case serve 2^10..2^24 bits: oracle products")
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        want = list(ex.map(lambda r: oracle.mul(r["a"], r["na"], r["b"], r["nb"]), reqs))
    for i, (r, w) in enumerate(zip(reqs, want)):
        assert np.array_equal(host(r["c"])[: P.out_words(r["na"], r["nb"])], w), (i, r["na"], r["nb"])
