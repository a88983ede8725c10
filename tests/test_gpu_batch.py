"""Batches on the GPU: every job of a batch equals the oracle and the single
gf2x_mul_dev call, on the one-shot entry point and on a reusable batch whose
hipGraph is replayed several times with eager work in between."""
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


def make_jobs(spec):
    jobs, ref = [], []
    for na, nb, sa, sb in spec:
        a, b = inputs.random_poly(sa, na), inputs.random_poly(sb, nb)
        c = torch.zeros(max(P.out_words(na, nb), 1), dtype=torch.int64, device="cuda")
        jobs.append((dev(a), na, dev(b), nb, c))
        ref.append((a, b))
    return jobs, ref


def check(jobs, ref):
    for (da, na, db, nb, c), (a, b) in zip(jobs, ref):
        got = host(c)[: P.out_words(na, nb)]
        assert np.array_equal(got, oracle.mul(a, na, b, nb)), (na, nb)


@pytest.mark.parametrize("persistent", [False, True], ids=["staged", "persistent"])
def test_reusable_batch_graph_replays(ctx, persistent):
    spec = inputs.batch_workload(96, 6, 17)
    jobs, ref = make_jobs(spec)
    say(f"case batch create (96 uneven jobs, persistent={persistent})")
    B = ctx.batch(jobs, persistent=persistent)
    st = B.stats()
    assert st["ops"] > 96 and st["launches"] < st["ops"]
    if persistent:
        assert st["launches"] == 2
    for rep in range(3):
        for j in jobs:
            j[4].zero_()
        torch.cuda.synchronize()
        say(f"case batch run {rep} (graph {'record' if rep == 0 else 'replay'})")
        B.run()
        torch.cuda.synchronize()
        B.check()
        check(jobs, ref)
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(x)
    B.close()


def test_one_shot_batch_matches_single_calls(ctx):
    spec = [(1, 1, 1, 2), (64, 64, 3, 4), (65, 7000, 5, 6), (1 << 16, 1 << 16, 7, 8), (12345, 99, 9, 10),
            (0, 5, 11, 12), (3 * 64 + 1, 5 * 64 - 1, 13, 14)]
    jobs, ref = make_jobs([s for s in spec])
    say("case one-shot batch with an empty job")
    ctx.mul_batch(jobs)
    torch.cuda.synchronize()
    for (da, na, db, nb, c), (a, b) in zip(jobs, ref):
        if na == 0 or nb == 0:
            assert (c == 0).all()
            continue
        single = ctx.mul(da, na, db, nb)
        torch.cuda.synchronize()
        assert torch.equal(single, c[: single.numel()])
        assert np.array_equal(host(single), oracle.mul(a, na, b, nb))
    # a second call frees the first plan after waiting for it
    ctx.mul_batch(jobs[:2])
    torch.cuda.synchronize()


def test_batch_results_independent_of_neighbours(ctx):
    """A job's product is the same alone and inside a mix."""
    spec = inputs.batch_workload(40, 8, 18)
    jobs, ref = make_jobs(spec)
    say("case batch mix vs alone")
    B = ctx.batch(jobs)
    B.run()
    torch.cuda.synchronize()
    mixed = [host(j[4]).copy() for j in jobs]
    for k in (0, 17, 39):
        alone, _ = make_jobs([spec[k]])
        Bk = ctx.batch(alone)
        Bk.run()
        torch.cuda.synchronize()
        assert np.array_equal(host(alone[0][4]), mixed[k])
        Bk.close()
    B.close()


def test_persistent_wait_timeout_is_reported(ctx):
    """Forced from the host: a spin limit of 0 abandons the run at its first
    barrier wait; the kernel exits and the error is reported."""
    spec = inputs.batch_workload(16, 10, 14)
    jobs, ref = make_jobs(spec)
    B = ctx.batch(jobs, persistent=True)
    B.set_spin_limit(0)
    say("case persistent batch forced timeout")
    B.run()
    torch.cuda.synchronize()
    with pytest.raises(P.Gf2xError):
        B.check()
    # a normal limit afterwards completes the batch
    B.set_spin_limit(1 << 26)
    B.run()
    torch.cuda.synchronize()
    B.check()
    check(jobs, ref)
    B.close()


def test_large_persistent_batch_headline_like(ctx):
    spec = inputs.batch_workload(256, 12, 20)
    jobs, ref = make_jobs(spec)
    say("case persistent batch of 256 jobs, 2^12..2^20 bits")
    B = ctx.batch(jobs, persistent=True)
    B.run()
    torch.cuda.synchronize()
    B.check()
    for k in range(0, 256, 37):
        (da, na, db, nb, c), (a, b) = jobs[k], ref[k]
        assert np.array_equal(host(c)[: P.out_words(na, nb)], oracle.mul(a, na, b, nb))
    B.close()


def oracle_all(ref, spec, threads=16):
    """The oracle's product of every job, computed by a pool of threads (one
    job per call, so the pool runs independent products side by side)."""
    with ThreadPoolExecutor(min(threads, os.cpu_count() or 1)) as ex:
        return list(ex.map(lambda x: oracle.mul(x[0][0], x[1][0], x[0][1], x[1][1]), zip(ref, spec)))


def test_configured_batch_every_job_both_modes_tuned():
    """The configured batch: 4096 jobs with operand lengths floor(2^u),
    u ~ U[12, 20] bits for a and b independently, planned after the
    autotuner picked the FFT schedules; staged and persistent, each run on
    outputs filled with a sentinel, every job compared with the oracle."""
    ctx = P.Context(0)
    try:
        spec = inputs.batch_workload(4096, 12, 20)
        jobs, ref = make_jobs(spec)
        say("case configured batch: oracle products of 4096 jobs")
        want = oracle_all(ref, spec)
        say("case configured batch: autotune 2^6..2^20")
        tuned = ctx.autotune(6, 20, reps=2)
        assert len(tuned) == 15
        for persistent in (False, True):
            for j in jobs:
                j[4].fill_(-1)
            say(f"case configured batch: 4096 jobs, persistent={persistent}")
            B = ctx.batch(jobs, persistent=persistent)
            B.run()
            B.run()  # the graph replay, on the first run's results
            torch.cuda.synchronize()
            B.check()
            B.close()
            for k, ((da, na, db, nb, c), w) in enumerate(zip(jobs, want)):
                assert np.array_equal(host(c)[: P.out_words(na, nb)], w), (k, na, nb, persistent)
    finally:
        torch.cuda.synchronize()
        ctx.close()
