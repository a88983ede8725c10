"""Benchmark: one 2^28 x 2^28-bit GF(2)[x] product per step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3a|c3b|c2|c1]

Prints ONE JSON line.  `value` is milliseconds per product (lower is better)
with both operands already resident in HBM; the whole hot path (Split,
BasisCvt, changeRepr, FFT, pointmul, iFFT, iBasisCvt, changeRepr back,
InterleavedCombine) runs inside every step.  The `roofline` object covers the
kernel with the largest share of the product's time, timed with HIP events on
the library's launch stream during the timed region; `cpu_baseline` times the
oracle (plain CPU Karatsuba) on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms per 2^28-bit GF(2)[x] product (bit-exact); batched products/s; p99 ms"
HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
PAPER_MS = {"c3a": 2302.0, "c3b": 4812.0}  # Tab. 2, TGF(2^128) row, Haswell (context)
WORKLOADS = {
    "c1": (1 << 16, "2^16 x 2^16-bit product"),
    "c2": (1 << 20, "2^20 x 2^20-bit product"),
    "c3a": (1 << 28, "2^28 x 2^28-bit product"),
    "c3b": (1 << 29, "2^29 x 2^29-bit product"),
}
COUNTERS = os.path.join(ROOT, "profiles", "k_fft_c3a_counters.txt")
# FFT pass schedules (bottom_log, col_rows_log) per transform size 2^m for the
# headline products, chosen by the autotuner (gf2x_autotune) and pinned here so
# that every timed, traced and profiled run executes the same launches; sizes
# not listed keep the library default (12, 6)
PINNED_SCHEDULES = {22: (12, 10), 23: (12, 6), 24: (12, 6)}
UTILISATION = os.path.join(ROOT, "profiles", "c3a_utilisation.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest():
    import hashlib

    h = hashlib.sha256()
    cs = os.path.join(ROOT, "paper_1708_09746_amd", "csrc")
    for f in sorted(os.listdir(cs)):
        with open(os.path.join(cs, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources; else None."""
    if not os.path.exists(COUNTERS):
        return None
    kv = {}
    with open(COUNTERS) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel") != kernel or kv.get("source_digest") != source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def counter_utilisation(kernel):
    """VALU/LDS utilisation of `kernel` from the committed rocprofv3 counter
    table, if it was taken on the current kernel sources; else None."""
    if not os.path.exists(UTILISATION):
        return None
    digest, row = None, None
    with open(UTILISATION) as f:
        for line in f:
            if line.startswith("source_digest:"):
                digest = line.split(":", 1)[1].strip()
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) == 8 and cells[0] == kernel:
                row = cells
    if row is None or digest != source_digest():
        return None
    return {"valu_issue": float(row[4]), "lds_busy": float(row[5]), "lds_bank_conflict_share": float(row[6]),
            "waves_waiting": float(row[7]), "source": "profiles/c3a_utilisation.md"}


def host_cores():
    """Host threads this process may use: its CPU affinity, capped at 16 (the
    CPU share a one-GPU machine gives a job, whatever nproc reports)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def golden_sha(name):
    path = os.path.join(ROOT, "tests", "golden", "product_sha256.txt")
    with open(path) as f:
        for line in f:
            if line.startswith(name + " "):
                return line.split()[6]
    return None


def cpu_baseline(workload, na, seeds):
    """The oracle timed on the whole product of the headline operands, on the
    host's cores: the top Karatsuba step of the oracle's own recursion
    (a = a0 + a1 x^h, b = b0 + b1 x^h, h = na/2) as three oracle products of
    h-bit halves, each on every core, then their XOR combination; one line
    per finished sub-product.  The product is checked against the SHA-256 the
    oracle recorded for these operands.  A one-thread figure is extrapolated
    from a 2^23-bit sample (Karatsuba: x3 per doubling) and labelled so."""
    import hashlib

    import numpy as np

    import oracle
    from paper_1708_09746_amd import inputs

    threads = host_cores()
    a = inputs.random_poly(seeds[0], na)
    b = inputs.random_poly(seeds[1], na)
    h = na // 2
    hw = h // 64
    a0, a1, b0, b1 = a[:hw], a[hw:], b[:hw], b[hw:]
    t0 = time.perf_counter()
    p0 = oracle.mul(a0, h, b0, h, threads=threads)
    log(f"bench: cpu baseline: sub-product a0 b0 done ({time.perf_counter() - t0:.1f} s)")
    p2 = oracle.mul(a1, h, b1, h, threads=threads)
    log(f"bench: cpu baseline: sub-product a1 b1 done ({time.perf_counter() - t0:.1f} s)")
    p1 = oracle.mul(a0 ^ a1, h, b0 ^ b1, h, threads=threads)
    log(f"bench: cpu baseline: sub-product (a0+a1)(b0+b1) done ({time.perf_counter() - t0:.1f} s)")
    c = np.zeros(4 * hw, dtype=np.uint64)
    c[: p0.size] ^= p0
    c[hw: hw + p0.size] ^= p0 ^ p1 ^ p2
    c[2 * hw: 2 * hw + p2.size] ^= p2
    dt = time.perf_counter() - t0
    sha = hashlib.sha256(c.tobytes()).hexdigest()
    want = golden_sha(workload)
    # one thread: the oracle on the low 2^23 bits of each operand, scaled
    n1 = min(na, 1 << 23)
    t1 = time.perf_counter()
    oracle.mul(a[: n1 // 64], n1, b[: n1 // 64], n1, threads=1)
    dt1 = time.perf_counter() - t1
    lv = (na.bit_length() - 1) - (n1.bit_length() - 1)
    log(f"bench: cpu baseline: {dt * 1e3:.0f} ms on {threads} threads; one-thread sample {dt1:.2f} s")
    return {
        "value": round(dt * 1e3, 1),
        "unit": "ms",
        "cores": threads,
        "kind": "oracle",
        "sample": f"the whole 2^{na.bit_length() - 1} x 2^{na.bit_length() - 1}-bit product of the headline "
                  f"operands, measured once: the oracle's top Karatsuba step as three oracle products of "
                  f"2^{h.bit_length() - 1}-bit halves on {threads} threads each, plus their XOR combination",
        "host_cpu": cpu_model(),
        "product_sha256_matches_oracle_record": sha == want,
        "one_thread_ms" + ("_extrapolated" if lv else ""): round(dt1 * 1e3 * 3 ** lv, 1),
        "one_thread_note": (f"extrapolation, not a measurement: one thread on the low 2^{n1.bit_length() - 1} "
                            f"bits of each operand ({dt1:.2f} s) times 3^{lv}") if lv else
                           "measured: the whole product on one thread",
    }


def bench_batched(ctx, njobs=4096, reps=5):
    """Configured batch: njobs products, operand lengths floor(2^u) with
    u ~ U[12, 20] bits independently for a and b.  Products/s of (1) a loop of
    gf2x_mul_dev calls, (2) the staged batch replayed as a hipGraph, (3) the
    persistent single-launch batch replayed as a hipGraph."""
    import numpy as np
    import torch

    import paper_1708_09746_amd as P
    from paper_1708_09746_amd import inputs

    spec = inputs.batch_workload(njobs, 12, 20)
    jobs = []
    for na, nb, sa, sb in spec:
        a = torch.from_numpy(inputs.random_poly(sa, na).view(np.int64).copy()).cuda()
        b = torch.from_numpy(inputs.random_poly(sb, nb).view(np.int64).copy()).cuda()
        c = torch.zeros(P.out_words(na, nb), dtype=torch.int64, device="cuda")
        jobs.append((a, na, b, nb, c))
    stream = torch.cuda.current_stream()
    res = {"jobs": njobs, "lengths": "floor(2^u), u ~ U[12, 20] bits, a and b independent"}

    def timed(run):
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def loop():
        for (a, na, b, nb, c) in jobs:
            ctx.mul_into(a, na, b, nb, c, stream)

    # the oracle's products of every job (a pool of host threads, one job per
    # call), computed once; every timed path is checked against all of them
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(host_cores()) as ex:
        want = list(ex.map(lambda j: oracle.mul(j[0].cpu().numpy().view(np.uint64), j[1],
                                                j[2].cpu().numpy().view(np.uint64), j[3]), jobs))
    log(f"bench: batched: oracle products of {njobs} jobs done")
    checked = []

    def verify(what):
        """Every job's output (filled with a sentinel before the run) against the oracle."""
        torch.cuda.synchronize()
        for k, ((_a, na, _b, nb, c), w) in enumerate(zip(jobs, want)):
            assert np.array_equal(c.cpu().numpy().view(np.uint64), w), f"{what}: job {k} differs from the oracle"
        checked.append(what)

    def sentinel():
        for j in jobs:
            j[4].fill_(-1)

    sentinel()
    t_loop = timed(loop)
    verify("loop")
    res["loop_products_per_s"] = round(njobs / t_loop, 1)
    out = {}

    def batches(tag):
        for name, persistent in (("staged_graph", False), ("persistent_graph", True)):
            B = ctx.batch(jobs, persistent=persistent)
            sentinel()
            t = timed(lambda: B.run(stream))
            B.check()
            verify(f"{name}{tag}")
            st = B.stats()
            out[f"{name}{tag}"] = t
            res[f"{name}{tag}_products_per_s"] = round(njobs / t, 1)
            if not tag.startswith("_trunc"):
                res[f"{name}_launches"] = st["launches"]
            else:
                res[f"{name}{tag}_launches"] = st["launches"]
            B.close()

    batches("_default_schedule")
    # the autotuner picks an FFT pass schedule per transform size, then the
    # batches are planned again with it
    tuned = ctx.autotune(6, 20, reps=3)
    res["schedule"] = {str(r["m"]): [r["bottom_log"], r["col_rows_log"]] for r in tuned}
    batches("")
    # truncated transforms: each product evaluated at n_c rounded up to a
    # multiple of 2^(m - levels) points instead of all N (the tuned schedules)
    res["truncation"] = {}
    for levels, min_log in ((2, 8), (3, 8), (3, 11)):
        ctx.set_truncation(levels, min_log)
        tag = f"_trunc_{levels}_{min_log}"
        batches(tag)
        res["truncation"][f"levels={levels},min_log2n={min_log}"] = {
            "staged_graph_products_per_s": res.pop(f"staged_graph{tag}_products_per_s"),
            "staged_graph_launches": res.pop(f"staged_graph{tag}_launches"),
            "persistent_graph_products_per_s": res.pop(f"persistent_graph{tag}_products_per_s")}
        res.pop(f"persistent_graph{tag}_launches")
        out.pop(f"staged_graph{tag}")
        out.pop(f"persistent_graph{tag}")
    ctx.set_truncation(3, 23, 2)  # the default
    best = min(out, key=out.get)
    res["best"] = best
    res["speedup_vs_loop"] = round(t_loop / out[best], 2)
    res["checked_against_oracle"] = {"jobs": njobs, "paths": checked,
                                     "how": "outputs filled with a sentinel before each path's runs, "
                                            "every job compared with the oracle after them"}
    return res


def bench_serving(ctx, nreq=10000, fracs=(0.1, 0.25, 0.5, 0.75, 0.9, 0.9, 0.9, 1.0, 1.2), arena_gib=16,
                  oracle_sample=32):
    """Serving: requests with operand lengths floor(2^u), u ~ U[10, 24] bits
    independently for a and b, Poisson arrivals.  First the saturation
    throughput of the continuous-batching server (all requests queued at
    once) for a few engine settings; then, for the best one, open-loop
    Poisson streams at fractions of that saturation rate, with latency taken
    from the scheduled arrival to the observed completion (first 10 % of each
    stream discarded).  The same streams go through the plain path (one
    gf2x_mul_dev call per request, FIFO on one stream) for comparison.  The
    0.9 point runs three times (its spread is reported).

    Checks: the output buffer is filled with a sentinel before every run; after
    the first run a seeded sample of requests is compared with the oracle and
    the whole buffer is kept, and every later run (other engine settings, the
    Poisson streams, the plain path) must reproduce it for all requests."""
    import math
    from collections import deque

    import numpy as np
    import torch

    import paper_1708_09746_amd as P
    from paper_1708_09746_amd import inputs

    spec = inputs.serve_workload(nreq, 0, 10, 24)
    # operands are windows of one seeded pool (timing does not depend on the
    # bits); every request has its own output buffer
    max_words = (1 << 24) // 64
    pool_words = 4 * max_words
    pool = torch.from_numpy(inputs.random_poly(inputs.SERVE_POOL_SEED, 64 * pool_words).view(np.int64).copy()).cuda()
    offs = inputs.splitmix64(inputs.SERVE_POOL_SEED + 1, 2 * nreq) % np.uint64(pool_words - max_words)
    ow = [P.out_words(na, nb) for na, nb, *_ in spec]
    cbuf = torch.empty(sum(ow) + 1, dtype=torch.int64, device="cuda")
    reqs, pos = [], 0
    for r, (na, nb, _sa, _sb, _u) in enumerate(spec):
        oa, ob = int(offs[2 * r]), int(offs[2 * r + 1])
        a = pool[oa: oa + (na + 63) // 64]
        b = pool[ob: ob + (nb + 63) // 64]
        reqs.append((a, na, b, nb, cbuf[pos: pos + ow[r]]))
        pos += ow[r]
    gaps = np.array([-math.log1p(-u) for *_x, u in spec])  # unit-rate exponential gaps
    torch.cuda.synchronize()
    arena = min(arena_gib << 30, int(torch.cuda.mem_get_info()[0] * 0.25))

    first = {}
    checked = []

    def sentinel():
        cbuf.fill_(-1)
        torch.cuda.synchronize()

    def verify(what):
        """The whole output buffer against the first run's (itself checked
        against the oracle on a sample)."""
        torch.cuda.synchronize()
        if not first:
            import oracle
            from concurrent.futures import ThreadPoolExecutor

            rng = np.random.default_rng(0x5EED)
            pick = sorted(set(int(i) for i in rng.choice(nreq, oracle_sample, replace=False)))
            host = [(reqs[i][0].cpu().numpy().view(np.uint64), reqs[i][1], reqs[i][2].cpu().numpy().view(np.uint64),
                     reqs[i][3]) for i in pick]
            with ThreadPoolExecutor(host_cores()) as ex:
                want = list(ex.map(lambda h: oracle.mul(*h), host))
            for i, w in zip(pick, want):
                got = reqs[i][4].cpu().numpy().view(np.uint64)
                assert np.array_equal(got, w), f"{what}: served request {i} differs from the oracle"
            first["buf"] = cbuf.clone()
            first["sample"] = pick
            log(f"bench: serving: {len(pick)} sampled requests of the first run equal the oracle")
        else:
            assert torch.equal(cbuf, first["buf"]), f"{what}: served results differ from the first run's"
        checked.append(what)

    def saturate(levels, persistent):
        srv = ctx.server(arena, max_active=4096, levels_per_iter=levels, persistent=persistent)
        sentinel()
        t0 = time.perf_counter()
        for i, (a, na, b, nb, c) in enumerate(reqs):
            srv.submit(a, na, b, nb, c, i)
        done = srv.drain()
        t = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        assert len(done) == nreq and all(d["status"] == 0 for d in done)
        verify(f"saturation levels={levels} mode={persistent}")
        return nreq / t, st

    def open_loop(rate, submit, poll, idle):
        """Latencies (ms) of one Poisson stream at `rate` requests/s."""
        t0 = P.now_ns() + 2_000_000
        arr = t0 + np.cumsum(gaps / rate * 1e9).astype(np.int64)
        lat = np.zeros(nreq)
        got, i = 0, 0
        while got < nreq:
            now = P.now_ns()
            while i < nreq and arr[i] <= now:
                submit(i)
                i += 1
            for tag, t_done in poll():
                lat[tag] = (t_done - arr[tag]) / 1e6
                got += 1
            idle(int(arr[i]) if i < nreq else now + 1_000_000)
        span = (arr[-1] - arr[nreq // 10]) / 1e9
        keep = lat[nreq // 10:]
        return dict(offered_per_s=round(rate, 1),
                    achieved_per_s=round(float(len(keep) / max(span, 1e-9)), 1),
                    p50_ms=round(float(np.percentile(keep, 50)), 3),
                    p99_ms=round(float(np.percentile(keep, 99)), 3))

    res = {"requests": nreq, "lengths": "floor(2^u), u ~ U[10, 24] bits, a and b independent",
           "arrivals": "Poisson (open loop), latency from scheduled arrival to completion, first 10 % discarded",
           "arena_bytes": arena}
    # engine settings: execution mode x dependency levels per iteration
    tune = {}
    for mode, levels in (("staged", 8), ("staged", 4), ("persistent", 2), ("adaptive", 2), ("adaptive", 4)):
        rate, st = saturate(levels, {"staged": False, "persistent": True, "adaptive": "adaptive"}[mode])
        key = f"{mode}_L{levels}"
        tune[key] = round(rate, 1)
        log(f"bench: serving saturation {key}: {rate:.0f} products/s, {st['iterations']} iterations")
    res["saturation_products_per_s"] = tune
    # the same with truncated transforms (evaluation at n_c rounded up to a
    # multiple of 2^(m - 3) points, transforms of 2^8 points and more)
    ctx.set_truncation(3, 8)
    rate, st = saturate(2, "adaptive")
    ctx.set_truncation(3, 23, 2)  # the default
    res["saturation_truncated_products_per_s"] = {"adaptive_L2": round(rate, 1),
                                                  "setting": "levels=3, min_log2n=8"}
    log(f"bench: serving saturation adaptive_L2 with truncation: {rate:.0f} products/s")
    sat = max(tune.values())
    # the open-loop streams run on the adaptive engine (persistent iterations
    # under load, staged ones when idle or backlogged), at fractions of the
    # best saturation rate of any setting
    res["engine"] = {"mode": "adaptive", "levels_per_iter": 2, "inflight": 2}
    srv = ctx.server(arena, max_active=4096, levels_per_iter=2, persistent="adaptive")

    def s_submit(i):
        a, na, b, nb, c = reqs[i]
        srv.submit(a, na, b, nb, c, i)

    def s_poll():
        return [(d["tag"], d["t_done_ns"]) for d in srv.poll()]

    rates = []
    for f in fracs:
        sentinel()
        r = open_loop(f * sat, s_submit, s_poll, lambda until: srv.step(until))
        verify(f"server Poisson stream at {f} x saturation")
        r["fraction_of_saturation"] = f
        rates.append(r)
        log(f"bench: serving at {f:.2f} x saturation: {r}")
    srv.close()
    res["server"] = rates
    spread = [r for r in rates if r["fraction_of_saturation"] == 0.9]
    res["server_0.9_spread"] = {"runs": len(spread), "p50_ms": [r["p50_ms"] for r in spread],
                                "p99_ms": [r["p99_ms"] for r in spread]}

    # plain path: one gf2x_mul_dev per request as it arrives, FIFO on one stream
    stream = torch.cuda.Stream()
    pending = deque()

    def p_submit(i):
        a, na, b, nb, c = reqs[i]
        ctx.mul_into(a, na, b, nb, c, stream)
        ev = torch.cuda.Event()
        ev.record(stream)
        pending.append((i, ev))

    def p_poll():
        out = []
        while pending and pending[0][1].query():
            out.append((pending[0][0], P.now_ns()))
            pending.popleft()
        return out

    def p_idle(until):
        while P.now_ns() < until and not (pending and pending[0][1].query()):
            pass

    sentinel()
    t0 = time.perf_counter()
    for i in range(nreq):
        p_submit(i)
    stream.synchronize()
    pending.clear()
    plain_sat = nreq / (time.perf_counter() - t0)
    verify("plain path saturation")
    res["plain_saturation_products_per_s"] = round(plain_sat, 1)
    plain = []
    for f in fracs:
        rate = f * sat
        if rate > 0.95 * plain_sat:
            plain.append({"offered_per_s": round(rate, 1), "fraction_of_saturation": f,
                          "note": "above the plain path's saturation rate: its queue grows without bound"})
            continue
        sentinel()
        r = open_loop(rate, p_submit, p_poll, p_idle)
        verify(f"plain path at {f} x saturation")
        r["fraction_of_saturation"] = f
        plain.append(r)
        log(f"bench: plain path at {f:.2f} x saturation: {r}")
    res["plain"] = plain
    res["speedup_saturation_vs_plain"] = round(sat / plain_sat, 2)
    res["saturation_products_per_s_best"] = sat
    res["checked"] = {"oracle_sample": first.get("sample", []), "runs_equal_to_first": checked,
                      "how": "output buffer filled with a sentinel before every run; the first run's results "
                             "compared with the oracle on the sampled requests; every run's whole buffer "
                             "equal to the first run's"}
    return res


def bench_sizes(P, ctx, runs=50):
    """Single products at the other configured sizes, operands resident: the
    latency of one call (2^16 and 2^20 bits: launch- and on-chip-bound; median
    and p99 of `runs` calls, each timed by events on its stream), also as a
    reusable one-job batch replayed as a graph, and the time per product at
    2^29 bits."""
    import numpy as np
    import torch

    from paper_1708_09746_amd import inputs

    out = {}
    for name, reps in (("c1", runs), ("c2", runs), ("c3b", 10)):
        n, desc = WORKLOADS[name]
        sa, sb = inputs.SEEDS[name]
        a = torch.from_numpy(inputs.random_poly(sa, n).view(np.int64).copy()).cuda()
        b = torch.from_numpy(inputs.random_poly(sb, n).view(np.int64).copy()).cuda()
        c = torch.empty(P.out_words(n, n), dtype=torch.int64, device="cuda")
        stream = torch.cuda.current_stream()
        for _ in range(3):
            ctx.mul_into(a, n, b, n, c, stream)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.mul_into(a, n, b, n, c, stream)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ts.sort()
        out[name] = {"workload": desc, "runs": reps, "median_ms": round(ts[len(ts) // 2], 4),
                     "p99_ms": round(ts[min(len(ts) - 1, int(0.99 * len(ts)))], 4),
                     "fft_points": 1 << P.fft_log2(n, n)}
        # the kernels one call launches (the library's trace), and its product
        # against the oracle's recorded SHA-256
        ctx.trace_begin(0x3FF)
        c.fill_(-1)
        ctx.mul_into(a, n, b, n, c, stream)
        recs = ctx.trace_end()
        import hashlib

        out[name]["sha256_equals_oracle_record"] = (
            hashlib.sha256(c.cpu().numpy().tobytes()).hexdigest() == golden_sha(name))
        out[name]["launches"] = len(recs)
        out[name]["kernels"] = sorted(set(r["kernel"] for r in recs))
        if name == "c1":
            # the same call as one launch: a single block runs every stage
            ctx.set_single_launch(12)
            c.fill_(-1)
            ctx.trace_begin(0x3FF)
            ctx.mul_into(a, n, b, n, c, stream)
            one = ctx.trace_end()
            same = hashlib.sha256(c.cpu().numpy().tobytes()).hexdigest() == golden_sha(name)
            ms = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                ctx.mul_into(a, n, b, n, c, stream)
                e1.record(stream)
                e1.synchronize()
                ms.append(e0.elapsed_time(e1))
            ctx.set_single_launch(-1)
            ms.sort()
            out[name]["single_launch"] = {"median_ms": round(ms[len(ms) // 2], 4), "launches": len(one),
                                          "kernels": sorted(set(r["kernel"] for r in one)),
                                          "sha256_equals_oracle_record": same}
        if name != "c3b":
            # the same product as a reusable one-job batch: its launches replay
            # as one hipGraph
            B = ctx.batch([(a, n, b, n, c)])
            for _ in range(3):
                B.run(stream)
            torch.cuda.synchronize()
            gs = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                B.run(stream)
                e1.record(stream)
                e1.synchronize()
                gs.append(e0.elapsed_time(e1))
            B.check()
            B.close()
            gs.sort()
            out[name]["graph_median_ms"] = round(gs[len(gs) // 2], 4)
            out[name]["graph_p99_ms"] = round(gs[min(len(gs) - 1, int(0.99 * len(gs)))], 4)
        if name in PAPER_MS:
            out[name]["paper_ms"] = PAPER_MS[name]
        del a, b, c
    return out


def bench_w128(P, a, b, n, ref, steps, warmup, tune):
    """Alg. 5 with 128-bit words over TGF(2^256) on the same operands: timed
    like the headline product (tuned schedules, operands resident), and
    checked equal to the w = 64 product `ref`."""
    import torch

    ctx = P.Context(0)
    ctx.set_word_bits(128)
    k = (n + 127) // 128
    m = max(1, (2 * k - 2).bit_length())
    m_op = max(1, (k - 1).bit_length())
    sched = ctx.autotune(min(m_op, m), m, reps=3) if m <= 26 and tune else []
    c = torch.empty_like(ref)
    for _ in range(warmup):
        ctx.mul_into(a, n, b, n, c)
    torch.cuda.synchronize()
    ctx.trace_begin(0xFF)
    ctx.mul_into(a, n, b, n, c)
    torch.cuda.synchronize()
    per_kernel = {}
    for r in ctx.trace_end():
        per_kernel[r["kernel"]] = per_kernel.get(r["kernel"], 0.0) + r["ms"]
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.mul_into(a, n, b, n, c)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    equal = bool(torch.equal(c, ref))
    ctx.close()
    assert equal, "the w = 128 product differs from the w = 64 one"
    return {"field": "TGF(2^256), w = 128", "ms_per_product": round(ms, 4), "fft_points": 1 << m,
            "stages_ms": {k2: round(v, 4) for k2, v in sorted(per_kernel.items(), key=lambda kv: -kv[1])},
            "fft_schedule": {str(r["m"]): [r["bottom_log"], r["col_rows_log"]] for r in sched},
            "equal_to_w64": equal}


VARIANTS = {
    "simple": ("simple_mul_into", "GF(2^128) polynomial basis, Cantor points"),
    "frobenius": ("frobenius_mul_into", "GF(2^128) polynomial basis, Frobenius partition: points beta_{m+64} + V_m"),
}


def bench_variant(P, name, a, b, n, ref, steps, warmup, other_sizes=True):
    """Alg. 4 (polynomial-basis GF(2^128), Cantor points) or the
    Frobenius-partition variant (App. C) on the same operands: timed like the
    headline product (operands resident), checked equal to the tower product
    `ref`; also the rate of full GF(2^128) products it sustains (butterflies
    of the three transforms plus the pointwise products)."""
    import torch

    meth, field = VARIANTS[name]
    ctx = P.Context(0)
    mul_into = getattr(ctx, meth)
    c = torch.empty_like(ref)
    for _ in range(warmup):
        mul_into(a, n, b, n, c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        mul_into(a, n, b, n, c)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    equal = bool(torch.equal(c, ref))
    assert equal, f"the {name} variant's product differs from the tower one"
    # the other configured sizes: one call's latency (median of `reps`,
    # events on the stream), product checked against the tower method's
    import numpy as np

    from paper_1708_09746_amd import inputs

    sizes = {}
    stream = torch.cuda.current_stream()
    for wl, reps in (("c1", 30), ("c2", 30), ("c3b", 5)) if other_sizes else ():
        n2, desc = WORKLOADS[wl]
        s1, s2 = inputs.SEEDS[wl]
        a2 = torch.from_numpy(inputs.random_poly(s1, n2).view(np.int64).copy()).cuda()
        b2 = torch.from_numpy(inputs.random_poly(s2, n2).view(np.int64).copy()).cuda()
        c2 = torch.empty(P.out_words(n2, n2), dtype=torch.int64, device="cuda")
        for _ in range(2):
            mul_into(a2, n2, b2, n2, c2, stream)
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            mul_into(a2, n2, b2, n2, c2, stream)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ts.sort()
        same = bool(torch.equal(c2, ctx.mul(a2, n2, b2, n2, stream)))
        assert same, f"the {name} variant's product differs from the tower one at {desc}"
        sizes[wl] = {"workload": desc, "runs": reps, "median_ms": round(ts[len(ts) // 2], 4), "equal_to_tower": same}
        del a2, b2, c2
    ctx.close()
    k = (n + 63) // 64
    if name == "simple":
        m = max(1, (2 * k - 2).bit_length())
        m_op = (k - 1).bit_length()
        N = 1 << m
        prods = (N // 2) * (2 * m_op + m) + N
    else:
        m = P.frobenius_log2n(n, n)
        N = 1 << m
        prods = (N // 2) * 3 * m + N
    return {"field": field, "ms_per_product": round(ms, 4), "fft_points": N,
            "field_products": prods, "field_products_per_s": round(prods / (ms * 1e-3), 1),
            "equal_to_tower": equal, "sizes": sizes}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3a", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-products measurement")
    ap.add_argument("--batch-jobs", type=int, default=4096)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--tune", action="store_true",
                    help="let the autotuner pick the headline product's FFT pass schedules instead of the pinned ones")
    ap.add_argument("--no-w128", action="store_true", help="skip the 128-bit-word (TGF(2^256)) variant")
    ap.add_argument("--no-simple", action="store_true", help="skip the simple variant (Alg. 4)")
    ap.add_argument("--no-frobenius", action="store_true", help="skip the Frobenius-partition variant (App. C)")
    ap.add_argument("--no-sizes", action="store_true", help="skip the single products at 2^16, 2^20, 2^29 bits")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent products shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1708_09746_amd as P
    from paper_1708_09746_amd import inputs

    n, desc = WORKLOADS[args.workload]
    seeds = inputs.SEEDS[args.workload]
    log(f"bench: workload {args.workload} ({desc}), steps {args.steps}, warmup {args.warmup}")
    if args.copy_mib:
        src = torch.ones(args.copy_mib << 17, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: calibration copy of {args.copy_mib} MiB done (3 dispatches)")
        del src, dst
    ctx = P.Context(0)
    a = torch.from_numpy(inputs.random_poly(seeds[0], n).view(np.int64).copy()).cuda()
    b = torch.from_numpy(inputs.random_poly(seeds[1], n).view(np.int64).copy()).cuda()
    c = torch.empty(P.out_words(n, n), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    # FFT pass schedules of this product's transform sizes (operand and
    # product): pinned, so that the timed run, the traced run and the
    # profiler runs execute the same launches (--tune: the autotuner's choice)
    m = P.fft_log2(n, n)
    m_op = max(1, (((n + 63) // 64) - 1).bit_length())
    if args.tune and m <= 26:
        sched = ctx.autotune(min(m_op, m), m, reps=3)
        log(f"bench: tuned FFT schedules {sched}")
    else:
        sched = []
        for mm in range(min(m_op, m), m + 1):
            bl, cr = PINNED_SCHEDULES.get(mm, ctx.get_schedule(mm))
            ctx.set_schedule(mm, bl, cr)
            sched.append({"m": mm, "bottom_log": bl, "col_rows_log": cr, "source": "pinned"})
    # warmup untraced, then one traced product: per-stage times and the dominant kernel
    for _ in range(args.warmup):
        ctx.mul_into(a, n, b, n, c, stream)
    torch.cuda.synchronize()
    ctx.trace_begin(0xFF)
    ctx.mul_into(a, n, b, n, c, stream)
    torch.cuda.synchronize()
    recs = ctx.trace_end()
    per_kernel, launches = {}, {}
    for r in recs:
        per_kernel[r["kernel"]] = per_kernel.get(r["kernel"], 0.0) + r["ms"]
        launches[r["kernel"]] = launches.get(r["kernel"], 0) + 1
    stages = {k: round(v, 4) for k, v in sorted(per_kernel.items(), key=lambda kv: -kv[1])}
    dominant = max(per_kernel, key=per_kernel.get) if per_kernel else "k_fft"
    kind_bit = 1 << P.KERNEL_OF_KIND.index(dominant)
    log(f"bench: per-kernel ms per product (one traced product after warmup): {stages}")

    # timed region: no instrumentation; K products back to back on one stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.mul_into(a, n, b, n, c, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    # the same K products again with the dominant kernel's launches bracketed
    # by HIP events inside their own dispatches on the launch stream
    ctx.trace_begin(kind_bit)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        ctx.mul_into(a, n, b, n, c, stream)
    torch.cuda.synchronize()
    ms_traced = (time.perf_counter() - t2) * 1e3 / args.steps
    recs = ctx.trace_end()

    # Algorithmic bytes of the method: read both operands and write the
    # product (B_floor), plus one HBM round trip of each of the three
    # N-point spectra (6T, T = 16 N bytes); the FFT passes' share of one
    # product is the 6T, spread over their launches.
    N = 1 << m
    T = 16 * N
    out_bytes = 8 * P.out_words(n, n)
    b_floor = 2 * (n // 8) + out_bytes
    b_alg = b_floor + 6 * T
    tot_ms = sum(r["ms"] for r in recs)
    nl = max(len(recs), 1)
    per_product = nl / args.steps
    avg_ms = tot_ms / nl
    alg_per_launch = (6 * T) / per_product if dominant == "k_fft" else \
        sum(r["bytes_read"] + r["bytes_written"] for r in recs) / nl
    achieved = alg_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    pass_bytes = sum(r["bytes_read"] + r["bytes_written"] for r in recs) / nl
    traffic = counter_traffic(dominant)
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": dominant,
        "launches": len(recs),
        "launches_per_product": per_product,
        "avg_launch_ms": round(avg_ms, 5),
        "alg_bytes_per_launch": int(alg_per_launch),
        "alg_bytes_rule": "6T / (k_fft launches per product), T = 16 N bytes: one HBM round trip of each of "
                          "the three N-point spectra",
        "traffic_over_alg": round(traffic / alg_per_launch, 3) if traffic else None,
        "pass_bytes_per_launch": int(pass_bytes),
        "pass_bytes_rule": "each element a pass covers read once and written once",
        "product": {"b_floor": b_floor, "b_alg": b_alg, "spectrum_bytes_T": T,
                    "achieved_GBs": round(b_alg / (ms * 1e-3) / 1e9, 1),
                    "frac": round(b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "utilisation": counter_utilisation(dominant),
        "timing": {"untraced_ms_per_product": round(ms, 4), "traced_ms_per_product": round(ms_traced, 4),
                   "how": "value: K products untimed by events; avg_launch_ms: the same K products again, "
                          "the dominant kernel's launches carrying two HIP events in their dispatches"},
    }
    # the unit that bounds the FFT passes: random byte lookups into LDS tables
    lk = sum(r["lookups"] for r in recs)
    if lk and tot_ms > 0:
        peak_lk = ctx.lookup_rate()
        ach_lk = lk / (tot_ms * 1e-3)
        roofline["lds_lookups"] = {"achieved": round(ach_lk / 1e12, 3), "peak": round(peak_lk / 1e12, 3),
                                   "unit": "T lookups/s", "frac": round(ach_lk / peak_lk, 4),
                                   "per_launch": int(lk / nl),
                                   "peak_source": "gf2x_lookup_rate: random byte lookups into a 64 KiB LDS "
                                                  "table on every CU, measured in this run"}

    # bit-exactness of the timed product: its SHA-256 against the oracle's
    # record for these operands, and two words from the convolution sum
    import hashlib

    import oracle

    got = c.cpu().numpy().view(np.uint64)
    an = a.cpu().numpy().view(np.uint64)
    bn = b.cpu().numpy().view(np.uint64)
    for k in (0, got.size // 3):
        assert int(got[k]) == oracle.word(an, n, bn, n, k), f"word {k} differs from the oracle"
    want_sha = golden_sha(args.workload)
    sha_ok = hashlib.sha256(got.tobytes()).hexdigest() == want_sha
    assert want_sha is None or sha_ok, "the timed product's SHA-256 differs from the oracle's record"

    out = {
        "metric": METRIC,
        "value": round(ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": round(ms / PAPER_MS[args.workload], 6) if args.workload in PAPER_MS else None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "na_bits": n,
            "nb_bits": n,
            "fft_points": 1 << P.fft_log2(n, n),
            "field": "TGF(2^128), w = 64",
            "seeds": [hex(s) for s in seeds],
        },
        "roofline": roofline,
        "stages_ms": stages,
        "launches_per_product": launches,
        "fft_schedule": {str(r["m"]): [r["bottom_log"], r["col_rows_log"]] for r in sched},
        "fft_schedule_source": "autotuned in this run" if args.tune else "pinned (PINNED_SCHEDULES)",
        "product_sha256_equals_oracle_record": sha_ok,
    }
    if not args.no_sizes and args.workload == "c3a":
        log("bench: single products at 2^16, 2^20 and 2^29 bits")
        out["sizes"] = bench_sizes(P, ctx)
    if not args.no_w128:
        log("bench: the same product with 128-bit words over TGF(2^256)")
        out["w128"] = bench_w128(P, a, b, n, c, args.steps, args.warmup, args.tune)
    if not args.no_simple:
        log("bench: the same product by the simple variant (polynomial basis, Cantor points)")
        out["simple"] = bench_variant(P, "simple", a, b, n, c, args.steps, args.warmup, not args.no_sizes)
    if not args.no_frobenius:
        log("bench: the same product by the Frobenius partition (App. C)")
        out["frobenius"] = bench_variant(P, "frobenius", a, b, n, c, args.steps, args.warmup, not args.no_sizes)
    if not args.no_batch:
        log(f"bench: batched products ({args.batch_jobs} jobs)")
        out["batched"] = bench_batched(ctx, args.batch_jobs)
    if not args.no_serve:
        log(f"bench: serving ({args.serve_requests} requests per stream)")
        out["serving"] = bench_serving(ctx, args.serve_requests)
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on the whole product")
        out["cpu_baseline"] = cpu_baseline(args.workload, n, seeds)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
