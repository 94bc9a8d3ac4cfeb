"""GPU tests of the serving loop (ces_server_*).

Bars: a served request's Y equals ces_sample of the same descriptor, seed
and range computed alone, bit for bit (the alone-versus-mix test: results
depend only on (plan, seed, sample), never on what else is being served);
served results match the oracle at the mixed-precision bar 1e-6; failure,
admission and accounting behave as documented.
"""

import numpy as np
import pytest

from oracle import sampler as osm
from paper_2306_13493_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ces():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_13493_amd as ces
    ces.load()
    return ces


@pytest.fixture(scope="module")
def ctx(ces):
    return ces.Context(0)


def mix():
    a = dict(cov="matern", nu=0.5, lam=0.05, m=16, level="single")
    b = dict(cov="matern", nu=1.0, lam=0.2, m=64, level="pair")
    c = dict(cov="matern", nu=1.5, lam=0.1, m=32, level="pair", tau_fine=-1, tau_coarse=-1)
    d = dict(cov="sepexp", lam=0.3, m=128, level="pair", qoi="point")
    e = dict(cov="matern", nu=2.3, lam=0.25, m=32, psd="grow")
    f = dict(W.c3_level(4))
    # a pair level whose coarse term comes from the coarse mesh's own embedding
    g = dict(cov="matern", nu=1.0, lam=0.1, m=64, level="pair", tau_fine=-1, tau_coarse=-1, coupling="embed")
    # (desc, seed, first, count): repeated descriptors share a plan
    return [(a, 1, 0, 37), (b, 2, 5, 20), (c, 3, 0, 64), (a, 4, 10, 9), (d, 5, 0, 7), (e, 6, 1, 30),
            (b, 7, 0, 3), (f, 8, 0, 12), (a, 1, 37, 11), (g, 9, 3, 21)]


def alone(ctx, ces, w, seed, first, count):
    p = ctx.plan(ces.level_desc(**w))
    out = p.sample(seed, first, count)
    torch.cuda.synchronize()
    return out["y"].cpu().numpy(), out["status"].cpu().numpy()


def test_served_equals_alone_bitwise(ctx, ces):
    srv = ces.Server(ctx, max_inflight=4)
    try:
        reqs = mix()
        ids = [srv.submit(w, s, f, c) for (w, s, f, c) in reqs]
        srv.drain()
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0
        for rid, (w, s, f, c) in zip(ids, reqs):
            state, lat = srv.poll(rid)
            assert state == 2 and lat > 0
            y, status = srv.result(rid)
            ya, sa = alone(ctx, ces, w, s, f, c)
            assert np.array_equal(y.view(np.uint64), ya.view(np.uint64)), (w, s, f, c)
            assert np.array_equal(status, sa) and np.all(status == 0)
    finally:
        srv.close()


def test_served_results_match_oracle(ctx, ces):
    srv = ces.Server(ctx)
    try:
        w = dict(cov="matern", nu=1.0, lam=0.2, m=32, level="pair")
        rid = srv.submit(w, 11, 0, 6)
        srv.drain()
        y, _ = srv.result(rid)
        ref = osm.Plan(W.to_oracle(w))
        yr = np.array([ref.sample(11, i)[0] for i in range(6)])
        assert np.max(np.abs(y - yr)) <= 1e-6 * np.max(np.abs(yr))
    finally:
        srv.close()


def test_tight_budget_limits_admitted_memory(ctx, ces):
    w = dict(cov="matern", nu=0.5, lam=0.1, m=128, level="pair")
    budget = 32 << 20
    srv = ces.Server(ctx, mem_budget=budget, max_inflight=8)
    try:
        ids = [srv.submit(dict(w, lam=0.1 + 0.01 * i), i, 0, 8) for i in range(5)]
        srv.drain()
        st = srv.stats()
        assert st["completed"] == 5 and st["failed"] == 0
        assert st["mem_peak"] <= budget
        for i, rid in enumerate(ids):
            ya, _ = alone(ctx, ces, dict(w, lam=0.1 + 0.01 * i), i, 0, 8)
            assert np.array_equal(srv.result(rid)[0].view(np.uint64), ya.view(np.uint64))
    finally:
        srv.close()


def test_failed_request_does_not_disturb_others(ctx, ces):
    srv = ces.Server(ctx)
    try:
        bad = dict(W.C1, psd="fail")              # negative eigenvalues at n = 2m
        good = dict(cov="matern", nu=0.5, lam=0.05, m=16)
        r1 = srv.submit(good, 1, 0, 5)
        r2 = srv.submit(bad, 1, 0, 5)
        r3 = srv.submit(good, 2, 0, 5)
        srv.drain()
        assert srv.poll(r2)[0] == -2               # CES_ERR_NOT_PSD
        assert srv.poll(r1)[0] == 2 and srv.poll(r3)[0] == 2
        st = srv.stats()
        assert st["failed"] == 1 and st["completed"] == 2 and st["samples_done"] == 10
        ya, _ = alone(ctx, ces, good, 2, 0, 5)
        assert np.array_equal(srv.result(r3)[0].view(np.uint64), ya.view(np.uint64))
    finally:
        srv.close()


def test_c4_trace_prefix_alone_vs_mix(ctx, ces):
    # first requests of the serving workload, submitted back to back
    full = W.c4_trace(duration_s=2.0)
    trace = [r for r in full if r["w"]["m"] <= 256][:10]
    # and the first large levels (grown embeddings, radix-3 DFT sizes)
    trace += [r for r in full if r["w"]["m"] >= 512][:2]
    srv = ces.Server(ctx, max_inflight=16)
    try:
        ids = [srv.submit(r["w"], r["seed"], r["first"], r["count"]) for r in trace]
        srv.drain()
        for rid, r in zip(ids, trace):
            ya, _ = alone(ctx, ces, r["w"], r["seed"], r["first"], r["count"])
            assert np.array_equal(srv.result(rid)[0].view(np.uint64), ya.view(np.uint64))
    finally:
        srv.close()


def test_requests_overlap_on_the_device(ctx, ces):
    # continuous batching: short requests submitted while a long one runs
    # are admitted next to it and complete before it does
    import time
    srv = ces.Server(ctx, max_inflight=8)
    try:
        big = dict(cov="matern", nu=1.0, lam=0.1, m=1024, level="pair")
        small = [dict(cov="matern", nu=0.5, lam=0.05, m=16, stream=1 + i) for i in range(4)]
        ra = srv.submit(big, 1, 0, 256)
        t0 = time.time()
        while srv.poll(ra)[0] == 0:
            assert time.time() - t0 < 60
        rs = [srv.submit(w, 2, 0, 8) for w in small]
        max_admitted, overtaken = 0, 0
        while True:
            st = srv.stats()
            max_admitted = max(max_admitted, st["admitted"])
            states = [srv.poll(r)[0] for r in rs]
            big_state = srv.poll(ra)[0]
            overtaken = max(overtaken, sum(s == 2 for s in states) if big_state == 1 else 0)
            if big_state == 2 and all(s == 2 for s in states):
                break
            assert big_state >= 0 and min(states) >= 0
            assert time.time() - t0 < 120
        srv.drain()
        assert max_admitted >= 2
        assert overtaken >= 1
        for r, w in zip(rs, small):
            ya, _ = alone(ctx, ces, w, 2, 0, 8)
            assert np.array_equal(srv.result(r)[0].view(np.uint64), ya.view(np.uint64))
    finally:
        srv.close()
