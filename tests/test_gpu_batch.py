"""GPU tests of the batch scheduler (ces_sample_batch, schedules, autotuner).

Bar: bit-exact.  A sample's arithmetic is fixed by its plan, so any batch
composition, schedule or lane interleaving must reproduce ces_sample on the
request alone to the last bit; parity of ces_sample itself against the
oracle is covered in test_gpu_parity.
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


# the C3 estimator's levels (m = 16 .. 256) at reduced sample counts
C3_SMALL_N = [600, 300, 120, 40, 10]


@pytest.fixture(scope="module")
def c3_plans(ctx, ces):
    return [ctx.plan(ces.level_desc(**W.c3_level(l))) for l in range(5)]


def bits(t):
    return t.cpu().numpy().view(np.uint64)


def alone(plans, seeds, firsts, counts):
    outs = []
    for p, s, f, c in zip(plans, seeds, firsts, counts):
        outs.append(p.sample(s, f, c))
    torch.cuda.synchronize()
    return outs


def assert_same(a, b):
    for k in ("y", "q_fine", "q_coarse"):
        assert np.array_equal(bits(a[k]), bits(b[k])), k
    for k in ("iters", "status"):
        assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()), k


def test_c3_batch_equals_alone(ctx, c3_plans):
    firsts = [3, 0, 1, 7, 2]          # odd starts split PAIR units
    seeds = [0] * 5
    ref = alone(c3_plans, seeds, firsts, C3_SMALL_N)
    got = ctx.sample_batch([(p, s, f, c) for p, s, f, c in zip(c3_plans, seeds, firsts, C3_SMALL_N)])
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert_same(a, b)
        assert np.all(b["status"].cpu().numpy() == 0)


def test_mixed_requests_same_plan_and_zero_count(ctx, c3_plans):
    p0, p2 = c3_plans[0], c3_plans[2]
    reqs = [(p2, 5, 11, 33), (p0, 1, 0, 50), (p2, 9, 0, 0), (p0, 1, 50, 17), (p2, 5, 44, 8)]
    got = ctx.sample_batch(reqs)
    ref = alone([r[0] for r in reqs if r[3] > 0], [r[1] for r in reqs if r[3] > 0],
                [r[2] for r in reqs if r[3] > 0], [r[3] for r in reqs if r[3] > 0])
    torch.cuda.synchronize()
    nz = [g for g, r in zip(got, reqs) if r[3] > 0]
    for a, b in zip(ref, nz):
        assert_same(a, b)
    # the contiguous split of one range equals the range in one request
    whole = p0.sample(1, 0, 67)
    torch.cuda.synchronize()
    y = np.concatenate([got[1]["y"].cpu().numpy(), got[3]["y"].cpu().numpy()])
    assert np.array_equal(y.view(np.uint64), bits(whole["y"]))


@pytest.mark.parametrize("sched", [(1, 0, 0, 0), (3, 1, 0, 0), (4, 2, 64, 0), (2, 0, 30, 0),
                                   (2, 0, 0, 1), (3, 0, 45, 1), (1, 1, 0, 1)])
def test_schedules_do_not_change_results(ctx, c3_plans, sched):
    # graphs = 1 replays captured iterations many times per solve and across
    # chunks of different sizes (45, 45, 30 at level 2), with eager work in
    # between; every replay must match the eagerly launched iterations
    reqs = [(p, 0, 0, c) for p, c in zip(c3_plans, C3_SMALL_N)]
    ref = ctx.sample_batch(reqs)
    torch.cuda.synchronize()
    old = ctx.schedule
    try:
        ctx.schedule = sched
        assert ctx.schedule[:2] == sched[:2] and ctx.schedule[3] == sched[3]
        got = ctx.sample_batch(reqs)
        torch.cuda.synchronize()
    finally:
        ctx.schedule = old
    for a, b in zip(ref, got):
        assert_same(a, b)


def test_autotune_picks_valid_schedule(ctx, c3_plans):
    reqs = [(p, 0, 0, c) for p, c in zip(c3_plans, C3_SMALL_N)]
    ref = ctx.sample_batch(reqs)
    torch.cuda.synchronize()
    old = ctx.schedule
    try:
        (depth, lanes, chunk, graphs), ms, outs = ctx.autotune(reqs)
        torch.cuda.synchronize()
        assert 1 <= depth <= 4 and lanes >= 0 and chunk >= 0 and graphs in (0, 1) and ms > 0
        assert ctx.schedule == (depth, lanes, chunk, graphs)
    finally:
        ctx.schedule = old
    for a, b in zip(ref, outs):
        assert_same(a, b)


def test_batch_level_samples_match_oracle(ctx, c3_plans):
    # small-mesh single launch (m = 16, 32) and tiled (m = 64) in one batch
    counts = [6, 6, 4]
    got = ctx.sample_batch([(c3_plans[l], 0, 0, counts[l]) for l in range(3)])
    torch.cuda.synchronize()
    for l in range(3):
        ref = osm.Plan(W.to_oracle(W.c3_level(l)))
        yr = np.array([ref.sample(0, i)[0] for i in range(counts[l])])
        y = got[l]["y"].cpu().numpy()
        assert np.max(np.abs(y - yr)) <= 1e-6 * np.max(np.abs(yr)), l


def test_busy_plan_in_two_requests_is_serialised(ctx, c3_plans):
    # one plan in several requests is fine (one lane, run in order)
    p = c3_plans[1]
    got = ctx.sample_batch([(p, 2, 0, 20), (p, 3, 0, 20)])
    torch.cuda.synchronize()
    a = p.sample(2, 0, 20)
    b = p.sample(3, 0, 20)
    torch.cuda.synchronize()
    assert_same(got[0], a)
    assert_same(got[1], b)


@pytest.mark.parametrize("m,level,qoi", [(32, "single", "l2"), (32, "pair", "l2"), (64, "pair", "integral")])
def test_iteration_cap_reports_nonconvergence(ctx, ces, m, level, qoi):
    # small-mesh and tiled solves agree on the status convention (at m = 32
    # only a QoI that is not linear in u runs the iterative small-mesh solve)
    plan = ctx.plan(ces.level_desc(cov="matern", nu=0.5, lam=0.05, m=m, level=level, qoi=qoi, cg_max_iter=2))
    out = plan.sample(0, 0, 6)
    torch.cuda.synchronize()
    assert np.all(out["status"].cpu().numpy() == -4)
    assert np.all(out["iters"].cpu().numpy() == -2)


@pytest.mark.parametrize("m,level,qoi", [(8, "single", "integral"), (16, "pair", "l2"), (16, "single", "point"),
                                         (32, "single", "integral"), (32, "pair", "outflux")])
def test_direct_solves_ignore_the_iteration_cap(ctx, ces, m, level, qoi):
    # meshes with m <= 16, and m <= 32 for a QoI linear in u, are solved
    # directly: one "iteration", never capped
    bc = "flowcell" if qoi == "outflux" else "dirichlet0"
    plan = ctx.plan(ces.level_desc(cov="matern", nu=0.5, lam=0.05, m=m, level=level, qoi=qoi, bc=bc, cg_max_iter=1))
    out = plan.sample(0, 0, 6)
    torch.cuda.synchronize()
    assert np.all(out["status"].cpu().numpy() == 0)
    assert np.all(out["iters"].cpu().numpy() == 1)
