"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars (stated per test): normals bit-exact; eigenvalues to 1e-12 of the
largest; masks equal up to ties within 1e-12; FP64 fields to 1e-11 of
max|Z|; mixed fields to 1e-5 of max|Z|; FP64 QoI to 1e-9 relative; mixed
QoI to 1e-6 relative (field rounding to float dominates; CG runs to
||r|| <= 1e-10 ||r0|| in double on both paths); the Y of a pair level also
to 1e-9 (FP64) / 2e-6 (mixed) of max|Y|, floored at 1% of max|Q_f|.
"""

import numpy as np
import pytest

from oracle import embedding as oem, fem as ofem, normals as onm, sampler as osm
from paper_2306_13493_amd import workloads as W
from tests.inputs import lognormal_k

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


def mkplan(ctx, ces, w):
    return ctx.plan(ces.level_desc(**w))


def oracle_plan(w):
    return osm.Plan(W.to_oracle(w))


# ------------------------------------------------------------------ normals
@pytest.mark.parametrize("seed,q,stream,first,count", [
    (0, 0, 0, 0, 4096),
    (12345678901, 7, 3, 1000, 5000),
    (2 ** 63 + 5, 2 ** 40 + 3, 9, 2 ** 31, 3000),
])
def test_normals_bit_exact(ces, seed, q, stream, first, count):
    g = ces.normals(seed, q, stream, first, count).cpu().numpy()
    e = np.arange(first, first + count, dtype=np.uint64)
    g0, g1 = onm.normals(seed, q, stream, e)
    ref = np.stack([g0, g1], axis=1)
    assert np.array_equal(g.view(np.uint64), ref.view(np.uint64))


# ----------------------------------------------------------- eigenvalues
EIG_CASES = {
    "c1_clamp": W.C1,
    "c2_grow": W.C2,
    "grow_pad_euclid": dict(cov="matern", nu=0.5, lam=0.3, m=32, psd="grow"),
    "grow_pad_inf": dict(cov="matern", nu=1.5, lam=0.3, m=32, psd="grow", period="inf"),
    "sepexp": dict(cov="sepexp", lam=0.1, m=32),
    "c3_l2_smoothed": W.c3_level(2),
    "c3_l4_finest": W.c3_level(4),
    # general nu (Bessel K from the device routine), periodised
    "matern_nu23_grow": dict(cov="matern", nu=2.3, lam=0.2, m=32, psd="grow"),
    "matern_nu1_grow_inf": dict(cov="matern", nu=1.0, lam=0.25, m=32, psd="grow", period="inf"),
    "sepexp_grow_m64": dict(cov="sepexp", lam=0.3, m=64, psd="grow"),
    # large embeddings: C5 (n = 4096) and a padded nu = 1 pair level (n = 1536)
    "c5_n4096": W.C5,
    "nu1_grow_m512_pair": dict(cov="matern", nu=1.0, lam=0.3, m=512, level="pair"),
}


def masks_agree(mg, mo, lam, tol=1e-12):
    if np.array_equal(mg, mo):
        return True
    diff = mg != mo
    lmax = lam.max()
    # disagreement only among values tied with the kept/dropped boundary
    boundary = lam[(mo == 0)].max() if (mo == 0).any() else 0.0
    return bool(np.all(np.abs(lam[diff] - boundary) <= tol * lmax))


@pytest.mark.parametrize("name", list(EIG_CASES))
def test_eigenvalues_and_masks(ctx, ces, name):
    w = EIG_CASES[name]
    p = mkplan(ctx, ces, w)
    o = oracle_plan(w)
    assert p.info.n == o.n and p.info.J == o.J
    assert p.info.n_clamped == o.info["n_clamped"]
    lam = p.eigenvalues()
    lmax = o.lam.max()
    assert np.max(np.abs(lam - o.lam)) <= 1e-12 * lmax
    assert abs(p.info.lam_min - o.info["lam_min"]) <= 1e-12 * lmax
    mf, mc = p.masks()
    assert masks_agree(mf, o.keep_f.astype(np.uint8), o.lam)
    if w.get("level") == "pair":
        assert masks_agree(mc, o.keep_c.astype(np.uint8), o.lam)


# ----------------------------------------------------------------- fields
FIELD_CASES = {
    "pair_single": dict(cov="matern", nu=1.0, lam=0.1, m=32, level="single"),
    "pair_level_smoothed_nf2": dict(cov="matern", nu=0.5, lam=0.03, m=16, level="pair", tau_fine=0, tau_coarse=-1),
    "pair_level_smoothed_nf1": dict(cov="matern", nu=0.5, lam=0.03, m=32, level="pair", tau_fine=-1, tau_coarse=-1),
    "hartley_pair_level": dict(cov="matern", nu=1.5, lam=0.2, m=16, level="pair", field="hartley"),
    "padded_n96": dict(cov="matern", nu=0.5, lam=0.3, m=32, level="pair", stream=3),
    "c2_size": dict(W.C2),
    # coarse field from the coarse mesh's own embedding (EMBED coupling)
    "embed_smoothed": dict(cov="matern", nu=1.5, lam=0.2, m=16, level="pair", tau_fine=-1, tau_coarse=-1,
                           coupling="embed"),
    "embed_finest_form_hartley": dict(cov="matern", nu=1.0, lam=0.1, m=64, level="pair", tau_fine=0,
                                      tau_coarse=-1, coupling="embed", field="hartley", stream=2),
    "embed_padded": dict(cov="matern", nu=0.5, lam=0.3, m=32, level="pair", coupling="embed", stream=3),
}


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("mixed", 1e-5)])
@pytest.mark.parametrize("name", list(FIELD_CASES))
def test_field_parity(ctx, ces, name, prec, tol):
    w = dict(FIELD_CASES[name], precision=prec)
    p = mkplan(ctx, ces, w)
    o = oracle_plan(w)
    for i in (0, 1, 5):
        zf, zc = p.field(seed=7, sample=i)
        rf, rc = o.fields(7, i)
        scale = np.abs(rf).max()
        assert np.max(np.abs(zf.cpu().numpy() - rf)) <= tol * scale, (name, i)
        if rc is not None:
            assert np.max(np.abs(zc.cpu().numpy() - rc)) <= tol * scale, (name, i)


# ------------------------------------------------------------------ solve
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
# single-level plans visit multigrid level 1 twice when it is a whole level:
# Dirichlet m = 64 (FP64), 128 and 256 (mixed) take that path
@pytest.mark.parametrize("bc,m", [("dirichlet0", 32), ("flowcell", 32), ("dirichlet0", 64), ("flowcell", 128),
                                  ("dirichlet0", 128), ("dirichlet0", 256)])
def test_solve_parity(ctx, ces, prec, bc, m):
    w = dict(cov="matern", nu=1.0, lam=0.2, m=m, bc=bc, precision=prec, cg_rtol=1e-12)
    p = mkplan(ctx, ces, w)
    k = lognormal_k(m, 3, seed=m + (bc == "flowcell"))
    u, it = p.solve(torch.from_numpy(k).cuda())
    u = u.cpu().numpy()
    it = it.cpu().numpy()
    assert np.all(it > 0) and np.all(it < 60), it
    # the mixed path stores k in float: the oracle solves with the same k
    kref = k if prec == "fp64" else k.astype(np.float32).astype(np.float64)
    for s in range(k.shape[0]):
        ref, _, _ = ofem.solve(kref[s], m, ofem.FLOWCELL if bc == "flowcell" else ofem.DIRICHLET0)
        assert np.max(np.abs(u[s] - ref)) <= 1e-9 * np.abs(ref).max(), (s, it[s])


# ---------------------------------------------------------- level samples
SAMPLE_CASES = {
    "c1": (dict(W.C1), 64),
    "c1_mixed": (dict(W.C1, precision="mixed"), 64),
    "pair_smoothed_nf2": (dict(cov="matern", nu=0.5, lam=0.03, m=16, level="pair", tau_fine=0,
                               tau_coarse=-1, stream=4), 24),
    "pair_smoothed_nf1": (dict(cov="matern", nu=0.5, lam=0.03, m=32, level="pair", tau_fine=-1,
                               tau_coarse=-1, stream=2), 16),
    "hartley": (dict(cov="matern", nu=1.0, lam=0.1, m=16, field="hartley"), 9),
    "flowcell_outflux": (dict(cov="matern", nu=1.5, lam=0.05, sigma2=2.0, m=32, bc="flowcell",
                              qoi="outflux"), 8),
    "point_qoi_pair": (dict(cov="sepexp", lam=0.3, m=32, level="pair", qoi="point"), 8),
    "l2_qoi": (dict(cov="matern", nu=1.5, lam=0.03, m=64, qoi="l2"), 6),
    # tiled solves of QoIs that are linear in u accumulate the QoI over the
    # CG steps instead of keeping the iterate.  The outflux is a boundary
    # functional of A u: a residual of 1e-10 of r0 (the flow cell's r0 is
    # large next to x1 = 0) bounds it only to a few 1e-9, so this case
    # solves to 1e-12 and checks the accumulation at the 1e-9 bar.
    "outflux_tiled_pair": (dict(cov="matern", nu=1.5, lam=0.05, sigma2=2.0, m=128, level="pair",
                                bc="flowcell", qoi="outflux", cg_rtol=1e-12), 4),
    "point_tiled_upper_triangle": (dict(cov="sepexp", lam=0.3, m=128, level="pair", qoi="point",
                                        qoi_x=0.3, qoi_y=0.71), 4),
    # EMBED coupling: smoothed level (small meshes) and the finest-level
    # form on a tiled mesh
    "embed_smoothed_small": (dict(cov="matern", nu=1.5, lam=0.2, m=16, level="pair", tau_fine=-1,
                                  tau_coarse=-1, coupling="embed"), 12),
    "embed_finest_tiled": (dict(cov="matern", nu=1.0, lam=0.1, m=128, level="pair", tau_fine=0,
                                tau_coarse=-1, coupling="embed"), 4),
    "integral_flowcell_tiled": (dict(cov="matern", nu=1.0, lam=0.1, m=64, bc="flowcell"), 6),
}


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-6)])
@pytest.mark.parametrize("name", list(SAMPLE_CASES))
def test_level_samples(ctx, ces, name, prec, tol):
    w, count = SAMPLE_CASES[name]
    w = dict(w, precision=prec)
    p = mkplan(ctx, ces, w)
    out = p.sample(seed=3, first=1, count=count)
    torch.cuda.synchronize()
    y = out["y"].cpu().numpy()
    yf = out["q_fine"].cpu().numpy()
    st = out["status"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    assert np.all(st == 0) and np.all(it > 0)
    o = oracle_plan(w)
    ref = np.array([o.sample(3, 1 + t) for t in range(count)])
    scale = np.abs(ref[:, 1]).max()
    assert np.max(np.abs(yf - ref[:, 1])) <= tol * scale
    assert np.max(np.abs(y - ref[:, 0])) <= tol * scale
    if w.get("level") == "pair":
        # Y = Q_f - Q_c on its own scale, floored at 1% of the QoI scale
        ybar = 2e-6 if prec == "mixed" else 1e-9
        yscale = max(np.abs(ref[:, 0]).max(), 1e-2 * scale)
        assert np.max(np.abs(y - ref[:, 0])) <= ybar * yscale


def test_batch_independence(ctx, ces):
    w = dict(cov="matern", nu=0.5, lam=0.05, m=32, level="pair", tau_fine=-1, tau_coarse=-1)
    p = mkplan(ctx, ces, w)
    a = p.sample(seed=11, first=0, count=20)["y"].cpu().numpy()
    b = p.sample(seed=11, first=5, count=7)["y"].cpu().numpy()
    c = p.sample(seed=11, first=19, count=1)["y"].cpu().numpy()
    assert np.array_equal(a[5:12], b) and a[19] == c[0]
    d = p.sample(seed=12, first=0, count=20)["y"].cpu().numpy()
    assert not np.array_equal(a, d)


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-6), ("fp64", 1e-9)])
def test_c2_full_size_sampled(ctx, ces, prec, tol):
    w = dict(W.C2, precision=prec)
    p = mkplan(ctx, ces, w)
    out = p.sample(seed=0, first=0, count=256)
    torch.cuda.synchronize()
    y = out["y"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    assert np.all(out["status"].cpu().numpy() == 0)
    print("C2 %s iterations: min %d max %d mean %.2f" % (prec, it.min(), it.max(), it.mean()))
    o = oracle_plan(w)
    for i in (0, 1, 255):
        ref = o.sample(0, i)[0]
        assert abs(y[i] - ref) <= tol * abs(ref), (i, y[i], ref)


def test_c5_full_size_field_and_flux_balance(ctx, ces):
    """C5 at its full size (2049^2 vertices, flow cell, outflow QoI): the
    field of a sample against the oracle's; the solution of the device
    solver satisfies the discrete flux balance of the flow cell (the
    operator's rows sum to zero, so the boundary fluxes add up to the
    integral of f = 1) and reproduces the sampled outflow QoI.  The
    operator is the oracle's element-by-element assembly on the float
    coefficients the mixed solver uses."""
    from oracle import fem as ofem2, qoi as oqoi
    w = W.C5
    m = w["m"]
    p = mkplan(ctx, ces, w)
    o = oracle_plan(w)
    assert (p.info.n, p.info.J) == (o.n, o.J) == (4096, 0)
    zf, _ = p.field(0, 0)
    z = zf.cpu().numpy()
    zr, _ = o.fields(0, 0)
    assert np.max(np.abs(z - zr)) <= 1e-5 * np.max(np.abs(zr))
    y = p.sample(0, 0, 2)["y"].cpu().numpy()
    k = np.exp(z).astype(np.float32).astype(np.float64)
    u, it = p.solve(torch.from_numpy(k).reshape(1, m + 1, m + 1).to("cuda"))
    assert int(it.cpu()[0]) > 0
    uu = u.cpu().numpy().reshape(-1)
    A, b = ofem2.assemble(k, m, 1.0)
    res = b - A @ uu
    i = np.arange((m + 1) ** 2) % (m + 1)
    influx, outflux = res[i == 0].sum(), res[i == m].sum()
    free = (i > 0) & (i < m)
    # CG stops at ||r|| <= 1e-10 ||r0|| (r0 of the Dirichlet lifting)
    r0 = b - A @ (i == 0).astype(np.float64)
    assert np.linalg.norm(res[free]) <= 1e-9 * np.linalg.norm(r0[free])
    # rows (and columns) of A sum to zero: the boundary fluxes balance the
    # load up to the sum of the free-node residuals
    assert abs(b.sum() - 1.0) <= 1e-12
    assert abs(influx + outflux - b.sum()) <= 1e-7
    q = oqoi.outflux(uu, m, A, b)
    assert abs(q - outflux) <= 1e-12 * abs(q)
    assert abs(y[0] - q) <= 1e-6 * abs(q)


@pytest.mark.timeout(400)   # the oracle's normals and DFT at 8192^2 take about a minute of CPU
def test_largest_mesh(ctx, ces):
    """The largest mesh a descriptor allows (4097^2 vertices, embedding
    8192^2, separable exponential: no padding): the field of a sample
    against the oracle's, and converged solves whose QoI agrees between
    the mixed and the FP64 path to the mixed bar.  Every kernel runs at
    its largest index range."""
    w = dict(cov="sepexp", lam=0.05, m=4096)
    p = mkplan(ctx, ces, w)
    o = oracle_plan(w)
    assert (p.info.n, p.info.J) == (o.n, o.J) == (8192, 0)
    zf, _ = p.field(0, 1)
    z = zf.cpu().numpy()
    zr, _ = o.fields(0, 1)
    assert np.max(np.abs(z - zr)) <= 1e-5 * np.max(np.abs(zr))
    del zf, z, zr, o
    out = p.sample(0, 0, 2)
    p64 = mkplan(ctx, ces, dict(w, precision="fp64"))
    out64 = p64.sample(0, 0, 2)
    torch.cuda.synchronize()
    for r in (out, out64):
        assert np.all(r["status"].cpu().numpy() == 0)
        it = r["iters"].cpu().numpy()
        assert np.all((it > 0) & (it < 60)), it
    y, y64 = out["y"].cpu().numpy(), out64["y"].cpu().numpy()
    assert np.max(np.abs(y - y64)) <= 1e-6 * np.max(np.abs(y64))


@pytest.mark.timeout(400)   # the oracle's normals and two DFTs at 4096^2 take about half a minute
def test_two_field_pair_level_at_4096(ctx, ces):
    """The largest pair level that draws both fields from one xi (the finest
    level of the smoothed estimator at 2049^2, embedding 4096^2): its DFT
    passes run one line per workgroup per field, 32 values per thread.  Both
    fields of a sample against the oracle's, and converged level samples
    whose Y agrees between the mixed and the FP64 path to the mixed bar."""
    w = dict(cov="sepexp", lam=0.05, m=2048, level="pair", tau_fine=0, tau_coarse=-1)
    p = mkplan(ctx, ces, w)
    o = oracle_plan(w)
    assert (p.info.n, p.info.J) == (o.n, o.J) == (4096, 0)
    zf, zc = p.field(0, 3)
    rf, rc = o.fields(0, 3)
    scale = np.abs(rf).max()
    assert np.max(np.abs(zf.cpu().numpy() - rf)) <= 1e-5 * scale
    assert np.max(np.abs(zc.cpu().numpy() - rc)) <= 1e-5 * scale
    del zf, zc, rf, rc, o
    out = p.sample(0, 0, 2)
    out64 = mkplan(ctx, ces, dict(w, precision="fp64")).sample(0, 0, 2)
    torch.cuda.synchronize()
    for r in (out, out64):
        assert np.all(r["status"].cpu().numpy() == 0)
    y, y64 = out["y"].cpu().numpy(), out64["y"].cpu().numpy()
    yq = out64["q_fine"].cpu().numpy()
    assert np.max(np.abs(y - y64)) <= 1e-6 * np.max(np.abs(yq))


def test_two_field_pair_level_beyond_4096_is_rejected(ctx, ces):
    # the finest level of the smoothed estimator at m = 4096 draws two fields
    w = dict(cov="sepexp", lam=0.05, m=4096, level="pair", tau_fine=0, tau_coarse=-1)
    with pytest.raises(ces.CesError):
        mkplan(ctx, ces, w)


def test_embed_plan_info_and_coarse_embedding(ctx, ces):
    w = dict(cov="matern", nu=0.5, lam=0.3, m=32, level="pair", coupling="embed", tau_coarse=-1)
    p = mkplan(ctx, ces, w)
    o = oracle_plan(w)
    # 32^2 needs padding (n = 96), the 16^2 coarse mesh does not (n = 32)
    assert (p.info.n, p.info.n_coarse) == (o.n, o.coarse_plan.n) == (96, 32)
    assert p.info.tau_coarse == o.coarse_plan.tau_f == o.coarse_plan.n
    # the coarse mask hook returns the coarse embedding's mask
    mf, mc = p.masks()
    assert mf.shape == (96, 96) and mc.shape == (32, 32)
    assert int((mc == 0).sum()) == o.coarse_plan.tau_f and int((mf == 0).sum()) == 0
    r = mkplan(ctx, ces, dict(w, coupling="restrict"))
    assert r.info.n_coarse == r.info.n
    with pytest.raises(ces.CesError):
        mkplan(ctx, ces, dict(w, level="single"))


# ------------------------------------------------------------- edge cases
def test_zero_count_is_a_no_op(ctx, ces):
    p = mkplan(ctx, ces, dict(cov="matern", nu=1.0, lam=0.1, m=64, level="pair"))
    out = p.sample(seed=1, first=5, count=0)
    torch.cuda.synchronize()
    assert out["y"].numel() == 0
    # the plan still samples normally afterwards
    y = p.sample(seed=1, first=5, count=3)["y"].cpu().numpy()
    yr = np.array([oracle_plan(dict(cov="matern", nu=1.0, lam=0.1, m=64, level="pair")).sample(1, 5 + t)[0]
                   for t in range(3)])
    assert np.max(np.abs(y - yr)) <= 1e-6 * np.max(np.abs(yr))


@pytest.mark.parametrize("m,level", [(16, "single"), (64, "pair")])
def test_every_eigenvalue_dropped_gives_the_constant_coefficient_qoi(ctx, ces, m, level):
    # tau = s: a zero field, k = exp(0) = 1 on every sample (Algorithm 2 with
    # all eigenvalues dropped); the QoIs equal the deterministic solve's
    from oracle import smoothing as osmo
    w = dict(cov="matern", nu=1.5, lam=0.2, m=m, level=level, precision="fp64")
    probe = mkplan(ctx, ces, w)
    s = probe.info.n ** 2
    probe.close()
    p = mkplan(ctx, ces, dict(w, tau_fine=s, tau_coarse=s))
    out = p.sample(seed=2, first=0, count=5)
    qf = out["q_fine"].cpu().numpy()
    d = W.to_oracle(w)
    assert np.allclose(qf, osmo.constant_coefficient_qoi(d), rtol=1e-9, atol=0)
    if level == "pair":
        qc = out["q_coarse"].cpu().numpy()
        assert np.allclose(qc, osmo.constant_coefficient_qoi(dict(d, m=m // 2)), rtol=1e-9, atol=0)


def test_sample_indices_beyond_32_bits(ctx, ces):
    # the pair index q = i / 2 spans two counter words
    w = dict(cov="matern", nu=1.0, lam=0.1, m=32, level="pair", precision="fp64")
    p = mkplan(ctx, ces, w)
    first = 2 ** 33 + 5
    y = p.sample(seed=7, first=first, count=4)["y"].cpu().numpy()
    o = oracle_plan(w)
    yr = np.array([o.sample(7, first + t)[0] for t in range(4)])
    scale = max(abs(o.sample(7, first)[1]), 1e-12)
    assert np.max(np.abs(y - yr)) <= 1e-9 * scale


# ------------------------------------------------------ multigrid cycle
@pytest.mark.parametrize("w", [
    dict(cov="matern", nu=1.0, lam=0.1, m=256, precision="mixed"),
    dict(cov="matern", nu=1.0, lam=0.1, m=128, level="pair", precision="fp64", stream=3),
    dict(cov="matern", nu=1.0, lam=0.2, m=128, bc="flowcell", qoi="outflux", precision="mixed", cg_rtol=1e-12),
    # a field the coarse levels do not resolve (length scale below 8 cells): AUTO keeps the V-cycle
    dict(cov="matern", nu=1.5, lam=0.01, m=256, precision="mixed", stream=1),
])
def test_cycle_choices_agree_with_oracle(ctx, ces, w):
    # the cycle changes the iterations, not the solution: V, W1 and the
    # automatic choice all meet the level-sample bar against the oracle
    count = 4
    o = oracle_plan(w)
    ref = np.array([o.sample(5, t)[0] for t in range(count)])
    tol = 1e-9 if w["precision"] == "fp64" else 1e-6
    its = {}
    for cyc in ("v", "w1", "auto"):
        p = mkplan(ctx, ces, dict(w, cycle=cyc))
        out = p.sample(seed=5, first=0, count=count)
        torch.cuda.synchronize()
        assert np.all(out["status"].cpu().numpy() == 0)
        y = out["y"].cpu().numpy()
        assert np.max(np.abs(y - ref)) <= tol * max(np.abs(ref).max(), 1e-3), cyc
        its[cyc] = out["iters"].cpu().numpy().mean()
    if w["lam"] == 0.01:
        assert its["auto"] == its["v"]
        return
    assert its["w1"] <= its["v"]
    if w["m"] == 256:
        assert its["w1"] < its["v"] and its["auto"] == its["w1"]


def test_cycle_rejects_unknown_value(ctx, ces):
    d = ces.level_desc(cov="matern", nu=1.0, lam=0.1, m=64)
    d.mg_cycle = 7
    with pytest.raises(ces.CesError):
        ctx.plan(d)
