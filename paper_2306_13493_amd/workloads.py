"""Synthetic workloads of the benchmark and the tests (pure data).

Each workload is a dict of level-descriptor fields plus sample counts and
seeds.  The same dict drives the HIP path (level_desc(**kw)) and, in the
tests, the CPU oracle (to_oracle).  No arithmetic of the method lives here.

C1  plain CE, Matern nu=1/2, sigma2=1, lambda=0.3, 33^2 vertices, fixed
    64^2 embedding (negative eigenvalues clamped), 64 samples, FP64,
    integral of u, single level.
C2  single-level MC, Matern nu=1, lambda=0.1, 257^2 vertices, embedding
    grown until nonnegative (512^2), 4096 samples, integral of u, run in
    FP64 and in mixed precision.
C3  MLMC with smoothing, Matern nu=1/2, lambda=0.03, levels h = 1/16 ..
    1/256 with N = 20000/5000/1200/300/80; level 0 single, levels 1..4
    pairs; tau = n on smoothed fields, the finest fine field unsmoothed.
C4  served requests: Poisson arrivals (rate 200/s), mesh m uniform on
    {32, ..., 1024}, count uniform on 1..256, Matern nu uniform on
    {1/2, 1, 3/2}, lambda uniform on [0.02, 0.3], sigma2=1, pair levels
    (m, m/2) except single at m=32, tau=0, embedding grown up to 4x, mixed;
    request r uses seed r+1 and samples 0..count-1.
C5  large fine level, Matern nu=3/2, sigma2=2, lambda=0.01, 2049^2
    vertices, embedding grown up to 4x, flow cell, outflow QoI, mixed.
"""

C1 = dict(cov="matern", nu=0.5, lam=0.3, sigma2=1.0, m=32, level="single", psd="clamp",
          precision="fp64", qoi="integral", bc="dirichlet0")
C1_COUNT = 64

C2 = dict(cov="matern", nu=1.0, lam=0.1, sigma2=1.0, m=256, level="single", psd="grow",
          precision="mixed", qoi="integral", bc="dirichlet0")
C2_COUNT = 4096

C3_M = [16, 32, 64, 128, 256]
C3_N = [20000, 5000, 1200, 300, 80]


def c3_level(l):
    """Level l of C3 (l = 0 .. 4): smoothed below the finest level."""
    base = dict(cov="matern", nu=0.5, lam=0.03, sigma2=1.0, m=C3_M[l], precision="mixed",
                qoi="integral", bc="dirichlet0", stream=l)
    if l == 0:
        return dict(base, level="single", tau_fine=-1, tau_coarse=-1)
    if l == len(C3_M) - 1:
        return dict(base, level="pair", tau_fine=0, tau_coarse=-1)
    return dict(base, level="pair", tau_fine=-1, tau_coarse=-1)


def c4_trace(duration_s=30.0, rate=200.0, seed=0, m_values=(32, 64, 128, 256, 512, 1024)):
    """Arrival trace of the serving workload: list of dicts with keys t
    (arrival time, s), w (level descriptor arguments), seed, first, count.
    Drawn from numpy.random.default_rng(seed)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration_s:
            break
        m = int(m_values[int(rng.integers(0, len(m_values)))])
        count = int(rng.integers(1, 257))
        nu = (0.5, 1.0, 1.5)[int(rng.integers(0, 3))]
        lam = float(rng.uniform(0.02, 0.3))
        r = len(out)
        w = dict(cov="matern", nu=nu, lam=lam, sigma2=1.0, m=m, level="single" if m == 32 else "pair",
                 tau_fine=0, tau_coarse=0, psd="grow", max_pad=4, precision="mixed", qoi="integral",
                 bc="dirichlet0")
        out.append(dict(t=t, w=w, seed=r + 1, first=0, count=count))
    return out


C5 = dict(cov="matern", nu=1.5, lam=0.01, sigma2=2.0, m=2048, level="single", psd="grow",
          max_pad=4, precision="mixed", qoi="outflux", bc="flowcell")
C5_COUNT = 1024

_ENUMS = {
    "cov": {"matern": 0, "sepexp": 1},
    "level": {"single": 0, "pair": 1},
    "psd": {"grow": 0, "clamp": 1, "fail": 2},
    "period": {"euclid": 0, "inf": 1},
    "field": {"pair": 0, "hartley": 1},
    "bc": {"dirichlet0": 0, "flowcell": 1},
    "qoi": {"integral": 0, "point": 1, "l2": 2, "outflux": 3},
    "coupling": {"restrict": 0, "embed": 1},
}


def to_oracle(w):
    """Translate a workload dict to the oracle's descriptor keys."""
    def e(key, default):
        v = w.get(key, default)
        return _ENUMS[key][v] if isinstance(v, str) else int(v)
    return dict(cov=e("cov", "matern"), nu=w.get("nu", 0.5), lam=w["lam"], sigma2=w.get("sigma2", 1.0),
                m=w["m"], level=e("level", "single"), tau_f=w.get("tau_fine", 0),
                tau_c=w.get("tau_coarse", 0), psd=e("psd", "grow"), period=e("period", "euclid"),
                max_pad=w.get("max_pad", 4), field_mode=e("field", "pair"), bc=e("bc", "dirichlet0"),
                qoi=e("qoi", "integral"), qx=w.get("qoi_x", 7.0 / 15.0), qy=w.get("qoi_y", 7.0 / 15.0),
                f=w.get("f", 1.0), stream=w.get("stream", 0), coupling=e("coupling", "restrict"))
