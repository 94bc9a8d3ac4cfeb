"""MI355X-native MLMC level sampler with (smoothed) circulant embedding.

Python binding of libcesmlmc (include/cesmlmc.h): argument marshalling
only.  Every step of the sampler runs in the library's HIP kernels; torch
provides device buffers and streams.

    import paper_2306_13493_amd as ces
    ctx = ces.Context(0)
    plan = ctx.plan(cov="matern", nu=1.0, lam=0.1, m=256, precision="mixed")
    out = plan.sample(seed=0, first=0, count=4096)   # torch tensors on cuda
"""

import ctypes

import numpy as np

from . import _lib
from ._lib import (CesError, LevelDesc, MlmcOpts, MlmcResult, MlqmcOpts, PlanInfo, Request, Schedule, ServerStats,
                   SmoothingStats, check, load)

COV = {"matern": 0, "sepexp": 1}
LEVEL = {"single": 0, "pair": 1}
PSD = {"grow": 0, "clamp": 1, "fail": 2}
PERIOD = {"euclid": 0, "inf": 1}
FIELD = {"pair": 0, "hartley": 1}
PREC = {"fp64": 0, "mixed": 1}
BC = {"dirichlet0": 0, "flowcell": 1}
QOI = {"integral": 0, "point": 1, "l2": 2, "outflux": 3}
COUPLE = {"restrict": 0, "embed": 1}
CYCLE = {"auto": 0, "v": 1, "w1": 2}


def _enum(table, v):
    return table[v] if isinstance(v, str) else int(v)


def level_desc(cov="matern", nu=0.5, lam=0.1, sigma2=1.0, m=32, level="single", tau_fine=0,
               tau_coarse=0, psd="grow", period="euclid", max_pad=4, field="pair", precision="mixed",
               bc="dirichlet0", qoi="integral", qoi_x=7.0 / 15.0, qoi_y=7.0 / 15.0, f=1.0, cg_rtol=1e-10,
               cg_max_iter=500, stream=0, coupling="restrict", cycle="auto"):
    """Build a ces_level_desc (library defaults, then the given fields)."""
    lib = load()
    d = LevelDesc()
    lib.ces_level_desc_default(ctypes.byref(d))
    d.cov_kind = _enum(COV, cov)
    d.nu = float(nu)
    d.lambda_ = float(lam)
    d.sigma2 = float(sigma2)
    d.m_fine = int(m)
    d.level_kind = _enum(LEVEL, level)
    d.tau_fine = int(tau_fine)
    d.tau_coarse = int(tau_coarse)
    d.psd_policy = _enum(PSD, psd)
    d.periodization = _enum(PERIOD, period)
    d.max_pad_factor = int(max_pad)
    d.field_mode = _enum(FIELD, field)
    d.precision = _enum(PREC, precision)
    d.bc = _enum(BC, bc)
    d.qoi = _enum(QOI, qoi)
    d.coupling = _enum(COUPLE, coupling)
    d.mg_cycle = _enum(CYCLE, cycle)
    d.qoi_x = float(qoi_x)
    d.qoi_y = float(qoi_y)
    d.f_value = float(f)
    d.cg_rtol = float(cg_rtol)
    d.cg_max_iter = int(cg_max_iter)
    d.stream = int(stream)
    return d


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """A device binding (ces_context)."""

    def __init__(self, device=0, mem_budget=0):
        self.lib = load()
        self.device = int(device)
        h = ctypes.c_void_p()
        check(self.lib.ces_context_create(self.device, int(mem_budget), ctypes.byref(h)))
        self.handle = h

    def plan(self, desc=None, **kw):
        return Plan(self, desc if desc is not None else level_desc(**kw))

    @property
    def schedule(self):
        """(depth, max_lanes, chunk_samples, graphs) of ces_sample / ces_sample_batch."""
        s = Schedule()
        check(self.lib.ces_schedule_get(self.handle, ctypes.byref(s)))
        return (s.depth, s.max_lanes, s.chunk_samples, s.graphs)

    @schedule.setter
    def schedule(self, v):
        v = tuple(v) + (0,) * (4 - len(v))
        s = Schedule(int(v[0]), int(v[1]), int(v[2]), int(v[3]), 0)
        check(self.lib.ces_schedule_set(self.handle, ctypes.byref(s)))

    def _requests(self, reqs, outs):
        torch = _torch()
        dev = torch.device("cuda", self.device)
        arr = (Request * len(reqs))()
        res = []
        for i, r in enumerate(reqs):
            plan, seed, first, count = r
            o = outs[i] if outs is not None else None
            if o is None:
                o = {"y": torch.empty(count, dtype=torch.float64, device=dev),
                     "q_fine": torch.empty(count, dtype=torch.float64, device=dev),
                     "q_coarse": torch.empty(count, dtype=torch.float64, device=dev),
                     "iters": torch.empty(count, dtype=torch.int32, device=dev),
                     "status": torch.empty(count, dtype=torch.int32, device=dev)}
            arr[i] = Request(plan.handle.value if plan is not None else None, int(seed), int(first), int(count),
                             o["y"].data_ptr(), o["q_fine"].data_ptr(), o["q_coarse"].data_ptr(),
                             o["iters"].data_ptr(), o["status"].data_ptr())
            res.append(o)
        return arr, res

    def sample_batch(self, reqs, stream=None, outs=None):
        """ces_sample_batch over [(plan, seed, first, count), ...]; returns
        one output dict per request (as Plan.sample)."""
        if not reqs:
            return []
        arr, res = self._requests(reqs, outs)
        check(self.lib.ces_sample_batch(self.handle, arr, len(reqs), _stream_ptr(stream)))
        return res

    def autotune(self, reqs, stream=None, outs=None):
        """ces_autotune over the requests: ((depth, max_lanes, chunk, graphs), best_ms, outputs)."""
        arr, res = self._requests(reqs, outs)
        s = Schedule()
        ms = ctypes.c_double()
        check(self.lib.ces_autotune(self.handle, arr, len(reqs), _stream_ptr(stream), ctypes.byref(s),
                                    ctypes.byref(ms)))
        return (s.depth, s.max_lanes, s.chunk_samples, s.graphs), ms.value, res

    def close(self):
        if self.handle:
            self.lib.ces_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """An immutable level plan (ces_plan): embedding, eigenvalues, masks."""

    def __init__(self, ctx, desc):
        self.ctx = ctx
        self.lib = ctx.lib
        self.desc = desc
        h = ctypes.c_void_p()
        check(self.lib.ces_plan_create(ctx.handle, ctypes.byref(desc), ctypes.byref(h)))
        self.handle = h
        info = PlanInfo()
        check(self.lib.ces_plan_info_get(h, ctypes.byref(info)))
        self.info = info

    @property
    def n(self):
        return self.info.n

    @property
    def m(self):
        return self.desc.m_fine

    def _outputs(self, count, out):
        if out is not None:
            return out
        torch = _torch()
        dev = torch.device("cuda", self.ctx.device)
        return {
            "y": torch.empty(count, dtype=torch.float64, device=dev),
            "q_fine": torch.empty(count, dtype=torch.float64, device=dev),
            "q_coarse": torch.empty(count, dtype=torch.float64, device=dev),
            "iters": torch.empty(count, dtype=torch.int32, device=dev),
            "status": torch.empty(count, dtype=torch.int32, device=dev),
        }

    def sample(self, seed, first, count, stream=None, out=None):
        """Y, Q_f, Q_c, iterations and status of samples first..first+count-1
        as device tensors (dict)."""
        out = self._outputs(count, out)
        check(self.lib.ces_sample(self.handle, int(seed), int(first), int(count), _ptr(out["y"]),
                                  _ptr(out.get("q_fine")), _ptr(out.get("q_coarse")), _ptr(out.get("iters")),
                                  _ptr(out.get("status")), _stream_ptr(stream)))
        return out

    def sample_noalloc(self, seed, first, count, stream=None, out=None):
        """ces_sample_noalloc: as sample(), with the library's workspace in
        its static device array (the outputs are the caller's: pass `out`
        to allocate nothing at all)."""
        out = self._outputs(count, out)
        check(self.lib.ces_sample_noalloc(self.handle, int(seed), int(first), int(count), _ptr(out["y"]),
                                          _ptr(out.get("q_fine")), _ptr(out.get("q_coarse")),
                                          _ptr(out.get("iters")), _ptr(out.get("status")), _stream_ptr(stream)))
        return out

    def eigenvalues(self):
        n = self.n
        a = np.empty((n, n), dtype=np.float64)
        check(self.lib.ces_plan_eigenvalues(self.handle, a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def masks(self):
        """(fine, coarse) keep masks; the coarse one is on the coarse
        embedding (n_coarse x n_coarse) for EMBED pairs."""
        n, nc = self.n, self.info.n_coarse
        f = np.empty((n, n), dtype=np.uint8)
        c = np.empty((nc, nc), dtype=np.uint8)
        check(self.lib.ces_plan_mask(self.handle, f.ctypes.data_as(ctypes.c_void_p),
                                     c.ctypes.data_as(ctypes.c_void_p)))
        return f, c

    def lattice_order(self, s):
        """(dims, lam): the s eigen indices with the largest eigenvalues."""
        d = np.empty(int(s), dtype=np.int64)
        lam = np.empty(int(s), dtype=np.float64)
        check(self.lib.ces_plan_lattice_order(self.handle, int(s), d.ctypes.data_as(ctypes.c_void_p),
                                              lam.ctypes.data_as(ctypes.c_void_p)))
        return d, lam

    def set_lattice(self, z=None, dims=None, shifts=16, s=None, log2_points=10):
        """Attach a randomly shifted lattice (HARTLEY plans).  With z given:
        ces_plan_set_lattice(z, dims or the default order); without:
        ces_plan_set_lattice_default(s, log2_points).  z = [] detaches."""
        if z is None:
            check(self.lib.ces_plan_set_lattice_default(self.handle, int(s), int(log2_points), int(shifts)))
            return
        z = np.ascontiguousarray(z, dtype=np.uint32)
        dp = None
        if dims is not None:
            dims = np.ascontiguousarray(dims, dtype=np.int64)
            if dims.size != z.size:
                raise ValueError("dims and z differ in length")
            dp = dims.ctypes.data_as(ctypes.c_void_p)
        check(self.lib.ces_plan_set_lattice(self.handle, int(z.size), z.ctypes.data_as(ctypes.c_void_p), dp,
                                            int(shifts)))

    def field(self, seed, sample, stream=None):
        """(Z_fine, Z_coarse or None) of one sample as float64 device tensors."""
        torch = _torch()
        dev = torch.device("cuda", self.ctx.device)
        m = self.m
        zf = torch.empty((m + 1, m + 1), dtype=torch.float64, device=dev)
        zc = None
        if self.desc.level_kind == LEVEL["pair"]:
            zc = torch.empty((m // 2 + 1, m // 2 + 1), dtype=torch.float64, device=dev)
        check(self.lib.ces_field(self.handle, int(seed), int(sample), _ptr(zf), _ptr(zc), _stream_ptr(stream)))
        return zf, zc

    def solve(self, k, grid=0, stream=None):
        """Solve for float64 device coefficients k of shape (count, m+1, m+1)."""
        torch = _torch()
        k = k.contiguous()
        count = k.shape[0]
        u = torch.empty_like(k)
        iters = torch.empty(count, dtype=torch.int32, device=k.device)
        check(self.lib.ces_solve(self.handle, int(grid), int(count), _ptr(k), _ptr(u), _ptr(iters),
                                 _stream_ptr(stream)))
        return u, iters

    def close(self):
        if self.handle:
            self.lib.ces_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """ces_server: continuous batching of level-sample requests with device
    memory admission.  Results land in host numpy arrays owned here."""

    QUEUED, ADMITTED, DONE = 0, 1, 2

    def __init__(self, ctx, mem_budget=0, max_inflight=0):
        self.ctx = ctx
        self.lib = ctx.lib
        h = ctypes.c_void_p()
        check(self.lib.ces_server_create(ctx.handle, int(mem_budget), int(max_inflight), ctypes.byref(h)))
        self.handle = h
        self._bufs = {}

    def submit(self, desc, seed, first, count):
        """Queue one request (desc: a LevelDesc or a dict of level_desc
        arguments); returns its id."""
        if isinstance(desc, dict):
            desc = level_desc(**desc)
        y = np.empty(int(count), dtype=np.float64)
        st = np.empty(int(count), dtype=np.int32)
        rid = ctypes.c_int64()
        check(self.lib.ces_server_submit(self.handle, ctypes.byref(desc), int(seed), int(first), int(count),
                                         y.ctypes.data_as(ctypes.c_void_p), st.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.byref(rid)))
        self._bufs[rid.value] = (y, st)
        return rid.value

    def poll(self, rid):
        """(state, latency_s): state 0 queued, 1 admitted, 2 done, < 0 error."""
        state = ctypes.c_int32()
        lat = ctypes.c_double()
        check(self.lib.ces_server_poll(self.handle, int(rid), ctypes.byref(state), ctypes.byref(lat)))
        return state.value, lat.value

    def result(self, rid):
        """(y, status) host arrays of a request (complete once poll says done)."""
        return self._bufs[rid]

    def drain(self):
        check(self.lib.ces_server_drain(self.handle))

    def stats(self):
        s = ServerStats()
        check(self.lib.ces_server_get_stats(self.handle, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_ if k != "reserved"}

    def close(self):
        if self.handle:
            self.lib.ces_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlmc_run(ctx, levels, finest=None, eps=1e-3, l_start=2, n_pilot=100, theta=0.5, alpha=0.0, cost_model=0,
             max_rounds=50, seed=0, stream=None, checkpoint=None, max_new_rounds=0):
    """ces_mlmc_run: adaptive MLMC over the given level plans (level 0
    single, levels >= 1 pairs); returns a dict of the result fields.  With
    `checkpoint` (a file path) ces_mlmc_run_checkpointed: the state is saved
    after every round and a run found there is continued; max_new_rounds > 0
    stops after that many rounds of this call."""
    lib = load()
    o = MlmcOpts()
    lib.ces_mlmc_opts_default(ctypes.byref(o))
    o.eps, o.l_start, o.n_pilot, o.theta = float(eps), int(l_start), int(n_pilot), float(theta)
    o.alpha, o.cost_model, o.max_rounds, o.seed = float(alpha), int(cost_model), int(max_rounds), int(seed)
    n = len(levels)
    lv = (ctypes.c_void_p * n)(*[p.handle.value for p in levels])
    fv = None if finest is None else (ctypes.c_void_p * n)(*[p.handle.value for p in finest])
    r = MlmcResult()
    if checkpoint is None:
        check(lib.ces_mlmc_run(ctx.handle, lv, fv, n, ctypes.byref(o), _stream_ptr(stream), ctypes.byref(r)))
    else:
        check(lib.ces_mlmc_run_checkpointed(ctx.handle, lv, fv, n, ctypes.byref(o), str(checkpoint).encode(),
                                            int(max_new_rounds), _stream_ptr(stream), ctypes.byref(r)))
    L = r.levels
    return {"estimate": r.estimate, "variance": r.variance, "bias": r.bias, "alpha": r.alpha, "beta": r.beta,
            "gamma": r.gamma, "levels": L, "converged": bool(r.converged), "rounds": r.rounds,
            "n": [r.n[i] for i in range(L)], "mean": [r.mean[i] for i in range(L)],
            "var": [r.var[i] for i in range(L)], "cost": [r.cost[i] for i in range(L)]}


def lattice_cbc(log2_points, gamma):
    """ces_lattice_cbc: generating vector (uint32 array) for 2^log2_points points."""
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    z = np.empty(g.size, dtype=np.uint32)
    check(load().ces_lattice_cbc(int(log2_points), int(g.size), g.ctypes.data_as(ctypes.c_void_p),
                                 z.ctypes.data_as(ctypes.c_void_p)))
    return z


def mlqmc_run(ctx, levels, finest=None, eps=1e-3, l_start=2, n_pilot=1, theta=0.5, alpha=0.0, cost_model=0,
              max_rounds=50, seed=0, stream=None):
    """ces_mlqmc_run: multilevel QMC over lattice plans; returns a dict of
    the result fields (n = points per shift x shifts)."""
    lib = load()
    o = MlqmcOpts()
    lib.ces_mlqmc_opts_default(ctypes.byref(o))
    o.eps, o.l_start, o.n_pilot, o.theta = float(eps), int(l_start), int(n_pilot), float(theta)
    o.alpha, o.cost_model, o.max_rounds, o.seed = float(alpha), int(cost_model), int(max_rounds), int(seed)
    n = len(levels)
    lv = (ctypes.c_void_p * n)(*[p.handle.value for p in levels])
    fv = None if finest is None else (ctypes.c_void_p * n)(*[p.handle.value for p in finest])
    r = MlmcResult()
    check(lib.ces_mlqmc_run(ctx.handle, lv, fv, n, ctypes.byref(o), _stream_ptr(stream), ctypes.byref(r)))
    L = r.levels
    return {"estimate": r.estimate, "variance": r.variance, "bias": r.bias, "alpha": r.alpha, "beta": r.beta,
            "gamma": r.gamma, "levels": L, "converged": bool(r.converged), "rounds": r.rounds,
            "n": [r.n[i] for i in range(L)], "mean": [r.mean[i] for i in range(L)],
            "var": [r.var[i] for i in range(L)], "cost": [r.cost[i] for i in range(L)]}


def coarsest_mesh(desc):
    """ces_mlmc_coarsest_mesh: m_0 of the coarsest-mesh rule for a descriptor."""
    m0 = ctypes.c_int32()
    check(load().ces_mlmc_coarsest_mesh(ctypes.byref(desc), ctypes.byref(m0)))
    return m0.value


def tau_rule(cov, m, alpha, cs_over_calpha, nu=0.5, J=0):
    """ces_tau_rule: eigenvalues to drop on mesh 1/m from the balance of
    discretisation and smoothing error; returns (tau, real root)."""
    t = ctypes.c_int64()
    tr = ctypes.c_double()
    check(load().ces_tau_rule(_enum(COV, cov), float(nu), int(m), int(J), float(alpha), float(cs_over_calpha),
                              ctypes.byref(t), ctypes.byref(tr)))
    return t.value, tr.value


def smoothing_error(ctx, full, smoothed, seed, first, count, stream=None):
    """ces_smoothing_error: statistics of Q_h - Q~_h over samples
    first..first+count-1 of two single plans that differ only in tau."""
    r = SmoothingStats()
    r.struct_size = ctypes.sizeof(SmoothingStats)
    check(load().ces_smoothing_error(ctx.handle, full.handle, smoothed.handle, int(seed), int(first), int(count),
                                     _stream_ptr(stream), ctypes.byref(r)))
    return {"n": r.n, "mean": r.mean, "mean_abs": r.mean_abs, "var": r.var, "mean_q": r.mean_q,
            "mean_q_smoothed": r.mean_q_smoothed}


def normals(seed, q, stream_tag, first_e, count, device=0, stream=None):
    """(count, 2) float64 device tensor of Box-Muller pairs (parity hook)."""
    torch = _torch()
    lib = load()
    out = torch.empty((count, 2), dtype=torch.float64, device=torch.device("cuda", device))
    check(lib.ces_normals(int(seed), int(q), int(stream_tag), int(first_e), int(count), _ptr(out),
                          _stream_ptr(stream)))
    return out


def profile_enable(on=True):
    """Start (clearing earlier records) or stop the library's launch profiler."""
    check(load().ces_profile_enable(1 if on else 0))


def profile_only(name=None):
    """Record only launches of the kernel with this profile name (None: all)."""
    check(load().ces_profile_only(name.encode() if name else None))


def profile_read(max_entries=64):
    """Per-kernel {name: (launches, total_ms, algorithmic_bytes)}; clears."""
    lib = load()
    buf = (_lib.ProfileEntry * max_entries)()
    n = ctypes.c_int32()
    check(lib.ces_profile_read(buf, max_entries, ctypes.byref(n)))
    return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms, buf[i].bytes)
            for i in range(min(n.value, max_entries))}


__all__ = ["Context", "Plan", "Server", "level_desc", "mlmc_run", "mlqmc_run", "lattice_cbc", "coarsest_mesh", "normals", "profile_enable", "profile_only", "profile_read", "CesError", "LevelDesc",
           "PlanInfo", "Request", "Schedule", "load"]
