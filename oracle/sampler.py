"""One MLMC level sample (oracle; test infrastructure only).

Algorithm 1 (level estimate with circulant embedding) and Algorithm 2
(smoothed variant) of Sections 3.4-3.5, per sample:

  Y = Q_f                       (SINGLE: level 0, or plain Monte Carlo)
  Y = Q_{h_l} - Q_{h_{l-1}}     (PAIR: both from the same field sample)

with the fine and coarse coefficients restricted from one field (step
4(e)).  Smoothing is expressed by two drop counts of the fine level's
embedding: tau_f for the field solved on the fine mesh and tau_c for the
field solved on the coarse mesh.  Reading of eq. (mlmc-estimator-smoothed):
on levels l < L both use tau_l; on the finest level
L the fine term is unsmoothed (tau_f = 0) and the coarse term keeps tau_L;
when tau_f != tau_c the two fields come from two DFTs of the same xi.
With coupling EMBED the coarse field instead comes from the coarse mesh's
own embedding (as a single level of mesh 2h with drop count tau_c) driven
by the fine xi at the same signed frequencies, so that the coarse term of
level l has the law of the fine term of level l-1 and the smoothed sum
telescopes exactly.

Sample index i maps to pair q = floor(i/2), component i mod 2 in PAIR field
mode, and to q = i in HARTLEY field mode.  A HARTLEY plan may carry a
lattice (qmc.py): its coordinates replace the normals at their eigen
indices.

desc keys: cov, nu, lam, sigma2, m, level (0 SINGLE / 1 PAIR), tau_f,
tau_c (-1 = default n), psd, period, max_pad, field_mode, bc, qoi, qx, qy,
f, stream, coupling (0 RESTRICT / 1 EMBED).
"""

import numpy as np

from . import embedding, field, fem, qmc, qoi

SINGLE = 0
PAIR_LEVEL = 1
RESTRICT = 0
EMBED = 1


class Plan:
    """Embedding set-up of a level (Algorithm 1 steps 1-3 + masks)."""

    def __init__(self, desc):
        self.desc = dict(desc)
        st = embedding.setup(self.desc)
        self.n = st["n"]
        self.J = st["J"]
        self.lam = st["lam"]
        self.info = st
        n = self.n
        tf = self.desc.get("tau_f", 0)
        tc = self.desc.get("tau_c", 0)
        self.tau_f = embedding.tau_default(n) if tf < 0 else int(tf)
        self.tau_c = embedding.tau_default(n) if tc < 0 else int(tc)
        self.coarse_plan = None
        if self.desc.get("coupling", 0) == EMBED and self.desc.get("level", SINGLE) == PAIR_LEVEL:
            # the coarse term from the coarse mesh's own embedding (a single
            # level of mesh 2h with the coarse drop count)
            cd = dict(self.desc, m=self.desc["m"] // 2, level=SINGLE, tau_f=tc, tau_c=tc, coupling=0)
            self.coarse_plan = Plan(cd)
            if n < 2 * self.coarse_plan.n:
                raise ValueError("EMBED coupling needs a fine embedding period at least the coarse one's")
            self.tau_c = self.coarse_plan.tau_f
        self.keep_f = embedding.mask(self.lam, self.tau_f)
        # the fine embedding's coarse-mesh field (RESTRICT only)
        self.keep_c = self.keep_f if self.coarse_plan is not None else embedding.mask(self.lam, self.tau_c)
        self.a_f = embedding.amplitudes(self.lam, self.keep_f)
        self.a_c = embedding.amplitudes(self.lam, self.keep_c)
        self.lattice = None

    def set_lattice(self, lat):
        """Quasi-Monte Carlo normals (qmc.Lattice) for a HARTLEY plan; None = Monte Carlo."""
        if lat is not None and self.desc.get("field_mode", field.PAIR) != field.HARTLEY:
            raise ValueError("a lattice needs the Hartley field mode")
        self.lattice = lat

    def fields(self, seed, i):
        """(Z_f, Z_c) nodal fields of sample i; Z_c is None for SINGLE."""
        d = self.desc
        m = d["m"]
        mode = d.get("field_mode", field.PAIR)
        if mode == field.PAIR:
            q, comp = i // 2, i % 2
        else:
            q, comp = i, 0
        if self.lattice is not None:
            xi = qmc.lattice_xi(self.lattice, seed, q, d.get("stream", 0), self.n)
        else:
            xi = field.xi(seed, q, d.get("stream", 0), self.n, mode)
        zf = field.fields(self.a_f, xi, m, mode)[comp]
        if d.get("level", SINGLE) == SINGLE:
            return zf, None
        if self.coarse_plan is not None:
            cp = self.coarse_plan
            return zf, field.fields(cp.a_f, field.embedded_xi(xi, cp.n), m // 2, mode)[comp]
        if self.tau_c == self.tau_f:
            zc_full = zf
        else:
            zc_full = field.fields(self.a_c, xi, m, mode)[comp]
        return zf, field.restrict_coarse(zc_full)

    def solve_q(self, z, m):
        d = self.desc
        k = np.exp(z)
        bc = d.get("bc", fem.DIRICHLET0)
        u, A, b = fem.solve(k, m, bc, d.get("f", 1.0))
        return qoi.evaluate(d.get("qoi", qoi.INTEGRAL), u, m, A, b,
                            d.get("qx", 7.0 / 15.0), d.get("qy", 7.0 / 15.0))

    def sample(self, seed, i):
        """(Y, Q_f, Q_c) of sample i (Q_c = 0 for SINGLE)."""
        m = self.desc["m"]
        zf, zc = self.fields(seed, i)
        qf = self.solve_q(zf, m)
        if zc is None:
            return qf, qf, 0.0
        qc = self.solve_q(zc, m // 2)
        return qf - qc, qf, qc


def level_samples(desc, seed, first, count):
    """Y, Q_f, Q_c arrays for samples first .. first+count-1."""
    plan = Plan(desc)
    out = np.array([plan.sample(seed, first + t) for t in range(count)])
    if count == 0:
        return np.zeros(0), np.zeros(0), np.zeros(0)
    return out[:, 0], out[:, 1], out[:, 2]
