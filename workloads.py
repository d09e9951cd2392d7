"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method: it only names the workloads
(mesh sizes, degree, separator spacing, number of eigenpairs) and draws the
per-element coefficient fields and loss weights from fixed seeds.  Both the
oracle and the HIP path receive the arrays it returns as plain inputs.

The paper's workload is the Dirichlet Laplace eigenproblem on the unit
square / cube with uniform meshes (Sec. 2.1 and Sec. 7); the coefficient
fields kappa_e, rho_e = exp(sigma Z), Z ~ N(0, 1) i.i.d. per element, extend it
to the heterogeneous problems the benchmark also covers.
"""
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2009_08167


@dataclass
class Workload:
    name: str
    dim: int
    ne: int
    p: int
    s: int                 # separator spacing in elements, 0 = plain IGA
    nev: int
    lognormal_sigma: float = 0.0
    seed: int = SEED_BASE
    extra: dict = field(default_factory=dict)

    @property
    def n_elem(self):
        return self.ne ** self.dim

    def n1(self):
        """Interior functions per direction."""
        n_c0 = 0 if self.s <= 0 else (self.ne - 1) // self.s
        return self.ne + self.p - 2 + n_c0 * (self.p - 1)

    @property
    def n_dof(self):
        return self.n1() ** self.dim

    def coefficients(self):
        """(kappa, rho) per element, x-fastest; ones if lognormal_sigma == 0."""
        if self.lognormal_sigma == 0.0:
            one = np.ones(self.n_elem)
            return one, one.copy()
        rng = np.random.default_rng(self.seed)
        kappa = np.exp(self.lognormal_sigma * rng.standard_normal(self.n_elem))
        rho = np.exp(self.lognormal_sigma * rng.standard_normal(self.n_elem))
        return kappa, rho

    def with_(self, **kw):
        d = dict(self.__dict__)
        d.update(kw)
        return Workload(**d)


def c1():
    """2D, 16x16, p=2 IGA, kappa=rho=1, lowest 10."""
    return Workload("2d_16x16_p2_iga", 2, 16, 2, 0, 10, 0.0, SEED_BASE + 0)


def c2(riga=True):
    """2D, 256x256, p=3; rIGA separators every 16 elements (or IGA);
    log-normal(0, 0.3) coefficients; lowest 200."""
    return Workload("2d_256x256_p3_" + ("riga16" if riga else "iga"), 2, 256, 3,
                    16 if riga else 0, 200, 0.3, SEED_BASE + 1)


def c3(riga=True):
    """3D, 32^3, p=2; rIGA separators every 8 elements (or IGA);
    kappa=rho=1; lowest 100."""
    return Workload("3d_32x32x32_p2_" + ("riga8" if riga else "iga"), 3, 32, 2,
                    8 if riga else 0, 100, 0.0, SEED_BASE + 2)


def c4(count=64):
    """64 uneven 2D rIGA instances: ne ~ U{32..192}, p ~ U{2,3,4},
    s ~ U{8,16}, log-normal(0, 0.5), lowest 20 each."""
    rng = np.random.default_rng(SEED_BASE + 3)
    out = []
    for i in range(count):
        ne = int(rng.integers(32, 193))
        p = int(rng.integers(2, 5))
        s = int(rng.choice([8, 16]))
        out.append(Workload("batch_%02d" % i, 2, ne, p, s, 20, 0.5,
                            SEED_BASE + 1000 + i))
    return out


def c5():
    """2D, 128x128, p=3, rIGA every 16, log-normal(0, 0.5); loss weights
    w ~ U(0,1)^20."""
    w = Workload("2d_128x128_p3_riga16_grad", 2, 128, 3, 16, 20, 0.5, SEED_BASE + 4)
    rng = np.random.default_rng(SEED_BASE + 5)
    w.extra["weights"] = rng.uniform(0.0, 1.0, 20)
    w.extra["fd_elements"] = rng.choice(w.n_elem, size=50, replace=False)
    return w


def small(dim, ne, p, s, nev, sigma=0.0, seed=SEED_BASE + 99):
    """A small case for parity tests."""
    return Workload("%dd_%d_p%d_s%d" % (dim, ne, p, s), dim, ne, p, s, nev, sigma, seed)
