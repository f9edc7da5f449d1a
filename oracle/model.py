"""Parameter set of one 2LPT problem (oracle side; test infrastructure only).

The paper states the problem as: a linear density field on a regular periodic
grid, a cosmology, a gravity model given by mu(k,a) and the expansion
coefficients M_k, and an output time (Sec. 3, the procedure paragraph;
Sec. 2.4, eq. d1 and eq. full-d2).  The fields below are those inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

GRAVITY = ("gr", "fr_hs", "mu_const")
FACTORISATION = ("eds", "t1", "triangle", "winther", "bouchet")


@dataclass(frozen=True)
class Model:
    n: int = 32                 # cells per side
    box: float = 128.0          # side in Mpc/h
    omega_m: float = 0.3        # flat: Omega_Lambda = 1 - Omega_m
    h: float = 0.7              # BBKS shape parameter Gamma = Omega_m h
    n_s: float = 0.96
    sigma8: float = 0.8
    gravity: str = "gr"         # "gr", "fr_hs" (Hu-Sawicki n=1), "mu_const" (test model)
    fr0_abs: float = 1e-5       # |f_R0| for fr_hs
    mu_const: float = 1.0       # mu for mu_const
    factorisation: str = "eds"  # how D2(k,a) is obtained
    tri_ratio: float = 1.0      # k1/k2 for "triangle"
    tri_theta_deg: float = 90.0  # angle between k1 and k2 for "triangle"
    nk: int = 256               # growth-table nodes, log-spaced
    kmin: float = 1e-3          # h/Mpc
    kmax: float = 10.0          # h/Mpc
    a_init: float = 1e-3
    ode_steps: int = 4096

    def __post_init__(self):
        if self.gravity not in GRAVITY:
            raise ValueError(f"unknown gravity model {self.gravity!r}")
        if self.factorisation not in FACTORISATION:
            raise ValueError(f"unknown factorisation {self.factorisation!r}")
        if self.n < 2 or self.n % 2:
            raise ValueError("grid size must be even")

    @property
    def omega_l(self) -> float:
        return 1.0 - self.omega_m

    @property
    def volume(self) -> float:
        return self.box ** 3

    def with_(self, **kw) -> "Model":
        return replace(self, **kw)


def preset(name: str) -> Model:
    """The five workload shapes used by tests and the benchmark.

    C1: GR, 32^3, L=128 Mpc/h, D2 = -3/7 D1^2.
    C2: Hu-Sawicki n=1, |f_R0|=1e-5, 256^3, L=512, T1 factorisation.
    C3: Hu-Sawicki n=1, |f_R0|=1e-6 (F6; F4 via with_), 512^3, L=1024, T1.
    C4: the batched mix uses C4a (128^3, L=256) and C4b (64^3, L=128), F5, T1.
    C5: adjoint workload, 128^3, L=256, F5, T1.
    """
    base = Model(omega_m=0.3, h=0.7, n_s=0.96, sigma8=0.8)
    table = {
        "C1": base.with_(n=32, box=128.0, gravity="gr", factorisation="eds"),
        "C2": base.with_(n=256, box=512.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1"),
        "C3": base.with_(n=512, box=1024.0, gravity="fr_hs", fr0_abs=1e-6, factorisation="t1"),
        "C4a": base.with_(n=128, box=256.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1"),
        "C4b": base.with_(n=64, box=128.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1"),
        "C5": base.with_(n=128, box=256.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1"),
    }
    return table[name]
