"""The five synthetic workloads and their seeds.

Each workload has the shape of the paper's measurements (4D lattices with
T = 2L, Ls of 8-24, 4^4 blocks, light masses); the physical gauge ensembles
are not available, so seeded SU(3) fields stand in for them.

Seeds: gauge = 1000*cfg + 1; source of right-hand side r = 1000*cfg + 100 + r;
random starting vector k of the subspace = 1000*cfg + 500 + k.
"""
from __future__ import annotations

from dataclasses import dataclass, field


@dataclass(frozen=True)
class Workload:
    cfg: int
    name: str
    dims: tuple  # (X, Y, Z, T)
    Ls: int
    M5: float
    mass: float
    eps: float
    bc: tuple = (1.0, 1.0, 1.0, -1.0)  # boundary phase per direction x, y, z, t
    block: tuple | None = None
    nvec: int = 0
    nrhs: int = 1
    tol: float = 1e-8

    @property
    def gauge_seed(self) -> int:
        return 1000 * self.cfg + 1

    def source_seed(self, r: int) -> int:
        return 1000 * self.cfg + 100 + r

    def subspace_seed(self, k: int) -> int:
        return 1000 * self.cfg + 500 + k

    @property
    def coarse_seed(self) -> int:
        """the coarse noise of the second deflation level"""
        return 1000 * self.cfg + 900


WORKLOADS = {
    1: Workload(1, "cg-fp64-4^4xLs8", (4, 4, 4, 4), 8, 1.8, 0.01, 0.5),
    2: Workload(2, "mpcdagmpc-16^4xLs16", (16, 16, 16, 16), 16, 1.8, 0.01, 0.7),
    3: Workload(3, "hdcg-16^3x32xLs16", (16, 16, 16, 32), 16, 1.8, 0.003, 0.7,
                block=(4, 4, 4, 4), nvec=24),
    4: Workload(4, "hdcg-24^3x48xLs16", (24, 24, 24, 48), 16, 1.8, 0.001, 0.7,
                block=(4, 4, 4, 4), nvec=48),
    5: Workload(5, "hdcg-mrhs16-24^3x48xLs16", (24, 24, 24, 48), 16, 1.8, 0.001, 0.7,
                block=(4, 4, 4, 4), nvec=48, nrhs=16),
}
