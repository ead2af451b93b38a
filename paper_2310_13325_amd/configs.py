"""Workload definitions (pure data; no arithmetic of the method).

Five workloads built around the paper's full-waveform-inversion example
(section 4.2: 2-D FD acoustic modelling, Ricker source, Gaussian noise, uniform
prior, SVGD / sSVGD) at sizes that exercise one GPU:

  c1  small plain SVGD-FWI: 64x64 at 10 m, nt 500, 4 shots, 64 receivers,
      8 particles, 20 SVGD steps (the size a CPU oracle finishes in seconds);
  c2  batched gradients: 200x120 at 20 m, nt 2000, 10 shots, 200 receivers,
      128 particles -- the geometry of the paper's Marmousi experiment
      (section 4.2: 20 m grid, 10 sources at 20 m depth, 200 receivers at 360 m
      on the seabed) with a synthetic faulted model standing in for Marmousi;
  c3  differentiation: 400x200 at 12.5 m, nt 4000, 20 shots, 400 receivers,
      64 particles, checkpoints every 50 steps;
  c4  uneven batching: three problems 96x96, 150x100, 256x128 at 10 m,
      nt 800/1200/1600, 4/6/8 shots, 32 particles each, sSVGD;
  c5  SVGD update precision: n = 2048 particles, d = 24000 (the c2 model).

Grids are written nx x nz (nx horizontal columns, nz depth rows).
"""
from __future__ import annotations

from dataclasses import dataclass, field

SEED_BASE = 231013325
SPONGE_WIDTH = 20
SPONGE_ALPHA = 0.015


@dataclass(frozen=True)
class Problem:
    """One FWI problem: grid, acquisition, ensemble size, synthetic recipe."""
    name: str
    nx: int
    nz: int
    dx: float
    nt: int
    dt: float
    ns: int
    np: int
    f0: float
    src_iz: int
    rec_iz: int
    model: str            # "layers_anomalies" | "faulted"
    prior: str            # "rowmean_pm500" | "background_2kms"
    noise: str            # "rms_1pct" | "median_max_2pct"
    seed: int
    water_rows: int = 0
    ckpt_every: int = 50
    nb: int = SPONGE_WIDTH
    alpha: float = SPONGE_ALPHA

    @property
    def nr(self) -> int:
        return self.nx          # one receiver per column

    @property
    def d(self) -> int:
        return self.nx * self.nz

    @property
    def NZ(self) -> int:
        return self.nz + 2 * self.nb

    @property
    def NX(self) -> int:
        return self.nx + 2 * self.nb

    @property
    def src_ix(self):
        return tuple(int(round((k + 0.5) * self.nx / self.ns)) for k in range(self.ns))

    @property
    def rec_ix(self):
        return tuple(range(self.nx))


C1 = Problem("c1", nx=64, nz=64, dx=10.0, nt=500, dt=1e-3, ns=4, np=8, f0=10.0,
             src_iz=1, rec_iz=2, model="layers_anomalies", prior="rowmean_pm500",
             noise="rms_1pct", seed=SEED_BASE + 1)
C2 = Problem("c2", nx=200, nz=120, dx=20.0, nt=2000, dt=2e-3, ns=10, np=128, f0=8.0,
             src_iz=1, rec_iz=18, model="faulted", prior="background_2kms",
             noise="median_max_2pct", seed=SEED_BASE + 2, water_rows=18)
C3 = Problem("c3", nx=400, nz=200, dx=12.5, nt=4000, dt=1e-3, ns=20, np=64, f0=10.0,
             src_iz=2, rec_iz=29, model="faulted", prior="background_2kms",
             noise="median_max_2pct", seed=SEED_BASE + 3, water_rows=29)
C4 = (
    Problem("c4a", nx=96, nz=96, dx=10.0, nt=800, dt=1e-3, ns=4, np=32, f0=10.0,
            src_iz=1, rec_iz=2, model="layers_anomalies", prior="rowmean_pm500",
            noise="median_max_2pct", seed=SEED_BASE + 4),
    Problem("c4b", nx=150, nz=100, dx=10.0, nt=1200, dt=1e-3, ns=6, np=32, f0=10.0,
            src_iz=1, rec_iz=2, model="layers_anomalies", prior="rowmean_pm500",
            noise="median_max_2pct", seed=SEED_BASE + 40),
    Problem("c4c", nx=256, nz=128, dx=10.0, nt=1600, dt=1e-3, ns=8, np=32, f0=10.0,
            src_iz=1, rec_iz=2, model="layers_anomalies", prior="rowmean_pm500",
            noise="median_max_2pct", seed=SEED_BASE + 41),
)


@dataclass(frozen=True)
class SvgdCase:
    name: str
    n: int
    d: int
    eps: float
    seed: int
    spread: float = 100.0


C5 = SvgdCase("c5", n=2048, d=24000, eps=1000.0, seed=SEED_BASE + 5)

SVGD_STEPS_C1 = 20
