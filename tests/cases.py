"""Seeded FWI problems for parity tests: the same synthetic inputs feed the
oracle (NumPy float64) and the library (torch device tensors)."""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np

from oracle import fwi as ofwi
from paper_2310_13325_amd import configs, synth


@dataclass
class Case:
    prob: configs.Problem
    v_true: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    particles: np.ndarray      # float32-representable, float64 dtype
    dobs: np.ndarray           # [ns][nt][nr] float32-representable
    sigma: float

    @property
    def ogrid(self):
        p = self.prob
        return ofwi.Grid(nz=p.nz, nx=p.nx, nb=p.nb, nt=p.nt, dx=p.dx, dz=p.dx, dt=p.dt, alpha=p.alpha)

    @property
    def ogeom(self):
        p = self.prob
        return ofwi.Geometry(src_iz=(p.src_iz,) * p.ns, src_ix=p.src_ix, rec_iz=(p.rec_iz,) * p.nr,
                             rec_ix=p.rec_ix, f0=p.f0)

    @property
    def vmax(self):
        return float(np.float32(self.hi.max()))


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def sigma_of(prob, clean):
    if prob.noise == "rms_1pct":
        return 0.01 * float(np.sqrt(np.mean(clean ** 2)))
    if prob.noise == "median_max_2pct":
        return 0.02 * float(np.median(np.abs(clean).max(axis=1)))
    raise ValueError(prob.noise)


@lru_cache(maxsize=None)
def build_case(prob: configs.Problem, n_particles: int | None = None) -> Case:
    """Observed data from the FP64 oracle on the true model plus seeded noise."""
    v, vb = synth.true_model(prob)
    lo, hi = synth.prior_bounds(prob, v, vb)
    lo, hi = f32(lo), f32(hi)
    parts = f32(synth.initial_particles(prob, lo, hi, n_particles))
    parts = np.clip(parts, lo, hi)
    case = Case(prob, f32(v), lo, hi, parts, None, 0.0)
    clean = ofwi.simulate(case.v_true, case.ogrid, case.ogeom)
    sigma = sigma_of(prob, clean)
    dobs = f32(clean + sigma * synth.noise(prob))
    case.dobs = dobs
    case.sigma = sigma
    return case


def small_problem(name="ragged", nx=70, nz=37, nt=180, ns=3, f0=18.0, dx=10.0, dt=1e-3, seed=7,
                  np_=3):
    """An odd-sized problem: tiles ragged in x and z, receivers on several rows."""
    return configs.Problem(name, nx=nx, nz=nz, dx=dx, nt=nt, dt=dt, ns=ns, np=np_, f0=f0,
                           src_iz=1, rec_iz=2, model="layers_anomalies", prior="rowmean_pm500",
                           noise="rms_1pct", seed=seed, nb=9)


def workers():
    from oracle import cpu_pool
    return cpu_pool.default_workers()


@lru_cache(maxsize=None)
def build_case_c(prob: configs.Problem, n_particles: int | None = None) -> Case:
    """As build_case, with the C oracle (threads) making the observed data."""
    from oracle import cref
    v, vb = synth.true_model(prob)
    lo, hi = synth.prior_bounds(prob, v, vb)
    lo, hi = f32(lo), f32(hi)
    parts = np.clip(f32(synth.initial_particles(prob, lo, hi, n_particles)), lo, hi)
    case = Case(prob, f32(v), lo, hi, parts, None, 0.0)
    clean = cref.simulate(case.v_true, case.ogrid, case.ogeom, workers=workers())
    case.sigma = sigma_of(prob, clean)
    case.dobs = f32(clean + case.sigma * synth.noise(prob))
    return case
