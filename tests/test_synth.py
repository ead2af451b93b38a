"""Seeded generators: reproducible, inside their stated ranges, and inside the
stability limit of the scheme for every workload."""
import hashlib

import numpy as np

from paper_2310_13325_amd import configs, synth


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_same_seed_same_bytes():
    for p in (configs.C1, configs.C2) + configs.C4:
        v1, b1 = synth.true_model(p)
        v2, b2 = synth.true_model(p)
        assert _sha(v1) == _sha(v2) and _sha(b1) == _sha(b2)
        lo, hi = synth.prior_bounds(p, v1, b1)
        assert _sha(synth.initial_particles(p, lo, hi, 4)) == _sha(synth.initial_particles(p, lo, hi, 4))
    assert _sha(synth.noise(configs.C1)) == _sha(synth.noise(configs.C1))
    assert _sha(synth.normals(5, 3, 7)) == _sha(synth.normals(5, 3, 7))
    assert _sha(synth.normals(5, 3, 7)) != _sha(synth.normals(6, 3, 7))


def test_models_priors_and_particles_in_range():
    for p in (configs.C1, configs.C2, configs.C3) + configs.C4:
        v, b = synth.true_model(p)
        assert v.shape == (p.nz, p.nx)
        vmax = 3000.0 if p.model == "layers_anomalies" else 4500.0
        assert v.min() >= 1500.0 and v.max() <= vmax
        lo, hi = synth.prior_bounds(p, v, b)
        assert np.all(hi - lo > 0) and np.all(lo >= 1000.0)
        x = synth.initial_particles(p, lo, hi, 3)
        assert np.all(x >= lo) and np.all(x <= hi)
        courant = hi.max() * p.dt / p.dx
        assert courant < np.sqrt(3.0 / 8.0), (p.name, courant)
    v, _ = synth.true_model(configs.C2)
    assert np.all(v[: configs.C2.water_rows] == 1500.0)


def test_acquisition_layout():
    p = configs.C2
    assert p.src_ix == (10, 30, 50, 70, 90, 110, 130, 150, 170, 190)
    assert len(p.rec_ix) == 200 and p.rec_iz * p.dx == 360.0 and p.src_iz * p.dx == 20.0


def test_precision_case_fields():
    case = configs.SvgdCase("tiny", n=6, d=0, eps=1.0, seed=11)
    v = np.full((12, 10), 3000.0)
    X, G = synth.svgd_precision_case(case, v)
    assert X.shape == (6, 120) and G.shape == (6, 120)
    zeta = (X - 3000.0) / 100.0
    assert np.allclose(np.sqrt(np.mean(zeta ** 2, axis=1)), 1.0)
