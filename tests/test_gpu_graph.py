"""hipGraph replay of vip_grad_logpost / vip_forward equals the eager launch
sequence bit for bit, over several replays with eager work and new input
values (same buffers) in between."""
import numpy as np
import pytest
import torch

from paper_2310_13325_amd import binding as vb
from paper_2310_13325_amd import configs
from tests.cases import build_case, small_problem
from tests.gpu_helpers import ctx, dev, grid_geom

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tile", [-1, 0, 3])
def test_graph_replays_match_eager(tile):
    case = build_case(small_problem("graph", nx=61, nz=45, nt=150, ns=3, np_=3))
    eager, graph = ctx(False), ctx(True)
    eager.set_tile(tile)
    graph.set_tile(tile)
    grid, geom = grid_geom(eager, case)
    x = dev(case.particles)
    dobs = dev(case.dobs)
    lp_g = torch.empty(3, dtype=torch.float64, device="cuda")
    g_g = torch.empty_like(x)
    for rep in range(4):
        with torch.no_grad():
            x.add_(float(rep))          # new values in the same buffer
        lp_e, g_e = vb.vip_grad_logpost(eager, grid, geom, x, dobs, case.sigma, ckpt_every=17,
                                        ws_tag="eager")
        lp_e, g_e = lp_e.clone(), g_e.clone()
        _ = torch.randn(1000, device="cuda").sum()   # unrelated eager work between replays
        vb.vip_grad_logpost(graph, grid, geom, x, dobs, case.sigma, ckpt_every=17,
                            logpost=lp_g, grad=g_g, ws_tag="graph")
        torch.cuda.synchronize()
        assert torch.equal(lp_e, lp_g) and torch.equal(g_e, g_g), rep
    assert len(graph._ws) >= 1
    eager.set_tile(-2)
    graph.set_tile(-2)


def test_graph_minibatch_subsets_differing_only_in_data_rows():
    """Graph mode keys its cache on the rows of d_obs a geometry reads: two
    one-shot minibatches with the same source position (shot 3 of the survey
    repeats shot 0's source with other recorded data) replay their own
    graphs, each equal to its eager result."""
    case = build_case(small_problem("graphmb", nx=61, nz=45, nt=150, ns=3, np_=2))
    eager, graph = ctx(False), ctx(True)
    grid, geom = grid_geom(eager, case)
    og = case.ogeom
    survey = vb.Geometry(list(og.src_iz) + [og.src_iz[0]], list(og.src_ix) + [og.src_ix[0]],
                         og.rec_iz, og.rec_ix, geom.wavelet)
    extra = case.dobs[:1] + case.sigma * np.random.default_rng(5).standard_normal(case.dobs[:1].shape)
    dobs = dev(np.concatenate([case.dobs, np.float32(extra)]))
    x = dev(case.particles)
    lp_g = torch.empty(2, dtype=torch.float64, device="cuda")
    g_g = torch.empty_like(x)
    first = {}
    for rep in range(3):
        for shots in ([0], [3], [3, 1]):
            lp_e, g_e = vb.vip_grad_logpost_minibatch(eager, grid, survey, x, dobs, case.sigma,
                                                      shots, ckpt_every=17, ws_tag="mbe")
            vb.vip_grad_logpost(graph, grid, survey.subset(shots), x, dobs, case.sigma,
                                ckpt_every=17, logpost=lp_g, grad=g_g, ws_tag="mbg")
            torch.cuda.synchronize()
            assert torch.equal(lp_e, lp_g) and torch.equal(g_e, g_g), (rep, shots)
            first.setdefault(tuple(shots), lp_e.clone())
    assert not torch.equal(first[(0,)], first[(3,)])
