"""Stream capture of the time step: lb_step allocates nothing, synchronises
nothing and clears nothing with memset, so a caller can capture n steps
into a HIP graph (torch.cuda.CUDAGraph) and replay them. An even n keeps the
ping-pong consistent from one replay to the next (the graph reads the buffer
it was captured reading). Each replay, with the program's own eager work
and synchronisations in between, must leave the same bytes as the same
steps run eagerly."""
import numpy as np
import pytest

from paper_1804_01918_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1804_01918_amd import lb  # noqa: E402

LX, LY = 64, 128  # a multiple of every clustered layout's vector length
CASES = [
    ("f64", "caosoa", {}),
    ("f32s", "soa", {}),
    ("f16s", "caosoa", {}),
    ("f64", "caosoa", dict(force=(0.0, -1e-4), walls=True, t_bottom=1.05, t_top=0.95)),
    ("f32s", "caosoa", "learned"),
]


def _make(stream, prec, layout, bc, fields, net):
    with torch.cuda.stream(stream):
        lat = lb.Lattice(LX, LY, 0.8, fields, precision=prec, layout=layout,
                         **(bc if isinstance(bc, dict) else {}))
        if bc == "learned":
            lat.set_surrogate(net, 1e9)
    return lat


@pytest.mark.parametrize("prec,layout,bc", CASES, ids=[f"{p}-{l}-{'plain' if b == {} else ('bc' if isinstance(b, dict) else b)}"
                                                       for p, l, b in CASES])
def test_graph_replay_equals_eager(prec, layout, bc):
    fields = [torch.from_numpy(a).cuda() for a in inputs.rayleigh_taylor(LX, LY, seed=3)]
    net = None
    if bc == "learned":
        net = lb.Mlp(1024)
        net.init(5)
        pre, post = lb.pairgen(4096, 7, 0.8)
        net.fit_normalization(pre, post, 0.8)
    cap = torch.cuda.Stream()
    eager_stream = torch.cuda.Stream()
    lat_g = _make(cap, prec, layout, bc, fields, net)
    lat_e = _make(eager_stream, prec, layout, bc, fields, net)
    with torch.cuda.stream(cap):
        lat_g.step(2)          # warm-up outside the capture
    with torch.cuda.stream(eager_stream):
        lat_e.step(2)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=cap):
        lat_g.step(8)
    torch.cuda.synchronize()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        with torch.cuda.stream(eager_stream):
            lat_e.step(8)
        junk = torch.randn(4096, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        a = lat_g.bufs[lat_g.current_buffer()]
        b = lat_e.bufs[lat_e.current_buffer()]
        assert torch.equal(a, b), f"replay {rep}: graph and eager steps differ"
        assert bool(torch.isfinite(junk))
    rho_g = lat_g.moments()[0]
    rho_e = lat_e.moments()[0]
    torch.cuda.synchronize()
    assert torch.equal(rho_g, rho_e)
    lat_g.close()
    lat_e.close()
    if net is not None:
        net.close()
