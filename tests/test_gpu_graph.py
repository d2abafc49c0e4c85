"""vl_step under HIP graph capture: one step captured (after an eager
warm-up step, which allocates the context's scratch on first use) and
replayed must advance the state exactly as eager steps do.  Two contexts
start from the same state; one is stepped eagerly, the other by replays of
its captured step, with the eager steps and a device synchronisation between
the replays, and every replay is compared bit for bit (f, moments, fields,
fluid state, clip and skip counters).  The step launches only kernels on the
caller's stream (with fitting off, one device-to-device copy of the moments)
and no memset."""
import numpy as np
import pytest

from gpu_util import ensure_lib
from paper_2109_06743_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_lib()


def _pair(cfg, f, fields, dtype):
    from paper_2109_06743_amd import vl
    out = []
    for _ in range(2):
        ctx = vl.Context(cfg, dtype)
        out.append((ctx, vl.StepState(ctx, f, fields)))
    return out


def _same(a, b):
    import torch
    for name in ("f", "mom_post", "mom_pre", "U"):
        for x, y in zip(getattr(a, name), getattr(b, name)):
            assert torch.equal(x, y), name
    assert torch.equal(a.fields, b.fields)
    assert torch.equal(a.counters, b.counters)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("case", ["2x3v_fit", "2x3v_nofit", "1x1v_fit"])
def test_step_graph_replays_match_eager(dtype, case):
    import torch
    from paper_2109_06743_amd import vl
    if case.startswith("2x3v"):
        cfg, f, F0 = W.gem(nx=16, ny=8, nv=8, dt=0.003, fit=case.endswith("_fit"), dtype=np.float64)
        fields = vl.yee_pack(F0)
    else:
        cfg, f = W.landau(nx=32, nv=32, fit=True)
        f, fields = [f], np.zeros(cfg["nx"])
    dt = cfg["dt"]
    (ca, sa), (cb, sb) = _pair(cfg, f, fields, dtype)
    ca.step(sa, dt)
    cb.step(sb, dt)
    torch.cuda.synchronize()
    _same(sa, sb)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=side):
        cb.step(sb, dt)                     # recorded, not run
    torch.cuda.synchronize()
    for k in range(4):
        g.replay()
        ca.step(sa, dt)
        torch.cuda.synchronize()
        _same(sa, sb)
