"""Executions enqueue kernel launches only (no allocation, copy, memset or
synchronisation), so a caller can capture them into a HIP graph.  A captured
transform is replayed several times, with the program's own eager work and
synchronisations between the replays, and every replay must give the eager
result bit for bit."""
import pytest
import torch

from paper_1409_5757_amd import api, inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


@pytest.mark.parametrize("q,dtype,inplace", [(20, torch.complex128, False), (16, torch.complex64, True),
                                             (24, torch.complex64, False)])
def test_captured_transform_replays_bitwise(q, dtype, inplace):
    n = 1 << q
    x = torch.empty(n, dtype=dtype, device=DEV)
    inputs.fill_uniform_torch(x, seed=q)
    plan = api.Plan(n, dtype, -1, inplace, device=DEV)
    ref = x.clone()
    ref = plan.execute(ref) if inplace else plan.execute(ref, out=torch.empty_like(ref))
    torch.cuda.synchronize()

    src = torch.empty_like(x)
    dst = src if inplace else torch.empty_like(x)
    src.copy_(x)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream(DEV)
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            if inplace:
                plan.execute(src)
            else:
                plan.execute(src, out=dst)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for r in range(3):
        src.copy_(x)                       # eager work between the replays
        dst.zero_() if not inplace else None
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(dst, ref), f"replay {r}"
    plan.close()
