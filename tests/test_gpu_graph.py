"""GPU: the per-coordinate entry point under HIP graph capture.

ss_grad_hess launches on the caller's stream and records no memset, so a
caller can capture a run of coordinates into a graph and replay it.  The
graph is replayed several times with eager calls of the library in between,
and every replay is compared with the eager results (the workspace epochs
advance inside the kernels, so a replay is the same computation as an
eager call).  The comparison allows last-bit differences: the decoupled
look-back forms a tile's prefix from whichever predecessor values are
visible first, so the rounding of the prefix can vary from run to run.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from test_gpu_parity import make_case, gpu_problem  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("model,n", [("cox", 50_001), ("fg", 30_000), ("cox", 5_000_000)])
def test_grad_hess_graph_replay(model, n):
    c = make_case(model, n, 6, 21, 0, 0.05, False)
    prob = gpu_problem(model, c)
    p = c["p"]
    eager = torch.empty(p, 3, dtype=torch.float64, device=DEV)
    for j in range(p):
        prob.grad_hess(j, out=eager[j])
    torch.cuda.synchronize()
    want = eager.cpu().numpy().copy()

    outs = torch.zeros(p, 3, dtype=torch.float64, device=DEV)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):          # warm-up on the capture stream
        for j in range(p):
            prob.grad_hess(j, out=outs[j])
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for j in range(p):
            prob.grad_hess(j, out=outs[j])
    for rep in range(3):
        outs.fill_(0.0)
        g.replay()
        torch.cuda.synchronize()
        got = outs.cpu().numpy()
        np.testing.assert_allclose(got, want, rtol=1e-11, atol=0.0)
        # eager work between replays, on the same workspace
        for j in (p - 1, 0):
            prob.grad_hess(j, out=eager[j])
        torch.cuda.synchronize()
        np.testing.assert_allclose(eager.cpu().numpy(), want, rtol=1e-11, atol=0.0)
    assert prob.workspace_error() == 0
