"""A full Strang step (REXI stage between two Heun half steps) captured in a HIP
graph: after one eager step the step only enqueues kernels (no allocation,
copy, memset or synchronisation), so it can be captured; three replays from
the same state, with eager work on the device between them, must each equal
an eager step bit for bit (every kernel sums in a fixed order)."""
import numpy as np
import pytest

from paper_1805_06557_amd.inputs import jet_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec_name", ["fp64", "fp32+bf16", "fp32+fp16"])
def test_strang_step_graph_replays_match_eager(prec_name):
    from paper_1805_06557_amd import api
    prec = {"fp64": 0, "fp32+bf16": api.PREC_FP32_SOLVE | api.PREC_BF16_SPLIT,
            "fp32+fp16": api.PREC_FP32_SOLVE | api.PREC_FP16_SPLIT}[prec_name]
    L, nlat, nlon, dt, N = 63, 96, 192, 1800.0, 160
    alpha, beta, _, _ = api.rexi_coefficients(api.FN_EXP, N, 6.0, 25.0)
    ctx = api.SWE(L, nlat, nlon, prec=prec)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        U = torch.from_numpy(jet_state(L, 5)).cuda()
        S0 = U.clone()
        V = torch.empty_like(U)
        ctx.strang_step(alpha, beta, dt, U, V, side)      # first call: allocations, caches
        U.copy_(S0)
        ctx.strang_step(alpha, beta, dt, U, V, side)
        ref = V.clone()
        side.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            ctx.strang_step(alpha, beta, dt, U, V, side)
        for rep in range(3):
            U.copy_(S0)
            V.fill_(float("nan"))
            side.synchronize()
            g.replay()
            side.synchronize()
            assert torch.equal(V, ref), (prec_name, rep)
            # eager device work between replays
            W = torch.empty_like(U)
            ctx.strang_step(alpha, beta, dt, S0, W, side)
            side.synchronize()
            assert torch.equal(W, ref)
    assert np.all(np.isfinite(ref.cpu().numpy()))
    ctx.close()
