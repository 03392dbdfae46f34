"""plbm_step inside a caller's HIP graph: on a stream the caller is capturing,
the step launches go into the caller's graph (the library captures no graph of
its own there).  The captured steps are replayed several times, with eager
work and synchronisation between the replays, and every replay must leave the
same populations, bitwise, as the same steps taken eagerly on a twin lattice:
the pseudopotential update and the well-balanced scheme (two launches per step)."""
import numpy as np
import pytest

from gpu_cases import fmt, lib_params, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scheme", ["pseudopotential", "well-balanced"])
def test_steps_captured_in_a_caller_graph_replay_like_eager_steps(scheme):
    require_gpu()
    import torch
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice

    fmt("graph_capture", scheme=scheme)
    dims = (40, 24, 18)
    if scheme == "pseudopotential":
        prm = lib_params()
        kw = {}
        W = 5.0
    else:
        prm = N.plbm_params_paper_lattice(0.0375, 1.187, 3.0, 2.0, 1.0, 1.0, 1.0, [0.0, 0.0, 0.0])
        kw = {"wb_k": 0.15}
        W = 6.0
    lats = [Lattice("D3Q19", dims, prm, collision="mrt", storage="f32", **kw) for _ in range(2)]
    for lat in lats:
        lat.init_shape(N.PLBM_SHAPE_DROPLET, prm.rho_l, prm.rho_v, W=W, R=7.0)
    captured, eager = lats
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=captured.stream):
        N.plbm_step(captured.h, 2)  # recorded, not run
    torch.cuda.synchronize()
    assert np.array_equal(captured.populations(), eager.populations())
    for k in range(4):
        g.replay()
        eager.step(2)
        torch.cuda.synchronize()
        _ = eager.reduce()  # eager work between replays
        got, ref = captured.populations(), eager.populations()
        fmt("graph_capture_replay", k=k, max_abs_diff=f"{np.max(np.abs(got - ref)):.1e}")
        assert np.array_equal(got, ref), k
    for lat in lats:
        lat.close()
