"""The serving loop on the GPU: requests arriving while others run are admitted
as memory frees up, never beyond the HBM budget, in arrival order within each
lattice kind (each kind has its own batch and stream), and each served result
is bitwise the same as the same solve run alone."""
import numpy as np
import pytest

from gpu_cases import fmt, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pattern", ["ab", "aa"])
def test_serving_small_stream_matches_solo_runs(pattern):
    """Served in place or not, every result equals a solo A-B run bitwise."""
    require_gpu()
    import plbm_synth as syn
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    from paper_2504_15018_amd.serving import Server, from_synth

    fmt("serving_small_stream", pattern=pattern)
    reqs = from_synth(syn.request_stream(10, 200.0, seed=3, side2d=(24, 72), side3d=(12, 24), t_range=(0.75, 0.9)))
    big = max(reqs, key=lambda r: r.nodes)
    srv = Server(budget_bytes=0, max_slots=4, max_tiles=4096, check_every=50, tol=1e-6, max_steps=6000,
                 keep_lattices=True, pattern=pattern)
    # budget: room for the largest request and a bit more, so later arrivals queue behind running ones
    sizes = [srv._desc_bytes(r) for r in reqs]
    srv.budget = int(max(sizes) * 1.5)
    out = srv.run(reqs, time_limit=120)
    print({k: v for k, v in out.items() if k != "records"}, flush=True)
    assert out["unfinished"] == 0 and out["rejected"] == 0 and out["failed"] == 0
    assert out["peak_bytes"] <= srv.budget
    for kind in ("D2Q9", "D3Q19"):  # FIFO within each lattice kind's lane
        order = sorted((r for r in reqs if r.lattice == kind), key=lambda r: r.arrival)
        admits = [r.admit for r in order]
        assert admits == sorted(admits)
    assert any(r.admit > r.arrival + 1e-3 for r in reqs)  # some requests waited for memory
    for r in reqs:
        assert r.status in ("converged", "capped")
        assert r.steps % 50 == 0 and r.lat.time == r.steps
        solo = Lattice(r.lattice, r.dims, r.params, collision="bgk", storage="f32")
        solo.init_shape(N.PLBM_SHAPE_DROPLET, r.params.rho_l, r.params.rho_v, W=5.0, R=r.radius,
                        centre=[n / 2.0 for n in r.dims])
        solo.step(r.steps)
        assert np.array_equal(solo.populations(), r.lat.populations()), r.record()
        solo.close()
        r.lat.close()
    assert big.status in ("converged", "capped")
    srv.close()


def test_serving_refuses_a_request_without_coexistence_and_serves_the_rest():
    """T/Tc >= 1 has no liquid-vapour coexistence: the parameter solve fails, the request is refused, the
    loop keeps serving the others."""
    require_gpu()
    from paper_2504_15018_amd.serving import Request, Server

    fmt("serving_reject")
    reqs = [Request(0, 0.0, "D2Q9", (48, 48), 0.85, 10.0), Request(1, 0.0, "D2Q9", (40, 40), 1.1, 8.0),
            Request(2, 0.0, "D3Q19", (16, 16, 16), 0.85, 4.0)]
    srv = Server(budget_bytes=1 << 34, max_slots=4, max_tiles=4096, check_every=50, tol=1e-6, max_steps=4000)
    out = srv.run(reqs, time_limit=60)
    srv.close()
    assert reqs[1].status == "rejected" and reqs[1].error
    assert reqs[0].status in ("converged", "capped") and reqs[2].status in ("converged", "capped")
    assert out["rejected"] == 1 and out["unfinished"] == 0
