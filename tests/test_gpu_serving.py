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


def test_served_results_match_the_plain_fp64_method():
    """Continuous batching in float32 against the plain float64 method on the same GPU: each request of a
    small stream is served (MRT, f32, converged at max|du|/step <= 1e-8 over 100 steps), then solved alone in
    float64 on the single-lattice path to the same test.  Bar: the droplet's coexistence densities (centre
    and far field) within 1e-3 relative; the Laplace jump p_EOS(centre) - p_EOS(far field) and the
    spurious-current maximum are reported beside them."""
    require_gpu()
    import plbm_synth as syn
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.serving import Server, from_synth, solve_alone

    fmt("serving_vs_fp64")
    reqs = from_synth(syn.request_stream(6, 50.0, seed=5, side2d=(48, 96), side3d=(20, 32), t_range=(0.75, 0.9)))
    srv = Server(budget_bytes=1 << 34, max_slots=8, max_tiles=1 << 16, check_every=100, tol=1e-8,
                 max_steps=400_000, collision="mrt", record_results=True)
    out = srv.run(reqs, time_limit=150)
    srv.close()
    print({k: v for k, v in out.items() if k != "records"}, flush=True)
    assert out["unfinished"] == 0 and out["failed"] == 0 and out["rejected"] == 0
    worst = 0.0
    for r in reqs:
        assert r.status == "converged", r.record()
        st, steps, ref = solve_alone(r, storage="f64", collision="mrt", tol=1e-8, max_steps=400_000)
        assert st == "converged", (r.record(), st, steps)
        prm = N.plbm_params_pr_lattice(r.T_over_Tc, 0.326, 2.0, 1.0, 1.0, 1.0)

        def p_eos(x):
            b = prm.pr_b
            return x * prm.pr_R * prm.pr_T / (1 - b * x) - prm.pr_a * prm.pr_alpha * x * x / (1 + 2 * b * x - b * b * x * x)

        e_in = abs(r.result["rho_in"] - ref["rho_in"]) / ref["rho_in"]
        e_out = abs(r.result["rho_out"] - ref["rho_out"]) / ref["rho_out"]
        dp, dp64 = (p_eos(r.result["rho_in"]) - p_eos(r.result["rho_out"]),
                    p_eos(ref["rho_in"]) - p_eos(ref["rho_out"]))
        fmt("serving_vs_fp64_case", id=r.id, lattice=r.lattice, dims=r.dims, T=f"{r.T_over_Tc:.3f}",
            steps_f32=r.steps, steps_f64=steps, rho_in_err=f"{e_in:.2e}", rho_out_err=f"{e_out:.2e}",
            laplace_err=f"{abs(dp - dp64) / abs(dp64):.2e}",
            max_u_err=f"{abs(r.result['max_u'] - ref['max_u']) / ref['max_u']:.2e}")
        worst = max(worst, e_in, e_out)
    assert worst <= 1e-3


def test_a_request_cancelled_mid_flight_leaves_the_rest_intact():
    """A running request withdrawn mid-flight is detached and its memory released once its lane's chunk has
    completed; the other requests are unaffected (bitwise the same as alone)."""
    require_gpu()
    import plbm_synth as syn
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    from paper_2504_15018_amd.serving import Server, from_synth

    fmt("serving_cancel")
    reqs = from_synth(syn.request_stream(5, 200.0, seed=4, side2d=(32, 64), side3d=(12, 20), t_range=(0.75, 0.9)))
    victim = max(reqs, key=lambda r: r.nodes)
    srv = Server(budget_bytes=1 << 34, max_slots=4, max_tiles=4096, check_every=50, tol=1e-7, max_steps=20_000,
                 keep_lattices=True)
    state = {"asked": None}

    def watch(_msg):
        if state["asked"] is None and victim.status == "running" and victim.steps >= 100:
            state["asked"] = victim.steps
            srv.cancel(victim.id)

    out = srv.run(reqs, time_limit=120, log=watch)
    print({k: v for k, v in out.items() if k != "records"}, flush=True)
    assert state["asked"] is not None
    assert victim.status == "cancelled" and victim.done is not None
    # at most one more chunk ran between the request and the release
    assert victim.steps <= state["asked"] + 50
    assert out["cancelled"] == 1 and out["unfinished"] == 0
    assert srv.used == 0 and not srv.resident
    for r in reqs:
        if r is victim:
            continue
        assert r.status in ("converged", "capped")
        solo = Lattice(r.lattice, r.dims, r.params, collision="bgk", storage="f32")
        solo.init_shape(N.PLBM_SHAPE_DROPLET, r.params.rho_l, r.params.rho_v, W=5.0, R=r.radius,
                        centre=[n / 2.0 for n in r.dims])
        solo.step(r.steps)
        assert np.array_equal(solo.populations(), r.lat.populations()), r.record()
        solo.close()
        r.lat.close()
    victim.lat.close()
    srv.close()


def test_served_channels_and_droplets_match_solo_runs_and_the_fp64_method():
    """A stream that sweeps channel width as well as droplet size (two-phase channels between walls, driven
    along x, beside periodic droplets, in the same lanes: the batch launches walled and periodic lattices as
    separate groups).  Each served result (f32, MRT, converged at max|du|/step <= 1e-8) is bitwise the same as
    the request run alone for the same number of steps, and its two coexisting densities (a channel's liquid
    and vapour layers) agree with the plain float64 method, solved alone to the same test, within 1e-3; the
    peak speed is reported beside them."""
    require_gpu()
    import plbm_synth as syn
    from paper_2504_15018_amd.serving import Server, from_synth, setup_lattice, solve_alone

    fmt("serving_channels")
    reqs = from_synth(syn.request_stream(8, 100.0, seed=24, side2d=(40, 64), side3d=(20, 28), t_range=(0.78, 0.85),
                                         r_frac=(0.3, 0.35), channel_frac=0.5, width2d=(24, 48), width3d=(16, 32),
                                         channel_len=8, body_force=1e-6))
    assert {(r.problem, r.lattice) for r in reqs} == {(p, k) for p in ("droplet", "channel") for k in ("D2Q9", "D3Q19")}
    srv = Server(budget_bytes=1 << 34, max_slots=8, max_tiles=1 << 16, check_every=100, tol=1e-8,
                 max_steps=300_000, collision="mrt", record_results=True, keep_lattices=True)
    out = srv.run(reqs, time_limit=150)
    print({k: v for k, v in out.items() if k != "records"}, flush=True)
    assert out["unfinished"] == 0 and out["failed"] == 0 and out["rejected"] == 0
    worst = 0.0
    for r in reqs:
        assert r.status == "converged", r.record()
        _, solo = setup_lattice(r, "f32", "mrt")
        solo.step(r.steps)
        assert np.array_equal(solo.populations(), r.lat.populations()), r.record()
        solo.close()
        r.lat.close()
        st, steps, ref = solve_alone(r, storage="f64", collision="mrt", tol=1e-8, max_steps=300_000)
        assert st == "converged", (r.record(), st, steps)
        e_in = abs(r.result["rho_in"] - ref["rho_in"]) / ref["rho_in"]
        e_out = abs(r.result["rho_out"] - ref["rho_out"]) / ref["rho_out"]
        fmt("serving_channels_case", id=r.id, problem=r.problem, lattice=r.lattice, dims=r.dims,
            T=f"{r.T_over_Tc:.3f}", steps_f32=r.steps, steps_f64=steps, rho_in_err=f"{e_in:.2e}",
            rho_out_err=f"{e_out:.2e}", max_u=f"{ref['max_u']:.3e}",
            max_u_err=f"{abs(r.result['max_u'] - ref['max_u']) / ref['max_u']:.2e}")
        worst = max(worst, e_in, e_out)
        assert ref["rho_in"] > 5 * ref["rho_out"]  # the droplet, or the liquid layer below the vapour, persists
    assert worst <= 1e-3
    srv.close()


def test_size_class_lanes_keep_fifo_and_solo_results():
    """With lanes split by lattice size, arrival order holds within each (kind, size class) lane, small and
    large lattices of one kind advance on their own streams, and every result is still bitwise the same as
    the request run alone."""
    require_gpu()
    import plbm_synth as syn
    from paper_2504_15018_amd.serving import Server, from_synth, setup_lattice

    fmt("serving_size_lanes")
    reqs = from_synth(syn.request_stream(10, 200.0, seed=3, side2d=(24, 72), side3d=(12, 24), t_range=(0.75, 0.9)))
    srv = Server(budget_bytes=1 << 34, max_slots=4, max_tiles=4096, check_every=50, tol=1e-6, max_steps=6000,
                 keep_lattices=True, split_nodes=(2500,))
    classes = {srv.lane_key(r) for r in reqs}
    assert ("D2Q9", 0) in classes and ("D2Q9", 1) in classes  # both D2Q9 size classes occur
    out = srv.run(reqs, time_limit=120)
    print({k: v for k, v in out.items() if k != "records"}, flush=True)
    assert out["unfinished"] == 0 and out["rejected"] == 0 and out["failed"] == 0
    assert set(srv.lanes) == classes
    for key in classes:
        order = sorted((r for r in reqs if srv.lane_key(r) == key), key=lambda r: r.arrival)
        admits = [r.admit for r in order]
        assert admits == sorted(admits)
    for r in reqs:
        assert r.status in ("converged", "capped")
        _, solo = setup_lattice(r, "f32", "bgk")
        solo.step(r.steps)
        assert np.array_equal(solo.populations(), r.lat.populations()), r.record()
        solo.close()
        r.lat.close()
    srv.close()
