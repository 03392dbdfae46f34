"""Host-side logic of the serving loop: FIFO admission under an HBM budget and
a slot limit, and the request stream it is fed (no GPU needed)."""
import numpy as np

import plbm_synth as syn
from paper_2504_15018_amd.serving import Request, admissible, from_synth, summarize


def _req(i, nbytes, arrival=0.0):
    r = Request(i, arrival, "D2Q9", (8, 8), 0.8, 2.0)
    r.bytes = nbytes
    return r


def test_admits_in_order_until_budget():
    q = [_req(0, 40), _req(1, 30), _req(2, 20), _req(3, 5)]
    assert admissible(q, 0, 0, 100, 8) == 4
    assert admissible(q, 0, 20, 100, 8) == 2
    assert admissible(q, 0, 40, 100, 8) == 1
    assert admissible(q, 0, 70, 100, 8) == 0  # head does not fit: nothing behind it overtakes


def test_slot_limit():
    q = [_req(i, 1) for i in range(10)]
    assert admissible(q, 5, 0, 10**9, 8) == 3
    assert admissible(q, 8, 0, 10**9, 8) == 0


def test_head_of_line_blocking_keeps_arrival_order():
    q = [_req(0, 90), _req(1, 1)]
    assert admissible(q, 1, 20, 100, 8) == 0


def test_empty_queue():
    assert admissible([], 0, 0, 100, 8) == 0


def test_summary_percentiles():
    reqs = [_req(i, 1, arrival=float(i)) for i in range(5)]
    for i, r in enumerate(reqs):
        r.status = "converged"
        r.done = r.arrival + (i + 1)
    reqs[4].status = "failed"
    s = summarize(reqs, 10.0, 1000)
    assert s["converged"] == 4 and s["failed"] == 1
    assert s["latency_p50_s"] == np.percentile([1, 2, 3, 4], 50)
    assert s["solves_per_s"] == 0.4
    assert s["served_site_updates_per_s"] == 100.0


def test_request_stream_statistics():
    """Poisson arrivals at the stated rate; both lattice kinds; sizes, T/Tc and radii in range."""
    reqs = syn.request_stream(4000, 50.0, seed=0)
    t = np.array([r["arrival"] for r in reqs])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 1 / 50.0) < 3 * (1 / 50.0) / np.sqrt(len(gaps))
    # exponential gaps: coefficient of variation 1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.06
    kinds = [r["lattice"] for r in reqs]
    assert 0.45 < kinds.count("D2Q9") / len(kinds) < 0.55
    for r in reqs:
        side = r["dims"][0]
        lo, hi = (64, 1024) if r["lattice"] == "D2Q9" else (64, 192)
        assert lo <= side <= hi and len(set(r["dims"])) == 1
        assert 0.6 <= r["T_over_Tc"] <= 0.9
        assert 0.15 * side <= r["radius"] <= 0.35 * side
    # fixed seed: same stream twice
    assert syn.request_stream(10, 50.0, seed=0) == syn.request_stream(10, 50.0, seed=0)
    assert all(r["problem"] == "droplet" for r in reqs)


def test_request_stream_with_channels():
    """A channel fraction turns that share of the requests into channels between walls (width on the last axis,
    channel_len nodes along the others, the body force along x); the droplet requests of the same seed are
    unchanged."""
    base = syn.request_stream(400, 50.0, seed=2)
    mixed = syn.request_stream(400, 50.0, seed=2, channel_frac=0.3, width2d=(32, 96), width3d=(24, 48),
                               channel_len=6, body_force=2e-6)
    chans = [r for r in mixed if r["problem"] == "channel"]
    assert 0.2 < len(chans) / len(mixed) < 0.4
    for r, b in zip(mixed, base):
        assert r["arrival"] == b["arrival"] and r["lattice"] == b["lattice"] and r["T_over_Tc"] == b["T_over_Tc"]
        if r["problem"] == "droplet":
            assert r == b
        else:
            lo, hi = (32, 96) if r["lattice"] == "D2Q9" else (24, 48)
            assert lo <= r["dims"][-1] <= hi and all(v == 6 for v in r["dims"][:-1])
            assert len(r["dims"]) == (2 if r["lattice"] == "D2Q9" else 3)
            assert r["body_force"] == 2e-6 and r["radius"] == 0.0
    req = from_synth(chans[:1])[0]
    assert req.problem == "channel" and req.walls and req.body_force == 2e-6


def test_unknown_problem_is_refused():
    import pytest
    with pytest.raises(ValueError):
        Request(0, 0.0, "D2Q9", (8, 8), 0.8, 2.0, problem="bubble")


def test_lane_key_splits_kinds_by_size():
    from paper_2504_15018_amd.serving import Server
    srv = Server.__new__(Server)  # lane_key needs only the thresholds
    srv.split_nodes = (262144,)
    small = Request(0, 0.0, "D2Q9", (511, 511), 0.8, 2.0)
    large = Request(1, 0.0, "D2Q9", (512, 512), 0.8, 2.0)
    cube = Request(2, 0.0, "D3Q19", (64, 64, 64), 0.8, 2.0)
    assert srv.lane_key(small) == ("D2Q9", 0) and srv.lane_key(large) == ("D2Q9", 1)
    assert srv.lane_key(cube) == ("D3Q19", 1)
    srv.split_nodes = ()
    assert {srv.lane_key(r) for r in (small, large)} == {("D2Q9", 0)}
