"""Host-side logic of the serving loop: FIFO admission under an HBM budget and
a slot limit, and the request stream it is fed (no GPU needed)."""
import numpy as np

import plbm_synth as syn
from paper_2504_15018_amd.serving import Request, admissible, summarize


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
