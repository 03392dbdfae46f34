"""Continuous-batching request loop for P-LBM solves (plbm_batch_*).

A request asks for one solve: lattice kind and size, reduced temperature of
the lattice Peng-Robinson EOS, and the problem: a static droplet of a given
radius (periodic box), or a two-phase channel (liquid below vapour between
half-way bounce-back walls on the last axis, whose extent is the channel
width, driven by a body force along x).  The loop

  * admits queued requests in arrival order while a batch slot is free and the
    device bytes of every resident lattice (plbm_lattice_bytes) plus the new
    one stay within the HBM budget; a request that does not fit waits;
  * gives each admitted request its own lattice (a PyTorch device buffer),
    initialised on the device (plbm_init_shape) and attached to the batch;
  * advances the resident lattices of each lattice kind together with
    plbm_batch_step (one batch and stream per kind, one launch per lattice
    type per step, replayed from a captured HIP graph); the kinds advance at
    their own rates;
  * every `check_every` steps reads the per-lattice diagnostics
    (plbm_batch_diag): a lattice whose residual max|u(t) - u(t-k)|/k is at or
    below `tol` is converged; NaN or rho <= 0 marks it failed; a lattice that
    reaches `max_steps` is capped.  Finished lattices are detached and their
    memory released at once, so queued requests can take their place.

Every lattice's result is bitwise the same as stepping it alone: the batch
only changes which workgroup computes which tile.  With `record_results`, a
converged lattice's droplet densities (centre and far corner) and maximum
speed are read on the device before it is released (a channel's liquid and
vapour layer densities and its peak speed); `solve_alone` runs one request by
itself on the plain single-lattice path (any storage, e.g. float64) to the
same convergence test, for comparison with the served result.  Both set a
request up with `setup_lattice`.
"""
import time

import numpy as np

from . import native as N
from .lattice import Lattice


class Request:
    def __init__(self, rid, arrival, lattice, dims, T_over_Tc, radius, problem="droplet", body_force=0.0):
        if problem not in ("droplet", "channel"):
            raise ValueError(f"unknown problem {problem!r}")
        self.id = rid
        self.arrival = float(arrival)
        self.lattice = lattice
        self.dims = tuple(int(v) for v in dims)
        self.T_over_Tc = float(T_over_Tc)
        self.radius = float(radius)
        self.problem = problem
        self.body_force = float(body_force)  # channel: along x, lattice units
        self.admit = None
        self.done = None
        self.steps = 0
        self.status = "queued"
        self.bytes = 0
        self.residual = None
        self.lat = None
        self.slot = None
        self.params = None
        self.error = None
        self.result = None  # rho_in / rho_out and max|u| at convergence (record_results)

    @property
    def nodes(self):
        return int(np.prod(self.dims))

    def record(self):
        return {"id": self.id, "arrival": self.arrival, "admit": self.admit, "done": self.done,
                "latency": None if self.done is None else self.done - self.arrival, "steps": self.steps,
                "status": self.status, "bytes": self.bytes, "nodes": self.nodes, "lattice": self.lattice,
                "dims": self.dims, "T_over_Tc": self.T_over_Tc, "problem": self.problem,
                "residual": self.residual, "error": self.error, "result": self.result}

    @property
    def walls(self):
        return self.problem == "channel"


def setup_lattice(req, storage, collision, stream=None, pattern="ab", width=5.0):
    """The request's lattice parameters and its initialised lattice: a tanh droplet of the request's radius
    at the box centre, or liquid below vapour at half the channel width (tanh width `width`) between walls on
    the last axis with the body force along x."""
    bf = [req.body_force, 0.0, 0.0] if req.walls else None
    prm = N.plbm_params_pr_lattice(req.T_over_Tc, 0.326, 2.0, 1.0, 1.0, 1.0, bf)
    lat = Lattice(req.lattice, req.dims, prm, collision=collision, storage=storage, stream=stream, pattern=pattern,
                  walls=req.walls)
    try:
        if req.walls:
            ax = len(req.dims) - 1
            lat.init_shape(N.PLBM_SHAPE_LAYERS, prm.rho_l, prm.rho_v, W=width, level=req.dims[ax] / 2.0, axis=ax)
        else:
            lat.init_shape(N.PLBM_SHAPE_DROPLET, prm.rho_l, prm.rho_v, W=width, R=req.radius,
                           centre=[n / 2.0 for n in req.dims])
    except BaseException:
        lat.close()
        raise
    return prm, lat


def result_readout(torch, lat, req, max_u):
    """The two coexisting densities of the request's current state, from its moments computed on the device:
    a droplet's centre (node dims // 2, rho_in) and far field (node 0, rho_out); a channel's liquid and vapour
    layers at a quarter and three quarters of the width (lateral node 0).  lat's stream must be idle or own
    the work before it."""
    dims = req.dims
    n = int(np.prod(dims))
    d = len(dims)
    rho = torch.empty(n, dtype=torch.float64, device="cuda")
    u = torch.empty(d * n, dtype=torch.float64, device="cuda")
    N.plbm_moments_device(lat.h, rho.data_ptr(), u.data_ptr())
    lat.stream.synchronize()

    def flat(idx):  # x fastest
        k, stride = 0, 1
        for i, ext in zip(idx, dims):
            k += i * stride
            stride *= ext
        return k

    if req.walls:
        h = dims[-1]
        i_in, i_out = flat((0,) * (d - 1) + (h // 4,)), flat((0,) * (d - 1) + ((3 * h) // 4,))
    else:
        i_in, i_out = flat([ext // 2 for ext in dims]), 0
    return {"rho_in": float(rho[i_in].item()), "rho_out": float(rho[i_out].item()), "max_u": float(max_u)}


def solve_alone(req, storage="f64", collision="mrt", check_every=100, tol=1e-8, max_steps=2_000_000, width=5.0,
                time_limit=None):
    """Run one request alone on the plain single-lattice path (plbm_step / plbm_reduce) until its residual
    max|u(t) - u(t-k)|/k is at or below tol; returns (status, steps, result)."""
    import torch

    _, lat = setup_lattice(req, storage, collision, width=width)
    t0 = time.perf_counter()
    try:
        lat.reduce()
        steps, status, d = 0, "capped", None
        while steps < max_steps:
            lat.step(check_every)
            steps += check_every
            d = lat.reduce(allow_unstable=True)
            if d.flags & (N.PLBM_FLAG_NAN | N.PLBM_FLAG_RHO_NONPOS):
                status = "failed"
                break
            if d.max_du_per_step <= tol:
                status = "converged"
                break
            if time_limit is not None and time.perf_counter() - t0 > time_limit:
                status = "timeout"
                break
        res = result_readout(torch, lat, req, d.max_u if d is not None else 0.0)
        return status, steps, res
    finally:
        lat.close()


def admissible(queue, n_resident, used, budget, max_slots):
    """How many requests at the head of the FIFO queue can be admitted now.

    Arrival order is kept: a head request that does not fit (no free slot, or
    its bytes would push the resident total over the budget) blocks the ones
    behind it, so a large request is never starved by smaller later ones."""
    k = 0
    for r in queue:
        if n_resident + k >= max_slots or used + r.bytes > budget:
            break
        used += r.bytes
        k += 1
    return k


def from_synth(reqs):
    return [Request(r["id"], r["arrival"], r["lattice"], r["dims"], r["T_over_Tc"], r["radius"],
                    r.get("problem", "droplet"), r.get("body_force", 0.0)) for r in reqs]


class Lane:
    """One batch of resident lattices of one lattice kind (and size class), on its own stream."""

    def __init__(self, torch, kind, max_slots, max_tiles):
        self.kind = kind
        self.stream = torch.cuda.Stream()  # default priority
        nb = N.plbm_batch_bytes(max_slots, max_tiles)
        self._bmem = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        ptr = (self._bmem.data_ptr() + 255) // 256 * 256
        self.batch = N.plbm_batch_create(max_slots, max_tiles, ptr, nb, self.stream.cuda_stream)
        self.resident = {}  # slot -> Request
        self.queue = []     # admitted in arrival order
        self.inflight = 0   # steps enqueued and not yet checked
        self.event = None


class Server:
    """Serving loop over one lane per lattice kind (D2Q9, D3Q19), or per kind and size class.

    Each lane is a batch on its own stream and advances at its own rate: a
    D2Q9 step of a few small lattices takes tens of microseconds, a D3Q19 step
    of large ones milliseconds, and lattices of one kind need similar step
    counts, so the cheap kind is not held to the other's pace.  The loop
    enqueues `check_every` steps on every idle lane without waiting, then
    polls the lanes' completion events; a finished chunk is checked (residual,
    health) and the lane's queue is admitted while that lane is idle.  The HBM
    budget is shared; each lane keeps arrival order in its own queue.  With
    `split_nodes` each kind is split further by lattice size, so that small
    lattices, which need few steps, are not held to the step rate of the
    largest lattice resident in their kind's lane.
    """

    def __init__(self, budget_bytes, max_slots=64, max_tiles=1 << 20, check_every=100, tol=1e-8,
                 max_steps=2_000_000, storage="f32", collision="bgk", keep_lattices=False, width=5.0,
                 pattern="ab", record_results=False, split_nodes=()):
        import torch

        self.torch = torch
        self.budget = int(budget_bytes)
        self.max_slots = max_slots  # per lane
        self.max_tiles = max_tiles
        self.check_every = int(check_every)
        self.tol = tol
        self.max_steps = int(max_steps)
        self.storage = storage
        self.collision = collision
        self.pattern = pattern  # "aa": in place, about half the population memory per resident lattice
        self.keep = keep_lattices
        self.record_results = record_results
        self.width = width
        # node-count thresholds that split each lattice kind into size classes with lanes of their own (a
        # small lattice then advances at its class's pace, not at that of the largest lattice of its kind)
        self.split_nodes = tuple(sorted(int(v) for v in split_nodes))
        self.lanes = {}
        self.used = 0
        self.peak_used = 0
        self.peak_resident = 0
        self._cancel = set()

    def cancel(self, rid):
        """Withdraw request `rid`.  A queued or not yet arrived request is dropped; a resident one is detached
        and its memory released once its lane's chunk in flight has completed (its kernels may still use the
        lattice until then).  It ends with status "cancelled"."""
        self._cancel.add(rid)

    def lane_key(self, req):
        """(lattice kind, size class) of a request; the class counts the thresholds at or below its nodes."""
        return (req.lattice, sum(req.nodes >= t for t in self.split_nodes))

    def _lane(self, key):
        if key not in self.lanes:
            self.lanes[key] = Lane(self.torch, key, self.max_slots, self.max_tiles)
        return self.lanes[key]

    @property
    def resident(self):
        return {(k, s): r for k, lane in self.lanes.items() for s, r in lane.resident.items()}

    def close(self):
        """Cancel what is still resident (its `done` stays None) and release the batches."""
        for lane in self.lanes.values():
            lane.stream.synchronize()
            for r in list(lane.resident.values()):
                self._retire(lane, r, "cancelled", None)
            N.plbm_batch_destroy(lane.batch)
            lane.batch = None
        self.lanes = {}

    # ---- admission ----
    def _desc_bytes(self, req):
        from .lattice import make_desc
        return N.plbm_lattice_bytes(make_desc(req.lattice, req.dims, self.collision, self.storage,
                                              walls=req.walls, pattern=self.pattern)) + 256

    def _admit(self, lane, req, now):
        req.params, lat = setup_lattice(req, self.storage, self.collision, stream=lane.stream, pattern=self.pattern,
                                        width=self.width)
        req.lat = lat
        lat.reduce()  # stores u(0) for the first residual
        req.slot = N.plbm_batch_attach(lane.batch, lat.h)
        req.admit = now
        req.status = "running"
        lane.resident[req.slot] = req
        self.used += req.bytes
        self.peak_used = max(self.peak_used, self.used)
        self.peak_resident = max(self.peak_resident, sum(len(ln.resident) for ln in self.lanes.values()))

    def _retire(self, lane, req, status, now, max_u=0.0):
        if status == "converged" and self.record_results:
            req.result = result_readout(self.torch, req.lat, req, max_u)
        N.plbm_batch_detach(lane.batch, req.slot)
        del lane.resident[req.slot]
        req.status = status
        req.done = now
        self.used -= req.bytes
        if not self.keep:
            req.lat.close()
            req.lat = None

    def _admit_queue(self, lane, now):
        for _ in range(admissible(lane.queue, len(lane.resident), self.used, self.budget, self.max_slots)):
            req = lane.queue.pop(0)
            try:
                self._admit(lane, req, now)
            except N.PlbmError as e:  # e.g. no coexistence at this T/Tc: refuse the request, keep serving
                if req.lat is not None:
                    req.lat.close()
                    req.lat = None
                req.status = "rejected"
                req.error = str(e)

    def _check(self, lane, now):
        """Residual and health of every lattice of a lane whose chunk has completed."""
        n = lane.inflight
        diag = N.plbm_batch_diag(lane.batch, self.max_slots)
        served = 0
        for slot, req in list(lane.resident.items()):
            d = diag[slot]
            req.steps += n
            served += req.nodes * n
            req.residual = d.max_du_per_step
            if d.flags & (N.PLBM_FLAG_NAN | N.PLBM_FLAG_RHO_NONPOS):
                self._retire(lane, req, "failed", now)
            elif req.residual <= self.tol:
                self._retire(lane, req, "converged", now, d.max_u)
            elif req.steps >= self.max_steps:
                self._retire(lane, req, "capped", now)
        lane.inflight = 0
        lane.event = None
        return served

    def _drop_cancelled(self, lane, now):
        """Cancelled requests of an idle lane: queued ones leave the queue, resident ones are released."""
        for r in [r for r in lane.queue if r.id in self._cancel]:
            lane.queue.remove(r)
            r.status, r.done = "cancelled", now
        for r in [r for r in lane.resident.values() if r.id in self._cancel]:
            self._retire(lane, r, "cancelled", now)

    # ---- the loop ----
    def run(self, requests, time_limit=None, log=None):
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            r.bytes = self._desc_bytes(r)
            if r.bytes > self.budget:
                r.status = "rejected"
        pending = [r for r in reqs if r.status != "rejected"]
        t0 = time.perf_counter()
        served_updates = 0
        i = 0

        def busy():
            return any(lane.resident or lane.queue or lane.inflight for lane in self.lanes.values())

        while i < len(pending) or busy():
            now = time.perf_counter() - t0
            if time_limit is not None and now > time_limit:
                break
            while i < len(pending) and pending[i].arrival <= now:
                r = pending[i]
                i += 1
                if r.id in self._cancel:
                    r.status, r.done = "cancelled", now
                    continue
                self._lane(self.lane_key(r)).queue.append(r)
            progressed = False
            for lane in self.lanes.values():
                if lane.inflight and lane.event.query():
                    served_updates += self._check(lane, time.perf_counter() - t0)
                    progressed = True
                if not lane.inflight:
                    if self._cancel:
                        self._drop_cancelled(lane, time.perf_counter() - t0)
                    if lane.queue:
                        self._admit_queue(lane, time.perf_counter() - t0)
                    if lane.resident:
                        N.plbm_batch_step(lane.batch, self.check_every)
                        lane.inflight = self.check_every
                        lane.event = self.torch.cuda.Event()
                        lane.event.record(lane.stream)
                        progressed = True
            if not progressed:
                # nothing completed: wait a little for the next chunk or arrival
                if not any(lane.inflight for lane in self.lanes.values()) and i < len(pending):
                    time.sleep(max(0.0, min(pending[i].arrival - now, 0.01)))
                else:
                    time.sleep(2e-5)
            if log is not None:
                log(f"[serve] t={now:.2f}s resident={len(self.resident)} "
                    f"queued={sum(len(ln.queue) for ln in self.lanes.values())} "
                    f"done={sum(r.done is not None for r in reqs)}/{len(reqs)}")
        for lane in self.lanes.values():
            lane.stream.synchronize()
        makespan = time.perf_counter() - t0
        out = summarize(reqs, makespan, served_updates)
        out.update(peak_bytes=self.peak_used, peak_resident=self.peak_resident, budget_bytes=self.budget)
        return out


def summarize(reqs, makespan, served_updates):
    done = [r for r in reqs if r.status == "converged"]
    lat = np.array([r.done - r.arrival for r in done]) if done else np.array([])
    pct = (lambda q: float(np.percentile(lat, q))) if len(lat) else (lambda q: None)
    return {
        "requests": len(reqs),
        "converged": len(done),
        "capped": sum(r.status == "capped" for r in reqs),
        "failed": sum(r.status == "failed" for r in reqs),
        "rejected": sum(r.status == "rejected" for r in reqs),
        "cancelled": sum(r.status == "cancelled" for r in reqs),
        "unfinished": sum(r.done is None and r.status != "rejected" for r in reqs),
        "makespan_s": makespan,
        "solves_per_s": len(done) / makespan if makespan > 0 else 0.0,
        "latency_p50_s": pct(50),
        "latency_p99_s": pct(99),
        "served_site_updates_per_s": served_updates / makespan if makespan > 0 else 0.0,
        "records": [r.record() for r in reqs],
    }
