"""Throughput of the fused P-LBM step on one MI355X.

Workload (the step the metric is quoted on): D3Q19 static droplet, 256^3
periodic lattice, float32 populations and arithmetic (psi evaluated in
float64), MRT collision with Guo forcing, lattice Peng-Robinson EOS at
T/Tc = 0.8 (acentric factor 0.326), eps = 2, kappa = 1, tau = 1, droplet
radius 48 with a tanh interface of width 5.  Synthetic input, resident in HBM
before timing starts.

A timed step is one fused update of every node (psi, force stencil, MRT
collision with forcing, streaming); the global reduction (mass, momentum,
max|u|, residual, health flags) runs every 100 steps inside the timed region,
as in a production run.

Prints one JSON line.  `roofline` reports the step kernel's algorithmic HBM
traffic (2 Q S bytes per node update: read and write 19 float32 populations)
over its average launch duration measured with HIP events on the lattice's
stream; `cpu_baseline` times the FP64 NumPy oracle on a bounded sample of the
same workload on the host (one single-threaded process per core, aggregated).

Before the step benchmark (--serve-first 0: after it), a bounded serving leg
runs the serving form at a sustainable rate (Poisson arrivals at 0.5 requests/s of the C5 mix for 40 s:
D2Q9 64^2..1024^2 and D3Q19 64^3..192^3 droplets, T/Tc in [0.6, 0.9], float32
MRT, converged at max|du|/step <= 1e-8) and reports solves/s and p50/p99
time to converged solution in the same line, with the accuracy of the
served results: the cheapest converged requests are solved again alone in
float64 on the single-lattice path, and their droplet densities compared.

`--pattern aa` times the in-place storage pattern instead (one population
array; a psi pass and the in-place update per step).  Its roofline covers the
two launches of a step together: 3 Q S + 2 C bytes per node (C = 4 bytes,
the psi value, 8 for float64) over the step's duration.

`--well-balanced` times the well-balanced scheme instead, on the same
lattice, droplet and storage with the paper's EOS (lattice densities 0.0375 /
1.187, interface width parameter 3, gradient coefficient 0.15; the lattice
Peng-Robinson fluid is too stiff for its explicit square-gradient force at
this interface width): two launches per step (the chemical-potential pass
reads the populations and writes mu, C bytes per node; the update reads the
populations and mu and writes the populations), 3 Q S + 2 C algorithmic bytes
per node over the step's duration.

`--precision` runs the precision form instead: the 384 x 384 x 128 channel
in every storage format (coexistence densities and u_x profile against the
float64 run), then static droplets (D2Q9 512^2, D3Q19 128^3; densities,
Laplace jump and spurious currents against float64).
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
REDUCE_EVERY = 100
PROFILE = os.path.join(ROOT, "profiles", "k_step_d3q19_256cubed_mrt_f32.json")
KERNEL_SOURCES = ["plbm_device.hpp", "plbm_step.hpp", "plbm_aux.hpp", "plbm_aa.hpp", "plbm_launch.hpp",
                  "plbm_kernels_inst.hpp", "plbm_k_f32.hip"]


def kernel_source_hash():
    """sha256 over the sources and compile flags of the float32 step kernel (identifies the kernel a profile
    was taken of)."""
    import hashlib
    from paper_2504_15018_amd import build
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2504_15018_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    # compile flags without the include directories (absolute paths differ between checkouts)
    flags = [a for a in build.COMMON[1:] + build.SOURCES["plbm_k_f32.hip"] if not a.startswith("-I")]
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


def profiled_traffic(storage, collision, size):
    """HBM bytes per update launch from the committed rocprofv3 counters, if they were taken of this kernel
    and workload; else None."""
    if (storage, collision, size) != ("f32", "mrt", 256) or not os.path.exists(PROFILE):
        return None
    with open(PROFILE) as fh:
        prof = json.load(fh)
    if prof.get("kernel_source_hash") != kernel_source_hash():
        return None
    return prof["traffic_bytes"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


CPU_CAP = 16  # host cores granted to one GPU's jobs on the measurement hosts


def cpu_baseline(seconds=12.0):
    """Time the oracle on a 48^3 D3Q19 MRT droplet (same physics): one single-threaded child process per host
    core available to this job (at most CPU_CAP, the host share of one GPU), each on its own lattice, run
    together; the aggregate rate is the baseline."""
    code = r"""
import os, sys, time, json
sys.path.insert(0, %r)
import numpy as np
import plbm_synth as syn
from oracle import eos as E, params as P, step as S
from oracle.lattice import D3Q19
e = E.PengRobinsonEOS(0.8, 0.326)
rv, rl, _ = P.coexistence(e, 2.0)
dims = (48, 48, 48)
co = syn.grid(dims)
rho = syn.droplet(co, dims, rv, rl, R=9.0, W=5.0)
p = S.StepParams(D3Q19, e, eps=2.0, kappa=1.0, tau_v=1.0, tau_l=1.0, rho_v=rv, rho_l=rl, collision="mrt")
f = S.init_equilibrium(D3Q19, rho)
f = S.step(p, f)
t0 = time.perf_counter(); n = 0
while time.perf_counter() - t0 < %f:
    f = S.step(p, f); n += 1
dt = time.perf_counter() - t0
print(json.dumps({"mlups": rho.size * n / dt / 1e6, "steps": n, "seconds": dt, "nodes": rho.size}))
""" % (ROOT, seconds)
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    nproc = max(1, min(CPU_CAP, ncpu))
    procs = [subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                              env=env) for _ in range(nproc)]
    outs = []
    for pr in procs:
        try:
            so, se = pr.communicate(timeout=600)
        except subprocess.TimeoutExpired:
            pr.kill()
            so, se = pr.communicate()
        if pr.returncode != 0:
            log(se[-2000:])
            continue
        outs.append(json.loads(so.strip().splitlines()[-1]))
    if not outs:
        return None
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    total = sum(o["mlups"] for o in outs)
    host = os.cpu_count() or 0
    return {"value": round(total, 4), "unit": "MLUPS", "cores": len(outs), "kind": "oracle",
            "host_cores": host, "cores_available": ncpu,
            "sample": f"FP64 NumPy oracle, D3Q19 48^3 MRT droplet (same EOS/physics): {len(outs)} independent "
                      f"single-threaded processes for {seconds:.0f} s each, {min(o['steps'] for o in outs)}-"
                      f"{max(o['steps'] for o in outs)} steps per process, {total / len(outs):.3f} MLUPS per "
                      f"process; {model}; host has {host} logical cores, {ncpu} available to this job, "
                      f"processes capped at {CPU_CAP} (the host share of one GPU)"}


def copy_probe(torch, nbytes=2 << 30, reps=20):
    """Plain device-to-device copy of nbytes: the measured HBM reference for the roofline."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3 / reps
    print(json.dumps({"copy_bytes": nbytes, "copy_ms": round(dt * 1e3, 4),
                      "copy_GBps_read_plus_write": round(2 * nbytes / dt / 1e9, 1)}), flush=True)


PR_OMEGA = 0.326  # acentric factor of the paper's fluid


def stream_probe(torch, nodes=256 ** 3, reps=50):
    """Reference rates of the population access pattern on this GPU (libplbm_probe.so): 19 float32 arrays in
    the blocked population layout read and written once per launch (the update's algorithmic bytes with no
    halo, stencil or collision), and a plain float4 copy of the same bytes."""
    import ctypes
    lib_path = os.path.join(ROOT, "paper_2504_15018_amd", "libplbm_probe.so")
    if not os.path.exists(lib_path):
        raise RuntimeError(f"{lib_path} is not built: run `python -m paper_2504_15018_amd.build`")
    lib = ctypes.CDLL(lib_path)
    lib.plbm_probe_stream19.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]
    lib.plbm_probe_copy4.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
    nfl = 19 * 32 * ((nodes + 31) // 32)
    a = torch.ones(nfl, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)

    def timed(fn):
        for _ in range(3):
            if fn() != 0:
                raise RuntimeError("probe launch failed")
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    lib.plbm_probe_stream19v.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int,
                                         ctypes.c_void_p]
    lib.plbm_probe_copy4u.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
    lib.plbm_probe_stream19s.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_void_p]
    lib.plbm_probe_stream19h.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int,
                                         ctypes.c_void_p]
    lib.plbm_probe_pingpong.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p]
    lib.plbm_probe_stream19_lds.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_void_p]
    lib.plbm_probe_read19.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p]
    lib.plbm_probe_copy4nt.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
    lib.plbm_probe_stream19x.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_uint32, ctypes.c_void_p]
    moved = 2 * 19 * 4 * nodes
    out = {"nodes": nodes}
    runs = [("stream19_blocked", lambda: lib.plbm_probe_stream19(a.data_ptr(), b.data_ptr(), nodes, sp)),
            ("stream19_blocked_2_per_thread", lambda: lib.plbm_probe_stream19v(a.data_ptr(), b.data_ptr(), nodes, 2, sp)),
            ("stream19_blocked_4_per_thread", lambda: lib.plbm_probe_stream19v(a.data_ptr(), b.data_ptr(), nodes, 4, sp)),
            ("stream19_blocks_of_64", lambda: lib.plbm_probe_stream19x(a.data_ptr(), b.data_ptr(), nodes, 64, 1, 0, sp)),
            ("stream19_blocks_of_64_2_per_thread",
             lambda: lib.plbm_probe_stream19x(a.data_ptr(), b.data_ptr(), nodes, 64, 2, 0, sp)),
            ("stream19_blocks_of_128", lambda: lib.plbm_probe_stream19x(a.data_ptr(), b.data_ptr(), nodes, 128, 1, 0, sp)),
            ("stream19_blocks_of_128_2_per_thread",
             lambda: lib.plbm_probe_stream19x(a.data_ptr(), b.data_ptr(), nodes, 128, 2, 0, sp)),
            ("stream19_blocks_of_128_4_per_thread",
             lambda: lib.plbm_probe_stream19x(a.data_ptr(), b.data_ptr(), nodes, 128, 4, 0, sp)),
            # the same with three workgroups per CU (unused LDS), the cap that suits the one-node stream
            *[(f"stream19_blocks_of_{xb}_{v}_per_thread_lds_53k",
               (lambda xb=xb, v=v: lib.plbm_probe_stream19x(a.data_ptr(), b.data_ptr(), nodes, xb, v, 53 * 1024, sp)))
              for xb, v in ((64, 2), (128, 2), (128, 4))],
            ("stream19_plain_stores", lambda: lib.plbm_probe_stream19s(a.data_ptr(), b.data_ptr(), nodes, 0, 0, sp)),
            ("stream19_plain_stores_interleaved",
             lambda: lib.plbm_probe_stream19s(a.data_ptr(), b.data_ptr(), nodes, 0, 1, sp)),
            ("stream19_interleaved", lambda: lib.plbm_probe_stream19s(a.data_ptr(), b.data_ptr(), nodes, 1, 1, sp)),
            ("copy4", lambda: lib.plbm_probe_copy4(a.data_ptr(), b.data_ptr(), 19 * 4 * nodes, sp)),
            # the one-node stream with its workgroups per CU capped by unused LDS (8, 5, 4, 3, 2 of 160 KiB)
            *[(f"stream19_lds_{k}k", (lambda k=k: lib.plbm_probe_stream19_lds(a.data_ptr(), b.data_ptr(), nodes,
                                                                               k * 1024, sp)))
              for k in (20, 32, 40, 53, 64)],
            # ping-pong pairs (two passes per call; rates of both passes' bytes): the second pass in the first's
            # order, or reversed so that it starts on the blocks the first wrote last
            ("pingpong_same_order", lambda: lib.plbm_probe_pingpong(a.data_ptr(), b.data_ptr(), nodes, 1, 0, sp)),
            ("pingpong_reversed", lambda: lib.plbm_probe_pingpong(a.data_ptr(), b.data_ptr(), nodes, 1, 1, sp)),
            ("pingpong_plain_stores_same_order",
             lambda: lib.plbm_probe_pingpong(a.data_ptr(), b.data_ptr(), nodes, 0, 0, sp)),
            ("pingpong_plain_stores_reversed",
             lambda: lib.plbm_probe_pingpong(a.data_ptr(), b.data_ptr(), nodes, 0, 1, sp)),
            # read-mostly passes (19 values read, one written per node); rates of those bytes
            ("read19_linear", lambda: lib.plbm_probe_read19(a.data_ptr(), b.data_ptr(), nodes, 0, sp)),
            ("read19_tiles_per_plane", lambda: lib.plbm_probe_read19(a.data_ptr(), b.data_ptr(), nodes, 1, sp)),
            ("read19_tile_columns_2", lambda: lib.plbm_probe_read19(a.data_ptr(), b.data_ptr(), nodes, 2, sp)),
            ("read19_tile_columns_16", lambda: lib.plbm_probe_read19(a.data_ptr(), b.data_ptr(), nodes, 3, sp)),
            # 16-bit populations: half the bytes (the rates below are of those bytes)
            ("half_stream19", lambda: lib.plbm_probe_stream19h(a.data_ptr(), b.data_ptr(), nodes, 1, sp)),
            ("half_stream19_2_per_thread", lambda: lib.plbm_probe_stream19h(a.data_ptr(), b.data_ptr(), nodes, 2, sp)),
            ("half_stream19_4_per_thread", lambda: lib.plbm_probe_stream19h(a.data_ptr(), b.data_ptr(), nodes, 4, sp)),
            ("copy4_nontemporal", lambda: lib.plbm_probe_copy4nt(a.data_ptr(), b.data_ptr(), 19 * 4 * nodes, sp)),
            ("copy4_4_per_thread", lambda: lib.plbm_probe_copy4u(a.data_ptr(), b.data_ptr(), 19 * 4 * nodes, sp))]
    if nodes != 256 ** 3:  # the read-mostly kernels index a cube of side 256 (and refuse other sizes)
        runs = [r for r in runs if not r[0].startswith("read19")]
    for name, fn in runs:
        t = timed(fn)
        out[name + "_us"] = round(t * 1e6, 1)
        nbytes = moved // 2 if name.startswith("half_") else (20 * 4 * nodes if name.startswith("read19") else moved)
        if name.startswith("pingpong"):
            nbytes = 2 * moved
        out[name + "_GBps"] = round(nbytes / t / 1e9, 1)
    return out


def droplet_precision_run(N, Lattice, lattice, n, R, steps, tr=0.8):
    """Static droplet (MRT, periodic) in every storage format: the Laplace jump p_EOS(centre) - p_EOS(far
    field), the droplet radius from its equivalent area or volume, the spurious-current maximum max|u| and
    the densities at the centre and in the far field, each against the float64 run."""
    import numpy as np

    def pr_pressure(prm, r):  # Peng-Robinson in the lattice parameters the library resolved
        b = prm.pr_b
        return r * prm.pr_R * prm.pr_T / (1.0 - b * r) - prm.pr_a * prm.pr_alpha * r * r / (1.0 + 2.0 * b * r - b * b * r * r)

    prm = N.plbm_params_pr_lattice(tr, PR_OMEGA, 2.0, 1.0, 1.0, 1.0)
    dims = (n, n) if lattice == "D2Q9" else (n, n, n)
    centre = [n / 2.0] * len(dims)
    rows = {}
    for st in ["f64", "f32", "f16s", "bf16s", "f16r", "bf16r"]:
        lat = Lattice(lattice, dims, prm, collision="mrt", storage=st)
        lat.init_shape(N.PLBM_SHAPE_DROPLET, prm.rho_l, prm.rho_v, W=5.0, R=R, centre=centre)
        lat.step(steps)
        rho, u = lat.moments()
        d = lat.reduce(allow_unstable=True)
        lat.close()
        mid = tuple(n // 2 for _ in dims)
        r_in, r_out = float(rho[mid]), float(rho[(0,) * len(dims)])
        frac = float(np.sum((rho - r_out) / (r_in - r_out)))
        radius = np.sqrt(frac / np.pi) if lattice == "D2Q9" else (3.0 * frac / (4.0 * np.pi)) ** (1.0 / 3.0)
        dp = pr_pressure(prm, r_in) - pr_pressure(prm, r_out)
        rows[st] = {"rho_in": r_in, "rho_out": r_out, "laplace_jump": dp, "radius": float(radius),
                    "spurious_max_u": float(np.sqrt((u ** 2).sum(axis=0)).max()), "flags": d.flags}
        log(f"[precision] {lattice} droplet {st}: dp {dp:.6e}, max|u| {rows[st]['spurious_max_u']:.3e}, flags {d.flags}")
    ref = rows["f64"]
    for st, r in rows.items():
        r["rho_in_rel_err"] = abs(r["rho_in"] - ref["rho_in"]) / ref["rho_in"]
        r["rho_out_rel_err"] = abs(r["rho_out"] - ref["rho_out"]) / ref["rho_out"]
        r["laplace_jump_rel_err"] = abs(r["laplace_jump"] - ref["laplace_jump"]) / abs(ref["laplace_jump"])
        r["spurious_max_u_rel_err"] = abs(r["spurious_max_u"] - ref["spurious_max_u"]) / ref["spurious_max_u"]
    name = f"{n}^2" if lattice == "D2Q9" else f"{n}^3"
    return {"workload": f"{lattice} static droplet {name} periodic, R = {R:g}, tanh width 5, PR T/Tc = {tr}, MRT, "
                        f"{steps} steps", "storages": rows}


def precision_run(torch, N, Lattice, steps):
    """Layered channel between plates, 384 x 384 x 128 (walls on z, F_g = 1e-6 x, BGK tau = 1), in every
    storage format; coexistence densities and the u_x profile against the float64 run."""
    dims = (384, 384, 128)
    prm = N.plbm_params_pr_lattice(0.8, 0.326, 2.0, 1.0, 1.0, 1.0, body_force=(1e-6, 0.0, 0.0))
    rows = {}
    cols = {}
    for st in ["f64", "f32", "f16s", "bf16s", "f16r", "bf16r"]:
        lat = Lattice("D3Q19", dims, prm, collision="bgk", storage=st, walls=True)
        lat.init_shape(N.PLBM_SHAPE_LAYERS, prm.rho_l, prm.rho_v, W=5.0, level=64.0, axis=2)
        rho = torch.empty(lat.N, dtype=torch.float64, device="cuda")
        u = torch.empty(3 * lat.N, dtype=torch.float64, device="cuda")
        lat.step(20)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        lat.step(steps - 20)
        e1.record(lat.stream)
        lat.stream.synchronize()
        ms = e0.elapsed_time(e1) / (steps - 20)
        N.plbm_moments_device(lat.h, rho.data_ptr(), u.data_ptr())
        lat.stream.synchronize()
        r = rho.view(128, 384, 384)
        ux = u.view(3, 128, 384, 384)[0]
        uniform = bool((r == r[:, :1, :1]).all()) and bool((ux == ux[:, :1, :1]).all())
        cols[st] = (r[:, 0, 0].cpu().numpy(), ux[:, 0, 0].cpu().numpy())
        d = lat.reduce(allow_unstable=True)
        S = {"f64": 8, "f32": 4}.get(st, 2)
        extra = 4 if st.endswith("r") else 0  # reference densities read and written
        rows[st] = {"ms_per_step": round(ms, 4), "MLUPS": round(lat.N / ms / 1e3, 1),
                    "GBps_algorithmic": round((2 * 19 * S + extra) * lat.N / ms / 1e6, 1),
                    "laterally_uniform": uniform, "flags": d.flags}
        log(f"[precision] {st}: {ms:.4f} ms/step, flags {d.flags}")
        lat.close()
        del rho, u
    r64, u64 = cols["f64"]
    for st in rows:
        r, uu = cols[st]
        rows[st]["rho_l_rel_err"] = float(abs(r[32] - r64[32]) / r64[32])
        rows[st]["rho_v_rel_err"] = float(abs(r[96] - r64[96]) / r64[96])
        rows[st]["ux_profile_rel_err"] = float(abs(uu - u64).max() / abs(u64).max())
    return {"workload": f"D3Q19 384x384x128 channel, half-way bounce-back plates on z, F_g = 1e-6 x, layered "
                        f"liquid below z = 64, PR T/Tc = 0.8, BGK tau = 1, {steps} steps",
            "rho_v_f64": float(r64[96]), "rho_l_f64": float(r64[32]), "ux_max_f64": float(abs(u64).max()),
            "storages": rows}


CHANNELS = dict(width2d=(64, 512), width3d=(64, 192), channel_len=8, body_force=1e-6)


def serve_run(N, seconds, budget_gb, collision="mrt", channel_frac=0.0, split_nodes=()):
    """Continuous-batching serving of the Poisson request stream (50 req/s, 500 requests, seed 0): D2Q9 64^2 to
    1024^2 and D3Q19 64^3 to 192^3 droplets, T/Tc in [0.6, 0.9], radius [0.15, 0.35] of the side, f32, BGK or
    MRT, converged at max|du|/step <= 1e-8 over 100 steps; with channel_frac > 0 that share of the requests are
    two-phase channels instead (width 64..512 in 2-D, 64..192 in 3-D, 8 nodes along the other axes, body force
    1e-6 along x).  Then a second stream at 0.8 x the measured capacity."""
    import plbm_synth as syn
    from paper_2504_15018_amd.serving import Server, from_synth

    def one(reqs, label):
        srv = Server(budget_bytes=int(budget_gb * 1e9), max_slots=64, max_tiles=1 << 21, check_every=100,
                     tol=1e-8, max_steps=2_000_000, collision=collision, split_nodes=split_nodes)
        last = [0.0]

        def progress(m):
            if time.perf_counter() - last[0] > 10:
                last[0] = time.perf_counter()
                log(f"[serve:{label}] {m}")

        out = srv.run(reqs, time_limit=seconds, log=progress)
        srv.close()
        out.pop("records")
        return out

    first = one(from_synth(syn.request_stream(500, 50.0, seed=0, channel_frac=channel_frac, **CHANNELS)), "c5")
    cap = first["solves_per_s"]
    rate = max(0.8 * cap, 1e-3)
    second = one(from_synth(syn.request_stream(max(4, int(rate * seconds * 1.2)), rate, seed=1,
                                               channel_frac=channel_frac, **CHANNELS)), "sustainable")
    return {"collision": collision, "channel_frac": channel_frac, "split_nodes": list(split_nodes), "stream": first,
            "sustainable": dict(second, rate_per_s=rate)}


def serving_leg(N, seconds=40.0, rate=0.5, seed=1, check_seconds=25.0, budget_gb=240.0, channel_frac=0.0,
                split_nodes=()):
    """Serving form at a sustainable rate, bounded: Poisson arrivals of the C5 mix for `seconds`, float32 MRT,
    converged at max|du|/step <= 1e-8 over 100 steps; then the cheapest converged requests solved again alone
    in float64 (within `check_seconds`) to state the served results' accuracy (droplet densities at the
    centre and in the far field; bar 1e-3 relative)."""
    import plbm_synth as syn
    from paper_2504_15018_amd.serving import Server, from_synth, solve_alone

    reqs = from_synth(syn.request_stream(max(4, int(rate * seconds * 1.2)), rate, seed=seed,
                                         channel_frac=channel_frac, **CHANNELS))
    srv = Server(budget_bytes=int(budget_gb * 1e9), max_slots=64, max_tiles=1 << 21, check_every=100, tol=1e-8,
                 max_steps=2_000_000, collision="mrt", record_results=True, split_nodes=split_nodes)
    out = srv.run(reqs, time_limit=seconds)
    srv.close()
    out.pop("records")
    conv = sorted([r for r in reqs if r.status == "converged"], key=lambda r: r.nodes * r.steps)
    bytes_per_node = {"D2Q9": 144, "D3Q19": 304}  # float64 populations read and written per update
    cases = []
    t0 = time.perf_counter()
    for r in conv:
        left = check_seconds - (time.perf_counter() - t0)
        est = r.steps * (max(1.2e-5, r.nodes * bytes_per_node[r.lattice] / 4e12) + 1e-6)
        if est > left:
            continue
        st, steps, ref = solve_alone(r, storage="f64", collision="mrt", tol=1e-8, max_steps=2 * r.steps + 1000,
                                     time_limit=left)
        row = {"lattice": r.lattice, "problem": r.problem, "dims": list(r.dims), "T_over_Tc": round(r.T_over_Tc, 4),
               "steps_f32": r.steps, "steps_f64": steps, "f64_status": st}
        if st == "converged":
            row["rho_in_rel_err"] = abs(r.result["rho_in"] - ref["rho_in"]) / ref["rho_in"]
            row["rho_out_rel_err"] = abs(r.result["rho_out"] - ref["rho_out"]) / ref["rho_out"]
            row["max_u_rel_err"] = abs(r.result["max_u"] - ref["max_u"]) / max(ref["max_u"], 1e-300)
        cases.append(row)
        log(f"[serve-leg] f64 check {row}")
    ok = [c for c in cases if "rho_in_rel_err" in c]
    worst = max([max(c["rho_in_rel_err"], c["rho_out_rel_err"]) for c in ok], default=None)
    out.update({
        "workload": f"Poisson arrivals at {rate} requests/s for {seconds:g} s (seed {seed}): D2Q9 64^2..1024^2 and "
                    f"D3Q19 64^3..192^3 static droplets, Peng-Robinson T/Tc in [0.6, 0.9], radius 0.15..0.35 of "
                    f"the side, f32 storage, MRT, converged at max|du|/step <= 1e-8 over 100 steps"
                    + (f"; {channel_frac:g} of the requests two-phase channels (width 64..512 / 64..192, 8 nodes "
                       f"along the other axes, body force 1e-6)" if channel_frac > 0 else ""),
        "rate_per_s": rate, "window_s": seconds,
        "accuracy_vs_f64": {"checked": len(ok), "max_coexistence_density_rel_err": worst, "bar": 1e-3,
                            "cases": cases},
    })
    for k in ("makespan_s", "solves_per_s", "latency_p50_s", "latency_p99_s"):
        if out.get(k) is not None:
            out[k] = round(out[k], 4)
    out["served_gsite_updates_per_s"] = round(out.pop("served_site_updates_per_s") / 1e9, 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--collision", default="mrt", choices=["mrt", "bgk"])
    ap.add_argument("--storage", default="f32", choices=["f64", "f32", "f16s", "bf16s", "f16r", "bf16r"])
    ap.add_argument("--pattern", default="ab", choices=["ab", "aa"],
                    help="population storage pattern: two arrays (ab) or in place (aa)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--well-balanced", action="store_true",
                    help="time the well-balanced scheme (paper EOS fluid, gradient coefficient 0.15)")
    ap.add_argument("--u0", type=float, default=0.0,
                    help="uniform initial velocity along x (0.05: the Galilean-invariance variant of the droplet)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain device-to-device copy of 2 GiB (HBM reference for the roofline)")
    ap.add_argument("--stream-probe", action="store_true",
                    help="reference rates: 19 arrays streamed in the population layout, and a float4 copy")
    ap.add_argument("--precision", action="store_true",
                    help="storage-format comparison on the 384x384x128 channel instead of the step benchmark")
    ap.add_argument("--precision-steps", type=int, default=20000)
    ap.add_argument("--precision-droplets", type=int, default=1,
                    help="with --precision: also the Laplace jump and spurious currents of static droplets "
                         "(D2Q9 512^2, D3Q19 128^3) by storage format (0 skips them)")
    ap.add_argument("--serve", action="store_true", help="serving-loop run instead of the step benchmark")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-budget-gb", type=float, default=240.0)
    ap.add_argument("--serve-leg-seconds", type=float, default=40.0,
                    help="length of the bounded serving leg (0 skips it)")
    ap.add_argument("--serve-first", type=int, default=1,
                    help="1 (default): run the serving leg before the step benchmark; 0: after it")
    ap.add_argument("--serve-split-nodes", default="262144",
                    help="comma-separated node counts that split each lattice kind's serving lane by size "
                         "(empty: one lane per kind)")
    ap.add_argument("--serve-channel-frac", type=float, default=0.0,
                    help="share of the served requests that are two-phase channels (width sweep) instead of droplets")
    ap.add_argument("--serve-collision", default="mrt", choices=["bgk", "mrt"],
                    help="collision of the served lattices (MRT: fewer unstable requests at low T/Tc)")
    args = ap.parse_args()
    split = tuple(int(v) for v in args.serve_split_nodes.split(",") if v.strip())
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the lattice update is not sharded across GPUs here); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice

    if args.copy_probe:
        copy_probe(torch)
        return
    if args.stream_probe:
        print(json.dumps({"metric": "reference rates of the population access pattern", **stream_probe(torch)}),
              flush=True)
        return
    N.load()
    if args.precision:
        out = {"metric": "coexistence density error vs float64 by storage format",
               **precision_run(torch, N, Lattice, args.precision_steps)}
        if args.precision_droplets:
            out["droplets"] = [droplet_precision_run(N, Lattice, "D2Q9", 512, 64.0, 20000),
                               droplet_precision_run(N, Lattice, "D3Q19", 128, 32.0, 10000)]
        print(json.dumps(out), flush=True)
        return
    if args.serve:
        print(json.dumps({"metric": "solves/s + p50/p99 time to converged solution",
                          **serve_run(N, args.serve_seconds, args.serve_budget_gb, args.serve_collision,
                                      args.serve_channel_frac, split)}),
              flush=True)
        return
    serving = None

    def run_serving_leg():
        out = serving_leg(N, seconds=args.serve_leg_seconds, channel_frac=args.serve_channel_frac, split_nodes=split)
        log(f"[bench] serving leg: {out['converged']} converged, {out['solves_per_s']} solves/s, "
            f"p50 {out['latency_p50_s']} s, p99 {out['latency_p99_s']} s")
        torch.cuda.empty_cache()
        return out

    if args.serve_leg_seconds > 0 and args.serve_first:
        serving = run_serving_leg()
    n = args.size
    dims = (n, n, n)
    wb = args.well_balanced
    if wb:
        prm = N.plbm_params_paper_lattice(0.0375, 1.187, 3.0, 2.0, 1.0, 1.0, 1.0)
    else:
        prm = N.plbm_params_pr_lattice(0.8, 0.326, 2.0, 1.0, 1.0, 1.0)
    log(f"[bench] coexistence rho_v={prm.rho_v:.6f} rho_l={prm.rho_l:.6f}")
    lat = Lattice("D3Q19", dims, prm, collision=args.collision, storage=args.storage, pattern=args.pattern,
                  wb_k=0.15 if wb else 0.0, wb_rho0=0.0375 if wb else 0.0)
    R = 48.0 * n / 256.0
    lat.init_shape(N.PLBM_SHAPE_DROPLET, prm.rho_l, prm.rho_v, W=6.0 if wb else 5.0, R=R, centre=[n / 2.0] * 3,
                   u0=(args.u0, 0.0, 0.0))
    stream = lat.stream
    lat.step(0)  # captures the replay graphs now, outside the timed region
    log(f"[bench] lattice {dims} D3Q19 {args.collision} {args.storage} pattern {args.pattern}, "
        f"{lat.nbytes / 2**30:.2f} GiB; "
        f"warmup {args.warmup}")
    lat.step(args.warmup)
    d0 = lat.reduce()
    torch.cuda.synchronize()
    log(f"[bench] warmup done: mass={d0.mass:.6e} max_u={d0.max_u:.3e}")

    ev = []
    K = args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    n_reduce = 0
    while done < K:
        chunk = min(REDUCE_EVERY, K - done)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.step(chunk)
        e1.record(stream)
        ev.append((e0, e1, chunk))
        done += chunk
        if done % REDUCE_EVERY == 0:
            d = lat.reduce()
            n_reduce += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    kernel_ms = sum(a.elapsed_time(b) for a, b, _ in ev)
    avg_kernel_s = kernel_ms / 1e3 / K
    nodes = lat.N
    ms_per_step = wall * 1e3 / K
    mlups = nodes * K / wall / 1e6
    S = {"f64": 8, "f32": 4}.get(args.storage, 2)
    # locally shifted storage also reads and writes a 2-byte reference density per node (twice in place: the
    # psi pass writes the new one, the update reads it for the encoder)
    RB = 0 if args.storage in ("f64", "f32", "f16s", "bf16s") else 2
    if wb:  # chemical-potential pass (Q S read, C written) + update (2 Q S, C of mu read)
        bytes_per_launch = (3 * 19 * S + 2 * (8 if args.storage == "f64" else 4)) * nodes
    elif args.pattern == "aa":  # psi pass (Q S read, C written) + in-place update (2 Q S, C of psi read)
        bytes_per_launch = (3 * 19 * S + 2 * (8 if args.storage == "f64" else 4) + 4 * RB) * nodes
    else:
        bytes_per_launch = (2 * 19 * S + 2 * RB) * nodes
    achieved = bytes_per_launch / avg_kernel_s / 1e9
    dfin = lat.reduce()
    log(f"[bench] {K} steps in {wall:.3f} s; step kernel avg {avg_kernel_s * 1e3:.4f} ms; "
        f"mass drift {(dfin.mass - d0.mass) / d0.mass:.2e}; flags {dfin.flags}")
    if dfin.flags & (N.PLBM_FLAG_NAN | N.PLBM_FLAG_RHO_NONPOS):
        log("[bench] lattice became unstable")
        sys.exit(3)

    nbytes = lat.nbytes
    lat.close()
    del lat
    torch.cuda.empty_cache()
    if args.serve_leg_seconds > 0 and not args.serve_first:
        serving = run_serving_leg()
    cpu = None if args.no_cpu_baseline else cpu_baseline()
    tb = profiled_traffic(args.storage, args.collision, n) if (args.pattern == "ab" and not wb) else None
    traffic = None if tb is None else round(tb / 1e9, 4)  # GB per update launch
    out = {
        "metric": "MLUPS & % HBM peak (D3Q19 P-LBM step); solves/s + p99 latency at fixed accuracy",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"D3Q19 static droplet {n}^3 periodic, {args.storage} populations"
                               f"{' (in place)' if args.pattern == 'aa' else ''}, "
                               + (f"well-balanced scheme (gradient coefficient 0.15), {args.collision.upper()} + Guo "
                                  f"forcing, paper EOS (0.0375 / 1.187, xi = 3), radius {R:g}, tanh width 6"
                                  if wb else
                                  f"{args.collision.upper()} + Guo forcing, Peng-Robinson T/Tc=0.8, radius {R:g}, "
                                  f"tanh width 5")
                               + f"{f', uniform initial u_x = {args.u0:g}' if args.u0 else ''}; "
                               f"reduction every {REDUCE_EVERY} steps",
                   "lattice": "D3Q19", "nodes": nodes, "storage": args.storage, "collision": args.collision,
                   "pattern": args.pattern, "lattice_bytes": nbytes,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
