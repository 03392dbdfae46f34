"""Continuous batching (plbm_batch_*) on the GPU.

Each lattice advanced inside a batch, whatever else shares the launches and
whenever it joins or leaves, must be bitwise identical to the same lattice
stepped alone (the kernels compute every node with the same arithmetic; the
batch only changes which workgroup handles which tile).  The per-slot
diagnostics must equal plbm_reduce of a solo lattice.  Covered at small,
ragged sizes with joins and leaves, and at the serving workload's extremes
(192^3 and 1024^2 beside 64^3 and 64^2).
"""
import numpy as np
import pytest

from gpu_cases import fmt, lib_params, random_state, require_gpu

pytestmark = pytest.mark.gpu

SPECS = [
    # lattice, dims, collision, storage, walls, seed
    ("D3Q19", (40, 24, 18), "mrt", "f32", False, 1),
    ("D3Q19", (33, 17, 12), "bgk", "f32", True, 2),
    ("D2Q9", (150, 40), "bgk", "f32", False, 3),
    ("D2Q9", (64, 64), "mrt", "f64", False, 4),
    ("D3Q19", (36, 20, 10), "mrt", "f32", False, 5),
    ("D3Q19", (36, 18, 12), "mrt", "f16r", True, 6),
    ("D2Q9", (96, 40), "bgk", "bf16s", False, 7),
]


def _make(spec, stream=None):
    from paper_2504_15018_amd.lattice import Lattice
    lattice, dims, coll, st, walls, seed = spec
    lat = Lattice(lattice, dims, lib_params(tau_v=0.9, tau_l=1.1), collision=coll, storage=st, walls=walls,
                  stream=stream)
    lat.write_populations(random_state(lattice, dims, seed))
    return lat


class Batch:
    def __init__(self, max_slots, max_tiles, stream):
        import torch
        from paper_2504_15018_amd import native as N
        self.N = N
        self.max_slots = max_slots
        nb = N.plbm_batch_bytes(max_slots, max_tiles)
        self.mem = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        ptr = (self.mem.data_ptr() + 255) // 256 * 256
        self.stream = stream
        self.h = N.plbm_batch_create(max_slots, max_tiles, ptr, nb, stream.cuda_stream)

    def attach(self, lat):
        return self.N.plbm_batch_attach(self.h, lat.h)

    def detach(self, slot):
        self.N.plbm_batch_detach(self.h, slot)

    def step(self, n):
        self.N.plbm_batch_step(self.h, n)

    def diag(self):
        return self.N.plbm_batch_diag(self.h, self.max_slots)

    def close(self):
        self.stream.synchronize()
        self.N.plbm_batch_destroy(self.h)


def test_batch_matches_solo_bitwise_with_joins_and_leaves():
    require_gpu()
    import torch
    fmt("batch_vs_solo")
    stream = torch.cuda.Stream()
    solo = [_make(s) for s in SPECS]
    mixed = [_make(s, stream=stream) for s in SPECS]
    b = Batch(8, 4096, stream)
    slots = {}
    # lattices 0..2, 5, 6 start together; 3 joins after 7 steps; 1 leaves after 12; 4 joins at 12
    for k in (0, 1, 2, 5, 6):
        slots[k] = b.attach(mixed[k])
    b.step(7)
    slots[3] = b.attach(mixed[3])
    b.step(5)
    b.detach(slots.pop(1))
    slots[4] = b.attach(mixed[4])
    b.step(9)  # odd count: graph pairs plus a single launch
    b.step(1)
    stream.synchronize()
    steps = {0: 22, 1: 12, 2: 22, 3: 15, 4: 10, 5: 22, 6: 22}
    for k, lat in enumerate(solo):
        lat.step(steps[k])
    for k in range(len(SPECS)):
        assert mixed[k].time == steps[k]
        assert np.array_equal(mixed[k].populations(), solo[k].populations()), SPECS[k]
    # a detached lattice keeps stepping on its own and stays identical
    mixed[1].step(3)
    solo[1].step(3)
    assert np.array_equal(mixed[1].populations(), solo[1].populations())
    # per-slot diagnostics equal the solo reductions
    d = b.diag()
    for k, s in slots.items():
        ref = solo[k].reduce()
        assert d[s].mass == ref.mass and d[s].max_u == ref.max_u and d[s].time == ref.time
        assert list(d[s].momentum) == list(ref.momentum)
    b.close()
    for lat in solo + mixed:
        lat.close()


def test_batch_detects_an_unstable_member_without_disturbing_others():
    """NaN injected into one lattice is flagged for that slot only; the others stay bitwise exact."""
    require_gpu()
    import torch
    from paper_2504_15018_amd import native as N
    fmt("batch_fault_isolation")
    stream = torch.cuda.Stream()
    specs = SPECS[:3]
    mixed = [_make(s, stream=stream) for s in specs]
    solo = [_make(s) for s in specs]
    f = mixed[1].populations()
    f[3, ...] = np.nan
    mixed[1].write_populations(f)
    b = Batch(4, 4096, stream)
    slots = [b.attach(m) for m in mixed]
    b.step(6)
    d = b.diag()
    assert d[slots[1]].flags & N.PLBM_FLAG_NAN
    for k in (0, 2):
        assert d[slots[k]].flags == 0
        solo[k].step(6)
        assert np.array_equal(mixed[k].populations(), solo[k].populations())
    b.close()
    for lat in solo + mixed:
        lat.close()


def test_batch_owns_its_lattices_until_detached():
    """An attached lattice refuses stepping and re-initialisation through its own
    handle and a second batch; destroying it detaches it; destroying the batch
    releases the rest."""
    require_gpu()
    import torch
    from paper_2504_15018_amd import native as N
    fmt("batch_ownership")
    stream = torch.cuda.Stream()
    specs = SPECS[:3]
    mixed = [_make(s, stream=stream) for s in specs]
    solo = [_make(s) for s in specs]
    b = Batch(4, 4096, stream)
    other = Batch(2, 4096, stream)
    slots = [b.attach(m) for m in mixed]
    f0 = mixed[0].populations()  # reads stay allowed
    for call in (lambda: mixed[0].step(1), lambda: mixed[0].write_populations(f0),
                 lambda: mixed[0].init_fields(np.ones(mixed[0].N)), lambda: other.attach(mixed[0])):
        with pytest.raises(N.PlbmError) as e:
            call()
        assert e.value.code == N.PLBM_E_INVALID
    b.step(4)
    # destroying an attached lattice frees its slot; the rest keep stepping
    mixed[1].close()
    b.step(3)
    d = b.diag()
    assert d[slots[1]].time == 0 and d[slots[1]].mass == 0.0
    assert b.attach(solo[1]) == slots[1]  # the freed slot is reused
    b.detach(slots[1])
    # destroying the batch releases the lattices still attached
    b.close()
    other.close()
    mixed[0].step(2)
    for k in (0, 2):
        steps = 9 if k == 0 else 7
        solo[k].step(steps)
        assert mixed[k].time == steps
        assert np.array_equal(mixed[k].populations(), solo[k].populations()), specs[k]
    for lat in solo + [mixed[0], mixed[2]]:
        lat.close()


def test_batch_of_the_serving_extremes_matches_solo_bitwise():
    """The serving workload's largest and smallest lattices in one batch (D3Q19 192^3 and 64^3, D2Q9 1024^2 and
    64^2; f32, MRT, static droplets as the serving loop initialises them), 21 steps: every lattice bitwise equal
    to the same lattice stepped alone, and the per-slot diagnostics equal to its solo reduction."""
    require_gpu()
    import torch
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    fmt("batch_serving_extremes")
    specs = [("D3Q19", (192, 192, 192)), ("D2Q9", (1024, 1024)), ("D3Q19", (64, 64, 64)), ("D2Q9", (64, 64))]
    prm = lib_params(tr=0.75)

    def make(lattice, dims, stream=None):
        lat = Lattice(lattice, dims, prm, collision="mrt", storage="f32", stream=stream)
        lat.init_shape(N.PLBM_SHAPE_DROPLET, prm.rho_l, prm.rho_v, W=5.0, R=0.3 * dims[0],
                       centre=[n / 2.0 for n in dims])
        return lat

    stream = torch.cuda.Stream()
    solo = [make(*s) for s in specs]
    mixed = [make(*s, stream=stream) for s in specs]
    b = Batch(4, 65536, stream)
    slots = [b.attach(lat) for lat in mixed]
    b.step(21)
    stream.synchronize()
    d = b.diag()
    for lat in solo:
        lat.step(21)
    for k, spec in enumerate(specs):
        assert np.array_equal(mixed[k].populations(), solo[k].populations()), spec
        ref = solo[k].reduce()
        assert d[slots[k]].mass == ref.mass and d[slots[k]].max_u == ref.max_u, spec
        assert d[slots[k]].flags == 0 and d[slots[k]].time == 21
    b.close()
    for lat in solo + mixed:
        lat.close()
