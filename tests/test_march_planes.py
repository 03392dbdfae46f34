"""Host replay of the z marches of the fused A-B update kernel (k_step) and of
the in-place update (k_aa_step, whose psi ring is loaded a plane ahead).

The kernel's tile waves and halo waves walk a chunk [z0, z1) of z planes
with one barrier per collided plane, loading each plane's populations ahead
of use (one phase ahead, or a full plane iteration ahead) and writing its psi
into a 4-plane LDS ring; the halo waves keep NH planes of loads in flight in
NH rotating register sets, and the well-balanced scheme's chemical-potential
pass runs its tile waves the same way (NM sets; its phase B reads only the
ring).  This test replays the same loop structures, in the same order, for
every prefetch depth the kernel can be built with, periodic and walled axes,
every axis length 1..9 and every chunk length, and checks:

* every stored plane the loads touch (the plane and its two neighbours) lies
  in [0, nz): the march loads up to as many planes past the last one the
  collision needs as it keeps in flight, unconditionally, and a periodic axis
  shorter than that window (nz = 1, 2, 3) must still wrap inside the array;
* a plane's psi is summed from the register set that was loaded with that
  plane, and a collided plane uses the set holding its own populations;
* tile waves and halo waves meet the same number of barriers;
* between two barriers no LDS ring slot is both written and read, and every
  slot read by the collision of plane z holds plane z - 1, z or z + 1,
  written (by tile and halo waves) before the preceding barrier.
"""
import pytest


def wrapz(zl, nz, walls):
    if walls:
        return 0 if zl < 0 else (nz - 1 if zl >= nz else zl)
    while zl < 0:
        zl += nz
    while zl >= nz:
        zl -= nz
    return zl


class Trace:
    def __init__(self, nz, walls, z0, z1):
        self.nz, self.walls, self.z0, self.z1 = nz, walls, z0, z1
        self.sets = {}          # register set -> plane loaded into it
        self.interval = 0       # barriers passed
        self.writes = []        # (interval, slot, plane, who)
        self.reads = []         # (interval, slot, plane)
        self.loaded = []

    def issue(self, zl, regset):
        pz = wrapz(zl, self.nz, self.walls)
        # neighbour planes as the kernel forms them
        zm = (0 if self.walls else self.nz - 1) if pz == 0 else pz - 1
        zp = (self.nz - 1 if self.walls else 0) if pz == self.nz - 1 else pz + 1
        for p in (pz, zm, zp):
            assert 0 <= p < self.nz, (zl, p, self.nz)
        self.loaded.append(zl)
        self.sets[regset] = zl

    def finish(self, zl, regset, who):
        assert self.sets.get(regset) == zl, f"psi of plane {zl} summed from set holding {self.sets.get(regset)}"
        slot = (zl - self.z0 + 1) & 3
        self.writes.append((self.interval, slot, zl, who))

    def barrier(self):
        self.interval += 1

    def collide(self, z, regset):
        assert self.sets.get(regset) == z, f"plane {z} collided from set holding {self.sets.get(regset)}"
        self.stencil(z)

    def stencil(self, z):
        # the stencil reads the ring values of planes z - 1, z, z + 1 from their slots
        for zz in (z - 1, z, z + 1):
            self.reads.append((self.interval, (zz - self.z0 + 1) & 3, zz))


def tile_march(tr, prefetch):
    z0, z1 = tr.z0, tr.z1
    if prefetch == 1:
        tr.issue(z0 - 1, "f0"); tr.finish(z0 - 1, "f0", "t")
        tr.issue(z0, "f0"); tr.finish(z0, "f0", "t")
        tr.issue(z0 + 1, "f1"); tr.finish(z0 + 1, "f1", "t")

        def stepz(z, cur, pf):
            tr.issue(z + 2, pf)
            tr.barrier()
            tr.collide(z, cur)
            tr.finish(z + 2, pf, "t")

        z = z0
        while z + 2 < z1:
            stepz(z, "f0", "f2"); stepz(z + 1, "f1", "f0"); stepz(z + 2, "f2", "f1")
            z += 3
        if z < z1:
            stepz(z, "f0", "f2")
            z += 1
        if z < z1:
            stepz(z, "f1", "f0")
    else:
        tr.issue(z0 - 1, "fa"); tr.finish(z0 - 1, "fa", "t")
        tr.issue(z0, "fa"); tr.finish(z0, "fa", "t")
        tr.issue(z0 + 1, "fb"); tr.finish(z0 + 1, "fb", "t")
        tr.issue(z0 + 2, "fc")

        def stepz(z, cur, f2, pf):
            tr.issue(z + 3, pf)
            tr.barrier()
            tr.collide(z, cur)
            tr.finish(z + 2, f2, "t")

        z = z0
        while z + 3 < z1:
            stepz(z, "fa", "fc", "fd"); stepz(z + 1, "fb", "fd", "fa")
            stepz(z + 2, "fc", "fa", "fb"); stepz(z + 3, "fd", "fb", "fc")
            z += 4
        if z < z1:
            stepz(z, "fa", "fc", "fd")
            z += 1
        if z < z1:
            stepz(z, "fb", "fd", "fa")
            z += 1
        if z < z1:
            stepz(z, "fc", "fa", "fb")


def rotating_march(tr, n, who, step_reads):
    """n register sets, plane z0+2+j in set j mod n: iteration z issues plane z+1+n, passes the plane barrier,
    (tile waves of the chemical-potential pass: evaluates the stencil of plane z,) and writes plane z+2."""
    z0, z1 = tr.z0, tr.z1
    for zl in range(z0 - 1, z0 + 2):
        tr.issue(zl, f"{who}0"); tr.finish(zl, f"{who}0", who)
    for j in range(n - 1):
        tr.issue(z0 + 2 + j, f"{who}{j}")

    def step(z, u):
        tr.issue(z + 1 + n, f"{who}{(u + n - 1) % n}")
        tr.barrier()
        if step_reads:
            tr.stencil(z)
        tr.finish(z + 2, f"{who}{u}", who)

    z = z0
    while z + n - 1 < z1:
        for u in range(n):
            step(z + u, u)
        z += n
    for u in range(n - 1):
        if z + u < z1:
            step(z + u, u)


def halo_march(tr, depth):
    rotating_march(tr, depth, "h", False)


def mu_march(tr, depth):
    rotating_march(tr, depth, "t", True)


def chunks(nz, cz):
    return [(z0, min(z0 + cz, nz)) for z0 in range(0, nz, cz)]


# (tile waves: update march of prefetch 1 or 2, or the chemical-potential pass with n sets; halo waves: n sets)
MARCHES = [("update", p, h) for p in (1, 2) for h in (1, 2, 3)] + [("mu", n, n) for n in (1, 2, 3, 4)]


@pytest.mark.parametrize("kind,tile_depth,halo_depth", MARCHES)
@pytest.mark.parametrize("walls", [False, True])
def test_march_stays_in_bounds_and_race_free(kind, tile_depth, halo_depth, walls):
    for nz in range(1, 10):
        for cz in range(1, nz + 1):
            for z0, z1 in chunks(nz, cz):
                tt = Trace(nz, walls, z0, z1)
                if kind == "update":
                    tile_march(tt, tile_depth)
                else:
                    mu_march(tt, tile_depth)
                th = Trace(nz, walls, z0, z1)
                halo_march(th, halo_depth)
                assert tt.interval == th.interval == z1 - z0
                # every collided plane, in order
                assert sorted({r[2] for r in tt.reads}) == list(range(z0 - 1, z1 + 1))
                # at most as many planes past the last one the collision reads as are kept in flight
                assert max(tt.loaded) <= z1 + tile_depth and max(th.loaded) <= z1 + halo_depth
                writes = tt.writes + th.writes
                for k, slot, zz in tt.reads:
                    # no write to a slot in the interval it is read
                    assert not any(w[0] == k and w[1] == slot for w in writes), (nz, cz, z0, k, slot)
                    # the latest earlier write of that slot, by each wave kind, is plane zz
                    for who in ("t", "h"):
                        prior = [w for w in writes if w[3] == who and w[1] == slot and w[0] < k]
                        assert prior and prior[-1][2] == zz, (nz, cz, z0, k, slot, zz, who, prior[-1:])


def test_short_periodic_axis_wraps_inside_the_array():
    # the window z0 - 1 .. z1 + 4 of a chunk, with neighbours, on axes of length 1 to 3
    for nz in (1, 2, 3):
        for zl in range(-1, nz + 6):
            p = wrapz(zl, nz, False)
            assert 0 <= p < nz and (p - zl) % nz == 0


def inplace_march(tr):
    """The in-place update's z march: psi of ring plane zl is loaded into a register set (issue) a plane
    iteration before it is written to its LDS slot (commit); iteration z commits plane z+1, issues the psi of
    plane z+2, loads the populations of plane z+1, passes the plane barrier and updates plane z."""
    z0, z1 = tr.z0, tr.z1
    tr.issue(z0 - 1, "pa"); tr.finish(z0 - 1, "pa", "t")
    tr.issue(z0, "pa"); tr.finish(z0, "pa", "t")
    tr.issue(z0 + 1, "pa")
    tr.issue(z0, "va")  # populations of plane z0

    def plane_step(z, cur, nxt, pc, pn):
        tr.finish(z + 1, pc, "t")
        tr.issue(z + 2, pn)
        if z + 1 < z1:
            tr.issue(z + 1, nxt)
        tr.barrier()
        tr.collide(z, cur)

    z = z0
    while z + 1 < z1:
        plane_step(z, "va", "vb", "pa", "pb")
        plane_step(z + 1, "vb", "va", "pb", "pa")
        z += 2
    if z < z1:
        plane_step(z, "va", "vb", "pa", "pb")


@pytest.mark.parametrize("walls", [False, True])
def test_inplace_march_stays_in_bounds_and_race_free(walls):
    for nz in range(1, 10):
        for cz in range(1, nz + 1):
            for z0, z1 in chunks(nz, cz):
                tr = Trace(nz, walls, z0, z1)
                inplace_march(tr)
                assert tr.interval == z1 - z0
                assert sorted({r[2] for r in tr.reads}) == list(range(z0 - 1, z1 + 1))
                assert max(tr.loaded) <= z1 + 1  # the psi of one plane past the last one the update reads
                for k, slot, zz in tr.reads:
                    assert not any(w[0] == k and w[1] == slot for w in tr.writes), (nz, cz, z0, k, slot)
                    prior = [w for w in tr.writes if w[1] == slot and w[0] < k]
                    assert prior and prior[-1][2] == zz, (nz, cz, z0, k, slot, zz, prior[-1:])
