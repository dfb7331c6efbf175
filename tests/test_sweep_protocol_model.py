"""A host-side model of the strip sweep's hand-off protocol (the dense-kernel sweep path), run
under random wavefront schedules on the CPU.

It reproduces what the gfx950 strip sweep does between wavefronts, not its arithmetic:

* persistent workgroups of NW wavefronts claim (wave-stream, band) tickets from one counter, in
  band-major order, with a workgroup barrier after each claim and at the end of each band;
* within a band, wave k sweeps strip band * NW + k chunk by chunk; a strip's top edge goes to the
  wave above through an LDS ring of RB slots (`produced` / `consumed` counters, the producer
  waits for the slot to be consumed RB chunks later), and the band's top edge goes to the next
  band through a global edge buffer behind an epoch-tagged progress counter;
* before its rows, a wave prefetches the next chunk's per-ordinate sources (addresses
  angular offset + cell * npad, checked against the pool here) and takes the chunk's bottom
  edge; several sweeps (epochs) reuse the same progress counters without clearing them.

Two chunk orders are modelled: the committed one (prefetch of chunk c + 1, then the bottom edge
of chunk c) and the reordered variant that hung once on the GPU (bottom edge first, then the
prefetch), each with the lane's angular offset read per ticket and read once per workgroup.
Every schedule must finish (no deadlock), never overwrite a ring slot before it is read, never
read an edge before it is written in the same sweep, and keep every address in range.
"""
import random
from dataclasses import dataclass, field

import pytest

WAIT = "wait"


@dataclass
class Shape:
    nx: int
    ny: int
    tx: int
    ty: int
    band: int
    n: int            # ordinates (a multiple of 4: mirrored quadrants)
    lanes: int        # lanes per ordinate group (16, 32, 64)
    wgs: int          # persistent workgroups
    rb: int = 1       # LDS ring slots per strip boundary (the library's kRingSlots)


@dataclass
class Plan:
    shape: Shape
    ws: list = field(default_factory=list)        # [(quadrant, [internal ordinate per lane])]
    tickets: list = field(default_factory=list)
    npad: int = 0
    nstrips: int = 0
    nchunks: int = 0
    nbands: int = 0


def build_plan(sh: Shape) -> Plan:
    """Wave-streams, lane ordinates and band-major tickets, as the host plan builds them for one
    system (ordinates grouped by quadrant, each quadrant padded to whole lane groups, G = 64 / L
    groups per wavefront)."""
    p = Plan(sh)
    m = sh.n // 4
    L = sh.lanes
    groups = []  # (quadrant, first internal ordinate)
    first = 0
    for q in range(4):
        for b in range(0, m, L):
            groups.append((q, first))
            first += L
    p.npad = (first + 127) // 128 * 128
    G = 64 // L
    for q in range(4):
        gq = [g for g in groups if g[0] == q]
        for g0 in range(0, len(gq), G):
            lanes = []
            for k in range(G):
                if g0 + k < len(gq):
                    lanes += [gq[g0 + k][1] + l for l in range(L)]
                else:
                    lanes += [gq[0][1]] * L  # empty groups alias ordinate 0 and never store
            p.ws.append((q, lanes))
    p.nstrips = (sh.ny + sh.ty - 1) // sh.ty
    p.nchunks = (sh.nx + sh.tx - 1) // sh.tx
    p.nbands = (p.nstrips + sh.band - 1) // sh.band
    p.tickets = [(w, b) for b in range(p.nbands) for w in range(len(p.ws))]
    return p


class Model:
    """One sweep per epoch: every wavefront is a generator of actions; WAIT means it is blocked on
    a counter; the scheduler runs the unblocked ones in a random order."""

    def __init__(self, plan: Plan, variant: bool, hoist_offset: bool, rng: random.Random, epochs: int = 3,
                 skip=()):
        self.p, self.variant, self.hoist, self.rng, self.epochs = plan, variant, hoist_offset, rng, epochs
        self.skip = set(skip)   # waits left out, to show that the checks catch a broken protocol
        self.prog = {}          # (ws, band) -> epoch << 24 | chunks published (never cleared)
        self.edge = {}          # (ws, band, chunk) -> epoch that wrote it
        self.errors = []
        self.pool = plan.shape.nx * plan.shape.ny * plan.npad

    def check_addresses(self, wsi, lanes_ord, c, strip):
        sh = self.p.shape
        for e in range(sh.tx * sh.ty):
            r, i = divmod(e, sh.tx)
            jj, ii = min(strip * sh.ty + r, sh.ny - 1), min(c * sh.tx + i, sh.nx - 1)
            cell = jj * sh.nx + ii
            for o in lanes_ord:
                a = cell * self.p.npad + o
                if not (0 <= a < self.pool):
                    self.errors.append(("address", wsi, c, strip, a))
                    return

    def barrier(self, wg):
        gen = wg["gen"]
        wg["arrived"] += 1
        if wg["arrived"] == self.p.shape.band:
            wg["arrived"] = 0
            wg["gen"] += 1
        while wg["gen"] == gen:
            yield WAIT

    def wave(self, wg, k, epoch, counter):
        p, sh = self.p, self.p.shape
        tag = epoch << 24
        hoisted = None
        while True:
            if k == 0:
                wg["ticket"] = counter[0]
                counter[0] += 1
            wg["produced"][k] = 0
            wg["consumed"][k] = 0
            yield from self.barrier(wg)
            t = wg["ticket"]
            if t >= len(p.tickets):
                return
            wsi, band = p.tickets[t]
            quad, lanes = p.ws[wsi]
            if hoisted is None:
                hoisted = lanes
            ords = hoisted if self.hoist else lanes
            strip = band * sh.band + k
            if strip < p.nstrips:
                from_global = k == 0 and strip > 0
                to_global = strip + 1 < p.nstrips and k == sh.band - 1
                has_out = strip + 1 < p.nstrips
                self.check_addresses(wsi, ords, 0, strip)
                for c in range(p.nchunks):
                    def take_edge():
                        if strip == 0:
                            return
                        if from_global:
                            while "edge" not in self.skip and self.prog.get((wsi, band - 1), 0) < (tag | (c + 1)):
                                yield WAIT
                            if self.edge.get((wsi, band - 1, c)) != epoch:
                                self.errors.append(("edge read before written", wsi, band, c, epoch))
                        else:
                            while wg["produced"][k - 1] < c + 1:
                                yield WAIT
                            slot = wg["ring"].get((k - 1, c % sh.rb))
                            if slot != (t, c, False):
                                self.errors.append(("ring slot", wsi, band, k, c, slot))
                            wg["ring"][(k - 1, c % sh.rb)] = (t, c, True)
                            wg["consumed"][k - 1] = c + 1

                    if self.variant:  # bottom edge first, then the next chunk's loads
                        yield from take_edge()
                        if c + 1 < p.nchunks:
                            self.check_addresses(wsi, ords, c + 1, strip)
                    else:
                        if c + 1 < p.nchunks:
                            self.check_addresses(wsi, ords, c + 1, strip)
                        yield from take_edge()
                    yield "rows"
                    if to_global:
                        self.edge[(wsi, band, c)] = epoch
                        self.prog[(wsi, band)] = tag | (c + 1)
                    elif has_out:
                        if c >= sh.rb:
                            while "ring" not in self.skip and wg["consumed"][k] < c + 1 - sh.rb:
                                yield WAIT
                        prev = wg["ring"].get((k, c % sh.rb))
                        if prev is not None and prev[0] == t and not prev[2]:
                            self.errors.append(("ring overwrite", wsi, band, k, c, prev))
                        wg["ring"][(k, c % sh.rb)] = (t, c, False)
                        wg["produced"][k] = c + 1
            yield from self.barrier(wg)

    def run_epoch(self, epoch):
        sh = self.p.shape
        counter = [0]
        waves = []
        for w in range(sh.wgs):
            wg = {"ticket": None, "arrived": 0, "gen": 0, "produced": [0] * sh.band, "consumed": [0] * sh.band,
                  "ring": {}}
            for k in range(sh.band):
                waves.append(self.wave(wg, k, epoch, counter))
        live = list(waves)
        idle = 0
        while live:
            self.rng.shuffle(live)
            still, progressed = [], False
            for g in live:
                try:
                    act = next(g)
                except StopIteration:
                    progressed = True
                    continue
                if act != WAIT:
                    progressed = True
                still.append(g)
            live = still
            idle = 0 if progressed else idle + 1
            if idle > 3:  # every live wave blocked, several rounds in a row: no progress possible
                self.errors.append(("deadlock", epoch, len(live)))
                return False
        return True

    def run(self):
        for e in range(1, self.epochs + 1):
            if not self.run_epoch(e):
                break
        return self.errors


SHAPES = [
    # the dense-kernel parity case (40 x 40, 128 ordinates: 32 per quadrant, 32-lane groups)
    Shape(40, 40, 8, 4, 4, 128, 32, 2), Shape(40, 40, 8, 8, 2, 128, 32, 1), Shape(40, 40, 16, 8, 8, 128, 32, 3),
    Shape(40, 40, 16, 16, 2, 128, 32, 2),
    # c4-like: 1024 ordinates in 64-lane groups, one workgroup and several
    Shape(64, 48, 8, 4, 4, 1024, 64, 1), Shape(64, 48, 8, 4, 4, 1024, 64, 5),
    # ragged strips and chunks, single-wave bands, more bands than workgroups
    Shape(37, 29, 8, 4, 1, 40, 16, 2), Shape(37, 29, 8, 4, 3, 40, 16, 1), Shape(23, 70, 16, 8, 2, 24, 16, 3),
    # two ring slots per boundary (the protocol allows any count)
    Shape(40, 40, 8, 4, 4, 128, 32, 2, rb=2), Shape(37, 29, 8, 4, 3, 40, 16, 1, rb=2),
]


@pytest.mark.parametrize("variant", [False, True], ids=["committed", "reordered"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s.nx}x{s.ny}_t{s.tx}x{s.ty}_b{s.band}_n{s.n}_L{s.lanes}_w{s.wgs}_rb{s.rb}")
def test_protocol_is_live_and_safe(shape, variant):
    plan = build_plan(shape)
    for seed in range(6):
        errs = Model(plan, variant, hoist_offset=False, rng=random.Random(seed)).run()
        assert not errs, errs[:3]


@pytest.mark.parametrize("shape", SHAPES[:6], ids=lambda s: f"{s.nx}x{s.ny}_t{s.tx}x{s.ty}_b{s.band}_n{s.n}_L{s.lanes}_w{s.wgs}_rb{s.rb}")
def test_offset_read_once_stays_in_range_but_is_wrong(shape):
    """Reading the lane's angular offset once per workgroup keeps every address inside the
    pool (the offsets of one system's wave-streams are all below npad): the variant cannot
    fault; a workgroup that takes tickets of several wave-streams then uses the first one's
    ordinates for the others, a wrong result, not a hang."""
    plan = build_plan(shape)
    errs = Model(plan, True, hoist_offset=True, rng=random.Random(1)).run()
    assert not errs, errs[:3]
    assert len({tuple(l) for _, l in plan.ws}) == len(plan.ws)  # distinct per wave-stream


@pytest.mark.parametrize("break_it", ["ring", "edge", "ticket_order"])
def test_model_detects_a_broken_protocol(break_it):
    """The checker is not vacuous: a producer that overwrites ring slots without back-pressure,
    a consumer that reads the band edge without waiting for its progress counter, and tickets
    claimed top band first (a consumer ahead of its producer with one workgroup) are caught."""
    # one workgroup runs bands one after another (a skipped edge wait then never shows); the
    # edge case needs bands in flight together
    plan = build_plan(Shape(16, 64, 8, 4, 2, 8, 16, 3 if break_it == "edge" else 1, rb=1))
    skip = (break_it,) if break_it in ("ring", "edge") else ()
    if break_it == "ticket_order":
        plan.tickets = sorted(plan.tickets, key=lambda t: (-t[1], t[0]))
    found = any(Model(plan, False, False, random.Random(seed), skip=skip).run() for seed in range(20))
    assert found
