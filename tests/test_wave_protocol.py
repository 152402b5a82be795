"""Model check of the progress-counter protocol of the two-level exchange
passes (FD_VARIANT_WAVE), on the CPU.

The kernel's tiles run concurrently and order their accesses to the
neighbours' data only through per-tile progress counters (paper Sec. 5.5 gets
the same order from the sequential order of its skewed tiles).  This test
restates the protocol as a state machine -- one workgroup per tile, each
iteration split into its two halves (wait, poll and issue the loads D
iterations ahead; then barrier, publish, store) -- and runs it under
adversarial and random schedules, checking:

* read after write: a ring load of the neighbours' level 1 at plane c is
  issued only once their store of that plane is complete;
* write after read: a workgroup overwrites u^n at plane c with level 2 only
  once every neighbour's ring loads of u^n at plane c have completed;
* progress: some workgroup can always move, and every one finishes.

The constants (prefetch distance, the level lags with their counter
publication intervals, compiled radii) are read from the kernel sources;
every radius is checked with every pair.  Mutations of the protocol
(a count published before the first complete iteration, a count one too high,
a lag one plane short of 2D + 3, an interval too coarse for its lag) must each
be caught, so the checker has teeth.
"""
import os
import random
import re

import pytest

CSRC = os.path.join(os.path.dirname(__file__), os.pardir, "paper_1707_02347_amd", "csrc")


def constant(name):
    text = open(os.path.join(CSRC, "fd_wave.h")).read()
    return int(re.search(rf"constexpr int {name} = (\d+);", text).group(1))


def compiled_radii():
    text = open(os.path.join(CSRC, "fd_stream_configs.h")).read()
    body = text[text.index("FDW_WAVE_CONFIGS(W)"):]
    return sorted({int(m.group(1)) for m in re.finditer(r"W\((\d+),\s*\d+,\s*\d+\)", body)})


D = constant("kWaveAhead")
LAGS = (constant("kWaveLagShort"), constant("kWaveLagLong"), constant("kWaveLagLonger"))
PUBS = (constant("kWavePubShort"), constant("kWavePubLong"), constant("kWavePubLong"))  # interval of each lag
MASK = (1 << 32) - 1
EPOCH = 7


class Violation(AssertionError):
    pass


class Model:
    """One pass over an nty x ntz grid of tiles, nx planes along x."""

    def __init__(self, M, nx, nty=3, ntz=3, lag=LAGS[0], pub=PUBS[0], publish="kernel"):
        self.M, self.nx, self.pub = M, nx, pub
        self.E = max(lag - M, 0)
        self.publish_rule = publish
        self.ibeg, self.iend = M, nx + 2 * M + self.E
        self.tiles = [(y, z) for y in range(nty) for z in range(ntz)]
        self.nbrs = {}
        for (y, z) in self.tiles:
            self.nbrs[(y, z)] = [t for t in ((y - 1, z), (y + 1, z), (y, z - 1), (y, z + 1)) if t in self.tiles]
        # counters start at a lower epoch's maximum: only this pass's counts admit anything
        self.counter = {t: ((EPOCH - 1) << 32) | MASK for t in self.tiles}
        self.it = {t: self.ibeg for t in self.tiles}
        self.half = {t: 0 for t in self.tiles}         # 0: wait/poll/issue; 1: barrier/publish/store
        self.flag = {t: {n: 0 for n in self.nbrs[t]} for t in self.tiles}
        self.stores_done = {t: -1 << 30 for t in self.tiles}  # stores of iterations <= this are complete
        self.loads_done = {t: -1 << 30 for t in self.tiles}   # loads of iterations <= this have returned
        self.l1_stored_at = {t: {} for t in self.tiles}     # level-1 plane -> iteration that stored it
        self.waits = 0

    # -- the protocol's arithmetic, as the kernel states it
    def publish(self, i):
        """Counter a workgroup stores at the barrier of iteration i, or None."""
        if i % self.pub:
            return None
        if self.publish_rule == "kernel":
            return (EPOCH << 32) | (i - D) if i > D else None
        if self.publish_rule == "negative":        # no lower bound: i - D < 0 wraps in the low word
            return (EPOCH << 32) | ((i - D) & MASK)
        if self.publish_rule == "one_high":        # claims one iteration more than is complete
            return (EPOCH << 32) | (i - D + 1) if i >= D else None
        raise ValueError(self.publish_rule)

    def want(self, i1):
        """Count every neighbour must show before the ring loads of iteration i1."""
        c2 = i1 - 2 * self.M - self.E
        if c2 < 0 or c2 >= self.nx:
            return 0
        return (EPOCH << 32) | (c2 + self.M + 1)

    # -- one half-iteration of tile t; False if it has to wait
    def advance(self, t):
        i = self.it[t]
        if i >= self.iend:
            return False
        if self.half[t] == 0:
            w = self.want(i + D)
            if w and not all(f >= w for f in self.flag[t].values()):
                self.poll(t)
                if not all(f >= w for f in self.flag[t].values()):
                    self.waits += 1
                    return False
            if not all(f >= self.want(i + D + 1) for f in self.flag[t].values()):
                self.poll(t)
            self.issue_loads(t, i + D)
            self.half[t] = 1
            return True
        # barrier: this iteration's loads (issued D iterations ago) have
        # returned, hence (in-order completion) every store issued before them
        self.loads_done[t] = i
        self.stores_done[t] = i - D - 1
        v = self.publish(i)
        if v is not None:
            self.counter[t] = v
        c1, c2 = i - self.M, i - 2 * self.M - self.E
        if 0 <= c1 < self.nx:
            self.l1_stored_at[t][c1] = i
        if 0 <= c2 < self.nx:
            # level 2 overwrites u^n at c2: the neighbours' u^n ring loads of
            # c2 (issued for their iteration c2 + M) must have returned
            for n in self.nbrs[t]:
                if self.loads_done[n] < c2 + self.M:
                    raise Violation(f"tile {t} overwrites u^n plane {c2} before tile {n} read its ring")
        self.it[t] += 1
        self.half[t] = 0
        return True

    def poll(self, t):
        for n in self.nbrs[t]:
            self.flag[t][n] = self.counter[n]

    def issue_loads(self, t, i1):
        c2 = i1 - 2 * self.M - self.E
        if not 0 <= c2 < self.nx:
            return
        for n in self.nbrs[t]:
            j = self.l1_stored_at[n].get(c2)
            if j is None or j > self.stores_done[n]:
                raise Violation(f"tile {t} loads level 1 plane {c2} of tile {n} before its store completed")

    def done(self):
        return all(self.it[t] >= self.iend for t in self.tiles)

    def prologue(self):
        # the loads of the first D iterations are issued before the loop,
        # without a wait (none of them reads a ring of level 1)
        for t in self.tiles:
            self.poll(t)
            for d in range(D):
                assert self.want(self.ibeg + d) == 0
                self.issue_loads(t, self.ibeg + d)


def run(model, order):
    """Drive the model: `order` yields tiles to try; stalls are detected."""
    model.prologue()
    stuck = 0
    for t in order(model):
        if model.done():
            return model
        if model.advance(t):
            stuck = 0
        else:
            stuck += 1
            if stuck > 4 * len(model.tiles) and not any(model.advance(u) for u in model.tiles):
                live = {u: model.it[u] for u in model.tiles if model.it[u] < model.iend}
                raise Violation(f"no workgroup can move: {live}")
    raise AssertionError("schedule ended early")


def random_order(seed):
    def gen(model):
        rng = random.Random(seed)
        speed = {t: rng.choice([1, 1, 2, 5, 20]) for t in model.tiles}
        while True:
            ts = model.tiles
            yield rng.choices(ts, weights=[speed[t] for t in ts])[0]
    return gen


def starve_order(victim, head_start):
    """The victim runs `head_start` half-iterations alone, is then frozen
    while the others run as far as they can, then everyone runs in turn."""
    def gen(model):
        for _ in range(head_start):
            yield victim
        others = [t for t in model.tiles if t != victim]
        while True:
            moved = False
            for t in others:
                if model.advance(t):
                    moved = True
            if not moved:
                break
        while True:
            for t in model.tiles:
                yield t
    return gen


def lockstep_order(model):
    while True:
        for t in model.tiles:
            yield t


def schedules(victims):
    out = [lockstep_order]
    out += [random_order(s) for s in range(6)]
    out += [starve_order(v, h) for v in victims for h in range(2 * (max(LAGS) + D) + 4)]
    return out


@pytest.mark.parametrize("lag,pub", list(zip(LAGS, PUBS)))
@pytest.mark.parametrize("M", compiled_radii())
def test_protocol_is_safe_and_live_for_every_compiled_radius(M, lag, pub):
    assert lag >= 2 * D + pub + 1
    nx = 3 * (2 * M + lag)
    for order in schedules([(1, 1), (0, 0)]):
        m = run(Model(M, nx, lag=lag, pub=pub), order)
        assert m.done()


def test_laggard_never_waits():
    """The workgroup furthest behind is never the one that waits."""
    for M, (lag, pub) in ((M, lp) for M in compiled_radii() for lp in zip(LAGS, PUBS)):
        m = Model(M, 40, lag=lag, pub=pub)
        m.prologue()
        rng = random.Random(M)
        while not m.done():
            live = [t for t in m.tiles if m.it[t] < m.iend]
            low = min((m.it[t], m.half[t]) for t in live)
            laggards = [t for t in live if (m.it[t], m.half[t]) == low]
            t = rng.choice(live)
            moved = m.advance(t)
            if t in laggards:
                assert moved, (M, t, m.it)


def find_violation(make):
    for order in schedules([(1, 1), (0, 0), (0, 1)]):
        try:
            run(make(), order)
        except Violation as e:
            return str(e)
    return None


@pytest.mark.parametrize("M", [1, 2])
def test_mutation_negative_count_is_caught(M):
    # first iteration i = M < D: an unguarded count i - D wraps to a huge value
    assert M < D
    assert find_violation(lambda: Model(M, 30, publish="negative")) is not None
    assert find_violation(lambda: Model(M, 30)) is None


def test_mutation_count_one_high_is_caught():
    msg = find_violation(lambda: Model(4, 30, publish="one_high"))
    assert msg is not None and "before its store completed" in msg


def test_mutation_short_lag_is_caught():
    # a lag below 2D + 3 lets neighbours wait on each other
    msg = find_violation(lambda: Model(4, 30, lag=2 * D + 2))
    assert msg is not None


def test_mutation_interval_too_coarse_for_the_lag_is_caught():
    # the long interval with the short lag: M + E < 2D + P + 1
    assert LAGS[0] < 2 * D + PUBS[1] + 1
    msg = find_violation(lambda: Model(4, 40, lag=LAGS[0], pub=PUBS[1]))
    assert msg is not None and "no workgroup can move" in msg
