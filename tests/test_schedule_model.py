"""Host-ordering check of the multi-stream sweep schedule that was tried and
withdrawn (launches per (parity, layer class) on four streams, each waiting
only on the launches that last updated a neighbouring layer).

The schedule is replayed here as its host code issued it: groups in key
order (4 * parity + class; class 0 = layers with one held neighbour, 1 = their
neighbours, 2 = the bulk), the bulk on the caller's stream, the edge classes
of each parity on a stream of their own and both neighbour classes on a third;
before a launch, a wait on the last recorded event of every neighbouring group
that was already issued on another stream; with observables recorded, the
caller's stream waits on every group and the other streams wait on it.

The launch graph (stream order + event waits) is then checked: any two
launches that touch the same layer, one of them writing it (a group writes
its own layers and reads the layers next to them), must be ordered in the
graph, in host issue order.  This passes for the shapes of the stress runs
that showed corruption (Lz = 4 and 6) and for the 32-layer workload, so the
event graph of that schedule was not the hazard.  The same check on a
deliberately broken rule (waits dropped for the neighbour classes) fails,
which shows the check can see a missing edge.
"""
import itertools

import pytest


def layer_class(Lz, z):
    if z == 0 or z == Lz - 1:
        return 0
    if z == 1 or z == Lz - 2:
        return 1
    return 2


def replay(Lz, n_sweeps, record, drop_class=None):
    """Returns (launches, edges): launches[i] = (sweep, parity, class, layers);
    edges: set of (i, j) meaning launch i is ordered before launch j."""
    groups = {}
    for p in (0, 1):
        for z in range(p, Lz, 2):
            groups.setdefault(4 * p + layer_class(Lz, z), []).append(z)
    keys = sorted(groups)
    owner = {z: k for k in keys for z in groups[k]}
    deps = {k: sorted({owner[z + dz] for z in groups[k] for dz in (-1, 1) if 0 <= z + dz < Lz}) for k in keys}

    def stream_of(k):
        cls, par = k % 4, k // 4
        return "s" if cls == 2 else ("aux%d" % par if cls == 0 else "aux2")

    launches, edges = [], set()
    last_on_stream = {}          # stream -> index of the last operation issued on it
    event_of = {}                # group -> launch index of its last recorded event
    entry = None                 # index of the entry marker on the caller's stream (observables)

    def issue(stream, waits, what):
        i = len(launches)
        launches.append(what)
        if stream in last_on_stream:
            edges.add((last_on_stream[stream], i))
        for w in waits:
            edges.add((w, i))
        last_on_stream[stream] = i
        return i

    for sw in range(n_sweeps):
        for k in keys:
            st = stream_of(k)
            waits = []
            for h in deps[k]:
                if h in event_of and stream_of(h) != st:
                    if drop_class is not None and k % 4 == drop_class:
                        continue
                    waits.append(event_of[h])
            if entry is not None and st != "s":
                waits.append(entry)
            event_of[k] = issue(st, waits, (sw, k // 4, k % 4, tuple(groups[k])))
        if record:
            waits = [event_of[k] for k in keys if stream_of(k) != "s"]
            entry = issue("s", waits, (sw, "observables", None, tuple(range(Lz))))
    return launches, edges


def reach(n, edges):
    succ = [[] for _ in range(n)]
    for a, b in edges:
        succ[a].append(b)
    out = []
    for a in range(n):
        seen, stack = set(), [a]
        while stack:
            u = stack.pop()
            for v in succ[u]:
                if v not in seen:
                    seen.add(v)
                    stack.append(v)
        out.append(seen)
    return out


def conflicts(a, b, Lz):
    """Whether launches a and b touch a common layer with at least one writing it."""
    def touched(l):
        if l[1] == "observables":
            return set(), set(range(Lz))
        writes = set(l[3])
        reads = {z + dz for z in l[3] for dz in (-1, 1) if 0 <= z + dz < Lz}
        return writes, reads
    wa, ra = touched(a)
    wb, rb = touched(b)
    return bool(wa & (wb | rb)) or bool(wb & ra)


def unordered_pairs(Lz, n_sweeps, record, drop_class=None):
    launches, edges = replay(Lz, n_sweeps, record, drop_class)
    r = reach(len(launches), edges)
    bad = []
    for i, j in itertools.combinations(range(len(launches)), 2):
        if conflicts(launches[i], launches[j], Lz) and j not in r[i]:
            bad.append((launches[i], launches[j]))
    return bad


@pytest.mark.parametrize("Lz", [4, 6, 7, 32])
@pytest.mark.parametrize("record", [False, True])
def test_withdrawn_schedule_orders_every_conflict(Lz, record):
    assert unordered_pairs(Lz, 3, record) == []


def test_check_sees_a_missing_wait():
    assert unordered_pairs(6, 2, False, drop_class=1)
