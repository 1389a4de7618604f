"""Checks an exported command-queue structure against the DAG it runs (test infrastructure).

Sec. III defines the command-queue structure Q = <Q, E_q> (Def. 4): in-order queues of write
(H2D), ndrange (kernel) and read (D2H) commands, plus precedence pairs <q_s[i], q_t[j]> across
queues; rules (i)-(iii) say which precedences must exist (write before the kernel that reads it,
kernel before the read of its output, producer kernel before consumer kernel over an edge), and
Def. 5 calls a schedule valid when kernels are dispatched in a topological order.

An exported schedule is ``{"n_streams": S, "ops": [op, ...]}`` with each op a dict
``{"id", "type" ("h2d"|"kernel"|"d2h"), "kernel" (index or -1), "buffer" (name or None),
"stream", "pos", "host_order", "waits": [op ids]}``: ``pos`` is the op's place in its in-order
stream, ``waits`` its cross-stream precedences, ``host_order`` the order in which the host
enqueues it.  The happens-before relation (HB) is the transitive closure of stream order and
waits.  A schedule may also say ``"in_order": False``: its queues run out of order (OpenCL's
out-of-order execution mode, a relaxation of Def. 4's in-order queues), a command may start
before earlier commands of its queue complete, and HB is the transitive closure of the waits
alone.

``check_schedule`` is the polynomial checker: the schedule is valid iff
  1. its structure is well formed (positions, host order, waits refer to ops enqueued earlier,
     which HIP requires because a wait sees only an event record already enqueued);
  2. every kernel appears once, every isolated input has one H2D covering it, every isolated
     output has one D2H;
  3. every pair of ops touching overlapping storage, at least one of them writing, is ordered by
     HB in the direction of the data flow (writer first), which covers rules (i)-(iii).
``brute_force`` enumerates every interleaving consistent with HB of a tiny schedule, executes it
on symbolic values, and reports the reads that can observe a value other than the one the
sequential execution gives.  Both return the set of reader ops that can read a wrong value.
"""
from __future__ import annotations

import itertools


def _buffers(spec):
    return {b["name"]: b for b in spec["buffers"]}


def _region(spec, name):
    by = _buffers(spec)
    b = by[name]
    rows, cols = b["rows"], b["cols"]
    r0 = c0 = 0
    while b["view_of"] is not None:
        r0 += b["row_off"]
        c0 += b["col_off"]
        b = by[b["view_of"]]
    return (b["name"], r0, c0, rows, cols)


def _overlap(a, b):
    return (a[0] == b[0] and a[1] < b[1] + b[3] and b[1] < a[1] + a[3]
            and a[2] < b[2] + b[4] and b[2] < a[2] + a[4])


def _covers(outer, inner):
    return (outer[0] == inner[0] and outer[1] <= inner[1] and outer[2] <= inner[2]
            and inner[1] + inner[3] <= outer[1] + outer[3]
            and inner[2] + inner[4] <= outer[2] + outer[4])


def isolated_io(spec):
    """Isolated writes (kernel, input buffer) and isolated reads (kernel, output buffer), Sec. III."""
    fed = {(t, tb) for (_, _, t, tb) in spec["edges"]}
    src = {(s, sb) for (s, sb, _, _) in spec["edges"]}
    writes, reads = [], []
    for ki, k in enumerate(spec["kernels"]):
        for b in k["inputs"]:
            if (ki, b) not in fed:
                writes.append((ki, b))
        for b in k["outputs"]:
            if (ki, b) not in src:
                reads.append((ki, b))
    return writes, reads


def accesses(spec, op):
    """List of (region, is_write) that an op touches."""
    t = op["type"]
    if t == "h2d":
        return [(_region(spec, op["buffer"]), True)]
    if t == "d2h":
        return [(_region(spec, op["buffer"]), False)]
    k = spec["kernels"][op["kernel"]]
    return ([(_region(spec, b), False) for b in k["inputs"]]
            + [(_region(spec, b), True) for b in k["outputs"]])


def hb_closure(sched):
    """ancestors[i] = bitmask of ops that happen before op i (requires a well-formed schedule)."""
    ops = sched["ops"]
    by_stream = {}
    for o in ops:
        by_stream.setdefault(o["stream"], []).append(o)
    prev = {}
    for s, lst in by_stream.items():
        lst.sort(key=lambda o: o["pos"])
        if sched.get("in_order", True):   # out-of-order queues: position orders nothing
            for a, b in zip(lst, lst[1:]):
                prev[b["id"]] = a["id"]
    anc = [0] * len(ops)
    for o in sorted(ops, key=lambda o: o["host_order"]):
        m = 0
        preds = list(o["waits"])
        if o["id"] in prev:
            preds.append(prev[o["id"]])
        for p in preds:
            m |= anc[p] | (1 << p)
        anc[o["id"]] = m
    return anc


def _structure(sched, n_kernels):
    errs = []
    ops = sched["ops"]
    n = len(ops)
    if sorted(o["id"] for o in ops) != list(range(n)):
        return ["op ids are not 0..n-1"]
    if sorted(o["host_order"] for o in ops) != list(range(n)):
        errs.append("host_order is not a permutation of 0..n-1")
    byid = {o["id"]: o for o in ops}
    streams = {}
    for o in ops:
        if not 0 <= o["stream"] < sched["n_streams"]:
            errs.append(f"op {o['id']}: stream {o['stream']} out of range")
        streams.setdefault(o["stream"], []).append(o)
    for s, lst in streams.items():
        if sorted(o["pos"] for o in lst) != list(range(len(lst))):
            errs.append(f"stream {s}: positions are not 0..len-1")
        lst = sorted(lst, key=lambda o: o["pos"])
        if any(a["host_order"] > b["host_order"] for a, b in zip(lst, lst[1:])):
            errs.append(f"stream {s}: stream order disagrees with host order")
    for o in ops:
        for w in o["waits"]:
            if w not in byid:
                errs.append(f"op {o['id']}: waits on unknown op {w}")
            elif byid[w]["host_order"] >= o["host_order"]:
                errs.append(f"op {o['id']}: waits on op {w} that is enqueued later")
        if o["type"] == "kernel" and not 0 <= o["kernel"] < n_kernels:
            errs.append(f"op {o['id']}: unknown kernel {o['kernel']}")
    return errs


def check_schedule(spec, sched):
    """Polynomial validity check.  Returns (ok, errors, bad_readers)."""
    errs = _structure(sched, len(spec["kernels"]))
    if errs:
        return False, errs, set()
    ops = sched["ops"]
    # completeness
    kcount = {}
    for o in ops:
        if o["type"] == "kernel":
            kcount[o["kernel"]] = kcount.get(o["kernel"], 0) + 1
    for ki in range(len(spec["kernels"])):
        if kcount.get(ki, 0) != 1:
            errs.append(f"kernel {ki} appears {kcount.get(ki, 0)} times")
    writes, reads = isolated_io(spec)
    h2d = [o for o in ops if o["type"] == "h2d"]
    d2h = [o for o in ops if o["type"] == "d2h"]
    produced = [(_region(spec, b)) for k in spec["kernels"] for b in k["outputs"]]
    for o in h2d:
        r = _region(spec, o["buffer"])
        if any(_overlap(r, p) for p in produced):
            errs.append(f"H2D of {o['buffer']} overwrites storage a kernel produces")
    for (ki, b) in writes:
        r = _region(spec, b)
        n_cover = sum(1 for o in h2d if _covers(_region(spec, o["buffer"]), r))
        if n_cover != 1:
            errs.append(f"isolated input {b} of kernel {ki} is covered by {n_cover} H2D ops")
    for (ki, b) in reads:
        n_rd = sum(1 for o in d2h if o["buffer"] == b)
        if n_rd != 1:
            errs.append(f"isolated output {b} of kernel {ki} has {n_rd} D2H ops")
    # ordering of every conflicting pair, writer first
    anc = hb_closure(sched)
    acc = [accesses(spec, o) for o in ops]
    bad_readers = set()
    for i, j in itertools.permutations(range(len(ops)), 2):
        for (ri, wi) in acc[i]:
            if not wi:
                continue
            for (rj, wj) in acc[j]:
                if not _overlap(ri, rj):
                    continue
                if wj and i > j:
                    continue  # each write-write pair once
                if not wj:
                    if not (anc[j] >> i) & 1:
                        errs.append(f"op {j} reads {rj[0]} without op {i}, which writes it, "
                                    f"happening before")
                        bad_readers.add(j)
                else:
                    if not ((anc[j] >> i) & 1 or (anc[i] >> j) & 1):
                        errs.append(f"ops {i} and {j} write {ri[0]} unordered")
    return (not errs), errs, bad_readers


def _cells(spec, ops):
    """Split every root into the grid cells that all op regions cut it into."""
    regs = [r for o in ops for (r, _) in accesses(spec, o)]
    cuts = {}
    for (root, r0, c0, rows, cols) in regs:
        rc, cc = cuts.setdefault(root, (set(), set()))
        rc.update((r0, r0 + rows))
        cc.update((c0, c0 + cols))
    grid = {root: (sorted(rc), sorted(cc)) for root, (rc, cc) in cuts.items()}

    def cells_of(reg):
        root, r0, c0, rows, cols = reg
        rc, cc = grid[root]
        out = []
        for a, b in zip(rc, rc[1:]):
            if r0 <= a and b <= r0 + rows:
                for c, d in zip(cc, cc[1:]):
                    if c0 <= c and d <= c0 + cols:
                        out.append((root, a, c))
        return out

    return cells_of


def _run_symbolic(spec, ops, order, cells_of):
    """Execute ops in ``order`` on symbolic values; returns {op id: tuple of values read}.

    The value of a storage cell is the identity of the op that last wrote it, so a read is
    correct exactly when it sees the writer the sequential execution makes it see.
    """
    val = {}
    seen = {}
    for oid in order:
        o = ops[oid]
        acc = accesses(spec, o)
        got = tuple(tuple(val.get(c, ("uninit", c)) for c in cells_of(r)) for (r, w) in acc if not w)
        seen[oid] = got
        tag = ("written-by", oid)
        for (r, w) in acc:
            if w:
                for c in cells_of(r):
                    val[c] = (tag, c)
    return seen


def brute_force(spec, sched, limit=200000):
    """Set of reader op ids that can observe a wrong value in some HB-consistent interleaving.

    The expected values are those of a sequential run in host order with every dependency
    respected, i.e. kernels in a topological order with writes before reads; the reference
    interleaving used is the kernels' Kahn order with H2D ops first and D2H ops last.
    """
    ops = sorted(sched["ops"], key=lambda o: o["id"])
    n = len(ops)
    cells_of = _cells(spec, ops)
    # reference sequential execution
    from .dag import topological_order
    korder = topological_order(spec)
    ref_order = ([o["id"] for o in ops if o["type"] == "h2d"]
                 + [next(o["id"] for o in ops if o["type"] == "kernel" and o["kernel"] == k)
                    for k in korder]
                 + [o["id"] for o in ops if o["type"] == "d2h"])
    expected = _run_symbolic(spec, ops, ref_order, cells_of)
    anc = hb_closure(sched)
    bad = set()
    count = 0

    def rec(done_mask, order):
        nonlocal count
        if count >= limit:
            return
        if len(order) == n:
            count += 1
            got = _run_symbolic(spec, ops, order, cells_of)
            for oid in range(n):
                if got[oid] != expected[oid]:
                    bad.add(oid)
            return
        for i in range(n):
            if not (done_mask >> i) & 1 and (anc[i] & ~done_mask) == 0:
                order.append(i)
                rec(done_mask | (1 << i), order)
                order.pop()

    rec(0, [])
    return bad
