"""Tiny schedule builders used by the validator tests (independent of the HIP library)."""
from oracle import dag
from oracle.validator import isolated_io


def _root(spec, name):
    return dag.resolve(spec, name)[0]


def naive_schedule(spec, assign, n_streams, order=None):
    """Ops for kernels in ``order`` with each kernel's isolated writes just before it and its
    isolated reads just after it on its stream; a wait on every cross-stream producer."""
    order = order or dag.topological_order(spec)
    writes, reads = isolated_io(spec)
    ops, pos = [], [0] * n_streams
    kop, h2d_of = {}, {}

    def emit(typ, kernel, buf, stream, waits):
        o = {"id": len(ops), "type": typ, "kernel": kernel, "buffer": buf, "stream": stream,
             "pos": pos[stream], "host_order": len(ops), "waits": sorted(set(waits))}
        pos[stream] += 1
        ops.append(o)
        return o["id"]

    for k in order:
        s = assign[k]
        for (ki, b) in writes:
            if ki == k and _root(spec, b) not in h2d_of:
                h2d_of[_root(spec, b)] = emit("h2d", -1, _root(spec, b), s, [])
        waits = [kop[src] for (src, _, dst, _) in spec["edges"] if dst == k]
        waits += [h2d_of[_root(spec, b)] for (ki, b) in writes if ki == k]
        waits = [w for w in waits if ops[w]["stream"] != s]
        kop[k] = emit("kernel", k, None, s, waits)
        for (ki, b) in reads:
            if ki == k:
                emit("d2h", -1, b, s, [])
    return {"n_streams": n_streams, "ops": ops}


def from_queues(spec, queues, eq):
    """Schedule from named queue lists ("kernel:k0", "h2d:b2", ...) and precedence pairs; the
    host enqueues round-robin across queues, which keeps every precedence pair in order here."""
    kid = {k["name"]: i for i, k in enumerate(spec["kernels"])}
    ops, name_to_id = [], {}
    for s, q in enumerate(queues):
        for p, item in enumerate(q):
            typ, name = item.split(":")
            o = {"id": len(ops), "type": typ, "kernel": kid[name] if typ == "kernel" else -1,
                 "buffer": None if typ == "kernel" else name, "stream": s, "pos": p,
                 "host_order": None, "waits": []}
            name_to_id[item] = o["id"]
            ops.append(o)
    for a, b in eq:
        ops[name_to_id[b]]["waits"].append(name_to_id[a])
    # host order: repeatedly take the first op of any queue whose waits are already enqueued
    heads = [0] * len(queues)
    placed, ho = set(), 0
    qids = [[name_to_id[i] for i in q] for q in queues]
    while ho < len(ops):
        progressed = False
        for s in range(len(queues)):
            if heads[s] < len(qids[s]):
                o = ops[qids[s][heads[s]]]
                if all(w in placed for w in o["waits"]):
                    o["host_order"] = ho
                    ho += 1
                    placed.add(o["id"])
                    heads[s] += 1
                    progressed = True
        if not progressed:
            raise ValueError("precedence pairs form a cycle with the queue order")
    return {"n_streams": len(queues), "ops": ops}, name_to_id
