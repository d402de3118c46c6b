"""Use-after-free detection by live sets (paper Sec. 4.3 and Sec. 5.3).

A data structure is live at a point if it has been allocated and not freed
before that point.  The host pass walks the host code with the set of live
buffers: ``malloc`` adds a buffer, ``free`` removes it, and after an
``if``/``else`` the set is the intersection of the sets that the two branches
leave, so a buffer freed on either path counts as freed.  A launch whose
pointer argument is not in the set is reported.  The kernel pass does the
same over a kernel body: parameters and arrays are live at entry, a device
``free`` removes a parameter, branches meet by intersection, a loop head
takes the intersection of its entry set and the set its body leaves (until
that no longer changes), and an access to a data structure that is not in
the set is reported.

The analysis is path-insensitive, as in the paper: two branches on the same
condition are taken as independent, so it can report a use that no single
run performs (it never misses one that some run performs).

Reports: ``("uaf", "launch", launch index, kernel, argument position)`` and
``("uaf", "access", kernel, access index)``; launches and accesses are
numbered in program order, then-branches first.
"""
from __future__ import annotations

from workloads.program import Program


def _host(prog, stmts, live, ptrs, counter, out):
    for s in stmts:
        k = s[0]
        if k == "malloc":
            live.add(s[1])
        elif k == "free":
            live.discard(s[1])
        elif k == "launch":
            li = counter[0]
            counter[0] += 1
            for pos, a in enumerate(s[5]):
                if a[0] == "ref" and a[1] in ptrs and a[1] not in live:
                    out.add(("uaf", "launch", li, s[1], pos))
        elif k == "hif":
            then = _host(prog, s[2], set(live), ptrs, counter, out)
            other = _host(prog, s[3], set(live), ptrs, counter, out)
            live = then & other
    return live


def _kernel(kname, stmts, live, counter, out):
    """Walks a statement list; ``counter`` maps each access statement to its
    program-order index (assigned on first sight)."""
    for s in stmts:
        k = s[0]
        if k in ("static", "dynshared", "partition"):
            live.add(s[1])
        elif k == "free":
            live.discard(s[1])
        elif k == "access":
            ai = counter.setdefault(id(s), len(counter))
            if s[2] not in live:
                out.add(("uaf", "access", kname, ai))
        elif k == "if":
            live = _kernel(kname, s[2], set(live), counter, out) & \
                _kernel(kname, s[3], set(live), counter, out)
        elif k == "for":
            head = set(live)
            while True:
                leave = _kernel(kname, s[3], set(head), counter, out)
                nxt = head & leave
                if nxt == head:
                    break
                head = nxt
            live = head
    return live


def _number(stmts, counter):
    for s in stmts:
        if s[0] == "access":
            counter.setdefault(id(s), len(counter))
        elif s[0] == "if":
            _number(s[2], counter)
            _number(s[3], counter)
        elif s[0] == "for":
            _number(s[3], counter)
    return counter


def analyse(prog: Program) -> set:
    """The set of reported uses after free."""
    out = set()
    ptrs = {s[1] for s in prog.host if s[0] == "malloc"}
    _host(prog, prog.host, set(), ptrs, [0], out)
    for kname, (params, body) in prog.kernels.items():
        _kernel(kname, body, set(params), _number(body, {}), out)
    return out
