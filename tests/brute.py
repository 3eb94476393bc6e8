"""Brute-force expected results written straight from kernel formulas.

A test describes a kernel as a Python function of one thread's coordinates
that returns the thread's event list -- ("acc", access_id, slot, index,
elem_bytes, i1, i2), ("site", site_index), ("hang",) -- in program order.  This
module turns those events into records, site counts and status exactly as the
checking definition says: every access checked against its own allocation,
record and continue, first violation = smallest (gtid, i1, i2).  It does not
read the IR at all, so it pins the oracle's decoder and interpreter.
"""
from __future__ import annotations

import itertools

import numpy as np

KIND_OVER, KIND_UNDER, KIND_FREED, KIND_NULL = 1, 2, 4, 8
U64MAX = (1 << 64) - 1


def kind_of(entry, idx, elem):
    base, size, _, flags = entry[0], entry[1], entry[2], entry[3]
    if base == 0:
        return KIND_NULL
    if flags & 1:
        return KIND_FREED
    if idx < 0:
        return KIND_UNDER
    if idx >= size // elem:
        return KIND_OVER
    return 0


def shadow(table, spaces):
    """Byte-level shadow memory of one input's table under the tripwire
    model, as an address sanitizer keeps it: per memory space the set of
    poisoned byte addresses (the redzone bytes around every live allocation,
    every byte of a freed allocation and its redzones) and the end of the
    space's window (largest allocation end with its redzone)."""
    poisoned, window = {}, {}
    for k, e in enumerate(table):
        base, size, flags = int(e[0]), int(e[1]), int(e[3])
        rz = int(e[4]) if len(e) > 4 else 0
        if base == 0:
            continue
        sp = spaces[k] if k < len(spaces) else 0
        P = poisoned.setdefault(sp, set())
        if flags & 1:
            P.update(range(base - rz, base + size + rz))
        else:
            P.update(range(base - rz, base))
            P.update(range(base + size, base + size + rz))
        window[sp] = max(window.get(sp, 0), base + size + rz)
    return poisoned, window


def tripwire_reports(table, spaces, sh, slot, idx, elem):
    """Whether an access out of exact bounds is reported: NULL always;
    otherwise one of its bytes is poisoned in its space, or (shared and local
    spaces) it leaves the space's window."""
    e = table[slot]
    if int(e[0]) == 0:
        return True
    sp = spaces[slot] if slot < len(spaces) else 0
    a = int(e[0]) + idx * elem
    poisoned, window = sh
    if any(b in poisoned.get(sp, ()) for b in range(a, a + elem)):
        return True
    return sp != 0 and (a < 0 or a + elem > window.get(sp, 0))


def threads(launch, mode="full"):
    gx, gy, gz, bx, by, bz = (int(v) for v in launch)
    nb, bs = gx * gy * gz, bx * by * bz

    def coords(blin, tlin):
        return ((tlin % bx, (tlin // bx) % by, tlin // (bx * by)),
                (blin % gx, (blin // gx) % gy, blin // (gx * gy)), blin * bs + tlin)

    if nb == 0 or bs == 0:
        return []
    if mode == "full":
        return [coords(b, t) for b in range(nb) for t in range(bs)]
    if mode == "corners":
        out = []
        for c in itertools.product(*[sorted({0, g - 1}) for g in (gx, gy, gz, bx, by, bz)]):
            blin = c[0] + gx * (c[1] + gy * c[2])
            tlin = c[3] + bx * (c[4] + by * c[5])
            out.append(coords(blin, tlin))
        return sorted(out, key=lambda x: x[2])
    if mode == "boundary":
        centre = gx // 2 + gx * (gy // 2 + gy * (gz // 2))
        out = []
        for b in range(nb):
            x, y, z = b % gx, (b // gx) % gy, b // (gx * gy)
            face = ((gx > 1 and x in (0, gx - 1)) or (gy > 1 and y in (0, gy - 1))
                    or (gz > 1 and z in (0, gz - 1)))
            if face or b == centre:
                out.extend(coords(b, t) for t in range(bs))
        return out
    raise ValueError(mode)


def run(kernel, launches, tables, n_acc, n_sites, mode="full", L=(0, 0), scalars=None, tripwire=False,
        spaces=()):
    """kernel(tid, bid, launch, scalars) -> events.  Returns (records as list of
    dicts per input, counts [n][n_sites], status list of dicts).  With
    ``tripwire`` an exact violation is recorded only when the shadow model
    reports it (``spaces``: memory space per slot, default global)."""
    recs, counts, status = [], [], []
    for i, launch in enumerate(launches):
        sh = shadow(tables[i], spaces) if tripwire else None
        rec = [dict(first_key=U64MAX, index=0, count=0, kinds=0, first_kind=0) for _ in range(n_acc)]
        cnt = [0] * n_sites
        st = dict(lanes=0, accesses_checked=0, hang_lanes=0, arith_faults=0)
        sc = None if scalars is None else scalars[i]
        for tid, bid, gtid in threads(launch, mode):
            st["lanes"] += 1
            for ev in kernel(tid, bid, launch, sc):
                if ev[0] == "site":
                    cnt[ev[1]] += 1
                elif ev[0] == "hang":
                    st["hang_lanes"] += 1
                    break
                elif ev[0] == "fault":
                    st["arith_faults"] += 1
                else:
                    _, acc, slot, idx, elem, i1, i2 = ev
                    st["accesses_checked"] += 1
                    k = kind_of(tables[i][slot], idx, elem)
                    if k and tripwire and not tripwire_reports(tables[i], spaces, sh, slot, idx, elem):
                        k = 0
                    if k:
                        r = rec[acc]
                        key = (gtid << (L[0] + L[1])) | (i1 << L[1]) | i2
                        r["count"] += 1
                        r["kinds"] |= k
                        if key < r["first_key"]:
                            r["first_key"], r["index"], r["first_kind"] = key, idx, k
        recs.append(rec)
        counts.append(cnt)
        status.append(st)
    return recs, counts, status


def assert_matches(out, expect, n_inputs=None):
    """Compare an oracle/GPU result dict with brute-force output."""
    recs, counts, status = expect
    n = len(recs) if n_inputs is None else n_inputs
    for i in range(n):
        for a, r in enumerate(recs[i]):
            got = out["records"][i, a]
            for f in ("first_key", "index", "count", "kinds", "first_kind"):
                assert int(got[f]) == r[f], (i, a, f, int(got[f]), r[f])
        assert [int(c) for c in out["counts"][i]] == counts[i], (i, list(out["counts"][i]), counts[i])
        for f in ("lanes", "accesses_checked", "hang_lanes", "arith_faults"):
            assert int(out["status"][i][f]) == status[i][f], (i, f)


def to_np_records(recs):
    from oracle.oracle import RECORD_DTYPE
    out = np.zeros((len(recs), len(recs[0]) if recs else 0), RECORD_DTYPE)
    for i, rr in enumerate(recs):
        for a, r in enumerate(rr):
            out[i, a] = (r["first_key"], r["index"], r["count"], r["kinds"], r["first_kind"])
    return out
