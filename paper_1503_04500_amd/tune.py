"""Autotuner of the batched build and the tuning table it writes.

The batched build has schedule choices that do not change its results: the
register tier the columns start in (tier0), how the first tier refills its waves
(refill), where spilled columns go (route), the size of the first tier's hash
tables (t0_hash, a tile choice) and the last register tier (last_tier, a class edge). ``autotune`` times every combination
on a matrix (rsai_autotune: median build time over repetitions, HIP events);
``main`` tunes a set of synthetic workloads and writes ``tuning.json``; ``choose``
looks a matrix up in it by mean column length, longest column and n (the same rule
the library applies when ``rsai.build`` hands it the table through rsai_params).
"""
from __future__ import annotations

import ctypes
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning.json")


class Choice(ctypes.Structure):
    _fields_ = [("tier0", ctypes.c_int32), ("refill", ctypes.c_int32), ("route", ctypes.c_int32),
                ("t0_hash", ctypes.c_int32), ("last_tier", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ms", ctypes.c_double)]

KEYS = ("tier0", "refill", "route", "t0_hash", "last_tier")


def autotune(A, reps: int = 3, **kw) -> dict:
    """Time every schedule choice for the batched build of A (a rsai.Matrix).
    Returns {"choices": [...], "best": {...}}."""
    from . import rsai
    lib = rsai.load()
    rsai._use_torch_allocator()
    prm = rsai.params(**kw)
    view = A.view()
    out = (Choice * 64)()
    cnt, best = ctypes.c_int32(), ctypes.c_int32()
    rsai._check(lib.rsai_autotune(ctypes.byref(view), ctypes.byref(prm), int(reps), rsai._stream(), out, 64,
                                  ctypes.byref(cnt), ctypes.byref(best)))
    ch = [dict(tier0=c.tier0, refill=c.refill, route=c.route, t0_hash=c.t0_hash, last_tier=c.last_tier, ms=c.ms)
          for c in out[:cnt.value]]
    return {"choices": ch, "best": ch[best.value]}


_table = None


def load_table(path: str = TABLE) -> list:
    """Entries of tuning.json (empty if absent); cached after the first call."""
    global _table
    if _table is None or path != TABLE:
        entries = []
        if os.path.exists(path):
            with open(path) as f:
                entries = json.load(f).get("entries", [])
        if path != TABLE:
            return entries
        _table = entries
    return _table


def choose(n: int, mean_len: float, max_len: int, table=None, eps: float = 0.4):
    """Schedule choices of the first table entry whose ranges hold (mean column
    length, longest column, n, eps); None if no entry matches."""
    for e in (load_table() if table is None else table):
        if (e["len_lo"] <= mean_len < e["len_hi"] and e["maxlen_lo"] <= max_len < e["maxlen_hi"]
                and e["n_lo"] <= n < e["n_hi"] and e.get("eps_lo", 0.0) <= eps < e.get("eps_hi", float("inf"))):
            return {k: e.get(k, -1) for k in KEYS}
    return None


def _workloads():
    """(name, matrix, parameters, the eps values tuned): the schedule that wins depends
    on eps as well as on the matrix (a smaller eps grows larger blocks)."""
    from . import gen
    return [("cd2d 512x512 (n=262144)", lambda: gen.cd2d(512, seed=0), dict(lmax=8), (0.4, 0.2)),
            ("cd3d 64^3 (n=262144)", lambda: gen.cd3d(64, seed=0), dict(lmax=8), (0.4,)),
            ("power-law n=10^6", lambda: gen.powerlaw(1_000_000, seed=0), dict(lmax=10), (0.4,)),
            ("cd2d 128x128", lambda: gen.cd2d(128, seed=1), dict(lmax=8), (0.4, 0.2)),
            ("power-law n=10^5", lambda: gen.powerlaw(100_000, seed=1), dict(lmax=10), (0.4,))]


def eps_ranges(eps_values):
    """Adjacent eps ranges around the tuned values, split at the midpoints."""
    ev = sorted(eps_values)
    cuts = [0.0] + [(a + b) / 2 for a, b in zip(ev, ev[1:])] + [float("inf")]
    return {e: (cuts[i], cuts[i + 1]) for i, e in enumerate(ev)}


def main(argv=None) -> int:
    """Tune the synthetic workloads on the current GPU and write tuning.json."""
    import torch
    from . import rsai
    out_path = TABLE if not argv else argv[0]
    results, entries = [], []
    for name, make, kw, epss in _workloads():
        H = make()
        A = rsai.Matrix.from_host(H, "cuda:0")
        mean_len = H.nnz / H.n
        maxlen = int((H.colptr[1:] - H.colptr[:-1]).max())
        rng = eps_ranges(epss)
        for eps in epss:
            r = autotune(A, reps=3, c=3, eps=eps, drop="fixed", tol=1e-3, validate=2, **kw)
            results.append(dict(workload=name, eps=eps, eps_lo=rng[eps][0], eps_hi=rng[eps][1], n=H.n,
                                mean_col_len=mean_len, max_col_len=maxlen, **r))
            print(name, "eps", eps, "best", r["best"], flush=True)
        del A
        torch.cuda.synchronize()
    # table: one entry per workload, keyed by mean column length, longest column and
    # n (ranges around the tuned point; the first match wins)
    for r in results:
        b = r["best"]
        entries.append(dict(len_lo=r["mean_col_len"] * 0.8, len_hi=r["mean_col_len"] * 1.25,
                            eps_lo=r["eps_lo"], eps_hi=r["eps_hi"] if r["eps_hi"] != float("inf") else 1e300,
                            maxlen_lo=max(1, r["max_col_len"] // 2), maxlen_hi=r["max_col_len"] * 2 + 1,
                            n_lo=r["n"] // 4, n_hi=r["n"] * 4, workload=r["workload"] + f" eps {r['eps']}",
                            **{k: b[k] for k in KEYS}))
    with open(out_path, "w") as f:
        json.dump({"device": torch.cuda.get_device_name(0), "entries": entries, "results": results}, f, indent=1)
    print("wrote", out_path)
    return 0


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1503_04500_amd import tune as _t
    sys.exit(_t.main(sys.argv[1:]))
