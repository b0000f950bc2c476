"""Host logic of the tuning table (no GPU)."""
import os

from paper_1503_04500_amd import tune
from paper_1503_04500_amd import rsai

TABLE = [
    dict(len_lo=4.0, len_hi=6.25, maxlen_lo=2, maxlen_hi=11, n_lo=1000, n_hi=10**6, tier0=0, refill=1, route=0),
    dict(len_lo=5.6, len_hi=8.75, maxlen_lo=100, maxlen_hi=401, n_lo=10**5, n_hi=10**7, tier0=1, refill=1, route=1),
    dict(len_lo=5.6, len_hi=8.75, maxlen_lo=3, maxlen_hi=15, n_lo=10**4, n_hi=10**7, tier0=0, refill=0, route=1),
]


def _sub(d):
    return {k: d[k] for k in ("tier0", "refill", "route")}


def test_choose_matches_ranges_in_order():
    assert _sub(tune.choose(262144, 5.0, 5, TABLE)) == dict(tier0=0, refill=1, route=0)
    # same mean length, told apart by the longest column
    assert _sub(tune.choose(10**6, 7.0, 200, TABLE)) == dict(tier0=1, refill=1, route=1)
    assert _sub(tune.choose(262144, 6.9, 7, TABLE)) == dict(tier0=0, refill=0, route=1)
    # fields an entry lacks come back as -1 (not applied)
    assert tune.choose(262144, 5.0, 5, TABLE)["t0_hash"] == -1
    # eps ranges: adjacent, split at the midpoints of the tuned values
    assert tune.eps_ranges((0.4, 0.2)) == {0.2: (0.0, 0.30000000000000004), 0.4: (0.30000000000000004, float("inf"))}
    t2 = [dict(TABLE[0], eps_lo=0.3, eps_hi=1.0, tier0=0), dict(TABLE[0], eps_lo=0.0, eps_hi=0.3, tier0=1)]
    assert tune.choose(262144, 5.0, 5, t2, eps=0.4)["tier0"] == 0
    assert tune.choose(262144, 5.0, 5, t2, eps=0.2)["tier0"] == 1
    # outside every range
    assert tune.choose(10, 5.0, 5, TABLE) is None
    assert tune.choose(262144, 20.0, 5, TABLE) is None


def test_committed_table_is_well_formed():
    entries = tune.load_table()
    if not os.path.exists(tune.TABLE):
        return
    assert entries
    for e in entries:
        assert e["len_lo"] < e["len_hi"] and e["maxlen_lo"] < e["maxlen_hi"] and e["n_lo"] < e["n_hi"]
        assert 0 <= e["tier0"] < 3 and e["refill"] in (0, 1) and e["route"] in (0, 1)
        assert e.get("t0_hash", -1) in (-1, 2, 4) and e.get("last_tier", -1) in (-1, 1, 2)


def test_tune_entries_layout_and_params_checks():
    """The binding's rsai_tune_entry matches the C layout (2 doubles, 4 int64, 6 int32)
    and the library rejects bad schedule fields on the host."""
    import ctypes
    assert ctypes.sizeof(rsai.TuneEntry) == 88
    if not os.path.exists(rsai.LIB_PATH):
        return
    arr, n = rsai.tune_entries(TABLE)
    assert n == 3 and arr[1].maxlen_lo == 100 and arr[1].tier0 == 1 and arr[0].t0_hash == -1
    lib = rsai.load()
    out = ctypes.c_void_p()
    v = rsai.CSCView(4, 4, 8, 8, 8)
    for field, val in (("t0_hash", 3), ("last_tier", 0), ("last_tier", 5), ("deterministic", 2), ("tune_count", -1)):
        q = rsai.params()
        setattr(q, field, val)
        assert lib.rsai_build(ctypes.byref(v), ctypes.byref(q), None, ctypes.byref(out)) == -1, field
    q = rsai.params(tier0=2)
    q.last_tier = 1
    assert lib.rsai_build(ctypes.byref(v), ctypes.byref(q), None, ctypes.byref(out)) == -1
    q = rsai.params()
    q.tune_count = 2   # a count without a table
    assert lib.rsai_build(ctypes.byref(v), ctypes.byref(q), None, ctypes.byref(out)) == -1


def test_params_route_field():
    if not os.path.exists(rsai.LIB_PATH):
        return
    p = rsai.params(route=0, refill=1, tier0=2)
    assert (p.route, p.refill, p.tier0) == (0, 1, 2)
    assert rsai.params().route == -1


def test_bench_traffic_requires_matching_kernel_sources(tmp_path, monkeypatch):
    """bench.py reports the counter-derived HBM traffic only while the tier kernel's
    sources hash to the value recorded beside the counters (a profile written for the
    current sources is read; a change to a source invalidates it)."""
    import hashlib
    import shutil
    import bench
    root = tmp_path
    (root / "profiles").mkdir()
    (root / "paper_1503_04500_amd" / "csrc").mkdir(parents=True)
    src = os.path.join(bench.ROOT, "paper_1503_04500_amd", "csrc")
    h = hashlib.sha256()
    for f in ("rsai_tier.hip", "rsai_tier_kernel.h", "rsai_tier.h", "rsai_dev.h"):
        shutil.copy(os.path.join(src, f), root / "paper_1503_04500_amd" / "csrc" / f)
        with open(os.path.join(src, f), "rb") as fh:
            h.update(fh.read())
    with open(root / "profiles" / "tier_kernel_cd2d512_pmc.md", "w") as f:
        f.write("# counters\n\n    kernel: tier_kernel\n    kernel_source_sha256: %s\n"
                "    traffic_bytes_per_launch: 12345\n" % h.hexdigest())
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic() == 12345.0
    with open(root / "paper_1503_04500_amd" / "csrc" / "rsai_tier.hip", "a") as f:
        f.write("\n// changed\n")
    assert bench.measured_traffic() is None
