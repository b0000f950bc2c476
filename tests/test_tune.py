"""Host logic of the tuning table (no GPU)."""
import os

from paper_1503_04500_amd import tune
from paper_1503_04500_amd import rsai

TABLE = [
    dict(len_lo=4.0, len_hi=6.25, maxlen_lo=2, maxlen_hi=11, n_lo=1000, n_hi=10**6, tier0=0, refill=1, route=0),
    dict(len_lo=5.6, len_hi=8.75, maxlen_lo=100, maxlen_hi=401, n_lo=10**5, n_hi=10**7, tier0=1, refill=1, route=1),
    dict(len_lo=5.6, len_hi=8.75, maxlen_lo=3, maxlen_hi=15, n_lo=10**4, n_hi=10**7, tier0=0, refill=0, route=1),
]


def test_choose_matches_ranges_in_order():
    assert tune.choose(262144, 5.0, 5, TABLE) == dict(tier0=0, refill=1, route=0)
    # same mean length, told apart by the longest column
    assert tune.choose(10**6, 7.0, 200, TABLE) == dict(tier0=1, refill=1, route=1)
    assert tune.choose(262144, 6.9, 7, TABLE) == dict(tier0=0, refill=0, route=1)
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
