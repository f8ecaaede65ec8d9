"""Host-side pieces of bench.py that need no GPU: the oracle baselines."""

import bench
from trs_workloads import generators as G


def test_all_cores_baseline_covers_the_batch():
    # a thread per core over independent terms: every term of a small batch
    # is normalised once, so the rule applications equal the one-core leg's
    w = G.cfg3(n_terms=40, pool_slots=1 << 20, scale="mini")
    one = bench.cpu_baseline(w, budget_s=60.0)
    many = bench.cpu_baseline_all_cores(w, budget_s=60.0, max_threads=4)
    assert one["sample"].startswith("40 of 40 terms")
    assert many["sample"].startswith("40 of 40 terms")
    apps_one = int(one["sample"].split(", ")[1].split()[0])
    apps_many = int(many["sample"].split(", ")[1].split()[0])
    assert apps_one == apps_many > 0
    assert 1 <= many["cores"] <= 4 and many["kind"] == "oracle"
