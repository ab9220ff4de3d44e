"""Host-side checks of the benchmark's bookkeeping: the interval union behind the stage kernel's launch time,
and that the committed rocprofv3 records are found for the setting they were taken on (and only for it), so
that the roofline fraction can be recomputed from the files under profiles/."""
import argparse
import json
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_interval_union():
    assert bench.interval_union([]) == 0
    assert bench.interval_union([(0, 10)]) == 10
    # disjoint, nested, overlapping and touching intervals, in any order
    assert bench.interval_union([(20, 30), (0, 10)]) == 20
    assert bench.interval_union([(0, 10), (2, 5)]) == 10
    assert bench.interval_union([(0, 10), (5, 15), (14, 20)]) == 20
    assert bench.interval_union([(0, 10), (10, 12)]) == 12
    assert bench.interval_union([(5.0, 6.5), (0.0, 1.0), (0.5, 2.0)]) == pytest.approx(3.5)


def test_timed_stage_waves():
    ns = argparse.Namespace
    assert bench.timed_stage_waves(ns(stage_waves=-1, streams=2)) == 6
    assert bench.timed_stage_waves(ns(stage_waves=-1, streams=1)) == 0
    assert bench.timed_stage_waves(ns(stage_waves=5, streams=2)) == 5


def _opts(rec, **over):
    import paper_2507_17094_amd as miann
    st = dict(rec["setting"], **over)
    return miann.SearchOptions(entry=st["entry"], dgs=True, search_width=st["search_width"],
                               ghost_every_stage=st["ghost_every_stage"], t_seeds=st["t_seeds"],
                               discard=st.get("discard", 0.5), cooldown=st.get("cooldown", 0.3),
                               stage_waves=st.get("stage_waves", 0))


def test_committed_records_match_their_setting_only():
    timing = json.load(open(os.path.join(ROOT, "profiles", "stage_kernel_sharded1m_timing.json")))
    traffic = json.load(open(os.path.join(ROOT, "profiles", "stage_kernel_sharded1m_traffic.json")))
    assert timing and traffic
    for rec in timing:
        st = rec["setting"]
        o = _opts(rec)
        got = bench.profiled_launch_us(rec["workload"], st["itopk"], st["T"], o, rec["streams"])
        if got == (None, None):
            continue  # taken on sources that have changed since
        assert got == (rec["stage_kernel_union_us_per_launch"], rec["stage_kernel_avg_us"])
        assert rec["stage_kernel_union_us_per_launch"] <= rec["stage_kernel_avg_us"] + 1e-9
        # another stream count, stage build or filter setting does not pick this record up
        other = bench.profiled_launch_us(rec["workload"], st["itopk"], st["T"], o, 3)
        assert other == (None, None)
        o2 = _opts(rec, cooldown=0.25)
        assert bench.profiled_launch_us(rec["workload"], st["itopk"], st["T"], o2, rec["streams"]) == (None, None)
    found = 0
    for rec in traffic:
        st = rec["setting"]
        o = _opts(rec)
        got = bench.measured_traffic(rec["workload"], st["itopk"], st["T"], o)
        if got is None:
            continue
        found += 1
        assert got == pytest.approx(rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"])
        assert bench.measured_traffic(rec["workload"], st["itopk"], st["T"] + 1000, o) is None
    assert found >= 1, "no traffic record matches the current stage kernel sources"
