"""Autotuner logic on the CPU: tuning validation through the C ABI, choice of
the fastest candidate, and the cache round trip (no device work)."""
import pytest


@pytest.fixture(scope="module")
def pc():
    from paper_1807_00399_amd import pcgpu
    yield pcgpu
    pcgpu.set_tuning(128, 16, 1.0)


def test_tuning_validation(pc):
    pc.set_tuning(64, 32, 0.5, 0)
    assert pc.get_tuning() == {"icp_block_threads": 64, "icp_leaf": 32, "node_budget": 0.5, "sort_queries": 0,
                               "icp_persistent": 0}
    # the persistent loop is switched off: only 0 is accepted
    for bad in ((96, 16, 1.0), (128, 12, 1.0), (128, 16, 1.5), (128, 16, 0.0), (128, 16, 1.0, 2),
                (128, 16, 1.0, 1, 1), (128, 16, 1.0, 1, 2)):
        with pytest.raises(pc.PcgpuError):
            pc.set_tuning(*bad)
    assert pc.get_tuning()["icp_block_threads"] == 64      # unchanged by rejected calls
    pc.set_tuning(128, 16, 1.0)


def test_tune_picks_fastest_and_caches(pc, tmp_path):
    from paper_1807_00399_amd import autotune
    # a fake step whose cost depends on the current tuning
    cost = {(b, l, nb): 1.0 + abs(b - 256) / 64 + abs(l - 8) / 8 + (1.0 - nb) for b, l, nb in autotune.CANDIDATES}
    clock = {"t": 0.0}

    def step():
        t = pc.get_tuning()
        # Morton-ordered queries save a little here
        clock["t"] += cost[(t["icp_block_threads"], t["icp_leaf"], t["node_budget"])] - 0.25 * t["sort_queries"]

    cache = str(tmp_path / "tune.json")
    r = autotune.tune(step, "fake", 1 << 20, device_name="dev0", cache_file=cache, sync=lambda: None,
                      clock=lambda: clock["t"])
    assert not r["from_cache"]
    assert r["tuning"] == {"icp_block_threads": 256, "icp_leaf": 8, "node_budget": 1.0, "sort_queries": 1,
                           "icp_persistent": 0}
    assert pc.get_tuning() == r["tuning"]
    assert len(r["timings"]) == len(autotune.CANDIDATES) + 1
    pc.set_tuning(128, 16, 1.0)
    # same device, tag and size bucket: served from the cache and applied
    r2 = autotune.tune(step, "fake", (1 << 20) + 5, device_name="dev0", cache_file=cache, sync=lambda: None,
                       clock=lambda: clock["t"])
    assert r2["from_cache"] and r2["tuning"] == r["tuning"] and pc.get_tuning() == r["tuning"]
    # another size bucket is tuned again
    r3 = autotune.tune(step, "fake", 1 << 10, device_name="dev0", cache_file=cache, sync=lambda: None,
                       clock=lambda: clock["t"])
    assert not r3["from_cache"]
    assert set(autotune.load_cache(cache)) == {"dev0|fake|20", "dev0|fake|10"}


def test_cache_entries_without_query_order_mean_input_order(pc, tmp_path):
    import json
    from paper_1807_00399_amd import autotune
    cache = str(tmp_path / "old.json")
    key = autotune.cache_key("dev0", "old", 1000)
    json.dump({key: {"tuning": {"icp_block_threads": 64, "icp_leaf": 16, "node_budget": 1.0}}}, open(cache, "w"))
    r = autotune.tune(lambda: None, "old", 1000, device_name="dev0", cache_file=cache)
    assert r["from_cache"] and pc.get_tuning()["sort_queries"] == 0 and pc.get_tuning()["icp_persistent"] == 0
    # an entry that chose the persistent loop (now switched off) is applied
    # without it
    key2 = autotune.cache_key("dev0", "pers", 1000)
    json.dump({key2: {"tuning": {"icp_block_threads": 128, "icp_leaf": 8, "node_budget": 0.5, "sort_queries": 1,
                                 "icp_persistent": 1}}}, open(cache, "w"))
    r = autotune.tune(lambda: None, "pers", 1000, device_name="dev0", cache_file=cache)
    assert r["from_cache"] and pc.get_tuning() == {"icp_block_threads": 128, "icp_leaf": 8, "node_budget": 0.5,
                                                   "sort_queries": 1, "icp_persistent": 0}
    pc.set_tuning(128, 16, 1.0)
