"""The benchmark configurations stored in workloads/configs.json: the five
records, the generators they name, and the instances the config functions
build from them (sizes of the configurations as specified)."""
import workloads as W


def test_records():
    cfg = W.configs()
    assert sorted(cfg) == ["C1", "C2", "C3", "C4", "C5"]
    for name, rec in cfg.items():
        assert {"what", "generator", "params", "seed", "run"} <= set(rec), name
    assert cfg["C3"]["params"]["n"] == 70_000_000 and cfg["C3"]["params"]["c"] == 32
    assert cfg["C5"]["params"]["requests"] == 4096


def test_c1_is_the_small_fp64_instance():
    wl = W.config_small_fp64()
    assert (wl.n, wl.c, wl.nnz) == (2000, 8, 40_000)   # 20,000 pairs, mirrored
    assert str(wl.val.dtype) == "torch.float64" and str(wl.U0.dtype) == "torch.float64"
    again = W.from_config("C1")
    assert bool((again.col_idx == wl.col_idx).all()) and bool((again.val == wl.val).all())


def test_smaller_instances_of_the_large_families():
    c2 = W.config_medium(n=20_000)
    assert (c2.n, c2.c) == (20_000, 32) and c2.meta["avg_deg"] == 30.0
    c3 = W.config_full_power_law(n=30_000)
    assert (c3.n, c3.c) == (30_000, 32) and c3.meta["pattern"] == "chung-lu"
    assert c3.meta["gamma"] == 2.1 and c3.meta["wmax"] == 50_000.0


def test_serving_requests_follow_the_stored_ranges():
    p = W.configs()["C5"]["params"]
    for i in range(12):
        r = W.serving_request(i)
        assert p["n_loguniform"][0] <= r.n <= p["n_loguniform"][1]
        assert r.c in p["c_choices"]
        assert p["avg_deg_uniform"][0] <= r.meta["avg_deg"] <= p["avg_deg_uniform"][1]
