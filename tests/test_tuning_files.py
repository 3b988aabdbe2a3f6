"""Tuning files (written by the autotuner on an MI355X) parse into context
options and server settings, and the autotuner's selection rules pick the
setting they state, with timings replaced by fixed values (CPU only)."""
import json
import os

import numpy as np
import pytest

from paper_2411_11244_amd import tune

TUNING = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2411_11244_amd", "tuning")


def test_server_config_reads_server_keys_only():
    cfg = {"best": {"max_slots": 128, "rounds_per_step": 8, "expand_budget": 1 << 20}}
    assert tune.server_config(cfg) == {"max_slots": 128, "rounds_per_step": 8}
    assert tune.server_config({"expand_budget": 4}) == {}


def test_committed_tuning_files_use_known_keys():
    files = [f for f in os.listdir(TUNING) if f.endswith(".json")]
    assert files
    for f in files:
        with open(os.path.join(TUNING, f)) as fh:
            best = json.load(fh)["best"]
        assert best and set(best) <= set(tune.KEYS) | set(tune.SERVER_KEYS), (f, best)
        assert all(isinstance(v, int) and v >= 0 for v in best.values()), (f, best)


def _record_options(monkeypatch):
    """Replace the binding's option setter with a recorder (no GPU)."""
    from paper_2411_11244_amd import gdist
    applied = {}
    monkeypatch.setattr(gdist, "gdist_set_option", lambda ctx, k, v: applied.__setitem__(k, v))
    return applied


def test_tune_keeps_the_fastest_setting_and_applies_it(monkeypatch):
    applied = _record_options(monkeypatch)
    # a made-up cost with its minimum at expand_budget 2^20, k_cap 8
    cost = {(1 << 18, 6): 3.0, (1 << 18, 8): 2.5, (1 << 20, 6): 2.2, (1 << 20, 8): 1.9, (1 << 22, 6): 2.0,
            (1 << 22, 8): 2.1}
    monkeypatch.setattr(tune, "time_setting", lambda ctx, descs, reps: cost[(applied["expand_budget"],
                                                                             applied["k_cap"])])
    grid = {"expand_budget": [1 << 18, 1 << 20, 1 << 22], "k_cap": [6, 8], "front_capacity": [1 << 26]}
    res = tune.tune(0, [], grid, reps=1, log=lambda *a: None)
    assert res["best"] == {"expand_budget": 1 << 20, "k_cap": 8, "front_capacity": 1 << 26}
    assert res["ms"] == 1.9 and len(res["results"]) == 6
    # the context is left at the best setting; the front capacity also sizes the leaf-pair buffers
    assert applied == {"expand_budget": float(1 << 20), "k_cap": 8.0, "front_capacity": float(1 << 26),
                       "leaf_capacity": float(1 << 26)}


def test_tune_server_prefers_low_latency_within_five_percent_of_capacity(monkeypatch):
    from paper_2411_11244_amd import gdist, serve
    applied = _record_options(monkeypatch)
    # (slots, rounds) -> (queries/s of the burst, p50 ms of the paced stream, all OK)
    table = {(64, 4): (20000.0, 0.25, True), (64, 8): (24000.0, 0.30, True), (256, 4): (25000.0, 0.40, True),
             (256, 8): (26000.0, 0.35, True), (256, 16): (30000.0, 0.20, False)}
    burst, paced = [None] * 1000, [None] * 100

    def fake_run_stream(ctx, handles, queries, max_slots=64, rounds_per_step=4, time_scale=1.0, **kw):
        qps, p50, ok = table[(max_slots, rounds_per_step)]
        status = gdist.GDIST_OK if ok else gdist.GDIST_E_CAPACITY
        return {"results": [{"status": status}] * len(queries), "wall_s": len(queries) / qps,
                "latency_ms": np.full(len(queries), p50)}

    monkeypatch.setattr(serve, "run_stream", fake_run_stream)
    grid = {"max_slots": [64, 256], "rounds_per_step": [4, 8, 16], "expand_budget": [1 << 22]}
    table[(64, 16)] = (10000.0, 0.1, True)
    res = tune.tune_server(0, [], burst, paced, grid, log=lambda *a: None)
    # (256, 16) fails a query and is out; the best capacity left is 26,000, and within 5% of it
    # (>= 24,700) (256, 8) has the lower p50 than (256, 4); (64, 16) is fast but far too slow
    assert res["best"] == {"max_slots": 256, "rounds_per_step": 8, "expand_budget": 1 << 22}
    assert applied["expand_budget"] == float(1 << 22)
    table.update({k: (q, p, False) for k, (q, p, _) in table.items()})
    with pytest.raises(RuntimeError):
        tune.tune_server(0, [], burst, paced, grid, log=lambda *a: None)
