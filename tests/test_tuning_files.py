"""Tuning files (written by the autotuner on an MI355X) parse into context
options and server settings (CPU only)."""
import json
import os

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
