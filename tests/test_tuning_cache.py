"""The committed autotuner cache for gfx950 names only launchable tile
variants (3 is withdrawn) and range widths the library accepts."""
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cache_entries_are_launchable():
    with open(os.path.join(ROOT, "paper_1402_3010_amd", "tuning", "gfx950.json")) as fh:
        cache = json.load(fh)
    assert cache
    kinds = set()
    for key, rec in cache.items():
        parts = key.split("|")
        assert parts[0] == "gfx950" and parts[1] in ("join", "screened"), key
        kinds.add(parts[1])
        assert rec["variant"] in (0, 1, 2), key
        # ranges are whole corpus blocks (1,024 or 2,048 rows per block)
        assert rec["range_rows"] >= 1024 and rec["range_rows"] % 1024 == 0, key
        assert rec["ms"] > 0, key
    # the benchmark's workloads: self-joins and the screened join
    assert {"join", "screened"} <= kinds
