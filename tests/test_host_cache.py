"""Host logic on the CPU: the autotuner's cache file is valid JSON, round-trips
every entry, and ignores lines it cannot read."""
import json
import subprocess

import pytest

from host_build import compile_harness


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    return compile_harness("cache_harness", tmp_path_factory.mktemp("cache"))


def _read(exe, path):
    out = subprocess.run([exe, "read", str(path)], capture_output=True, text=True, check=True).stdout
    rows = [line.split() for line in out.strip().split("\n") if line]
    return {r[0]: (int(r[1]), int(r[2]), int(r[3]), float(r[4])) for r in rows}


def test_cache_round_trip_is_json(harness, tmp_path):
    path = tmp_path / "tune.json"
    subprocess.run([harness, "write", str(path)], check=True)
    doc = json.load(open(path))
    assert doc["sigA|R=1024"] == {"tn": 64, "persistent": 1, "blocks_per_cu": 4, "ms": 0.123456}
    assert set(doc) == {"sigA|R=1024", "sigA|R=256", "sigB|R=64"}
    got = _read(harness, path)
    assert got == {k: (v["tn"], v["persistent"], v["blocks_per_cu"], v["ms"]) for k, v in doc.items()}


def test_cache_skips_unreadable_entries(harness, tmp_path):
    path = tmp_path / "tune.json"
    path.write_text('{\n'
                    '"good|R=64": {"tn": 128, "persistent": 0, "blocks_per_cu": 2, "ms": 1.000000},\n'
                    '"bad_tn|R=64": {"tn": 96, "persistent": 0, "blocks_per_cu": 2, "ms": 1.0},\n'
                    '"bad_pe|R=64": {"tn": 64, "persistent": 3, "blocks_per_cu": 2, "ms": 1.0},\n'
                    'garbage line\n'
                    '"short|R=64": {"tn": 64}\n'
                    '}\n')
    assert _read(harness, path) == {"good|R=64": (128, 0, 2, 1.0)}


def test_missing_cache_reads_empty(harness, tmp_path):
    assert _read(harness, tmp_path / "absent.json") == {}
