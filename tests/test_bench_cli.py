"""Host-side checks of the benchmark's command line (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_kernel_hash_names_the_kernel_sources():
    r = run("--print-kernel-hash")
    assert r.returncode == 0
    h = r.stdout.strip()
    assert len(h) == 16 and int(h, 16) >= 0


def test_tuned_table_matches_the_search_spaces():
    """Every committed tuned entry names a device (ISA x compute units), a
    workload, a net count and one of the tuner's current search spaces, and
    its configuration sets only knobs of that space to values it searches."""
    import json
    sys.path.insert(0, ROOT)
    from paper_1404_0076_amd import autotune
    with open(autotune.TUNED) as f:
        table = json.load(f)
    assert table
    spaces = {autotune.space_signature(sp): sp for sp in (autotune.BATCH_SPACE, autotune.SINGLE_SPACE)}
    for key, entry in table.items():
        dev, sig, n, space = key.split("/", 3)
        assert dev.startswith("gfx") and "x" in dev
        assert len(sig) == 16 and int(n) >= 1
        assert space in spaces, key
        allowed = dict(spaces[space])
        for k, v in entry["config"].items():
            assert v in allowed[k], (key, k, v)
        assert entry["seconds"] > 0
