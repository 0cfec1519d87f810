"""CPU checks of the measurement side: the HBM-traffic figures bench.py
reports belong to the compute source they were measured on (bench.py drops
them to null otherwise),
every rocprofv3 summary under profiles/ gives the command that produced it,
and a request for more than one GPU is refused before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_traffic_figure_belongs_to_the_compute_source():
    import bench
    t = bench.TRAFFIC_PROFILE
    # the figure is the FETCH and WRITE counters scaled by the copy-probe factors
    assert t["bytes_per_launch"] == t["fetch_kib"] * 1024 * t["fetch_factor"] + t["write_kib"] * 1024 * t["write_factor"]
    # reported only for the source it was measured on, null otherwise
    if t["source"] == bench.source_hash(bench.TRAFFIC_SOURCE):
        assert bench.traffic_bytes() == t["bytes_per_launch"]
    else:
        assert bench.traffic_bytes() is None


def test_profiles_give_their_commands():
    pdir = os.path.join(ROOT, "profiles")
    names = sorted(f for f in os.listdir(pdir) if f.endswith((".md", ".txt")))
    assert names, "no profile summaries"
    for f in names:
        text = open(os.path.join(pdir, f)).read()
        assert "rocprofv3 " in text, f"{f}: no rocprofv3 command"
        assert "_work" not in text, f"{f}: refers to working files"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
