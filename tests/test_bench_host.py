"""Host logic of bench.py that needs no GPU: the traffic figure it reads from
the committed counter summary (only while the kernel source it was measured
on is unchanged) and the medians it reports from the iteration timeline."""
import hashlib
import importlib.util
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def write_profile(root, kernel, source_rel, sha, nbytes):
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    with open(os.path.join(root, "profiles", "backproject_traffic_512.md"), "w") as f:
        f.write("# counters\n\nRead by bench.py:\n\n")
        f.write(f"    kernel: {kernel}\n    kernel_source: {source_rel}\n")
        f.write(f"    kernel_source_sha256: {sha}\n    traffic_bytes_per_launch: {nbytes}\n")


def test_traffic_is_read_only_for_the_measured_source(tmp_path):
    bench = load_bench()
    src = tmp_path / "k.hip"
    src.write_text("__global__ void k() {}\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    write_profile(str(tmp_path), "k_backproject_sym8", "k.hip", sha, 29439952)
    bench.ROOT = str(tmp_path)
    assert bench.measured_traffic("k_backproject_sym8") == 29439952.0
    assert bench.measured_traffic("k_project4") is None          # another kernel
    src.write_text("__global__ void k() { /* changed */ }\n")
    assert bench.measured_traffic("k_backproject_sym8") is None  # source changed since
    os.remove(os.path.join(str(tmp_path), "profiles", "backproject_traffic_512.md"))
    assert bench.measured_traffic("k_backproject_sym8") is None  # no summary


def test_committed_summary_names_an_existing_source():
    bench = load_bench()
    kv = {}
    for line in open(os.path.join(ROOT, "profiles", "backproject_traffic_512.md")):
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            kv[k.strip()] = v.strip()
    assert kv["kernel"] == "k_backproject_sym8"
    assert os.path.exists(os.path.join(ROOT, kv["kernel_source"]))
    assert float(kv["traffic_bytes_per_launch"]) > 0
    got = bench.measured_traffic("k_backproject_sym8")
    sha = hashlib.sha256(open(os.path.join(ROOT, kv["kernel_source"]), "rb").read()).hexdigest()
    assert got == (float(kv["traffic_bytes_per_launch"]) if sha == kv["kernel_source_sha256"] else None)


def test_timeline_summary_medians_and_slack():
    bench = load_bench()
    # rows: gradient reached, projection done, update done (the period),
    # PCG set-up done, PCG done; microseconds after the previous update
    tl = np.array([[190.0, 400.0, 415.0, 105.0, 430.0],
                   [188.0, 398.0, 413.0, 110.0, 425.0],
                   [192.0, 405.0, 420.0, 100.0, 440.0],
                   [189.0, 401.0, 416.0, 108.0, 431.0]])
    s = bench.timeline_summary(tl)
    assert s["iterations"] == 4
    assert s["period"] == float(np.median(tl[:, 2]))
    assert s["gradient_reached"] == float(np.median(tl[:, 0]))
    # slack: the next gradient's time minus how long after that iteration's
    # update the PCG ended
    slack = tl[1:, 0] - (tl[:-1, 4] - tl[:-1, 2])
    assert s["pcg_slack_before_next_gradient"] == float(np.median(slack))
    assert bench.timeline_summary(tl[:2]) is None
