"""bench.py's contract pieces that run without a GPU: one GPU only, the roofline arithmetic and
the rule that committed counters count only on the kernel source they were taken on."""
import importlib.util
import json
import os
import subprocess
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_roofline_arithmetic():
    b = load_bench()
    R = types.SimpleNamespace
    # two steps of one plain design: 10 launches each, 5 of them timed (0.5 ms in all)
    step = [R(n_cells=1000, n_visits=500, n_candidates=100, n_span_launches=10, n_timed_launches=5,
              t_span_kernels_s=5e-4)]
    roof = b.roofline_for([step, step], None, False)
    alg = 2 * (72 * 1000 + 20 * 500 + 12 * 100)
    assert roof["launches"] == 20 and roof["timed_launches"] == 10
    assert abs(roof["alg_bytes_per_launch"] - alg / 20) < 1e-9
    assert abs(roof["avg_launch_us"] - 100.0) < 1e-9  # 1 ms over 10 timed launches
    assert abs(roof["achieved"] - (alg / 20) / 1e-4 / 1e9) < 1e-12
    assert roof["frac"] == roof["achieved"] / 8000.0 and roof["peak"] == 8000.0
    assert roof["traffic"] is None and roof["bound"] == "hbm" and roof["unit"] == "GB/s"
    # a batched step is one persistent launch, timed whole
    bstep = [R(n_cells=1000, n_visits=500, n_candidates=100, n_span_launches=0, n_timed_launches=0,
               t_span_kernels_s=0.25), R(n_cells=3000, n_visits=0, n_candidates=0, n_span_launches=0,
                                         n_timed_launches=0, t_span_kernels_s=0.25)]
    roof = b.roofline_for([bstep], {"hbm_bytes_per_launch": 123.0}, True)
    assert roof["launches"] == 1 and roof["timed_launches"] == 1 and abs(roof["avg_launch_us"] - 5e5) < 1e-6
    assert roof["alg_bytes_per_launch"] == 72 * 4000 + 20 * 500 + 12 * 100 and roof["traffic"] == 123.0


def test_counter_records_count_only_on_their_kernel_source(monkeypatch):
    b = load_bench()
    for name, fn in b.COUNTER_FILES.items():
        rec = json.load(open(os.path.join(ROOT, "profiles", fn)))
        monkeypatch.setattr(b, "kernel_source_sha", lambda rec=rec: rec["kernel_source_sha256"])
        assert b.profile_record(name)["hbm_bytes_per_launch"] == rec["hbm_bytes_per_launch"]
        monkeypatch.setattr(b, "kernel_source_sha", lambda: "0" * 64)
        assert b.profile_record(name) is None
