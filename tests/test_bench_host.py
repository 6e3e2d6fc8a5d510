"""Host-side logic of bench.py (no GPU): the counter summaries it reports are the ones taken on
the current kernel source and on launches of the timed length; its JSON line carries every
field of the line contract; a request for more than one GPU is refused before any GPU work."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counter_entries_match_source_and_launch_length(tmp_path):
    B = _bench()
    src = tmp_path / "paper_2607_24234_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "qs_spectral.hip").write_text("// kernel source stand-in\n")
    (tmp_path / "profiles").mkdir()
    B.ROOT = str(tmp_path)
    h = B.kernel_source_hash()
    valu = {"fp32": {"kernel_sha256_16": h, "steps_per_dispatch": 500, "wave_instructions_per_cell_update": 2.71},
            "fp32_steps20": {"kernel_sha256_16": h, "steps_per_dispatch": 20, "wave_instructions_per_cell_update": 2.78},
            "fp32_stale": {"kernel_sha256_16": "0" * 16, "steps_per_dispatch": 100,
                           "wave_instructions_per_cell_update": 9.0}}
    traffic = {"fp32": {"kernel_sha256_16": h, "steps_per_dispatch": 500, "bytes_per_step": 2.0e10},
               "fp32_steps20": {"kernel_sha256_16": h, "steps_per_dispatch": 20, "bytes_per_step": 2.1e10}}
    (tmp_path / "profiles" / "march_spectral3d_valu.json").write_text(json.dumps(valu))
    (tmp_path / "profiles" / "march_spectral3d_traffic.json").write_text(json.dumps(traffic))
    assert B.read_valu("fp32", 500) == 2.71
    assert B.read_valu("fp32", 20) == 2.78
    assert B.read_valu("fp32", 20.0) == 2.78
    assert B.read_valu("fp32", 100) is None        # taken on another source
    assert B.read_valu("fp32", 19) is None         # no counters for this length
    assert B.read_valu("fp64", 500) is None
    assert B.read_traffic("fp32", 500) == 2.0e10 * 500
    assert B.read_traffic("fp32", 20) == 2.1e10 * 20
    assert B.read_traffic("fp32", 7) is None
    # a changed source invalidates every entry
    (src / "qs_spectral.hip").write_text("// changed\n")
    assert B.read_valu("fp32", 500) is None and B.read_traffic("fp32", 20) is None


def test_line_carries_the_contract_fields(capsys):
    B = _bench()
    B._line("m", 1.5, "u", 20, 5, 4.2, "f32", {"workload": "w"},
            {"bound": "alu", "achieved": 1.0, "peak": 2.0, "unit": "TFLOP/s", "frac": 0.5, "traffic": None},
            {"value": 3.0, "unit": "u", "cores": 16, "kind": "oracle", "sample": "s"}, extra=1)
    d = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["warmup"] == 5 and d["extra"] == 1
    assert set(d["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert set(d["cpu_baseline"]) >= {"value", "unit", "cores", "kind", "sample"}


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""
