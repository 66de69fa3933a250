"""Every bench.py workload emits one JSON line with the required fields
(small settings; the numbers themselves are not checked)."""

import json
import sys

import pytest

pytestmark = pytest.mark.gpu

REQUIRED = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
            "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config")


def _run(monkeypatch, capsys, argv):
    import bench
    monkeypatch.setattr(sys, "argv", ["bench.py"] + argv)
    print(f"bench {' '.join(argv)}", file=sys.stderr, flush=True)
    bench.main()
    lines = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    line = json.loads(lines[-1])
    for k in REQUIRED:
        assert k in line, k
    assert line["n_gpus"] == 1 and line["value"] > 0 and "workload" in line["config"]
    return line


def test_scale_workload_line(monkeypatch, capsys):
    line = _run(monkeypatch, capsys, ["--workload", "scale", "--steps", "2", "--warmup", "1",
                                      "--no-plain", "--no-graph", "--cpu-sample", "200"])
    r = line["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["peak"] == 8000.0 and 0 < r["frac"] < 1
    c = line["cpu_baseline"]
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in c, k
    assert c["kind"] == "oracle"
    assert line["separate_calls"]["identical_matches"]
    assert 0 < line["mutual"]["mutual_matches"] <= line["mutual"]["forward_matches"]


def test_batch_workload_line(monkeypatch, capsys):
    """The default line (the batching configuration) on a few pairs: roofline
    and CPU baseline present, every other form identical, the oracle sample
    identical."""
    line = _run(monkeypatch, capsys, ["--pairs", "8", "--steps", "2", "--warmup", "1",
                                      "--cold-steps", "2", "--no-tune", "--cpu-every", "2"])
    r = line["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["peak"] == 8000.0 and 0 < r["frac"] < 1
    c = line["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0
    assert line["oracle_check"]["identical"] and line["oracle_check"]["pairs"] == 4
    for k in ("graph", "fp32_masters_fused", "fp8_rows_fused", "separate_calls_bf16"):
        assert line[k]["identical_matches"], k
    assert line["step_ms_cold"]["steps"] == 2
    assert line["speedup_vs_plain"] > 1


def test_precision_workload_line(monkeypatch, capsys):
    line = _run(monkeypatch, capsys, ["--workload", "precision", "--steps", "1", "--warmup", "0"])
    assert set(line["paths"]) == {"f32", "f32_plain", "bf16", "fp8", "bf16_measured",
                                  "fp8_measured", "bin256", "f32_fused", "bf16_fused",
                                  "fp8_fused"}
    for name, entry in line["paths"].items():
        if name != "bin256":
            assert entry["identical_to_plain"], name
    assert set(line["error_vs_fp64"]) == {"f32_canonical", "bf16_mfma", "fp8_mfma", "pairs"}


def test_learned_workload_line(monkeypatch, capsys):
    line = _run(monkeypatch, capsys, ["--workload", "learned", "--train-pairs", "8",
                                      "--test-pairs", "2", "--epochs", "1", "--steps", "1",
                                      "--warmup", "0"])
    assert line["training"]["residual_samples"] > 0
    assert len(line["held_out"]["fixed"]) > 3


def test_paper_workload_line(monkeypatch, capsys):
    line = _run(monkeypatch, capsys, ["--workload", "paper", "--steps", "1", "--warmup", "0",
                                      "--no-plain", "--no-separate", "--cpu-sample", "20"])
    assert line["roofline"]["kernel"].startswith("k_wide_tile")
    assert line["config"]["wide_rows"] > 0.9 * line["config"]["queries_per_step"]
    assert line["cpu_baseline"]["kind"] == "oracle"
