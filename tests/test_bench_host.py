"""Host-side parts of bench.py (no GPU): the one-GPU guard, the kernel-name
rule and the reading of committed counter summaries."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2 and "one GPU" in out.stdout


def test_kernel_name_follows_the_schedule():
    b = load_bench()

    class A:
        pass
    a = A()
    a.rv_lanes, a.tile_nnz, a.max_row_nnz, a.nnz = 0, 1024, 7, 5000
    # one table, 3-bit index in the column word: the instance with the split
    # folded in; any other table size, layout or block tables: the general one
    a.block_rows, a.idx_bits, a.idx_layout = 0, 3, 1
    assert b.kernel_name(a) == "k_spmv_rows<1, 7, false, 3>"
    for m, bw in ((1, 3), (3, 3), (4, 5), (5, 5), (6, 7), (8, 8)):
        a.max_row_nnz = m
        assert b.kernel_name(a) == f"k_spmv_rows<1, {bw}, false, 3>"
    a.max_row_nnz = 7
    for bits, lay, blk, name in ((4, 1, 0, "false"), (3, 2, 0, "false"), (3, 1, 256, "true")):
        a.idx_bits, a.idx_layout, a.block_rows = bits, lay, blk
        assert b.kernel_name(a) == f"k_spmv_rows<1, 7, {name}, -1>"
    a.block_rows, a.idx_bits, a.idx_layout = 0, 3, 1
    for m in (9, 24):
        a.max_row_nnz = m
        assert b.kernel_name(a) == "k_spmv_ring<1>"
    a.max_row_nnz = 7
    a.nnz = 900
    assert b.kernel_name(a) == "k_spmv_short<1, 4>"
    a.tile_nnz = 2048
    assert b.kernel_name(a) == "k_spmv_short<1, 8>"
    a.tile_nnz, a.max_row_nnz = 1024, 100
    assert b.kernel_name(a) == "k_spmv<1, 4>"
    a.rv_lanes = 8
    assert b.kernel_name(a) == "k_spmv_rv<1, 8>"


def test_traffic_summary_is_used_only_while_sources_match(tmp_path, monkeypatch):
    b = load_bench()
    prof = tmp_path / "profiles"
    prof.mkdir()
    for rel in b.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(ROOT, rel), "rb").read())
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    digest = b.source_digest()
    text = ("- kernel: `k_spmv_short<1, 4>`\n- workload: `w`\n"
            f"- source_digest: `{digest}`\n- hbm_bytes_per_launch: `123456`\n")
    (prof / "traffic_spmv_s1_diffusion3d_128.md").write_text(text)
    assert b.measured_traffic("k_spmv_short<1, 4>", "w") == 123456
    assert b.measured_traffic("k_spmv<1, 4>", "w") is None      # another kernel
    assert b.measured_traffic("k_spmv_short<1, 4>", "v") is None  # another workload
    (tmp_path / b.KERNEL_SOURCES[0]).write_text("// changed\n")
    assert b.measured_traffic("k_spmv_short<1, 4>", "w") is None  # kernel changed since


def test_cpu_baseline_threads_keep_the_sequential_result():
    """The CPU baseline runs the oracle's row routine over contiguous row
    blocks on several host threads; each row keeps its order, so the result
    equals the sequential oracle's bit for bit (the leg reports that)."""
    from workloads import diffusion3d
    b = load_bench()
    r = b.cpu_baseline(diffusion3d(12, 0), 0.2)
    assert r["kind"] == "oracle" and r["cores"] >= 1 and r["value"] > 0
    assert "sequential result: True" in r["sample"]


def test_bench_line_stays_strict_json():
    import json
    b = load_bench()
    v = b.json_safe({"a": float("inf"), "b": [1.0, float("nan")], "c": {"d": -float("inf")}})
    assert json.loads(json.dumps(v, allow_nan=False)) == {"a": "inf", "b": [1.0, "nan"],
                                                          "c": {"d": "-inf"}}
