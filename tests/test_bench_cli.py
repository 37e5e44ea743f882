"""bench.py on the host: its command line (one GPU only) and the lookup of
committed counter summaries."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_counter_summaries_apply_only_to_their_kernel_sources_and_workload(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    k = "k_fused<approx, int16 in, uniform, int16 levels, int16 out>"
    c = {"kernel": k, "source_sha256": bench.kernel_source_hash(k), "frames": 8, "q": 16,
         "fetch_kib": 150.0, "write_kib": 200.0, "copy_fetch_kib": 50.0, "copy_write_kib": 100.0, "copy_bytes": 102400,
         "strips": 10, "sq_insts_valu": 6144.0, "sq_insts_valu_f64": 1024.0}
    path = tmp_path / "c.json"
    path.write_text(json.dumps(c))
    wl = {"frames": 8, "q": 16}
    # 100 KiB copy: FETCH x 2, WRITE x 1
    assert bench._traffic(k, str(path), wl) == (300.0 + 200.0) * 1024
    assert bench._traffic(k, str(path), {"frames": 1, "q": 16}) is None
    assert bench._traffic("k_mfma_fused<false, true, 1, true>", str(path), wl) is None
    comp = bench._compute(k, 1e-6, str(path), wl)
    assert comp["valu_instr_per_strip"] == 614.4 and comp["valu_f64_share"] == round(1024 / 6144, 4)
    assert "mfma_busy_frac" not in comp
    c["source_sha256"] = "0" * 64
    path.write_text(json.dumps(c))
    assert bench._traffic(k, str(path), wl) is None and bench._compute(k, 1e-6, str(path), wl) is None
    assert bench._traffic(k, str(tmp_path / "absent.json"), wl) is None
