"""Host logic of the measurement records (CPU): the HBM traffic record and the
instruction-mix summary are read back only while their source digest is the
current one, kernel names match with or without the spaces rocprofv3 prints,
and the bench refuses more than one GPU before touching any device."""
import json
import os
import subprocess
import sys

from paper_2606_11529_amd import profiling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _traffic_file(tmp_path, digest):
    tab = {"fetch_factor": 2.0, "write_factor": 1.0,
           "kernels": {"xpr::k_render_bwd<16, 16, 64, 4, false>":
                       {"launches": 3, "fetch_kib": 10.0, "write_kib": 4.0, "bytes": 24.0 * 1024}}}
    p = tmp_path / "traffic.txt"
    p.write_text(profiling.traffic_text(tab, "cmd", digest))
    return str(p)


def test_traffic_record_follows_the_source_digest(tmp_path):
    good = _traffic_file(tmp_path, profiling.sources_digest())
    assert profiling.traffic_of(good, "xpr::k_render_bwd<16,16,64,4,false>") == 24.0 * 1024
    assert profiling.traffic_of(good, "xpr::k_render_fwd<16,16,256,1,false>") is None
    stale = _traffic_file(tmp_path, "0" * 64)
    assert profiling.traffic_of(stale, "xpr::k_render_bwd<16,16,64,4,false>") is None
    assert profiling.traffic_of(str(tmp_path / "missing.txt"), "xpr::k") is None


def test_valu_busy_summary_follows_the_source_digest(tmp_path):
    def write(digest):
        p = tmp_path / f"sq_{digest[:4]}.md"
        p.write_text("\n".join([
            "# summary", "", f"sources_sha256: {digest}", "",
            "| kernel | waves | VALU busy | LDS conflict cyc/instr |",
            "|---|---:|---:|---:|",
            "| `xpr::k_render_bwd<16, 16, 64, 4, false>` | 6700 | 0.77 | 0.06 |",
            "| `xpr::k_render_fwd<16, 16, 256, 1, false>` | 26800 | 0.84 | 0.01 |", ""]))
        return str(p)
    good = write(profiling.sources_digest())
    assert profiling.valu_busy_of(good, "xpr::k_render_bwd<16,16,64,4,false>") == 0.77
    assert profiling.valu_busy_of(good, "xpr::k_render_fwd<16,16,256,1,false>") == 0.84
    assert profiling.valu_busy_of(good, "xpr::k_project<3>") is None
    assert profiling.valu_busy_of(write("f" * 64), "xpr::k_render_bwd<16,16,64,4,false>") is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1]
    out = json.loads(line)
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]
