"""Host logic of bench.py (no GPU): the single-GPU guard and the keying of the
measured HBM traffic to the kernel sources it was taken on."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "single-GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_is_read_only_for_matching_sources(tmp_path):
    b = _bench()
    src = b.kernel_source_hash()
    f = tmp_path / "traffic.md"
    f.write_text("# summary\n"
                 f"traffic: kernel=k_conv64 dtype=f32 workload=block-256x256x32 bytes_per_launch=123456 "
                 f"source_sha256={src}\n"
                 f"traffic: kernel=k_fft512 dtype=f32 workload=block-256x256x32 bytes_per_launch=777 "
                 f"source_sha256={'0' * 64}\n")
    b.TRAFFIC_FILE = str(f)
    assert b.measured_traffic("k_conv64", "f32", "block-256x256x32") == 123456.0
    # stale sources, another workload, another precision, an absent summary
    assert b.measured_traffic("k_fft512", "f32", "block-256x256x32") is None
    assert b.measured_traffic("k_conv64", "f32", "film-128x64") is None
    assert b.measured_traffic("k_conv64", "f64", "block-256x256x32") is None
    b.TRAFFIC_FILE = str(tmp_path / "absent.md")
    assert b.measured_traffic("k_conv64", "f32", "block-256x256x32") is None


def test_source_hash_covers_every_native_source():
    # the kernels, their launchers and the plan that sets launch parameters
    b = _bench()
    names = sorted(os.path.basename(p) for p in b.KERNEL_SOURCES)
    csrc = os.path.join(ROOT, "paper_2606_28113_amd", "csrc")
    assert names == sorted(n for n in os.listdir(csrc) if n.endswith((".hip", ".h")))
