"""Host-side parts of bench.py, on the CPU.

* More than one GPU (by flag or by a WORLD_SIZE above 1) is refused with
  exit status 2 and a message, before anything touches a GPU.
* The HBM traffic figure of the roofline line comes from the committed
  counter summary only while the digest of the factor kernel's sources and
  the precision recorded there match; otherwise it is reported as null.
"""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                       env=e, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _record(path, sha, precision, nbytes):
    with open(path, "w") as f:
        f.write("# comment: ignored\n")
        f.write(f"precision: {precision}\n")
        f.write(f"kernel_sources_sha256: {sha}\n")
        f.write(f"hbm_bytes_per_launch: {nbytes}\n")


def test_traffic_is_read_only_for_the_current_sources(tmp_path, monkeypatch):
    b = _bench_module()
    rec = tmp_path / "traffic.txt"
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(rec))
    assert b.read_traffic("fp32_ir") is None                      # no record
    _record(rec, b.src_sha(), "fp32_ir", 33708459)
    assert b.read_traffic("fp32_ir") == 33708459.0
    assert b.read_traffic("fp64") is None                         # taken for another precision
    _record(rec, "0" * 64, "fp32_ir", 33708459)
    assert b.read_traffic("fp32_ir") is None                      # sources changed since
    _record(rec, b.src_sha(), "fp32_ir", "n/a")
    assert b.read_traffic("fp32_ir") is None                      # unreadable figure


def test_source_digest_follows_the_kernel_sources(tmp_path, monkeypatch):
    b = _bench_module()
    files = []
    for k in range(2):
        p = tmp_path / f"src{k}.hip"
        p.write_text(f"// kernel source {k}\n")
        files.append(str(p))
    monkeypatch.setattr(b, "KERNEL_SRCS", files)
    d0 = b.src_sha()
    assert d0 == b.src_sha()
    (tmp_path / "src1.hip").write_text("// kernel source 1, edited\n")
    assert b.src_sha() != d0
