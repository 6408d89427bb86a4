"""Host logic of bench.py (CPU): the roofline's measured HBM traffic is read from the committed
rocprofv3 counter summary only while the kernel's sources match the hash recorded there."""
import importlib.util
import os
import shutil

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(root=ROOT):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    m.ROOT = root
    return m


def test_traffic_from_current_summary():
    b = _bench()
    t = b.measured_traffic("k_tsqr_factor", "n65535_r20_mixed")
    assert isinstance(t, int) and t > 0
    assert b.measured_traffic("k_core", "n65535_r20_mixed") is None
    assert b.measured_traffic("k_tsqr_factor", "n65535_r20_fp64") is None


def test_traffic_is_null_once_the_kernel_source_changes(tmp_path):
    root = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "profiles"), root / "profiles")
    csrc = root / "paper_2607_06021_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("tsqr.hip", "lrp_internal.h", "lrp_kernels.h"):
        shutil.copy(os.path.join(ROOT, "paper_2607_06021_amd", "csrc", f), csrc / f)
    b = _bench(str(root))
    assert b.measured_traffic("k_tsqr_factor", "n65535_r20_mixed") is not None
    with open(csrc / "tsqr.hip", "a") as f:
        f.write("\n// edited\n")
    assert b.measured_traffic("k_tsqr_factor", "n65535_r20_mixed") is None
