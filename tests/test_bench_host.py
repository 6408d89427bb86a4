"""Host logic of bench.py (CPU): the roofline's measured HBM traffic is read from a committed
rocprofv3 counter summary only while the kernel's sources match the hash recorded there."""
import hashlib
import importlib.util
import os
import re
import shutil

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUMMARY = "tsqr_factor_n65535_mixed_traffic.md"


def _bench(root=ROOT):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    m.ROOT = root
    return m


def _fresh_copy(tmp_path):
    """The profiles and the summary's sources in a scratch tree, with the recorded hash set to
    the sources as they are now (as if the counters had just been taken)."""
    root = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "profiles"), root / "profiles")
    path = root / "profiles" / SUMMARY
    text = path.read_text()
    srcs = re.search(r"^- sources: (.*)$", text, flags=re.M).group(1).split()
    h = hashlib.sha256()
    for src in srcs:
        dst = root / src
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, src), dst)
        h.update(dst.read_bytes())
    path.write_text(re.sub(r"^- source_sha256: \w+$", f"- source_sha256: {h.hexdigest()}", text, flags=re.M))
    return root, srcs


def test_traffic_read_while_the_sources_match(tmp_path):
    root, _ = _fresh_copy(tmp_path)
    b = _bench(str(root))
    t = b.measured_traffic("k_tsqr_factor", "n65535_r20_mixed")
    assert isinstance(t, int) and t > 0
    assert b.measured_traffic("k_core", "n65535_r20_mixed") is None
    assert b.measured_traffic("k_tsqr_factor", "n65535_r20_fp64") is None


def test_traffic_is_null_once_the_kernel_source_changes(tmp_path):
    root, srcs = _fresh_copy(tmp_path)
    b = _bench(str(root))
    assert b.measured_traffic("k_tsqr_factor", "n65535_r20_mixed") is not None
    with open(root / srcs[0], "a") as f:
        f.write("\n// edited\n")
    assert b.measured_traffic("k_tsqr_factor", "n65535_r20_mixed") is None
