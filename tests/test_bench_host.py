"""Host logic of bench.py (no GPU): the counter-traffic lookup is used only
while the kernel sources match the hashes its profile recorded, and an
optional leg that fails reports the failure instead of ending the run."""
import hashlib
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _profile(path, value, sources, root):
    lines = ["# traffic", "", f"traffic-bytes-per-launch: {value:.6e}"]
    for f in sources:
        sha = hashlib.sha256(open(f, "rb").read()).hexdigest()
        lines.append(f"source-sha256 ({os.path.relpath(f, root)}): {sha}")
    open(path, "w").write("\n".join(lines) + "\n")


def test_traffic_used_only_for_the_recorded_sources(tmp_path):
    b = _bench()
    b.ROOT = str(tmp_path)
    src1 = tmp_path / "k1.hip"
    src2 = tmp_path / "k2.h"
    src1.write_text("kernel one\n")
    src2.write_text("header two\n")
    prof = tmp_path / "prof.md"
    _profile(str(prof), 4.25e9, [str(src1), str(src2)], str(tmp_path))
    b.TRAFFIC_PROFILE = {("gather", "w"): (str(prof), [str(src1), str(src2)])}
    assert b.measured_traffic("gather", "w") == 4.25e9
    # another kernel family or workload has no profile
    assert b.measured_traffic("deposit", "w") is None
    assert b.measured_traffic("gather", "other") is None
    # a changed source voids the figure
    src2.write_text("header two, edited\n")
    assert b.measured_traffic("gather", "w") is None
    # a profile that names fewer sources than the kernel has is not used either
    src2.write_text("header two\n")
    _profile(str(prof), 4.25e9, [str(src1)], str(tmp_path))
    assert b.measured_traffic("gather", "w") is None
    # a missing profile
    os.remove(prof)
    assert b.measured_traffic("gather", "w") is None


def test_failed_leg_is_reported_not_raised():
    b = _bench()
    assert b._leg("ok leg", lambda: {"x": 1}) == {"x": 1}
    out = b._leg("bad leg", lambda: 1 / 0)
    assert set(out) == {"failed"} and out["failed"].startswith("ZeroDivisionError")
