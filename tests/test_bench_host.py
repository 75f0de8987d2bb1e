"""Host-side checks of the benchmark contract and of the committed profile
summaries (no GPU needed)."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2410_09739_amd import profiling as P  # noqa: E402

TRAFFIC = os.path.join(ROOT, "profiles", "traffic_stream_collide_taylor_green_512.md")
TRACE = os.path.join(ROOT, "profiles", "stream_collide_taylor_green_512_kernel_trace.md")


@pytest.mark.parametrize("n", [2, 8])
def test_bench_refuses_more_than_one_gpu(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert r.stdout.strip() == ""  # no JSON line for a multi-GPU request
    assert "one GPU" in r.stderr + r.stdout


def test_traffic_summary_matches_the_kernel_sources():
    """The HBM byte counts the benchmark reports as roofline.traffic were taken
    with the stream-collide sources as they are now (else the benchmark reports
    null): a kernel change must come with a new measurement.  FP32 and FP64 run
    in the XCD-aware block order and fetch within 2 % of the algorithmic bytes;
    the 16-bit forms run in the plain order, where the two halves of a 512-node
    row sit on different XCDs and the cache lines at their seams are fetched
    by both (8 % more reads; the plain order still runs faster for them)."""
    t = P.read_traffic_md(TRAFFIC)
    assert t is not None
    assert t["kernel_source_sha"] == P.kernel_source_hash()
    for form, algo, bound in (("f32", 216, 1.02), ("f64", 432, 1.02), ("f16dev", 108, 1.10), ("bf16dev", 108, 1.10)):
        f = t["forms"][form]
        assert f["algorithmic_bytes_per_launch"] == algo * 512 ** 3
        assert 0.99 < f["traffic_over_algorithmic"] < bound, form


def test_kernel_trace_summary_covers_the_timed_kernel():
    text = open(TRACE).read()
    assert "rocprofv3 --kernel-trace --stats" in text
    # FP32, periodic, no force, unit higher-order rates: the benchmark's kernel
    assert "k_stream_collide<1, 0, false, false, 1>" in text
    assert "512x512x512" in text


def test_source_hash_ignores_comments_but_not_code():
    a = 'int f(int x) { return x + 1; } // one\n/* block\n comment */\nconst char* s = "// kept /* too */";\n'
    b = 'int f(int x)\n{\n  return x + 1;   // another comment\n}\nconst char* s = "// kept /* too */";\n'
    c = 'int f(int x) { return x + 2; }\nconst char* s = "// kept /* too */";\n'
    assert P._code_only(a) == P._code_only(b)
    assert P._code_only(a) != P._code_only(c)
    assert '"// kept /* too */"' in P._code_only(a)


def test_closure_errors_file_matches_the_kept_networks():
    """The benchmark's closure cost at equal error uses the study's held-out
    errors only while the kept networks are the ones they were measured with
    (else it reports nothing): a retrained network must come with new errors."""
    import hashlib
    import json
    data = os.path.join(ROOT, "paper_2410_09739_amd", "data")
    d = json.load(open(os.path.join(data, "closure_channel_errors.json")))
    assert set(d["networks_sha256"]) == {"closure_channel_192x96x96.npy", "closure_channel_128x64x64_refined.npy"}
    for name, sha in d["networks_sha256"].items():
        assert hashlib.sha256(open(os.path.join(data, name), "rb").read()).hexdigest() == sha, name


def test_closure_cost_at_equal_error_follows_its_definition(tmp_path, monkeypatch):
    """cost = r^4 x (closure MLUPS / plain FP32 MLUPS) with r = (e_plain /
    e_closure)^(1/p), p from the plain errors of the two coarse grids (spacing
    ratio 1.5); nothing when a network's hash does not match its errors."""
    import importlib.util
    import json
    import shutil
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    data = tmp_path / "paper_2410_09739_amd" / "data"
    data.mkdir(parents=True)
    src = os.path.join(ROOT, "paper_2410_09739_amd", "data")
    for name in ("closure_channel_192x96x96.npy", "closure_channel_128x64x64_refined.npy"):
        shutil.copy(os.path.join(src, name), data / name)
    d = json.load(open(os.path.join(src, "closure_channel_errors.json")))
    d["grids"] = {"192x96x96": {"plain_f32": [0.06, 0.06], "closure_f16dev": [0.02, 0.02]},
                  "128x64x64": {"plain_f32": [0.135, 0.135], "closure_f16dev": [0.03, 0.03]}}
    (data / "closure_channel_errors.json").write_text(json.dumps(d))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    cg = {"f32": {"mlups": 26000.0}, "f16dev+closure": {"mlups": 13000.0}}
    c = b.closure_cost_at_equal_error(cg)
    p = np.log(0.135 / 0.06) / np.log(1.5)  # = 2 exactly: errors go as dx^2
    assert c["plain_error_order"] == pytest.approx(p, abs=1e-3) and p == pytest.approx(2.0)
    assert c["plain_refinement_for_equal_error"] == pytest.approx(3.0 ** 0.5, abs=1e-3)
    assert c["plain_f32_cost_over_closure_cost"] == pytest.approx(9.0 * 0.5, rel=1e-3)
    d["networks_sha256"]["closure_channel_192x96x96.npy"] = "0" * 64
    (data / "closure_channel_errors.json").write_text(json.dumps(d))
    assert b.closure_cost_at_equal_error(cg) is None
