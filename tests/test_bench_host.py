"""Host-side checks of the benchmark script: it refuses more than one GPU
with a message, its JSON output stays valid when a figure is not finite, and
the algorithmic byte models match their definitions on small sizes."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_json_line_has_no_nan():
    import bench
    out = {"value": float("nan"), "roofline": {"frac": float("inf")}, "x": [1.0, float("-inf")]}
    from io import StringIO
    import contextlib
    buf = StringIO()
    with contextlib.redirect_stdout(buf):
        bench.emit(out)
    d = json.loads(buf.getvalue())
    assert d == {"value": None, "roofline": {"frac": None}, "x": [1.0, None]}


def test_byte_models():
    import bench
    n, nnz, B = 1000, 20000, 1024
    W = 16
    assert bench.algorithmic_bytes_per_step("sir", n, nnz, B, False) == \
        4 * nnz + 8 * W * nnz + 4 * (n + 1) + 32 * W * n
    assert bench.algorithmic_bytes_per_step("ic", n, nnz, 64, True) == 4 * nnz + n / 8
    assert bench.hk_algorithmic_bytes(n, nnz, 256) == 4 * 256 * nnz + 8 * 256 * n + 4 * nnz + 4 * (n + 1)
    # finalize: IC with a frontier bitmap reads the ever-active plane only
    assert bench.finalize_bytes("ic", n, 64, True, True) == n * (8 + 64 + 4) + n / 8
    assert bench.finalize_bytes("sir", n, 1024, True, False) == n * (8 * 16 * 2 + 1024 + 4)
    assert bench.finalize_bytes("seir", n, 64, False, False) == n * (8 * 3 + 4)


def test_kernel_hash_is_per_workload():
    import bench
    h = {w: bench.kernel_source_hash(w) for w in ("c2", "c4", "hk", "c5")}
    assert h["c2"] == h["c4"] and h["hk"] != h["c2"] and h["c5"] != h["hk"]


def test_host_cpu_record():
    import bench
    hc = bench.host_cpu()
    assert hc["threads"] >= 1 and hc["threads"] <= hc["visible_cpus"]
    if (os.environ.get("OMP_NUM_THREADS") or "").isdigit():
        assert hc["threads"] <= int(os.environ["OMP_NUM_THREADS"])
    assert isinstance(hc["cpu_model"], str) and hc["cpu_model"]
    f = bench.cpu_fields(hc)
    assert f["cores"] == hc["threads"]


def test_kernel_source_hash_ignores_comments_not_code():
    """A counter record stays valid across comment and layout edits of the
    kernels' sources, and not across code edits; literals are kept."""
    sys.path.insert(0, ROOT)
    import bench
    src = ('int a = 1; // one\n/* block\n comment */ const char *s = "x // y /* z */";\n'
           "char q = '\\''; int  b =\n 2;")
    assert bench.strip_comments(src) == \
        'int a = 1; const char *s = "x // y /* z */"; char q = \'\\\'\'; int b = 2;'
    assert bench.strip_comments("a/* c */b") == "a b"
    assert bench.strip_comments(src.replace("// one", "// two")) == bench.strip_comments(src)
    assert bench.strip_comments(src.replace(" 2;", " 3;")) != bench.strip_comments(src)
