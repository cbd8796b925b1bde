"""Host logic of bench.py (no GPU): the code hash that ties committed
hardware-counter figures to the kernel source, the lookup that reports
`traffic` only while that hash matches, and the one-GPU guard."""
import importlib.util
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load_bench(path):
    spec = importlib.util.spec_from_file_location("bench_copy", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_source_hash_ignores_comments_and_whitespace(tmp_path):
    bench = _load_bench(os.path.join(ROOT, "bench.py"))
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f(int x) {\n  return x + 1;  // one\n}\n")
    b.write_text("/* block\n comment */ int f(int x)\n{ return x + 1; }\n")
    c.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.kernel_source_hash(str(a)) == bench.kernel_source_hash(str(b))
    assert bench.kernel_source_hash(str(a)) != bench.kernel_source_hash(str(c))


def test_traffic_reported_only_for_the_profiled_source(tmp_path):
    """A copy of bench.py beside fake library sources and a fake counter
    summary: the figure comes back while the summary's hash is that of the
    sources, and None once any of them changes its code (a comment change
    keeps it)."""
    shutil.copy(os.path.join(ROOT, "bench.py"), tmp_path / "bench.py")
    csrc = tmp_path / "paper_1007_4591_amd" / "csrc"
    csrc.mkdir(parents=True)
    bench = _load_bench(str(tmp_path / "bench.py"))
    for name in bench.TRAFFIC_SOURCES:
        (csrc / name).write_text(f"// {name}\nint v_{name.replace('.', '_')} = 1;\n")
    src = csrc / "fmm.hip"
    src.write_text("__global__ void k(float *y) { y[0] = 1.f; }\n")
    sha = bench.library_source_hash()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "pmc_traffic_crowded.md").write_text(
        "| kernel | fetch bytes | write bytes | total bytes | code sha256 | launches |\n"
        "|---|---|---|---|---|---|\n"
        f"| `k<float, 0>` | 100 | 20 | 120 | {sha} | 3 of 3 |\n")
    assert bench.pmc_traffic("k<float, 0>", "crowded") == 120.0
    assert bench.pmc_traffic("k<float, 1>", "crowded") is None
    assert bench.pmc_traffic("k<float, 0>", "blobby") is None
    src.write_text("__global__ void k(float *y) { y[0] = 1.f; }  // a comment\n")
    assert bench.pmc_traffic("k<float, 0>", "crowded") == 120.0
    (csrc / "tree_build.hip").write_text("int v = 2;\n")
    assert bench.pmc_traffic("k<float, 0>", "crowded") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
