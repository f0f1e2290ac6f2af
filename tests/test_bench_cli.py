"""bench.py's command line, checked without a GPU: more than one GPU is
refused before anything touches a device, the profiling modes exist, and
the kernel-source hash behind the stored traffic figures ignores comments."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_profiling_modes_are_listed():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--only-main", "--only-zoom-to", "--only-fwd-bwd", "--only-u8", "--copy-calib",
                 "--no-cpu"):
        assert flag in r.stdout, flag


def test_source_hash_ignores_comments_only():
    # the stored traffic figures stay valid across comment edits, not code edits
    sys.path.insert(0, ROOT)
    import bench
    a = 'int f() { return 1; }  // one\n/* block\n */ const char* s = "a // b";\n'
    b = '// header\nint f() {   return 1; }\n\nconst char* s = "a // b"; /* trailing */\n'
    assert bench.strip_comments(a) == 'int f() { return 1; }\nconst char* s = "a // b";'
    assert bench.strip_comments(a) != bench.strip_comments(a.replace("return 1", "return 2"))
    assert bench.strip_comments(b) == 'int f() {   return 1; }\nconst char* s = "a // b";'
    assert bench.strip_comments("char c = '\\''; int x; // y") == "char c = '\\''; int x;"
