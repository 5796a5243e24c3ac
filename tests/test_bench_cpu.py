"""bench.py's command-line contract, checked without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    """One GPU only: --gpus 2 exits with status 2 and says why, before it
    imports torch or touches a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_hash_ignores_comments_only(tmp_path, monkeypatch):
    """The hash that ties committed counter runs to the kernel sources changes
    with the code and not with its comments or blank space."""
    sys.path.insert(0, ROOT)
    import bench
    f = tmp_path / "k.hpp"
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(f)])

    def hash_of(text):
        f.write_text(text)
        return bench.kernel_hash()

    base = hash_of("int a = 1;  // one\n/* block */ int b = 2;\n")
    assert hash_of("int a = 1;  // uno\n\n/* other\n block */   int b = 2;\n") == base
    assert hash_of("int a = 1;\nint b = 3;\n") != base
