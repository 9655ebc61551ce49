"""Host-side checks of bench.py: the fingerprint that ties the committed rocprofv3 summaries to the
kernel code ignores comments and blank lines but not code."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_kernel_code_sha_ignores_comments_only():
    code = "int f(int a) {\n  return a + 1;  // add one\n}\n"
    assert bench.kernel_code_sha(code) == bench.kernel_code_sha("/* header */\n" + code.replace("// add one", "") + "\n\n")
    assert bench.kernel_code_sha(code) == bench.kernel_code_sha("int f(int a) {\n    return a + 1;\n}\n")
    assert bench.kernel_code_sha(code) != bench.kernel_code_sha(code.replace("a + 1", "a + 2"))


def test_kernel_code_sha_of_the_sources():
    sha = bench.kernel_code_sha(bench.kernel_sources_text())
    assert len(sha) == 16 and int(sha, 16) >= 0


def test_more_than_one_gpu_is_refused_with_a_message():
    import subprocess
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)
