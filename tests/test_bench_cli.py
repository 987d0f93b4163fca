"""The bench's command-line contract on the host: more than one GPU and the
profiling-only options outside a profiling run exit with a message before
anything touches a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_several_gpus_exit_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_profiling_options_need_a_profiling_run():
    for opt in (["--level", "8"], ["--sparse-adam"]):
        r = _run(*opt)
        assert r.returncode == 2, opt
        assert "--profile-steps" in r.stderr, opt
