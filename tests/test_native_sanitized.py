"""Host code under AddressSanitizer and UBSan (CPU only): the context arena
allocator against a byte-map model, and the oracle on a small problem (both
projection forms, the evaluation metrics and top-k, a tetrahedron mesh)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-g", "-O1"]


def build_and_run(tmp_path, name, srcs, incs, extra=()):
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17"] + SAN + list(extra) + [f"-I{i}" for i in incs] + srcs + ["-o", exe]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    return out.stdout


def test_arena_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2306_08132_amd", "csrc")
    out = build_and_run(tmp_path, "arena_check", [os.path.join(ROOT, "tests", "native", "arena_check.cpp"),
                                                   os.path.join(csrc, "arena.cpp")], [csrc])
    assert "arena ok" in out


def test_oracle_under_sanitizers(tmp_path):
    od = os.path.join(ROOT, "oracle")
    out = build_and_run(tmp_path, "oracle_check", [os.path.join(ROOT, "tests", "native", "oracle_check.cpp"),
                                                    os.path.join(od, "oracle.cpp"), os.path.join(od, "mesh.cpp")],
                        [od], extra=["-fopenmp"])
    assert "oracle ok" in out


def test_serving_loop_under_thread_sanitizer(tmp_path):
    """The serving loop's host core with an executor that computes each step on
    the CPU through the oracle: concurrent submit, poll and cancel; admission
    under a full arena; the candidate capacity and job limit; an executor that
    throws; shutdown with jobs in flight (tests/native/sched_check.cpp)."""
    csrc = os.path.join(ROOT, "paper_2306_08132_amd", "csrc")
    od = os.path.join(ROOT, "oracle")
    exe = str(tmp_path / "sched_check")
    srcs = [os.path.join(ROOT, "tests", "native", "sched_check.cpp"), os.path.join(csrc, "serve_core.cpp"),
            os.path.join(csrc, "arena.cpp"), os.path.join(od, "oracle.cpp"), os.path.join(od, "mesh.cpp")]
    cmd = ["g++", "-std=c++17", "-fsanitize=thread", "-g", "-O1", "-Wno-unknown-pragmas", f"-I{csrc}", f"-I{od}",
           f"-I{os.path.join(ROOT, 'include')}"] + \
        srcs + ["-o", exe, "-lpthread"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1")
    for _ in range(3):  # a few schedules of the same threads
        out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert out.returncode == 0, out.stdout + out.stderr[-4000:]
        assert "sched ok" in out.stdout
