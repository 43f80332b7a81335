"""Host-only checks of the job queue behind Algorithm 1's crossover threads
(Section 3.1): a capped number of threads, queued jobs that never block the
thread queueing them, and a cancel that drops the jobs not yet started.
Built with g++ from the library's header; no GPU."""
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_24429_amd", "csrc")


def _run(tmp_path):
    exe = tmp_path / "job_queue_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-pthread", "-I", CSRC,
                           os.path.join(ROOT, "tests", "cpp", "job_queue_check.cpp"),
                           "-o", str(exe)])
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True,
                         timeout=60).stdout
    return {line.split()[0]: dict(re.findall(r"(\w+) ([-\d.]+)", line))
            for line in out.strip().splitlines()}


def test_job_queue(tmp_path):
    r = _run(tmp_path)
    cap = r["cap1"]
    assert float(cap["push_s"]) < 0.02          # queueing never waits for a job
    assert int(cap["peak"]) == 1 and int(cap["done"]) == 5 and int(cap["started"]) == 5
    assert float(cap["total_s"]) >= 5 * 0.04
    c = r["cancel"]
    assert int(c["started"]) == 2 and int(c["ran"]) == 2   # the other 4 were dropped
    assert float(c["total_s"]) < 5
    assert int(r["nocap"]["peak"]) == 8 and int(r["nocap"]["started"]) == 8
    e = r["external"]
    assert int(e["before"]) == 0 and int(e["done"]) == 3
