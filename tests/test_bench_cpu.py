"""The benchmark's command-line contract, without a GPU: one GPU only (a
clear message and exit status 2 for more), and the documented options."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_contract_options():
    r = run("--help")
    assert r.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--legs", "--no-cpu", "--batch-config"):
        assert opt in r.stdout


def test_serve_sample_starts_follow_the_leg_order():
    """The serving leg's oracle windows assume each request starts at its
    stream's cursor after the warm-up, three Poisson loads and the capacity
    run (the same request list each time), admitted in arrival order; here
    that order is replayed as one first-come list over every run."""
    sys.path.insert(0, ROOT)
    import bench
    import workloads
    n = 300
    warm = workloads.serve_requests(64, 1.0, seed=6)
    runs = workloads.serve_requests(n, 1.0)
    seq = warm + runs * 5
    cur, start = {}, []
    for r in seq:
        start.append(cur.get(r.stream_id, 0))
        cur[r.stream_id] = start[-1] + r.count
    check_run = start[len(warm) + 4 * n:]
    sample = bench.serve_sample(n)
    assert len(sample) == 16
    for i, (sid, p, count, wins) in sample:
        assert sid == runs[i].stream_id and count == runs[i].count and p == bench.P
        assert wins[0][0] == check_run[i]                        # the request's first value
        for w, m in wins:                                        # windows stay inside the request
            assert check_run[i] <= w and w + m <= check_run[i] + count and m == min(512, count)
