"""The benchmark's command-line contract, on the CPU (no GPU work is started)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_measured_counters_match_the_kernel_sources():
    """Each recorded counter figure names the kernel source it was measured on; a
    stale figure is reported null rather than attributed to changed code."""
    sys.path.insert(0, ROOT)
    import hashlib

    import bench

    for (kernel, workload), m in bench.MEASURED.items():
        with open(os.path.join(ROOT, m["src"]), "rb") as f:
            current = hashlib.sha256(f.read()).hexdigest()[:16]
        for field in ("read", "write", "valu_insts"):
            got = bench.measured(kernel, workload, field)
            if current == m["sha256"] and m.get(field) is not None:
                assert got == m[field] and got > 0, (kernel, workload, field)
            else:
                assert got is None, (kernel, workload, field)
