"""Host-side checks of bench.py: the event sampling of the plain steps, the
comment-insensitive kernel source hash that keys the committed traffic
figure, and the single-GPU refusal."""
import math
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_event_groups_visit_every_window():
    for windows in range(1, 65):
        period = bench.event_period(windows)
        assert period > bench.EVENT_GROUP
        assert math.gcd(period, windows) == 1 or period == bench.EVENT_GROUP
        steps = 40
        starts = range(0, steps - bench.EVENT_GROUP + 1, period)
        seen = {(s + j) % windows for s in starts for j in range(bench.EVENT_GROUP)}
        if windows <= 8:
            assert seen == set(range(windows)), (windows, period, sorted(seen))


def test_code_only_ignores_comments_and_blank_space():
    a = "int f(int x) {  // add one\n  return x + 1; /* the\n answer */\n}\n"
    b = "int f(int x) { return x + 1; }"
    assert bench.code_only(a) == bench.code_only(b)
    assert bench.code_only("return x + 1;") != bench.code_only("return x + 2;")


def test_kernel_source_hash_and_traffic_figure():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    t = bench.load_traffic()
    assert t is None or t > 280e6  # at least the algorithmic bytes of a 10 M window


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
