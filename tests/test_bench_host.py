"""bench.py's host logic (no GPU): the buffer rotation that keeps a launch
from rewriting the lines the launch before it wrote, and the refusal of
more than one GPU."""
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))
import bench  # noqa: E402


def test_rotation_takes_input_and_output_sets_in_turn():
    seen = []
    f = bench.rotating(lambda i, o: seen.append((i, o)), ["in0", "in1"], ["o0", "o1", "o2", "o3"])
    for _ in range(9):
        f()
    assert seen == [("in%d" % (k % 2), "o%d" % (k % 4)) for k in range(9)]
    # no launch writes the output set the launch before it wrote, and the
    # same (input, output) pair comes back only after 4 launches
    assert all(seen[k][1] != seen[k + 1][1] for k in range(8))
    assert len(set(seen[:4])) == 4


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=str(ROOT))
    assert r.returncode != 0 and "one GPU" in r.stderr and not r.stdout.strip()
