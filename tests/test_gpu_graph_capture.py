"""The library keeps no stream or event of its own: a fresh process can make
its first gs_bin_sort call inside a HIP graph capture (with the caller's side
stream for the depth sort, and with one stream), and the replays equal an
eager call bit for bit.  Each case runs in a child process so that its
gs_bin_sort is the process's first."""
import os
import subprocess
import sys

import pytest

from gpu_common import note

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("mode", ["side", "single"])
def test_first_bin_sort_of_a_process_captured_in_a_graph(mode):
    note(f"first gs_bin_sort of a fresh process under graph capture ({mode})")
    r = subprocess.run([sys.executable, os.path.join(HERE, "_capture_child.py"), mode], capture_output=True,
                       text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-2000:]
    assert "CAPTURE_OK" in r.stdout
