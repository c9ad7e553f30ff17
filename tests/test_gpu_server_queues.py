"""The server's resident kernels must not hold back the caller's work.

HIP runs each hardware queue in order, so work on a stream that shares a
hardware queue with a resident kernel waits until that kernel ends.  In a
process whose streams are the caller's null stream and the server's three
(PILA builds run on the null stream), a copy on the caller's stream and
requests on new geometries finish within deadlines while long chains occupy
two queues, one of them needing its queue's kernel launched.  The scenario runs in a child process so that no stream
of the other tests is present; the child cancels its chains and destroys
the server before it exits.
"""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_caller_copy_and_new_request_not_held_behind_resident_chains():
    print("server queues: child process", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "serve_queues_child.py")],
                       capture_output=True, text=True, timeout=400)
    assert r.returncode == 0, r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    print(out, flush=True)
    assert out["ok"], out
    assert all(out["long_running"]), out
    assert out["copy_done"] and out["copy_s"] < 5.0, out
    assert out["small_long_done"] and out["small_long_s"] < 20.0, out
    assert out["small_long_body"] == 2, out  # the long-row body
    assert out["small_piped_done"] and out["small_piped_s"] < 20.0, out
    assert out["small_piped_body"] == 1, out
    assert out["left"] == 0, out
