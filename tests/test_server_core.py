"""The serving scheduler (paper_2607_06731_amd/csrc/server_core.h) on the
CPU: tests/server_harness.cpp drives it against a simulated device on a
fake clock and checks its bookkeeping after every step (arenas within
capacity and equal to the blocks held, no double or misplaced delivery, no
delivery for a failed or cancelled request).  Built twice: optimized, and
under AddressSanitizer + UndefinedBehaviorSanitizer (no recovery).

Scenarios: continuous batching with chunking (chunk and launch caps
respected, every program's value delivered to its request), backpressure
(a small device budget makes requests wait; the arena never overflows),
one launch per request (the comparison mode), launch failures at enqueue
and at completion and upload failures for poisoned requests (only those
fail; requests batched with them are retried alone and succeed),
cancellation (at submit and in flight; cancelled requests never receive
results and release their memory), and a randomized mix of all of these."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "server_harness.cpp")
INC = os.path.join(ROOT, "paper_2607_06731_amd", "csrc")


def _build(tmp, sanitize):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    exe = str(tmp / ("server_harness_san" if sanitize else "server_harness"))
    flags = ["-std=c++17", "-I", INC]
    flags += (["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
              if sanitize else ["-O2"])
    subprocess.check_call([cxx] + flags + [SRC, "-o", exe])
    return exe


@pytest.fixture(scope="module", params=[False, True], ids=["O2", "asan-ubsan"])
def harness(request, tmp_path_factory):
    return _build(tmp_path_factory.mktemp("srv"), request.param)


def _run(exe, scenario, seed=1):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, scenario, str(seed)], stdout=subprocess.PIPE,
                       stderr=subprocess.PIPE, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    out = {}
    for kv in r.stdout.split():
        k, v = kv.split("=", 1)
        try:
            out[k] = float(v) if "." in v else int(v)
        except ValueError:
            out[k] = v
    assert out["checks_failed"] == 0
    assert out["wrong"] == 0
    return out


def test_batching_and_chunking(harness):
    o = _run(harness, "plain")
    assert o["ok"] == o["requests"]
    assert o["max_chunk_work"] <= o["chunk_cap"]
    assert o["max_launch_work"] <= o["batch_cap"]
    assert o["max_chunks"] <= 64
    assert o["launches"] < sum([o["requests"], 1000])


def test_backpressure(harness):
    o = _run(harness, "backpressure")
    assert o["ok"] == o["requests"]
    assert o["max_waiting"] > 0                    # requests had to wait for memory
    assert o["max_dev_used"] <= o["dev_capacity"]


def test_one_launch_per_request(harness):
    o = _run(harness, "oneshot")
    assert o["ok"] == o["requests"]
    assert o["max_chunks"] == 1 and o["launches"] == o["requests"]


@pytest.mark.parametrize("where", ["fail_enqueue", "fail_poll", "fail_upload"])
def test_failures_stay_with_their_requests(harness, where):
    o = _run(harness, where)
    assert o["poisoned"] > 0
    assert o["failed"] == o["poisoned"] and o["poisoned_ok"] == 0
    assert o["innocent_failed"] == 0
    assert o["ok"] == o["requests"] - o["poisoned"]
    if where != "fail_upload":
        assert o["retried"] >= o["poisoned"]


def test_cancellation(harness):
    o = _run(harness, "cancel")
    assert o["cancelled"] > 0
    assert o["ok"] + o["cancelled"] == o["requests"]


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_randomized_mix(harness, seed):
    o = _run(harness, "random", seed)
    assert o["innocent_failed"] == 0 and o["poisoned_ok"] == 0
    assert o["ok"] + o["failed"] + o["cancelled"] + o["rejected"] == o["requests"]
    assert o["max_waiting"] > 0
