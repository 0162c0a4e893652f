"""Host emulations of two protocols whose failures hang rather than fail
(no GPU): the persistent kernels' work list (claim in order, wait for the
job's previous pass, publish; the watchdog's expiry path) and the serving
loop's admission wait. Both programs compile the library's own protocol
headers (worklist.hpp, server_admission.hpp) for the host; threads stand in
for workgroups and for the server's scheduler, collector and submitter."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2305_07390_amd", "csrc")


@pytest.fixture(scope="module")
def programs(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("host_protocols")
    built = {}
    for name in ("worklist_emu", "admission_emu"):
        exe = str(out / name)
        subprocess.run([hipcc, "-std=c++17", "-O1", "-pthread", "-I", CSRC,
                        os.path.join(HERE, "host", name + ".cpp"), "-o", exe],
                       check=True, capture_output=True, timeout=300)
        built[name] = exe
    return built


def _run(exe, *args, timeout=60):
    p = subprocess.run([exe, *args], capture_output=True, text=True, timeout=timeout)
    line = [l for l in p.stdout.splitlines() if l.startswith("result")]
    return p.returncode, (line[-1] if line else p.stdout + p.stderr)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_worklist_runs_every_item_after_its_previous_pass(programs, seed):
    rc, line = _run(programs["worklist_emu"], "ok", str(seed))
    assert rc == 0, line
    assert "violations=0" in line and "status=0" in line and "complete=1" in line


@pytest.mark.parametrize("seed", [1, 2])
def test_worklist_held_back_workgroup_trips_the_watchdog(programs, seed):
    # a workgroup holds an early item without publishing: the waits behind it
    # expire, the rest of the launch drains, and the report is a timeout
    rc, line = _run(programs["worklist_emu"], "held", str(seed))
    assert rc == 0, line
    assert "err=1" in line and "status=-7" in line and "complete=0" in line  # STENCIL_ERR_TIMEOUT


def test_admission_wait_makes_progress(programs):
    rc, line = _run(programs["admission_emu"], "fixed")
    assert rc == 0, line


def test_admission_wait_on_a_nonempty_queue_livelocks(programs):
    # the predicate the server's scheduler must not use: the emulation detects
    # the live-lock (no collection for 2 s) instead of hanging
    rc, line = _run(programs["admission_emu"], "queue")
    assert rc == 2, line
