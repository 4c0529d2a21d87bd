"""Race and ordering checks of the supernodal schedule on the host (no GPU): tests/sched_sim.cpp
replays every launch of the refactorization sweep and of the sparse L and U solves from the
schedule records as the memory accesses of its workgroups (their kernels' reads and writes of
factor entries, solution rows and the scratch blocks of split supernodes).

- exact mode, on every circuit and knob setting: no word is written by two units of one launch
  or read by one while another writes it (a split supernode's units against its last part
  excepted), a panel touches only its own columns, an update only reads columns finalised by
  an earlier launch and writes only its target, a solve reads only final rows, and every
  column and row is finalised exactly once; the same under AddressSanitizer and UBSan;
- threads mode under ThreadSanitizer: the launches' units on eight threads, split supernodes
  meeting through an arrival counter as the kernels' do (Section IV-B's concern that a thread
  never waits on work that has not been ordered before it, here within one launch);
- the checks are not blind: mistakes planted in the simulated launches (two sweep levels
  swapped, two solve levels merged, a split supernode finished without its counter) fail.
"""
import os
import subprocess

import pytest

from helpers import SCHEDULE_CASES as CASES, SCHEDULE_KNOBS as KNOBS, build_host_tool, write_csc_binary


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    return build_host_tool(tmp_path_factory, "sched_sim.cpp")


@pytest.fixture(scope="module")
def sim_asan(tmp_path_factory):
    return build_host_tool(tmp_path_factory, "sched_sim.cpp", ("-fsanitize=address,undefined",), "_asan")


@pytest.fixture(scope="module")
def sim_tsan(tmp_path_factory):
    return build_host_tool(tmp_path_factory, "sched_sim.cpp", ("-fsanitize=thread",), "_tsan")


@pytest.fixture(scope="module")
def matrices(tmp_path_factory):
    d = tmp_path_factory.mktemp("circuits")
    out = {}
    for name, make in CASES.items():
        out[name] = str(d / (name + ".bin"))
        write_csc_binary(out[name], make())
    return out


def _run(exe, path, knobs, mode, extra=(), env=None):
    return subprocess.run([exe, path, *[str(v) for v in knobs], mode, *[str(v) for v in extra]],
                          capture_output=True, text=True, timeout=600, env=env)


def _tsan_env():
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1 exitcode=66"
    return env


def _skip_if_tsan_cannot_run(r):
    if "ThreadSanitizer" in r.stderr and "data race" not in r.stderr:
        pytest.skip("ThreadSanitizer cannot run here: " + r.stderr[-300:])


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("knobs", KNOBS, ids=lambda k: "tail%d_split%d_rows%d" % k)
def test_launches_race_free_and_ordered(sim, matrices, name, knobs):
    r = _run(sim, matrices[name], knobs, "exact")
    assert r.returncode == 0 and r.stdout.startswith("OK"), (r.stdout + r.stderr)[-4000:]


def test_launches_under_address_sanitizer(sim_asan, matrices):
    r = _run(sim_asan, matrices["power_grid_200x200"], KNOBS[1], "exact")
    assert r.returncode == 0 and r.stdout.startswith("OK"), (r.stdout + r.stderr)[-4000:]


@pytest.mark.parametrize("stride", [1, 8])
@pytest.mark.parametrize("name,knobs", [("power_grid_200x200", KNOBS[0]), ("mesh_transistor_50x50", KNOBS[1])])
def test_launches_under_thread_sanitizer(sim_tsan, matrices, name, knobs, stride):
    r = _run(sim_tsan, matrices[name], knobs, "threads", (8, stride, 0), _tsan_env())
    _skip_if_tsan_cannot_run(r)
    assert r.returncode == 0 and r.stdout.startswith("OK") and "ThreadSanitizer" not in r.stderr, \
        (r.stdout + r.stderr)[-4000:]


@pytest.mark.parametrize("plant,expect", [(1, "an update touches a finalised column"),
                                          (2, "reads a row not yet final")])
def test_planted_ordering_mistakes_fail(sim, matrices, plant, expect):
    r = _run(sim, matrices["power_grid_200x200"], KNOBS[0], "exact", (8, 1, plant))
    assert r.returncode == 1 and r.stdout.startswith("FAIL") and expect in r.stdout, r.stdout[-2000:]


def test_planted_race_is_seen_by_thread_sanitizer(sim_tsan, matrices):
    r = _run(sim_tsan, matrices["power_grid_200x200"], KNOBS[1], "threads", (8, 1, 3), _tsan_env())
    _skip_if_tsan_cannot_run(r)
    assert r.returncode == 66 and "data race" in r.stderr, (r.stdout + r.stderr)[-2000:]
