"""Host checks of the supernodal schedule (no GPU): the records the sweep and solve kernels
index without bounds checks are rebuilt from the factor on the CPU and checked one by one by
tests/schedule_check.cpp, compiled here against the in-tree library.

What is checked, per level of the sweep (Section IV's right-looking supernodal update):
singletons, small and wide panels in their ranges; panel units covering every panel once and
carrying their supernode's record; every update item's suffix at consecutive slots of its
target column holding the source's rows, and its map sending R's rows to the same rows of the
target (rows below the dense tail only, for a dense target); within a task, suffix slots
distinct and never a slot of any item's rows of R, and each item's rows of R on distinct
slots (what lets the suffix solves go first and a pass load its target values up front);
heavy groups covering each of their tasks' items exactly once with the sources ascending.  Per level of the L and U solves:
the singletons left out of the L launches pull nothing, and the runs of every workgroup
supernode hold exactly its entries outside the diagonal block, each at a position that holds
its row.
"""
import subprocess

import pytest

from helpers import SCHEDULE_CASES as CASES, SCHEDULE_KNOBS as KNOBS, build_host_tool, write_csc_binary


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    return build_host_tool(tmp_path_factory, "schedule_check.cpp")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("knobs", KNOBS, ids=lambda k: "tail%d_split%d_rows%d" % k)
def test_schedule_records(checker, tmp_path, name, knobs):
    c = CASES[name]()
    path = str(tmp_path / (name + ".bin"))
    write_csc_binary(path, c)
    r = subprocess.run([checker, path] + [str(v) for v in knobs], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("OK"), (r.stdout + r.stderr)[-4000:]
    st = dict((k, int(v)) for k, v in (f.split("=") for f in r.stdout.split()[1:]))
    # the checks were not vacuous: every case has tiny update items and L singletons left out
    # of the launches; the tail setting decides the dense targets; the power grid has heavy
    # groups and solve supernodes pulled by several units
    assert st["tiny_items"] > 0 and st["lskip"] > 0
    if knobs[0] == -1:
        assert st["T"] == st["n"] and st["dense_items"] == 0
    elif st["T"] < st["n"]:
        assert st["dense_items"] > 0
    if knobs[2] == 16:
        assert st["split_panels"] > 0          # panels over 16 rows below the block are split
    if name.startswith("power_grid"):
        assert st["groups"] > 0 and st["split_solves"] > 0 and st["runs"] > 0
