"""Host checks of the supernodal schedule (no GPU): the records the sweep and solve kernels
index without bounds checks are rebuilt from the factor on the CPU and checked one by one by
tests/schedule_check.cpp, compiled here against the in-tree library.

What is checked, per level of the sweep (Section IV's right-looking supernodal update):
singletons, small and wide panels in their ranges; panel units covering every panel once and
carrying their supernode's record; every update item's suffix at consecutive slots of its
target column holding the source's rows, and its map sending R's rows to the same rows of the
target (rows below the dense tail only, for a dense target); heavy groups covering each of
their tasks' items exactly once with the sources ascending.  Per level of the L and U solves:
the singletons left out of the L launches pull nothing, and the runs of every workgroup
supernode hold exactly its entries outside the diagonal block, each at a position that holds
its row.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import mnagen
import paper_2411_14082_amd as ck

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2411_14082_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("g++ or the HIP headers are not available")
    if not os.path.exists(ck.LIB_PATH):
        pytest.skip("libcktlu.so is not built")
    out = str(tmp_path_factory.mktemp("schedcheck") / "schedule_check")
    libdir = os.path.dirname(ck.LIB_PATH)
    cmd = ["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, os.path.join(HERE, "schedule_check.cpp"),
           "-o", out, "-L" + libdir, "-l:libcktlu.so", "-Wl,-rpath," + libdir,
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _write(path, c):
    with open(path, "wb") as f:
        np.array([c.n], dtype=np.int32).tofile(f)
        np.array([c.nnz], dtype=np.int64).tofile(f)
        np.asarray(c.colptr, dtype=np.int32).tofile(f)
        np.asarray(c.rowind, dtype=np.int32).tofile(f)
        np.asarray(c.values, dtype=np.float64).tofile(f)


CASES = {
    "power_grid_200x200": lambda: mnagen.power_grid(200, 200, n_src=200, nrhs=1, seed=3),
    "mesh_transistor_50x50": lambda: mnagen.mesh_transistor(50, 50, seed=5),
    "layered_rc_3x24x24": lambda: mnagen.layered_rc(24, 24, 3, seed=7),
    "mesh_vsrc_30x30": lambda: mnagen.mesh_vsrc(30, 30, n_vsrc=6, seed=2),
}

# (dense_tail_size, solve_split_entries, sweep_panel_rows): the defaults; a dense tail of 256
# with small solve units (several units per supernode) and split panels; no dense tail
KNOBS = [(0, 0, 0), (256, 64, 16), (-1, 256, 64)]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("knobs", KNOBS, ids=lambda k: "tail%d_split%d_rows%d" % k)
def test_schedule_records(checker, tmp_path, name, knobs):
    c = CASES[name]()
    path = str(tmp_path / (name + ".bin"))
    _write(path, c)
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
