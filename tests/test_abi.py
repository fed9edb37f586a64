"""The C-ABI library loads and exports every entry point that include/gmapp.h
declares; without a device, context creation reports GMAPP_EDEVICE.  No compute
call is made here (these run on the CPU-only host)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmapp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gmapp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("gmapp_create", "gmapp_destroy", "gmapp_last_error", "gmapp_rollout", "gmapp_force_probe"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2606_12579_amd import gmapp
    lib = gmapp.load_library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", gmapp.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\b(gmapp_[a-z0-9_]+)\b", out))
    assert set(declared_functions()) <= exported


def test_version_and_no_device_error():
    import torch
    from paper_2606_12579_amd import gmapp
    lib = gmapp.load_library()
    assert lib.gmapp_version().startswith(b"gmapp")
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    assert lib.gmapp_create(0, 0, ctypes.byref(h)) == gmapp.EDEVICE
    assert lib.gmapp_create(0, 0, None) == gmapp.EINVAL
    lib.gmapp_destroy(None)                       # NULL is accepted
    assert lib.gmapp_last_error(None) == b"no context"


def test_struct_layouts_match_header():
    """ctypes mirrors of the C structs have the sizes the C compiler gives them."""
    from paper_2606_12579_amd import gmapp
    src = r'''
#include <stdio.h>
#include "gmapp.h"
#include <stddef.h>
int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %d\n", sizeof(gmapp_scene),
 sizeof(gmapp_agents), sizeof(gmapp_query), sizeof(gmapp_params), sizeof(gmapp_outputs), sizeof(gmapp_tiling),
 sizeof(gmapp_job), sizeof(gmapp_batch_tuning), sizeof(gmapp_server_config), sizeof(gmapp_request),
 sizeof(gmapp_completion), sizeof(gmapp_server_stats), sizeof(gmapp_loop_config), sizeof(gmapp_loop_outputs),
 sizeof(gmapp_pose_agents), sizeof(gmapp_pose_query), sizeof(gmapp_arm),
 offsetof(gmapp_job, state), offsetof(gmapp_job, k_end),
 offsetof(gmapp_request, deadline_s), offsetof(gmapp_agents, heuristic), GMAPP_STATE_FLOATS);
 return 0;}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "s")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        sizes = [int(x) for x in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    mine = [ctypes.sizeof(s) for s in (gmapp.Scene, gmapp.Agents, gmapp.Query, gmapp.Params, gmapp.Outputs,
                                       gmapp.Tiling, gmapp.Job, gmapp.BatchTuning, gmapp.ServerConfig,
                                       gmapp.Request, gmapp.Completion, gmapp.ServerStats, gmapp.LoopConfig,
                                       gmapp.LoopOutputs, gmapp.PoseAgents, gmapp.PoseQuery, gmapp.Arm)]
    mine += [gmapp.Job.state.offset, gmapp.Job.k_end.offset, gmapp.Request.deadline_s.offset,
             gmapp.Agents.heuristic.offset, gmapp.STATE_FLOATS]
    assert sizes == mine


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and a message, before any
    device is touched."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
