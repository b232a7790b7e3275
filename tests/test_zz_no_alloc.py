"""mesh_visibility_noalloc (the visibility entry point that allocates
nothing: its workspace is the library's fixed device array) against
mesh_visibility with a caller workspace, bit-exact, on two calls in a row,
the second with a smaller input; sizes beyond the array are refused before
any launch."""

import numpy as np
import pytest
import torch

from oracle import cpu
from paper_2407_10707_amd import rga
from tests.conftest import scene

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _inputs(s):
    vx, _, _ = cpu.lbs_f32(s["skin"], s["mesh_jidx"], s["mesh_jw"], s["verts"])
    return dev(vx), dev(s["faces"]), dev(s["view_dirs"]), s["vis_res"], dev(s["knn_v"])


def test_noalloc_matches_workspace_entry_point_on_two_calls():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    big = scene(2, n_gauss=1000)     # 6,840 vertices, 512 views at 128^2
    small = scene(1)                 # about 500 vertices, 64 views at 64^2
    ib, is_ = _inputs(big), _inputs(small)
    nv_b, V_b = ib[0].shape[1], ib[2].shape[0]
    nv_s, V_s = is_[0].shape[1], is_[2].shape[0]
    assert nv_s < nv_b and V_s < V_b
    assert rga.lib().mesh_visibility_workspace(nv_b, V_b) <= rga.lib().mesh_visibility_noalloc_limit()
    # outputs allocated up front, so the two no-alloc calls allocate nothing
    cb = torch.empty((nv_b, V_b), dtype=torch.uint8, device="cuda")
    rb = torch.empty((nv_b, (V_b + 31) // 32), dtype=torch.int32, device="cuda")
    cs = torch.empty((nv_s, V_s), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    print(f"[noalloc] call 1: nv={nv_b} V={V_b} res={ib[3]}", flush=True)
    rga.mesh_visibility_noalloc(*ib, count=cb, raw=rb)
    print(f"[noalloc] call 2: nv={nv_s} V={V_s} res={is_[3]} (no raw bits)", flush=True)
    rga.mesh_visibility_noalloc(*is_, count=cs)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    ecb, erb = rga.mesh_visibility(*ib, want_raw=True)
    ecs, _ = rga.mesh_visibility(*is_)
    assert np.array_equal(host(rb), host(erb))
    assert np.array_equal(host(cb), host(ecb))
    assert np.array_equal(host(cs), host(ecs))
    # and the small case against the oracle itself
    s = small
    vx, _, _ = cpu.lbs_f32(s["skin"], s["mesh_jidx"], s["mesh_jw"], s["verts"])
    _, ecnt = cpu.mesh_visibility(vx, s["faces"], s["view_dirs"], s["vis_res"], s["knn_v"])
    assert np.array_equal(host(cs), ecnt)


def test_noalloc_refuses_sizes_beyond_its_array():
    L = rga.lib()
    limit = L.mesh_visibility_noalloc_limit()
    nv, V = 200000, 2048
    assert L.mesh_visibility_workspace(nv, V) > limit
    # refused on the host before any pointer is read or kernel launched
    rc = L.mesh_visibility_noalloc(None, nv, 10, None, None, V, None, 128, None, 19, None, None)
    assert rc == -2
    assert "scratch" in rga.last_error()
