"""The C ABI library loads and exports every entry point include/rga.h
declares; host-only behaviour (workspace sizing, argument validation before
any launch) is checked without a GPU."""

import ctypes as C
import os
import re

import pytest

from paper_2407_10707_amd import rga

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rga.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 18, names
    L = rga.lib()
    for name in names:
        assert hasattr(L, name), f"{name} declared in rga.h but not exported"
    for name in names:
        assert name in rga._SIGS, f"{name} has no ctypes signature in the binding"


def test_abi_version_and_error_string():
    L = rga.lib()
    assert L.rga_abi_version() == 3
    assert isinstance(L.rga_last_error(), bytes)


def test_workspace_sizes_are_monotone():
    L = rga.lib()
    a = L.splat_workspace_size(100000, 512, 512, 1 << 20)
    b = L.splat_workspace_size(100000, 512, 512, 1 << 21)
    assert 0 < a < b
    assert L.splat_workspace_size(-1, 512, 512, 10) == 0
    assert L.mesh_visibility_workspace(6840, 512) > 6840 * 512 // 8
    assert L.shade_gaussians_workspace(100000, 16, 32) > 0
    assert L.l1_loss_workspace(3 * 512 * 512) > 0
    assert L.knn_workspace(6840) > 6840 * 16
    assert 0 < L.mlp_workspace(100) < L.mlp_workspace(10000)
    assert L.image_loss_workspace(3, 512, 512) >= 3 * 3 * 512 * 512 * 4
    assert L.image_loss_workspace(0, 512, 512) == 0
    assert L.mlp_workspace(-1) == 0


def test_argument_errors_are_reported_before_any_launch():
    L = rga.lib()
    assert L.lbs_skin(None, 10, 0, None, None, None, None, None, None, None, None, None) == -1
    assert "n_joints" in rga.last_error()
    assert L.lbs_skin(None, 0, 24, None, None, None, None, None, None, None, None, None) == 0
    assert L.pose_to_skin_backward(None, 0, None, None, None, None, None, 1) == -1
    assert L.mesh_visibility(None, 10, 10, None, None, 8, None, 256, None, 19, None, None, None, 0) == -4
    assert "res" in rga.last_error()
    assert L.mesh_visibility(None, 10, 10, None, None, 8, None, 64, None, 18, None, None, None, 0) == -1
    cam = rga.Camera()
    cam.width, cam.height = 0, 10
    assert L.splat_forward(None, 10, C.byref(cam), None, None, None, None, None, None, None, None,
                           0, 100, None, None) == -1
    assert "image size" in rga.last_error()
    cp = (C.c_float * 3)(0, 0, 3)
    assert L.shade_gaussians(None, 10, None, None, None, None, None, None, None, None, 7000, 19,
                             16, 32, 5, 32, None, C.cast(cp, C.c_void_p), 0, None, None, None,
                             0) == -1
    assert "divide" in rga.last_error()
    assert L.l1_loss(None, 0, None, None, None, None, None, 0) == -1
    assert L.knn_query(None, 10, None, 5, 6, None, None, None, 0, None, 0) == -1
    assert "k must be" in rga.last_error()
    assert L.knn_query(None, 10, None, 5, 0, None, None, None, 0, None, 0) == -1
    assert L.knn_query_workspace(1000) >= 3 * 4000
    assert L.knn_build(None, 0, None, None, 0) == -1
    assert L.knn_interpolate(None, 10, 33, None, None, 3, 5, None, None) == -1
    assert L.knn_interpolate_backward(None, 10, 3, None, None, 3, 5, None, None) == -1
    assert L.regularisers(None, 0, 10, 19, 3, *([None] * 7), 0.005, 0.002, 0.1, 0.02, 10.0,
                          *([None] * 5), 0, None, None, 0) == -1
    assert L.regularisers(None, 10, 10, 19, 3, *([None] * 7), 0.005, 0.002, 0.1, 0.02, 10.0,
                          *([None] * 5), 1, None, None, 0) == -1
    assert "kv" in rga.last_error()
    assert L.mesh_visibility_shadowmap(None, 10, 10, None, None, 8, None, 64, None, 19, -1.0,
                                       None, None, None, 0) == -1
    assert "bias_px" in rga.last_error()
    assert L.adam_step(None, 10, None, None, None, None, 1e-3, 0.9, 0.999, 1e-8, 0) == -1
    assert L.adam_step(None, 10, None, None, None, None, 1e-3, 1.0, 0.999, 1e-8, 1) == -1
    assert L.image_loss(None, 3, 0, 8, None, None, 0.2, None, None, None, 0) == -1
    assert L.image_loss(None, 3, 8, 8, None, None, 1.5, None, None, None, 0) == -1
    assert "lambda" in rga.last_error()
    assert L.mlp_forward(None, -1, None, None, None, None, None, 0, None) == -1
    assert L.mlp_forward(None, 10, None, None, None, None, None, 0, None) == -1
    assert "null" in rga.last_error()
    fake = C.c_void_p(16)   # never dereferenced: the size check fails first
    assert L.mlp_forward(None, 10, fake, fake, fake, fake, fake, 16, fake) == -2
    assert "workspace" in rga.last_error()
    assert L.mlp_backward(None, 10, fake, fake, fake, fake, fake, fake, 16, fake, None) == -1
