"""Pins of the densification oracle (App. B, Alg. 1): the random-number
generator against its published reference outputs, the vertex counts and
triangle densities of a hand-counted mesh, the number of added Gaussians,
no addition where every triangle is dense enough, multinomial counts whose
frequencies follow P / sum(P), and placements inside their triangles with
uniform barycentric statistics."""

import math
import os

import numpy as np
import pytest

from oracle import cpu
from paper_2407_10707_amd import synth
from tests.conftest import scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_outputs():
    rows = [line.split() for line in open(os.path.join(GOLDEN, "splitmix64.txt"))
            if line.strip() and not line.startswith("#")]
    assert len(rows) >= 4
    for seed, k, out in rows:
        assert cpu.splitmix64(int(seed), int(k)) == int(out)


def _quad():
    """Two triangles sharing the edge 1-2 of a unit square in the z = 0 plane."""
    verts = np.array([[0.0, 1.0, 0.0, 1.0], [0.0, 0.0, 1.0, 1.0], [0.0, 0.0, 0.0, 0.0]],
                     np.float32)
    faces = np.array([[0, 1, 2], [1, 3, 2]], np.int32)
    return verts, faces


def test_hand_counted_mesh():
    """K_g = 2, four Gaussians with nearest-vertex sets {0,1}, {0,2}, {0,1},
    {3,1}: D_v = (3, 3, 1, 1); d_f = (3+3+1)/12 = 7/12 and (3+1+1)/12 = 5/12;
    P = (5/12, 7/12), sum P = 1, so p0 = 0.02 adds floor(0.02) = 0 Gaussians
    and p0 = 30 adds 30."""
    verts, faces = _quad()
    sg = np.array([[0, 0, 0, 3], [1, 2, 1, 1]], np.int32)
    r = cpu.densify(sg, verts, faces, d0=1.0, p0=0.02, seed=1)
    assert r["Dv"].tolist() == [3, 3, 1, 1]
    assert r["df"].tolist() == [np.float32(7 / 12), np.float32(5 / 12)]
    assert r["n_added"] == 0 and r["ng"].tolist() == [0, 0]
    r = cpu.densify(sg, verts, faces, d0=1.0, p0=30.0, seed=1, cap=64)
    assert r["n_added"] == 30 and int(r["ng"].sum()) == 30
    assert np.array_equal(np.bincount(r["face"], minlength=2), r["ng"])


def test_dense_mesh_gets_no_gaussians():
    """Every triangle's density at or above d0: P = 0 everywhere, nothing is
    added whatever p0; lowering d0 below the smallest density does the
    same, raising it above gives additions."""
    s = scene(2)
    faces = s["faces"]
    r = cpu.densify(s["vidx"], s["verts"], faces, d0=1.0, p0=0.02, seed=3)
    dmin = float(r["df"].min())
    assert dmin > 0
    r0 = cpu.densify(s["vidx"], s["verts"], faces, d0=dmin * 0.999, p0=50.0, seed=3)
    assert r0["n_added"] == 0 and not r0["ng"].any()
    r1 = cpu.densify(s["vidx"], s["verts"], faces, d0=float(r["df"].max()) * 1.5, p0=0.02,
                     seed=3)
    assert r1["n_added"] > 0


def test_count_and_zero_probability_triangles():
    """N' = floor(sum(P) p0), the counts add up to N', and triangles with
    P = 0 receive nothing (the avatar workload's mesh and Gaussians, with a
    threshold that leaves about half the triangles dense enough)."""
    s = scene(2)
    base = cpu.densify(s["vidx"], s["verts"], s["faces"], seed=0)
    d0 = float(np.median(base["df"]))
    r = cpu.densify(s["vidx"], s["verts"], s["faces"], d0=d0, p0=0.5, seed=5,
                    cap=len(s["faces"]) * 4)
    P = np.maximum(0.0, d0 - base["df"].astype(np.float64))
    want = math.floor(P.sum() * 0.5)
    assert abs(r["n_added"] - want) <= 1           # P held to 2^-16 / (6 K_g)
    assert int(r["ng"].sum()) == r["n_added"]
    assert not r["ng"][P == 0].any()
    assert np.array_equal(np.bincount(r["face"], minlength=len(P)), r["ng"])


def test_multinomial_frequencies_follow_P():
    """About 200k draws over the avatar mesh: the counts of 20 groups of
    triangles (by quantile of P) against N' P_group / sum(P), chi-square
    with 19 degrees of freedom below 50 (p ~ 1e-4)."""
    s = scene(2)
    base = cpu.densify(s["vidx"], s["verts"], s["faces"], seed=0)
    d0 = float(np.quantile(base["df"], 0.7))
    P = np.maximum(0.0, d0 - base["df"].astype(np.float64))
    p0 = 2e5 / P.sum()
    r = cpu.densify(s["vidx"], s["verts"], s["faces"], d0=d0, p0=p0, seed=11, cap=1)
    N = r["n_added"]
    assert N > 150000
    live = np.nonzero(P > 0)[0]
    order = live[np.argsort(P[live], kind="stable")]
    chi2 = 0.0
    for grp in np.array_split(order, 20):
        exp = N * P[grp].sum() / P.sum()
        chi2 += (r["ng"][grp].sum() - exp) ** 2 / exp
    assert chi2 < 50.0, chi2


def test_placements_lie_in_their_triangles_uniformly():
    verts, faces = synth.body_mesh(12, 6)
    verts = np.ascontiguousarray(verts.T, np.float32)
    faces = np.ascontiguousarray(faces, np.int32)
    sg = np.zeros((3, 0), np.int32)                   # no Gaussians: P = d0 everywhere
    r = cpu.densify(sg, verts, faces, d0=1.0, p0=20.0, seed=9, cap=1 << 20)
    N = r["n_added"]
    assert N == 20 * len(faces)
    x = r["x"].astype(np.float64)
    f = faces[r["face"]]
    a, b, c = (verts[:, f[:, k]].astype(np.float64) for k in range(3))
    e1, e2, q = b - a, c - a, x - a
    d11, d12, d22 = (e1 * e1).sum(0), (e1 * e2).sum(0), (e2 * e2).sum(0)
    q1, q2 = (q * e1).sum(0), (q * e2).sum(0)
    den = d11 * d22 - d12 * d12
    b1 = (d22 * q1 - d12 * q2) / den
    b2 = (d11 * q2 - d12 * q1) / den
    b0 = 1 - b1 - b2
    resid = q - b1 * e1 - b2 * e2
    assert np.abs(resid).max() < 1e-5
    for bb in (b0, b1, b2):
        assert bb.min() > -1e-4 and bb.max() < 1 + 1e-4
        assert abs(bb.mean() - 1 / 3) < 0.01
    # the corner region b0 > 1/2 holds a quarter of a uniform triangle's area
    assert abs((b0 > 0.5).mean() - 0.25) < 0.01
