"""Pins of the pose-to-skinning-matrix oracle (forward kinematics of the
axis-angle pose, the quantity pose optimisation differentiates): Rodrigues
against the matrix exponential, the rest pose, a rigid root rotation, the
synthetic skeleton's own matrices, and finite differences."""

import math

import numpy as np
import scipy.linalg
import torch

from oracle import ref64
from paper_2407_10707_amd import synth


def test_rodrigues_is_the_matrix_exponential():
    rng = np.random.default_rng(1)
    th = rng.normal(size=(6, 3))
    th[0] = 0.0
    th[1] = [1e-8, 0, 0]
    R = ref64.rodrigues(th).numpy()
    for k in range(6):
        Kx = np.array([[0, -th[k, 2], th[k, 1]], [th[k, 2], 0, -th[k, 0]],
                       [-th[k, 1], th[k, 0], 0]])
        assert np.allclose(R[k], scipy.linalg.expm(Kx), atol=1e-13)


def test_rest_pose_and_rigid_root_rotation():
    J = len(synth.PARENTS)
    S = ref64.pose_to_skin(np.zeros(3 * J), synth.JOINTS_REST, synth.PARENTS).numpy()
    want = np.zeros((J, 12))
    want[:, [0, 5, 10]] = 1.0
    assert np.allclose(S, want, atol=1e-15)
    th = np.zeros(3 * J)
    th[:3] = [0.0, 0.0, math.pi / 2]
    S = ref64.pose_to_skin(th, synth.JOINTS_REST, synth.PARENTS).numpy().reshape(J, 3, 4)
    Rz = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1.0]])
    root = synth.JOINTS_REST[0]
    for j in range(J):                 # every joint moves with the root
        assert np.allclose(S[j, :, :3], Rz, atol=1e-15)
        assert np.allclose(S[j, :, 3], root - Rz @ root, atol=1e-15)


def test_matches_the_skeletons_own_matrices():
    rng = np.random.default_rng(2)
    th = rng.normal(0.0, 0.3, (len(synth.PARENTS), 3))
    R = ref64.rodrigues(th).numpy()
    want = synth.skinning_matrices(R).reshape(-1, 12)
    got = ref64.pose_to_skin(th.reshape(-1), synth.JOINTS_REST, synth.PARENTS).numpy()
    assert np.allclose(got, want, atol=1e-13)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    J = len(synth.PARENTS)
    th0 = rng.normal(0.0, 0.3, 3 * J)
    th0[3:6] = 0.0                      # a joint at the rest pose
    C = rng.normal(size=(J, 12))
    th = torch.tensor(th0, requires_grad=True)
    (g,) = torch.autograd.grad((ref64.pose_to_skin(th, synth.JOINTS_REST, synth.PARENTS) *
                                torch.tensor(C)).sum(), (th,))
    for k in [0, 4, 5, 17, 40, 71]:
        e = np.zeros_like(th0)
        e[k] = 1e-6
        f = lambda v: float((ref64.pose_to_skin(v, synth.JOINTS_REST, synth.PARENTS).numpy() * C).sum())
        fd = (f(th0 + e) - f(th0 - e)) / 2e-6
        assert abs(fd - float(g[k])) < 1e-6 * max(1.0, abs(fd))
