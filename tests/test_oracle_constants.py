"""The oracle and the synthetic workloads use the numbers the paper prints
for the hot path (tests/golden/paper_constants.txt, each with its passage):
the 16 x 32 light probe of 512 lights, K_g and K_v, and the constants of the
App. A BRDF.  A mistyped digit in the oracle's Fresnel or Smith term, or a
workload with the wrong probe or neighbour counts, fails here."""

import math
import os

import numpy as np
import torch

from oracle import ref64
from paper_2407_10707_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def _constants():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, value = line.split()[:2]
        out[name] = float(value)
    return out


def test_probe_and_neighbour_counts():
    c = _constants()
    cfg = synth.CONFIGS[2]               # the avatar workload: the paper's probe
    assert (cfg.he, cfg.we) == (c["env_rows"], c["env_cols"])
    assert cfg.he * cfg.we == c["num_lights"]
    assert cfg.hv * cfg.wv == c["vis_directions"]
    for cfg in synth.CONFIGS.values():
        assert cfg.kg == c["knn_gaussian"] and cfg.kv == c["knn_vertex"]


def test_oracle_fresnel_uses_printed_constants():
    c = _constants()
    assert ref64.F0 == c["fresnel_f0"]
    for oh in (0.0, 0.25, 0.5, 0.8, 1.0):
        want = c["fresnel_f0"] + (1 - c["fresnel_f0"]) * 2.0 ** (
            (c["fresnel_c1"] * oh + c["fresnel_c2"]) * oh)
        got = float(ref64.fresnel(torch.tensor(oh, dtype=torch.float64)))
        assert abs(got - want) <= 1e-15 * want


def test_oracle_brdf_uses_printed_smith_k():
    """Specular lobe at n = w_o, n.w_i = 0.5 against the App. A terms built
    from the printed constants (G1 depends on k only off normal incidence)."""
    c = _constants()
    n = torch.tensor([0.0, 1.0, 0.0], dtype=torch.float64)
    wo = n.clone()
    wi = torch.tensor([math.sqrt(0.75), 0.5, 0.0], dtype=torch.float64)
    for gamma in (0.2, 0.5, 0.9):
        R = ref64.brdf(wi, wo, n, torch.zeros(3, dtype=torch.float64), torch.tensor(gamma,
                       dtype=torch.float64), torch.tensor(1.0, dtype=torch.float64))
        h = (wi + wo) / torch.linalg.norm(wi + wo)
        nh, oh, ci, co = float(n @ h), float(wo @ h), 0.5, 1.0
        a2 = gamma ** 4
        D = a2 / (math.pi * (nh * nh * (a2 - 1) + 1) ** 2)
        F = c["fresnel_f0"] + (1 - c["fresnel_f0"]) * 2.0 ** (
            (c["fresnel_c1"] * oh + c["fresnel_c2"]) * oh)
        k = (gamma + 1) ** 2 / c["smith_k_div"]
        g1 = lambda x: x / (x * (1 - k) + k)
        want = D * F * g1(ci) * g1(co) / (4 * ci * co)
        assert np.allclose(R.numpy(), want, rtol=1e-13, atol=0)


def test_training_loss_and_network_constants():
    """The loss weights, the scale threshold and the network's shape of the
    training section and the implementation details."""
    import inspect
    c = _constants()
    assert ref64.REG_LAMBDAS == (c["lambda_smooth"], c["lambda_mdist"], c["lambda_disp"],
                                 c["lambda_scale"])
    assert ref64.REG_S0 == c["scale_s0"]
    assert inspect.signature(ref64.image_loss).parameters["lam"].default == c["lambda_img"]
    hidden = [s for s in ref64.MLP_SHAPES if s[0] == ref64.MLP_WIDTH]
    assert len(hidden) == c["mlp_layers"] and ref64.MLP_WIDTH == c["mlp_width"]
    assert ref64.MLP_POSE == c["pose_dim"] and ref64.MLP_SHAPES[0][1] == 2 * ref64.MLP_FREQS + 72


def test_densification_defaults_are_the_printed_ones():
    """App. B: d0 = 1, p0 = 0.02 are the oracle's defaults, and the density
    of a triangle divides its vertex sum by 6 K_g (six triangles per vertex):
    one Gaussian whose K_g = 3 nearest vertices are a lone triangle's gives
    d_f = 3 / (6 3)."""
    import inspect

    from oracle import cpu
    c = _constants()
    sig = inspect.signature(cpu.densify)
    assert sig.parameters["d0"].default == c["dens_d0"]
    assert sig.parameters["p0"].default == c["dens_p0"]
    verts = np.eye(3, dtype=np.float32)
    faces = np.array([[0, 1, 2]], np.int32)
    r = cpu.densify(np.array([[0], [1], [2]], np.int32), verts, faces)
    assert r["df"][0] == np.float32(3 / (c["dens_incidence"] * c["knn_gaussian"]))
