"""Pins of the FP64 shading oracle (Sec. 3.1 rendering equation, App. A BRDF)
against closed forms and textbook properties of its terms."""

import math

import numpy as np
import pytest
import torch
from scipy import integrate

from oracle import ref64

f64 = torch.float64


def _one(n_vec, cam_dir, albedo, rough, tint, he, we, env, kv=1, count_val=None, x=(0, 0, 0)):
    """Shade one Gaussian at x with normal n, camera 3 units along cam_dir."""
    n_vec = np.asarray(n_vec, float)
    cam = np.asarray(x, float) + 3.0 * np.asarray(cam_dir, float) / np.linalg.norm(cam_dir)
    K = he * we
    cnt = np.full((1, K), kv if count_val is None else count_val, np.uint8)
    col, Lo = ref64.shade(
        torch.tensor(np.asarray(x, float).reshape(3, 1)), torch.tensor(n_vec.reshape(3, 1)),
        torch.tensor(np.asarray(albedo, float).reshape(3, 1)), torch.tensor([float(rough)]),
        torch.tensor([float(tint)]), np.zeros((3, 1), np.int32),
        np.array([[1.0], [0.0], [0.0]]), cnt, kv, he, we, he, we, env, cam, np.array([1]))
    return col[:, 0].numpy(), Lo[:, 0].numpy()


def test_solid_angles_and_directions():
    for he, we in ((8, 16), (16, 32), (32, 64)):
        d, a = ref64.env_geometry(he, we)
        assert abs(a.sum().item() - 4 * math.pi) < 1e-12
        assert torch.allclose(torch.linalg.norm(d, dim=1), torch.ones(he * we, dtype=f64))
        assert torch.allclose((a[:, None] * d).sum(0), torch.zeros(3, dtype=f64), atol=1e-12)


def test_lambertian_white_environment_converges_to_albedo():
    """Uniform unit radiance, full visibility, no specular: L_o = (a/pi)
    * sum_k A_k max(0, w_k.n) -> a as the light grid is refined (the
    cosine-weighted hemisphere integral is pi)."""
    rng = np.random.default_rng(0)
    albedo = np.array([0.2, 0.5, 0.9])
    for trial in range(3):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        errs = []
        for he, we in ((8, 16), (16, 32), (64, 128)):
            env = np.ones((he * we, 3))
            _, Lo = _one(n, n, albedo, 0.5, 0.0, he, we, env)
            errs.append(np.abs(Lo - albedo).max())
        assert errs[2] < errs[0]
        assert errs[2] < 2e-3


def test_specular_at_normal_incidence_closed_form():
    """n = w_i = w_o: D = 1/(pi alpha^2), F = F0 + (1 - F0) 2^-12.53789, G = 1,
    so the lit texel contributes p E F / (4 pi alpha^2) (zero albedo)."""
    he, we = 8, 16
    d, area = ref64.env_geometry(he, we)
    k0 = 37
    n = d[k0].numpy()
    env = np.zeros((he * we, 3))
    env[k0] = [1.0, 2.0, 3.0]
    gamma, p = 0.6, 0.7
    _, Lo = _one(n, n, [0, 0, 0], gamma, p, he, we, env)
    alpha = gamma ** 2
    F = 0.04 + 0.96 * 2.0 ** (-5.55473 - 6.98316)
    want = p * env[k0] * area[k0].item() * F / (4 * math.pi * alpha ** 2)
    assert np.allclose(Lo, want, rtol=1e-12)


@pytest.mark.parametrize("alpha", [0.05, 0.2, 0.5, 0.9])
def test_ggx_distribution_is_normalised(alpha):
    """Projected-area normalisation of a microfacet NDF: int D(h) (n.h) dw = 1."""
    def f(th):
        c = torch.tensor(math.cos(th), dtype=f64)
        return float(ref64.ggx_d(c, alpha)) * math.cos(th) * math.sin(th) * 2 * math.pi
    val, _ = integrate.quad(f, 0, math.pi / 2, limit=400, points=[0.001, 0.01, 0.1])
    assert abs(val - 1.0) < 1e-6


def test_fresnel_spherical_gaussian_tracks_schlick():
    oh = torch.linspace(0, 1, 1001, dtype=f64)
    F = ref64.fresnel(oh)
    schlick = 0.04 + 0.96 * (1 - oh) ** 5
    assert (F - schlick).abs().max() < 0.01
    assert abs(F[0].item() - 1.0) < 1e-12          # grazing: total reflection
    assert abs(F[-1].item() - 0.04) < 2e-4          # normal incidence ~ F0


def test_smith_g1_limits():
    k = 0.3
    x = torch.tensor([0.0, 1.0], dtype=f64)
    g = ref64.smith_g1(x, k)
    assert g[0].item() == 0.0 and abs(g[1].item() - 1.0) < 1e-15


def test_brdf_reciprocity():
    rng = np.random.default_rng(1)
    for _ in range(20):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        wi, wo = rng.normal(size=3), rng.normal(size=3)
        wi = wi * np.sign(wi @ n) / np.linalg.norm(wi)
        wo = wo * np.sign(wo @ n) / np.linalg.norm(wo)
        t = lambda a: torch.tensor(a, dtype=f64)
        r1 = ref64.brdf(t(wi), t(wo), t(n), t([0.3, 0.4, 0.5]), 0.4, 0.8)
        r2 = ref64.brdf(t(wo), t(wi), t(n), t([0.3, 0.4, 0.5]), 0.4, 0.8)
        assert torch.allclose(r1, r2, rtol=1e-13)


def test_shade_is_the_rendering_equation_sum():
    """shade() equals the literal sum over lights of L A R v max(0, w.n)."""
    rng = np.random.default_rng(2)
    he, we = 4, 8
    d, area = ref64.env_geometry(he, we)
    env = np.exp(rng.normal(-1, 1, size=(he * we, 3)))
    kv = 19
    for _ in range(5):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        cd = n + 0.5 * rng.normal(size=3)
        alb = rng.random(3)
        gam, p = rng.uniform(0.2, 0.9), rng.random()
        cnt = rng.integers(0, kv + 1, size=he * we)
        cam = 3 * cd / np.linalg.norm(cd)
        col, Lo = ref64.shade(torch.zeros(3, 1, dtype=f64), torch.tensor(n.reshape(3, 1)),
                              torch.tensor(alb.reshape(3, 1)), torch.tensor([gam]),
                              torch.tensor([p]), np.zeros((3, 1), np.int32),
                              np.array([[1.0], [0.0], [0.0]]), cnt[None].astype(np.uint8), kv, he,
                              we, he, we, env, cam, np.array([1]))
        wo = torch.tensor(cam / np.linalg.norm(cam))
        nn = torch.tensor(n)
        want = torch.zeros(3, dtype=f64)
        for k in range(he * we):
            c = float(d[k] @ nn)
            if c <= 0 or cnt[k] == 0:
                continue
            R = ref64.brdf(d[k], wo, nn, torch.tensor(alb), gam, p)
            want += torch.tensor(env[k]) * area[k] * R * (cnt[k] / kv) * c
        assert torch.allclose(Lo[:, 0], want, rtol=1e-10)
        assert torch.allclose(col[:, 0], ref64.srgb_oetf(want), rtol=1e-10)


def test_zero_visibility_and_back_facing_give_black():
    he, we = 4, 8
    env = np.ones((he * we, 3))
    n = np.array([0, 0, 1.0])
    _, Lo = _one(n, n, [1, 1, 1], 0.5, 1.0, he, we, env, kv=19, count_val=0)
    assert np.all(Lo == 0)
    col, Lo = ref64.shade(torch.zeros(3, 1, dtype=f64), torch.tensor([[0.0], [0.0], [1.0]]),
                          torch.ones(3, 1, dtype=f64), torch.tensor([0.5]), torch.tensor([1.0]),
                          np.zeros((3, 1), np.int32), np.array([[1.0], [0.0], [0.0]]),
                          np.full((1, he * we), 19, np.uint8), 19, he, we, he, we, env,
                          np.array([0, 0, 3.0]), np.array([0]))
    assert torch.all(col == 0)


def test_srgb_transfer_curve():
    x = torch.tensor([0.0, 0.0031308, 1.0], dtype=f64)
    y = ref64.srgb_oetf(x)
    assert y[0].item() == 0.0
    assert abs(y[1].item() - 0.0404500) < 1e-6     # both branches meet at the knee
    assert abs(y[2].item() - 1.0) < 1e-12


@pytest.mark.parametrize("grid", [(8, 16, 8, 8), (32, 64, 32, 32), (16, 32, 16, 32),
                                  (12, 24, 4, 6)])
def test_texel_view_lies_in_its_view_cell(grid):
    """The coarse texel -> view map (views fewer than light directions): the
    direction of every texel lies inside the lat-long cell of the view it is
    given, measured from the direction itself (polar angle from +Y, azimuth
    from +Z towards +X), not from the integer formula."""
    he, we, hv, wv = grid
    dirs, _ = ref64.env_geometry(he, we)
    view = ref64.texel_view(he, we, hv, wv).numpy()
    d = dirs.numpy()
    th = np.arccos(np.clip(d[:, 1], -1.0, 1.0))
    ph = np.mod(np.arctan2(d[:, 0], d[:, 2]), 2 * math.pi)
    vr, vc = view // wv, view % wv
    assert view.min() >= 0 and view.max() < hv * wv
    assert np.all(th >= vr * math.pi / hv) and np.all(th < (vr + 1) * math.pi / hv)
    assert np.all(ph >= vc * 2 * math.pi / wv) and np.all(ph < (vc + 1) * 2 * math.pi / wv)
    # every view cell receives the same number of texels
    assert np.all(np.bincount(view, minlength=hv * wv) == (he // hv) * (we // wv))


def test_texel_view_identity_when_grids_coincide():
    for he, we in ((8, 16), (16, 32), (32, 64)):
        assert np.array_equal(ref64.texel_view(he, we, he, we).numpy(), np.arange(he * we))


def test_bf16_rounding_and_operand_emulation():
    """bfloat16 rounding (8 significant bits, ties to even) on hand-checked
    values, and the emulated contraction forms: exact for operands that
    bfloat16 holds exactly; for positive sums the plain bf16 form's relative
    error is bounded by two roundings per product (2 * 2^-9 + 2^-18) and the
    split hi + lo form's by its dropped lo.lo product and the rounding of the
    lo parts (< 2^-15), and the split is far closer than the plain form."""
    vals = torch.tensor([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7, 3.0,
                         -(1.0 + 2.0 ** -9), 2.0 ** -130], dtype=f64)
    want = [1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, 3.0, -1.0, 2.0 ** -130]
    assert ref64.bf16_round(vals).tolist() == want
    rng = np.random.default_rng(3)
    Wi = torch.tensor(rng.integers(0, 64, (17, 40)), dtype=f64) / 8
    Ei = torch.tensor(rng.integers(0, 64, (40, 3)), dtype=f64) * 4
    for op in ("bf16", "bf16x3"):
        assert torch.equal(ref64.contract(Wi, Ei, op), Wi @ Ei)
    W = torch.tensor(rng.random((64, 512)))
    E = torch.tensor(np.exp(rng.normal(-1, 1, (512, 3))))
    ex = W @ E
    e1 = ((ref64.contract(W, E, "bf16") - ex).abs() / ex).max().item()
    e3 = ((ref64.contract(W, E, "bf16x3") - ex).abs() / ex).max().item()
    assert e1 <= 2 * 2.0 ** -9 + 2.0 ** -18
    assert e3 < 2.0 ** -15 and e3 < e1 / 50


def test_bf16_shading_forms_against_exact():
    """The shaded colours of a scene with each emulated operand precision:
    plain bf16 loses several 1e-3 relative, the split form stays within
    2e-5 (its dropped lo.lo product is about 2^-16 of each term)."""
    from tests import helpers
    from tests.conftest import scene
    s = scene(1)
    xo, no, _ = helpers.cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    _, _, cnt = helpers.oracle_visibility(s)
    front = helpers.front_flags(s)
    args = (ref64.t64(xo), ref64.t64(no), s["albedo"], s["rough"], s["tint"], s["vidx"], s["vw"],
            cnt, s["kv"], s["he"], s["we"], s["hv"], s["wv"], s["env"],
            s["cam"].centre.astype(np.float32).astype(np.float64), front)
    ex, _ = ref64.shade(*args)
    lit = ex > 1e-3
    errs = {}
    for op in ("bf16", "bf16x3"):
        c, _ = ref64.shade(*args, operands=op)
        errs[op] = ((c - ex).abs()[lit] / ex[lit]).max().item()
    assert errs["bf16"] > 1e-3 and errs["bf16x3"] < 2e-5, errs
