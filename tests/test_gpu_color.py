"""Colour network at the hits of a geometry render, against the FP64 oracle
(run with -m gpu).

Free running: the GPU renders its own geometry and the oracle its own; colours
and colour gradients are compared on the pixels that are hits in both with
the same step count (there the two Eq. 1 points agree to the render's depth
tolerance).  FP32: colour within 1e-5, dL/dz within 1e-3 relative; BF16
(bf16 colour network, split-bf16 recompute in the backward): colour within
2e-2 at worst and 2e-3 at the median, dL/dz within 1e-2.
"""
import sys

import numpy as np
import pytest

import dist_inputs as di
from oracle import dist_oracle as O
from _common import gpu_ctx, oracle_decoder

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_13225_amd import _native
    _native.load()


CASES = {
    "fp32-c1": (di.C1_SPEC, di.C1_COLOR_SPEC, 0, 24, 0),
    "bf16-deepsdf": (di.DEEPSDF_SPEC, di.COLOR_SPEC, 1, 32, 1),
}


@pytest.mark.parametrize("case", list(CASES))
def test_color_and_its_gradient_match_oracle(case):
    from paper_1911_13225_amd import api
    gspec, cspec, precision, H, levels = CASES[case]
    _log("case:", case)
    gctx = gpu_ctx(gspec)
    Wc, bc = di.make_decoder(cspec, seed=7)
    cctx = gpu_ctx(cspec, Ws=Wc, bs=bc)
    cdec = O.ColorDecoder(cspec, Wc, bc)
    cams = di.random_sphere_cameras(2, H, H)
    Z = di.make_latents(2, gspec.latent_dim, sigma=0.05)
    Zc = di.make_latents(2, cspec.latent_dim, sigma=0.3, base_seed=6000)
    prm = di.TraceParams(alpha=1.5, eps=5e-4, max_steps=40, c2f_levels=levels, k_samples=1, precision=precision,
                         want_normals=0)
    pairs = [(i // 2, i % 2) for i in range(4)]
    rs = O.render(oracle_decoder(gspec), Z, cams, pairs, prm)
    out = api.dist_render_fwd(gctx, cams, torch.tensor(Z, device="cuda"), prm, save=True)
    zc = torch.tensor(Zc, device="cuda")
    rgb = api.dist_render_color(cctx, out["saved"], zc, precision).double().cpu().numpy()
    ref = O.render_color(cdec, Zc, rs, pairs)
    same = [(out["status"][i].cpu().numpy() == 1) & (r.status == 1) & (out["nsteps"][i].cpu().numpy() == r.nsteps)
            for i, r in enumerate(rs)]
    err = np.concatenate([np.abs(rgb[i] - ref[i])[same[i]].reshape(-1) for i in range(4)])
    off = np.concatenate([rgb[i][(out["status"][i].cpu().numpy() != 1)].reshape(-1) for i in range(4)])
    _log("colour: pixels", int(sum(m.sum() for m in same)), "max err", float(err.max()), "median", float(np.median(err)))
    assert err.size > 100 and np.all(off == 0.0)
    if precision == 0:
        assert err.max() <= 1e-5
    else:
        assert err.max() <= 2e-2 and np.median(err) <= 2e-3
    # backward: a random colour gradient on the agreeing hit pixels
    rng = np.random.Generator(np.random.PCG64(8))
    g = [rng.standard_normal((H, H, 3)) * same[i][..., None] for i in range(4)]
    g_ref = O.color_backward(cdec, Zc, rs, pairs, g)
    gt = torch.tensor(np.stack(g).astype(np.float32), device="cuda")
    g_gpu = api.dist_render_color_bwd(cctx, out["saved"], zc, gt, precision).double().cpu().numpy()
    g_gpu2 = api.dist_render_color_bwd(cctx, out["saved"], zc, gt, precision).double().cpu().numpy()
    out["saved"].free()
    rel = np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref)
    _log("colour gradient rel", rel)
    assert np.array_equal(g_gpu, g_gpu2)
    assert rel <= (1e-3 if precision == 0 else 1e-2)


def test_color_and_geometry_networks_are_not_interchangeable():
    from paper_1911_13225_amd import api, _native as N
    gctx = gpu_ctx(di.C1_SPEC)
    cctx = gpu_ctx(di.C1_COLOR_SPEC, seed=7)
    cams = [di.front_camera(16, 16)]
    Z = torch.tensor(di.make_latents(1, di.C1_SPEC.latent_dim), device="cuda")
    prm = di.TraceParams(alpha=1.5, eps=5e-4, max_steps=20, c2f_levels=0, precision=0, want_normals=0)
    with pytest.raises(N.DistError) as e:
        api.dist_render_fwd(cctx, cams, torch.zeros(1, di.C1_COLOR_SPEC.latent_dim, device="cuda"), prm)
    assert e.value.code == -1
    out = api.dist_render_fwd(gctx, cams, Z, prm, save=True)
    with pytest.raises(N.DistError):
        api.dist_render_color(gctx, out["saved"], Z, 0)
    with pytest.raises(N.DistError):        # one colour code per latent of the render
        api.dist_render_color(cctx, out["saved"], torch.zeros(2, di.C1_COLOR_SPEC.latent_dim, device="cuda"), 0)
    rgb = api.dist_render_color(cctx, out["saved"], torch.zeros(1, di.C1_COLOR_SPEC.latent_dim, device="cuda"), 0)
    out["saved"].free()
    assert rgb.shape == (1, 16, 16, 3) and float(rgb.max()) <= 1.0 and float(rgb.min()) >= 0.0
