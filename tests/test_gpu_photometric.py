"""Cross-view photometric loss on the GPU against the FP64 oracle (run with -m gpu).

Same inputs on both sides (closed-form sphere depth maps scaled by 1.003 and
a procedurally textured sphere), so the comparison is of the loss itself: the
total to 1e-5 relative, dL/d(depth) per pixel to 1e-4 of its largest value on
all but 0.1% of the pixels (float32 and float64 may take a visibility or
footprint decision differently at a boundary).  End to end, the tracer's
depth (float32), the loss and the paper's backward give the loss within 1e-4
and dL/dz within 1e-3 (the float32 dL/dz bound) of the oracle's free-running
pipeline.
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


def _ring_inputs(n, H, freq=4.0, scale=1.003):
    cams = di.ring_cameras(n, H, H)
    im = di.textured_sphere_images(cams, 0.45, freq=freq)
    D = np.stack([di.sphere_target_maps(c, 0.45)[0] for c in cams]) * np.float32(scale)
    return cams, D.astype(np.float32), im


@pytest.mark.parametrize("n,H", [(8, 64), (4, 37)])
def test_photometric_loss_matches_oracle(n, H):
    from paper_1911_13225_amd import api
    cams, D, im = _ring_inputs(n, H)
    pairs = [(i, (i + 1) % n) for i in range(n)] + [(i, (i + n - 1) % n) for i in range(n)]
    _log("case: views", n, "H", H, "pairs", len(pairs))
    L_o, g_o = O.photometric_loss(cams, list(D), list(im), pairs, weight=5.0)
    g_o = np.stack(g_o)
    loss, g = api.dist_photometric_loss(cams, torch.tensor(D, device="cuda"), torch.tensor(im, device="cuda"), pairs,
                                        weight=5.0)
    loss2, g2 = api.dist_photometric_loss(cams, torch.tensor(D, device="cuda"), torch.tensor(im, device="cuda"),
                                          pairs, weight=5.0)
    L = float(loss.item())
    g = g.double().cpu().numpy()
    assert torch.equal(loss, loss2) and np.array_equal(g, g2.double().cpu().numpy())
    bad = np.abs(g - g_o) > 1e-4 * np.abs(g_o).max()
    _log("loss", L, "oracle", L_o, "pixels off", int(bad.sum()), "of", bad.size)
    assert abs(L - L_o) <= 1e-5 * abs(L_o)
    assert int(bad.sum()) <= max(1, bad.size // 1000)


def test_photometric_pipeline_gradient_matches_oracle():
    """Render depth (float32 tracer), photometric loss, paper backward: dL/dz
    against the oracle's pipeline on the oracle's own render."""
    from paper_1911_13225_amd import api
    spec = di.C1_SPEC
    ctx = gpu_ctx(spec)
    n, H = 4, 40
    cams = di.ring_cameras(n, H, H)
    im = di.textured_sphere_images(cams, 0.45, freq=4.0)
    Z = di.make_latents(1, spec.latent_dim, sigma=0.05)
    prm = di.TraceParams(alpha=1.5, eps=5e-4, max_steps=40, c2f_levels=0, k_samples=1, precision=0, want_normals=0)
    pairs = [(i, (i + 1) % n) for i in range(n)]
    dec = oracle_decoder(spec)
    rs = O.render(dec, Z, cams, [(v, 0) for v in range(n)], prm)
    L_o, gd_o = O.photometric_loss(cams, [r.depth for r in rs], list(im), pairs, weight=5.0)
    zero = np.zeros((H, H))
    ref = O.backward(dec, Z, rs, [(v, 0) for v in range(n)], prm,
                     [(g, np.zeros((H, H, 3)), zero) for g in gd_o], want_theta=False)[0]
    out = api.dist_render_fwd(ctx, cams, torch.tensor(Z, device="cuda"), prm, save=True)
    loss, gd = api.dist_photometric_loss(cams, out["depth"], torch.tensor(im, device="cuda"), pairs, weight=5.0)
    g = api.dist_render_bwd(ctx, out["saved"], gd, None, None, n_latents=1).double().cpu().numpy()
    out["saved"].free()
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    _log("photometric loss", float(loss.item()), "oracle", L_o, "dL/dz rel", rel)
    assert abs(float(loss.item()) - L_o) <= 1e-4 * L_o
    assert rel <= 1e-3


def test_photometric_invalid_arguments():
    from paper_1911_13225_amd import api, _native as N
    cams, D, im = _ring_inputs(4, 16)
    d, i = torch.tensor(D, device="cuda"), torch.tensor(im, device="cuda")
    for pairs in ([(0, 4)], [(-1, 0)], []):
        with pytest.raises(N.DistError) as e:
            api.dist_photometric_loss(cams, d, i, pairs)
        assert e.value.code == -1
    many = di.ring_cameras(17, 16, 16)
    with pytest.raises(N.DistError):
        api.dist_photometric_loss(many, torch.zeros(17, 16, 16, device="cuda"), torch.zeros(17, 16, 16, 3,
                                                                                           device="cuda"), [(0, 1)])
    # still usable afterwards, loss only
    loss, g = api.dist_photometric_loss(cams, d, i, [(0, 1)], want_grad=False)
    assert g is None and np.isfinite(float(loss.item()))
