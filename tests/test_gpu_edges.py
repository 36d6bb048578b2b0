"""Edge cases and degenerate inputs of the HIP path (run with -m gpu).

Views that see nothing, single-pixel and odd-sized images, the largest K,
one marching step, zero gradients, empty query batches and invalid
arguments.  Results are compared with the FP64 oracle under the float32
tolerances of test_gpu_parity.py.
"""
import sys

import numpy as np
import pytest

import dist_inputs as di
from oracle import dist_oracle as O
from _common import cfg_params, compare_render, gpu_ctx, oracle_decoder

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


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx(di.DEEPSDF_SPEC)


def _away_camera(H, W):
    """A camera at radius 2 looking away from the origin: every ray misses."""
    cam = di.front_camera(H, W)
    R = cam.R_wc.astype(np.float64) @ np.diag([-1.0, 1.0, -1.0])     # still a rotation
    return di.Camera(cam.fx, cam.fy, cam.cx, cam.cy, R.astype(np.float32), cam.c, H, W)


def _prm(**kw):
    p = di.TraceParams(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=2, k_samples=1, precision=0, want_normals=1)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _np(out, i):
    return {k: out[k][i].cpu().numpy() for k in ("depth", "sil", "status", "nsteps")}


def test_view_that_sees_nothing(ctx):
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    cams = [_away_camera(16, 16)]
    Z = di.make_latents(1, spec.latent_dim)
    prm = _prm()
    out = api.dist_render_fwd(ctx, cams, torch.tensor(Z, device="cuda"), prm, save=True)
    o = O.render(oracle_decoder(spec), Z, cams, [(0, 0)], prm)[0]
    st = out["status"][0].cpu().numpy()
    assert np.all(st == O.MISS) and np.all(o.status == O.MISS)
    assert int(out["queries"].sum()) == 0
    assert np.all(np.isinf(out["depth"][0].cpu().numpy()))
    np.testing.assert_allclose(out["sil"][0].cpu().numpy(), o.sil, rtol=0, atol=1e-6)
    # no shape gradient from rays that miss the unit sphere; the camera still
    # gets the background-silhouette gradient
    g_s = torch.ones_like(out["sil"]) * 1e-2
    g = api.dist_render_bwd(ctx, out["saved"], None, None, g_s, n_latents=1)
    gc = api.dist_render_bwd_camera(ctx, out["saved"], 1, None, g_s).double().cpu().numpy()
    out["saved"].free()
    assert float(g.abs().max()) == 0.0
    g_c, g_R = O.camera_backward(oracle_decoder(spec), Z, [o], cams, [(0, 0)], prm,
                                 [(np.zeros((16, 16)), np.full((16, 16), 1e-2))])
    ref = np.concatenate([g_c[0], g_R[0].reshape(9)])
    assert np.linalg.norm(gc[0] - ref) <= 1e-5 * np.linalg.norm(ref)


@pytest.mark.parametrize("H,W,levels", [(1, 1, 0), (17, 9, 0), (12, 20, 2)])
def test_small_and_odd_images(ctx, H, W, levels):
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    cam = di.look_at_camera((0.3, -0.2, 1.9), H, W, fov_deg=30.0 if H == 1 else 50.0)
    Z = di.make_latents(1, spec.latent_dim, sigma=0.05)
    prm = _prm(c2f_levels=levels)
    out = api.dist_render_fwd(ctx, [cam], torch.tensor(Z, device="cuda"), prm)
    o = O.render(oracle_decoder(spec), Z, [cam], [(0, 0)], prm)[0]
    st = compare_render(o, _np(out, 0), prm.eps)
    _log("image", H, W, "levels", levels, st["hits"], "hits, flips", st["flips"], "depth max", st["depth_max"])
    assert st["unexplained"] == 0
    assert st["depth_max"] <= 1e-4
    assert int(out["queries"].sum()) == o.queries or st["flips"] > 0


def test_largest_k_and_one_step(ctx):
    """K = 4 records (the maximum) in the backward; a single marching step."""
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    H = 24
    cams = di.random_sphere_cameras(2, H, H)
    Z = di.make_latents(1, spec.latent_dim, sigma=0.05)
    dec = oracle_decoder(spec)
    pairs = [(0, 0), (1, 0)]
    # K = 4
    prm = _prm(k_samples=4, c2f_levels=1, want_normals=0)
    out = api.dist_render_fwd(ctx, cams, torch.tensor(Z, device="cuda"), prm, save=True)
    rs = O.render(dec, Z, cams, pairs, prm)
    grads, gd, gs = [], [], []
    for r, (v, l) in zip(rs, pairs):
        dt, nt, stt = di.sphere_target_maps(cams[v], 0.45)
        _, g_d, g_n, g_s = O.loss_and_grads(r, dt, nt, stt, w_d=10.0, w_s=1.0)
        grads.append((g_d, g_n, g_s))
        gd.append(g_d)
        gs.append(g_s)
    go = O.backward(dec, Z, rs, pairs, prm, grads, want_theta=False)[0]
    T = lambda a: torch.tensor(np.stack(a).astype(np.float32), device="cuda")
    g = api.dist_render_bwd(ctx, out["saved"], T(gd), None, T(gs), n_latents=1).double().cpu().numpy()
    out["saved"].free()
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    _log("K=4 backward rel", rel)
    assert rel <= 1e-3
    # one step: every ray that meets the sphere is queried once and stops
    prm1 = _prm(max_steps=1, c2f_levels=0, want_normals=0)
    out = api.dist_render_fwd(ctx, cams, torch.tensor(Z, device="cuda"), prm1)
    rs = O.render(dec, Z, cams, pairs, prm1)
    for i, r in enumerate(rs):
        st = compare_render(r, _np(out, i), prm1.eps)
        assert st["unexplained"] == 0
        assert set(np.unique(out["status"][i].cpu().numpy())) <= {O.HIT, O.MISS, O.UNCONVERGED}
        assert int(out["queries"][i]) == int((r.status != O.MISS).sum())


def test_zero_gradients_and_empty_batches(ctx):
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    cams = di.random_sphere_cameras(2, 16, 16)
    Z = torch.tensor(di.make_latents(2, spec.latent_dim), device="cuda")
    out = api.dist_render_fwd(ctx, cams, Z, _prm(precision=1), save=True)
    zeros = torch.zeros_like(out["depth"])
    g = api.dist_render_bwd(ctx, out["saved"], zeros, torch.zeros_like(out["normal"]), zeros, n_latents=2)
    g2 = api.dist_render_bwd(ctx, out["saved"], None, None, None, n_latents=2)
    out["saved"].free()
    assert float(g.abs().max()) == 0.0 and float(g2.abs().max()) == 0.0
    P = torch.zeros(0, 3, device="cuda")
    lat = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert api.dist_sdf_eval(ctx, P, lat, Z, 1).numel() == 0
    gz = api.dist_sdf_vjp(ctx, P, lat, torch.zeros(0, device="cuda"), Z, 1)
    assert float(gz.abs().max()) == 0.0


def test_sdf_vjp_device_grouping(ctx):
    """The VJP entry point groups its samples by latent on the device (stable
    sort, per-latent segments padded to whole tiles): each latent's gradient
    equals, bit for bit, that of a call holding only its own samples; ids
    outside [0, n_latents) are clamped; a repeated call is identical."""
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    g = np.random.default_rng(11)
    n, L = 1000, 3
    P = torch.tensor(g.uniform(-0.6, 0.6, (n, 3)).astype(np.float32), device="cuda")
    ids = g.integers(0, L, n).astype(np.int32)
    seeds = torch.tensor(g.normal(size=n).astype(np.float32), device="cuda")
    Z = torch.tensor(di.make_latents(L, spec.latent_dim), device="cuda")
    for prec in (0, 1):
        lat = torch.tensor(ids, device="cuda")
        gz = api.dist_sdf_vjp(ctx, P, lat, seeds, Z, prec)
        assert torch.equal(gz, api.dist_sdf_vjp(ctx, P, lat, seeds, Z, prec))
        for l in range(L):
            sel = torch.tensor(np.nonzero(ids == l)[0], device="cuda")
            one = api.dist_sdf_vjp(ctx, P[sel], torch.zeros(len(sel), dtype=torch.int32, device="cuda"), seeds[sel],
                                   Z[l:l + 1].contiguous(), prec)
            assert torch.equal(gz[l], one[0]), (prec, l)
        wild = ids.copy()
        wild[ids == 0] = -5
        wild[ids == L - 1] = L + 7
        gw = api.dist_sdf_vjp(ctx, P, torch.tensor(wild, device="cuda"), seeds, Z, prec)
        assert torch.equal(gw, gz)


def test_many_small_images_in_one_launch(ctx):
    """4,096 images of 8 x 8 (64 views x 64 latents) in one launch: every
    per-image grid row and descriptor is used; sampled images agree with the
    oracle in status and step count and, on hits, in depth; 65,536 images are
    refused (an image is one row of the per-image launch grids)."""
    from paper_1911_13225_amd import api, _native as N
    spec = di.C1_SPEC
    c = api.Context.from_spec(spec, *di.make_decoder(spec, seed=0))
    try:
        cams = di.random_sphere_cameras(64, 8, 8)
        Z = di.make_latents(64, spec.latent_dim)
        prm = _prm(precision=0, c2f_levels=1, want_normals=0)
        out = api.dist_render_fwd(c, cams, torch.tensor(Z, device="cuda"), prm)
        assert out["depth"].shape[0] == 4096
        dec = O.Decoder(spec, *di.make_decoder(spec, seed=0))
        for i in (0, 1, 2047, 4095):
            v, l = i // 64, i % 64
            o = O.render(dec, Z, cams, [(v, l)], prm)[0]
            st = out["status"][i].cpu().numpy()
            ns = out["nsteps"][i].cpu().numpy()
            same = (o.status == st) & (o.nsteps == ns)
            assert np.all(same | (o.margin < 2e-5)), i
            h = same & (st == 1)
            if h.any():
                assert np.abs(o.depth[h] - out["depth"][i].cpu().numpy()[h]).max() <= 1e-4
        with pytest.raises(N.DistError) as e:
            api.dist_render_fwd(c, di.random_sphere_cameras(256, 4, 4), torch.tensor(
                di.make_latents(256, spec.latent_dim), device="cuda"), _prm(precision=0, c2f_levels=0))
        assert e.value.code == -1
    finally:
        c.close()


def test_invalid_arguments_are_rejected(ctx):
    from paper_1911_13225_amd import api, _native as N
    spec = di.DEEPSDF_SPEC
    Z = torch.tensor(di.make_latents(1, spec.latent_dim), device="cuda")
    cam = di.front_camera(16, 16)
    bad = [
        ([di.front_camera(18, 18)], _prm(c2f_levels=2)),       # 18 is not a multiple of 4
        ([cam], _prm(alpha=0.0)),
        ([cam], _prm(k_samples=5)),
        ([cam], _prm(max_steps=0)),
        ([di.front_camera(16, 16, radius=0.5)], _prm()),       # camera inside the unit sphere
    ]
    for cams, prm in bad:
        with pytest.raises(N.DistError) as e:
            api.dist_render_fwd(ctx, cams, Z, prm)
        assert e.value.code == -1
    # a mixed-size view set
    with pytest.raises(N.DistError) as e:
        api.dist_render_fwd(ctx, [cam, di.front_camera(32, 32)], Z, _prm())
    assert e.value.code == -1
    # the library is still usable afterwards
    out = api.dist_render_fwd(ctx, [cam], Z, _prm())
    assert int(out["queries"].sum()) > 0
