"""Serving loop (continuous batching) on the GPU.

* A request's result is bitwise the same whether it runs alone or pooled with
  other requests of different resolutions (each ray's decoder evaluation and
  march update is independent of the other rays in its tile, and the
  per-request reductions run in a fixed order).
* A served render equals the batch render of the same images.
* A latent-optimisation request returns the same code alone and in the mix.
* Admission errors: a request larger than the budget is refused (ENOMEM).
"""
import sys
import time

import numpy as np
import pytest

import dist_inputs as di

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    c = api.Context.from_spec(spec, Ws, bs)
    yield c
    c.close()


def _prm(**kw):
    p = di.TraceParams(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=2, k_samples=1, precision=1, want_normals=1)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _render_req(res, n_views, seed, normals=True):
    from paper_1911_13225_amd import api, _native as N
    cams = di.random_sphere_cameras(n_views, res, res, base_seed=2000 + seed)
    z = torch.tensor(di.make_latents(1, 256, sigma=0.01, base_seed=5000 + seed)[0], device="cuda")
    return api.ServeRequest(N.REQ_RENDER, cams, z, _prm(), want_normals=normals), cams, z


def test_served_render_alone_equals_mix_and_batch(ctx):
    from paper_1911_13225_amd import api
    _log("serving: alone")
    a, cams, z = _render_req(64, 2, 1)
    api.dist_submit(ctx, a)
    ra = api.dist_poll(ctx, a, 60_000_000)
    assert ra is not None and ra["status"] == 0
    _log("  alone", ra)
    # the same request pooled with others of different resolutions
    _log("serving: mix")
    b, _, _ = _render_req(64, 2, 1)
    others = [_render_req(res, nv, 10 + i)[0] for i, (res, nv) in enumerate([(128, 1), (32, 3), (256, 1), (64, 4)])]
    for o in others[:2]:
        api.dist_submit(ctx, o)
    api.dist_submit(ctx, b)
    for o in others[2:]:
        api.dist_submit(ctx, o)
    rb = api.dist_poll(ctx, b, 60_000_000)
    for o in others:
        ro = api.dist_poll(ctx, o, 60_000_000)
        assert ro is not None and ro["status"] == 0
    _log("  mix", rb)
    assert torch.equal(a.depth, b.depth)
    assert torch.equal(a.sil, b.sil)
    assert torch.equal(a.status, b.status)
    assert torch.equal(a.normal, b.normal)
    assert ra["queries"] == rb["queries"]
    # the batch path renders the same images bit for bit
    out = api.dist_render_fwd(ctx, cams, z[None], _prm())
    torch.cuda.synchronize()
    assert torch.equal(out["depth"], a.depth)
    assert torch.equal(out["status"], a.status)
    assert torch.equal(out["normal"], a.normal)
    assert int(out["queries"].sum()) == ra["queries"]


def test_served_zopt_alone_equals_mix(ctx):
    from paper_1911_13225_amd import api, _native as N
    cams = di.random_sphere_cameras(2, 64, 64, base_seed=2100)
    spec = di.DEEPSDF_SPEC
    z_star = torch.tensor(di.make_latents(1, 256, sigma=0.1, base_seed=3000)[0], device="cuda")
    tgt = api.dist_render_fwd(ctx, cams, z_star[None], _prm(want_normals=0))
    torch.cuda.synchronize()
    td = torch.where(torch.isfinite(tgt["depth"]), tgt["depth"], torch.zeros_like(tgt["depth"]))
    ts = (tgt["sil"] < 0).float()
    z0 = torch.tensor(di.make_latents(1, 256, sigma=0.01, base_seed=1000)[0], device="cuda")

    def make():
        return api.ServeRequest(N.REQ_ZOPT, cams, z0, _prm(want_normals=0), want_normals=False,
                                targets=(td, ts), iters=3, lr=1e-2)

    a = make()
    api.dist_submit(ctx, a)
    ra = api.dist_poll(ctx, a, 120_000_000)
    assert ra["status"] == 0
    b = make()
    others = [_render_req(res, nv, 20 + i)[0] for i, (res, nv) in enumerate([(128, 2), (64, 1)])]
    api.dist_submit(ctx, others[0])
    api.dist_submit(ctx, b)
    api.dist_submit(ctx, others[1])
    rb = api.dist_poll(ctx, b, 120_000_000)
    for o in others:
        assert api.dist_poll(ctx, o, 120_000_000)["status"] == 0
    _log("zopt alone", ra, "mix", rb, "|dz|", float((a.z_out - z0).norm()))
    assert torch.equal(a.z_out, b.z_out)
    assert ra["queries"] == rb["queries"]
    assert float((a.z_out - z0).norm()) > 0
    assert abs(ra["final_loss"] - rb["final_loss"]) <= 1e-6 * max(1.0, abs(ra["final_loss"]))


def test_admission_refuses_requests_beyond_the_budget():
    from paper_1911_13225_amd import api, _native as N
    spec = di.C1_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    # a small budget: enough for the decoder and a small pool
    c = api.Context.from_spec(spec, Ws, bs, hbm_budget=256 << 20)
    try:
        cams = di.random_sphere_cameras(1, 32, 32)
        z = torch.zeros(64, device="cuda")
        ok = api.ServeRequest(N.REQ_RENDER, cams, z, _prm(precision=1), want_normals=False)
        api.dist_submit(c, ok)
        assert api.dist_poll(c, ok, 60_000_000)["status"] == 0
        big = api.ServeRequest(N.REQ_RENDER, di.random_sphere_cameras(16, 512, 512), z, _prm(precision=1),
                               want_normals=True)
        with pytest.raises(N.DistError) as e:
            api.dist_submit(c, big)
        assert e.value.code == -2
        bad = api.ServeRequest(N.REQ_RENDER, cams, z, _prm(precision=0), want_normals=False)
        with pytest.raises(N.DistError) as e:
            api.dist_submit(c, bad)
        assert e.value.code == -1
    finally:
        c.close()
