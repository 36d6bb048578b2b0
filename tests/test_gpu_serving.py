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


def _oracle_fit(dec, cams, pairs, prm, z0, dt, st, iters, lr=1e-2):
    """The oracle's latent fit: render -> loss_and_grads -> backward -> Adam."""
    from oracle import dist_oracle as O
    zo = z0.astype(np.float64).copy()
    m = np.zeros_like(zo)
    v = np.zeros_like(zo)
    losses, gs, renders = [], [], []
    for it in range(iters):
        rs = O.render(dec, zo[None], cams, pairs, prm)
        grads, L = [], 0.0
        for r, d_t, s_t in zip(rs, dt, st):
            l, g_d, g_n, g_s = O.loss_and_grads(r, d_t, np.zeros(d_t.shape + (3,)), s_t, w_d=10.0, w_s=1.0)
            grads.append((g_d, g_n, g_s))
            L += l
        g = O.backward(dec, zo[None], rs, pairs, prm, grads, want_theta=False)[0][0]
        losses.append(L)
        gs.append(g)
        renders.append(rs)
        zo, m, v = O.adam_step(zo, g, m, v, it + 1, lr=lr)
    return zo, losses, gs, renders


def test_served_zopt_matches_oracle_loop(ctx):
    """A served latent-optimisation job (bf16 march, split-precision recompute,
    device loss, adjoint and Adam) against the oracle's own loop from the same
    start and targets.

    Adam is invariant to the scale of the gradient and its first step moves
    every coordinate by lr sign(g), so the code it returns checks the
    gradient's direction coordinate by coordinate: after one iteration every
    coordinate whose oracle gradient is clear of the bf16 gradient error
    (|g_j| > 5% of max |g|) must have moved by exactly -lr sign(g_j), and none
    by more than lr.  After three iterations those coordinates (clear at every
    iteration, one sign) must agree with the oracle's code to 0.3 lr (each
    step is lr m/sqrt(v), a ratio of gradients that agree to a few percent per
    coordinate), and every coordinate to 2 lr per step.  The loss the job
    reports is the loss of its last render: it must equal the loss of the maps
    it returned (float32 summation order), and the oracle's loss at the same
    iteration up to what the bf16 render tolerances allow, w_d 2e-3 per
    foreground pixel plus w_s 2e-3 per pixel inside the unit sphere, per H W."""
    from paper_1911_13225_amd import api, _native as N
    from _common import oracle_decoder
    spec = di.DEEPSDF_SPEC
    dec = oracle_decoder(spec)
    H = 32
    cams = di.random_sphere_cameras(2, H, H, base_seed=2100)
    pairs = [(0, 0), (1, 0)]
    prm = _prm(want_normals=0)
    from oracle import dist_oracle as O
    zs = di.make_latents(1, 256, sigma=0.1, base_seed=3000)
    tg = O.render(dec, zs, cams, pairs, prm)
    dt = np.stack([np.where(np.isfinite(t.depth), t.depth, 0.0) for t in tg]).astype(np.float32)
    st = np.stack([(t.sil < 0).astype(np.float32) for t in tg])
    z0 = di.make_latents(1, 256, sigma=0.01, base_seed=1000)[0]
    td, ts = torch.tensor(dt, device="cuda"), torch.tensor(st, device="cuda")
    lr = 1e-2
    for iters in (1, 3):
        _log("served z-opt vs oracle loop, iterations", iters)
        req = api.ServeRequest(N.REQ_ZOPT, cams, torch.tensor(z0, device="cuda"), prm, want_normals=False,
                               targets=(td, ts), iters=iters, lr=lr)
        api.dist_submit(ctx, req)
        res = api.dist_poll(ctx, req, 120_000_000)
        assert res is not None and res["status"] == 0
        zo, losses, grads, renders = _oracle_fit(dec, cams, pairs, prm, z0, dt.astype(np.float64),
                                                 st.astype(np.float64), iters, lr)
        zg = req.z_out.double().cpu().numpy()
        # the reported loss is that of the returned maps (last iteration)
        depth, sil = req.depth.double().cpu().numpy(), req.sil.double().cpu().numpy()
        fg = (sil < 0) & (st > 0.5)
        L_maps = (10.0 * np.abs(np.where(fg, depth - dt, 0.0)).sum()
                  + (st * np.maximum(sil, 0) + (1 - st) * np.maximum(-sil, 0)).sum()) / (H * H)
        _log("  final loss", res["final_loss"], "of its maps", L_maps, "oracle", losses[-1])
        assert abs(res["final_loss"] - L_maps) <= 1e-5 * L_maps
        n_fg = sum(int((r.status == O.HIT).sum()) for r in renders[-1])
        n_in = sum(int((r.status != O.MISS).sum()) for r in renders[-1])
        bound = (10.0 * 2e-3 * n_fg + 2e-3 * n_in) / (H * H)
        assert abs(res["final_loss"] - losses[-1]) <= bound, (res["final_loss"], losses[-1], bound)
        gmax = [np.abs(g).max() for g in grads]
        clear = np.all([np.abs(g) > 0.05 * m for g, m in zip(grads, gmax)], axis=0)
        clear &= np.all([np.sign(g) == np.sign(grads[0]) for g in grads], axis=0)
        assert clear.sum() >= 10
        dz = zg - z0.astype(np.float64)
        if iters == 1:
            np.testing.assert_allclose(dz[clear], -lr * np.sign(grads[0][clear]), rtol=1e-4, atol=0)
            assert np.all(np.abs(dz) <= lr * (1 + 1e-4))
        else:
            err = np.abs(zg - zo)
            _log("  |z - z_oracle| on", int(clear.sum()), "clear coordinates: max", err[clear].max() / lr, "lr")
            assert np.all(err[clear] <= 0.3 * lr)
            assert np.all(err <= 2 * lr * iters)


def test_slot_reuse_after_a_request_ends_by_max_steps():
    """A request that stops at max_steps leaves its stopped rays in the last
    pooled list; a request of another resolution admitted into the freed ray
    slots at the next tick must render exactly as it does alone."""
    from paper_1911_13225_amd import api, _native as N
    spec = di.C1_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    budget = 18 << 20           # a pool of 65536 ray slots: A or B, never both

    def b_request():
        cams = di.random_sphere_cameras(1, 224, 224, base_seed=2300)
        z = torch.tensor(di.make_latents(1, 64, sigma=0.02, base_seed=5300)[0], device="cuda")
        return api.ServeRequest(N.REQ_RENDER, cams, z, _prm(c2f_levels=2), want_normals=True)

    c = api.Context.from_spec(spec, Ws, bs, hbm_budget=budget)
    try:
        alone = b_request()
        api.dist_submit(c, alone)
        assert api.dist_poll(c, alone, 60_000_000)["status"] == 0
        cams_a = di.random_sphere_cameras(3, 128, 128, base_seed=2400)
        za = torch.tensor(di.make_latents(1, 64, sigma=0.02, base_seed=5400)[0], device="cuda")
        a = api.ServeRequest(N.REQ_RENDER, cams_a, za, _prm(c2f_levels=0, max_steps=4), want_normals=False)
        b = b_request()
        api.dist_submit(c, a)
        api.dist_submit(c, b)
        ra = api.dist_poll(c, a, 60_000_000)
        rb = api.dist_poll(c, b, 60_000_000)
        assert ra["status"] == 0 and rb["status"] == 0
        n_unconv = int((a.status == 4).sum())
        _log("slot reuse: A rays stopped at max_steps", n_unconv)
        assert n_unconv > 1000
        assert torch.equal(alone.depth, b.depth)
        assert torch.equal(alone.sil, b.sil)
        assert torch.equal(alone.status, b.status)
        assert torch.equal(alone.normal, b.normal)
    finally:
        c.close()


def test_non_finite_queries_are_reported():
    """A decoder whose output layer holds a NaN returns a non-finite f at
    every query: the forward marks every ray that meets the unit sphere
    DIST_ERROR (background, depth +inf, silhouette +inf, no gradient samples,
    so dL/dz is zero), and a served render or z-opt request ends with
    DIST_ENUMERIC."""
    from paper_1911_13225_amd import api, _native as N
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    Ws = [w.copy() for w in Ws]
    Ws[-1][0, 7] = np.nan
    c = api.Context.from_spec(spec, Ws, bs)
    try:
        cams = [di.front_camera(32, 32)]
        Z = torch.tensor(di.make_latents(1, spec.latent_dim), device="cuda")
        for prec in (0, 1):
            _log("non-finite decoder: forward and backward, precision", prec)
            out = api.dist_render_fwd(c, cams, Z, _prm(precision=prec, c2f_levels=0), save=True)
            st = out["status"].cpu().numpy()
            assert set(np.unique(st).tolist()) <= {N.ERROR, N.MISS} and (st == N.ERROR).any()
            assert bool(torch.isinf(out["depth"]).all()) and bool((out["sil"] > 0).all())
            err = torch.tensor(st == N.ERROR, device="cuda")
            assert bool(torch.isinf(out["sil"][err]).all())
            ones = torch.ones_like(out["depth"])
            g = api.dist_render_bwd(c, out["saved"], ones, torch.ones_like(out["normal"]), ones, n_latents=1)
            out["saved"].free()
            assert float(g.abs().max()) == 0.0
        _log("non-finite decoder: served render and z-opt")
        r = api.ServeRequest(N.REQ_RENDER, cams, Z[0], _prm(c2f_levels=0), want_normals=True)
        api.dist_submit(c, r)
        res = api.dist_poll(c, r, 60_000_000)
        assert res is not None and res["status"] == N.DIST_ENUMERIC
        assert bool((r.status == N.ERROR).any())
        tgt = (torch.full((1, 32, 32), 1.5, device="cuda"), torch.ones(1, 32, 32, device="cuda"))
        q = api.ServeRequest(N.REQ_ZOPT, cams, Z[0], _prm(c2f_levels=0), want_normals=False, targets=tgt, iters=3)
        api.dist_submit(c, q)
        res = api.dist_poll(c, q, 60_000_000)
        assert res is not None and res["status"] == N.DIST_ENUMERIC
    finally:
        c.close()
