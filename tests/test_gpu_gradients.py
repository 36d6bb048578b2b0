"""Gradient checks of the HIP adjoint (run with -m gpu).

* The adjoint of the decoder at fixed points against central differences of
  the HIP forward (float32), h = 1e-3 and 1e-4, on 16 random latent
  coordinates: the frozen-sample surrogate L(z) = sum_k seed_k f(p_k, z) of the
  paper's first-term gradient (Eq. 2).
* Latent-code fitting (App. B.4: Adam, lr 1e-2; depth L1 x 10 + silhouette):
  the HIP path and the FP64 oracle each run their own 50-iteration fit from
  the same seeded start against the same oracle-rendered targets; the
  gradients agree at the start and the two loss curves agree along the way.
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


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx(di.DEEPSDF_SPEC)


def test_adjoint_matches_central_differences(ctx):
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    n = 4096
    rng = np.random.Generator(np.random.PCG64(31))
    d = rng.standard_normal((n, 3))
    P = (d / np.linalg.norm(d, axis=1, keepdims=True) * rng.uniform(0.35, 0.7, (n, 1))).astype(np.float32)
    seeds = rng.standard_normal(n).astype(np.float32)
    z = torch.tensor(di.make_latents(1, spec.latent_dim, sigma=0.01, base_seed=1000), device="cuda")
    Pt = torch.tensor(P, device="cuda")
    lat = torch.zeros(n, dtype=torch.int32, device="cuda")
    st = torch.tensor(seeds, device="cuda")
    g = api.dist_sdf_vjp(ctx, Pt, lat, st, z, 0)[0].double().cpu().numpy()
    coords = rng.choice(spec.latent_dim, 16, replace=False)
    s64 = seeds.astype(np.float64)
    for h, tol in ((1e-3, 2e-3), (1e-4, 2e-2)):
        fd = np.zeros(16)
        for a, i in enumerate(coords):
            zp = z.clone()
            zm = z.clone()
            zp[0, i] += h
            zm[0, i] -= h
            fp = api.dist_sdf_eval(ctx, Pt, lat, zp, 0).double().cpu().numpy()
            fm = api.dist_sdf_eval(ctx, Pt, lat, zm, 0).double().cpu().numpy()
            # the step actually taken in float32
            hh = (float(zp[0, i]) - float(zm[0, i])) / 2.0
            fd[a] = np.dot(s64, fp - fm) / (2.0 * hh)
        rel = np.linalg.norm(fd - g[coords]) / np.linalg.norm(g[coords])
        _log("central differences h", h, "rel", rel, "|g|", np.linalg.norm(g[coords]))
        assert rel <= tol


def _fit_targets(spec, cams, prm):
    dec = oracle_decoder(spec)
    zs = di.make_latents(1, spec.latent_dim, sigma=0.1, base_seed=3000)
    pairs = [(v, 0) for v in range(len(cams))]
    tg = O.render(dec, zs, cams, pairs, prm)
    dt = np.stack([np.where(np.isfinite(t.depth), t.depth, 0.0) for t in tg])
    st = np.stack([(t.sil < 0).astype(np.float64) for t in tg])
    return dec, zs, pairs, dt, st


def test_latent_fit_matches_oracle(ctx):
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    cams = di.random_sphere_cameras(2, 32, 32)
    prm = di.TraceParams(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=2, k_samples=1, precision=0,
                         want_normals=0)
    dec, zs, pairs, dt, st = _fit_targets(spec, cams, prm)
    z0 = di.make_latents(1, spec.latent_dim, sigma=0.01, base_seed=1000)
    iters, checks = 50, (0, 1, 10, 49)

    # HIP path: DistRender + torch Adam
    z = torch.tensor(z0, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([z], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    dtt = torch.tensor(dt.astype(np.float32), device="cuda")
    stt = torch.tensor(st.astype(np.float32), device="cuda")
    nz = torch.zeros(dtt.shape + (3,), device="cuda")
    loss_g, g0_gpu = {}, None
    for it in range(iters):
        depth, normal, sil, _ = api.DistRender.apply(z, ctx, cams, prm)
        L = api.render_loss(depth, nz, sil, dtt, nz, stt, w_d=10.0, w_s=1.0, w_n=0.0)
        opt.zero_grad()
        L.backward()
        if it == 0:
            g0_gpu = z.grad.detach().double().cpu().numpy()[0]
        loss_g[it] = float(L)
        opt.step()
    zg = z.detach().double().cpu().numpy()

    # oracle: its own render, loss gradient, backward and Adam in float64
    zo = z0.astype(np.float64).copy()
    m = np.zeros_like(zo)
    v = np.zeros_like(zo)
    loss_o, g0_or = {}, None
    for it in range(iters):
        rs = O.render(dec, zo, cams, pairs, prm)
        grads, L = [], 0.0
        for r, d_t, s_t in zip(rs, dt, st):
            l, gd, gn, gs = O.loss_and_grads(r, d_t, np.zeros(d_t.shape + (3,)), s_t, w_d=10.0, w_s=1.0, w_n=0.0)
            grads.append((gd, gn, gs))
            L += l
        g, _, _ = O.backward(dec, zo, rs, pairs, prm, grads, want_theta=False)
        if it == 0:
            g0_or = g[0]
        loss_o[it] = L
        zo, m, v = O.adam_step(zo, g, m, v, it + 1)

    rel0 = np.linalg.norm(g0_gpu - g0_or) / np.linalg.norm(g0_or)
    dz_g = np.linalg.norm(zg - zs) / np.linalg.norm(z0 - zs)
    dz_o = np.linalg.norm(zo - zs) / np.linalg.norm(z0 - zs)
    _log("latent fit: gradient at start rel", rel0)
    for it in checks:
        _log("  it", it, "loss hip", loss_g[it], "oracle", loss_o[it])
    _log("  |z - z*| / |z0 - z*|: hip", dz_g, "oracle", dz_o)
    assert rel0 <= 1e-3
    for it in checks:
        assert abs(loss_g[it] - loss_o[it]) <= 2e-2 * loss_o[0]
    assert loss_g[iters - 1] < loss_g[0] and loss_o[iters - 1] < loss_o[0]
