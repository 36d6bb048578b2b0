"""The image-space loss of the latent fit and the Adam step on the GPU (run
with -m gpu), against the FP64 oracle's loss_and_grads and adam_step on the
same inputs: oracle-rendered maps (rounded to float32) and sphere targets."""
import sys

import numpy as np
import pytest

import dist_inputs as di
from oracle import dist_oracle as O
from _common import oracle_decoder

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


@pytest.mark.parametrize("w", [(10.0, 1.0, 0.0), (10.0, 1.0, 1.0), (0.0, 2.5, 0.5)], ids=["d+s", "d+s+n", "s+n"])
def test_render_loss_matches_oracle(w):
    from paper_1911_13225_amd import api
    w_d, w_s, w_n = w
    spec = di.C1_SPEC
    dec = oracle_decoder(spec)
    H = 24
    cams = di.random_sphere_cameras(3, H, H)
    Z = di.make_latents(1, spec.latent_dim, sigma=0.05)
    prm = di.TraceParams(alpha=1.5, eps=1e-3, max_steps=30, c2f_levels=1, want_normals=1)
    rs = O.render(dec, Z, cams, [(v, 0) for v in range(3)], prm)
    maps = {k: np.stack([getattr(r, k) for r in rs]).astype(np.float32) for k in ("depth", "normal", "sil")}
    # targets: a sphere of another radius, with a soft target silhouette on part of the image
    tg = [di.sphere_target_maps(c, 0.47) for c in cams]
    dt = np.stack([t[0] for t in tg])
    nt = np.stack([t[1] for t in tg])
    st = np.stack([t[2] for t in tg])
    st[:, :4, :] = 0.3
    T = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda")
    loss, gd, gn, gs = api.dist_render_loss(T(maps["depth"]), T(maps["normal"]), T(maps["sil"]), T(dt), T(nt),
                                            T(st), w_d=w_d, w_s=w_s, w_n=w_n)
    loss2, gd2, gn2, gs2 = api.dist_render_loss(T(maps["depth"]), T(maps["normal"]), T(maps["sil"]), T(dt), T(nt),
                                                T(st), w_d=w_d, w_s=w_s, w_n=w_n)
    assert torch.equal(loss, loss2) and torch.equal(gd, gd2) and torch.equal(gs, gs2) and torch.equal(gn, gn2)
    for i, r in enumerate(rs):
        r.depth, r.sil, r.normal = (maps[k][i].astype(np.float64) for k in ("depth", "sil", "normal"))
        L, g_d, g_n, g_s = O.loss_and_grads(r, dt[i], nt[i], st[i], w_d=w_d, w_s=w_s, w_n=w_n)
        _log("image", i, "loss gpu", float(loss[i]), "oracle", L)
        assert abs(float(loss[i]) - L) <= 2e-6 * max(abs(L), 1e-3)
        np.testing.assert_allclose(gd[i].cpu().numpy(), g_d, rtol=1e-6, atol=0)
        np.testing.assert_allclose(gs[i].cpu().numpy(), g_s, rtol=1e-6, atol=0)
        np.testing.assert_allclose(gn[i].cpu().numpy(), g_n, rtol=1e-6, atol=0)


def test_render_loss_rejects_bad_arguments():
    from paper_1911_13225_amd import api, _native as N
    x = torch.zeros(1, 4, 4, device="cuda")
    with pytest.raises(N.DistError) as e:
        api.dist_render_loss(x, None, x, x, None, x, w_n=1.0)
    assert e.value.code == -1
    lib = N.load()
    assert lib.dist_render_loss(0, 4, 4, None, None, None, None, None, None, 1.0, 1.0, 0.0, None, None, None, None,
                                None) == -1


def test_adam_step_matches_oracle():
    from paper_1911_13225_amd import api
    rng = np.random.Generator(np.random.PCG64(8))
    n = 256
    z = rng.standard_normal(n).astype(np.float32)
    zt = torch.tensor(z, device="cuda")
    m = torch.zeros(n, device="cuda")
    v = torch.zeros(n, device="cuda")
    zo, mo, vo = z.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        g = (rng.standard_normal(n) * 10.0 ** (-t)).astype(np.float32)
        api.dist_adam_step(zt, m, v, torch.tensor(g, device="cuda"), t)
        zo, mo, vo = O.adam_step(zo, g.astype(np.float64), mo, vo, t)
    np.testing.assert_allclose(zt.cpu().numpy(), zo, rtol=0, atol=2e-6)
