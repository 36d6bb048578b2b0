"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: the paper's
worked examples (tests/golden/worked_examples.txt), closed forms of analytic
fields, brute-force dense marching, central finite differences and an
independent autograd evaluation.  A plausible mistake in the oracle (a dropped
term, a wrong sign, a swapped operand, an off-by-one step count) fails one of
these.
"""
import math

import numpy as np
import pytest

import dist_inputs as di
from oracle import dist_oracle as O
from conftest import load_golden


def _prm(**kw):
    p = di.TraceParams()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# ----------------------------------------------------------------------------
# Paper worked examples (App. A.1, App. A.2, Sec. 3.2)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("alpha", [1.0, 1.5])
def test_kmin_worked_example_through_march(alpha):
    """App. A.1: plane SDF, d=1, eps=5e-5, theta=10deg -> 52 (alpha 1) / 33 (alpha 1.5) steps.

    Runs the oracle's own march loop on one ray against a plane; the number of
    position updates before the converging query must equal the paper's count.
    """
    g = load_golden("worked_examples.txt")
    th = math.radians(g["kmin.theta_deg"])
    d0, eps = g["kmin.d"], g["kmin.eps"]
    want = int(g["kmin.steps.alpha%.1f" % alpha])
    # plane z = 0, ray starting at height d0 with angle theta to the plane
    Ov = np.array([[0.0, 0.0, d0]])
    D = np.array([[math.cos(th), 0.0, -math.sin(th)]])

    def plane(idx, P):
        return P[:, 2]

    st = O.new_state(Ov, D, np.zeros(1), np.array([-1e9]), np.array([1e9]),
                     np.array([O.ACTIVE]), 1, np.array([np.inf]))
    O.march(plane, st, 0, 200, alpha, eps, 200)
    assert st.status[0] == O.HIT
    updates = int(st.nsteps[0]) - 1       # queries minus the converging one
    assert updates == want
    assert math.ceil(O.k_min(eps, d0, alpha, th)) == want


def test_eps_worked_example():
    """App. A.2: eps = d_min S cos^2 / (2 f R) ~ 0.5e-4 m; Sec. 3.2: 2 eps ~ 1e-4 m."""
    g = load_golden("worked_examples.txt")
    e = O.eps_for_camera(g["eps.dmin_m"], g["eps.sensor_m"], g["eps.focal_m"], int(g["eps.res"]))
    assert abs(e - g["eps.approx_m"]) / g["eps.approx_m"] < 0.05
    assert abs(2 * e - g["spacing.approx_m"]) / g["spacing.approx_m"] < 0.05
    assert abs(e - 5.2083333e-5) < 1e-10


# ----------------------------------------------------------------------------
# Analytic base field: output layer zeroed -> f = 0.5 (|p| - 0.5)
# ----------------------------------------------------------------------------
def _base_decoder(spec=di.C1_SPEC):
    Ws, bs = di.make_decoder(spec, seed=0)
    Ws[-1][:] = 0.0
    return O.Decoder(spec, Ws, bs)


@pytest.mark.parametrize("c2f,alpha,H", [(0, 1.0, 32), (2, 1.5, 32), (1, 1.5, 24)])
def test_base_field_closed_forms(c2f, alpha, H):
    spec = di.C1_SPEC
    dec = _base_decoder(spec)
    z = di.make_latents(1, spec.latent_dim)
    cam = di.front_camera(H, H)
    prm = _prm(alpha=alpha, eps=1e-3, max_steps=40, c2f_levels=c2f, want_normals=1)
    r = O.render(dec, z, [cam], [(0, 0)], prm)[0]
    depth_t, normal_t, sil_t = di.sphere_target_maps(cam, 0.5)

    hit = r.status == O.HIT
    assert hit.sum() > 50
    # fg <=> S < 0 <=> HIT (the silhouette sign rule of Sec. 3.3)
    assert np.array_equal(r.sil < 0, hit)
    # |f| at every hit < eps, and the hit point is within 2 eps of the 0.5-sphere
    R = cam.R_wc.astype(np.float64)
    c = cam.c.astype(np.float64)
    d = r.dist[hit]
    dirs = r.dirs.reshape(H, H, 3)[hit]
    P = c + d[:, None] * dirs
    assert np.all(np.abs(np.linalg.norm(P, axis=1) - 0.5) < 2.0 * prm.eps * (1 + 1e-9))
    # depth = camera-frame z of the hit point (independent of the 1/sqrt formula)
    zc = ((P - c) @ R)[:, 2]
    np.testing.assert_allclose(r.depth[hit], zc, rtol=0, atol=1e-12)
    # closed-form sphere depth: |d - t*| <= 2 eps / s with s = -v . p_hat at the root
    t_star = depth_t[hit].astype(np.float64) * np.sqrt(r.xt.reshape(H, H)[hit] ** 2 + r.yt.reshape(H, H)[hit] ** 2 + 1)
    proot = c + t_star[:, None] * dirs
    s = -np.sum(dirs * proot / 0.5, axis=1)
    ok = s > 0.05
    assert np.all(np.abs(d - t_star)[ok] <= 2.0 * prm.eps / s[ok] + 1e-6)
    # hit pixels off the closed-form sphere are the eps-dilation of App. A.2: their
    # ray passes the origin closer than 0.5 + 2 eps
    off = sil_t[hit] < 0.5
    perp_h = c - (dirs @ c)[:, None] * dirs
    assert np.all(np.linalg.norm(perp_h[off], axis=1) < 0.5 + 2 * prm.eps)
    # normals: central differences of 0.5|p| point along p
    n = r.normal[hit]
    cosang = np.sum(n * P / np.linalg.norm(P, axis=1, keepdims=True), axis=1)
    assert np.all(cosang > 1 - 1e-6)
    # MISS: S + 1 = distance of the ray line from the origin = |c - (c.v) v|
    miss = r.status == O.MISS
    assert miss.sum() > 0
    dm = r.dirs.reshape(H, H, 3)[miss]
    perp = c - (dm @ c)[:, None] * dm
    np.testing.assert_allclose(r.sil[miss] + 1.0, np.linalg.norm(perp, axis=1), rtol=0, atol=1e-12)
    # S inside the sphere is min |f| - eps over the pixel's queries, and min |f| >= 0
    ins = ~miss
    assert np.all(r.sil[ins] >= -prm.eps)
    # per-step query counts add up
    assert sum(r.queries_per_step) == r.queries


def test_base_field_trajectory_is_monotone_and_bounded():
    """On f0 = 0.5(|p| - 0.5) with alpha * Lip(f0) = 0.75 < 1 the march is a
    contraction towards the first root: t increases and never passes the root."""
    dec = _base_decoder()
    cam = di.front_camera(16, 16)
    prm = _prm(alpha=1.5, eps=1e-4, max_steps=60, c2f_levels=0, want_normals=0)
    z = di.make_latents(1, 64)
    r = O.render(dec, z, [cam], [(0, 0)], prm)[0]
    depth_t, _, _ = di.sphere_target_maps(cam, 0.5)
    hit = r.status == O.HIT
    t_star = depth_t[hit] * np.sqrt(r.xt.reshape(16, 16)[hit] ** 2 + r.yt.reshape(16, 16)[hit] ** 2 + 1)
    # the last query t stays in front of the root (f > 0 side) for head-on rays
    rec_t = r.rec_t[0].reshape(16, 16)[hit]
    assert np.all(rec_t <= t_star + 1e-9)
    # and the number of queries follows the scalar contraction |f_{n+1}| <= 0.75 |f_n| bound
    assert np.all(r.nsteps[hit] <= 60)


# ----------------------------------------------------------------------------
# Linear-regime decoder: m(z, p) = a + u.z exactly -> sphere of radius R(z)
# ----------------------------------------------------------------------------
def _linear_decoder(spec):
    rng = np.random.Generator(np.random.PCG64(7))
    Ws, bs = di.make_decoder(spec, seed=0)
    L = spec.latent_dim
    Ws2, bs2 = [], []
    for l, (W, b) in enumerate(zip(Ws, bs)):
        W = np.abs(W).astype(np.float64) * 0.3
        if l == 0:
            W[:, L:] = 0.0                                  # no point dependence
        if spec.skip_layer is not None and l == spec.skip_layer:
            W[:, -3:] = 0.0
        b = 0.5 + rng.random(W.shape[0])
        if l == len(Ws) - 1:
            b = np.array([0.0])
        Ws2.append(W)
        bs2.append(b)
    dec = O.Decoder(spec, Ws2, bs2)
    # scale the output layer so that m(0) = 0.3: tanh stays in its sloped range
    m0, _, _ = dec.layer_inputs(np.zeros((1, L)), np.zeros((1, 3)), keep=False)
    dec.W[-1] *= 0.1 / m0[0]
    dec.b[-1][:] = 0.2
    return dec


@pytest.mark.parametrize("spec", [di.C1_SPEC, di.DEEPSDF_SPEC], ids=["c1", "deepsdf"])
def test_linear_regime_depth_and_gradient_closed_form(spec):
    dec = _linear_decoder(spec)
    L = spec.latent_dim
    z = di.make_latents(1, L, sigma=0.01)
    z64 = z[0].astype(np.float64)
    # m is affine in z: recover (a, u) from the forward at z = 0 and z = e_j (exact for affine maps)
    P0 = np.zeros((L + 1, 3))
    Zs = np.vstack([np.zeros(L), np.eye(L)])
    m_all, _, _ = dec.layer_inputs(Zs, P0, keep=False)
    a = m_all[0]
    u = m_all[1:] - a
    mz = a + u @ z64
    Rz = 0.5 - 0.1 * math.tanh(mz)
    # f = 0.5(|p| - 0.5) + 0.05 tanh(mz) = 0.5 (|p| - Rz): a sphere of radius Rz
    H = 24
    cam = di.front_camera(H, H)
    prm = _prm(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=1, want_normals=0, k_samples=1)
    r = O.render(dec, z, [cam], [(0, 0)], prm)[0]
    depth_t, _, sil_t = di.sphere_target_maps(cam, Rz)
    hit = r.status == O.HIT
    assert hit.sum() > 100
    nrm = np.sqrt(r.xt.reshape(H, H) ** 2 + r.yt.reshape(H, H) ** 2 + 1)
    t_star = depth_t[hit] * nrm[hit]
    dirs = r.dirs.reshape(H, H, 3)[hit]
    proot = cam.c.astype(np.float64) + t_star[:, None] * dirs
    s = -np.sum(dirs * proot / Rz, axis=1)
    ok = s > 0.1
    assert np.all(np.abs(r.dist[hit] - t_star)[ok] <= 2 * prm.eps / s[ok] + 1e-6)
    # paper gradient of an L1 depth loss (K = 1): every hit pixel contributes
    # alpha * g_d / |(xt,yt,1)| * df/dz with df/dz = 0.05 sech^2(mz) u for all p.
    dt = np.where(sil_t > 0.5, depth_t + 0.01, np.inf).astype(np.float32)
    _, g_d, g_n, g_s = O.loss_and_grads(r, dt, np.zeros((H, H, 3)), sil_t, w_d=10.0, w_s=0.0)
    gz, _, _ = O.backward(dec, z, [r], [(0, 0)], prm, [(g_d, g_n, g_s)], want_theta=False)
    seed_sum = prm.alpha * np.sum(g_d[hit] / nrm[hit])
    expect = 0.05 * (1 - math.tanh(mz) ** 2) * u * seed_sum
    np.testing.assert_allclose(gz[0], expect, rtol=1e-9, atol=1e-15)
    assert np.linalg.norm(expect) > 0


# ----------------------------------------------------------------------------
# Brute force: dense marching on tiny images
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("spec,H,dt", [(di.C1_SPEC, 16, 2e-3), (di.DEEPSDF_SPEC, 8, 4e-3)],
                         ids=["c1-16", "deepsdf-8"])
def test_brute_force_dense_march(spec, H, dt):
    Ws, bs = di.make_decoder(spec, seed=0)
    dec = O.Decoder(spec, Ws, bs)
    z = di.make_latents(1, spec.latent_dim)
    cam = di.front_camera(H, H)
    prm = _prm(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=0, want_normals=0)
    r = O.render(dec, z, [cam], [(0, 0)], prm)[0]
    c = cam.c.astype(np.float64)
    zz = z[0].astype(np.float64)

    def f(P):
        return dec.sdf(np.broadcast_to(zz, (P.shape[0], zz.size)), P)

    D = r.dirs
    b = D @ c
    disc = b * b - (c @ c - 1)
    n_checked = 0
    for i in range(H * H):
        if disc[i] <= 0:
            assert r.status.reshape(-1)[i] == O.MISS
            continue
        t0, t1 = -b[i] - math.sqrt(disc[i]), -b[i] + math.sqrt(disc[i])
        ts = np.arange(t0, t1, dt)
        fv = f(c + ts[:, None] * D[i])
        sc = np.nonzero(np.sign(fv[:-1]) != np.sign(fv[1:]))[0]
        st = r.status.reshape(-1)[i]
        if sc.size == 0:
            # no crossing: the ray may only be foreground if it came within eps of the surface
            if st == O.HIT:
                assert np.min(np.abs(fv)) < 5 * prm.eps
            continue
        lo, hi = ts[sc[0]], ts[sc[0] + 1]
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if np.sign(f((c + mid * D[i])[None])[0]) == np.sign(fv[sc[0]]):
                lo = mid
            else:
                hi = mid
        t_bf = 0.5 * (lo + hi)
        if st != O.HIT:
            continue       # erosion at grazing rays (App. A.2) is allowed
        g = np.zeros(3)
        p = c + t_bf * D[i]
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1e-5
            g[k] = (f((p + e)[None])[0] - f((p - e)[None])[0]) / 2e-5
        s = abs(g @ D[i])
        assert abs(r.dist.reshape(-1)[i] - t_bf) <= (prm.eps / s) * (1 + s) + 1e-9
        n_checked += 1
    assert n_checked > H * H // 8


# ----------------------------------------------------------------------------
# VJP: hand-derived chain rule vs central differences and vs torch autograd
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("spec", [di.C1_SPEC, di.DEEPSDF_SPEC], ids=["c1", "deepsdf"])
def test_vjp_against_central_differences(spec):
    Ws, bs = di.make_decoder(spec, seed=0)
    rng = np.random.Generator(np.random.PCG64(11))
    bs = [(rng.standard_normal(b.shape) * 0.05).astype(np.float32) for b in bs]
    dec = O.Decoder(spec, Ws, bs)
    n = 16
    Z = rng.standard_normal((n, spec.latent_dim)) * 0.3
    P = rng.uniform(-0.6, 0.6, (n, 3))
    seeds = rng.standard_normal(n)
    gZ, gW, gb = dec.sdf_vjp(Z, P, seeds)
    h = 1e-6
    for j in rng.choice(spec.latent_dim, 8, replace=False):
        Zp, Zm = Z.copy(), Z.copy()
        Zp[:, j] += h
        Zm[:, j] -= h
        fd = (dec.sdf(Zp, P) - dec.sdf(Zm, P)) / (2 * h) * seeds
        np.testing.assert_allclose(gZ[:, j], fd, rtol=1e-6, atol=1e-9)
    # weights and biases of every layer, a few entries each
    for l in range(dec.nl):
        for _ in range(3):
            o = rng.integers(dec.W[l].shape[0])
            i = rng.integers(dec.W[l].shape[1])
            Wsave = dec.W[l][o, i]
            dec.W[l][o, i] = Wsave + h
            fp = dec.sdf(Z, P) @ seeds
            dec.W[l][o, i] = Wsave - h
            fm = dec.sdf(Z, P) @ seeds
            dec.W[l][o, i] = Wsave
            assert abs((fp - fm) / (2 * h) - gW[l][o, i]) <= 1e-6 * max(1.0, abs(gW[l][o, i]))
        o = rng.integers(dec.b[l].shape[0])
        bsave = dec.b[l][o]
        dec.b[l][o] = bsave + h
        fp = dec.sdf(Z, P) @ seeds
        dec.b[l][o] = bsave - h
        fm = dec.sdf(Z, P) @ seeds
        dec.b[l][o] = bsave
        assert abs((fp - fm) / (2 * h) - gb[l][o]) <= 1e-6 * max(1.0, abs(gb[l][o]))


def test_vjp_against_torch_autograd():
    torch = pytest.importorskip("torch")
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    dec = O.Decoder(spec, Ws, bs)
    rng = np.random.Generator(np.random.PCG64(12))
    n = 32
    Z = rng.standard_normal((n, spec.latent_dim)) * 0.1
    P = rng.uniform(-0.6, 0.6, (n, 3))
    seeds = rng.standard_normal(n)
    gZ, gW, _ = dec.sdf_vjp(Z, P, seeds)
    Zt = torch.tensor(Z, requires_grad=True)
    Pt = torch.tensor(P)
    Wt = [torch.tensor(W.astype(np.float64), requires_grad=True) for W in Ws]
    x = torch.cat([Zt, Pt], 1)
    h = x
    for l, W in enumerate(Wt):
        inp = torch.cat([h, Zt, Pt], 1) if l == spec.skip_layer else h
        a = inp @ W.T
        h = torch.relu(a) if l < len(Wt) - 1 else a
    f = 0.5 * (Pt.norm(dim=1) - 0.5) + 0.05 * torch.tanh(h[:, 0])
    (f * torch.tensor(seeds)).sum().backward()
    np.testing.assert_allclose(gZ, Zt.grad.numpy(), rtol=1e-10, atol=1e-14)
    for l in range(len(Wt)):
        np.testing.assert_allclose(gW[l], Wt[l].grad.numpy(), rtol=1e-10, atol=1e-14)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.Generator(np.random.PCG64(3))
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-6, 3, 5000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0])])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O._bf16_round(x), ref)


# ----------------------------------------------------------------------------
# Seeds of the silhouette loss (App. A.3) and the sample rule (Sec. 3.4)
# ----------------------------------------------------------------------------
def test_silhouette_hinge_gradient_by_finite_differences():
    """dL/dS of the hinge loss of App. A.3 against central differences of the loss."""
    rng = np.random.Generator(np.random.PCG64(5))
    H = 8
    S = rng.uniform(-0.1, 0.1, (H, H))
    St = (rng.random((H, H)) > 0.5).astype(np.float64)
    r = O.Render(H=H, W=H, depth=np.ones((H, H)), dist=np.ones((H, H)),
                 normal=np.zeros((H, H, 3)), nraw=np.zeros((H, H, 3)), sil=S,
                 status=np.full((H, H), O.ESCAPED, np.int8), nsteps=np.zeros((H, H), np.int32),
                 margin=np.zeros((H, H)), xt=np.zeros(H * H), yt=np.zeros(H * H), dirs=np.zeros((H * H, 3)),
                 c=np.zeros(3), rec_absf=np.zeros((1, H * H)), rec_t=np.zeros((1, H * H)),
                 rec_f=np.zeros((1, H * H)), rec_n=np.zeros((1, H * H), np.int32), queries=0)
    L0, _, _, g_s = O.loss_and_grads(r, np.zeros((H, H)), np.zeros((H, H, 3)), St, w_d=0, w_s=1.0)
    h = 1e-7
    for _ in range(10):
        i, j = rng.integers(H), rng.integers(H)
        r.sil[i, j] += h
        Lp = O.loss_and_grads(r, np.zeros((H, H)), np.zeros((H, H, 3)), St, w_d=0, w_s=1.0)[0]
        r.sil[i, j] -= 2 * h
        Lm = O.loss_and_grads(r, np.zeros((H, H)), np.zeros((H, H, 3)), St, w_d=0, w_s=1.0)[0]
        r.sil[i, j] += h
        assert abs((Lp - Lm) / (2 * h) - g_s[i, j]) < 1e-6


def test_normal_seeds_match_finite_differences_of_normal_loss():
    """The six normal samples with seeds +-(I - nn^T) g / (|n| 2 delta) reproduce the
    derivative of the normal loss -n~ . n~* through the central-difference normal."""
    spec = di.C1_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    dec = O.Decoder(spec, Ws, bs)
    H = 12
    cam = di.front_camera(H, H)
    z = di.make_latents(1, spec.latent_dim)
    prm = _prm(alpha=1.5, eps=1e-3, max_steps=30, c2f_levels=0, want_normals=1)
    r = O.render(dec, z, [cam], [(0, 0)], prm)[0]
    _, nt, st = di.sphere_target_maps(cam, 0.5)
    _, g_d, g_n, g_s = O.loss_and_grads(r, np.zeros((H, H)), nt, st, w_d=0.0, w_s=0.0, w_n=1.0)
    gz, _, _ = O.backward(dec, z, [r], [(0, 0)], prm, [(np.zeros_like(g_d), g_n, np.zeros_like(g_s))],
                          want_theta=False)
    # surrogate: points frozen, normals recomputed from the decoder at z +- h e_j
    hit = (r.status == O.HIT).reshape(-1)
    p = r.c + r.dist.reshape(-1)[hit, None] * r.dirs[hit]
    fg = ((r.sil < 0) & (st > 0.5)).reshape(-1)[hit]
    ntf = nt.reshape(-1, 3)[hit]

    def loss(zv):
        fn = lambda P: dec.sdf(np.broadcast_to(zv, (P.shape[0], zv.size)), P)
        n = O.surface_normals(fn, p, prm.normal_delta)
        n = n / np.linalg.norm(n, axis=1, keepdims=True)
        return -(np.sum(n * ntf, axis=1) * fg).sum() / (H * H)

    h = 1e-6      # small enough that no ReLU kink is crossed by the perturbation
    z0 = z[0].astype(np.float64)
    for j in range(0, spec.latent_dim, 9):
        zp, zm = z0.copy(), z0.copy()
        zp[j] += h
        zm[j] -= h
        fd = (loss(zp) - loss(zm)) / (2 * h)
        assert abs(fd - gz[0, j]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


def test_subset_render_equals_full_render():
    """Tracing only a subset of pixels (with their coarse ancestors) reproduces
    the full render exactly at those pixels (self-consistency of the C2F chain)."""
    spec = di.C1_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    dec = O.Decoder(spec, Ws, bs)
    z = di.make_latents(1, spec.latent_dim)
    cam = di.front_camera(32, 32)
    prm = _prm(alpha=1.5, eps=5e-4, max_steps=30, c2f_levels=2, want_normals=1, k_samples=3)
    full = O.render(dec, z, [cam], [(0, 0)], prm)[0]
    pix = np.random.Generator(np.random.PCG64(1)).choice(32 * 32, 50, replace=False)
    sub = O.render(dec, z, [cam], [(0, 0)], prm, pixels=[pix])[0]
    # discrete decisions exactly; values up to BLAS rounding order (batch size differs)
    for name in ("status", "nsteps"):
        np.testing.assert_array_equal(getattr(sub, name).reshape(-1)[pix], getattr(full, name).reshape(-1)[pix])
    np.testing.assert_array_equal(sub.rec_n[:, pix], full.rec_n[:, pix])
    for name in ("depth", "sil"):
        np.testing.assert_allclose(getattr(sub, name).reshape(-1)[pix], getattr(full, name).reshape(-1)[pix],
                                   rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(sub.rec_t[:, pix], full.rec_t[:, pix], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(sub.normal.reshape(-1, 3)[pix], full.normal.reshape(-1, 3)[pix], rtol=0, atol=1e-9)


def test_adam_step_matches_torch_adam():
    """The oracle's Adam (paper's optimiser) against torch.optim.Adam, float64."""
    import torch
    rng = np.random.Generator(np.random.PCG64(21))
    z = rng.standard_normal(7)
    zt = torch.tensor(z.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([zt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(7)
    v = np.zeros(7)
    for t in range(1, 6):
        g = rng.standard_normal(7) * (10.0 ** -t)
        z, m, v = O.adam_step(z, g, m, v, t)
        opt.zero_grad()
        zt.grad = torch.tensor(g)
        opt.step()
        assert np.allclose(z, zt.detach().numpy(), rtol=0, atol=1e-14)


# ----------------------------------------------------------------------------
# camera-extrinsic gradient (detached march points)
# ----------------------------------------------------------------------------
def test_grad_p_against_autograd_and_differences():
    torch = pytest.importorskip("torch")
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    dec = O.Decoder(spec, Ws, bs)
    rng = np.random.Generator(np.random.PCG64(22))
    n = 24
    Z = rng.standard_normal((n, spec.latent_dim)) * 0.1
    P = rng.uniform(-0.6, 0.6, (n, 3))
    seeds = rng.standard_normal(n)
    gP = dec.sdf_grad_p(Z, P, seeds)
    Pt = torch.tensor(P, requires_grad=True)
    Zt = torch.tensor(Z)
    h = torch.cat([Zt, Pt], 1)
    for l, W in enumerate(Ws):
        Wt = torch.tensor(W.astype(np.float64))
        inp = torch.cat([h, Zt, Pt], 1) if l == spec.skip_layer else h
        a = inp @ Wt.T
        h = torch.relu(a) if l < len(Ws) - 1 else a
    f = 0.5 * (Pt.norm(dim=1) - 0.5) + 0.05 * torch.tanh(h[:, 0])
    (f * torch.tensor(seeds)).sum().backward()
    np.testing.assert_allclose(gP, Pt.grad.numpy(), rtol=1e-10, atol=1e-14)
    e = 1e-6
    for i in range(3):
        Pp, Pm = P.copy(), P.copy()
        Pp[:, i] += e
        Pm[:, i] -= e
        fd = (dec.sdf(Z, Pp) - dec.sdf(Z, Pm)) / (2 * e) * seeds
        np.testing.assert_allclose(gP[:, i], fd, rtol=1e-6, atol=1e-9)


def test_camera_gradient_against_frozen_sample_differences():
    """dL/d(c, R) of the oracle against central differences of the surrogate in
    which the samples keep their seeds, ray parameters t and pixel directions u
    (p = c + t R u) and background pixels keep S = sqrt(|c|^2 - (c.Ru)^2) - 1."""
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    dec = O.Decoder(spec, Ws, bs)
    prm = di.TraceParams(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=1, k_samples=2, precision=0, want_normals=0)
    cams = di.random_sphere_cameras(2, 12, 12)
    Z = di.make_latents(1, spec.latent_dim, sigma=0.05)
    pairs = [(0, 0), (1, 0)]
    rs = O.render(dec, Z, cams, pairs, prm)
    grads = []
    for r, (v, _) in zip(rs, pairs):
        dt, nt, st = di.sphere_target_maps(cams[v], 0.45)
        _, gd, _, gs = O.loss_and_grads(r, dt, nt, st, w_d=10.0, w_s=1.0)
        grads.append((gd, gs))
    g_c, g_R = O.camera_backward(dec, Z, rs, cams, pairs, prm, grads)
    assert np.linalg.norm(g_c) > 0 and np.linalg.norm(g_R) > 0
    for vi in range(2):
        r, (gd, gs) = rs[vi], grads[vi]
        P, s, t, u = O.camera_samples(r, prm, gd, gs)
        gsf = np.asarray(gs).reshape(-1)
        miss = (r.status.reshape(-1) == O.MISS) & (gsf != 0)
        nrm = np.sqrt(r.xt[miss] ** 2 + r.yt[miss] ** 2 + 1.0)
        um = np.stack([r.xt[miss] / nrm, r.yt[miss] / nrm, 1.0 / nrm], axis=1)
        R0 = cams[vi].R_wc.astype(np.float64).reshape(3, 3)
        c0 = r.c.copy()

        def surrogate(c, R):
            p = c[None, :] + t[:, None] * (u @ R.T)
            val = np.dot(s, dec.sdf(np.broadcast_to(Z[0], (p.shape[0], Z.shape[1])), p)) if p.shape[0] else 0.0
            v = um @ R.T
            b = v @ c
            dist = np.where(b < 0, np.sqrt(c @ c - b * b), np.sqrt(c @ c))
            return val + np.dot(gsf[miss], dist - 1.0)

        # a step of 1e-7 keeps every ReLU unit on its side (1e-6 already
        # crosses a kink for one of these samples); rounding stays ~1e-9
        e = 1e-7
        for i in range(3):
            cp, cm = c0.copy(), c0.copy()
            cp[i] += e
            cm[i] -= e
            fd = (surrogate(cp, R0) - surrogate(cm, R0)) / (2 * e)
            assert abs(fd - g_c[vi, i]) <= 1e-6 * max(1.0, abs(g_c[vi, i])) + 1e-9
        for i in range(3):
            for j in range(3):
                Rp, Rm = R0.copy(), R0.copy()
                Rp[i, j] += e
                Rm[i, j] -= e
                fd = (surrogate(c0, Rp) - surrogate(c0, Rm)) / (2 * e)
                assert abs(fd - g_R[vi, i, j]) <= 1e-6 * max(1.0, abs(g_R[vi, i, j])) + 1e-9


# ----------------------------------------------------------------------------
# exact (implicit-function) depth gradient
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("spec", [di.C1_SPEC, di.DEEPSDF_SPEC], ids=["c1", "deepsdf"])
def test_implicit_depth_gradient_closed_form(spec):
    """On the linear-regime decoder the surface is the sphere |p| = R(z),
    R = 0.5 - 0.1 tanh(a + u.z): the hit distance t* solves |c + t v| = R, so
    dt*/dz = -0.1 sech^2(m) u / (p_hat . v).  The oracle's implicit gradient
    equals that formula at its Eq. 1 points and the true derivative at the
    exact roots to within the convergence tolerance."""
    dec = _linear_decoder(spec)
    L = spec.latent_dim
    z = di.make_latents(1, L, sigma=0.01)
    z64 = z[0].astype(np.float64)
    P0 = np.zeros((L + 1, 3))
    Zs = np.vstack([np.zeros(L), np.eye(L)])
    m_all, _, _ = dec.layer_inputs(Zs, P0, keep=False)
    a, u = m_all[0], m_all[1:] - m_all[0]
    mz = a + u @ z64
    Rz = 0.5 - 0.1 * math.tanh(mz)
    H = 24
    cam = di.front_camera(H, H)
    prm = _prm(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=1, want_normals=0, k_samples=1)
    r = O.render(dec, z, [cam], [(0, 0)], prm)[0]
    depth_t, _, sil_t = di.sphere_target_maps(cam, Rz)
    dt = np.where(sil_t > 0.5, depth_t + 0.01, np.inf).astype(np.float32)
    _, g_d, g_n, g_s = O.loss_and_grads(r, dt, np.zeros((H, H, 3)), sil_t, w_d=10.0, w_s=0.0)
    gz = O.implicit_backward(dec, z, [r], [(0, 0)], prm, [(g_d, g_n, g_s)])[0]
    hit = (r.status == O.HIT).reshape(-1) & (g_d.reshape(-1) != 0)
    nrm = np.sqrt(r.xt[hit] ** 2 + r.yt[hit] ** 2 + 1)
    v = r.dirs[hit]
    sech2 = 1 - math.tanh(mz) ** 2
    # formula at the Eq. 1 points (what the oracle evaluates)
    p = cam.c.astype(np.float64) + r.dist.reshape(-1)[hit, None] * v
    pv = np.sum(p / np.linalg.norm(p, axis=1, keepdims=True) * v, axis=1)
    w = g_d.reshape(-1)[hit] / nrm
    expect = -0.1 * sech2 * u * np.sum(w / pv)
    np.testing.assert_allclose(gz, expect, rtol=1e-9, atol=1e-14)
    # the true derivative at the exact roots
    c = cam.c.astype(np.float64)
    b = v @ c
    t_star = -b - np.sqrt(b * b - (c @ c - Rz * Rz))
    ps = c[None, :] + t_star[:, None] * v
    true = -0.1 * sech2 * u * np.sum(w / np.sum(ps / Rz * v, axis=1))
    # the Eq. 1 point lies within eps / s of the root (s = -p_hat . v), which
    # moves 1 / (p_hat . v) by O(eps / (R s^2)) per pixel: 0.7% here
    assert np.linalg.norm(gz - true) <= 2e-2 * np.linalg.norm(true)
    # the paper's approximation differs (it omits the 1 / (grad f . v) factor)
    gp_, _, _ = O.backward(dec, z, [r], [(0, 0)], prm, [(g_d, g_n, g_s)], want_theta=False)
    assert np.linalg.norm(gp_[0] - gz) > 1e-2 * np.linalg.norm(gz)


def test_view_facing_away_is_background():
    """A camera outside the sphere looking away from it: the ray lines of some
    pixels cross the sphere behind the camera, but no ray meets it; every pixel
    is background with S = |c| - 1 - the distance from the origin to the ray
    (App. A.3) - and the camera gradient of S is c / |c| per pixel."""
    spec = di.C1_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    dec = O.Decoder(spec, Ws, bs)
    cam = di.front_camera(8, 8)
    R = cam.R_wc.astype(np.float64) @ np.diag([-1.0, 1.0, -1.0])
    away = di.Camera(cam.fx, cam.fy, cam.cx, cam.cy, R.astype(np.float32), cam.c, 8, 8)
    prm = _prm(alpha=1.0, eps=1e-3, max_steps=20, c2f_levels=0, want_normals=0, k_samples=1)
    Z = di.make_latents(1, spec.latent_dim)
    r = O.render(dec, Z, [away], [(0, 0)], prm)[0]
    c = away.c.astype(np.float64)
    assert np.all(r.status == O.MISS) and r.queries == 0
    # some pixel lines do cross the sphere (behind the camera)
    b = r.dirs @ c
    assert np.any(b * b - (c @ c - 1.0) > 0)
    np.testing.assert_allclose(r.sil, np.linalg.norm(c) - 1.0, rtol=0, atol=1e-15)
    gs = np.full((8, 8), 0.5)
    g_c, g_R = O.camera_backward(dec, Z, [r], [away], [(0, 0)], prm, [(np.zeros((8, 8)), gs)])
    np.testing.assert_allclose(g_c[0], 64 * 0.5 * c / np.linalg.norm(c), rtol=1e-12)
    assert np.all(g_R == 0)


# ----------------------------------------------------------------------------
# exact gradient through the unrolled march (Eq. 2 with both terms)
# ----------------------------------------------------------------------------
def _render_loss(r, g_d, g_s):
    hit = r.status == O.HIT
    return float(np.sum(np.where(hit, g_d * np.where(hit, r.depth, 0.0), 0.0))
                 + np.sum(np.where(r.status != O.MISS, g_s * np.where(r.status != O.MISS, r.sil, 0.0), 0.0)))


@pytest.mark.parametrize("spec,c2f", [(di.C1_SPEC, 0), (di.C1_SPEC, 1), (di.DEEPSDF_SPEC, 1)],
                         ids=["c1", "c1-c2f", "deepsdf-c2f"])
def test_unrolled_gradient_against_render_differences(spec, c2f):
    """The unrolled derivative (Eq. 2, both terms, carried through every step
    and the coarse-to-fine splits) equals central differences of the oracle's
    own render along a random direction in z, on the pixels whose discrete
    trajectory (status, step count, minimum-|f| step) is the same at z +- h u
    and whose decisions are not within 1e-5 of a threshold.  The difference
    shrinks in proportion to h (a ReLU unit of some query changing side within
    the step), so h is small: 1e-8, where rounding of the loss adds ~5e-8."""
    Ws, bs = di.make_decoder(spec, seed=0)
    dec = O.Decoder(spec, Ws, bs)
    z = di.make_latents(1, spec.latent_dim, sigma=0.05).astype(np.float64)
    H = 16
    cam = di.look_at_camera((0.4, -0.3, 1.9), H, H, fov_deg=45.0)
    prm = _prm(alpha=1.5, eps=1e-3, max_steps=30, c2f_levels=c2f, want_normals=0, k_samples=1)
    rng = np.random.Generator(np.random.PCG64(11))
    u = rng.standard_normal(spec.latent_dim)
    u /= np.linalg.norm(u)
    h = 1e-8
    r0, rp, rm = (O.render(dec, zz, [cam], [(0, 0)], prm)[0] for zz in (z, z + h * u, z - h * u))
    same = ((r0.status == rp.status) & (r0.status == rm.status) & (r0.nsteps == rp.nsteps)
            & (r0.nsteps == rm.nsteps) & (r0.margin > 1e-5))
    same &= (r0.rec_n[0] == rp.rec_n[0]).reshape(H, H) & (r0.rec_n[0] == rm.rec_n[0]).reshape(H, H)
    g_d = rng.standard_normal((H, H)) * same
    g_s = rng.standard_normal((H, H)) * same
    fd = (_render_loss(rp, g_d, g_s) - _render_loss(rm, g_d, g_s)) / (2 * h)
    gz = O.unrolled_backward(dec, z, [cam], [(0, 0)], prm, [(g_d, g_s)])[0]
    assert int(same.sum()) > H * H // 4 and int((r0.status == O.HIT)[same].sum()) > 10
    assert abs(gz @ u - fd) <= 2e-6 * abs(fd) + 2e-7
    # the paper's first-term gradient is a different number here
    gp_ = O.backward(dec, z, [r0], [(0, 0)], prm, [(g_d, np.zeros((H, H, 3)), g_s)], want_theta=False)[0][0]
    assert abs(gp_ @ u - fd) > 1e-3 * abs(fd)


def test_unrolled_gradient_converges_to_the_implicit_one():
    """Marched to a tight threshold, the unrolled derivative of a hit's depth
    tends to the derivative of the exact root: on the linear-regime decoder
    (surface |p| = R(z)) dt*/dz = -0.1 sech^2(m) u / (p_hat . v)."""
    spec = di.C1_SPEC
    dec = _linear_decoder(spec)
    L = spec.latent_dim
    z = di.make_latents(1, L, sigma=0.01).astype(np.float64)
    P0 = np.zeros((L + 1, 3))
    m_all, _, _ = dec.layer_inputs(np.vstack([np.zeros(L), np.eye(L)]), P0, keep=False)
    a, uz = m_all[0], m_all[1:] - m_all[0]
    mz = a + uz @ z[0]
    Rz = 0.5 - 0.1 * math.tanh(mz)
    H = 12
    cam = di.front_camera(H, H)
    prm = _prm(alpha=1.0, eps=1e-10, max_steps=200, c2f_levels=0, want_normals=0, k_samples=1)
    r = O.render(dec, z, [cam], [(0, 0)], prm)[0]
    hit = r.status == O.HIT
    assert int(hit.sum()) > 20
    g_d = np.where(hit, 1.0, 0.0)
    gz = O.unrolled_backward(dec, z, [cam], [(0, 0)], prm, [(g_d, np.zeros((H, H)))])[0]
    h = hit.reshape(-1)
    v = r.dirs[h]
    c = cam.c.astype(np.float64)
    b = v @ c
    t_star = -b - np.sqrt(b * b - (c @ c - Rz * Rz))
    ps = c[None, :] + t_star[:, None] * v
    nrm = np.sqrt(r.xt[h] ** 2 + r.yt[h] ** 2 + 1)
    true = -0.1 * (1 - math.tanh(mz) ** 2) * uz * np.sum(1.0 / nrm / np.sum(ps / Rz * v, axis=1))
    assert np.linalg.norm(gz - true) <= 1e-6 * np.linalg.norm(true)


# ----------------------------------------------------------------------------
# multi-view photometric loss
# ----------------------------------------------------------------------------
def test_photometric_warp_of_an_identical_view_is_the_identity():
    """Warping a view into an identical camera lands every surface point on its
    own pixel centre: the warped image is the source image, every foreground
    pixel whose 2x2 footprint lies inside the image is visible, and with a zero
    target image the loss is weight / (H W) times the source's colour sum."""
    H = 40
    cam = di.ring_cameras(8, H, H)[3]
    im = di.textured_sphere_images([cam], 0.45)[0]
    D = di.sphere_target_maps(cam, 0.45)[0]
    L, g = O.photometric_loss([cam, cam], [D, D], [np.zeros_like(im), im], [(0, 1)], weight=5.0)
    fg = np.isfinite(D)
    fg[:, -1] = False
    fg[-1, :] = False
    expect = 5.0 / (H * H) * float(im[fg].astype(np.float64).sum())
    assert abs(L - expect) <= 1e-5 * expect
    L2, g2 = O.photometric_loss([cam, cam], [D, D], [im, im], [(0, 1)])
    assert L2 <= 1e-5 * expect


def test_photometric_gradient_against_central_differences():
    """dL/d(depth) of the photometric loss against central differences of the
    loss in single depth values (step 1e-6), on random visible pixels."""
    H = 48
    cams = di.ring_cameras(8, H, H)
    im = di.textured_sphere_images(cams, 0.45, freq=4.0)
    D = [di.sphere_target_maps(c, 0.45)[0].astype(np.float64) * 1.003 for c in cams]
    pairs = [(i, (i + 1) % 8) for i in range(8)] + [(i, (i + 7) % 8) for i in range(8)]
    L, g = O.photometric_loss(cams, D, im, pairs)
    rng = np.random.Generator(np.random.PCG64(3))
    checked = 0
    for _ in range(60):
        v = int(rng.integers(8))
        nz = np.argwhere(np.abs(g[v]) > 1e-4)
        if nz.size == 0:
            continue
        y, x = nz[int(rng.integers(len(nz)))]
        h = 1e-6
        Dp = [d.copy() for d in D]
        Dm = [d.copy() for d in D]
        Dp[v][y, x] += h
        Dm[v][y, x] -= h
        fd = (O.photometric_loss(cams, Dp, im, pairs)[0] - O.photometric_loss(cams, Dm, im, pairs)[0]) / (2 * h)
        assert abs(fd - g[v][y, x]) <= 1e-5 * abs(g[v][y, x]) + 1e-9
        checked += 1
    assert checked >= 30


# ----------------------------------------------------------------------------
# colour network at the hit points
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("spec", [di.C1_COLOR_SPEC, di.COLOR_SPEC], ids=["c1", "deepsdf"])
def test_color_vjp_against_torch_autograd_and_differences(spec):
    """The colour network's VJP w.r.t. the code against torch float64 autograd
    of an independent torch forward, and against central differences."""
    torch = pytest.importorskip("torch")
    Ws, bs = di.make_decoder(spec, seed=3)
    dec = O.ColorDecoder(spec, Ws, bs)
    rng = np.random.Generator(np.random.PCG64(9))
    n = 40
    Z = np.repeat(rng.standard_normal((1, spec.latent_dim)) * 0.3, n, 0)
    P = rng.uniform(-0.6, 0.6, (n, 3))
    seeds = rng.standard_normal((n, 3))
    g = dec.color_vjp(Z, P, seeds).sum(0)
    Wt = [torch.tensor(np.asarray(W, np.float64)) for W in Ws]
    bt = [torch.tensor(np.asarray(b, np.float64)) for b in bs]
    z = torch.tensor(Z[0], requires_grad=True)
    Pt = torch.tensor(P)
    Zt = z[None, :].expand(n, -1)
    h = torch.cat([Zt, Pt], 1)
    for l in range(len(Wt)):
        x = torch.cat([h, Zt, Pt], 1) if (spec.skip_layer is not None and l == spec.skip_layer) else h
        a = x @ Wt[l].T + bt[l]
        h = torch.relu(a) if l < len(Wt) - 1 else a
    c = 0.5 * (1 + torch.tanh(h))
    (c * torch.tensor(seeds)).sum().backward()
    np.testing.assert_allclose(g, z.grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(dec.color(Z, P), c.detach().numpy(), rtol=1e-12, atol=1e-14)
    k = int(np.argmax(np.abs(g)))
    e = np.zeros(spec.latent_dim)
    e[k] = 1e-6
    fd = ((dec.color(Z + e, P) - dec.color(Z - e, P)) * seeds).sum() / 2e-6
    assert abs(fd - g[k]) <= 1e-6 * abs(g[k]) + 1e-9


# ----------------------------------------------------------------------------
# silhouette seed, coarse-to-fine schedule, bf16-rounding decoder
# ----------------------------------------------------------------------------
def test_silhouette_seed_against_frozen_point_differences():
    """Sec. 3.4 / App. A.3: S = min_n |f(p_n, z)| - eps, so with the minimising
    query p* held fixed dS/dz = sign f(p*) df(p*, z)/dz.  The oracle's backward
    given only dL/dS must equal central differences of the surrogate
    sum_pix g_S (|f(p*, z)| - eps), and p* must be the query of smallest |f|
    along the pixel's ray, found here by an independent scalar re-trace.  A
    dropped sign, the sign of another record or the point of another record
    fails this.  The step factor alpha = 2.5 makes many rays overshoot, so
    that many argmin queries have f < 0 (with the workloads' alpha = 1.5 the
    residual form never overshoots and every sign would be +1)."""
    spec = di.C1_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    dec = O.Decoder(spec, Ws, bs)
    H = 14
    cam = di.front_camera(H, H)
    z = di.make_latents(1, spec.latent_dim, sigma=0.05)
    prm = _prm(alpha=2.5, eps=1e-3, max_steps=30, c2f_levels=0, k_samples=3, want_normals=0)
    r = O.render(dec, z, [cam], [(0, 0)], prm)[0]
    z0 = z[0].astype(np.float64)
    fn = lambda P, zv=z0: dec.sdf(np.broadcast_to(zv, (P.shape[0], zv.size)), P)
    st = r.status.reshape(-1)
    # independent re-trace: one ray at a time, every query kept
    c = cam.c.astype(np.float64)
    inside = np.nonzero(st != O.MISS)[0]
    for q in inside:
        v = r.dirs[q]
        b = float(v @ c)
        t = -b - math.sqrt(b * b - (c @ c - 1.0))
        t_hi = -b + math.sqrt(b * b - (c @ c - 1.0))
        seen = []
        for n in range(prm.max_steps):
            f = float(fn((c + t * v)[None])[0])
            seen.append((abs(f), n, t))
            if abs(f) < prm.eps or n == prm.max_steps - 1:
                break
            t += prm.alpha * f
            if t > t_hi or t < -b - math.sqrt(b * b - (c @ c - 1.0)):
                break
        best = min(seen, key=lambda s: (s[0], s[1]))
        assert abs(best[0] - r.rec_absf[0, q]) <= 1e-12
        assert best[1] == r.rec_n[0, q]
        assert abs(best[2] - r.rec_t[0, q]) <= 1e-12
    rng = np.random.Generator(np.random.PCG64(31))
    g_s = rng.standard_normal((H, H)) / (H * H)
    gz, _, _ = O.backward(dec, z, [r], [(0, 0)], prm, [(np.zeros((H, H)), np.zeros((H, H, 3)), g_s)],
                          want_theta=False)
    sel = inside
    p_star = c[None, :] + r.rec_t[0, sel, None] * r.dirs[sel]
    neg = (r.rec_f[0, sel] < 0) & (st[sel] == O.HIT)
    assert neg.sum() >= 5, "the pin needs hits whose minimum-|f| query is negative"
    gsel = g_s.reshape(-1)[sel]

    def surrogate(zv):
        return float(np.dot(gsel, np.abs(fn(p_star, zv)) - prm.eps))

    h = 1e-7
    for j in range(0, spec.latent_dim, 5):
        zp, zm = z0.copy(), z0.copy()
        zp[j] += h
        zm[j] -= h
        fd = (surrogate(zp) - surrogate(zm)) / (2 * h)
        assert abs(fd - gz[0, j]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10, (j, fd, gz[0, j])


@pytest.mark.parametrize("H,L", [(32, 2), (48, 2), (40, 1)])
def test_coarse_to_fine_schedule_query_counts(H, L):
    """Sec. 3.2 coarse-to-fine: tracing starts at 1/2^L of the resolution per
    side and every ray splits into four after every three steps, every child
    that meets the unit sphere being traced again.  So on the analytic base
    field, where no ray converges within three steps of the sphere entry, the
    queries of step 0 count the level-L rays that meet the unit sphere, those of
    step 3 the level-(L-1) rays and those of step 6 the full-resolution rays.
    The counts come from the closed form of a camera at distance |c| looking at
    the origin: the ray through (xt, yt) meets the unit sphere iff
    xt^2 + yt^2 < 1 / (|c|^2 - 1)."""
    dec = _base_decoder()
    z = di.make_latents(1, di.C1_SPEC.latent_dim)
    cam = di.front_camera(H, H)
    prm = _prm(alpha=1.5, eps=1e-3, max_steps=12, c2f_levels=L, want_normals=0)
    r = O.render(dec, z, [cam], [(0, 0)], prm)[0]
    cc = float(np.sum(cam.c.astype(np.float64) ** 2))

    def meeting(level):
        s = 2 ** level
        ctr = s * np.arange(H // s, dtype=np.float64) + 0.5 * s
        xt = (ctr[None, :] - cam.cx) / cam.fx
        yt = (ctr[:, None] - cam.cy) / cam.fy
        return int(np.sum(xt * xt + yt * yt < 1.0 / (cc - 1.0)))

    for seg in range(L + 1):
        assert r.queries_per_step[3 * seg] == meeting(L - seg), (seg, r.queries_per_step)
    # between the splits the count only falls (rays stop, none start)
    for n in range(1, prm.max_steps):
        if n % 3 or n > 3 * L:
            assert r.queries_per_step[n] <= r.queries_per_step[n - 1]


@pytest.mark.parametrize("spec", [di.C1_SPEC, di.DEEPSDF_SPEC], ids=["c1", "deepsdf"])
def test_bf16_emulated_decoder_matches_torch_bfloat16(spec):
    """The bf16-rounding oracle decoder against an independent torch
    evaluation: hidden-layer products take torch.bfloat16 casts of the input
    activations and of the hidden part of the weights (exact float64
    products and sums); layer 0, the skip layer's [z, p] columns, biases and the
    output layer stay float64."""
    torch = pytest.importorskip("torch")
    Ws, bs = di.make_decoder(spec, seed=0)
    rng = np.random.Generator(np.random.PCG64(41))
    bs = [rng.standard_normal(b.shape).astype(np.float32) * 0.1 for b in bs]
    emu = O.DecoderBF16Emulated(spec, Ws, bs)
    n = 64
    Z = rng.standard_normal((n, spec.latent_dim)) * 0.1
    P = rng.uniform(-0.6, 0.6, (n, 3))
    got = emu.sdf(Z, P)

    def r16(x):
        return x.to(torch.bfloat16).to(torch.float64)

    Zt, Pt = torch.tensor(Z), torch.tensor(P)
    zp = torch.cat([Zt, Pt], 1)
    nl = len(Ws)
    h = None
    for l in range(nl):
        W = torch.tensor(Ws[l].astype(np.float64))
        b = torch.tensor(bs[l].astype(np.float64))
        if l == 0:
            a = zp @ W.T + b
        elif l == nl - 1:
            a = h @ W.T + b
        elif spec.skip_layer is not None and l == spec.skip_layer:
            nh = Ws[l - 1].shape[0]
            a = r16(h) @ r16(W[:, :nh]).T + zp @ W[:, nh:].T + b
        else:
            a = r16(h) @ r16(W).T + b
        h = torch.relu(a) if l < nl - 1 else a
    want = (0.5 * (Pt.norm(dim=1) - 0.5) + 0.05 * torch.tanh(h[:, 0])).numpy()
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    # and it is not the float64 decoder
    assert np.abs(got - O.Decoder(spec, Ws, bs).sdf(Z, P)).max() > 1e-6
