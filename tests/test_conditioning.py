"""How well-conditioned each term of the paper gradient is (CPU, oracle only).

These measurements back the bounds the GPU gradient tests can assert.  The
paper gradient (Sec. 3.4, Eq. 2 first term) is taken at detached sample
points, and df/dz of a ReLU network jumps wherever a unit changes side, so a
term whose samples each count on their own -- the normal term (a central
difference over +-delta, Sec. 3.3, seeded +-dL/dn / 2 delta) and the
silhouette term at hit pixels (seeds dL/dS sign f) -- moves by a finite
amount when the samples move by the rounding of a reduced-precision march.
Nothing here touches the GPU path.
"""
import numpy as np
import pytest

import dist_inputs as di
from oracle import dist_oracle as O
from _common import cfg_params, oracle_decoder, well_conditioned


def _setup(prm, H=32, n_views=1, n_lat=2):
    spec = di.DEEPSDF_SPEC
    cams = di.random_sphere_cameras(n_views, H, H)
    Z = di.make_latents(n_lat, spec.latent_dim, sigma=0.05)
    pairs = [(i // n_lat, i % n_lat) for i in range(n_views * n_lat)]
    return spec, cams, Z, pairs


def _grad(dec, Z, rs, pairs, prm, cams, w, keep=None):
    grads = []
    for i, (r, (v, l)) in enumerate(zip(rs, pairs)):
        dt, nt, stt = di.sphere_target_maps(cams[v], 0.5)
        _, g_d, g_n, g_s = O.loss_and_grads(r, dt, nt, stt, w_d=w[0], w_s=w[1], w_n=w[2])
        if keep is not None:
            g_d, g_s, g_n = g_d * keep[i], g_s * keep[i], g_n * keep[i][..., None]
        grads.append((g_d, g_n, g_s))
    return O.backward(dec, Z, rs, pairs, prm, grads, want_theta=False)[0]


def test_relu_margin_against_an_independent_forward():
    """Decoder.relu_margin is the smallest |pre-activation| of the hidden
    units: checked against a torch forward written here from the layer
    layout (z, p at layer 0; [h, z, p] at the skip layer)."""
    torch = pytest.importorskip("torch")
    spec = di.DEEPSDF_SPEC
    Ws, bs = di.make_decoder(spec, seed=0)
    dec = O.Decoder(spec, Ws, bs)
    rng = np.random.Generator(np.random.PCG64(3))
    P = rng.uniform(-0.6, 0.6, (64, 3))
    Z = rng.normal(0, 0.05, (64, spec.latent_dim))
    x0 = torch.tensor(np.concatenate([Z, P], 1))
    h = x0
    mins = []
    for l in range(len(Ws)):
        x = torch.cat([h, x0], 1) if l == spec.skip_layer else h
        a = x @ torch.tensor(np.asarray(Ws[l], np.float64)).T + torch.tensor(np.asarray(bs[l], np.float64))
        if l < len(Ws) - 1:
            mins.append(a.abs().min(1).values)
            h = torch.relu(a)
    want = torch.stack(mins, 1).min(1).values.numpy()
    np.testing.assert_allclose(dec.relu_margin(Z, P), want, rtol=1e-12, atol=0)


def test_normal_term_is_ill_conditioned_under_float32_rounding():
    """Moving the hit distances by 3e-7 (float32 rounding of t ~ 1.5) moves
    the normal-term gradient by far more than the dL/dz bound allows at the
    pixels whose stencil units sit near a kink, and by nothing measurable
    at the pixels the oracle finds well-conditioned."""
    prm = cfg_params("c2", precision=0)
    spec, cams, Z, pairs = _setup(prm, H=48, n_views=2)
    dec = oracle_decoder(spec)
    rs = O.render(dec, Z, cams, pairs, prm)
    rng = np.random.Generator(np.random.PCG64(5))
    moved = []
    for r in rs:
        r2 = O.Render(**{k: getattr(r, k) for k in r.__dataclass_fields__})
        r2.dist = r.dist + rng.normal(0, 3e-7, r.dist.shape)
        moved.append(r2)
    w = (0.0, 0.0, 1.0)
    keep = [well_conditioned(dec, Z[l], r, prm) for r, (_, l) in zip(rs, pairs)]
    g0 = _grad(dec, Z, rs, pairs, prm, cams, w)
    g1 = _grad(dec, Z, moved, pairs, prm, cams, w)
    k0 = _grad(dec, Z, rs, pairs, prm, cams, w, keep)
    k1 = _grad(dec, Z, moved, pairs, prm, cams, w, keep)
    rel_all = np.linalg.norm(g1 - g0) / np.linalg.norm(g0)
    rel_kept = np.linalg.norm(k1 - k0) / np.linalg.norm(k0)
    hits = sum(int((r.status == O.HIT).sum()) for r in rs)
    kept = sum(int((k & (r.status == O.HIT)).sum()) for k, r in zip(keep, rs))
    print("normal term, 3e-7 move: all pixels", rel_all, "well-conditioned", rel_kept, "kept", kept, "of", hits)
    assert rel_kept <= 1e-6
    assert kept >= 0.6 * hits
    assert rel_all >= 10 * rel_kept


def test_bf16_trajectory_moves_the_normal_term_but_not_the_depth_term():
    """The FP64 paper gradient taken at the samples of a bf16-rounding render
    (DecoderBF16Emulated: the march's hit points move by ~1e-4) against the
    same gradient at the FP64 render's samples, each with its own loss seeds:
    the depth term stays within the bf16 bound, the normal term does not."""
    prm = cfg_params("c3", precision=1)
    spec, cams, Z, pairs = _setup(prm)
    dec = oracle_decoder(spec)
    decb = oracle_decoder(spec, bf16=True)
    ro = O.render(dec, Z, cams, pairs, prm)
    rb = O.render(decb, Z, cams, pairs, prm)
    out = {}
    for name, w in [("depth", (10.0, 0.0, 0.0)), ("normal", (0.0, 0.0, 1.0))]:
        ga = _grad(dec, Z, ro, pairs, prm, cams, w)
        gb = _grad(dec, Z, rb, pairs, prm, cams, w)
        out[name] = np.linalg.norm(gb - ga) / np.linalg.norm(ga)
    print("fp64 gradient at bf16-rounding samples vs fp64 samples:", out)
    assert out["depth"] <= 1e-2
    assert out["normal"] >= 0.1
