"""Shared test helpers: seeded workloads, oracle runs and comparisons."""
import copy

import numpy as np

import dist_inputs as di


def params(**kw):
    p = di.TraceParams()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def cfg_params(name, **kw):
    p = copy.deepcopy(di.CONFIGS[name]["params"])
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def gpu_ctx(spec, seed=0, Ws=None, bs=None):
    import torch
    from paper_1911_13225_amd import api
    if Ws is None:
        Ws, bs = di.make_decoder(spec, seed=seed)
    return api.Context.from_spec(spec, Ws, bs)


def oracle_decoder(spec, seed=0, bf16=False):
    from oracle import dist_oracle as O
    Ws, bs = di.make_decoder(spec, seed=seed)
    return (O.DecoderBF16Emulated if bf16 else O.Decoder)(spec, Ws, bs)


def compare_render(o, g, eps, mu=2e-5, depth_tol=1e-4):
    """Compare one oracle render `o` with GPU maps `g` (numpy dict of one image).

    Pixels whose discrete trajectory (status, step count) agrees must match in
    depth to `depth_tol`; disagreeing pixels ("flips") must be explained by a
    decision of the oracle within `mu` of its threshold.  Returns a dict of
    statistics.
    """
    st_o = o.status.reshape(-1)
    st_g = g["status"].reshape(-1)
    ns_o = o.nsteps.reshape(-1)
    ns_g = g["nsteps"].reshape(-1)
    same = (st_o == st_g) & (ns_o == ns_g)
    flips = ~same
    hit = same & (st_o == 1)
    dd = np.abs(o.depth.reshape(-1)[hit] - g["depth"].reshape(-1)[hit])
    ds = np.abs(o.sil.reshape(-1)[same] - g["sil"].reshape(-1)[same])
    fg_o = o.sil.reshape(-1) < 0
    fg_g = g["sil"].reshape(-1) < 0
    return dict(n=st_o.size, flips=int(flips.sum()),
                unexplained=int((flips & (o.margin.reshape(-1) >= mu)).sum()),
                depth_max=float(dd.max()) if dd.size else 0.0,
                sil_max=float(ds.max()) if ds.size else 0.0,
                sil_mismatch=int((fg_o != fg_g).sum()), hits=int((st_o == 1).sum()),
                flip_idx=np.nonzero(flips)[0])


def well_conditioned(dec, z, r, prm, depth_t=None, sil_t=None, mu_march=2e-5, mu_relu=1e-6, mu_f=1e-6,
                     mu_res=1e-5):
    """[H,W] bool: pixels whose paper gradient is a well-conditioned function
    of the render, judged from the oracle alone (no GPU value enters).

    A pixel is kept when every floating-point decision its gradient depends
    on is farther from its threshold than the rounding of a float32 path can
    move it: the march decisions (status, step count; ``Render.margin``), the
    ReLU patterns at every gradient sample (``O.sample_relu_margin``), the
    sign of f at the minimum-|f| query (silhouette seed) and, given a target
    depth, the sign of the depth residual."""
    from oracle import dist_oracle as O
    keep = r.margin > mu_march
    if mu_relu > 0:
        keep &= O.sample_relu_margin(dec, z, r, prm) > mu_relu
    f0 = r.rec_f[0].reshape(r.H, r.W)
    keep &= (r.status == O.MISS) | (np.abs(f0) > mu_f)
    if depth_t is not None:
        fg = (r.sil < 0) & ((np.asarray(sil_t) > 0.5) if sil_t is not None else True)
        res = np.where(fg, r.depth - np.where(fg, depth_t, 0.0), np.inf)
        keep &= ~fg | (np.abs(res) > mu_res)
    return keep
