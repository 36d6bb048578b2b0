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
