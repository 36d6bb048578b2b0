"""Thin Python binding over the C ABI: argument marshalling only.

Every computation of the tracer runs in the HIP library; PyTorch provides
device memory (tensors) and the current stream.  If the library is missing
the calls raise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _native as N
from ._native import check


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("tensors passed to the library must be contiguous GPU tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_camera(cam) -> N.dist_camera:
    """Convert an object with fx, fy, cx, cy, R_wc [3,3], c [3], H, W to the C struct."""
    c = N.dist_camera()
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R_wc, np.float32).reshape(9)
    for i in range(9):
        c.R_wc[i] = float(R[i])
    cc = np.asarray(cam.c, np.float32).reshape(3)
    for i in range(3):
        c.c[i] = float(cc[i])
    c.H, c.W = int(cam.H), int(cam.W)
    return c


def make_params(p) -> N.dist_trace_params:
    q = N.dist_trace_params()
    q.alpha, q.eps, q.normal_delta = float(p.alpha), float(p.eps), float(p.normal_delta)
    q.near_, q.far_ = float(p.near), float(p.far)
    q.max_steps, q.c2f_levels, q.k_samples = int(p.max_steps), int(p.c2f_levels), int(p.k_samples)
    q.precision, q.want_normals = int(p.precision), int(p.want_normals)
    q.keep_history = int(getattr(p, "keep_history", 0))
    return q


class Context:
    """A decoder resident on the GPU (dist_create / dist_destroy)."""

    def __init__(self, out_dims: Sequence[int], latent_dim: int, skip_layer: Optional[int],
                 Ws: Sequence[torch.Tensor], bs: Sequence[torch.Tensor], hbm_budget: int = 0):
        self.lib = N.load()
        self.out_dims = list(out_dims)
        self.latent_dim = int(latent_dim)
        self.skip_layer = -1 if skip_layer is None else int(skip_layer)
        self._Ws = [w.detach().float().contiguous().cuda() for w in Ws]
        self._bs = [b.detach().float().contiguous().cuda() for b in bs]
        dims = (ctypes.c_int32 * len(self.out_dims))(*self.out_dims)
        desc = N.dist_decoder_desc(len(self.out_dims), self.latent_dim, self.skip_layer, dims)
        Wp = (ctypes.c_void_p * len(self._Ws))(*[w.data_ptr() for w in self._Ws])
        bp = (ctypes.c_void_p * len(self._bs))(*[b.data_ptr() for b in self._bs])
        h = ctypes.c_void_p()
        check(self.lib.dist_create(ctypes.byref(h), ctypes.byref(desc), Wp, bp, int(hbm_budget), _stream()))
        self.handle = h

    @classmethod
    def from_spec(cls, spec, Ws, bs, hbm_budget: int = 0, device="cuda"):
        Wt = [torch.as_tensor(np.asarray(w), dtype=torch.float32, device=device) for w in Ws]
        bt = [torch.as_tensor(np.asarray(b), dtype=torch.float32, device=device) for b in bs]
        return cls(spec.out_dims, spec.latent_dim, spec.skip_layer, Wt, bt, hbm_budget)

    def close(self):
        if getattr(self, "handle", None):
            check(self.lib.dist_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, Ws, bs):
        self._Ws = [w.detach().float().contiguous().cuda() for w in Ws]
        self._bs = [b.detach().float().contiguous().cuda() for b in bs]
        Wp = (ctypes.c_void_p * len(self._Ws))(*[w.data_ptr() for w in self._Ws])
        bp = (ctypes.c_void_p * len(self._bs))(*[b.data_ptr() for b in self._bs])
        check(self.lib.dist_set_weights(self.handle, Wp, bp, _stream()))


def dist_timing_enable(ctx: Context, on: bool = True):
    check(ctx.lib.dist_timing_enable(ctx.handle, 1 if on else 0))


def dist_timing_read(ctx: Context, kernel: int):
    """(launches, milliseconds, rows) of kernel class 0 march, 1 eval, 2 adjoint, 3 VJP from saved masks,
    4 weight-gradient contraction (rows not counted)."""
    t = N.dist_kernel_time()
    check(ctx.lib.dist_timing_read(ctx.handle, int(kernel), ctypes.byref(t)))
    return int(t.launches), float(t.ms), int(t.rows)


class Saved:
    """Owner of a dist_saved handle."""

    def __init__(self, lib, handle, shape=None):
        self.lib, self.handle = lib, handle
        self.shape = shape          # (n_img, H, W) of the render

    def free(self):
        if self.handle:
            check(self.lib.dist_saved_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def dist_render_fwd(ctx: Context, cams, z: torch.Tensor, params, pairs=None, save: bool = False):
    """Render; returns a dict of output tensors (and a Saved handle if save)."""
    cams_c = (N.dist_camera * len(cams))(*[make_camera(c) for c in cams])
    n_lat = z.shape[0]
    if pairs is None:
        n_img = len(cams) * n_lat
        pairs_c = None
    else:
        pairs = np.asarray(pairs, np.int32).reshape(-1, 2)
        n_img = pairs.shape[0]
        pairs_c = (ctypes.c_int32 * (2 * n_img))(*pairs.reshape(-1).tolist())
    H, W = int(cams[0].H), int(cams[0].W)
    dev = z.device
    out = dict(
        depth=torch.empty(n_img, H, W, device=dev), dist=torch.empty(n_img, H, W, device=dev),
        normal=torch.empty(n_img, H, W, 3, device=dev), sil=torch.empty(n_img, H, W, device=dev),
        status=torch.empty(n_img, H, W, dtype=torch.uint8, device=dev),
        nsteps=torch.empty(n_img, H, W, dtype=torch.uint8, device=dev),
        queries=torch.empty(n_img, dtype=torch.int64, device=dev))
    if not int(params.want_normals):
        out["normal"].zero_()
    prm = make_params(params)
    sv = ctypes.c_void_p()
    zc = z.detach().float().contiguous()
    check(ctx.lib.dist_render_fwd(ctx.handle, cams_c, len(cams), _ptr(zc), n_lat, pairs_c, n_img, ctypes.byref(prm),
                                  _ptr(out["depth"]), _ptr(out["dist"]),
                                  _ptr(out["normal"]) if int(params.want_normals) else None,
                                  _ptr(out["sil"]), _ptr(out["status"]), _ptr(out["nsteps"]), _ptr(out["queries"]),
                                  ctypes.byref(sv) if save else None, _stream()))
    if save:
        out["saved"] = Saved(ctx.lib, sv, (n_img, H, W))
        out["_z"] = zc          # keep the latent buffer alive for the backward
    return out


def _theta_buffers(ctx: Context):
    gW = [torch.empty_like(w) for w in ctx._Ws]
    gb = [torch.empty_like(b) for b in ctx._bs]
    Wp = (ctypes.c_void_p * len(gW))(*[t.data_ptr() for t in gW])
    bp = (ctypes.c_void_p * len(gb))(*[t.data_ptr() for t in gb])
    return gW, gb, Wp, bp


def dist_render_bwd(ctx: Context, saved: Saved, g_depth=None, g_normal=None, g_sil=None, n_latents=None,
                    want_theta: bool = False):
    """Paper gradient w.r.t. the latent codes (g_z [n_latents, L]); with
    want_theta also w.r.t. the decoder weights: returns (g_z, gW list, gb list)."""
    g_z = torch.empty(n_latents, ctx.latent_dim, device="cuda")
    args = [None if g is None else g.detach().float().contiguous() for g in (g_depth, g_normal, g_sil)]
    if want_theta:
        gW, gb, Wp, bp = _theta_buffers(ctx)
        check(ctx.lib.dist_render_bwd(ctx.handle, saved.handle, *[_ptr(a) for a in args], _ptr(g_z), Wp, bp,
                                      _stream()))
        return g_z, gW, gb
    check(ctx.lib.dist_render_bwd(ctx.handle, saved.handle, *[_ptr(a) for a in args], _ptr(g_z), None, None,
                                  _stream()))
    return g_z


def dist_render_bwd_implicit(ctx: Context, saved: Saved, g_depth=None, g_normal=None, g_sil=None, n_latents=None):
    """dL/dz with the exact (implicit-function) depth derivative at each hit;
    silhouette and normal terms as dist_render_bwd."""
    g_z = torch.empty(n_latents, ctx.latent_dim, device="cuda")
    args = [None if g is None else g.detach().float().contiguous() for g in (g_depth, g_normal, g_sil)]
    check(ctx.lib.dist_render_bwd_implicit(ctx.handle, saved.handle, *[_ptr(a) for a in args], _ptr(g_z), _stream()))
    return g_z


def dist_render_bwd_unrolled(ctx: Context, saved: Saved, g_depth=None, g_sil=None, n_latents=None):
    """Exact dL/dz of the depth and silhouette terms through the unrolled march
    (the forward must have run with keep_history = 1)."""
    g_z = torch.empty(n_latents, ctx.latent_dim, device="cuda")
    args = [None if g is None else g.detach().float().contiguous() for g in (g_depth, g_sil)]
    check(ctx.lib.dist_render_bwd_unrolled(ctx.handle, saved.handle, *[_ptr(a) for a in args], _ptr(g_z),
                                           _stream()))
    return g_z


def dist_render_color(cctx: Context, saved: Saved, zc: torch.Tensor, precision: int = 1):
    """Colour [n_img, H, W, 3] of the hits of a saved geometry render, by the
    colour network ``cctx`` with one code per latent of the render."""
    zc_ = zc.detach().float().contiguous()
    rgb = torch.empty(saved.shape + (3,), device=zc.device)
    check(cctx.lib.dist_render_color(cctx.handle, saved.handle, _ptr(zc_), zc.shape[0], int(precision), _ptr(rgb),
                                     _stream()))
    return rgb


def dist_render_color_bwd(cctx: Context, saved: Saved, zc: torch.Tensor, g_rgb: torch.Tensor, precision: int = 1):
    """dL/d(code) [n_lat, code width] of the colour at the hits (hit points detached)."""
    zc_ = zc.detach().float().contiguous()
    g = g_rgb.detach().float().contiguous()
    g_zc = torch.empty_like(zc_)
    check(cctx.lib.dist_render_color_bwd(cctx.handle, saved.handle, _ptr(zc_), zc.shape[0], int(precision), _ptr(g),
                                         _ptr(g_zc), _stream()))
    return g_zc


def dist_photometric_loss(cams, depth: torch.Tensor, images: torch.Tensor, pairs, weight=5.0, want_grad=True):
    """Cross-view photometric loss of rendered depth maps [n, H, W] and colour
    images [n, H, W, 3]; pairs (i, j) warp view j into view i.  Returns
    (loss tensor [1], dL/d(depth) [n, H, W] or None)."""
    lib = N.load()
    n = len(cams)
    cams_c = (N.dist_camera * n)(*[make_camera(c) for c in cams])
    flat = [int(v) for p in pairs for v in p]
    pairs_c = (ctypes.c_int32 * len(flat))(*flat)
    d = depth.detach().float().contiguous()
    im = images.detach().float().contiguous()
    loss_map = torch.empty_like(d)
    loss = torch.empty(1, device=d.device)
    g = torch.empty_like(d) if want_grad else None
    check(lib.dist_photometric_loss(cams_c, n, _ptr(d), _ptr(im), pairs_c, len(pairs), float(weight), _ptr(loss_map),
                                    _ptr(loss), _ptr(g), _stream()))
    return loss, g


def dist_render_bwd_camera(ctx: Context, saved: Saved, n_views: int, g_depth=None, g_sil=None):
    """Gradient of the depth and silhouette terms w.r.t. each view's camera
    extrinsics: a tensor [n_views, 12] = (dL/dc, dL/dR_wc row-major)."""
    g_cam = torch.empty(n_views, 12, device="cuda")
    args = [None if g is None else g.detach().float().contiguous() for g in (g_depth, g_sil)]
    check(ctx.lib.dist_render_bwd_camera(ctx.handle, saved.handle, *[_ptr(a) for a in args], _ptr(g_cam),
                                         _stream()))
    return g_cam


def dist_sdf_eval(ctx: Context, points: torch.Tensor, latent_ids: torch.Tensor, z: torch.Tensor, precision: int):
    n = points.shape[0]
    f = torch.empty(n, device=points.device)
    pts = points.detach().float().contiguous()
    ids = latent_ids.to(torch.int32).contiguous()
    zc = z.detach().float().contiguous()
    check(ctx.lib.dist_sdf_eval(ctx.handle, _ptr(pts), _ptr(ids), _ptr(zc), z.shape[0], n, int(precision), _ptr(f),
                                _stream()))
    return f


def dist_sdf_eval_noalloc(ctx: Context, points: torch.Tensor, latent_ids: torch.Tensor, z: torch.Tensor,
                          precision: int, out: torch.Tensor):
    """dist_sdf_eval into the caller's `out` [n] with no allocation anywhere:
    inputs must already be contiguous float32 / int32 device tensors."""
    check(ctx.lib.dist_sdf_eval_noalloc(ctx.handle, _ptr(points), _ptr(latent_ids), _ptr(z), z.shape[0],
                                        points.shape[0], int(precision), _ptr(out), _stream()))
    return out


def dist_sdf_vjp(ctx: Context, points, latent_ids, seeds, z, precision: int, want_theta: bool = False):
    n = points.shape[0]
    g_z = torch.empty(z.shape[0], ctx.latent_dim, device=points.device)
    pts = points.detach().float().contiguous()
    ids = latent_ids.to(torch.int32).contiguous()
    sd = seeds.detach().float().contiguous()
    zc = z.detach().float().contiguous()
    if want_theta:
        gW, gb, Wp, bp = _theta_buffers(ctx)
        check(ctx.lib.dist_sdf_vjp(ctx.handle, _ptr(pts), _ptr(ids), _ptr(sd), _ptr(zc), z.shape[0], n,
                                   int(precision), _ptr(g_z), Wp, bp, _stream()))
        return g_z, gW, gb
    check(ctx.lib.dist_sdf_vjp(ctx.handle, _ptr(pts), _ptr(ids), _ptr(sd), _ptr(zc), z.shape[0], n, int(precision),
                               _ptr(g_z), None, None, _stream()))
    return g_z


class DistRender(torch.autograd.Function):
    """Differentiable render of depth, normal and soft silhouette w.r.t. z.

    forward(z, ctx, cams, params, pairs) -> (depth, normal, sil, status)
    backward applies the paper's approximate gradient via dist_render_bwd.
    """

    @staticmethod
    def forward(actx, z, ctx, cams, params, pairs=None):
        out = dist_render_fwd(ctx, cams, z, params, pairs=pairs, save=True)
        actx.saved_handle = out["saved"]
        actx.ctx = ctx
        actx.n_lat = z.shape[0]
        actx.keep = out["_z"]
        actx.mark_non_differentiable(out["status"])
        return out["depth"], out["normal"], out["sil"], out["status"]

    @staticmethod
    def backward(actx, g_depth, g_normal, g_sil, g_status):
        g_z = dist_render_bwd(actx.ctx, actx.saved_handle, g_depth, g_normal, g_sil, n_latents=actx.n_lat)
        actx.saved_handle.free()
        return g_z, None, None, None, None


def dist_render_loss(depth, normal, sil, depth_t, normal_t, sil_t, w_d=10.0, w_s=1.0, w_n=0.0, want_grad=True):
    """Per-image loss [n] of the latent fit (L1 depth, silhouette hinge,
    normal term) and, with want_grad, its map gradients (g_depth, g_normal,
    g_sil); normals may be None when w_n = 0."""
    lib = N.load()
    d, s, dt, st = [x.detach().float().contiguous() for x in (depth, sil, depth_t, sil_t)]
    n_img, H, W = d.shape
    use_n = float(w_n) != 0.0
    nr = normal.detach().float().contiguous() if use_n and normal is not None else None
    ntr = normal_t.detach().float().contiguous() if use_n and normal_t is not None else None
    loss = torch.empty(n_img, device=d.device)
    gd = torch.empty_like(d) if want_grad else None
    gs = torch.empty_like(d) if want_grad else None
    gn = torch.empty(n_img, H, W, 3, device=d.device) if want_grad else None
    check(lib.dist_render_loss(n_img, H, W, _ptr(d), _ptr(nr), _ptr(s), _ptr(dt), _ptr(ntr), _ptr(st), float(w_d),
                               float(w_s), float(w_n), _ptr(loss), _ptr(gd), _ptr(gn), _ptr(gs), _stream()))
    return loss, gd, gn, gs


def dist_eps_for_camera(d_min: float, sensor: float, focal: float, resolution: int, theta: float = 0.0) -> float:
    """Convergence threshold of App. A.2 (host arithmetic in the library)."""
    lib = N.load()
    e = ctypes.c_double()
    check(lib.dist_eps_for_camera(float(d_min), float(sensor), float(focal), int(resolution), float(theta),
                                  ctypes.byref(e)))
    return e.value


def dist_adam_step(z: torch.Tensor, m: torch.Tensor, v: torch.Tensor, g: torch.Tensor, t: int, lr=1e-2,
                   beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam step t (>= 1) on z in place; m and v are the moment buffers."""
    lib = N.load()
    gg = g.detach().float().contiguous()
    check(lib.dist_adam_step(_ptr(z), _ptr(m), _ptr(v), _ptr(gg), z.numel(), float(lr), float(beta1), float(beta2),
                             float(eps), int(t), _stream()))


# ----------------------------------------------------------------------------
# serving
# ----------------------------------------------------------------------------
class ServeRequest:
    """Host-side holder of one submitted request and the buffers it references."""

    def __init__(self, kind, cams, z, params, want_normals=True, targets=None, iters=0, lr=1e-2,
                 w_depth=10.0, w_sil=1.0):
        n = len(cams)
        H, W = int(cams[0].H), int(cams[0].W)
        dev = z.device
        self.kind = kind
        self.cams_c = (N.dist_camera * n)(*[make_camera(c) for c in cams])
        self.z = z.detach().float().contiguous()
        self.depth = torch.empty(n, H, W, device=dev)
        self.sil = torch.empty(n, H, W, device=dev)
        self.normal = torch.zeros(n, H, W, 3, device=dev) if want_normals else None
        self.status = torch.empty(n, H, W, dtype=torch.uint8, device=dev)
        self.targets = None if targets is None else tuple(t.float().contiguous() for t in targets)
        self.z_out = torch.empty_like(self.z) if kind == N.REQ_ZOPT else None
        r = N.dist_request()
        r.kind = kind
        r.n_views = n
        r.cams = self.cams_c
        r.prm = make_params(params)
        r.prm.want_normals = 1 if want_normals else 0
        r.z = self.z.data_ptr()
        r.depth = self.depth.data_ptr()
        r.sil = self.sil.data_ptr()
        r.normal = self.normal.data_ptr() if want_normals else None
        r.status = self.status.data_ptr()
        if kind == N.REQ_ZOPT:
            r.target_depth = self.targets[0].data_ptr()
            r.target_sil = self.targets[1].data_ptr()
            r.iters = int(iters)
            r.lr, r.w_depth, r.w_sil = float(lr), float(w_depth), float(w_sil)
            r.z_out = self.z_out.data_ptr()
        self.c = r
        self.ticket = None
        self.result = None


def dist_submit(ctx: Context, req: ServeRequest):
    """Queue a request (buffers must be ready: the server reads them on its own stream)."""
    torch.cuda.current_stream().synchronize()
    t = ctypes.c_uint64()
    check(ctx.lib.dist_submit(ctx.handle, ctypes.byref(req.c), ctypes.byref(t)))
    req.ticket = t.value
    return t.value


def dist_poll(ctx: Context, req: ServeRequest, timeout_us: int = -1):
    """Wait for a request; returns a dict (status, latency_ms, queries, final_loss) or None if pending."""
    res = N.dist_result()
    rc = check(ctx.lib.dist_poll(ctx.handle, ctypes.c_uint64(req.ticket), ctypes.byref(res), int(timeout_us)))
    if rc == N.DIST_PENDING:
        return None
    req.result = dict(status=int(res.status), latency_ms=res.latency_ns / 1e6, queries=int(res.queries),
                      final_loss=float(res.final_loss))
    return req.result
