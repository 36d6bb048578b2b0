"""Seeded synthetic inputs for the DIST sphere tracer.

This module only *generates data*: decoder weights, latent codes, pinhole
cameras, request streams and closed-form target images of an analytic sphere.
It contains none of the tracing method's arithmetic (no marching, no decoder
evaluation, no gradients), so both the FP64 oracle and the HIP path can take
their inputs from here without sharing any of the method's code.

All random draws use numpy's PCG64 generator in float64 and are rounded to
float32 once, so every consumer sees identical bit patterns.

Seed plan: decoder weights 0, latent i -> 1000+i, camera i -> 2000+i,
target latent i -> 3000+i, request stream -> 4000.

The decoder follows the DeepSDF-style network of the paper's implementation
appendix (B.1: nine fully connected layers, hidden width 512, the latent code
and the point concatenated at the input and again at a middle layer), in the
residual form f(p) = 0.5 (|p| - 0.5) + 0.05 tanh(m(z, p)) used by the
synthetic workloads so that a randomly initialised network still describes a
closed surface inside the unit sphere (Sec. 3.2 "Initialization" bounds all
shapes by the unit sphere).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "DecoderSpec", "C1_SPEC", "DEEPSDF_SPEC", "make_decoder", "make_latents",
    "Camera", "look_at_camera", "front_camera", "random_sphere_cameras",
    "sphere_target_maps", "poisson_requests", "TraceParams", "CONFIGS",
]


# ----------------------------------------------------------------------------
# Decoder architecture and weights
# ----------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class DecoderSpec:
    """Layer sizes of a DeepSDF-style decoder.

    ``out_dims[l]`` is the output width of linear layer ``l``; the last entry
    is 1 for a signed distance network, 3 for a colour network.  Layer 0 reads ``[z, p]`` (latent_dim + 3 values).  If
    ``skip_layer`` is set, that layer reads ``[h, z, p]`` where ``h`` is the
    previous layer's output.
    """
    latent_dim: int
    out_dims: tuple
    skip_layer: Optional[int] = None

    @property
    def n_layers(self) -> int:
        return len(self.out_dims)

    def in_dims(self) -> List[int]:
        ins = []
        for l in range(self.n_layers):
            if l == 0:
                ins.append(self.latent_dim + 3)
            else:
                d = self.out_dims[l - 1]
                if self.skip_layer is not None and l == self.skip_layer:
                    d += self.latent_dim + 3
                ins.append(d)
        return ins


# Small decoder of the smallest workload: 67 -> 128 x4 -> 1, no skip.
C1_SPEC = DecoderSpec(latent_dim=64, out_dims=(128, 128, 128, 128, 1), skip_layer=None)
# DeepSDF scale: 259 -> 512 x8 (layer 3 emits 253 so that [h3, z, p] is 512 wide) -> 1.
DEEPSDF_SPEC = DecoderSpec(latent_dim=256,
                           out_dims=(512, 512, 512, 253, 512, 512, 512, 512, 1),
                           skip_layer=4)


# Colour network of texture rendering: the geometry network's layout reading
# the concatenated shape and texture codes (256 + 256) and emitting 3 channels.
COLOR_SPEC = DecoderSpec(latent_dim=512,
                         out_dims=(512, 512, 512, 253, 512, 512, 512, 512, 3),
                         skip_layer=4)
# A small colour network for quick tests: codes 32 + 32, 128 x4, 3 channels.
C1_COLOR_SPEC = DecoderSpec(latent_dim=64, out_dims=(128, 128, 128, 128, 3), skip_layer=None)


def make_decoder(spec: DecoderSpec, seed: int = 0):
    """Kaiming-normal (fan_in, std sqrt(2/fan_in)) weights, zero biases, float32.

    Returns ``(Ws, bs)``: lists of row-major ``[out, in]`` weight matrices and
    ``[out]`` bias vectors.  Draw order: W_0, W_1, ... from one PCG64 stream.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    Ws, bs = [], []
    for l, (fin, fout) in enumerate(zip(spec.in_dims(), spec.out_dims)):
        std = math.sqrt(2.0 / fin)
        W = (rng.standard_normal((fout, fin)) * std).astype(np.float32)
        Ws.append(W)
        bs.append(np.zeros(fout, dtype=np.float32))
    return Ws, bs


def make_latents(n: int, dim: int, sigma: float = 0.01, base_seed: int = 1000) -> np.ndarray:
    """Latent codes z_i ~ N(0, sigma^2 I), one PCG64 stream per code (seed base+i)."""
    out = np.empty((n, dim), dtype=np.float32)
    for i in range(n):
        rng = np.random.Generator(np.random.PCG64(base_seed + i))
        out[i] = (rng.standard_normal(dim) * sigma).astype(np.float32)
    return out


# ----------------------------------------------------------------------------
# Cameras (pinhole, OpenCV axes: x right, y down, z forward)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    R_wc: np.ndarray     # [3,3] float32, camera-to-world rotation (columns = camera axes)
    c: np.ndarray        # [3] float32, camera centre in world coordinates
    H: int
    W: int

    def as_tuple(self):
        return (self.fx, self.fy, self.cx, self.cy, self.R_wc, self.c, self.H, self.W)


def look_at_camera(center, H: int, W: int, fov_deg: float = 50.0) -> Camera:
    """Camera at ``center`` looking at the origin; ``fov_deg`` is the full angle
    of both image axes; principal point at the image centre."""
    c = np.asarray(center, dtype=np.float64)
    fwd = -c / np.linalg.norm(c)
    up = np.array([0.0, 1.0, 0.0])
    if abs(float(fwd @ up)) > 0.99:
        up = np.array([1.0, 0.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd], axis=1)      # columns: camera x, y, z in world
    f = (W / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    fy = (H / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return Camera(fx=float(np.float32(f)), fy=float(np.float32(fy)),
                  cx=float(W) / 2.0, cy=float(H) / 2.0,
                  R_wc=R.astype(np.float32), c=c.astype(np.float32), H=H, W=W)


def front_camera(H: int, W: int, radius: float = 2.0) -> Camera:
    """The single-view workloads' camera: at (0, 0, radius) looking at the origin."""
    return look_at_camera((0.0, 0.0, radius), H, W)


def random_sphere_cameras(n: int, H: int, W: int, radius: float = 2.0,
                          base_seed: int = 2000) -> List[Camera]:
    """Cameras whose direction is normalize(N(0, I3)) (seed base+i) at ``radius``."""
    cams = []
    for i in range(n):
        rng = np.random.Generator(np.random.PCG64(base_seed + i))
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        cams.append(look_at_camera(radius * d, H, W))
    return cams


def sphere_target_maps(cam: Camera, radius: float = 0.5):
    """Closed-form images of a sphere of ``radius`` at the origin, seen by ``cam``.

    Returns float32 ``depth`` (inf off the sphere), ``normal`` [H,W,3] (0 off
    the sphere) and ``sil`` (1 on the sphere, 0 elsewhere).  Used as synthetic
    supervision targets; computed in float64 from the camera description.
    """
    H, W = cam.H, cam.W
    u = np.arange(W, dtype=np.float64) + 0.5
    v = np.arange(H, dtype=np.float64) + 0.5
    xt = (u[None, :] - cam.cx) / cam.fx
    yt = (v[:, None] - cam.cy) / cam.fy
    xt, yt = np.broadcast_to(xt, (H, W)), np.broadcast_to(yt, (H, W))
    dc = np.stack([xt, yt, np.ones_like(xt)], axis=-1)
    norm = np.linalg.norm(dc, axis=-1)
    R = cam.R_wc.astype(np.float64)
    dw = (dc / norm[..., None]) @ R.T
    c = cam.c.astype(np.float64)
    b = dw @ c
    disc = b * b - (c @ c - radius * radius)
    hit = disc > 0
    t = np.where(hit, -b - np.sqrt(np.maximum(disc, 0.0)), np.inf)
    depth = np.where(hit, t / norm, np.inf)
    pts = c[None, None, :] + np.where(hit, t, 0.0)[..., None] * dw
    normal = np.where(hit[..., None], pts / radius, 0.0)
    return (depth.astype(np.float32), normal.astype(np.float32), hit.astype(np.float32))


def ring_cameras(n: int, H: int, W: int, radius: float = 2.0, elevation_deg: float = 20.0) -> List[Camera]:
    """``n`` cameras evenly spaced over 360 degrees of azimuth around the
    vertical axis, at ``radius`` and a fixed elevation, looking at the origin
    (the multi-view setting's views "uniformly distributed around the object")."""
    cams = []
    el = math.radians(elevation_deg)
    for i in range(n):
        az = 2.0 * math.pi * i / n
        cams.append(look_at_camera((radius * math.cos(el) * math.sin(az), -radius * math.sin(el),
                                    radius * math.cos(el) * math.cos(az)), H, W))
    return cams


def texture_params(seed: int = 5000, freq: float = 8.0):
    """A procedural colour field on R^3: channel k is 0.5 + 0.5 sin(w_k . X + phi_k)
    with w_k ~ N(0, freq^2 I3) and phi_k ~ U[0, 2 pi) (PCG64 ``seed``)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((3, 3)) * freq
    phi = rng.random(3) * 2.0 * math.pi
    return w, phi


def textured_sphere_images(cams: Sequence[Camera], radius: float = 0.45, seed: int = 5000,
                           background: float = 0.0, freq: float = 8.0) -> np.ndarray:
    """Colour images [n, H, W, 3] (float32) of a sphere of ``radius`` at the
    origin painted with the procedural colour field of ``texture_params``:
    every view sees the same colour at the same surface point, as photometric
    consistency across views assumes.  Pixels off the sphere get
    ``background``."""
    w, phi = texture_params(seed, freq)
    out = []
    for cam in cams:
        H, W = cam.H, cam.W
        u = np.arange(W, dtype=np.float64) + 0.5
        v = np.arange(H, dtype=np.float64) + 0.5
        xt = np.broadcast_to((u[None, :] - cam.cx) / cam.fx, (H, W))
        yt = np.broadcast_to((v[:, None] - cam.cy) / cam.fy, (H, W))
        dc = np.stack([xt, yt, np.ones_like(xt)], axis=-1)
        dw = (dc / np.linalg.norm(dc, axis=-1, keepdims=True)) @ cam.R_wc.astype(np.float64).T
        c = cam.c.astype(np.float64)
        b = dw @ c
        disc = b * b - (c @ c - radius * radius)
        hit = disc > 0
        t = np.where(hit, -b - np.sqrt(np.maximum(disc, 0.0)), 0.0)
        X = c[None, None, :] + t[..., None] * dw
        col = 0.5 + 0.5 * np.sin(X @ w.T + phi[None, None, :])
        out.append(np.where(hit[..., None], col, background))
    return np.stack(out).astype(np.float32)


# ----------------------------------------------------------------------------
# Trace parameters per workload
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class TraceParams:
    alpha: float = 1.5
    eps: float = 5e-4
    normal_delta: float = 1e-3
    near: float = 0.5
    far: float = 3.5
    max_steps: int = 50
    c2f_levels: int = 2
    k_samples: int = 1
    precision: int = 0          # 0 = FP32 plain, 1 = BF16 MFMA
    want_normals: int = 1
    keep_history: int = 0       # 1: the saved forward keeps t per step (unrolled backward)


CONFIGS = {
    # 32x32, one front view, alpha 1, 20 steps, eps 1e-3, no coarse-to-fine.
    "c1": dict(spec=C1_SPEC, H=32, W=32, n_views=1, n_latents=1, latent_sigma=0.01,
               params=TraceParams(alpha=1.0, eps=1e-3, max_steps=20, c2f_levels=0,
                                  want_normals=0, precision=0)),
    # 256x256 single front view at DeepSDF scale, FP32 plain.
    "c2": dict(spec=DEEPSDF_SPEC, H=256, W=256, n_views=1, n_latents=1, latent_sigma=0.01,
               params=TraceParams(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=2,
                                  want_normals=1, precision=0)),
    # 8 random views x 4 latents = 32 images of 256x256, BF16 MFMA.
    "c3": dict(spec=DEEPSDF_SPEC, H=256, W=256, n_views=8, n_latents=4, latent_sigma=0.01,
               params=TraceParams(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=2,
                                  want_normals=1, precision=1)),
    # inverse optimisation: 4 views, depth + silhouette loss.
    "c4": dict(spec=DEEPSDF_SPEC, H=256, W=256, n_views=4, n_latents=1, latent_sigma=0.01,
               target_sigma=0.1,
               params=TraceParams(alpha=1.5, eps=5e-4, max_steps=50, c2f_levels=2,
                                  want_normals=0, precision=1)),
}


def poisson_requests(rate: float, n: int, seed: int = 4000, zopt_frac: float = 0.1,
                     sizes: Sequence[int] = (64, 128, 256, 512), max_views: int = 8):
    """Arrival times and shapes of a serving request stream.

    Returns a list of dicts with ``t_arrive`` (s), ``kind`` ("render"/"zopt"),
    ``res``, ``n_views`` and ``latent_seed``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps)
    res = rng.choice(np.asarray(sizes), size=n)
    views = rng.integers(1, max_views + 1, size=n)
    kinds = rng.random(n) < zopt_frac
    return [dict(t_arrive=float(t[i]), kind="zopt" if kinds[i] else "render",
                 res=int(res[i]), n_views=int(views[i]), latent_seed=5000 + i)
            for i in range(n)]
