"""FP64 CPU oracle of DIST's differentiable sphere tracing (arXiv 1911.13225).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference that the HIP path is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
library never calls it and shares no code with it (the two meet only through
the seeded inputs of ``dist_inputs``).

Everything is numpy float64.  Each function cites the passage of the paper it
follows.  Where the paper is silent or ambiguous the reading taken is stated
in the docstring (tagged "Reading:"); the same readings are implemented by the
GPU path from their own description.

Parity pins (what checks this oracle against something other than itself) live
in ``tests/test_oracle_pins.py``.  The coarse-to-fine schedule (which steps
run at which level, every child re-traced) is pinned by closed-form query
counts on the analytic base field.  Parity unpinned: the start of a split
child and its empty minimum-|f| records (Reading C2F), the alpha coefficient
of the depth gradient (Reading G1) and the K-sample rule (Reading G2) are
checked only for self-consistency; the paper gives no numbers for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

# Ray status codes (Alg. 1 termination cases + unit-sphere initialisation).
ACTIVE, HIT, MISS, ESCAPED, UNCONVERGED = 0, 1, 2, 3, 4


# ============================================================================
# Decoder: DeepSDF-style MLP in the residual form of the synthetic workloads
# ============================================================================
class Decoder:
    """f(p, z) = 0.5 (|p| - 0.5) + 0.05 tanh(m(z, p)).

    ``m`` is a stack of fully connected layers with ReLU between them (App. B.1,
    following DeepSDF): layer 0 reads [z, p]; the skip layer reads [h, z, p].
    Weights are row-major [out, in] as given; all arithmetic in float64.
    """

    def __init__(self, spec, Ws, bs):
        self.spec = spec
        self.L = spec.latent_dim
        self.skip = spec.skip_layer
        self.W = [np.asarray(W, dtype=np.float64) for W in Ws]
        self.b = [np.asarray(b, dtype=np.float64) for b in bs]
        self.nl = len(self.W)

    # -- forward ------------------------------------------------------------
    def layer_inputs(self, Z, P, keep):
        """Run the MLP; return pre-activation m and (if keep) per-layer inputs
        and pre-activations for the backward pass."""
        h = np.concatenate([Z, P], axis=1)
        inputs, pre = [], []
        a = None
        for l in range(self.nl):
            if l == 0:
                x = h
            elif self.skip is not None and l == self.skip:
                x = np.concatenate([h, Z, P], axis=1)
            else:
                x = h
            a = x @ self.W[l].T + self.b[l]
            if keep:
                inputs.append(x)
                pre.append(a)
            if l < self.nl - 1:
                h = np.maximum(a, 0.0)
        return a[:, 0], inputs, pre

    def sdf(self, Z, P):
        """Signed distance at points P [n,3] with per-point latents Z [n,L]."""
        Z = np.asarray(Z, np.float64)
        P = np.asarray(P, np.float64)
        if P.shape[0] == 0:
            return np.zeros(0)
        m, _, _ = self.layer_inputs(Z, P, keep=False)
        return 0.5 * (np.linalg.norm(P, axis=1) - 0.5) + 0.05 * np.tanh(m)

    # -- reverse mode (hand-derived chain rule) -------------------------------
    def sdf_vjp(self, Z, P, seeds, want_theta=True):
        """Return (gZ [n,L], gW list, gb list) = sum_i seeds_i d f(P_i, Z_i)/d(z, theta).

        Points are treated as constants (the paper differentiates f at detached
        sample locations, Sec. 3.4).  ReLU'(0) is taken as 0.
        """
        Z = np.asarray(Z, np.float64)
        P = np.asarray(P, np.float64)
        seeds = np.asarray(seeds, np.float64)
        n = P.shape[0]
        gZ = np.zeros((n, self.L))
        gW = [np.zeros_like(W) for W in self.W]
        gb = [np.zeros_like(b) for b in self.b]
        if n == 0:
            return gZ, gW, gb
        m, inputs, pre = self.layer_inputs(Z, P, keep=True)
        th = np.tanh(m)
        delta = (seeds * 0.05 * (1.0 - th * th))[:, None]          # d/d(pre-activation of last layer)
        for l in range(self.nl - 1, -1, -1):
            if want_theta:
                gW[l] = delta.T @ inputs[l]
                gb[l] = delta.sum(axis=0)
            g_in = delta @ self.W[l]                               # gradient w.r.t. layer input
            if l == 0:
                gZ += g_in[:, : self.L]
                break
            if self.skip is not None and l == self.skip:
                nh = self.W[l - 1].shape[0]
                gZ += g_in[:, nh: nh + self.L]
                g_h = g_in[:, :nh]
            else:
                g_h = g_in
            delta = g_h * (pre[l - 1] > 0.0)
        return gZ, gW, gb

    def relu_margin(self, Z, P):
        """Smallest |pre-activation| over all hidden units at each point [n].

        A ReLU pattern is an integer decision taken in floating point: the
        derivative of f jumps when a unit crosses zero, so a gradient sample
        whose margin is below the rounding error of its point (or of the
        arithmetic) is ill-conditioned, and two correct implementations may
        disagree there by a finite amount."""
        Z = np.asarray(Z, np.float64)
        P = np.asarray(P, np.float64)
        if P.shape[0] == 0:
            return np.zeros(0)
        _, _, pre = self.layer_inputs(Z, P, keep=True)
        return np.min(np.stack([np.abs(a).min(axis=1) for a in pre[:-1]], axis=1), axis=1)

    def sdf_grad_p(self, Z, P, seeds):
        """seeds_i * grad_p f(P_i, Z_i) [n,3]: the spatial gradient of f through
        the residual term 0.5 |p| and the point columns of layer 0 and of the
        skip layer.  ReLU'(0) is taken as 0."""
        Z = np.asarray(Z, np.float64)
        P = np.asarray(P, np.float64)
        seeds = np.asarray(seeds, np.float64)
        n = P.shape[0]
        if n == 0:
            return np.zeros((0, 3))
        m, inputs, pre = self.layer_inputs(Z, P, keep=True)
        th = np.tanh(m)
        gP = (0.5 * seeds / np.linalg.norm(P, axis=1))[:, None] * P
        delta = (seeds * 0.05 * (1.0 - th * th))[:, None]
        for l in range(self.nl - 1, -1, -1):
            g_in = delta @ self.W[l]
            if l == 0:
                gP += g_in[:, self.L: self.L + 3]
                break
            if self.skip is not None and l == self.skip:
                nh = self.W[l - 1].shape[0]
                gP += g_in[:, nh + self.L: nh + self.L + 3]
                g_h = g_in[:, :nh]
            else:
                g_h = g_in
            delta = g_h * (pre[l - 1] > 0.0)
        return gP


def _bf16_round(x):
    """Round float64 values to the nearest bfloat16 (ties to even), via float32."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


class DecoderBF16Emulated(Decoder):
    """The decoder evaluated the way a BF16 tensor-core implementation rounds.

    Not the reference for accuracy claims (that is :class:`Decoder`); this
    variant only separates rounding effects from implementation mistakes.  The
    latent part of layer 0 and of the skip layer, the point part of both, all
    biases and the final 1-wide layer stay at full precision; every matrix
    product between hidden layers takes bfloat16-rounded weights and a
    bfloat16-rounded input and is accumulated exactly.
    """

    def layer_inputs(self, Z, P, keep):
        h = None
        a = None
        inputs, pre = [], []
        for l in range(self.nl):
            W, b = self.W[l], self.b[l]
            if l == 0:
                a = np.concatenate([Z, P], 1) @ W.T + b
            elif l == self.nl - 1:
                a = h @ W.T + b
            else:
                nh = W.shape[1] if not (self.skip is not None and l == self.skip) else self.W[l - 1].shape[0]
                a = _bf16_round(h) @ _bf16_round(W[:, :nh]).T + b
                if self.skip is not None and l == self.skip:
                    a = a + np.concatenate([Z, P], 1) @ W[:, nh:].T
            if l < self.nl - 1:
                h = np.maximum(a, 0.0)
        return a[:, 0], inputs, pre


# ============================================================================
# Cameras and rays  (Sec. 3.3 depth formula; one ray through each pixel centre)
# ============================================================================
@dataclass
class Cam:
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray   # camera-to-world rotation [3,3]
    c: np.ndarray   # centre [3]
    H: int
    W: int


def cam_from(camera) -> Cam:
    return Cam(float(camera.fx), float(camera.fy), float(camera.cx), float(camera.cy),
               np.asarray(camera.R_wc, np.float64), np.asarray(camera.c, np.float64),
               int(camera.H), int(camera.W))


def level_rays(cam: Cam, level: int, U: np.ndarray, V: np.ndarray):
    """Rays of the coarse-to-fine level ``level`` at block coordinates (U, V).

    A level-l ray passes through the centre of its 2^l x 2^l block of
    full-resolution pixels; at level 0 that is the pixel centre (u + 1/2,
    v + 1/2).  Returns (xt, yt, unit world direction [n,3]) where
    (xt, yt, 1) = K^-1 (x, y, 1) (Sec. 3.3).
    """
    s = float(1 << level)
    u = s * U.astype(np.float64) + 0.5 * s
    v = s * V.astype(np.float64) + 0.5 * s
    xt = (u - cam.cx) / cam.fx
    yt = (v - cam.cy) / cam.fy
    dc = np.stack([xt, yt, np.ones_like(xt)], axis=1)
    dc /= np.linalg.norm(dc, axis=1, keepdims=True)
    return xt, yt, dc @ cam.R.T


def unit_sphere_init(c, D, near, far):
    """Initialisation of Sec. 3.2: start each ray where it enters the unit sphere.

    Returns (inside mask, t_lo, t_hi, dist of the ray line from the origin,
    |disc| margin).  Rays that do not meet the sphere are background (MISS);
    App. A.3 gives them the soft silhouette (distance to origin) - 1.
    """
    b = D @ c
    cc = float(c @ c)
    disc = b * b - (cc - 1.0)
    # Reading R16: the camera is outside the sphere, so the two roots of the
    # line share a sign; the ray meets the sphere only if they lie ahead (b < 0)
    inside = (disc > 0.0) & (b < 0.0)
    sq = np.sqrt(np.maximum(disc, 0.0))
    t_lo = np.maximum(-b - sq, near)
    t_hi = np.minimum(-b + sq, far)
    dist = ray_origin_distance(c, b)
    return inside, t_lo, t_hi, dist, np.abs(disc)


def ray_origin_distance(c, b):
    """Distance from the origin to the ray c + t v, t >= 0, with b = c . v:
    the foot of the perpendicular if it lies ahead (b < 0), else the camera
    centre (App. A.3 uses it for the soft silhouette of rays that miss)."""
    cc = float(c @ c)
    return np.where(b < 0.0, np.sqrt(np.maximum(cc - b * b, 0.0)), math.sqrt(cc))


# ============================================================================
# Marching (Alg. 1 with the Sec. 3.2 strategies)
# ============================================================================
@dataclass
class RayState:
    """Per-ray state of the tracer (the "location of each query is saved
    globally" of App. B.2 is kept here as the top-K records)."""
    O: np.ndarray            # [n,3] origins
    D: np.ndarray            # [n,3] unit directions
    t: np.ndarray
    t_lo: np.ndarray
    t_hi: np.ndarray
    status: np.ndarray       # int8 status codes
    nsteps: np.ndarray       # global step count at termination (N for hits)
    f_last: np.ndarray
    rec_absf: np.ndarray     # [K,n] ascending |f| of the K best queries (inf = empty)
    rec_n: np.ndarray        # [K,n] global step of each record
    rec_t: np.ndarray        # [K,n] ray parameter of each record
    rec_f: np.ndarray        # [K,n] signed f of each record
    margin: np.ndarray       # smallest distance of any decision value to its threshold
    queries: int = 0


def new_state(O, D, t0, t_lo, t_hi, status, K, margin):
    n = D.shape[0]
    return RayState(O=O, D=D, t=t0.copy(), t_lo=t_lo, t_hi=t_hi, status=status.astype(np.int8),
                    nsteps=np.zeros(n, np.int32), f_last=np.zeros(n),
                    rec_absf=np.full((K, n), np.inf), rec_n=np.full((K, n), -1, np.int32),
                    rec_t=np.zeros((K, n)), rec_f=np.zeros((K, n)), margin=margin.copy())


def march(sdf_fn: Callable, st: RayState, n_begin: int, n_end: int, alpha: float, eps: float,
          max_steps: int):
    """Global steps n_begin .. n_end-1 of sphere tracing on every ACTIVE ray.

    Per step and ray (Alg. 1, Sec. 3.2, Eq. 1):
      * query f at p = c + t v  (dynamic synchronized inference: only
        unfinished rays are evaluated, in one batch);
      * record the query among the ray's K smallest |f| (App. B.2; ties keep
        the earlier step);
      * |f| < eps -> converged (HIT), N = n + 1, ray distance d = t + f: Eq. 1
        with the unit-weight last step, alpha sum_{n<N-1} f + f_{N-1} plus the
        start offset t_0;
      * else if n is the last allowed step -> UNCONVERGED (background);
      * else aggressive step t += alpha f (Sec. 3.2); leaving the unit-sphere
        interval [t_lo, t_hi] -> ESCAPED (App. B.2 "gets out of the unit
        sphere"), background.
    Reading: the stop test precedes the step, so no query is made outside the
    unit sphere and d uses the last query (Alg. 1 queries, then updates, then
    checks).
    """
    K = st.rec_absf.shape[0]
    for n in range(n_begin, min(n_end, max_steps)):
        idx = np.nonzero(st.status == ACTIVE)[0]
        if idx.size == 0:
            continue
        P = st.O[idx] + st.t[idx, None] * st.D[idx]
        f = np.asarray(sdf_fn(idx, P), np.float64)
        st.queries += idx.size
        af = np.abs(f)
        # --- running top-K of (|f|, step): insertion keeps ties in step order
        pos = (st.rec_absf[:, idx] <= af[None, :]).sum(axis=0)
        for j in range(K - 1, -1, -1):
            shift = pos < j
            put = pos == j
            if j > 0:
                for arr in (st.rec_absf, st.rec_n, st.rec_t, st.rec_f):
                    arr[j, idx[shift]] = arr[j - 1, idx[shift]]
            st.rec_absf[j, idx[put]] = af[put]
            st.rec_n[j, idx[put]] = n
            st.rec_t[j, idx[put]] = st.t[idx[put]]
            st.rec_f[j, idx[put]] = f[put]
        st.f_last[idx] = f
        st.margin[idx] = np.minimum(st.margin[idx], np.abs(af - eps))
        hit = af < eps
        h_idx = idx[hit]
        st.status[h_idx] = HIT
        st.nsteps[h_idx] = n + 1
        rest = idx[~hit]
        if n == max_steps - 1:
            st.status[rest] = UNCONVERGED
            st.nsteps[rest] = n + 1
            continue
        t_new = st.t[rest] + alpha * f[~hit]
        st.t[rest] = t_new
        st.margin[rest] = np.minimum(st.margin[rest],
                                     np.minimum(np.abs(t_new - st.t_hi[rest]), np.abs(t_new - st.t_lo[rest])))
        esc = (t_new > st.t_hi[rest]) | (t_new < st.t_lo[rest])
        st.status[rest[esc]] = ESCAPED
        st.nsteps[rest[esc]] = n + 1


# ============================================================================
# Rendering an image (Sec. 3.2 + 3.3)
# ============================================================================
@dataclass
class Render:
    H: int
    W: int
    depth: np.ndarray        # [H,W] z_c, inf for background
    dist: np.ndarray         # [H,W] ray distance d, inf for background
    normal: np.ndarray       # [H,W,3] unit normal, 0 for background
    nraw: np.ndarray         # [H,W,3] unnormalised central-difference gradient
    sil: np.ndarray          # [H,W] soft silhouette S (negative = foreground)
    status: np.ndarray       # [H,W] int8
    nsteps: np.ndarray       # [H,W] int32
    margin: np.ndarray       # [H,W] smallest decision margin along the pixel's chain
    xt: np.ndarray
    yt: np.ndarray
    dirs: np.ndarray         # [H*W,3]
    c: np.ndarray
    rec_absf: np.ndarray     # [K,H*W]
    rec_t: np.ndarray
    rec_f: np.ndarray
    rec_n: np.ndarray
    queries: int
    queries_per_step: List[int] = field(default_factory=list)


def render_image(sdf_fn: Callable, cam: Cam, prm, pixels: Optional[np.ndarray] = None) -> Render:
    """Render one image of a signed distance function.

    ``sdf_fn(P)`` maps points [n,3] to f [n].  ``prm`` carries alpha, eps,
    normal_delta, near, far, max_steps, c2f_levels, k_samples, want_normals.

    Coarse-to-fine (Sec. 3.2, Fig. 3a): tracing starts at 1/2^L of the
    resolution per side; after every three steps each ray is split into its
    four children, so after 3L steps every full-resolution pixel has its own
    ray.  Reading C2F: a child starts from its parent's current t clamped into
    the child's own unit-sphere interval (a parent that missed the sphere
    contributes -inf, i.e. the child starts at its own entry), every child that
    meets the sphere is re-activated whatever the parent's status, and the
    running minimum-|f| records start empty for each ray ("the minimum absolute
    signed distance value for each pixel along its ray", Sec. 3.3).  Decision
    margins are inherited because the ancestors' decisions shape the child's
    start.

    ``pixels`` (optional flat indices into H*W) restricts the work to those
    pixels and their coarse ancestors; the result at those pixels is identical
    to the full render, other pixels are left as MISS.
    """
    H, W, L = cam.H, cam.W, int(prm.c2f_levels)
    K = int(prm.k_samples)
    c = cam.c
    sel0 = np.zeros(H * W, bool)
    if pixels is None:
        sel0[:] = True
    else:
        sel0[np.asarray(pixels)] = True
    total_queries = 0
    per_step = [0] * int(prm.max_steps)

    def wrapped(idx, P):
        return sdf_fn(P)

    parent = None           # (state, Hl, Wl, index map) of the previous level
    for seg in range(L + 1):
        level = L - seg
        Hl, Wl = H >> level, W >> level
        # which rays of this level exist (ancestors of selected pixels)
        vv, uu = np.divmod(np.nonzero(sel0)[0], W)
        keys = np.unique((vv >> level) * Wl + (uu >> level))
        V, U = np.divmod(keys, Wl)
        xt, yt, D = level_rays(cam, level, U, V)
        inside, t_lo, t_hi, dist, dmarg = unit_sphere_init(c, D, prm.near, prm.far)
        margin = dmarg.copy()
        t0 = t_lo.copy()
        if parent is not None:
            pst, pWl, pmap = parent
            pidx = pmap[(V >> 1) * pWl + (U >> 1)]
            tp = np.where(pst.status[pidx] == MISS, -np.inf, pst.t[pidx])
            t0 = np.minimum(np.maximum(tp, t_lo), t_hi)
            margin = np.minimum(margin, pst.margin[pidx])
        status = np.where(inside, ACTIVE, MISS)
        O = np.broadcast_to(c, D.shape)
        st = new_state(O, D, t0, t_lo, t_hi, status, K, margin)
        n_begin = 3 * seg
        n_end = 3 * (seg + 1) if level > 0 else int(prm.max_steps)
        before = st.queries
        for n in range(n_begin, min(n_end, int(prm.max_steps))):
            q0 = st.queries
            march(wrapped, st, n, n + 1, float(prm.alpha), float(prm.eps), int(prm.max_steps))
            per_step[n] += st.queries - q0
        total_queries += st.queries - before
        if level > 0:
            imap = np.full(Hl * Wl, -1, np.int64)
            imap[keys] = np.arange(keys.size)
            parent = (st, Wl, imap)

    # ---- outputs at full resolution (level 0): `st`, rays at `keys`
    n = H * W
    depth = np.full(n, np.inf)
    distv = np.full(n, np.inf)
    sil = np.full(n, np.inf)
    status_img = np.full(n, MISS, np.int8)
    nsteps_img = np.zeros(n, np.int32)
    margin_img = np.full(n, np.inf)
    xt_img = np.zeros(n)
    yt_img = np.zeros(n)
    dirs = np.zeros((n, 3))
    rec_absf = np.full((K, n), np.inf)
    rec_t = np.zeros((K, n))
    rec_f = np.zeros((K, n))
    rec_n = np.full((K, n), -1, np.int32)
    status_img[keys] = st.status
    nsteps_img[keys] = st.nsteps
    margin_img[keys] = st.margin
    xt_img[keys], yt_img[keys], dirs[keys] = xt, yt, D
    rec_absf[:, keys], rec_t[:, keys], rec_f[:, keys], rec_n[:, keys] = st.rec_absf, st.rec_t, st.rec_f, st.rec_n
    hit = st.status == HIT
    d = st.t + st.f_last                                   # Eq. 1 (see march)
    inv = 1.0 / np.sqrt(xt * xt + yt * yt + 1.0)          # z_c = d / sqrt(xt^2 + yt^2 + 1)
    depth[keys[hit]] = d[hit] * inv[hit]
    distv[keys[hit]] = d[hit]
    # soft silhouette (Sec. 3.3, App. A.3): min |f| - eps inside the unit
    # sphere; (distance of the ray from the origin) - 1 for rays that miss it.
    miss = st.status == MISS
    b = D @ c
    sil[keys[miss]] = ray_origin_distance(c, b[miss]) - 1.0
    sil[keys[~miss]] = st.rec_absf[0, ~miss] - float(prm.eps)

    normal = np.zeros((n, 3))
    nraw = np.zeros((n, 3))
    if int(prm.want_normals):
        hk = keys[hit]
        Ph = c[None, :] + d[hit, None] * D[hit]
        nrm = surface_normals(sdf_fn, Ph, float(prm.normal_delta))
        nraw[hk] = nrm
        ln = np.linalg.norm(nrm, axis=1)
        ok = ln > 0
        normal[hk[ok]] = nrm[ok] / ln[ok, None]

    return Render(H=H, W=W, depth=depth.reshape(H, W), dist=distv.reshape(H, W),
                  normal=normal.reshape(H, W, 3), nraw=nraw.reshape(H, W, 3), sil=sil.reshape(H, W),
                  status=status_img.reshape(H, W), nsteps=nsteps_img.reshape(H, W),
                  margin=margin_img.reshape(H, W), xt=xt_img, yt=yt_img, dirs=dirs, c=c.copy(),
                  rec_absf=rec_absf, rec_t=rec_t, rec_f=rec_f, rec_n=rec_n,
                  queries=total_queries, queries_per_step=per_step)


def surface_normals(sdf_fn: Callable, P: np.ndarray, delta: float) -> np.ndarray:
    """Central differences of f with step delta along each world axis (Sec. 3.3);
    returns the unnormalised vector n (the caller normalises)."""
    out = np.zeros((P.shape[0], 3))
    for i in range(3):
        e = np.zeros(3)
        e[i] = delta
        out[:, i] = (sdf_fn(P + e) - sdf_fn(P - e)) / (2.0 * delta)
    return out


def render(dec: Decoder, Z: np.ndarray, cams: Sequence, pairs: Sequence, prm,
           pixels: Optional[Sequence] = None) -> List[Render]:
    """Render images given as (view, latent) pairs."""
    out = []
    for i, (vi, li) in enumerate(pairs):
        z = np.asarray(Z[li], np.float64)
        cam = cam_from(cams[vi])

        def fn(P, z=z):
            return dec.sdf(np.broadcast_to(z, (P.shape[0], z.size)), P)

        out.append(render_image(fn, cam, prm, None if pixels is None else pixels[i]))
    return out


# ============================================================================
# Losses on the rendered observations (Sec. 4.2.1, App. A.3, App. B.3)
# ============================================================================
def loss_and_grads(r: Render, depth_t, normal_t, sil_t, w_d=10.0, w_s=1.0, w_n=0.0):
    """Loss of one image and its gradient w.r.t. the rendered maps.

    L = (1/HW) [ w_d sum_{fg_r & fg_t} |z_c - z_c*|                 (L1 depth)
               + w_s sum_pix S* max(0,S) + (1-S*) max(0,-S)         (App. A.3)
               + w_n sum_{fg_r & fg_t} (-n . n*) ]                  (App. B.3)
    Reading: a fixed 1/(HW) normaliser; fg_r is the rendered binary
    silhouette (S < 0), fg_t the target's.  sign(0) = 0, max'(0) = 0.
    """
    HW = r.H * r.W
    fg_r = r.sil < 0
    fg_t = np.asarray(sil_t) > 0.5
    m = fg_r & fg_t
    dt = np.asarray(depth_t, np.float64)
    diff = np.where(m, r.depth - np.where(m, dt, 0.0), 0.0)
    S = r.sil
    St = np.asarray(sil_t, np.float64)
    L_d = w_d / HW * np.abs(diff).sum()
    # a term whose weight S* or 1 - S* is zero contributes zero even where S is
    # infinite (pixels left out of a partial render)
    L_s = w_s / HW * (St * np.maximum(np.where(St > 0, S, 0.0), 0)
                      + (1 - St) * np.maximum(-np.where(St < 1, S, 0.0), 0)).sum()
    nt = np.asarray(normal_t, np.float64)
    L_n = w_n / HW * (-(r.normal * nt).sum(-1) * m).sum()
    g_depth = w_d / HW * np.sign(diff)
    g_sil = w_s / HW * (St * (S > 0) - (1 - St) * (S < 0))
    g_normal = np.where(m[..., None], -w_n / HW * nt, 0.0)
    return L_d + L_s + L_n, g_depth, g_normal, g_sil


# ============================================================================
# The paper's approximate gradient (Sec. 3.4, Eq. 2 first term; App. B.2)
# ============================================================================
def gradient_samples(r: Render, prm, g_depth, g_normal, g_sil):
    """Detached sample points and their seeds for one rendered image.

    * depth: d' = alpha sum_n f(p_n) (Eq. 1 without the residual e).  Only the
      K queries of smallest |f| on the ray are kept (Sec. 3.4) and each gets
      the first term of Eq. 2, so the seed is alpha dL/dz_c / sqrt(xt^2 +
      yt^2 + 1) at each of them.  Reading G1: the coefficient is alpha for
      every kept sample (dropping e removes the (1 - alpha) part).  Reading
      G2: a ray with fewer than K queries contributes all of them.
    * silhouette: S = |f(p*)| - eps at the minimum-|f| query p*, so the seed
      is dL/dS * sign(f(p*)); rays that miss the unit sphere do not depend on
      the shape.
    * normal: n_i = (f(p + delta e_i) - f(p - delta e_i)) / (2 delta) at the
      detached surface point p = c + d v; dL/dn = (I - n~ n~^T) dL/dn~ / |n|
      and the six queries get seeds +-(dL/dn_i) / (2 delta).
    Returns (points [m,3], seeds [m]).
    """
    K = int(prm.k_samples)
    alpha = float(prm.alpha)
    delta = float(prm.normal_delta)
    c = r.c
    st = r.status.reshape(-1)
    gd = np.asarray(g_depth, np.float64).reshape(-1)
    gs = np.asarray(g_sil, np.float64).reshape(-1)
    gn = np.asarray(g_normal, np.float64).reshape(-1, 3)
    inv = 1.0 / np.sqrt(r.xt ** 2 + r.yt ** 2 + 1.0)
    pts, seeds = [], []
    hit = st == HIT
    for j in range(K):
        sel = hit & np.isfinite(r.rec_absf[j]) & (gd != 0)
        pts.append(c[None, :] + r.rec_t[j, sel, None] * r.dirs[sel])
        seeds.append(alpha * gd[sel] * inv[sel])
    sel = (st != MISS) & np.isfinite(r.rec_absf[0]) & (gs != 0)
    pts.append(c[None, :] + r.rec_t[0, sel, None] * r.dirs[sel])
    seeds.append(gs[sel] * np.sign(r.rec_f[0, sel]))
    if int(prm.want_normals):
        nraw = r.nraw.reshape(-1, 3)
        ln = np.linalg.norm(nraw, axis=1)
        sel = hit & (ln > 0) & np.any(gn != 0, axis=1)
        nt = nraw[sel] / ln[sel, None]
        g = gn[sel]
        gnr = (g - (g * nt).sum(1, keepdims=True) * nt) / ln[sel, None]
        p = c[None, :] + r.dist.reshape(-1)[sel, None] * r.dirs[sel]
        for i in range(3):
            e = np.zeros(3)
            e[i] = delta
            pts.append(p + e)
            seeds.append(gnr[:, i] / (2.0 * delta))
            pts.append(p - e)
            seeds.append(-gnr[:, i] / (2.0 * delta))
    return np.concatenate(pts, 0), np.concatenate(seeds, 0)


def sample_relu_margin(dec: Decoder, z, r: Render, prm) -> np.ndarray:
    """[H,W] smallest ReLU margin (Decoder.relu_margin) over every point at
    which the paper gradient of a pixel may evaluate the decoder: its K
    minimum-|f| records (the first is also the silhouette sample) and, for
    hits, the six central-difference queries around c + d v (Sec. 3.3, 3.4).
    Background pixels without samples get +inf."""
    n = r.H * r.W
    out = np.full(n, np.inf)
    st = r.status.reshape(-1)
    c = r.c
    for j in range(int(prm.k_samples)):
        sel = (st != MISS) & np.isfinite(r.rec_absf[j])
        P = c[None, :] + r.rec_t[j, sel, None] * r.dirs[sel]
        mg = dec.relu_margin(np.broadcast_to(z, (P.shape[0], z.shape[0])), P)
        out[sel] = np.minimum(out[sel], mg)
    if int(prm.want_normals):
        hit = st == HIT
        p = c[None, :] + r.dist.reshape(-1)[hit, None] * r.dirs[hit]
        zz = np.broadcast_to(z, (p.shape[0], z.shape[0]))
        for i in range(3):
            e = np.zeros(3)
            e[i] = float(prm.normal_delta)
            out[hit] = np.minimum(out[hit], np.minimum(dec.relu_margin(zz, p + e), dec.relu_margin(zz, p - e)))
    return out.reshape(r.H, r.W)


def backward(dec: Decoder, Z, renders: Sequence[Render], pairs, prm, grads, want_theta=True):
    """dL/dz per latent (and dL/dtheta) from per-image map gradients.

    ``grads[i] = (g_depth, g_normal, g_sil)`` for image i.  Re-evaluates the
    decoder at the detached samples (the recompute of App. B.2) and applies the
    chain rule exactly in float64.
    """
    Z = np.asarray(Z, np.float64)
    gz = np.zeros_like(Z)
    gW = [np.zeros_like(W) for W in dec.W]
    gb = [np.zeros_like(b) for b in dec.b]
    for r, (vi, li), (g_d, g_n, g_s) in zip(renders, pairs, grads):
        P, s = gradient_samples(r, prm, g_d, g_n, g_s)
        if P.shape[0] == 0:
            continue
        Zr = np.broadcast_to(Z[li], (P.shape[0], Z.shape[1]))
        gZ, gWi, gbi = dec.sdf_vjp(Zr, P, s, want_theta=want_theta)
        gz[li] += gZ.sum(0)
        for l in range(len(gW)):
            gW[l] += gWi[l]
            gb[l] += gbi[l]
    return gz, gW, gb


GRAZING = 1e-2     # |grad f . v| <= GRAZING |grad f|: no implicit depth term (Reading X1)


def implicit_backward(dec: Decoder, Z, renders: Sequence[Render], pairs, prm, grads):
    """dL/dz with the exact derivative of the depth instead of the paper's
    approximation (the gap that Sec. 3.4 accepts by dropping the second term of
    Eq. 2): at a hit the surface point p = c + d v satisfies f(p, z) = 0, so by
    the implicit function theorem dd/dz = -(df/dz) / (grad_p f . v), evaluated
    at the Eq. 1 point.  Silhouette and normal terms are the paper's.

    Reading X1: pixels whose ray grazes the surface (|grad f . v| <= 1e-2
    |grad f|) get no depth term (the derivative is singular there).
    Returns g_z [n_lat, L].
    """
    Z = np.asarray(Z, np.float64)
    gz = np.zeros_like(Z)
    for r, (vi, li), (g_d, g_n, g_s) in zip(renders, pairs, grads):
        # the paper's silhouette and normal terms
        P, s = gradient_samples(r, prm, np.zeros_like(np.asarray(g_d, np.float64)), g_n, g_s)
        if P.shape[0]:
            gz[li] += dec.sdf_vjp(np.broadcast_to(Z[li], (P.shape[0], Z.shape[1])), P, s,
                                  want_theta=False)[0].sum(0)
        gd = np.asarray(g_d, np.float64).reshape(-1)
        sel = (r.status.reshape(-1) == HIT) & (gd != 0)
        if not np.any(sel):
            continue
        v = r.dirs[sel]
        p = r.c[None, :] + r.dist.reshape(-1)[sel, None] * v
        Zr = np.broadcast_to(Z[li], (p.shape[0], Z.shape[1]))
        gp = dec.sdf_grad_p(Zr, p, np.ones(p.shape[0]))
        gv = (gp * v).sum(1)
        ok = np.abs(gv) > GRAZING * np.linalg.norm(gp, axis=1)
        nrm = np.sqrt(r.xt[sel] ** 2 + r.yt[sel] ** 2 + 1.0)
        seed = np.where(ok, -gd[sel] / nrm / np.where(ok, gv, 1.0), 0.0)
        gz[li] += dec.sdf_vjp(Zr, p, seed, want_theta=False)[0].sum(0)
    return gz


def unrolled_backward(dec: Decoder, Z, cams: Sequence, pairs, prm, grads):
    """dL/dz of the depth and silhouette terms differentiated exactly through
    the unrolled march: Eq. 2 with both of its terms (Sec. 3.4).

    Eq. 2 splits the derivative of a query f(p^(i)(z), z) into the part at the
    detached point, df/dz, and the part through the point, grad_p f . dp/dz
    with dp^(i)/dz = v dt^(i)/dz.  The ray parameter accumulates the steps,
    t^(i+1) = t^(i) + alpha f^(i) (Sec. 3.2), so dt/dz is carried along the
    march in forward mode:
        df^(i)/dz   = df/dz(p^(i)) + (grad_p f(p^(i)) . v) dt^(i)/dz
        dt^(i+1)/dz = dt^(i)/dz + alpha df^(i)/dz.

    Reading U1: the result is the exact derivative of the rendered outputs
    along the forward's discrete trajectory (its step counts, statuses, record
    steps and coarse-to-fine decisions held fixed): the depth through Eq. 1
    with its residual term, d = t^(N-1) + f^(N-1), and the silhouette through
    the minimum-|f| query, S = |f^(k)| - eps, dS/dz = sign f^(k) df^(k)/dz.  A
    child ray of the coarse-to-fine split starts from its parent's t and
    inherits dt/dz unless the clamp into its own interval binds or the parent
    missed the sphere (then 0).  Rays that miss the unit sphere add nothing.

    ``grads[i] = (g_depth, g_sil)``.  Returns g_z [n_lat, L].
    """
    Z = np.asarray(Z, np.float64)
    gz = np.zeros_like(Z)
    for (vi, li), (g_d, g_s) in zip(pairs, grads):
        cam = cam_from(cams[vi])
        dd, ds, st, _ = unrolled_image(dec, Z[li], cam, prm)
        gd = np.asarray(g_d, np.float64).reshape(-1)
        gs = np.asarray(g_s, np.float64).reshape(-1)
        xt, yt, _ = level_rays(cam, 0, *np.divmod(np.arange(cam.H * cam.W), cam.W)[::-1])
        nrm = np.sqrt(xt * xt + yt * yt + 1.0)
        hit = st == HIT
        gz[li] += ((gd * hit / nrm)[:, None] * np.nan_to_num(dd)).sum(0)
        gz[li] += (gs[:, None] * np.nan_to_num(ds)).sum(0)
    return gz


def unrolled_image(dec: Decoder, z, cam: Cam, prm):
    """The march of ``render_image`` carrying dt/dz per ray (see
    ``unrolled_backward``).  Returns, per full-resolution pixel, dd/dz [n, L]
    (hits; NaN elsewhere), dS/dz [n, L] (rays inside the unit sphere; 0 for
    misses), the status and the final t."""
    z = np.asarray(z, np.float64)
    L = z.size
    H, W, Lv = cam.H, cam.W, int(prm.c2f_levels)
    alpha, eps, max_steps = float(prm.alpha), float(prm.eps), int(prm.max_steps)
    c = cam.c
    parent = None
    for seg in range(Lv + 1):
        level = Lv - seg
        Hl, Wl = H >> level, W >> level
        V, U = np.divmod(np.arange(Hl * Wl), Wl)
        _, _, D = level_rays(cam, level, U, V)
        inside, t_lo, t_hi, _, _ = unit_sphere_init(c, D, prm.near, prm.far)
        n = D.shape[0]
        t = t_lo.copy()
        J = np.zeros((n, L))
        if parent is not None:
            pt, pst, pJ, pWl = parent
            pi = (V >> 1) * pWl + (U >> 1)
            tp = np.where(pst[pi] == MISS, -np.inf, pt[pi])
            t = np.minimum(np.maximum(tp, t_lo), t_hi)
            free = (pst[pi] != MISS) & (tp > t_lo) & (tp < t_hi)
            J = np.where(free[:, None], pJ[pi], 0.0)
        status = np.where(inside, ACTIVE, MISS).astype(np.int8)
        rec_absf = np.full(n, np.inf)
        rec_f = np.zeros(n)
        rec_df = np.zeros((n, L))
        dd = np.full((n, L), np.nan)
        n_begin = 3 * seg
        n_end = 3 * (seg + 1) if level > 0 else max_steps
        for step in range(n_begin, min(n_end, max_steps)):
            idx = np.nonzero(status == ACTIVE)[0]
            if idx.size == 0:
                continue
            P = c[None, :] + t[idx, None] * D[idx]
            Zr = np.broadcast_to(z, (idx.size, L))
            f = dec.sdf(Zr, P)
            fz = dec.sdf_vjp(Zr, P, np.ones(idx.size), want_theta=False)[0]
            fp = dec.sdf_grad_p(Zr, P, np.ones(idx.size))
            df = fz + (fp * D[idx]).sum(1)[:, None] * J[idx]          # Eq. 2, both terms
            af = np.abs(f)
            better = af < rec_absf[idx]                               # ties keep the earlier step
            b = idx[better]
            rec_absf[b], rec_f[b], rec_df[b] = af[better], f[better], df[better]
            hit = af < eps
            status[idx[hit]] = HIT
            dd[idx[hit]] = J[idx[hit]] + df[hit]                      # d = t + f (Eq. 1)
            rest, fr, dfr = idx[~hit], f[~hit], df[~hit]
            if step == max_steps - 1:
                status[rest] = UNCONVERGED
                continue
            t[rest] = t[rest] + alpha * fr
            J[rest] = J[rest] + alpha * dfr
            esc = (t[rest] > t_hi[rest]) | (t[rest] < t_lo[rest])
            status[rest[esc]] = ESCAPED
        if level > 0:
            parent = (t, status, J, Wl)
    sgn = np.sign(rec_f)
    ds = np.where((status != MISS)[:, None] & np.isfinite(rec_absf)[:, None], sgn[:, None] * rec_df, 0.0)
    return dd, ds, status, t


def camera_samples(r: Render, prm, g_depth, g_sil):
    """The depth and silhouette samples of ``gradient_samples`` with, for each,
    its ray parameter t and the pixel's camera-frame unit direction u (so that
    p = c + t R u).  Returns (points [m,3], seeds [m], t [m], u [m,3])."""
    K = int(prm.k_samples)
    alpha = float(prm.alpha)
    c = r.c
    st = r.status.reshape(-1)
    gd = np.asarray(g_depth, np.float64).reshape(-1)
    gs = np.asarray(g_sil, np.float64).reshape(-1)
    nrm = np.sqrt(r.xt ** 2 + r.yt ** 2 + 1.0)
    u = np.stack([r.xt / nrm, r.yt / nrm, 1.0 / nrm], axis=1)
    pts, seeds, ts, us = [], [], [], []
    hit = st == HIT
    for j in range(K):
        sel = hit & np.isfinite(r.rec_absf[j]) & (gd != 0)
        t = r.rec_t[j, sel]
        pts.append(c[None, :] + t[:, None] * r.dirs[sel])
        seeds.append(alpha * gd[sel] / nrm[sel])
        ts.append(t)
        us.append(u[sel])
    sel = (st != MISS) & np.isfinite(r.rec_absf[0]) & (gs != 0)
    t = r.rec_t[0, sel]
    pts.append(c[None, :] + t[:, None] * r.dirs[sel])
    seeds.append(gs[sel] * np.sign(r.rec_f[0, sel]))
    ts.append(t)
    us.append(u[sel])
    return np.concatenate(pts, 0), np.concatenate(seeds, 0), np.concatenate(ts, 0), np.concatenate(us, 0)


def camera_backward(dec: Decoder, Z, renders: Sequence[Render], cams: Sequence, pairs, prm, grads):
    """dL/d(camera extrinsics) per view, (g_c [n_views,3], g_R [n_views,3,3]),
    for the depth and silhouette terms (the quantities the paper's camera-pose
    experiment optimises, Sec. 4.1 "Back-Propagation Effectiveness"; App. A.3:
    the silhouette is differentiable w.r.t. the extrinsics).

    Reading F1: as for z (Sec. 3.4), the march points are detached: each
    depth/silhouette sample keeps its ray parameter t, and only its position
    p = c + t R u moves with the camera, so a sample adds
    s grad_p f(p) to dL/dc and s t grad_p f(p) u^T to dL/dR (R_wc, row-major).
    Rays that miss the unit sphere have S = (distance from the origin to the
    ray) - 1, i.e. sqrt(|c|^2 - (c.v)^2) - 1 with v = R u when the foot of the
    perpendicular lies ahead (c.v < 0), else |c| - 1; differentiated exactly.  Normal terms are not included (g_normal
    is not an input here).
    """
    Z = np.asarray(Z, np.float64)
    nv = len(cams)
    g_c = np.zeros((nv, 3))
    g_R = np.zeros((nv, 3, 3))
    for r, (vi, li), (g_d, g_s) in zip(renders, pairs, grads):
        P, s, t, u = camera_samples(r, prm, g_d, g_s)
        if P.shape[0]:
            gp = dec.sdf_grad_p(np.broadcast_to(Z[li], (P.shape[0], Z.shape[1])), P, s)
            g_c[vi] += gp.sum(0)
            g_R[vi] += np.einsum("ki,kj->ij", gp * t[:, None], u)
        # background silhouette of rays that miss the unit sphere
        gs = np.asarray(g_s, np.float64).reshape(-1)
        sel = (r.status.reshape(-1) == MISS) & (gs != 0)
        if np.any(sel):
            c = r.c
            v = r.dirs[sel]
            nrm = np.sqrt(r.xt[sel] ** 2 + r.yt[sel] ** 2 + 1.0)
            uu = np.stack([r.xt[sel] / nrm, r.yt[sel] / nrm, 1.0 / nrm], axis=1)
            b = v @ c
            ahead = b < 0.0
            # foot ahead: S = sqrt(|c|^2 - b^2) - 1; else S = |c| - 1
            q = np.where(ahead, np.sqrt(np.maximum(c @ c - b * b, 0.0)), math.sqrt(c @ c))
            w = gs[sel] / q
            bb = np.where(ahead, b, 0.0)
            g_c[vi] += (w[:, None] * (c[None, :] - bb[:, None] * v)).sum(0)
            dv = -(w * bb)[:, None] * c[None, :]
            g_R[vi] += np.einsum("ki,kj->ij", dv, uu)
    return g_c, g_R


# ============================================================================
# Colour rendering at the hit points (Sec. 3.3 "Color and Semantics"; App. C)
# ============================================================================
class ColorDecoder(Decoder):
    """The colour network of texture rendering: the geometry network's layout
    (App. C) reading the concatenated shape and texture codes, three outputs.

    Reading C1: each channel is c = 0.5 (1 + tanh(m)) (the DeepSDF-style tanh
    output mapped to [0, 1]); the code z is [z_shape, z_tex]; the colour is
    evaluated at the Eq. 1 point of every hit, which the backward treats as
    detached (the principle of Sec. 3.4).
    """

    def color(self, Z, P):
        Z = np.asarray(Z, np.float64)
        P = np.asarray(P, np.float64)
        if P.shape[0] == 0:
            return np.zeros((0, 3))
        h = self._hidden(Z, P)
        m = h @ self.W[-1].T + self.b[-1]
        return 0.5 * (1.0 + np.tanh(m))

    def _hidden(self, Z, P, keep=None):
        x0 = np.concatenate([Z, P], axis=1)
        h = x0
        for l in range(self.nl - 1):
            x = np.concatenate([h, Z, P], axis=1) if (self.skip is not None and l == self.skip) else h
            a = x @ self.W[l].T + self.b[l]
            if keep is not None:
                keep.append((x, a))
            h = np.maximum(a, 0.0)
        return h

    def color_vjp(self, Z, P, seeds):
        """sum_i seeds_i . d c(P_i, Z_i) / dZ_i per row: gZ [n, L]."""
        Z = np.asarray(Z, np.float64)
        P = np.asarray(P, np.float64)
        seeds = np.asarray(seeds, np.float64)
        n = P.shape[0]
        gZ = np.zeros((n, self.L))
        if n == 0:
            return gZ
        keep = []
        h = self._hidden(Z, P, keep)
        m = h @ self.W[-1].T + self.b[-1]
        th = np.tanh(m)
        delta = seeds * 0.5 * (1.0 - th * th)                   # d/dm of the output channels
        g_h = delta @ self.W[-1]
        for l in range(self.nl - 2, -1, -1):
            x, a = keep[l]
            d = g_h * (a > 0.0)
            g_in = d @ self.W[l]
            if l == 0:
                gZ += g_in[:, : self.L]
                break
            if self.skip is not None and l == self.skip:
                nh = self.W[l - 1].shape[0]
                gZ += g_in[:, nh: nh + self.L]
                g_h = g_in[:, :nh]
            else:
                g_h = g_in
        return gZ


def render_color(dec: ColorDecoder, Zc, renders: Sequence[Render], pairs):
    """Colour images [n][H, W, 3] of the hits of geometry renders (image i uses
    code Zc[pairs[i][1]]); 0 off the hits."""
    out = []
    for r, (vi, li) in zip(renders, pairs):
        hit = (r.status == HIT).reshape(-1)
        P = r.c[None, :] + r.dist.reshape(-1)[hit, None] * r.dirs[hit]
        rgb = np.zeros((r.H * r.W, 3))
        rgb[hit] = dec.color(np.broadcast_to(np.asarray(Zc[li], np.float64), (P.shape[0], dec.L)), P)
        out.append(rgb.reshape(r.H, r.W, 3))
    return out


def color_backward(dec: ColorDecoder, Zc, renders: Sequence[Render], pairs, g_rgb):
    """dL/dZc [n_lat, L] from per-image dL/d(colour) [H, W, 3] (hit points detached)."""
    Zc = np.asarray(Zc, np.float64)
    gz = np.zeros_like(Zc)
    for r, (vi, li), g in zip(renders, pairs, g_rgb):
        hit = (r.status == HIT).reshape(-1)
        P = r.c[None, :] + r.dist.reshape(-1)[hit, None] * r.dirs[hit]
        s = np.asarray(g, np.float64).reshape(-1, 3)[hit]
        gz[li] += dec.color_vjp(np.broadcast_to(Zc[li], (P.shape[0], dec.L)), P, s).sum(0)
    return gz


# ============================================================================
# Multi-view photometric loss (Sec. 4, multi-view reconstruction; App. C loss)
# ============================================================================
PHOTO_VIS = 1e-3       # Delta_d^2 below this: the point is visible in both views


def photometric_loss(cams: Sequence, depth, images, pairs, weight=5.0):
    """Cross-view photometric loss and its gradient w.r.t. the rendered depth.

    For every ordered pair (i, j) and every pixel x of view i with a rendered
    depth, the surface point X = c_i + d v_i(x) (d = z_c |(xt, yt, 1)|, Sec. 3.3)
    is projected into view j; the colour of view j there, by bilinear
    interpolation, is the warped image I_{j->i}(x), and the loss adds
    weight / (H W) * sum_channels |I_i(x) - I_{j->i}(x)| (the L1 photometric
    error of the multi-view objective, weight 5.0).

    Reading P1 (visibility, "Delta_d^2 < 0.001"): Delta_d is the depth of X
    in view j's frame minus view j's rendered depth at the pixel nearest to the
    projection; the pixel counts only if that depth is finite and
    Delta_d^2 < 1e-3, X lies in front of view j and the 2x2 interpolation
    footprint lies inside the image.  Reading P2: the visibility decision and
    view j's depth are constants; the gradient flows only through X (the depth
    of view i) and the interpolation weights.

    ``depth``: [n][H,W] z_c (inf = background); ``images``: [n][H,W,3].
    Returns (L, g_depth [n][H,W]).
    """
    cs = [cam_from(c) for c in cams]
    n = len(cs)
    H, W = cs[0].H, cs[0].W
    scale = float(weight) / (H * W)
    g = [np.zeros(H * W) for _ in range(n)]
    L = 0.0
    V, U = np.divmod(np.arange(H * W), W)
    for i, j in pairs:
        ci, cj = cs[i], cs[j]
        zi = np.asarray(depth[i], np.float64).reshape(-1)
        Ii = np.asarray(images[i], np.float64).reshape(-1, 3)
        Ij = np.asarray(images[j], np.float64)
        Dj = np.asarray(depth[j], np.float64)
        xt, yt, Dir = level_rays(ci, 0, U, V)
        nrm = np.sqrt(xt * xt + yt * yt + 1.0)
        fg = np.isfinite(zi)
        X = ci.c[None, :] + np.where(fg, zi * nrm, 0.0)[:, None] * Dir
        Xc = (X - cj.c[None, :]) @ cj.R                 # R^T (X - c) per row
        front = Xc[:, 2] > 0.0
        zc = np.where(front, Xc[:, 2], 1.0)
        a = cj.fx * Xc[:, 0] / zc + cj.cx - 0.5           # pixel-index coordinates in view j
        b = cj.fy * Xc[:, 1] / zc + cj.cy - 0.5
        an = np.floor(a + 0.5).astype(np.int64)
        bn = np.floor(b + 0.5).astype(np.int64)
        a0 = np.floor(a).astype(np.int64)
        b0 = np.floor(b).astype(np.int64)
        ok = fg & front & (an >= 0) & (an < W) & (bn >= 0) & (bn < H)
        ok &= (a0 >= 0) & (a0 + 1 < W) & (b0 >= 0) & (b0 + 1 < H)
        dj = np.where(ok, Dj[np.clip(bn, 0, H - 1), np.clip(an, 0, W - 1)], np.inf)
        ok &= np.isfinite(dj)
        ok &= (Xc[:, 2] - np.where(ok, dj, 0.0)) ** 2 < PHOTO_VIS
        idx = np.nonzero(ok)[0]
        if idx.size == 0:
            continue
        al, be = (a - a0)[idx], (b - b0)[idx]
        A0, B0 = a0[idx], b0[idx]
        I00, I01 = Ij[B0, A0], Ij[B0, A0 + 1]
        I10, I11 = Ij[B0 + 1, A0], Ij[B0 + 1, A0 + 1]
        Iw = ((1 - be)[:, None] * ((1 - al)[:, None] * I00 + al[:, None] * I01)
              + be[:, None] * ((1 - al)[:, None] * I10 + al[:, None] * I11))
        r = Ii[idx] - Iw
        L += scale * float(np.abs(r).sum())
        dIa = (1 - be)[:, None] * (I01 - I00) + be[:, None] * (I11 - I10)
        dIb = (1 - al)[:, None] * (I10 - I00) + al[:, None] * (I11 - I01)
        q = Xc[idx]
        dX = (Dir[idx] * nrm[idx, None]) @ cj.R            # d Xc / d z_c of view i
        da = cj.fx * (dX[:, 0] / q[:, 2] - q[:, 0] * dX[:, 2] / q[:, 2] ** 2)
        db = cj.fy * (dX[:, 1] / q[:, 2] - q[:, 1] * dX[:, 2] / q[:, 2] ** 2)
        dIw = dIa * da[:, None] + dIb * db[:, None]
        g[i][idx] += scale * (-np.sign(r) * dIw).sum(1)
    return L, [gi.reshape(H, W) for gi in g]


# ============================================================================
# Closed forms from the appendix
# ============================================================================
def eps_for_camera(d_min, sensor, focal, resolution, theta=0.0):
    """App. A.2: eps = d_min S cos^2(theta) / (2 f R), the radius at which the
    eps-balls around the front ends of neighbouring pixel rays stop overlapping."""
    return d_min * sensor * math.cos(theta) ** 2 / (2.0 * focal * resolution)


def k_min(eps, d, alpha, theta):
    """App. A.1: smallest k with |d (1 - alpha sin theta)^k| < eps is the first
    integer above (log eps - log d) / log|1 - alpha sin theta|."""
    return (math.log(eps) - math.log(d)) / math.log(abs(1.0 - alpha * math.sin(theta)))


def adam_step(z, g, m, v, t, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Alg. 1), the optimiser the paper uses
    for latent-code fitting (App. B.4: learning rate 1e-2).  t counts from 1.
    Returns the new (z, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return z - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
