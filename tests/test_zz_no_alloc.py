"""The allocation-free decoder query (dist_sdf_eval_noalloc) against
dist_sdf_eval, called through the C ABI (run with -m gpu).

Both run the same kernels on the same folded biases, so their outputs must be
identical bit for bit.  Two calls in a row, the second with fewer points and
fewer latents, check that the shared scratch array keeps no state that
matters from one call to the next; a request beyond the scratch is refused.
Captured in a HIP graph (the callers it is for), a call replays to the eager
result bit for bit, with eager work between the replays, and follows its
inputs when they change in place.
"""
import ctypes
import sys

import numpy as np
import pytest

import dist_inputs as di
from _common import gpu_ctx

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


def _inputs(n, n_lat, L, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    P = torch.tensor(rng.uniform(-0.8, 0.8, (n, 3)).astype(np.float32), device="cuda")
    ids = torch.tensor(rng.integers(0, n_lat, n).astype(np.int32), device="cuda")
    Z = torch.tensor(rng.normal(0, 0.05, (n_lat, L)).astype(np.float32), device="cuda")
    return P, ids, Z


@pytest.mark.parametrize("spec", [di.DEEPSDF_SPEC, di.C1_SPEC], ids=["deepsdf", "c1"])
@pytest.mark.parametrize("precision", [0, 1, 2], ids=["fp32", "bf16", "split"])
def test_noalloc_eval_equals_eval(spec, precision):
    from paper_1911_13225_amd import api
    ctx = gpu_ctx(spec)
    lib = ctx.lib
    s = torch.cuda.current_stream().cuda_stream
    # the second call is smaller in both points (a ragged tail) and latents
    for call, (n, n_lat, seed) in enumerate([(5000, 6, 11), (1733, 2, 12)]):
        P, ids, Z = _inputs(n, n_lat, spec.latent_dim, seed)
        _log("case", spec.out_dims[0], "precision", precision, "call", call, "n", n, "latents", n_lat)
        ref = api.dist_sdf_eval(ctx, P, ids, Z, precision)
        out = torch.full((n,), float("nan"), device="cuda")
        rc = lib.dist_sdf_eval_noalloc(ctx.handle, ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(ids.data_ptr()),
                                       ctypes.c_void_p(Z.data_ptr()), n_lat, n, precision,
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s))
        assert rc == 0, lib.dist_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), float((out - ref).abs().max())
    ctx.close()


def test_noalloc_eval_refuses_beyond_the_scratch():
    from paper_1911_13225_amd import api, _native as N
    spec = di.DEEPSDF_SPEC
    ctx = gpu_ctx(spec)
    P, ids, Z = _inputs(64, 257, spec.latent_dim, 13)
    out = torch.empty(64, device="cuda")
    with pytest.raises(N.DistError) as e:
        api.dist_sdf_eval_noalloc(ctx, P, ids, Z, 1, out)
    assert e.value.code == -1
    # the largest request that fits still works afterwards
    P, ids, Z = _inputs(300, 256, spec.latent_dim, 14)
    out = torch.empty(300, device="cuda")
    api.dist_sdf_eval_noalloc(ctx, P, ids, Z, 1, out)
    ref = api.dist_sdf_eval(ctx, P, ids, Z, 1)
    assert torch.equal(out, ref)
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1, 2], ids=["fp32", "bf16", "split"])
def test_noalloc_eval_replays_in_a_captured_graph(precision):
    from paper_1911_13225_amd import api
    spec = di.DEEPSDF_SPEC
    ctx = gpu_ctx(spec)
    P, ids, Z = _inputs(4000, 5, spec.latent_dim, 21)
    out = torch.full((4000,), float("nan"), device="cuda")
    ref = api.dist_sdf_eval(ctx, P, ids, Z, precision)
    # one call outside the capture first, on the stream the capture will use
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        api.dist_sdf_eval_noalloc(ctx, P, ids, Z, precision, out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    _log("graph capture, precision", precision)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        api.dist_sdf_eval_noalloc(ctx, P, ids, Z, precision, out)
    for k in range(4):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), k
    # the graph reads its inputs where they are: change them in place
    P.mul_(0.9)
    Z.mul_(1.1)
    ref2 = api.dist_sdf_eval(ctx, P, ids, Z, precision)
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(out, ref2)
    del g
    ctx.close()
