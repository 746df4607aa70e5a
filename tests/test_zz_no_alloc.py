"""The no-allocation LRB-3 backward (lt_backward_lrb3_noalloc) against the
ordinary entry point (lt_backward_lrb3), through the C ABI: two calls in a
row on the same GPU, the second with fewer paths (the static scratch keeps
the first call's contents, so anything that must start at zero is cleared by
the call itself), detached (fused and two-kernel forms) and attached (the
two-kernel form, its hand-off in the scratch).  Same kernels on both sides,
so results agree to FP32 atomic summation order: max rel 1e-4 (the bar of
the oracle comparisons), measured ~1e-6.  Sizes beyond the scratch and
guided calls are rejected before anything is enqueued."""
import numpy as np
import pytest
import torch

from paper_2609_32920_amd import lt, scenes

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _maxrel(a, b):
    a, b = a.double(), b.double()
    den = b.abs().max().item()
    assert den > 0
    return (a - b).abs().max().item() / den


def _case(sc, flags, sizes, split):
    dev = torch.device("cuda", 0)
    ctx = lt.Context(0).scene_upload(sc)
    ctx.set_tuning(lrb3_split=split)
    f32 = lambda x: torch.as_tensor(np.asarray(x, np.float32), device=dev).contiguous()
    alb, Le = f32(sc["albedo"]), f32(sc["Le"])
    h = f32(sc["heights"]) if sc.get("heights") is not None else None
    p = ctx.params(alb, Le, h)
    H, W = sc["camera"]["height"], sc["camera"]["width"]
    gen = torch.Generator(device=dev).manual_seed(3)
    dI = (torch.randn((H, W, 3), device=dev, generator=gen) * 1e-2).contiguous()
    for k, n in enumerate(sizes):
        a = ctx.args(40 + k, n, 6, flags)
        out = {}
        for name, fn in (("noalloc", ctx.backward_lrb3_noalloc), ("ordinary", ctx.backward_lrb3)):
            ga, gl = torch.zeros_like(alb), torch.zeros_like(Le)
            gh = torch.zeros_like(h) if h is not None else None
            fn(a, p, dI, ga, gl, gh)
            torch.cuda.synchronize()
            out[name] = (ga, gl, gh)
        e = [_maxrel(out["noalloc"][i], out["ordinary"][i]) for i in range(3) if out["ordinary"][i] is not None]
        print(f"{sc['name']} flags {flags} split {split} call {k} ({n} paths): "
              f"max rel {' '.join(f'{x:.1e}' for x in e)}", flush=True)
        assert max(e) <= TOL
    return ctx, p, alb, Le, h, dI


@pytest.mark.parametrize("split", [0, 1])
def test_noalloc_matches_ordinary_detached(split):
    _case(scenes.box_scene(width=64, height=64), 0, (300_000, 100_000), split)


def test_noalloc_matches_ordinary_attached():
    ctx, p, alb, Le, h, dI = _case(scenes.caustic_scene(G=32, width=64, height=64), lt.ATTACHED,
                                   (400_000, 150_000), 2)
    # beyond the scratch's hand-off capacity: rejected, nothing written
    ga, gl, gh = torch.zeros_like(alb), torch.zeros_like(Le), torch.zeros_like(h)
    with pytest.raises(lt.LTError) as e:
        ctx.backward_lrb3_noalloc(ctx.args(1, 600_000, 6, lt.ATTACHED), p, dI, ga, gl, gh)
    assert e.value.status == lt.LT_ERR_ARG
    # a guided call is refused (its emission records would be allocated)
    gw = torch.as_tensor(scenes.guide_weights(), dtype=torch.float32, device=alb.device)
    with pytest.raises(lt.LTError) as e:
        ctx.backward_lrb3_noalloc(ctx.args(1, 1000, 6, lt.ATTACHED), ctx.params(alb, Le, h, gw), dI, ga, gl, gh)
    assert e.value.status == lt.LT_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert not ga.any() and not gl.any() and not gh.any()
