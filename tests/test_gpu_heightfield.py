"""GPU parity of the heightfield's grid walk: scenes whose only geometry is
a rough heightfield (no BVH at all), seen from above and at a grazing
angle, against the FP64 oracle (which finds hits its own way), detached
and attached, through the C ABI."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_32920_amd import lt, scenes
from gpu_common import GpuRun, matched_paths, maxrel

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def hf_only_scene(G=12, width=32, height=32, sigma=0.08, seed=5, cam=(0.0, 2.2, 0.3), target=(0.0, 0.0, 0.0),
                  up=(0.0, 0.0, 1.0)):
    """A rough Lambertian heightfield over x, z in [-1, 1] (heights
    N(0, sigma)), a point light above it, no other geometry."""
    rng = np.random.default_rng(seed)
    h = rng.normal(0.0, sigma, size=(G, G))
    return dict(
        name="hf_only", tri_v=np.zeros((0, 3, 3)), tri_uv=np.zeros((0, 3, 2)), tri_mat=np.zeros(0, np.int32),
        mat_type=np.array([scenes.MAT_LAMBERT], np.int32), mat_tex=np.array([0], np.int32), mat_ior=np.array([1.0]),
        n_tex=1, tex_res=1,
        emitter=dict(type=scenes.EMIT_POINT, o=np.array([0.2, 1.2, -0.1]), e1=np.zeros(3), e2=np.zeros(3)),
        camera=dict(pos=np.array(cam), target=np.array(target), up=np.array(up), fov_deg=60.0, width=width,
                    height=height),
        hf=dict(G=G, x0=-1.0, z0=-1.0, dx=2.0 / (G - 1), base=0.0, mat=0),
        albedo=np.full((1, 1, 1, 3), 0.7), Le=np.full(3, 3.0), heights=h.reshape(-1).copy(),
        albedo_target=None, heights_target=None)


@pytest.mark.parametrize("view", ["above", "grazing"])
def test_heightfield_only_detached(view):
    kw = {} if view == "above" else dict(cam=(-1.6, 0.25, -1.4), target=(0.5, 0.0, 0.4), up=(0.0, 1.0, 0.0))
    sc = hf_only_scene(**kw)
    g = GpuRun(sc)
    seed, n, D = 7, 1 << 16, 3
    mask, ids, mis = matched_paths(sc, g, seed, n, D)
    assert mis <= 2e-3, mis
    gi = g.trace(seed, n, D, mask=mask)["image"]
    oi = O.render(sc, seed, n, D, path_list=ids)["image"]
    assert np.abs(oi).max() > 0
    assert maxrel(gi, oi) <= TOL
    dI = np.random.default_rng(seed).normal(size=oi.shape)
    on = O.gradient(sc, seed, n, D, dI, path_list=ids)
    for mode in ("naive", "lrb3"):
        gg = g.backward(mode, seed, n, D, dI, mask=mask)
        assert maxrel(gg["albedo"], on["albedo"]) <= TOL, mode
        assert maxrel(gg["Le"], on["Le"]) <= TOL, mode


def test_attached_lambertian_heightfield_is_rejected():
    # attached derivatives cover dielectric and rough-conductor heightfields
    # (the surfaces the paper differentiates); a Lambertian heightfield's
    # facet-normal and frame terms are not carried, so the call refuses
    import torch
    sc = hf_only_scene()
    g = GpuRun(sc)
    img = torch.empty((32, 32, 3), dtype=torch.float32, device=g.dev)
    with pytest.raises(lt.LTError, match="LT_ERR_UNSUPPORTED"):
        g.ctx.trace(g.ctx.args(1, 1024, 3, lt.ATTACHED), g.params(), img)
