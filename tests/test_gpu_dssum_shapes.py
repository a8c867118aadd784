"""Gather-scatter parity over the mesh shapes that select its implementation
(N = 7: two lanes per element-row segment while 2 nelx <= 256, one lane up
to nelx = 256, with x-face values exchanged by shuffles while a row fits a
wavefront and through LDS beyond; the table-driven passes when an axis is
periodic with a single element or the row is longer).  FP64 is bit-exact
against the oracle; FP32 is bit-exact against the same ascending-local-index
sum taken in float32 (numpy's unbuffered ufunc.at adds in index order)."""
import numpy as np
import pytest

from paper_2405_05640_amd import sem
from paper_2405_05640_amd import workloads as wl
from tests.gpu_util import dev, host, pair

pytestmark = pytest.mark.gpu

SHAPES = [
    wl.box(1, 2, 2, 7),                                                            # nelx = 1
    wl.random_deformed_box(2, 2, 3, 7, seed=5, amp=0.2, periodic=(1, 1, 0),
                           dirichlet=0x30),                                        # two-element wraps
    wl.random_deformed_box(32, 1, 2, 7, seed=6, amp=0.2, periodic=(1, 0, 0)),      # 2 nelx = 64 exactly
    wl.random_deformed_box(33, 2, 1, 7, seed=7, amp=0.2),                          # two wavefronts per row
    wl.random_deformed_box(64, 1, 2, 7, seed=8, amp=0.2, periodic=(1, 0, 1),
                           dirichlet=wl.DIRICHLET_Y_WALLS),                        # nelx = 64, periodic
    wl.random_deformed_box(65, 1, 1, 7, seed=9, amp=0.2),                          # two lanes, LDS exchange
    wl.random_deformed_box(130, 1, 1, 7, seed=10, amp=0.2, periodic=(1, 0, 0)),    # one lane, LDS exchange
    wl.random_deformed_box(257, 1, 1, 7, seed=11, amp=0.2),                        # row too long: table passes
    wl.box(2, 1, 3, 7, periodic=(0, 1, 0)),                                        # table-driven passes
]
IDS = ["nelx1", "wrap2", "nelx32_per", "nelx33", "nelx64_per", "nelx65", "nelx130_per", "nelx257",
       "per_single_y"]


@pytest.fixture(scope="module", params=list(range(len(SHAPES))), ids=IDS)
def meshes(request):
    spec = SHAPES[request.param]
    print("mesh", spec.name, spec.nelx, spec.nely, spec.nelz, flush=True)
    return pair(spec)


def dssum_f32_reference(om, u32, mask):
    s = np.zeros(om.n_global, dtype=np.float32)
    np.add.at(s, om.glo.ravel(), u32.ravel())
    out = s[om.glo.ravel()].reshape(om.shape)
    single = (om.mult == 1)
    out[single] = u32[single]            # a node with one copy keeps its value
    if mask:
        out[om.mask.astype(bool)] = 0.0
    return out


def test_dssum_f64_shapes(meshes):
    om, gm = meshes
    rng = np.random.default_rng(50)
    u = rng.standard_normal(om.shape)
    for mask in (False, True):
        t = dev(u)
        gm.dssum(t, mask=mask)
        ref = om.dssum(u)
        if mask:
            ref = om.apply_mask(ref)
        assert np.array_equal(host(t), ref)


def test_dssum_f32_shapes(meshes):
    import torch
    om, gm = meshes
    rng = np.random.default_rng(51)
    u32 = rng.standard_normal(om.shape).astype(np.float32)
    for mask in (False, True):
        t = dev(u32, torch.float32)
        gm.dssum(t, mask=mask, dtype=sem.SEM_F32)
        assert np.array_equal(host(t), dssum_f32_reference(om, u32, mask))
