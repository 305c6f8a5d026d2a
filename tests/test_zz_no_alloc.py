"""The allocation-free edge evaluation (gba_eval_edges_noalloc) through the C
ABI: the same outputs as gba_eval_edges on two calls in a row (the second on
a smaller graph, so stale scratch contents would show), no call of the
device allocator during the call, and its limits reported as errors.
"""
import numpy as np
import pytest

from paper_2509_26581_amd import gba, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gba.load()


class _CountingAllocator(gba._Allocator):
    """PyTorch's caching allocator behind callbacks that count their calls."""

    def __init__(self):
        import torch
        self.n_alloc = 0

        def _alloc(nbytes, ctx):
            self.n_alloc += 1
            return torch.cuda.caching_allocator_alloc(int(nbytes), 0,
                                                      torch.cuda.current_stream(0).cuda_stream)

        def _free(ptr, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        super().__init__(_alloc, _free)


def _handle(sc, allocator, active=None):
    h = gba.gba_create(gba.GBA_FP64, 0, allocator)
    gba.gba_set_stream(h, gba.torch_stream(0))
    gba.gba_add_cameras(h, np.arange(sc.n_cams), sc.cams0)
    gba.gba_add_points(h, np.arange(sc.n_pts), sc.pts0)
    gba.gba_add_edges(h, sc.cam_idx, sc.pt_idx, sc.obs)
    gba.gba_set_robust_kernel(h, gba.GBA_LOSS_HUBER, 1.0)
    if active is not None:
        for e in np.flatnonzero(~active):
            gba.gba_set_edge_active(h, int(e), False)
    return h


def test_noalloc_edge_evaluation_equals_the_allocating_call():
    import torch
    torch.cuda.set_device(0)
    alloc = _CountingAllocator()
    big = synth.make_scene("small", seed=61, n_cams=12, n_pts=3000)     # ~16k edges
    act = np.ones(big.n_obs, bool)
    act[::11] = False
    small = synth.make_scene("small", seed=62, n_cams=5, n_pts=200)     # ~1k edges
    for sc, active in ((big, act), (small, None)):
        h = _handle(sc, alloc, active)
        gba.gba_prepare(h)
        want = gba.gba_eval_edges(h, sc.n_obs)
        torch.cuda.synchronize()
        before = alloc.n_alloc
        got = gba.gba_eval_edges_noalloc(h, sc.n_obs)
        assert alloc.n_alloc == before, "the allocation-free call used the allocator"
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b)
        if active is not None:
            assert not got[0][~active].any() and not got[1][~active].any()
            assert np.abs(got[1][active]).max() > 0
        gba.gba_destroy(h)


def test_noalloc_limits_are_errors():
    alloc = _CountingAllocator()
    sc = synth.make_scene("small", seed=63, n_cams=4, n_pts=50)
    h = _handle(sc, alloc)
    with pytest.raises(gba.GbaError) as e:
        gba.gba_eval_edges_noalloc(h, sc.n_obs)          # not prepared yet
    assert e.value.status == -7
    gba.gba_destroy(h)
    # more edges than the scratch holds
    n = gba.GBA_NOALLOC_MAX_EDGES + 1
    h = gba.gba_create(gba.GBA_FP64, 0, None)
    try:
        gba.gba_add_cameras(h, [0], np.array([[0, 0, 0, 0, 0, 0, 500.0, 0, 0]]))
        gba.gba_add_points(h, np.arange(n), np.tile([0.0, 0.0, -10.0], (n, 1)))
        gba.gba_add_edges(h, np.zeros(n, np.int64), np.arange(n), np.zeros((n, 2)))
        gba.gba_prepare(h)
        with pytest.raises(gba.GbaError) as e:
            gba.gba_eval_edges_noalloc(h, n)
        assert e.value.status == -8
    finally:
        gba.gba_destroy(h)
