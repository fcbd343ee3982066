"""The allocation-free batched entry point (bn_estimate_normals_batch_noalloc)
against the plan-based one it varies (bn_batch_launch on a small list): the
same bits for every output and count, on two calls in a row, the second with
a smaller input, and both against the oracle."""
import numpy as np
import pytest

import oracle
import paper_2209_08241_amd as bn
from gpu_util import assert_parity, log, to_gpu
from synth import scenes

pytestmark = pytest.mark.gpu


def _frames(shapes, seed0):
    host = [scenes.sized_frame(H, W, seed=seed0 + k) for k, (H, W) in enumerate(shapes)]
    return host, [bn.BatchFrame(to_gpu(s.depth), s.fx, s.fy, s.cx, s.cy) for s in host]


def _outputs(frames):
    return [(f.normals.cpu().numpy().copy(), f.mask.cpu().numpy().copy(),
             f.stats.cpu().numpy().copy()) for f in frames]


def _plan_reference(frames, **kw):
    """The same frames through a plan's bn_batch_launch (small-list path)."""
    import torch
    with bn.BatchPlan(frames, **kw) as plan:
        plan.launch()
        torch.cuda.synchronize()
    return _outputs(frames)


@pytest.mark.parametrize("method,alpha,K", [("four_pair", 2, 0), ("pair_removal", 1, 0),
                                           ("multiscale", 2, 3)])
def test_noalloc_equals_plan_launch_twice(method, alpha, K):
    import torch
    kw = dict(alpha=alpha, mode="rel", tau=4.0, method=method, scales=K)
    # call 1: 16 frames (the maximum) of mixed sizes and layouts, 1080p
    # included; call 2: a smaller input (3 small frames)
    big_shapes = [(1080, 1920), (480, 640), (97, 131), (240, 320), (33, 64), (720, 1280),
                  (5, 7), (480, 640)] * 2
    small_shapes = [(240, 320), (61, 83), (120, 160)]
    for call, (shapes, seed0) in enumerate(((big_shapes, 4100), (small_shapes, 4200))):
        host, frames = _frames(shapes, seed0)
        want = _plan_reference(frames, **kw)
        for f in frames:
            f.normals.fill_(7.0)
            f.mask.fill_(9)
            f.stats.fill_(-1)
        torch.cuda.synchronize()
        bn.estimate_normals_batch_noalloc(frames, **kw)
        torch.cuda.synchronize()
        got = _outputs(frames)
        for k, ((gn, gm, gs), (wn, wm, ws), s) in enumerate(zip(got, want, host)):
            what = f"call {call} frame {k} {s.depth.shape} {method}"
            assert np.array_equal(gn.view(np.uint32), wn.view(np.uint32)), what + " normals"
            assert np.array_equal(gm, wm), what + " mask"
            assert np.array_equal(gs, ws), what + " counts"
            ref = oracle.variant_f32(s.depth, s.fx, s.fy, s.cx, s.cy, alpha, "rel", 4.0,
                                     method=method, scales=K)
            assert_parity(ref, gn, gm, gs, what=what + " vs oracle")
        log(f"no-alloc call {call}: {len(frames)} frames equal the plan launch and the oracle")


def test_noalloc_rejects_too_many_frames_and_bad_arguments():
    import torch
    host, frames = _frames([(24, 32)] * 17, 4300)
    with pytest.raises(bn.BnError) as e:
        bn.estimate_normals_batch_noalloc(frames)
    assert e.value.status == bn.BN_ERR_UNSUPPORTED
    with pytest.raises(bn.BnError) as e:
        bn.estimate_normals_batch_noalloc(frames[:2], alpha=0)
    assert e.value.status == bn.BN_ERR_INVALID_ARG
    with pytest.raises(bn.BnError) as e:
        bn.estimate_normals_batch_noalloc([])
    assert e.value.status == bn.BN_ERR_INVALID_ARG
    # nothing was written by the rejected calls
    torch.cuda.synchronize()
    assert all(int(f.stats.sum()) == 0 for f in frames)
