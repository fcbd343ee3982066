"""The autotuner picks among variants / grids that all give identical output."""
import os

import numpy as np
import pytest

import oracle
import paper_2209_08241_amd as bn
from gpu_util import assert_parity, gpu_normals, log, to_gpu
from synth import scenes

pytestmark = pytest.mark.gpu


def test_autotune_plain_and_cache(tmp_path):
    bn.autotune_reset()
    v, us = bn.autotune_plain(1080, 1920, alpha=2)
    log(f"plain 1920x1080 tuned: variant {v} ({dict(bn.variants())[v]}), {us:.2f} us")
    assert v in dict(bn.variants()) and us > 0
    assert bn.autotune_entries() == 1
    s = scenes.frame_1920x1080(seed=3)
    ref = oracle.normals_f32(s.depth, *s.intrinsics, 2, "rel", 4.0)
    n, m, st = gpu_normals(s.depth, *s.intrinsics, 2, "rel", 4.0, 0)
    assert_parity(ref, n, m, st, what="after plain autotune")
    p = str(tmp_path / "tune.json")
    bn.autotune_save(p)
    bn.autotune_reset()
    assert bn.autotune_entries() == 0
    bn.autotune_load(p)
    assert bn.autotune_entries() == 1
    bn.autotune_reset()


def test_autotune_batch_grid():
    import torch
    bn.autotune_reset()
    frs = scenes.batch_frames(seed0=1000, indices=range(0, 256, 8))
    frames = [bn.BatchFrame(to_gpu(s.depth), s.fx, s.fy, s.cx, s.cy) for s in frs]
    with bn.BatchPlan(frames) as plan:
        k, us = plan.autotune()
        tuned_wg = plan.info()["workgroups"]
        log(f"batch grid tuned: shape {k}, {us:.1f} us")
        assert k in (0, -2, -4, 2, 4, 8)
        info = plan.info()
        per = max(1, -k)
        assert info["workgroups"] == ((info["tiles"] + per - 1) // per if k <= 0 else 256 * k)
        for f in frames:
            f.stats.zero_()
        plan.run()
        torch.cuda.synchronize()
        for s, f in zip(frs, frames):
            ref = oracle.normals_f32(s.depth, *s.intrinsics, 2, "rel", 4.0)
            assert_parity(ref, f.normals.cpu().numpy(), f.mask.cpu().numpy(),
                          f.stats.cpu().numpy(), what="after batch autotune")
    # a new plan of the same size class starts from the tuned grid
    with bn.BatchPlan(frames) as plan2:
        assert plan2.info()["workgroups"] == tuned_wg
    bn.autotune_reset()


@pytest.mark.parametrize("shape", [-1, -2, -4, 2, 4, 8])
def test_every_batch_shape_is_bit_identical(tmp_path, shape):
    """Each grid shape the batch autotuner chooses among, forced through a
    recorded table entry, gives the plain launches' outputs bit for bit."""
    import json
    import torch
    frs = scenes.batch_frames(seed0=1000, indices=range(0, 256, 8))
    frames = [bn.BatchFrame(to_gpu(s.depth), s.fx, s.fy, s.cx, s.cy) for s in frs]
    px = sum(s.depth.size for s in frs)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    entry = {"arch": arch, "kind": "batch", "method": 0, "alpha": 2, "class": px.bit_length(),
             "value": shape, "us": 1.0}
    path = tmp_path / "shape.json"
    path.write_text('{"entries": [\n ' + json.dumps(entry) + "\n]}\n")
    bn.autotune_reset()
    bn.autotune_load(str(path))
    try:
        with bn.BatchPlan(frames) as plan:
            info = plan.info()
            per = max(1, -shape)
            want_wg = (info["tiles"] + per - 1) // per if shape < 0 else 256 * shape
            assert info["workgroups"] == want_wg, (shape, info)
            plan.run()
            torch.cuda.synchronize()
            for k, f in enumerate(frames):
                n, m, st = bn.estimate_normals(f.depth, f.fx, f.fy, f.cx, f.cy, 2)
                torch.cuda.synchronize()
                assert torch.equal(f.normals.view(torch.int32), n.view(torch.int32)), (shape, k)
                assert torch.equal(f.mask, m), (shape, k)
                assert torch.equal(f.stats, st), (shape, k)
    finally:
        bn.autotune_reset()
