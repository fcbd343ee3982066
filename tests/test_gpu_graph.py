"""The plain and batched entry points inside a captured HIP graph: every
replay, with eager work and synchronisations between replays, equals the
eager result (the path records no memset node)."""
import numpy as np
import pytest

import paper_2209_08241_amd as bn
from synth import scenes

pytestmark = pytest.mark.gpu


def test_plain_launches_replayed_from_a_graph():
    import torch
    s = scenes.frame_640x480(seed=1)
    d = torch.from_numpy(s.depth).cuda()
    n, m, st = bn.estimate_normals(d, *s.intrinsics, 2)
    torch.cuda.synchronize()
    ref = (n.clone(), m.clone(), st[:3].clone())
    n2 = torch.full_like(n, 7.0)
    m2 = torch.full_like(m, 9)
    st2 = bn.new_stats(device="cuda")
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        bn.estimate_normals(d, *s.intrinsics, 2, normals=n2, mask=m2, stats=st2,
                            stream=torch.cuda.current_stream())
    for rep in range(4):
        n2.fill_(float(rep))            # eager work between replays
        m2.fill_(200 + rep)
        st2.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(n2, ref[0]) and torch.equal(m2, ref[1]), f"replay {rep}"
        assert torch.equal(st2[:3], ref[2]), f"replay {rep} counts"


def test_batch_plan_runs_repeatedly_with_eager_work_between():
    import torch
    frames_h = [scenes.sized_frame(H, W, 70 + k) for k, (H, W) in
                enumerate([(240, 320), (480, 640), (97, 131)])]
    frames = [bn.BatchFrame(torch.from_numpy(s.depth).cuda(), s.fx, s.fy, s.cx, s.cy)
              for s in frames_h]
    refs = []
    for s, f in zip(frames_h, frames):
        n, m, st = bn.estimate_normals(f.depth, s.fx, s.fy, s.cx, s.cy, 2)
        refs.append((n, m, st[:3].clone()))
    torch.cuda.synchronize()
    with bn.BatchPlan(frames, 2, "rel", 4.0) as plan:
        for rep in range(4):
            for f in frames:
                f.normals.fill_(float(rep))
                f.mask.fill_(99)
            torch.cuda.synchronize()
            plan.run()
            torch.cuda.synchronize()
            for f, (n, m, st) in zip(frames, refs):
                assert torch.equal(f.normals, n) and torch.equal(f.mask, m), f"replay {rep}"
                assert torch.equal(f.stats[:3], st), f"replay {rep} counts"
