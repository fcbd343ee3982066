"""GPU parity of the batched entry points (bn_batch_plan_*): each frame's
outputs equal the plain entry point's bit for bit and the oracle's (masks
and counts exact, normals within 1e-5)."""
import numpy as np
import pytest

import oracle
import paper_2209_08241_amd as bn
from gpu_util import assert_parity, log, to_gpu
from synth import scenes

pytestmark = pytest.mark.gpu


def _plain(fr, alpha, mode, tau):
    n, m, st = bn.estimate_normals(fr.depth, fr.fx, fr.fy, fr.cx, fr.cy, alpha, mode, tau)
    return n, m, st


def _check_against_plain(frames, alpha=2, mode="rel", tau=4.0):
    import torch
    for k, fr in enumerate(frames):
        n, m, st = _plain(fr, alpha, mode, tau)
        torch.cuda.synchronize()
        assert torch.equal(fr.mask, m), f"frame {k}: mask differs from plain"
        assert torch.equal(fr.normals.view(torch.int32), n.view(torch.int32)), \
            f"frame {k}: normals differ from plain"
        if fr.stats is not None:
            assert torch.equal(fr.stats[:3], st[:3]), f"frame {k}: counts differ from plain"


@pytest.fixture(scope="module")
def mixed_batch():
    log("generating the 256-frame mixed batch")
    return scenes.batch_frames(seed0=1000, workers=8)


def test_mixed_256(mixed_batch):
    """The 256-frame mix (64x 320x240, 96x 640x480, 64x 1280x720,
    32x 1920x1080) in one launch, as the benchmark runs it."""
    import torch
    frames = [bn.BatchFrame(to_gpu(s.depth), s.fx, s.fy, s.cx, s.cy) for s in mixed_batch]
    with bn.BatchPlan(frames, alpha=2, mode="rel", tau=4.0) as plan:
        info = plan.info()
        assert info["pixels"] == 159_744_000
        plan.run()
        torch.cuda.synchronize()
        log("batch ran; checking every frame against the oracle")
        for k, (s, fr) in enumerate(zip(mixed_batch, frames)):
            ref = oracle.normals_f32(s.depth, s.fx, s.fy, s.cx, s.cy, 2, "rel", 4.0)
            st = fr.stats.cpu()
            assert st[:3].tolist() == [int(c) for c in ref["counts"]], f"frame {k} counts"
            assert int(st[3]) == 0, f"frame {k}: reserved word not stored as 0"
            assert_parity(ref, fr.normals.cpu().numpy(), fr.mask.cpu().numpy(),
                          what=f"batch frame {k}")
        log("checking every frame against the plain entry point")
        for fr in frames:
            fr.stats.zero_()
        plan.run()
        torch.cuda.synchronize()
        _check_against_plain(frames)


def _odd_frames(rng, alpha):
    import torch
    frames, host = [], []
    shapes = [(7, 9), (1, 1), (0, 5), (5, 0), (33, 65), (64, 64), (17, 1028), (240, 321),
              (2 * alpha, 50), (120, 160), (3, 4), (480, 640)]
    for H, W in shapes:
        d = rng.uniform(0.7, 3.0, size=(H, W)).astype(np.float32)
        if d.size:
            d[rng.random((H, W)) < 0.03] = 0.0
        host.append(d)
    for k, d in enumerate(host):
        H, W = d.shape
        pad = 3 if k % 3 == 1 else 0          # strided rows -> scalar tiles
        t = to_gpu(d, stride_pad=pad)
        fx = 200.0 + 10 * k
        fr = bn.BatchFrame(t, fx, fx * 1.05, (W - 1) / 2, (H - 1) / 2,
                           want_stats=(k % 4 != 2))
        frames.append(fr)
    return frames, host


@pytest.mark.parametrize("alpha", [1, 2, 3, 6])
@pytest.mark.parametrize("mode,tau", [("rel", 4.0), ("abs", 5e-4), ("none", 1.0)])
def test_mixed_layouts(alpha, mode, tau):
    """Vector and scalar tiles, empty and tiny frames, frames without counts."""
    import torch
    rng = np.random.default_rng(alpha * 7 + len(mode))
    frames, host = _odd_frames(rng, alpha)
    with bn.BatchPlan(frames, alpha=alpha, mode=mode, tau=tau) as plan:
        plan.run()
        torch.cuda.synchronize()
        for k, (d, fr) in enumerate(zip(host, frames)):
            ref = oracle.normals_f32(d, fr.fx, fr.fy, fr.cx, fr.cy, alpha, mode, tau)
            st = fr.stats.cpu().numpy() if fr.stats is not None else None
            assert_parity(ref, fr.normals.cpu().numpy(), fr.mask.cpu().numpy(), st,
                          what=f"odd frame {k} {d.shape}")
        for fr in frames:
            if fr.stats is not None:
                fr.stats.zero_()
        plan.run()
        torch.cuda.synchronize()
        _check_against_plain(frames, alpha, mode, tau)


def test_update_and_repeat():
    import torch
    rng = np.random.default_rng(11)
    frames, host = _odd_frames(rng, 2)
    with bn.BatchPlan(frames, alpha=2) as plan:
        for _ in range(3):
            plan.run()
        torch.cuda.synchronize()
        for k, (d, fr) in enumerate(zip(host, frames)):
            if fr.stats is None:
                continue
            ref = oracle.normals_f32(d, fr.fx, fr.fy, fr.cx, fr.cy, 2, "rel", 4.0)
            st = fr.stats.cpu()
            # each run stores the frame's counts (not added up over the runs)
            assert st[:3].tolist() == [int(c) for c in ref["counts"]]
            assert int(st[3]) == 0
        # a different, shorter list through the same plan (same graph)
        new = [scenes.sized_frame(240, 320, seed=77), scenes.sized_frame(480, 640, seed=78)]
        nf = [bn.BatchFrame(to_gpu(s.depth), s.fx, s.fy, s.cx, s.cy) for s in new]
        plan.update(nf)
        plan.run()
        torch.cuda.synchronize()
        assert plan.info()["pixels"] == 240 * 320 + 480 * 640
        for s, fr in zip(new, nf):
            ref = oracle.normals_f32(s.depth, s.fx, s.fy, s.cx, s.cy, 2, "rel", 4.0)
            assert_parity(ref, fr.normals.cpu().numpy(), fr.mask.cpu().numpy(),
                          fr.stats.cpu().numpy(), what="updated frame")
        with pytest.raises(bn.BnError):
            plan.update(nf * 20)        # over capacity


def test_plan_errors():
    import torch
    d = torch.ones((8, 8), dtype=torch.float32, device="cuda")
    good = bn.BatchFrame(d, 500.0, 500.0, 3.5, 3.5)
    bad = bn.BatchFrame(d, -1.0, 500.0, 3.5, 3.5)
    for frames, kw, status in (([good, bad], {}, bn.BN_ERR_INVALID_ARG),
                               ([good], {"alpha": 9}, bn.BN_ERR_UNSUPPORTED),
                               ([good], {"alpha": 0}, bn.BN_ERR_INVALID_ARG),
                               ([good], {"tau": -1.0}, bn.BN_ERR_INVALID_ARG)):
        with pytest.raises(bn.BnError) as e:
            bn.BatchPlan(frames, **kw)
        assert e.value.status == status
    with pytest.raises(bn.BnError):
        bn.BatchPlan([])


def test_graph_replay_deterministic(mixed_batch):
    import torch
    sub = mixed_batch[::16]
    frames = [bn.BatchFrame(to_gpu(s.depth), s.fx, s.fy, s.cx, s.cy) for s in sub]
    with bn.BatchPlan(frames) as plan:
        plan.run()
        torch.cuda.synchronize()
        first = [(f.normals.clone(), f.mask.clone(), f.stats[:3].clone()) for f in frames]
        for _ in range(4):
            for f in frames:
                f.stats.zero_()
            plan.run()
            torch.cuda.synchronize()
            for (n0, m0, s0), f in zip(first, frames):
                assert torch.equal(n0.view(torch.int32), f.normals.view(torch.int32))
                assert torch.equal(m0, f.mask)
                assert torch.equal(s0, f.stats[:3])


def test_direct_launch_equals_graph_replay():
    """bn_batch_launch writes what bn_batch_run writes, across updates that
    change the frame list in between (the graph picks its new parameters up
    at its next replay, whichever call came before)."""
    import torch
    lists = [[scenes.sized_frame(240, 320, seed=90), scenes.sized_frame(97, 131, seed=91)],
             [scenes.sized_frame(480, 640, seed=92)],
             [scenes.sized_frame(120, 160, seed=93), scenes.sized_frame(720, 1280, seed=94),
              scenes.sized_frame(33, 65, seed=95)]]
    first = [bn.BatchFrame(to_gpu(s.depth), s.fx, s.fy, s.cx, s.cy) for s in lists[0]]
    with bn.BatchPlan(first + first[:1], alpha=2) as plan:
        for k, lst in enumerate(lists):
            frames = [bn.BatchFrame(to_gpu(s.depth), s.fx, s.fy, s.cx, s.cy) for s in lst]
            plan.update(frames)
            order = ("launch", "run") if k % 2 == 0 else ("run", "launch")
            got = {}
            for how in order:
                for f in frames:
                    f.normals.fill_(7.0)
                    f.mask.fill_(9)
                    f.stats.zero_()
                getattr(plan, how)()
                torch.cuda.synchronize()
                got[how] = [(f.normals.clone(), f.mask.clone(), f.stats.clone()) for f in frames]
            for (n0, m0, s0), (n1, m1, s1) in zip(got["run"], got["launch"]):
                assert torch.equal(n0.view(torch.int32), n1.view(torch.int32))
                assert torch.equal(m0, m1)
                assert torch.equal(s0, s1)
            for s, (n, m, st) in zip(lst, got["launch"]):
                ref = oracle.normals_f32(s.depth, s.fx, s.fy, s.cx, s.cy, 2, "rel", 4.0)
                assert_parity(ref, n.cpu().numpy(), m.cpu().numpy(), st.cpu().numpy(),
                              what=f"list {k} {s.depth.shape}")


def _plain_outputs(fr, alpha, mode, tau, method="four_pair", scales=0):
    import torch
    n, m, st = bn.estimate_normals(fr.depth, fr.fx, fr.fy, fr.cx, fr.cy, alpha, mode, tau,
                                   method=method, scales=scales)
    torch.cuda.synchronize()
    return n, m, st


def _assert_equal_plain(frames, alpha, mode, tau, method="four_pair", scales=0, times=1):
    import torch
    for k, fr in enumerate(frames):
        n, m, st = _plain_outputs(fr, alpha, mode, tau, method, scales)
        assert torch.equal(fr.normals.view(torch.int32), n.view(torch.int32)), f"frame {k}"
        assert torch.equal(fr.mask, m), f"frame {k}"
        if fr.stats is not None:
            assert fr.stats[:3].tolist() == [times * c for c in st[:3].tolist()], f"frame {k}"


@pytest.mark.parametrize("method,alpha,K", [("four_pair", 2, 0), ("pair_removal", 1, 0),
                                           ("multiscale", 2, 3), ("multiscale", 3, 3)])
def test_small_lists(method, alpha, K):
    """Lists of at most 16 frames carry their descriptors in the kernel
    arguments and reduce their counts in the same kernel: outputs and counts
    equal the plain launches, through the graph and through plain launches,
    and repeated runs with the accumulate flag add the counts (the work
    areas return to zero)."""
    import torch
    rng = np.random.default_rng(alpha * 10 + K)
    sizes = [(97, 131), (240, 320), (0, 8), (33, 64), (480, 640), (5, 7)]
    host = [scenes.sized_frame(H, W, seed=300 + k) if H > 0 else None
            for k, (H, W) in enumerate(sizes)]
    frames = []
    for s, (H, W) in zip(host, sizes):
        if s is None:
            frames.append(bn.BatchFrame(torch.empty((0, W), device="cuda"), 100.0, 100.0,
                                        3.5, 0.0))
        else:
            frames.append(bn.BatchFrame(to_gpu(s.depth), s.fx, s.fy, s.cx, s.cy))
    for n in (1, 4, len(frames)):
        sub = frames[:n]
        with bn.BatchPlan(sub, alpha, "rel", 4.0, method=method, scales=K,
                          accumulate_counts=True) as plan:
            for how in ("run", "launch"):
                for f in sub:
                    f.stats.zero_()
                for _ in range(3):
                    getattr(plan, how)()
                torch.cuda.synchronize()
                _assert_equal_plain(sub, alpha, "rel", 4.0, method, K, times=3)
    log(f"small lists {method} alpha={alpha} K={K} ok (rng {rng.integers(9)})")


def test_small_and_table_lists_through_one_plan():
    """One plan alternates between lists above and below the small-list
    limit; every list's outputs equal the plain launches, and every list
    stores its counts over whatever the stats held."""
    import torch
    pool = [scenes.sized_frame(H, W, seed=400 + k) for k, (H, W) in
            enumerate([(120, 160), (97, 131), (240, 320), (64, 64)] * 6)]
    frames = [bn.BatchFrame(to_gpu(s.depth), s.fx, s.fy, s.cx, s.cy) for s in pool]
    with bn.BatchPlan(frames, 2, "rel", 4.0) as plan:
        for n, how in ((3, "launch"), (24, "run"), (16, "run"), (17, "launch"), (1, "run"),
                       (24, "launch"), (2, "launch")):
            sub = frames[:n]
            plan.update(sub)
            for f in sub:
                f.normals.fill_(5.0)
                f.mask.fill_(7)
                f.stats.fill_(3)   # stored over: counts and reserved word
            getattr(plan, how)()
            torch.cuda.synchronize()
            info = plan.info()
            assert info["tiles"] == sum(
                (f.depth.shape[0] * (f.depth.shape[1] // 4 if f.depth.shape[1] % 4 == 0
                                     else f.depth.shape[1]) + 255) // 256 for f in sub)
            for k, f in enumerate(sub):
                n_, m_, st_ = _plain_outputs(f, 2, "rel", 4.0)
                assert torch.equal(f.normals.view(torch.int32), n_.view(torch.int32)), (n, k)
                assert torch.equal(f.mask, m_), (n, k)
                assert f.stats.tolist() == st_.tolist(), (n, k)


def test_large_frame_counts_in_chunks():
    """A frame of more than 4096 tiles has its counts summed in chunks that
    combine through the plan's work area: counts equal the plain launch's,
    stored by default and added over repeated runs with the accumulate
    flag."""
    import torch
    big = scenes.sized_frame(3072, 4096, seed=700)
    small = [scenes.sized_frame(40, 64, seed=701 + k) for k in range(16)]
    frames = [bn.BatchFrame(to_gpu(s.depth), s.fx, s.fy, s.cx, s.cy) for s in [big] + small]
    want = [_plain_outputs(f, 2, "rel", 4.0)[2][:3].tolist() for f in frames]
    for accumulate in (True, False):
        with bn.BatchPlan(frames, 2, "rel", 4.0, accumulate_counts=accumulate) as plan:
            for f in frames:
                f.stats.zero_()
            for how in ("run", "launch", "run"):
                getattr(plan, how)()
            torch.cuda.synchronize()
            times = 3 if accumulate else 1
            for k, f in enumerate(frames):
                assert f.stats[:3].tolist() == [times * c for c in want[k]], (accumulate, k)
    n, m, _ = _plain_outputs(frames[0], 2, "rel", 4.0)
    assert torch.equal(frames[0].normals.view(torch.int32), n.view(torch.int32))
    assert torch.equal(frames[0].mask, m)
