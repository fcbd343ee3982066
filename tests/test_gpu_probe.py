"""The bandwidth probes run and move the bytes they claim."""
import pytest

import paper_2209_08241_amd as bn

pytestmark = pytest.mark.gpu


def test_stream_copy_copies():
    import torch
    src = torch.randn(1 << 20, device="cuda")
    dst = torch.zeros_like(src)
    bn.stream_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


def test_stream_pattern_writes_every_output():
    import torch
    px = 64 * 1024
    depth = torch.full((px,), 1.5, device="cuda")
    normals = torch.zeros(3 * px, device="cuda")
    mask = torch.full((px,), 7, dtype=torch.uint8, device="cuda")
    bn.stream_pattern(depth, normals, mask)
    torch.cuda.synchronize()
    n = normals.view(px // 4, 12)
    # each thread's 4 pixels: centre, 2x centre, 3x centre
    assert torch.all(n[:, 0:4] == 1.5) and torch.all(n[:, 4:8] == 3.0) and torch.all(n[:, 8:12] == 4.5)
    assert torch.all(mask == 0) or torch.all(mask < 2)


def test_alu_probe_computes_its_chains():
    """Each thread's output is the binary32 sum of its 8 chains, each chain
    multiplied by m `iters` times in order, as numpy computes it."""
    import numpy as np
    import torch
    out = torch.zeros(2 * 256, device="cuda")
    iters, m = 37, np.float32(1.0001)
    n = bn.alu_probe(out, iters, float(m))
    torch.cuda.synchronize()
    assert n == 2 * 256 * 8 * iters
    t = np.arange(256, dtype=np.float32)
    want = np.zeros(256, dtype=np.float32)
    for c in range(8):
        x = np.float32(1.0) + np.float32(1e-3) * (t + np.float32(c))
        for _ in range(iters):
            x = (x * m).astype(np.float32)
        want = (want + x).astype(np.float32)
    got = out.cpu().numpy().reshape(2, 256)
    assert np.array_equal(got[0], want) and np.array_equal(got[1], want)
