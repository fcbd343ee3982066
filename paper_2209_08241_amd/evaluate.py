"""Accuracy of the estimators on synthetic depth, in the paper's terms
(Section 4): the mean squared error of the theta and phi angle images
(Eqs. 14-15) against a ground truth, over the pixels each estimator keeps.

Two ground truths are used: the analytic normals of the generated scene, and
the 25-neighbour local plane fit that the paper uses on real data.  The
sweep covers the methods of this library (four-pair, pair removal,
multi-scale single pair), alpha, and the depth noise level.  Everything on
the estimator side runs on the GPU through the library's entry points.

    python -m paper_2209_08241_amd.evaluate [--frames 4] [--json out.json]
"""
from __future__ import annotations

import argparse
import json
import sys

CONFIGS = [
    ("four_pair", 1, 0), ("four_pair", 2, 0), ("four_pair", 3, 0),
    ("pair_removal", 1, 0), ("pair_removal", 2, 0),
    ("multiscale", 1, 1), ("multiscale", 2, 1), ("multiscale", 1, 3),
]
NOISE = (0.0, 0.0005, 0.001, 0.002)


def accuracy_table(frames: int = 4, noise_levels=NOISE, configs=CONFIGS, mode: str = "rel",
                   tau: float = 4.0, H: int = 480, W: int = 640, seed0: int = 4000):
    """Rows of {noise_k, method, alpha, scales, coverage, mse_theta, mse_phi,
    mse_theta_fit, mse_phi_fit}: MSEs averaged over `frames` scenes (by
    pixel), coverage = fraction of pixels VALID."""
    import numpy as np
    import torch
    import paper_2209_08241_amd as bn
    from synth import scenes

    f = 525.0 * W / 640.0
    acc = {}
    for k in noise_levels:
        for i in range(frames):
            s = scenes.make_scene(H, W, fx=f, seed=seed0 + i, noise_k=k,
                                  n_planes=2, n_spheres=3, n_boxes=1)
            d = torch.from_numpy(s.depth).cuda()
            gt = torch.from_numpy(s.normals.astype(np.float32)).cuda()
            fit_n, fit_m = bn.plane_fit_normals(d, s.fx, s.fy, s.cx, s.cy, 2)
            for (method, alpha, K) in configs:
                n, m, _ = bn.estimate_normals(d, s.fx, s.fy, s.cx, s.cy, alpha, mode, tau,
                                              method=method, scales=K, want_stats=False)
                t, p, c = bn.angle_mse(n, m, gt, None)
                tf, pf, cf = bn.angle_mse(n, m, fit_n, fit_m)
                a = acc.setdefault((k, method, alpha, K), [0.0, 0.0, 0, 0.0, 0.0, 0, 0])
                a[0] += t * c
                a[1] += p * c
                a[2] += c
                a[3] += tf * cf
                a[4] += pf * cf
                a[5] += cf
                a[6] += H * W
    rows = []
    for (k, method, alpha, K), a in acc.items():
        rows.append({"noise_k": k, "method": method, "alpha": alpha, "scales": K,
                     "coverage": a[2] / a[6],
                     "mse_theta": a[0] / max(a[2], 1), "mse_phi": a[1] / max(a[2], 1),
                     "mse_theta_fit": a[3] / max(a[5], 1), "mse_phi_fit": a[4] / max(a[5], 1)})
    return rows


def markdown(rows) -> str:
    out = ["| noise k | method | alpha | K | valid | MSE theta (analytic) | MSE phi (analytic) "
           "| MSE theta (5x5 fit) | MSE phi (5x5 fit) |", "|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| {r['noise_k']:g} | {r['method']} | {r['alpha']} | {r['scales'] or '-'} | "
                   f"{100 * r['coverage']:.1f}% | {r['mse_theta']:.3g} | {r['mse_phi']:.3g} | "
                   f"{r['mse_theta_fit']:.3g} | {r['mse_phi_fit']:.3g} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=4)
    ap.add_argument("--json", default="")
    a = ap.parse_args()
    rows = accuracy_table(a.frames)
    print(markdown(rows), flush=True)
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(rows, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
