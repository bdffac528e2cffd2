"""Plain FP64 oracle of quadtree seeding and Gaussian initialisation (GSFusion Sec. III-B-2).

TEST INFRASTRUCTURE ONLY: the product library never imports or calls anything here.
It shares no code with the HIP path.

What it computes, in the paper's order:

* a quadtree over each input image (Sec. III-B-2, Fig. 3): every root cell of
  ``root`` pixels is split into four quadrants while its measure exceeds a threshold
  (0.1 in Sec. IV-A-4) and its side exceeds ``min_side``; leaves are kept;
* the back-projection of each leaf's centre pixel with the depth map,
  p_q = T_WC pi^-1(u_q, D[u_q])  (Eq. 10);
* the initial Gaussian: R = I, S = diag(d, d, d) with d the back-projected length from
  the quadrant centre to its corner, opacity 0.5, and the DC spherical-harmonic
  coefficients set from the pixel colour (the paragraph after Eq. 10).

Readings where the paper is silent (each is an argument):

* measure ``"contrast"``: the range (max - min) of the per-pixel mean of the three
  colour channels in the cell; a leaf has contrast lower than the threshold, so a cell
  splits when its contrast is >= the threshold;
* measure ``"depth_variance"``: the population variance (m^2) of the cell's valid depths
  (> 0); a cell splits when it is > the threshold (the rule used to seed the synthetic
  workloads); cells without a valid depth are dropped;
* roots are ``root``-pixel squares aligned at (0, 0) and clipped at the image border;
  children are the four quadrants of the nominal square (top-left, top-right,
  bottom-left, bottom-right), dropped when they start outside the image;
* the centre pixel is (x0 + w // 2, y0 + h // 2), pixels sampled at integer
  coordinates; a leaf whose centre depth is not valid yields no Gaussian;
* d is the distance from the back-projected centre to the back-projected top-left
  pixel (x0, y0) of the leaf at the centre's depth;
* colour = 0.5 + sh_0 * Y_00 (the rasterizer's SH convention), so sh_0 = (c - 0.5) / Y_00
  with Y_00 = 1 / (2 sqrt(pi)); the other coefficients are zero.

The check against duplicating primitives (the paragraph after Eq. 10): given a TSDF map
that has fused the frame (oracle/tsdf.py), a Gaussian is kept only where the voxel holding
its mean (rounded to binary32) has weight exactly 1, i.e. was observed for the first time;
without a map every leaf with a valid centre depth gives one.
"""
from __future__ import annotations

import math

import numpy as np

Y00 = 0.5 / math.sqrt(math.pi)


def cell_measure(rgb, depth, x0, y0, x1, y1, measure):
    """(number of samples, measure) of the pixels [y0, y1) x [x0, x1)."""
    if measure == "contrast":
        g = rgb[:, y0:y1, x0:x1].astype(np.float64).mean(axis=0)
        return g.size, float(g.max() - g.min())
    d = depth[y0:y1, x0:x1].astype(np.float64)
    d = d[d > 0]
    if d.size == 0:
        return 0, 0.0
    return d.size, float(((d - d.mean()) ** 2).mean())


def splits(n, m, side, threshold, min_side, measure):
    if n == 0 or side <= min_side:
        return False
    return m >= threshold if measure == "contrast" else m > threshold


def quadtree(rgb, depth, measure="contrast", threshold=0.1, root=64, min_side=4):
    """Leaves (x0, y0, w, h) in depth-first order (roots in raster order, quadrants
    top-left, top-right, bottom-left, bottom-right), and every visited cell as
    (x0, y0, side, n, measure, split)."""
    H, W = depth.shape
    leaves, cells = [], []

    def visit(x0, y0, side):
        if x0 >= W or y0 >= H:
            return
        x1, y1 = min(x0 + side, W), min(y0 + side, H)
        n, m = cell_measure(rgb, depth, x0, y0, x1, y1, measure)
        s = splits(n, m, side, threshold, min_side, measure)
        cells.append((x0, y0, side, n, m, s))
        if s:
            h = side // 2
            for dy in (0, h):
                for dx in (0, h):
                    visit(x0 + dx, y0 + dy, h)
        elif n > 0:
            leaves.append((x0, y0, x1 - x0, y1 - y0))

    for y0 in range(0, H, root):
        for x0 in range(0, W, root):
            visit(x0, y0, root)
    return np.array(leaves, np.int64).reshape(-1, 4), cells


def initial_gaussians(leaves, rgb, depth, cam, opacity=0.5, sh_degree=0, tsdf_map=None):
    """Gaussians of the leaves whose centre depth is valid (and, with a TSDF map, whose
    mean's voxel has weight 1): dict of means [n,3], scales [n,3], quats [n,4],
    opacities [n], sh [n,K,3], and the kept leaves."""
    R = np.asarray(cam.R, np.float64).reshape(3, 3)   # world -> camera
    t = np.asarray(cam.t, np.float64)
    K = (sh_degree + 1) ** 2
    means, scales, sh, kept = [], [], [], []
    for x0, y0, w, h in leaves:
        xc, yc = x0 + w // 2, y0 + h // 2
        d = float(depth[yc, xc])
        if not d > 0:
            continue
        pc = np.array([(xc - cam.cx) / cam.fx * d, (yc - cam.cy) / cam.fy * d, d])   # pi^-1(u_q, D[u_q])
        corner = np.array([(x0 - cam.cx) / cam.fx * d, (y0 - cam.cy) / cam.fy * d, d])
        mean = R.T @ (pc - t)                                                          # T_WC
        if tsdf_map is not None and tsdf_map.voxel_weight(mean.astype(np.float32)[None])[0] != 1.0:
            continue                                                                   # seen before
        means.append(mean)
        scales.append(np.linalg.norm(pc - corner))
        c = np.zeros((K, 3))
        c[0] = (rgb[:, yc, xc].astype(np.float64) - 0.5) / Y00
        sh.append(c)
        kept.append((x0, y0, w, h))
    n = len(means)
    return dict(means=np.array(means).reshape(n, 3), scales=np.repeat(np.array(scales).reshape(n, 1), 3, 1),
                quats=np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)), opacities=np.full(n, float(opacity)),
                sh=np.array(sh).reshape(n, K, 3), leaves=np.array(kept, np.int64).reshape(n, 4))
