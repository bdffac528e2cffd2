"""Plain oracle of TSDF fusion on a voxel-block map (GSFusion Sec. III-B-1, Eq. 6-9) and of
the voxel-weight check that gates new Gaussians (Sec. III-B-2).

TEST INFRASTRUCTURE ONLY: the product library never imports or calls anything here.
It shares no code with the HIP path.

The map is a set of voxel blocks of 8 x 8 x 8 voxels of side ``voxel``, each voxel holding
a truncated signed distance and a weight (both 0 until first updated).  One depth frame is
fused in the paper's order:

1. allocation: the viewing ray of every pixel with a depth d > 0 is marched through the
   band [d - eps, d + eps]; every block that a sample falls in is allocated (if new) and
   marked as met by this frame;
2. integration, for every voxel of the blocks met by the frame: its centre p_v is taken to
   the camera, projected, and, where the nearest pixel holds a depth D > 0,
     sdf = D - z_v                                  (Eq. 6)
     tsdf = min(1, sdf / eps) if sdf > 0, else max(-1, sdf / eps)          (Eq. 7)
     w_k = min(w_max, w_(k-1) + 1)                  (Eq. 8)
     tsdf_k = (tsdf_(k-1) w_(k-1) + tsdf w_k) / (w_(k-1) + w_k)      (Eq. 9 as printed)
   The prose calls the update a simple running weighted average, which Eq. 9 as printed
   is not (it weighs the new measurement by w_k); ``weighting="unit"`` gives the running
   average with unit measurement weight, (tsdf_(k-1) w_(k-1) + tsdf) / (w_(k-1) + 1),
   and "eq9" (default) the printed form.

Readings where the paper is silent (each a setting or stated here):

* the march samples camera depths z_i = (d - eps) + i * step, i = 0 .. n - 1 with
  n = floor(2 eps / step) + 1, and skips z_i <= 0; a sample's world point is
  R^T ((u - cx) / fx * z_i - t_x, (v - cy) / fy * z_i - t_y, z_i - t_z) for pixel (u, v);
  its block is floor(p / (8 voxel)) per axis;
* voxel (gx, gy, gz) (global integer index) has centre ((g + 0.5) voxel); the nearest
  pixel of a camera point (x, y, z > 0) is (floor(fx (x/z) + cx + 0.5), floor(fy (y/z) +
  cy + 0.5)); voxels that project outside the image or onto a pixel without depth keep
  their values; every other voxel of a met block is updated, also behind the surface
  (Eq. 7 clamps those to -1);
* the block allocation and the projection of a voxel are integer decisions; both are
  taken in binary32, one correctly rounded operation at a time in the order written
  below (sums left to right), so any implementation that follows the same sequence
  allocates the same blocks and reads the same pixels; the values (Eq. 6-9) are FP64;
* defaults: voxel 0.01 m (Sec. IV-A-4), eps = 8 voxels, w_max = 100, step = one voxel;
* the seeding check: the voxel nearest to a point p (the voxel floor(p / voxel) that
  contains it) is looked up after the frame's fusion; a new Gaussian is placed only where
  that voxel's weight is exactly 1 (first observed by this frame); an unallocated voxel
  has weight 0 and gets none.
"""
from __future__ import annotations

import numpy as np

F = np.float32
BLOCK = 8


def _f(x):
    return F(x)


def camera_arrays(cam):
    R = np.asarray(cam.R, np.float32).reshape(3, 3)
    t = np.asarray(cam.t, np.float32).reshape(3)
    return R, t, F(cam.fx), F(cam.fy), F(cam.cx), F(cam.cy)


def band_samples(eps, step):
    """n = floor(2 eps / step) + 1, with the quotient in binary32."""
    return int(np.floor(F(F(2) * F(eps)) / F(step))) + 1


def sample_blocks(depth, cam, voxel, eps, step):
    """Block coordinates [k, 3] (int64) met by the band samples of every valid pixel."""
    H, W = depth.shape
    R, t, fx, fy, cx, cy = camera_arrays(cam)
    eps, step, voxel = F(eps), F(step), F(voxel)
    bsize = F(F(BLOCK) * voxel)
    v, u = np.nonzero(depth > 0)
    d = depth[v, u].astype(np.float32)
    xn = ((u.astype(np.float32) - cx) / fx).astype(np.float32)
    yn = ((v.astype(np.float32) - cy) / fy).astype(np.float32)
    a = (d - eps).astype(np.float32)
    out = []
    for i in range(band_samples(eps, step)):
        z = (a + F(F(i) * step)).astype(np.float32)
        ok = z > 0
        zz, x, y = z[ok], xn[ok], yn[ok]
        xc = (x * zz).astype(np.float32)
        yc = (y * zz).astype(np.float32)
        dx, dy, dz = (xc - t[0]).astype(F), (yc - t[1]).astype(F), (zz - t[2]).astype(F)
        blk = []
        for j in range(3):   # row j of R^T is column j of R
            pw = (((R[0, j] * dx).astype(F) + (R[1, j] * dy).astype(F)).astype(F) + (R[2, j] * dz).astype(F)).astype(F)
            blk.append(np.floor((pw / bsize).astype(F)).astype(np.int64))
        out.append(np.stack(blk, 1))
    return np.concatenate(out) if out else np.zeros((0, 3), np.int64)


def project_voxels(gidx, cam, voxel, W, H):
    """For global voxel indices [n, 3]: (valid mask, pixel x, pixel y, camera z as binary32)."""
    R, t, fx, fy, cx, cy = camera_arrays(cam)
    voxel = F(voxel)
    p = ((gidx.astype(np.float32) + F(0.5)).astype(F) * voxel).astype(F)
    c = []
    for r in range(3):
        c.append(((((R[r, 0] * p[:, 0]).astype(F) + (R[r, 1] * p[:, 1]).astype(F)).astype(F)
                   + (R[r, 2] * p[:, 2]).astype(F)).astype(F) + t[r]).astype(F))
    x, y, z = c
    ok = z > 0
    with np.errstate(divide="ignore", invalid="ignore"):
        u = ((fx * (x / z).astype(F)).astype(F) + cx).astype(F)
        v = ((fy * (y / z).astype(F)).astype(F) + cy).astype(F)
        uh = (u + F(0.5)).astype(F)
        vh = (v + F(0.5)).astype(F)
    ok &= (uh >= 0) & (uh < F(W)) & (vh >= 0) & (vh < F(H))
    px = np.where(ok, np.floor(np.where(ok, uh, 0)), 0).astype(np.int64)
    py = np.where(ok, np.floor(np.where(ok, vh, 0)), 0).astype(np.int64)
    return ok, px, py, z


class TsdfMap:
    """Blocks as a dict: block coordinate (bx, by, bz) -> (tsdf [8,8,8] z-y-x order,
    weight [8,8,8]), FP64."""

    def __init__(self, voxel=0.01, eps=None, w_max=100.0, step=None, weighting="eq9"):
        self.voxel = float(voxel)
        self.eps = float(8 * voxel if eps is None else eps)
        self.w_max = float(w_max)
        self.step = float(voxel if step is None else step)
        assert weighting in ("eq9", "unit")
        self.weighting = weighting
        self.blocks: dict = {}

    def integrate(self, depth, cam):
        """Fuse one depth frame [H, W] (binary32 metres, <= 0 = no depth).  Returns the
        set of blocks met."""
        depth = np.asarray(depth, np.float32)
        H, W = depth.shape
        met = {tuple(b) for b in np.unique(sample_blocks(depth, cam, self.voxel, self.eps, self.step), axis=0)}
        for b in met:
            if b not in self.blocks:
                self.blocks[b] = (np.zeros((BLOCK,) * 3), np.zeros((BLOCK,) * 3))
        if not met:
            return met
        order = sorted(met)
        k, j, i = np.meshgrid(np.arange(BLOCK), np.arange(BLOCK), np.arange(BLOCK), indexing="ij")
        local = np.stack([i.ravel(), j.ravel(), k.ravel()], 1)           # x fastest
        gidx = (np.asarray(order, np.int64)[:, None, :] * BLOCK + local[None]).reshape(-1, 3)
        ok, px, py, z = project_voxels(gidx, cam, self.voxel, W, H)
        D = np.where(ok, depth[py, px], 0).astype(np.float64)
        ok &= D > 0
        sdf = D - z.astype(np.float64)                                     # Eq. 6
        tsdf = np.where(sdf > 0, np.minimum(1.0, sdf / self.eps), np.maximum(-1.0, sdf / self.eps))   # Eq. 7
        T = np.stack([self.blocks[b][0].ravel() for b in order]).reshape(-1)
        Wt = np.stack([self.blocks[b][1].ravel() for b in order]).reshape(-1)
        w_new = np.minimum(self.w_max, Wt + 1.0)                           # Eq. 8
        if self.weighting == "eq9":
            t_new = (T * Wt + tsdf * w_new) / (Wt + w_new)                 # Eq. 9
        else:
            t_new = (T * Wt + tsdf) / (Wt + 1.0)
        T = np.where(ok, t_new, T)
        Wt = np.where(ok, w_new, Wt)
        for n, b in enumerate(order):
            s = slice(n * BLOCK ** 3, (n + 1) * BLOCK ** 3)
            self.blocks[b] = (T[s].reshape((BLOCK,) * 3), Wt[s].reshape((BLOCK,) * 3))
        return met

    def voxel_weight(self, points):
        """Weight of the voxel containing each point [n, 3] (binary32 coordinates divided
        by the binary32 voxel side, then floored); 0 where unallocated."""
        g = np.floor((np.asarray(points, np.float32) / F(self.voxel)).astype(F)).astype(np.int64)
        out = np.zeros(len(g))
        for n, (x, y, z) in enumerate(g):
            b = (x // BLOCK, y // BLOCK, z // BLOCK)
            if b in self.blocks:
                out[n] = self.blocks[b][1][z % BLOCK, y % BLOCK, x % BLOCK]
        return out
