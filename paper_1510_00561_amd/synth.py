"""Seeded synthetic inputs shaped like the paper's workloads.

The paper evaluates on QCIF conferencing/surveillance clips and times a VGA
frame (section 4); neither is available here. These generators stand in for
them with the same kind of content: a static textured background, moving
objects with sharp edges, and sensor noise, on 8-bit RGB or luma frames.

This module holds only input synthesis (NumPy, none of the method's
arithmetic): frames come out as 8-bit RGB; the conversion to the Y, Co, Cg
planes the contourlet transform runs on is the library's (or, in tests,
the oracle's).
Random draws use numpy's default_rng with seed 1510_00561 + workload number.
"""
import numpy as np

SEED_BASE = 151000561


def rng_for(workload):
    return np.random.default_rng(SEED_BASE + workload)


def luma_edges(height=256, width=256, seed=None, n_edges=8, noise=5.0):
    """Smooth gradient (32..224) + oriented half-plane edges + Gaussian noise, uint8.

    Each edge is a step of height amp centred on its line (+-amp/2 on the
    two sides), so that the frame stays mostly inside 0..255.
    """
    rng = rng_for(1) if seed is None else np.random.default_rng(seed)
    r, c = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    img = 32.0 + 192.0 * c / max(width - 1, 1)
    for _ in range(n_edges):
        th = rng.uniform(0, np.pi)
        r0, c0 = rng.uniform(0, height), rng.uniform(0, width)
        amp = rng.uniform(20, 60) * rng.choice([-1.0, 1.0])
        dist = (r - r0) * np.cos(th) + (c - c0) * np.sin(th)
        img += amp * (np.clip(dist + 0.5, 0.0, 1.0) - 0.5)   # 1-pixel soft step, +-amp/2
    img += rng.normal(0, noise, img.shape)
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


class ClipGenerator:
    """Moving ellipses/rectangles over a textured background, RGB uint8.

    Background: 3-4 colour gratings plus smooth value noise. Six objects with
    random colours move 2 pixels per frame in seeded directions. Additive
    Gaussian noise (sigma 3) per frame.
    """

    def __init__(self, height, width, seed, n_objects=6, speed=2.0, noise=3.0):
        self.h, self.w = height, width
        rng = np.random.default_rng(seed)
        self.rng = rng
        r, c = np.meshgrid(np.arange(height, dtype=np.float32),
                           np.arange(width, dtype=np.float32), indexing="ij")
        bg = np.full((height, width, 3), 110.0, np.float32)
        for _ in range(rng.integers(3, 5)):
            th = rng.uniform(0, np.pi)
            freq = rng.uniform(0.02, 0.25)
            phase = rng.uniform(0, 2 * np.pi)
            amp = rng.uniform(10, 35, size=3).astype(np.float32)
            wave = np.sin(freq * (r * np.cos(th) + c * np.sin(th)) + phase)
            bg += wave[..., None] * amp
        # smooth value noise: bilinear upsampling of a coarse random grid
        gh, gw = height // 32 + 2, width // 32 + 2
        grid = rng.uniform(-30, 30, size=(gh, gw, 3)).astype(np.float32)
        gy, gx = r / 32.0, c / 32.0
        y0, x0 = np.floor(gy).astype(int), np.floor(gx).astype(int)
        fy, fx = (gy - y0)[..., None], (gx - x0)[..., None]
        bg += ((1 - fy) * (1 - fx) * grid[y0, x0] + (1 - fy) * fx * grid[y0, x0 + 1]
               + fy * (1 - fx) * grid[y0 + 1, x0] + fy * fx * grid[y0 + 1, x0 + 1])
        self.bg = bg
        self.objs = []
        for _ in range(n_objects):
            self.objs.append(dict(
                kind=rng.choice(["ellipse", "rect"]),
                cy=rng.uniform(0, height), cx=rng.uniform(0, width),
                ry=rng.uniform(0.05, 0.2) * height, rx=rng.uniform(0.05, 0.2) * width,
                color=rng.uniform(0, 255, size=3).astype(np.float32),
                dy=speed * np.sin(ang := rng.uniform(0, 2 * np.pi)), dx=speed * np.cos(ang)))
        self.noise = noise
        self._r, self._c = r, c

    def frame(self, t):
        img = self.bg.copy()
        r, c = self._r, self._c
        for o in self.objs:
            cy = (o["cy"] + o["dy"] * t) % self.h
            cx = (o["cx"] + o["dx"] * t) % self.w
            if o["kind"] == "ellipse":
                m = ((r - cy) / o["ry"]) ** 2 + ((c - cx) / o["rx"]) ** 2 <= 1.0
            else:
                m = (np.abs(r - cy) <= o["ry"]) & (np.abs(c - cx) <= o["rx"])
            img[m] = o["color"]
        img += self.rng.normal(0, self.noise, img.shape).astype(np.float32)
        return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def clip_rgb(n_frames, height, width, workload):
    """[n_frames, height, width, 3] uint8 RGB frames of a synthetic clip."""
    gen = ClipGenerator(height, width, SEED_BASE + workload)
    return np.stack([gen.frame(t) for t in range(n_frames)])


def subband_steps(nsub, n_channels=3, workload=3, low=4, high=64):
    """Per-channel step table drawn uniformly from low..high (inclusive)."""
    return rng_for(workload).integers(low, high + 1, size=(n_channels, nsub)).astype(np.float32)


def mixed_streams(n_streams=64, workload=4):
    """Stream list of the mixed-resolution batch: (height, width, levels, dirs).

    Resolution uniform over 320x240, 640x480, 1280x720; LP depth uniform
    over 2..4; finest direction count 8 or 16, halving per coarser level
    with a floor of 8.
    """
    rng = rng_for(workload)
    sizes = [(240, 320), (480, 640), (720, 1280)]
    out = []
    for _ in range(n_streams):
        h, w = sizes[rng.integers(0, 3)]
        J = int(rng.integers(2, 5))
        d0 = int(rng.choice([8, 16]))
        dirs = [max(8, d0 >> j) for j in range(J)]
        out.append((h, w, J, dirs))
    return out
