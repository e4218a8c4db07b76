"""Seeded synthetic images for the evaluation workloads.

Input generation only: nothing here evaluates a formula or any operator of
the logic.  Both the GPU path and the oracle receive these arrays unchanged.
All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).

Layout of every image: numpy array (C, H, W), float32, uint8 or uint16;
volumes (C, D, H, W).
"""
import hashlib

import numpy as np
from scipy import ndimage


def smoothed_noise(rng, h, w, sigma=4.0):
    """Uniform noise smoothed by a Gaussian (sigma px, reflect border,
    truncate 4.0) in float64, min-max scaled to [0, 1], cast to float32."""
    u = rng.random((h, w))
    s = ndimage.gaussian_filter(u, sigma=sigma, mode="reflect", truncate=4.0)
    lo, hi = s.min(), s.max()
    s = (s - lo) / (hi - lo) if hi > lo else np.zeros_like(s)
    return s.astype(np.float32)


def paint_ellipses(canvas, rng, n, axis_range, intensities):
    """Paint `n` filled ellipses in order (later ones on top).  Centre
    ~ U(image), semi-axes ~ U[axis_range], angle ~ U[0, pi).  `intensities`
    gives the value of ellipse i."""
    h, w = canvas.shape
    for i in range(n):
        cy, cx = rng.uniform(0, h), rng.uniform(0, w)
        a, b = rng.uniform(*axis_range), rng.uniform(*axis_range)
        th = rng.uniform(0, np.pi)
        r = max(a, b)
        y0, y1 = max(0, int(cy - r) - 1), min(h, int(cy + r) + 2)
        x0, x1 = max(0, int(cx - r) - 1), min(w, int(cx + r) + 2)
        if y0 >= y1 or x0 >= x1:
            continue
        yy, xx = np.mgrid[y0:y1, x0:x1]
        dy, dx = yy + 0.5 - cy, xx + 0.5 - cx
        c, s = np.cos(th), np.sin(th)
        u = (dx * c + dy * s) / a
        v = (-dx * s + dy * c) / b
        inside = u * u + v * v <= 1.0
        canvas[y0:y1, x0:x1][inside] = intensities[i]
    return canvas


def serpentine_maze(h, w):
    """One 8-connected, 1-px-wide corridor: even rows are all open; odd rows
    are walls with one opening, at x = w-1 when y % 4 == 1 and at x = 0 when
    y % 4 == 3."""
    m = np.zeros((h, w), np.float32)
    m[0::2, :] = 1.0
    for y in range(1, h, 2):
        m[y, w - 1 if y % 4 == 1 else 0] = 1.0
    return m


def plain_image(seed=1, size=256):
    """One-channel smoothed-noise image (sigma = 4 px)."""
    rng = np.random.default_rng(seed)
    return smoothed_noise(rng, size, size)[None]


def ellipse_maze_image(seed=2, size=4096, n_ellipses=200):
    """Three channels:
    0: smoothed noise scaled to [0, 0.5] with `n_ellipses` filled ellipses of
       distinct intensities 0.5 + (p_i + 1) / (2 * n_ellipses) painted on top
       (p a random permutation), semi-axes scaled with the image side;
    1: serpentine maze (0/1);
    2: seed marker, 1 only at pixel (0, 0)."""
    rng = np.random.default_rng(seed)
    ch0 = smoothed_noise(rng, size, size) * np.float32(0.5)
    perm = rng.permutation(n_ellipses)
    inten = (0.5 + (perm + 1) / (2.0 * n_ellipses)).astype(np.float32)
    scale = size / 4096.0
    paint_ellipses(ch0, rng, n_ellipses, (max(2.0, 20 * scale), max(3.0, 300 * scale)), inten)
    maze = serpentine_maze(size, size)
    seed_ch = np.zeros((size, size), np.float32)
    seed_ch[0, 0] = 1.0
    return np.stack([ch0, maze, seed_ch]).astype(np.float32)


def ellipse_intensities(n_ellipses=200):
    """The distinct ellipse intensities used by ellipse_maze_image, sorted."""
    return (0.5 + (np.arange(n_ellipses) + 1) / (2.0 * n_ellipses)).astype(np.float32)


def random_mask_image(seed=3, size=1024, density=0.5):
    """uint8 Bernoulli(density) image with values in {0, 1}, one channel."""
    rng = np.random.default_rng(seed)
    return (rng.random((size, size)) < density).astype(np.uint8)[None]


def phantom_image(rng, h, w, channels=4, sigma_noise=0.05):
    """Ellipse phantom per channel (10-40 ellipses, per-channel intensities in
    [0.2, 1]) with Rician-like noise sqrt((s + sigma n1)^2 + (sigma n2)^2)."""
    out = np.empty((channels, h, w), np.float32)
    side = min(h, w)
    for c in range(channels):
        n = int(rng.integers(10, 41))
        canvas = np.zeros((h, w), np.float32)
        inten = rng.uniform(0.2, 1.0, n).astype(np.float32)
        paint_ellipses(canvas, rng, n, (max(2.0, 0.03 * side), max(3.0, 0.3 * side)), inten)
        n1 = rng.standard_normal((h, w), dtype=np.float32)
        n2 = rng.standard_normal((h, w), dtype=np.float32)
        s = np.float32(sigma_noise)
        out[c] = np.sqrt((canvas + s * n1) ** 2 + (s * n2) ** 2)
    return out


def batch_sizes(seed=4, n=512, lo=128, hi=2048, square=False):
    """Image sides for the uneven batch: H, W ~ independent U{lo..hi}
    (square=True draws one side and uses it for both)."""
    rng = np.random.default_rng(seed)
    if square:
        s = rng.integers(lo, hi + 1, n)
        return [(int(v), int(v)) for v in s]
    hs = rng.integers(lo, hi + 1, n)
    ws = rng.integers(lo, hi + 1, n)
    return [(int(a), int(b)) for a, b in zip(hs, ws)]


def batch_image(seed, index, h, w, channels=4):
    """Image `index` of the uneven batch; seeded by (seed, index) so images can
    be produced one at a time."""
    rng = np.random.default_rng([seed, index])
    return phantom_image(rng, h, w, channels)


def digest(arr):
    """SHA-256 of an array's bytes (for input manifests)."""
    return hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()


def phantom_image_device(seed, index, h, w, channels=4, sigma_noise=0.05, device="cuda"):
    """Same recipe as `phantom_image`, generated directly in device memory
    with torch (for batches too large to synthesise on the host in time).
    Ellipse parameters come from ``default_rng([seed, index])``; the noise
    from a torch generator on the device seeded from that rng.  The values
    differ from `phantom_image`'s; copy an image to the host to hand the
    identical array to the oracle."""
    import torch
    rng = np.random.default_rng([seed, index])
    gen = torch.Generator(device=device)
    gen.manual_seed(int(rng.integers(0, 2**62)))
    out = torch.empty((channels, h, w), dtype=torch.float32, device=device)
    side = min(h, w)
    lo_ax, hi_ax = max(2.0, 0.03 * side), max(3.0, 0.3 * side)
    s = float(sigma_noise)
    for c in range(channels):
        n = int(rng.integers(10, 41))
        canvas = torch.zeros((h, w), dtype=torch.float32, device=device)
        inten = rng.uniform(0.2, 1.0, n).astype(np.float32)
        for i in range(n):
            cy, cx = rng.uniform(0, h), rng.uniform(0, w)
            a, b = rng.uniform(lo_ax, hi_ax), rng.uniform(lo_ax, hi_ax)
            th = rng.uniform(0, np.pi)
            r = max(a, b)
            y0, y1 = max(0, int(cy - r) - 1), min(h, int(cy + r) + 2)
            x0, x1 = max(0, int(cx - r) - 1), min(w, int(cx + r) + 2)
            if y0 >= y1 or x0 >= x1:
                continue
            dy = torch.arange(y0, y1, device=device, dtype=torch.float64)[:, None] + (0.5 - cy)
            dx = torch.arange(x0, x1, device=device, dtype=torch.float64)[None, :] + (0.5 - cx)
            cs, sn = np.cos(th), np.sin(th)
            u = (dx * cs + dy * sn) / a
            v = (-dx * sn + dy * cs) / b
            inside = u * u + v * v <= 1.0
            view = canvas[y0:y1, x0:x1]
            view.masked_fill_(inside, float(inten[i]))
        n1 = torch.randn((h, w), generator=gen, device=device, dtype=torch.float32)
        n2 = torch.randn((h, w), generator=gen, device=device, dtype=torch.float32)
        out[c] = torch.sqrt((canvas + s * n1) ** 2 + (s * n2) ** 2)
    return out


def paper_slice_u16(side=7680, seed=6, device="cuda"):
    """A uint16 stand-in for the paper's MRI slice (Sect. 4.2, Fig.
    specification: a 2-D uint16 image thresholded at 62258 and 56360): the
    device phantom (one channel) scaled by 65535, rounded and clamped to the
    uint16 range.  Returns the (1, side, side) numpy uint16 array."""
    import torch
    t = phantom_image_device(seed, 0, side, side, channels=1, device=device)
    t = torch.round(t * 65535.0).clamp_(0.0, 65535.0).to(torch.int32)
    out = t.cpu().numpy().astype(np.uint16)
    del t
    return out


def volume_phantom_device(seed, d, h, w, channels=2, sigma_noise=0.05, device="cuda"):
    """A volume (channels, d, h, w) float32 in device memory: per channel
    10-40 filled ellipsoids (semi-axes 3-30% of the smallest side, random
    orientation about the slice axis) with intensities in [0.2, 1], plus the
    Rician-like noise of `phantom_image`.  Parameters from
    ``default_rng([seed, 7])``, noise from a device generator seeded from it."""
    import torch
    rng = np.random.default_rng([seed, 7])
    gen = torch.Generator(device=device)
    gen.manual_seed(int(rng.integers(0, 2**62)))
    out = torch.empty((channels, d, h, w), dtype=torch.float32, device=device)
    side = min(d, h, w)
    lo_ax, hi_ax = max(1.5, 0.03 * side), max(2.0, 0.3 * side)
    zz = torch.arange(d, device=device, dtype=torch.float32)[:, None, None] + 0.5
    yy = torch.arange(h, device=device, dtype=torch.float32)[None, :, None] + 0.5
    xx = torch.arange(w, device=device, dtype=torch.float32)[None, None, :] + 0.5
    for c in range(channels):
        canvas = torch.zeros((d, h, w), dtype=torch.float32, device=device)
        n = int(rng.integers(10, 41))
        inten = rng.uniform(0.2, 1.0, n).astype(np.float32)
        for i in range(n):
            cz, cy, cx = rng.uniform(0, d), rng.uniform(0, h), rng.uniform(0, w)
            a, b, e = rng.uniform(lo_ax, hi_ax, 3)
            th = rng.uniform(0, np.pi)
            cs, sn = float(np.cos(th)), float(np.sin(th))
            dy, dx = yy - cy, xx - cx
            u = (dx * cs + dy * sn) / a
            v = (-dx * sn + dy * cs) / b
            t = (zz - cz) / e
            canvas.masked_fill_(u * u + v * v + t * t <= 1.0, float(inten[i]))
        n1 = torch.randn((d, h, w), generator=gen, device=device, dtype=torch.float32)
        n2 = torch.randn((d, h, w), generator=gen, device=device, dtype=torch.float32)
        out[c] = torch.sqrt((canvas + sigma_noise * n1) ** 2 + (sigma_noise * n2) ** 2)
    return out


def serve_image(index, side):
    """Image `index` of the serving mix: one float32 channel, the ellipse
    recipe (60 ellipses on smoothed noise) at `side` x `side`."""
    return np.ascontiguousarray(ellipse_maze_image(50 + index, side, n_ellipses=60)[:1])
