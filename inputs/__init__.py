"""Seeded synthetic inputs shaped like the paper's 2-D/3-D photoacoustic grids.

This module holds no arithmetic of the method (no filters, transforms or
weights): it only draws test and benchmark inputs.  Both the HIP path and the
oracle receive the same arrays from here.

The paper's own phantom (Sec. 5: circular and rectangular inclusions in a
square domain) and its simulated data are not available, so random-disc and
random-ellipsoid phantoms stand in for them, at the paper's grid sizes
(512^2 reconstruction grid, 128^2 small grid) and its noise level (Gaussian
with a standard deviation of 5 % of the maximum amplitude).

Every generator takes an explicit numpy Generator; `rng(config, instance,
stream)` derives one from a SeedSequence so that instances can be generated
independently and in any order.  Values are drawn in float64; callers that feed
a float32 kernel cast once and give the oracle the cast values.
"""

import math

import numpy as np

# Shape pool of the ragged batch: every 2-D pair of {128..2048} plus two cubes.
RAGGED_2D_SIDES = (128, 256, 512, 1024, 2048)
RAGGED_3D_SIDES = (64, 128)
RAGGED_ORDERS = (2, 4, 8)
RAGGED_S = (0.5, 1.0, 2.0)


def rng(config, instance=0, stream=0):
    return np.random.default_rng(np.random.SeedSequence([int(config), int(instance), int(stream)]))


def disc_phantom(shape, n_discs, gen, radius=(5.0, 20.0), amplitude=(0.5, 1.0), noise_sigma=0.0):
    """Sum of `n_discs` filled discs on an (n0, n1) grid plus white noise of std `noise_sigma`.

    Radius ~ U[radius], centre ~ U[r, n - r] per axis, amplitude ~ U[amplitude];
    pixel centres sit at integer coordinates and a pixel belongs to a disc when
    (i - ci)^2 + (j - cj)^2 <= r^2.  Overlapping discs add.
    """
    n0, n1 = shape
    img = np.zeros(shape, dtype=np.float64)
    for _ in range(n_discs):
        r = gen.uniform(*radius)
        ci = gen.uniform(r, n0 - r)
        cj = gen.uniform(r, n1 - r)
        amp = gen.uniform(*amplitude)
        i0, i1 = max(0, int(math.floor(ci - r))), min(n0, int(math.ceil(ci + r)) + 1)
        j0, j1 = max(0, int(math.floor(cj - r))), min(n1, int(math.ceil(cj + r)) + 1)
        ii = np.arange(i0, i1)[:, None]
        jj = np.arange(j0, j1)[None, :]
        img[i0:i1, j0:j1] += amp * (((ii - ci) ** 2 + (jj - cj) ** 2) <= r * r)
    if noise_sigma:
        img += gen.normal(0.0, noise_sigma, size=shape)
    return img


def ellipsoid_phantom(shape, n_ellipsoids, gen, semi_axes=(4.0, 32.0), centre=None, amplitude=(0.0, 1.0)):
    """Sum of randomly rotated filled ellipsoids on an (n0, n1, n2) grid.

    Semi-axes ~ U[semi_axes]; rotation = Q factor of a 3x3 standard normal
    matrix with the signs fixed by diag(R) > 0; centre ~ U[centre] per axis
    (default: the middle 3/4 of each side); amplitude ~ U[amplitude].
    """
    n = np.array(shape)
    lo_c, hi_c = centre if centre is not None else (n.min() / 8.0, n.min() * 7.0 / 8.0)
    vol = np.zeros(shape, dtype=np.float64)
    for _ in range(n_ellipsoids):
        ax = gen.uniform(*semi_axes, size=3)
        q, r = np.linalg.qr(gen.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))[None, :]
        c = gen.uniform(lo_c, hi_c, size=3)
        amp = gen.uniform(*amplitude)
        ext = ax.max()
        lo = np.maximum(0, np.floor(c - ext)).astype(int)
        hi = np.minimum(n, np.ceil(c + ext) + 1).astype(int)
        g = np.stack(np.meshgrid(*[np.arange(lo[k], hi[k]) for k in range(3)], indexing="ij"), axis=-1)
        local = (g - c) @ q  # coordinates in the ellipsoid's own frame
        inside = np.sum((local / ax) ** 2, axis=-1) <= 1.0
        vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += amp * inside
    return vol


def white_noise(shape, gen, sigma=1.0):
    return gen.normal(0.0, sigma, size=shape)


def bernoulli_mask(shape, p, gen):
    """1 = observed pixel with probability p."""
    return (gen.random(shape) < p).astype(np.float64)


def ragged_descriptors(count, seed):
    """Instance list of the ragged batch: (shape, order, levels, s) per instance.

    Shape uniform over the 25 ordered 2-D pairs of RAGGED_2D_SIDES and the two
    cubes of RAGGED_3D_SIDES (27 choices); order uniform over RAGGED_ORDERS;
    s uniform over RAGGED_S; levels = log2(min side) - 3 (coarsest side 8).
    """
    gen = rng(4, 0, seed)
    pool = [(a, b) for a in RAGGED_2D_SIDES for b in RAGGED_2D_SIDES] + [(c, c, c) for c in RAGGED_3D_SIDES]
    out = []
    for _ in range(count):
        shape = pool[int(gen.integers(len(pool)))]
        order = RAGGED_ORDERS[int(gen.integers(len(RAGGED_ORDERS)))]
        s = RAGGED_S[int(gen.integers(len(RAGGED_S)))]
        levels = int(math.log2(min(shape))) - 3
        out.append((tuple(shape), order, levels, s))
    return out


# ---------------------------------------------------------------------------
# The five workloads.  Each returns float32 arrays (the device inputs) plus the
# scalar parameters; the oracle is given the same float32 values.

def small_image(seed=0):
    """128x128 image: 5 discs, amplitudes U[0.5,1], N(0, 0.01) noise; db4, 5 levels, s = 1."""
    img = disc_phantom((128, 128), 5, rng(1, 0, seed), amplitude=(0.5, 1.0), noise_sigma=0.01)
    return dict(x=img.astype(np.float32), order=4, levels=5, s=1.0)


def image_batch(count=64, side=1024, seed=0):
    """`count` images of side^2: 20 discs each plus N(0, 0.05) noise; db8, 7 levels, s = 1.5."""
    x = np.empty((count, side, side), dtype=np.float32)
    for b in range(count):
        x[b] = disc_phantom((side, side), 20, rng(2, b, seed), amplitude=(0.5, 1.0), noise_sigma=0.05)
    return dict(x=x, order=8, levels=7, s=1.5)


def volume_autograd(side=256, seed=0, n_ellipsoids=50):
    """side^3 volume of 50 ellipsoids (amplitude U[0,1]) and an N(0,1) target; db4, 5 levels, s = 2."""
    vol = ellipsoid_phantom((side,) * 3, n_ellipsoids, rng(3, 0, seed))
    y = white_noise((side,) * 3, rng(3, 1, seed))
    return dict(x=vol.astype(np.float32), y=y.astype(np.float32), order=4, levels=5, s=2.0)


def ragged_batch(count=200, seed=0):
    """Ragged instances with N(0,1) inputs (see `ragged_descriptors`)."""
    descs = ragged_descriptors(count, seed)
    xs = [white_noise(d[0], rng(4, i + 1, seed)).astype(np.float32) for i, d in enumerate(descs)]
    return dict(descs=descs, xs=xs)


def map_gradient_batch(count=256, side=512, seed=0):
    """`count` images of side^2: xi ~ N(0,1), mask ~ Bernoulli(0.3), y = mask * (20-disc phantom).

    Sampler parameters: db6, 6 levels, s = 1.5.
    """
    xi = np.empty((count, side, side), dtype=np.float32)
    mask = np.empty_like(xi)
    y = np.empty_like(xi)
    for b in range(count):
        xi[b] = white_noise((side, side), rng(5, b, seed))
        mask[b] = bernoulli_mask((side, side), 0.3, rng(5, b, seed + 1000003))
        y[b] = mask[b] * disc_phantom((side, side), 20, rng(5, b, seed + 2000003))
    return dict(xi=xi, mask=mask, y=y, order=6, levels=6, s=1.5)
