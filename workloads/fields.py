"""Seeded synthetic fields.  Arrays are (nz, ny, nx) with x fastest, or
(ny, nx) for 2D.  The ``*_into`` variants fill a caller-owned array (for
example a pinned host tensor viewed through numpy) block by block along the
slowest axis, so a field of tens of GiB is never held twice."""
import numpy as np


def uniform(shape, seed, dtype=np.float64):
    """U[0, 1) field from PCG64(seed)."""
    dt = np.dtype(dtype)
    if dt not in (np.float32, np.float64):
        raise TypeError("uniform draws float32 or float64")
    return np.random.default_rng(seed).random(shape, dtype=dt.type)


def uniform_into(out, seed, block=16):
    """Fill ``out`` (float32 or float64, slowest axis first) with U[0, 1) drawn
    block by block along axis 0 from one PCG64(seed) stream.  For a given
    dtype, shape and ``block`` the values are fixed by the seed."""
    rng = np.random.default_rng(seed)
    dt = out.dtype
    if dt not in (np.float32, np.float64):
        raise TypeError("uniform_into needs a float32 or float64 array")
    for z0 in range(0, out.shape[0], block):
        z1 = min(out.shape[0], z0 + block)
        rng.random(out[z0:z1].shape, dtype=dt.type, out=out[z0:z1])
    return out


def _mode_params(seed, n_modes=8, kmax=16):
    rng = np.random.default_rng(seed)
    kx = rng.integers(1, kmax + 1, n_modes)
    ky = rng.integers(1, kmax + 1, n_modes)
    m = rng.integers(1, kmax + 1, n_modes)
    a = rng.uniform(0.5, 1.0, n_modes) / n_modes
    phi = rng.uniform(0.0, 2 * np.pi, n_modes)
    return kx, ky, m, a, phi


def fourier_modes_into(out, seed, noise_std=0.01, block=8):
    """sum_j a_j cos(2 pi (kx_j x/nx + ky_j y/ny) + phi_j) sin(pi m_j (z+1)/(nz+1))
    plus N(0, noise_std^2) noise.  kx, ky, m are integers in [1, 16],
    a_j ~ U[0.5, 1)/8, phi_j ~ U[0, 2 pi).  Mode parameters come from
    PCG64(seed), the noise from PCG64(seed + 1), block by block along z."""
    nz, ny, nx = out.shape
    kx, ky, m, a, phi = _mode_params(seed)
    noise = np.random.default_rng(seed + 1)
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    planes = [np.cos(2 * np.pi * (kx[j] * x / nx + ky[j] * y / ny) + phi[j]) * a[j]
              for j in range(len(a))]
    for z0 in range(0, nz, block):
        z1 = min(nz, z0 + block)
        zz = np.arange(z0, z1)
        blk = np.zeros((z1 - z0, ny, nx))
        for j in range(len(a)):
            s = np.sin(np.pi * m[j] * (zz + 1) / (nz + 1))
            blk += s[:, None, None] * planes[j][None]
        blk += noise.normal(0.0, noise_std, blk.shape)
        out[z0:z1] = blk
    return out


def fourier_modes(shape, seed, noise_std=0.01):
    out = np.empty(shape)
    return fourier_modes_into(out, seed, noise_std)


def gaussian_bump_into(out, seed, noise=1e-3, block=32):
    """exp(-|x - c|^2 / (2 sigma^2)) with c the grid centre ((n-1)/2 per axis)
    and sigma = n/8 per axis, plus U[-noise, noise) from PCG64(seed), block by
    block along the slowest axis."""
    rng = np.random.default_rng(seed)
    shp = out.shape
    coords = [np.arange(n) for n in shp]
    gs = [np.exp(-((c - (n - 1) / 2.0) ** 2) / (2 * (n / 8.0) ** 2)) for c, n in zip(coords, shp)]
    for z0 in range(0, shp[0], block):
        z1 = min(shp[0], z0 + block)
        g = gs[0][z0:z1]
        for ax in range(1, len(shp)):
            g = np.multiply.outer(g, gs[ax])
        g = g + rng.uniform(-noise, noise, g.shape)
        out[z0:z1] = g
    return out


def gaussian_bump(shape, seed, noise=1e-3):
    out = np.empty(shape)
    return gaussian_bump_into(out, seed, noise)
