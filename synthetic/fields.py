"""Seeded synthetic scalar fields that stand in for the paper's datasets.

The paper evaluates on CT/MRI scans and simulation volumes (Sec. 4.6,
table ``tab:mc_benchmark_data``) that are not available here.  This module
draws fields with the same character -- a noisy sphere distance field,
Fourier-mode turbulence with a k^(-5/3) energy spectrum, Gaussian blobs and a
channel-flow-like sheet -- from ``numpy.random.default_rng(seed)``.

It holds none of the extraction method's arithmetic (no compression, no
culling, no marching cubes); it is the one module that both the CPU oracle and
the GPU path take their inputs from.

Layout of every returned array: ``[nz][ny][nx]`` (x fastest); sample
``(x, y, z)`` sits at position ``(x, y, z)`` in voxel units.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "sphere_sdf_noisy",
    "sphere_sdf",
    "plane_z",
    "tilted_plane",
    "turbulence",
    "turbulence_modes",
    "gaussian_blobs",
    "batched_dims",
    "percentile_iso",
    "turbulence_torch",
    "percentile_iso_torch",
    "channel_flow_slab",
    "CHANNEL_FLOW_DIMS",
    "random_block_stream",
]

# Large channel-flow-like volume: (nx, ny, nz) in voxels.
CHANNEL_FLOW_DIMS = (5120, 3840, 768)


def _grid(nx, ny, nz):
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    z = np.arange(nz, dtype=np.float64)
    return x, y, z


def sphere_sdf(n=64, radius=20.0, center=None, dtype=np.float32):
    """f(p) = |p - c| - radius on an n^3 grid (c = grid centre by default)."""
    nx = ny = nz = int(n)
    c = (np.array([nx - 1, ny - 1, nz - 1], dtype=np.float64) / 2.0
         if center is None else np.asarray(center, dtype=np.float64))
    x, y, z = _grid(nx, ny, nz)
    d2 = ((z - c[2])[:, None, None] ** 2 + (y - c[1])[None, :, None] ** 2
          + (x - c[0])[None, None, :] ** 2)
    return (np.sqrt(d2) - radius).astype(dtype)


def sphere_sdf_noisy(n=64, radius=20.0, noise=0.5, seed=1, dtype=np.float32):
    """Sphere distance field plus ``noise * N(0,1)`` per voxel (seeded)."""
    f = sphere_sdf(n, radius, dtype=np.float64)
    rng = np.random.default_rng(seed)
    f = f + noise * rng.standard_normal(f.shape)
    return f.astype(dtype)


def plane_z(nx, ny, nz, z0, dtype=np.float32):
    """f(p) = z - z0 (an axis-aligned plane)."""
    z = np.arange(nz, dtype=np.float64) - z0
    f = np.broadcast_to(z[:, None, None], (nz, ny, nx))
    return np.ascontiguousarray(f).astype(dtype)


def tilted_plane(nx, ny, nz, normal, d, dtype=np.float32):
    """f(p) = normal . p - d (a linear field)."""
    nrm = np.asarray(normal, dtype=np.float64)
    x, y, z = _grid(nx, ny, nz)
    f = (nrm[2] * z[:, None, None] + nrm[1] * y[None, :, None]
         + nrm[0] * x[None, None, :] - d)
    return f.astype(dtype)


def turbulence_modes(seed, n_modes=256, kmin=1.0 / 512.0, kmax=1.0 / 16.0):
    """Random Fourier modes: wave vectors k (cycles/voxel), amplitudes, phases.

    |k| is uniform in [kmin, kmax] with a uniform direction on the sphere, so
    the mode density is flat in |k|; amplitude |k|^(-5/6) then gives an
    energy spectrum E(k) ~ a^2 ~ k^(-5/3).
    """
    rng = np.random.default_rng(seed)
    kmag = rng.uniform(kmin, kmax, n_modes)
    d = rng.standard_normal((n_modes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    k = d * kmag[:, None]
    phase = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    amp = kmag ** (-5.0 / 6.0)
    return k, amp, phase


def _mode_sum(nx, ny, nz, k, amp, phase, slab=32):
    """sum_m amp_m cos(2 pi k_m . p + phase_m), evaluated separably.

    cos(2 pi k.p + phi) = Re(e^{i phi} X(x) Y(y) Z(z)) with per-axis complex
    exponentials, so each z-slab is one complex matrix product over modes.
    """
    x, y, z = _grid(nx, ny, nz)
    X = np.exp(2j * np.pi * np.outer(k[:, 0], x))            # [M, nx]
    Y = np.exp(2j * np.pi * np.outer(k[:, 1], y))            # [M, ny]
    Z = np.exp(2j * np.pi * np.outer(k[:, 2], z))            # [M, nz]
    c = amp * np.exp(1j * phase)                              # [M]
    out = np.empty((nz, ny, nx), dtype=np.float64)
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        # G[zz, y, m] = c_m Z[m, zz] Y[m, y]
        G = (c[None, None, :] * Z[:, z0:z1].T[:, None, :]) * Y.T[None, :, :]
        out[z0:z1] = np.real(G.reshape(-1, len(amp)) @ X).reshape(z1 - z0, ny, nx)
    return out


def turbulence(nx, ny=None, nz=None, seed=2, n_modes=256, dtype=np.float32,
               kmin=1.0 / 512.0, kmax=1.0 / 16.0):
    """Sum of random Fourier modes (k^-5/3 spectrum) normalised to mean 0, var 1."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    k, amp, phase = turbulence_modes(seed, n_modes, kmin, kmax)
    f = _mode_sum(nx, ny, nz, k, amp, phase)
    f -= f.mean()
    f /= f.std()
    return f.astype(dtype)


def gaussian_blobs(n=256, n_blobs=16, seed=3, dtype=np.float32):
    """sum_i A_i exp(-|p - c_i|^2 / (2 sigma_i^2)); c_i ~ U[0,n)^3,
    sigma_i ~ U[8,24], A_i ~ U[0.5,1.5]."""
    rng = np.random.default_rng(seed)
    cen = rng.uniform(0.0, float(n), (n_blobs, 3))
    sig = rng.uniform(8.0, 24.0, n_blobs)
    amp = rng.uniform(0.5, 1.5, n_blobs)
    x = np.arange(n, dtype=np.float64)
    f = np.zeros((n, n, n), dtype=np.float64)
    for i in range(n_blobs):
        g = [np.exp(-((x - cen[i, a]) ** 2) / (2.0 * sig[i] ** 2)) for a in range(3)]
        f += amp[i] * (g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :])
    return f.astype(dtype)


def batched_dims(n_volumes=48, seed=4, lo=32, hi=256):
    """Per-volume (nx, ny, nz), each axis an independent integer in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in row) for row in rng.integers(lo, hi + 1, size=(n_volumes, 3))]


def random_block_stream(dims, rate, is_f64=False, density=0.5, seed=0, exp_spread=20,
                        zero_every=0):
    """Random fixed-rate block words for a (nx, ny, nz) volume: every bit of
    every block drawn independently with P(1) = density, except the block
    header (the nonzero flag, set, and the biased exponent, drawn within
    +-exp_spread of the bias so that every decoded value is finite).  With
    zero_every > 0 every zero_every-th block is flagged all-zero.  Exercises
    the decoders on bit patterns a smooth field rarely produces (long zero
    runs, budgets that end inside a run).  Returns uint64 words, rate per
    block, blocks x-fastest."""
    nx, ny, nz = dims
    nb = ((nx + 3) // 4) * ((ny + 3) // 4) * ((nz + 3) // 4)
    rng = np.random.default_rng(seed)
    bits = rng.random((nb, 64 * rate)) < density
    ebits, bias = (11, 1023) if is_f64 else (8, 127)
    e = bias + rng.integers(-exp_spread, exp_spread + 1, size=nb)
    bits[:, 0] = True
    for i in range(ebits):
        bits[:, 1 + i] = ((e >> i) & 1).astype(bool)
    if zero_every > 0:
        bits[::zero_every, 0] = False
    return np.packbits(bits, axis=1, bitorder="little").view("<u8").reshape(-1).copy()


def percentile_iso(values, p):
    """Isovalue at the p-th percentile (linear interpolation) of ``values``,
    taken in float64 and rounded to float32."""
    v = np.asarray(values, dtype=np.float64).ravel()
    return np.float32(np.percentile(v, p, method="linear"))


def turbulence_torch(nx, ny=None, nz=None, seed=2, n_modes=256, device="cuda",
                     kmin=1.0 / 512.0, kmax=1.0 / 16.0, slab=64):
    """Same field as ``turbulence`` (same seeded modes), summed on ``device``
    with torch in float64; returns a float32 tensor [nz, ny, nx].  The result
    matches the numpy version up to the rounding of the mode sum."""
    import torch
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    k, amp, phase = turbulence_modes(seed, n_modes, kmin, kmax)
    kt = torch.tensor(k, dtype=torch.float64, device=device)
    c = torch.tensor(amp * np.exp(1j * phase), dtype=torch.complex128, device=device)

    def axis(n, col):
        x = torch.arange(n, dtype=torch.float64, device=device)
        return torch.exp(2j * np.pi * torch.outer(kt[:, col], x))      # [M, n]

    X, Y, Z = axis(nx, 0), axis(ny, 1), axis(nz, 2)
    out = torch.empty((nz, ny, nx), dtype=torch.float64, device=device)
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        G = (c[None, None, :] * Z[:, z0:z1].T[:, None, :]) * Y.T[None, :, :]
        out[z0:z1] = torch.real(G.reshape(-1, n_modes) @ X).reshape(z1 - z0, ny, nx)
    out -= out.mean()
    out /= out.std(unbiased=False)
    return out.to(torch.float32)


def percentile_iso_torch(values, p):
    """``percentile_iso`` for a (possibly huge) torch tensor: sort on the
    device, then numpy's linear interpolation in float64 between the two
    neighbouring order statistics."""
    import torch
    v = values.reshape(-1)
    n = v.numel()
    h = (n - 1) * (p / 100.0)
    lo = int(np.floor(h))
    hi = min(lo + 1, n - 1)
    s = torch.sort(v.to(torch.float32)).values
    a, b = float(s[lo].item()), float(s[hi].item())
    del s
    t = h - lo
    # numpy's linear interpolation, including its form for t >= 1/2
    return np.float32(b - (b - a) * (1.0 - t) if t >= 0.5 else a + (b - a) * t)


def channel_flow_slab(z0, z1, dims=CHANNEL_FLOW_DIMS, seed=5, n_modes=256, delta=None,
                      rel_amp=0.1, kmin=1.0 / 1024.0, kmax=1.0 / 16.0, device="cuda"):
    """z-planes [z0, z1) of a channel-flow-like float64 field, generated on
    ``device`` with torch so that the whole volume never exists at once:

        f(p) = tanh((y - (ny - 1)/2) / delta) + rel_amp * T(p) / sigma_T

    T is a sum of random Fourier modes with the k^(-5/3) law of
    ``turbulence_modes`` (wavelengths 16..1024 voxels by default) and
    sigma_T = sqrt(sum a_m^2 / 2) its analytic standard deviation; delta
    defaults to ny / 10.  Returns a float64 tensor [z1 - z0, ny, nx]; the
    value of a sample does not depend on which slab it is generated in, up to
    the rounding of the mode sum."""
    import torch
    nx, ny, nz = (int(d) for d in dims)
    delta = ny / 10.0 if delta is None else float(delta)
    k, amp, phase = turbulence_modes(seed, n_modes, kmin, kmax)
    sigma = float(np.sqrt(np.sum(amp ** 2) / 2.0))
    kt = torch.tensor(k, dtype=torch.float64, device=device)
    c = torch.tensor(amp * np.exp(1j * phase) * (rel_amp / sigma), dtype=torch.complex128,
                     device=device)

    def axis(lo, hi, col):
        x = torch.arange(lo, hi, dtype=torch.float64, device=device)
        return torch.exp(2j * np.pi * torch.outer(kt[:, col], x))      # [M, n]

    X, Y, Z = axis(0, nx, 0), axis(0, ny, 1), axis(z0, z1, 2)
    yv = torch.arange(ny, dtype=torch.float64, device=device)
    mean = torch.tanh((yv - (ny - 1) / 2.0) / delta)                  # [ny]
    out = torch.empty((z1 - z0, ny, nx), dtype=torch.float64, device=device)
    for zz in range(z1 - z0):
        G = c[None, :] * Z[:, zz][None, :] * Y.T                       # [ny, M]
        out[zz] = torch.real(G @ X)
        out[zz] += mean[:, None]
    return out
