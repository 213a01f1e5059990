"""Small shared helpers for the test suite (no operator arithmetic)."""
import numpy as np


def plane_wave(dims, n):
    """e^{i p.x} on a [Nt][Nz][Ny][Nx] lattice with p_mu = 2 pi n_mu / N_mu."""
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    p = [2 * np.pi * n[i] / dims[i] for i in range(4)]
    return np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t)), np.array(p)


def coords(dims):
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x, y, z, t])


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def random_gauge(dims, seed):
    import synthetic
    shape = synthetic.lattice_shape(dims)
    return synthetic.haar_su3(int(np.prod(shape)), seed).reshape(shape + (3, 3))


def dag(u):
    return np.conj(np.swapaxes(u, -1, -2))


def read_golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def bf16_bits(a):
    """Round complex a to bfloat16 (RNE) on the host; returns uint16 [..., 2]."""
    f = np.stack([a.real, a.imag], -1).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return u


def from_bf16_bits(u):
    f = (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return f[..., 0] + 1j * f[..., 1]


def f16_pairs(a):
    return np.stack([a.real, a.imag], -1).astype(np.float32).astype(np.float16)


def from_f16_pairs(h):
    h = h.astype(np.float64)
    return h[..., 0] + 1j * h[..., 1]
