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


# The library's launch rule for its row-staged kernels, restated so that a test
# can require them (DSLASH_ROWS=2) exactly where they apply.
WORD_BYTES = {"c64": 8, "c128": 16, "bf16": 4, "f16": 4}


def row_sites(nx, nv):
    """Default chunk length: fewest chunks of at most 16 sites (more where
    fewer than 128 threads would result), at most 256 threads, split evenly."""
    want, lim = -(-128 // nv), 256 // nv
    cap = min(want, lim) if want > 16 else min(16, lim)
    k = -(-nx // cap)
    r = -(-nx // k)
    rmin = min(want, cap)
    if r < rmin:
        r = nx if nx < rmin else rmin
    return min(r, nx)


def wilson_rows_cover(nx, nv, dt):
    """D_W t-marching kernel (FP32 arithmetic storages): N_v in 4, 8, 12, 16,
    24, 64 .. 256 threads, and the own row's two halo sites in the extra
    register groups (one, or two at N_v > 16 with 8-byte words or where the
    link words need them)."""
    if dt not in ("c64", "bf16", "f16") or nv not in (4, 8, 12, 16, 24):
        return False
    r, wb = row_sites(nx, nv), WORD_BYTES[dt]
    links = (-(-9 // nv) * wb + 15) // 16
    halo = (24 * wb // 16 + 7) // 8 if nv > 16 else 1
    return 64 <= r * nv <= 256 and r * 16 * max(links, halo) >= 24 * wb


def staggered_rows_cover(nx, nv, dt):
    """D_S t-marching kernel (C64, C128): N_v in 4, 8, 12, 16, 24, 64 .. 256
    threads and at least 6 sites per chunk."""
    if dt not in ("c64", "c128") or nv not in (4, 8, 12, 16, 24):
        return False
    r = row_sites(nx, nv)
    return r >= 6 and 64 <= r * nv <= 256


def brillouin_rows_cover(nx, nv, dt):
    """D_B row-staged kernels: FP32 storage at N_v in 4, 8, 12, 16, 24 with
    64 .. 256 threads and the halo in HK pieces a thread (R HK >= 12, HK = 2
    above N_v = 16); FP64 storage at N_v = 12 (chunks of 16 sites)."""
    if dt == "c128":
        return nv == 12
    if dt != "c64" or nv not in (4, 8, 12, 16, 24):
        return False
    r = row_sites(nx, nv)
    hk = 2 if nv > 16 else 1
    return r * hk >= 12 and 64 <= r * nv <= 256


def grad_rows_cover(nx, nv, op, dt):
    """Link-gradient row kernel: D_W in C64, D_S in C64 and C128; N_v in 4, 8,
    12, 16, 24, 64 .. 256 threads and at least 6 sites per chunk."""
    if nv not in (4, 8, 12, 16, 24):
        return False
    if not (dt == "c64" or (dt == "c128" and op == "staggered")):
        return False
    r = row_sites(nx, nv)
    return r >= 6 and 64 <= r * nv <= 256
