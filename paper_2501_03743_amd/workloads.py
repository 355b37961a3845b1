"""Seeded synthetic inputs for the s-step CG solver (host side, numpy).

This module only generates problems: grid operators in CSR form, right-hand
sides, manufactured solutions and random coefficient fields.  It holds none
of the solver's arithmetic, and both the HIP path and the CPU oracle take
their inputs from it.

The paper's own workload is the Poisson equation on a cube with Dirichlet
boundary conditions and right-hand side 1 (Sec. V); the other inputs here are
seeded synthetic stand-ins of the same kind.

Operators (unscaled, lexicographic index x + nx*(y + ny*z), Dirichlet zero
outside the grid, column indices ascending within a row):
  2d5       diagonal 4, neighbours -1 (2D)
  3d7       diagonal 6, neighbours -1
  3d27      diagonal 26, the 26 neighbours -1
  3d7_vark  -div(k grad u): face weight 2 k_p k_q / (k_p + k_q), weight k_p on
            faces to the boundary, diagonal = sum of the six face weights
"""
from __future__ import annotations

import numpy as np

DEFAULT_COEF = {"2d5": (4.0, -1.0), "3d7": (6.0, -1.0), "3d27": (26.0, -1.0)}


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def normal_rhs(n: int, seed: int) -> np.ndarray:
    """b ~ N(0, 1), FP64."""
    return rng(seed).standard_normal(n)


def uniform_solution(n: int, seed: int) -> np.ndarray:
    """x* ~ U(-1, 1), FP64."""
    return rng(seed).uniform(-1.0, 1.0, n)


def _grid(shape):
    if len(shape) == 2:
        return int(shape[0]), int(shape[1]), 1
    return int(shape[0]), int(shape[1]), int(shape[2])


def stencil_csr(kind: str, shape, k=None, coef=None):
    """(rowptr int32[n+1], colind int32[nnz], val float64[nnz]) of a grid operator."""
    nx, ny, nz = _grid(shape)
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    X = idx % nx
    Y = (idx // nx) % ny
    Z = idx // (nx * ny)
    if kind == "3d27":
        offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    elif kind == "2d5":
        offs = [(0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0)]
    elif kind in ("3d7", "3d7_vark"):
        offs = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    else:
        raise ValueError(kind)
    # offsets are listed in ascending index order, so per-row columns ascend
    cols, vals, masks = [], [], []
    d, o = coef if coef is not None else DEFAULT_COEF.get(kind, (0.0, 0.0))
    if kind == "3d7_vark":
        kk = np.asarray(k, dtype=np.float64).reshape(-1)
        diag = np.zeros(n)
    for (dx, dy, dz) in offs:
        qx, qy, qz = X + dx, Y + dy, Z + dz
        m = (qx >= 0) & (qx < nx) & (qy >= 0) & (qy < ny) & (qz >= 0) & (qz < nz)
        q = np.where(m, qx + nx * (qy + ny * qz), 0)
        if kind == "3d7_vark":
            if (dx, dy, dz) == (0, 0, 0):
                v = None
            else:
                w = np.where(m, 2.0 * kk * kk[q] / (kk + kk[q]), kk)
                diag += w
                v = -w
        else:
            v = np.full(n, d if (dx, dy, dz) == (0, 0, 0) else o)
        cols.append(q)
        vals.append(v)
        masks.append(m)
    if kind == "3d7_vark":
        vals[3] = diag
    M = np.stack(masks, axis=1)
    Cc = np.stack(cols, axis=1)[M]
    V = np.stack(vals, axis=1)[M]
    cnt = M.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=rowptr[1:])
    if rowptr[-1] >= 2 ** 31:
        raise ValueError("nnz exceeds int32 indexing")
    return rowptr.astype(np.int32), Cc.astype(np.int32), V.astype(np.float64)


def csr_matvec(csr, x):
    """y = A x for a CSR triple (scipy), used to manufacture b = A x*."""
    import scipy.sparse as sp
    rowptr, colind, val = csr
    n = len(rowptr) - 1
    A = sp.csr_matrix((val, colind, rowptr), shape=(n, n))
    return A @ np.asarray(x, dtype=np.float64)


def gaussian_random_field(shape, sigma: float, ell: float, seed: int) -> np.ndarray:
    """Stationary Gaussian field on the unit cube with squared-exponential
    covariance sigma^2 exp(-r^2 / (2 ell^2)), by FFT spectral synthesis on a
    periodic grid twice the size (cropped), normalised to sample std sigma."""
    nx, ny, nz = _grid(shape)
    g = rng(seed)
    ext = [2 * nx, 2 * ny, 2 * nz] if nz > 1 else [2 * nx, 2 * ny]
    h = 1.0 / (max(nx, ny, nz) + 1)
    freqs = np.meshgrid(*[np.fft.fftfreq(m, d=h) for m in ext], indexing="ij")
    k2 = sum(f * f for f in freqs) * (2.0 * np.pi) ** 2
    spec = np.exp(-0.25 * k2 * ell * ell)       # sqrt of the SE spectral density (unnormalised)
    noise = g.standard_normal(ext)
    field = np.real(np.fft.ifftn(np.fft.fftn(noise) * spec))
    if nz > 1:
        field = field[:nx, :ny, :nz]
    else:
        field = field[:nx, :ny]
    field = field - field.mean()
    field *= sigma / max(field.std(), 1e-300)
    # return in lexicographic (x fastest) order
    return np.ascontiguousarray(field.transpose()).reshape(-1)


def fourier_source(shape, seed: int, modes: int = 16) -> np.ndarray:
    """f(x) = sum_m a_m prod_d sin(pi kappa_{m,d} x_d), a_m ~ N(0,1),
    kappa ~ U{1..4}, sampled at the interior nodes x_d = (i+1) h."""
    nx, ny, nz = _grid(shape)
    g = rng(seed)
    a = g.standard_normal(modes)
    kap = g.integers(1, 5, size=(modes, 3))
    xs = [(np.arange(m) + 1.0) / (m + 1.0) for m in (nx, ny, nz)]
    f = np.zeros((nz, ny, nx))
    for m in range(modes):
        sx = np.sin(np.pi * kap[m, 0] * xs[0])
        sy = np.sin(np.pi * kap[m, 1] * xs[1])
        sz = np.sin(np.pi * kap[m, 2] * xs[2])
        f += a[m] * sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return f.reshape(-1)


def batch_sides(seed: int, count: int = 32, lo: int = 32, hi: int = 160) -> np.ndarray:
    """Side lengths L_i ~ U{lo..hi} for a batch of cubic grids."""
    return rng(seed).integers(lo, hi + 1, size=count)


# ---------------------------------------------------------------------------
# Device-side generators for large sample sets (same definitions as the host
# ones above; the noise comes from torch's seeded device generator, so values
# differ from the host versions but follow the same distribution).
# ---------------------------------------------------------------------------

_SPEC_CACHE = {}


def gaussian_random_field_device(shape, sigma: float, ell: float, seed: int, device="cuda"):
    """gaussian_random_field() on the device (torch FFTs; float64 tensor of
    n entries, x fastest)."""
    import torch
    nx, ny, nz = _grid(shape)
    ext = (2 * nz, 2 * ny, 2 * nx)            # (z, y, x): x fastest in memory
    key = (ext, float(ell), str(device))
    spec = _SPEC_CACHE.get(key)
    if spec is None:
        h = 1.0 / (max(nx, ny, nz) + 1)
        fz = torch.fft.fftfreq(ext[0], d=h, dtype=torch.float64, device=device)
        fy = torch.fft.fftfreq(ext[1], d=h, dtype=torch.float64, device=device)
        fx = torch.fft.rfftfreq(ext[2], d=h, dtype=torch.float64, device=device)
        k2 = (fz[:, None, None] ** 2 + fy[None, :, None] ** 2 + fx[None, None, :] ** 2) \
            * (2.0 * np.pi) ** 2
        spec = torch.exp(-0.25 * k2 * ell * ell)
        _SPEC_CACHE[key] = spec
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    noise = torch.randn(ext, generator=gen, device=device, dtype=torch.float64)
    field = torch.fft.irfftn(torch.fft.rfftn(noise) * spec, s=ext)
    field = field[:nz, :ny, :nx].contiguous()
    field = field - field.mean()
    field = field * (sigma / torch.clamp(field.std(unbiased=False), min=1e-300))
    return field.reshape(-1)


def fourier_source_device(shape, seed: int, modes: int = 16, device="cuda"):
    """fourier_source() on the device (same coefficients, float64 tensor)."""
    import torch
    nx, ny, nz = _grid(shape)
    g = rng(seed)
    a = g.standard_normal(modes)
    kap = g.integers(1, 5, size=(modes, 3))
    xs = [(torch.arange(m, dtype=torch.float64, device=device) + 1.0) / (m + 1.0)
          for m in (nx, ny, nz)]
    f = torch.zeros((nz, ny, nx), dtype=torch.float64, device=device)
    for m in range(modes):
        sx = torch.sin(np.pi * float(kap[m, 0]) * xs[0])
        sy = torch.sin(np.pi * float(kap[m, 1]) * xs[1])
        sz = torch.sin(np.pi * float(kap[m, 2]) * xs[2])
        f += float(a[m]) * sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return f.reshape(-1)


def warm_start_problem(shape, seed: int, sigma: float = 1.0, ell: float = 0.1, device="cuda"):
    """One variable-coefficient Poisson problem -div(k grad u) = f on the unit
    cube's interior grid: log k a Gaussian random field, f a random sum of
    Fourier modes, and b = h^2 f for the unscaled 3d7_vark operator
    (h = 1 / (N + 1)).  Returns float64 device tensors (log k, k, f, b)."""
    import torch
    nx, ny, nz = _grid(shape)
    logk = gaussian_random_field_device(shape, sigma, ell, 2 * seed, device)
    f = fourier_source_device(shape, 2 * seed + 1, device=device)
    h = 1.0 / (max(nx, ny, nz) + 1)
    return logk, torch.exp(logk), f, f * (h * h)


def random_graph_laplacian(n: int, seed: int, mean_degree: float = 6.0, hub_fraction: float = 0.01,
                           hub_degree: int = 60):
    """CSR (rowptr, colind, val) of L + I for a random undirected graph: most
    vertices get ~mean_degree random neighbours, a few hubs many more, so row
    lengths are irregular (1 to ~hub_degree + 1).  SPD (diagonally dominant)."""
    g = rng(seed)
    m = int(n * mean_degree / 2)
    src = g.integers(0, n, size=m)
    dst = g.integers(0, n, size=m)
    hubs = g.choice(n, size=max(1, int(n * hub_fraction)), replace=False)
    hs = np.repeat(hubs, hub_degree)
    hd = g.integers(0, n, size=hs.size)
    src = np.concatenate([src, hs])
    dst = np.concatenate([dst, hd])
    keep = src != dst
    src, dst = src[keep], dst[keep]
    a = np.concatenate([src, dst])
    b = np.concatenate([dst, src])
    key = np.unique(a.astype(np.int64) * n + b)
    rows, cols = key // n, key % n
    w = np.full(rows.size, -1.0)
    deg = np.bincount(rows, minlength=n).astype(np.float64)
    rows = np.concatenate([rows, np.arange(n)])
    cols = np.concatenate([cols, np.arange(n)])
    vals = np.concatenate([w, deg + 1.0])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return rowptr.astype(np.int32), cols.astype(np.int32), vals


def stencil_with_long_rows(shape, seed: int, every: int = 4, extra: int = 10):
    """The 3D 7-point CSR matrix plus, in one row of every `every`-th block of
    64 rows, `extra` symmetric long-range couplings (-0.05, diagonals raised
    to keep diagonal dominance): SPD, with a few rows longer than the 8-entry
    load chunk in otherwise regular slices."""
    rp, ci, va = stencil_csr("3d7", shape)
    n = len(rp) - 1
    g = rng(seed)
    rows = np.repeat(np.arange(n), np.diff(rp)).astype(np.int64)
    cols = ci.astype(np.int64)
    vals = va.copy()
    add_r, add_c = [], []
    for sl in range(0, (n + 63) // 64, every):
        r = min(sl * 64 + int(g.integers(0, 64)), n - 1)
        cand = g.choice(n, size=extra * 3, replace=False)
        cand = [int(c) for c in cand if abs(int(c) - r) > 1][:extra]
        for c in cand:
            add_r += [r, c]
            add_c += [c, r]
    key_old = rows * n + cols
    key_new = np.array(add_r, dtype=np.int64) * n + np.array(add_c, dtype=np.int64)
    key_new = np.setdiff1d(np.unique(key_new), key_old)
    nr, nc = key_new // n, key_new % n
    diag_add = np.bincount(nr, minlength=n) * 0.05
    rows = np.concatenate([rows, nr])
    cols = np.concatenate([cols, nc])
    vals = np.concatenate([vals, np.full(nr.size, -0.05)])
    vals[rows == cols] += diag_add[rows[rows == cols]]
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return rowptr.astype(np.int32), cols.astype(np.int32), vals
