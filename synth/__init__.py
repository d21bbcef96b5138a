"""Seeded synthetic velocity snapshots on hexahedral spectral-element meshes.

Shared by the tests, the bench and the oracle checks; it holds none of the
compression method's arithmetic (no transform, norm, energy or threshold), only
the input recipe.  It stands in for the paper's NEKO Taylor-Green snapshots
(arXiv 2407.20731, Sec. IV-A/IV-B: 64^3 elements on GPUs), which are not
available: a divergence-free sum of random Fourier modes with a k^-5/3
amplitude spectrum plus small Gaussian noise, sampled at the GLL points of
each element.

Recipe (all draws from ``numpy.random.default_rng(seed)`` in this order):
  1. modes: ``n_modes`` integer wave vectors uniform in the ball
     0 < |k| <= kmax (rejection from the cube [-kmax, kmax]^3), amplitude
     |k|^(-5/3); then one phase per mode, U[0, 2 pi); then one direction per
     mode: a standard normal 3-vector with its k-component removed,
     normalised (so each mode is divergence free).
  2. field: u_c(x) = sum_m a_m d_{m,c} cos(k_m . x + phi_m) at every GLL
     point; each component is scaled to unit RMS over its stored values.
  3. noise: i.i.d. N(0, noise^2) added to every stored value, drawn in
     [c][e][k][j][i] order.
Mesh: E cubes of edge h = 2 pi / 8 on an nx * ny * nz block grid with
nx = ny = ceil(E^(1/3)), nz = ceil(E / (nx ny)); element e sits at
(e mod nx, (e div nx) mod ny, e div (nx ny)).  E = 512 is exactly the
8^3 box [0, 2 pi)^3.

The node positions use numpy's own Legendre root finder (they only decide
where the synthetic field is sampled).
"""

from __future__ import annotations

import math
from functools import lru_cache

import numpy as np

__all__ = ["mesh_dims", "gll_points", "modes", "field", "element_pool"]


def mesh_dims(n_elem: int):
    nx = int(math.ceil(round(n_elem ** (1.0 / 3.0), 12)))
    while nx ** 3 < n_elem:
        nx += 1
    while nx > 1 and (nx - 1) ** 3 >= n_elem:
        nx -= 1
    ny = nx
    nz = int(math.ceil(n_elem / (nx * ny)))
    return nx, ny, nz


@lru_cache(maxsize=None)
def gll_points(order: int) -> np.ndarray:
    """Sampling positions on [-1, 1]: endpoints plus the roots of P_N'."""
    if order == 1:
        return np.array([-1.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(order).deriv().roots()
    return np.concatenate(([-1.0], np.sort(inner.real), [1.0]))


def modes(rng: np.random.Generator, n_modes: int, kmax: float):
    ks = []
    r = int(math.floor(kmax))
    while len(ks) < n_modes:
        k = rng.integers(-r, r + 1, size=3)
        kk = float(np.dot(k, k))
        if 0.0 < kk <= kmax * kmax:
            ks.append(k)
    k = np.array(ks, dtype=np.float64)
    knorm = np.sqrt((k * k).sum(axis=1))
    amp = knorm ** (-5.0 / 3.0)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    g = rng.standard_normal(size=(n_modes, 3))
    khat = k / knorm[:, None]
    d = g - (g * khat).sum(axis=1, keepdims=True) * khat
    d /= np.sqrt((d * d).sum(axis=1, keepdims=True))
    return k, amp, phase, d


def _axis_phasors(k_axis: np.ndarray, nblk: int, xi: np.ndarray, h: float) -> np.ndarray:
    """exp(i k x) for every mode and every sampled coordinate along one axis,
    coordinates ordered (block, node): shape [n_modes, nblk * n]."""
    x = (np.arange(nblk)[:, None] * h + (xi[None, :] + 1.0) * (0.5 * h)).ravel()
    return np.exp(1j * k_axis[:, None] * x[None, :])


def field(n_elem: int, order: int, ncomp: int = 3, seed: int = 1, n_modes: int = 64,
          kmax: float = 4.0, noise: float = 1e-6, dtype=np.float64) -> np.ndarray:
    """Synthetic snapshot u[ncomp, n_elem, n, n, n] (C order, i fastest)."""
    if ncomp > 3:
        raise ValueError("the Fourier-mode recipe defines at most 3 components")
    rng = np.random.default_rng(seed)
    k, amp, phase, d = modes(rng, n_modes, kmax)
    n = order + 1
    xi = gll_points(order)
    h = 2.0 * math.pi / 8.0
    nx, ny, nz = mesh_dims(n_elem)
    EX = _axis_phasors(k[:, 0], nx, xi, h)  # [M, nx*n]
    EY = _axis_phasors(k[:, 1], ny, xi, h)
    EZ = _axis_phasors(k[:, 2], nz, xi, h)
    e = np.arange(n_elem)
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    out = np.empty((ncomp, n_elem, n, n, n), dtype=np.float64)
    for c in range(ncomp):
        coef = amp * d[:, c] * np.exp(1j * phase)          # [M]
        # grid[zk, yj, xi] = Re sum_m coef_m EZ[m,zk] EY[m,yj] EX[m,xi]
        W = (coef[:, None, None] * EZ[:, :, None] * EY[:, None, :])  # [M, Z, Y]
        M = W.shape[0]
        grid = (W.reshape(M, -1).T @ EX).real.reshape(nz * n, ny * n, nx * n)
        g = grid.reshape(nz, n, ny, n, nx, n)
        # element e -> [k][j][i] block of the grid
        out[c] = g[ez, :, ey, :, ex, :]
        rms = math.sqrt(float(np.mean(out[c] * out[c])))
        if rms > 0:
            out[c] /= rms
    if noise:
        out += rng.normal(0.0, noise, size=out.shape)
    return out.astype(dtype, copy=False)


def field_torch(n_elem: int, order: int, ncomp: int = 3, seed: int = 1, n_modes: int = 64,
                kmax: float = 4.0, noise: float = 1e-6, device: str = "cuda", chunk: int = 8192):
    """The same recipe evaluated with torch on a device, for large element pools
    (bench workloads).  Mode draws use the same numpy generator; the field is
    summed per element chunk as a batched complex product, and the noise comes
    from torch's generator seeded with `seed` (so values differ from `field`
    in rounding and noise, not in distribution)."""
    import torch

    if ncomp > 3:
        raise ValueError("the Fourier-mode recipe defines at most 3 components")
    rng = np.random.default_rng(seed)
    k, amp, phase, d = modes(rng, n_modes, kmax)
    n = order + 1
    xi = gll_points(order)
    h = 2.0 * math.pi / 8.0
    nx, ny, nz = mesh_dims(n_elem)
    cd = torch.complex128
    EX = torch.from_numpy(_axis_phasors(k[:, 0], nx, xi, h).reshape(n_modes, nx, n)).to(device, cd)
    EY = torch.from_numpy(_axis_phasors(k[:, 1], ny, xi, h).reshape(n_modes, ny, n)).to(device, cd)
    EZ = torch.from_numpy(_axis_phasors(k[:, 2], nz, xi, h).reshape(n_modes, nz, n)).to(device, cd)
    out = torch.empty((ncomp, n_elem, n, n, n), dtype=torch.float64, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    for c in range(ncomp):
        coef = torch.from_numpy(amp * d[:, c] * np.exp(1j * phase)).to(device, cd)  # [M]
        for e0 in range(0, n_elem, chunk):
            e = torch.arange(e0, min(n_elem, e0 + chunk), device=device)
            ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
            zk = (coef[:, None, None] * EZ[:, ez, :]).permute(1, 2, 0).contiguous()      # [B, n(k), M]
            yx = (EY[:, ey, :, None] * EX[:, ex, None, :]).permute(1, 0, 2, 3)            # [B, M, n(j), n(i)]
            yx = yx.reshape(e.numel(), n_modes, n * n).contiguous()
            out[c, e0:e0 + e.numel()] = torch.bmm(zk, yx).real.reshape(-1, n, n, n)
        rms = torch.sqrt(torch.mean(out[c] * out[c]))
        if rms > 0:
            out[c] /= rms
    if noise:
        out += noise * torch.randn(out.shape, generator=gen, dtype=torch.float64, device=device)
    return out


def element_pool(n_elem: int, order: int, seed: int, ncomp: int = 3) -> np.ndarray:
    """A pool of elements from which request windows are taken."""
    return field(n_elem, order, ncomp=ncomp, seed=seed)


def flat_spectrum(n_elem: int, order: int, ncomp: int = 1, seed: int = 1, spread: float = 1e-3) -> np.ndarray:
    """Nodal fields whose Legendre coefficients all carry nearly the same
    energy: c_pqr = s (1 + spread * U) / sqrt(gamma_p gamma_q gamma_r), random
    signs s and U uniform in [0, 1), with the discrete GLL norms gamma_k =
    2/(2k+1) and 2/N for k = N; u = sum c P_p(xi_i) P_q(xi_j) P_r(xi_k)
    (numpy's Legendre evaluator at gll_points).  Every energy lies in
    [1, (1 + spread)^2): one exponent bin holds (nearly) all of them, the
    worst case for candidate lists built around a few bins."""
    rng = np.random.default_rng(seed)
    n = order + 1
    x = gll_points(order)
    P = np.polynomial.legendre.legvander(x, order)  # [node, degree]
    gam = 2.0 / (2.0 * np.arange(n) + 1.0)
    gam[-1] = 2.0 / order
    g3 = gam[:, None, None] * gam[None, :, None] * gam[None, None, :]  # [r, q, p]
    sign = rng.choice([-1.0, 1.0], size=(ncomp, n_elem, n, n, n))
    c = sign * (1.0 + spread * rng.random((ncomp, n_elem, n, n, n))) / np.sqrt(g3)
    return np.ascontiguousarray(np.einsum("kr,jq,ip,cerqp->cekji", P, P, P, c, optimize=True))
