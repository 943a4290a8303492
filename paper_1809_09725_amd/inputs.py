"""Seeded synthetic inputs: moving-ellipsoid phantoms and random operands.

This module only *makes data*; it holds none of the reconstruction method's
arithmetic (no projector, no basis, no solver).  Sinograms are the exact
line integrals of ellipse cross-sections (the textbook closed form of the
Radon transform of an ellipse, Kak & Slaney ch. 3), sampled on a continuous
rotation: projection i is taken at angle i*pi/Ntheta0 and time i/Ntheta, the
acquisition protocol of the paper (Sec. 2: angle and time are linked,
Sec. 5: a phantom of moving circles captured over several half-turns).

It works with numpy or torch arrays: ``sinogram`` evaluates on any torch
device so that full-size benchmark data can be synthesised on the GPU.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Phantom:
    """A set of z-aligned ellipsoids with linear in-plane motion.

    All lengths are in pixel units, centred coordinates (x = column - (N-1)/2,
    y = row - (N-1)/2, zc = slice - (Nz-1)/2).  Time t runs over [0, 1).
    """
    cx: np.ndarray
    cy: np.ndarray
    cz: np.ndarray
    ax: np.ndarray          # in-plane semi-axis along the rotated x'
    ay: np.ndarray          # in-plane semi-axis along the rotated y'
    az: np.ndarray          # semi-axis along z
    psi: np.ndarray         # in-plane rotation
    rho: np.ndarray         # density
    vx: np.ndarray          # velocity, pixels per unit time
    vy: np.ndarray
    drift: np.ndarray       # density drift: rho(t) = rho (1 + drift t)
    grow: np.ndarray        # radius growth: semi-axes scale (1 + grow t)
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.rho)


def make_phantom(N: int, Nz: int, Npi: int, n_ell: int, seed: int, *,
                 axis_range=(2.0, 8.0), z_axis_range=None, rho_range=(0.5, 1.0),
                 speed_per_halfturn=1.0, drift=0.0, sphere=None,
                 radius_frac=0.45) -> Phantom:
    """Random moving ellipsoids whose whole path stays inside radius_frac*N.

    axis_range          in-plane semi-axes, uniform
    z_axis_range        z semi-axes (None: same as in-plane, Nz=1 makes it moot)
    speed_per_halfturn  maximum displacement per half-turn, random direction
    drift               density drift amplitude d: rho(t) = rho (1 + d t), d ~ U(-drift, drift)
    sphere              (r0, r1, rho): a centred sphere whose radius grows r0 -> r1 over t
    """
    rs = np.random.default_rng(seed)
    n = n_ell
    ax = rs.uniform(*axis_range, n)
    ay = rs.uniform(*axis_range, n)
    zr = z_axis_range if z_axis_range is not None else axis_range
    az = rs.uniform(*zr, n) if Nz > 1 else np.full(n, 1e6)
    psi = rs.uniform(0.0, math.pi, n)
    rho = rs.uniform(*rho_range, n)
    speed = rs.uniform(0.0, speed_per_halfturn, n) * Npi          # pixels over t in [0,1)
    ang = rs.uniform(0.0, 2 * math.pi, n)
    vx, vy = speed * np.cos(ang), speed * np.sin(ang)
    # start point such that the whole segment [c, c + v] stays inside the disc
    rmax = radius_frac * N - np.maximum(ax, ay)
    rmax = np.maximum(rmax, 0.0)
    cx = np.empty(n); cy = np.empty(n)
    for j in range(n):
        for _ in range(1000):
            r = rmax[j] * math.sqrt(rs.uniform())
            a = rs.uniform(0, 2 * math.pi)
            x0, y0 = r * math.cos(a), r * math.sin(a)
            if math.hypot(x0 + vx[j], y0 + vy[j]) <= rmax[j]:
                break
        else:
            x0 = y0 = 0.0
            vx[j] = vy[j] = 0.0
        cx[j], cy[j] = x0, y0
    cz = rs.uniform(-0.5 * (Nz - 1), 0.5 * (Nz - 1), n) if Nz > 1 else np.zeros(n)
    dr = rs.uniform(-drift, drift, n) if drift else np.zeros(n)
    grow = np.zeros(n)
    ph = Phantom(cx, cy, cz, ax, ay, az, psi, rho, vx, vy, dr, grow)
    if sphere is not None:
        r0, r1, rho_s = sphere
        ph = Phantom(*(np.append(getattr(ph, k), v) for k, v in (
            ("cx", 0.0), ("cy", 0.0), ("cz", 0.0), ("ax", r0), ("ay", r0),
            ("az", r0 if Nz > 1 else 1e6), ("psi", 0.0), ("rho", rho_s), ("vx", 0.0),
            ("vy", 0.0), ("drift", 0.0), ("grow", (r1 - r0) / r0))))
    return ph


def sinogram(ph: Phantom, N: int, Nz: int, Ns: int, Ntheta: int, Npi: int, *,
             noise: float = 0.01, seed: int = 0, device: str = "cpu",
             chunk: int = 64):
    """Exact line integrals of the phantom on the continuous-rotation grid,
    plus Gaussian noise of standard deviation noise*max(g); float32 torch
    tensor of shape (Ntheta, Nz, Ns).  Evaluated in float64."""
    import torch
    dev = torch.device(device)
    n0 = Ntheta // Npi
    out = torch.empty((Ntheta, Nz, Ns), dtype=torch.float32, device=dev)
    s = torch.arange(Ns, dtype=torch.float64, device=dev) - 0.5 * (Ns - 1)
    zc = torch.arange(Nz, dtype=torch.float64, device=dev) - 0.5 * (Nz - 1)
    P = {k: torch.as_tensor(getattr(ph, k), dtype=torch.float64, device=dev)
         for k in ("cx", "cy", "cz", "ax", "ay", "az", "psi", "rho", "vx", "vy", "drift", "grow")}
    # cross-section scale of each ellipsoid at each slice centre: (Nz, n)
    dz = (zc[:, None] - P["cz"][None, :]) / P["az"][None, :]
    zs2 = torch.clamp(1.0 - dz * dz, min=0.0)
    for i0 in range(0, Ntheta, chunk):
        i = torch.arange(i0, min(i0 + chunk, Ntheta), dtype=torch.float64, device=dev)
        th = (i * math.pi) / n0                       # angle of projection i
        t = i / Ntheta                                # its time
        acc = torch.zeros((len(i), Nz, Ns), dtype=torch.float64, device=dev)
        for j in range(ph.n):
            g = 1.0 + P["grow"][j] * t                # (T,)
            A = P["ax"][j] * g
            B = P["ay"][j] * g
            x0 = P["cx"][j] + P["vx"][j] * t
            y0 = P["cy"][j] + P["vy"][j] * t
            rho = P["rho"][j] * (1.0 + P["drift"][j] * t)
            c, sn = torch.cos(th), torch.sin(th)
            d = th - P["psi"][j]
            a2 = (A * torch.cos(d)) ** 2 + (B * torch.sin(d)) ** 2   # (T,)
            sh = x0 * c + y0 * sn                                      # (T,)
            zz = zs2[:, j]                                             # (Nz,)
            # ellipse scaled by sqrt(zz): semi-axes A', B' and a'^2 = zz a2
            a2z = a2[:, None] * zz[None, :]                            # (T,Nz)
            ABz = (A * B)[:, None] * zz[None, :]
            sp = s[None, None, :] - sh[:, None, None]                  # (T,1,Ns)
            rad = torch.clamp(a2z[:, :, None] - sp * sp, min=0.0)
            val = 2.0 * rho[:, None, None] * ABz[:, :, None] * torch.sqrt(rad) / \
                torch.clamp(a2z[:, :, None], min=1e-300)
            acc += torch.where(a2z[:, :, None] > 0, val, torch.zeros_like(val))
        out[i0:i0 + len(i)] = acc.to(torch.float32)
    if noise > 0:
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed)
        sig = noise * float(out.max())
        out += sig * torch.randn(out.shape, generator=gen, device=dev, dtype=torch.float32)
    return out


def frames(ph: Phantom, N: int, Nz: int, t: float) -> np.ndarray:
    """Point-sampled object state at time t, shape (Nz, N, N), float64."""
    x = np.arange(N) - 0.5 * (N - 1)
    zc = np.arange(Nz) - 0.5 * (Nz - 1)
    X, Y = np.meshgrid(x, x, indexing="xy")       # X[r,q] = x_q, Y[r,q] = y_r
    out = np.zeros((Nz, N, N))
    for j in range(ph.n):
        gr = 1.0 + ph.grow[j] * t
        A, B = ph.ax[j] * gr, ph.ay[j] * gr
        x0, y0 = ph.cx[j] + ph.vx[j] * t, ph.cy[j] + ph.vy[j] * t
        rho = ph.rho[j] * (1.0 + ph.drift[j] * t)
        c, s = math.cos(ph.psi[j]), math.sin(ph.psi[j])
        u = (X - x0) * c + (Y - y0) * s
        v = -(X - x0) * s + (Y - y0) * c
        for z in range(Nz):
            zz = 1.0 - ((zc[z] - ph.cz[j]) / ph.az[j]) ** 2
            if zz <= 0:
                continue
            inside = (u / A) ** 2 + (v / B) ** 2 <= zz
            out[z][inside] += rho
    return out


def uniform(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Seeded uniform float32 values (numpy PCG64)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape).astype(np.float32)


def smooth_coeffs(N: int, Nz: int, K: int, seed: int, n_ell: int = 6) -> np.ndarray:
    """Structured coefficient volumes (Nz, N, N, K), float32: each channel k is
    a random ellipse image scaled by 2^-k, so the low basis indices dominate
    as they do for slowly moving objects."""
    rs = np.random.default_rng(seed)
    out = np.zeros((Nz, N, N, K), np.float32)
    for k in range(K):
        ph = make_phantom(N, Nz, 1, n_ell, int(rs.integers(1 << 30)),
                          axis_range=(N / 16 + 1, N / 5 + 1), rho_range=(-1.0, 1.0),
                          speed_per_halfturn=0.0, z_axis_range=(Nz / 4 + 1, Nz + 1))
        out[..., k] = (frames(ph, N, Nz, 0.0) * 2.0 ** (-k)).astype(np.float32)
    return out
