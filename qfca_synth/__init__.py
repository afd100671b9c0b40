"""Seeded synthetic feature maps for the QFCA hot path.

This module is shared input infrastructure: it makes stationary Gaussian
random-field textures with inserted anomalies and holds none of the method's
arithmetic (no PCA, no quantisation, no histograms).  Both the HIP path and the
FP64 oracle are fed from here.

Recipe (stand-in for Wide-ResNet-50 layer-2 features of texture images, which
are not available here):

1. Z ~ N(0, 1) of shape [C, H, W] from numpy's PCG64 with the given seed.
2. Periodic Gaussian blur of every channel through the FFT.  Either isotropic
   (sigma px) or anisotropic with (sigma_u, sigma_v, theta) drawn once per seed:
   sigma_u ~ U[1.5, 6], sigma_v ~ U[0.5, 1.5], theta ~ U[0, pi), which makes the
   texture directional.
3. Standardise every channel to zero mean and unit variance.
4. Mix across channels: X = M Z with M_ij ~ N(0, 1/C).
5. Insert axis-aligned, non-overlapping anomalous squares, recording a mask:
   * "shift":   +1.5 sigma_c on a channel subset S,
   * "scale":   x <- mu_c + sqrt(3) (x - mu_c) on S (variance x3),
   * "permute": X[S] <- X[pi(S)] inside the square (local channel permutation).
6. Cast to float32, layout [C][H][W] (channel-planar).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

ANOMALY_KINDS = ("shift", "scale", "permute")


@dataclass
class Texture:
    X: np.ndarray            # [C, H, W] float32
    mask: np.ndarray         # [H, W] uint8, 1 inside an anomaly
    anomalies: list = field(default_factory=list)  # (kind, y, x, size)
    seed: int = 0

    def digest(self) -> str:
        return hashlib.sha256(self.X.tobytes()).hexdigest()[:16]


def _blur_fft(Z: np.ndarray, sig_u: float, sig_v: float, theta: float) -> np.ndarray:
    C, H, W = Z.shape
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.rfftfreq(W)[None, :]
    ct, st = np.cos(theta), np.sin(theta)
    fu = ct * fx + st * fy
    fv = -st * fx + ct * fy
    # Fourier transform of a unit-mass anisotropic Gaussian.
    g = np.exp(-2.0 * np.pi ** 2 * ((sig_u * fu) ** 2 + (sig_v * fv) ** 2))
    out = np.empty_like(Z)
    for c in range(C):
        out[c] = np.fft.irfft2(np.fft.rfft2(Z[c]) * g, s=(H, W))
    return out


def _place_squares(rng, H, W, sizes, margin=0):
    placed = []
    for s in sizes:
        for _ in range(1000):
            y = int(rng.integers(margin, max(margin + 1, H - s - margin + 1)))
            x = int(rng.integers(margin, max(margin + 1, W - s - margin + 1)))
            ok = all(y + s <= py or py + ps <= y or x + s <= px or px + ps <= x
                     for (py, px, ps) in placed)
            if ok:
                placed.append((y, x, s))
                break
        else:
            raise RuntimeError("could not place anomaly squares without overlap")
    return placed


def make_texture(C: int, H: int, W: int, seed: int, *, iso_sigma: float | None = None,
                 anomalies=(), subset: int | None = None, class_seed: int | None = None,
                 dtype=np.float32) -> Texture:
    """Make one texture.

    iso_sigma: isotropic blur width in px; None draws the anisotropic blur.
    anomalies: sequence of (kind, size) or (kind, size_lo, size_hi).
    subset: number of channels an anomaly touches (default C // 4, at least 1).
    class_seed: when given, the blur parameters and the mixing matrix come from
        this seed (a texture class) and only the noise and anomalies from `seed`.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    crng = rng if class_seed is None else np.random.Generator(np.random.PCG64(class_seed))
    if iso_sigma is not None:
        su = sv = float(iso_sigma)
        th = 0.0
    else:
        su = float(crng.uniform(1.5, 6.0))
        sv = float(crng.uniform(0.5, 1.5))
        th = float(crng.uniform(0.0, np.pi))
    M = crng.standard_normal((C, C)) / np.sqrt(C)
    Z = rng.standard_normal((C, H, W))
    Z = _blur_fft(Z, su, sv, th)
    Z -= Z.mean(axis=(1, 2), keepdims=True)
    Z /= Z.std(axis=(1, 2), keepdims=True)
    X = (M @ Z.reshape(C, -1)).reshape(C, H, W)

    sizes, kinds = [], []
    for a in anomalies:
        kind = a[0]
        if kind not in ANOMALY_KINDS:
            raise ValueError(kind)
        s = int(a[1]) if len(a) == 2 else int(rng.integers(a[1], a[2] + 1))
        kinds.append(kind)
        sizes.append(min(s, H, W))
    mask = np.zeros((H, W), np.uint8)
    info = []
    if sizes:
        placed = _place_squares(rng, H, W, sizes)
        ns = subset if subset is not None else max(1, C // 4)
        ns = min(ns, C)
        mu = X.mean(axis=(1, 2))
        sd = X.std(axis=(1, 2))
        for kind, (y, x, s) in zip(kinds, placed):
            S = rng.choice(C, size=ns, replace=False)
            win = (slice(y, y + s), slice(x, x + s))
            if kind == "shift":
                X[S, win[0], win[1]] += 1.5 * sd[S, None, None]
            elif kind == "scale":
                X[S, win[0], win[1]] = mu[S, None, None] + np.sqrt(3.0) * (
                    X[S, win[0], win[1]] - mu[S, None, None])
            else:
                perm = S[rng.permutation(ns)] if ns > 1 else S
                if ns > 1 and np.all(perm == S):
                    perm = np.roll(S, 1)
                X[S, win[0], win[1]] = X[perm, win[0], win[1]].copy()
            mask[win] = 1
            info.append((kind, y, x, s))
    return Texture(X=np.ascontiguousarray(X.astype(dtype)), mask=mask, anomalies=info, seed=seed)


# ---------------------------------------------------------------------------
# Named workloads.  Each returns (textures, params) where params is a dict with
# C, k, B, T, q_lo, q_hi, sigma_s.

def workload_small(seed: int = 1):
    """64x64 map, C=64, isotropic blur sigma=2, one 8x8 mean-shift square on 16
    channels.  PCA to 16, B=16, T=7."""
    t = make_texture(64, 64, 64, seed, iso_sigma=2.0, anomalies=[("shift", 8)], subset=16)
    return [t], dict(C=64, k=16, B=16, T=7, q_lo=0.01, q_hi=0.99, sigma_s=1.0)


def workload_256(seed: int = 100):
    """256x256 map, C=256, anisotropic blur, three anomalies (shift, scale,
    permute) of side 8..32.  PCA to 32, B=32, T=15."""
    t = make_texture(256, 256, 256, seed,
                     anomalies=[("shift", 8, 32), ("scale", 8, 32), ("permute", 8, 32)])
    return [t], dict(C=256, k=32, B=32, T=15, q_lo=0.01, q_hi=0.99, sigma_s=1.0)


BATCH_SIDES = (128, 192, 256, 384, 512)


def batch_sides(n: int = 64, seed: int = 3):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(s) for s in rng.choice(BATCH_SIDES, size=n)]


def workload_batch(n: int = 64, C: int = 256, first_seed: int = 300, sides=None):
    """n images with sides drawn from {128,192,256,384,512}, C=256, anisotropic
    blur, one anomaly of each kind.  PCA to 32, B=32, T=15."""
    sides = sides if sides is not None else batch_sides(n)
    texs = [make_texture(C, s, s, first_seed + i,
                         anomalies=[("shift", 8, 32), ("scale", 8, 32), ("permute", 8, 32)])
            for i, s in enumerate(sides)]
    return texs, dict(C=C, k=32, B=32, T=15, q_lo=0.01, q_hi=0.99, sigma_s=1.0)


def poisson_arrivals(rate: float, duration: float, seed: int = 4, sides=(128, 256, 512),
                     n_classes: int = 8):
    """Open-loop Poisson request schedule: list of (t_arrival_s, side, class_id)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        out.append((t, int(rng.choice(sides)), int(rng.integers(0, n_classes))))
    return out


# ---------------------------------------------------------------------------
# Device-side generator for large batches: the same recipe (blur, standardise,
# mix, anomalous squares) drawn with torch's generator on the GPU.  It does
# not reproduce the numpy streams above; it is used where generating on the
# host would take minutes (64 images up to 512x512x256).

def make_texture_torch(C: int, H: int, W: int, seed: int, device="cuda", *, anomalies=(),
                       subset: int | None = None, class_seed: int | None = None):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    cg = g if class_seed is None else torch.Generator(device=device)
    if class_seed is not None:
        cg.manual_seed(int(class_seed))
    su = float(torch.empty(1, device=device).uniform_(1.5, 6.0, generator=cg))
    sv = float(torch.empty(1, device=device).uniform_(0.5, 1.5, generator=cg))
    th = float(torch.empty(1, device=device).uniform_(0.0, float(np.pi), generator=cg))
    M = torch.randn((C, C), generator=cg, device=device, dtype=torch.float32) / np.sqrt(C)
    Z = torch.randn((C, H, W), generator=g, device=device, dtype=torch.float32)
    fy = torch.fft.fftfreq(H, device=device)[:, None]
    fx = torch.fft.rfftfreq(W, device=device)[None, :]
    ct, st = np.cos(th), np.sin(th)
    fu = ct * fx + st * fy
    fv = -st * fx + ct * fy
    filt = torch.exp(-2.0 * np.pi ** 2 * ((su * fu) ** 2 + (sv * fv) ** 2))
    Z = torch.fft.irfft2(torch.fft.rfft2(Z) * filt, s=(H, W))
    Z = (Z - Z.mean(dim=(1, 2), keepdim=True)) / Z.std(dim=(1, 2), keepdim=True)
    X = (M @ Z.reshape(C, -1)).reshape(C, H, W)
    mask = torch.zeros((H, W), dtype=torch.uint8, device=device)
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes, kinds = [], []
    for a in anomalies:
        s = int(a[1]) if len(a) == 2 else int(rng.integers(a[1], a[2] + 1))
        kinds.append(a[0])
        sizes.append(min(s, H, W))
    info = []
    if sizes:
        placed = _place_squares(rng, H, W, sizes)
        ns = min(subset if subset is not None else max(1, C // 4), C)
        mu = X.mean(dim=(1, 2))
        sd = X.std(dim=(1, 2))
        for kind, (y, x, s) in zip(kinds, placed):
            S = torch.from_numpy(rng.choice(C, size=ns, replace=False)).to(device)
            if kind == "shift":
                X[S, y:y + s, x:x + s] += 1.5 * sd[S, None, None]
            elif kind == "scale":
                X[S, y:y + s, x:x + s] = mu[S, None, None] + np.sqrt(3.0) * (X[S, y:y + s, x:x + s] - mu[S, None, None])
            else:
                perm = S[torch.from_numpy(rng.permutation(ns)).to(device)]
                X[S, y:y + s, x:x + s] = X[perm, y:y + s, x:x + s].clone()
            mask[y:y + s, x:x + s] = 1
            info.append((kind, y, x, s))
    return X.contiguous(), mask, info


def workload_batch_torch(n: int = 64, C: int = 256, first_seed: int = 300, sides=None, device="cuda"):
    """The 64-image uneven batch generated on the device."""
    sides = sides if sides is not None else batch_sides(n)
    out = [make_texture_torch(C, s, s, first_seed + i, device,
                              anomalies=[("shift", 8, 32), ("scale", 8, 32), ("permute", 8, 32)])
           for i, s in enumerate(sides)]
    return out, dict(C=C, k=32, B=32, T=15, q_lo=0.01, q_hi=0.99, sigma_s=1.0)
