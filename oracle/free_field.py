"""Free-field (unit links) closed forms, NumPy FFT.

TEST INFRASTRUCTURE ONLY.

With U_mu(x) = 1 the staggered phases anticommute between directions, so the
cross terms of D^2 cancel and only the mu = nu terms survive:
  (D^2 chi)(x) = 1/4 sum_mu [chi(x + 2mu) - 2 chi(x) + chi(x - 2mu)],
which is diagonal on plane waves e^{i p.x}:
  (m^2 - D^2) e^{i p.x} c = (m^2 + sum_mu sin^2 p_mu) e^{i p.x} c,
with p_mu = 2 pi n / L_mu in the periodic directions and
p_t = 2 pi (n + 1/2) / L_t when t is antiperiodic.  This gives the exact
spectrum and an exact solver at any lattice size, independent of the
operator code.
"""

from __future__ import annotations

import numpy as np


def _momenta(dims, antiperiodic_t=True):
    L = [int(v) for v in dims]
    ps = []
    for mu in range(4):
        n = np.arange(L[mu], dtype=np.float64)
        shift = 0.5 if (mu == 3 and antiperiodic_t) else 0.0
        ps.append(2.0 * np.pi * (n + shift) / L[mu])
    return ps


def spectrum(dims, m, antiperiodic_t=True) -> np.ndarray:
    """All eigenvalues of m^2 - D^2 on the full lattice (3 colours each),
    sorted ascending."""
    px, py, pz, pt = _momenta(dims, antiperiodic_t)
    s = (np.sin(pt)[:, None, None, None] ** 2 + np.sin(pz)[None, :, None, None] ** 2
         + np.sin(py)[None, None, :, None] ** 2 + np.sin(px)[None, None, None, :] ** 2)
    ev = m * m + s.reshape(-1)
    return np.sort(np.repeat(ev, 3))


def solve(dims, m, b, antiperiodic_t=True) -> np.ndarray:
    """x = (m^2 - D^2)^{-1} b for unit links, exactly, via 4-d FFT.
    b, x: complex128 [V,3], sites lexicographic (x fastest)."""
    Lx, Ly, Lz, Lt = [int(v) for v in dims]
    f = np.asarray(b, dtype=np.complex128).reshape(Lt, Lz, Ly, Lx, 3)
    t = np.arange(Lt)
    twist = np.exp(1j * np.pi * t / Lt) if antiperiodic_t else np.ones(Lt)
    f = f * np.conj(twist)[:, None, None, None, None]
    fh = np.fft.fftn(f, axes=(0, 1, 2, 3))
    px, py, pz, pt = _momenta(dims, antiperiodic_t)
    den = (m * m + np.sin(pt)[:, None, None, None] ** 2 + np.sin(pz)[None, :, None, None] ** 2
           + np.sin(py)[None, None, :, None] ** 2 + np.sin(px)[None, None, None, :] ** 2)
    xh = fh / den[..., None]
    x = np.fft.ifftn(xh, axes=(0, 1, 2, 3)) * twist[:, None, None, None, None]
    return x.reshape(-1, 3)


def plane_wave(dims, n, colour_vec, antiperiodic_t=True) -> np.ndarray:
    """e^{i p.x} c for the integer momentum label n = (nx, ny, nz, nt);
    returns (vector [V,3], eigenvalue of -D^2)."""
    Lx, Ly, Lz, Lt = [int(v) for v in dims]
    px, py, pz, pt = _momenta(dims, antiperiodic_t)
    p = (px[n[0]], py[n[1]], pz[n[2]], pt[n[3]])
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    v = ph.reshape(-1)[:, None] * np.asarray(colour_vec, dtype=np.complex128)[None, :]
    lam = float(sum(np.sin(q) ** 2 for q in p))
    return v, lam
