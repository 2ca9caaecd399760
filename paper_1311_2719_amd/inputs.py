"""Seeded synthetic inputs: SU(3) gauge fields and Gaussian colour-vector sources.

This module produces host arrays only.  It holds none of the operator's or the
solver's arithmetic, so the same arrays can be handed both to the library and
to the CPU oracle.

Array conventions (shared by every consumer):
  links  complex128 [V, 4, 3, 3]   U_mu(x)[a, b], sites lexicographic
                                   s = x + Lx*(y + Ly*(z + Lz*t)), mu = x,y,z,t
  vector complex128 [V, 3]         one colour vector per site

All draws use numpy's PCG64 (`default_rng(seed)`) in the order sites, then mu,
then the entries of one 3x3 draw (row-major, real part before imaginary part).

The paper's production fields (thermalised N_f=2 staggered ensembles with the
Wilson gauge action, Sec. 6) are not given; these synthetic fields stand in
for them: Haar-random links are the roughest possible field, and
proj_SU3(exp(i eps H)) links are smooth fields whose roughness is set by eps.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "volume",
    "haar_su3",
    "smooth_su3",
    "unit_links",
    "gaussian_source",
    "gaussian_spinor",
    "proj_su3",
    "masses_uniform",
    "gaussian_momenta",
]


def volume(dims) -> int:
    d = [int(v) for v in dims]
    if len(d) != 4:
        raise ValueError("dims must have 4 entries (Lx, Ly, Lz, Lt)")
    return d[0] * d[1] * d[2] * d[3]


def _complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """Entries (N(0,1) + i N(0,1)) / sqrt(2)."""
    g = rng.standard_normal(tuple(shape) + (2,))
    return (g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0)


def haar_su3(dims, seed: int) -> np.ndarray:
    """Haar-random SU(3) links.

    QR of a complex Gaussian matrix, with the phases of R's diagonal moved
    into Q (Mezzadri, Notices AMS 54 (2007) 592) so Q is Haar on U(3); then
    Q is divided by the principal cube root of det Q, which leaves the
    distribution Haar on SU(3).
    """
    V = volume(dims)
    rng = np.random.default_rng(seed)
    Z = _complex_gaussian(rng, (V, 4, 3, 3))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    ph = d / np.abs(d)
    Q = Q * ph[..., None, :]
    det = np.linalg.det(Q)
    Q = Q / (det ** (1.0 / 3.0))[..., None, None]
    return np.ascontiguousarray(Q, dtype=np.complex128)


def proj_su3(M: np.ndarray) -> np.ndarray:
    """Project 3x3 matrices onto SU(3): Gram-Schmidt on rows 0 and 1, then
    row 2 = conj(row0 x row1)."""
    r0 = M[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = M[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.ascontiguousarray(np.stack([r0, r1, r2], axis=-2), dtype=np.complex128)


def smooth_su3(dims, eps: float, seed: int, chunk: int = 1 << 18) -> np.ndarray:
    """Links proj_SU3(exp(i eps H)), H random traceless Hermitian.

    H = (A + A^dagger)/2 - tr(...)/3 with A complex Gaussian; the exponential
    is taken through the eigen-decomposition of H, then projected to SU(3) to
    remove rounding.  Generated in chunks of sites to bound host memory.
    """
    V = volume(dims)
    rng = np.random.default_rng(seed)
    out = np.empty((V, 4, 3, 3), dtype=np.complex128)
    eye = np.eye(3)
    for s0 in range(0, V, chunk):
        n = min(chunk, V - s0)
        A = _complex_gaussian(rng, (n, 4, 3, 3))
        H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
        tr = np.trace(H, axis1=-2, axis2=-1)
        H = H - (tr / 3.0)[..., None, None] * eye
        w, Vv = np.linalg.eigh(H)
        E = (Vv * np.exp(1j * eps * w)[..., None, :]) @ np.conj(np.swapaxes(Vv, -1, -2))
        out[s0:s0 + n] = proj_su3(E)
    return out


def unit_links(dims) -> np.ndarray:
    """The free field: U_mu(x) = 1."""
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def gaussian_source(dims, seed: int) -> np.ndarray:
    """Colour-vector source with Re, Im ~ N(0,1) on every component."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((V, 3, 2))
    return np.ascontiguousarray(g[..., 0] + 1j * g[..., 1], dtype=np.complex128)


def gaussian_spinor(dims, seed: int) -> np.ndarray:
    """Spin-colour source [V, 4, 3] (Wilson fermions) with Re, Im ~ N(0,1)."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((V, 4, 3, 2))
    return np.ascontiguousarray(g[..., 0] + 1j * g[..., 1], dtype=np.complex128)


def masses_uniform(lo: float, hi: float, n: int) -> np.ndarray:
    """n masses evenly spread over [lo, hi], end points included."""
    return np.linspace(lo, hi, n)


def random_su3_gauge_transform(dims, seed: int) -> np.ndarray:
    """One Haar SU(3) matrix per site, complex128 [V, 3, 3]."""
    V = volume(dims)
    g = haar_su3((V, 1, 1, 1), seed)  # [V, 4, 3, 3]; use mu = 0
    return np.ascontiguousarray(g[:, 0])


def gaussian_momenta(dims, seed: int) -> np.ndarray:
    """Molecular-dynamics momenta [V, 4, 3, 3]: Q = i sum_a g_a T_a with
    g_a ~ N(0,1) (eight per link, drawn in the order sites, mu, a) and
    T_a = lambda_a / 2 the Gell-Mann generators, so Q is anti-Hermitian and
    traceless with <-tr Q^2> = 4 per link."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((V, 4, 8))
    s3 = 1.0 / np.sqrt(3.0)
    lam = np.array([
        [[0, 1, 0], [1, 0, 0], [0, 0, 0]],
        [[0, -1j, 0], [1j, 0, 0], [0, 0, 0]],
        [[1, 0, 0], [0, -1, 0], [0, 0, 0]],
        [[0, 0, 1], [0, 0, 0], [1, 0, 0]],
        [[0, 0, -1j], [0, 0, 0], [1j, 0, 0]],
        [[0, 0, 0], [0, 0, 1], [0, 1, 0]],
        [[0, 0, 0], [0, 0, -1j], [0, 1j, 0]],
        [[s3, 0, 0], [0, s3, 0], [0, 0, -2 * s3]],
    ], dtype=np.complex128)
    return np.ascontiguousarray(0.5j * np.einsum("...a,aij->...ij", g, lam), dtype=np.complex128)
