"""Dense-matrix brute force for tiny lattices (NumPy only).

TEST INFRASTRUCTURE ONLY.  Builds the staggered operator D of the paper's
Sec. 3 matrix-vector routine as an explicit (3V x 3V) complex matrix, one
3x3 block per hop, so that small problems can be solved directly (LU via
numpy.linalg.solve) and diagonalised (eigvalsh).  Written independently of
stag_oracle.c: coordinates come from numpy.unravel_index and blocks are
placed one hop at a time.

Convention (shared with the rest of the oracle, by definition of the
operator): (D chi)(x) = 1/2 sum_mu eta_mu(x) [U_mu(x) chi(x+mu)
- U_mu(x-mu)^dagger chi(x-mu)], eta_mu(x) = (-1)^(x_0+...+x_{mu-1}),
antiperiodic in t when requested, sites lexicographic with x fastest.

`mutation` exists only so a test can plant a plausible mistake in this
builder and show that the pins catch it; production callers leave it None.
"""

from __future__ import annotations

import numpy as np

MUTATIONS = (
    "drop_direction",      # leave out the z hops
    "backward_sign",       # + instead of - on the backward hop
    "eta_order",           # eta_mu from the coordinates after mu
    "transpose_link",      # U^T instead of U on the forward hop
    "no_dagger",           # U instead of U^dagger on the backward hop
    "periodic_t",          # forget the antiperiodic sign
    "no_half",             # drop the factor 1/2
    "wrong_backward_link", # U_mu(x)^dagger instead of U_mu(x-mu)^dagger
)


def _lex(c, L):
    return int(np.ravel_multi_index(tuple(int(v) for v in c[::-1]), tuple(int(v) for v in L[::-1])))


def _coords(s, L):
    # lexicographic with x fastest: unravel over (Lt, Lz, Ly, Lx)
    t, z, y, x = np.unravel_index(int(s), tuple(int(v) for v in L[::-1]))
    return np.array([x, y, z, t])


def dense_dslash(dims, U, antiperiodic_t=True, mutation=None) -> np.ndarray:
    """D as a dense complex matrix, row/column index 3*site + colour."""
    if mutation is not None and mutation not in MUTATIONS:
        raise ValueError("unknown mutation %r" % mutation)
    L = np.asarray(dims, dtype=np.int64)
    V = int(np.prod(L))
    U = np.asarray(U).reshape(V, 4, 3, 3)
    D = np.zeros((3 * V, 3 * V), dtype=np.complex128)
    half = 1.0 if mutation == "no_half" else 0.5
    for s in range(V):
        c = _coords(s, L)
        for mu in range(4):
            if mutation == "drop_direction" and mu == 2:
                continue
            if mutation == "eta_order":
                eta = (-1.0) ** int(np.sum(c[mu + 1:]))
            else:
                eta = (-1.0) ** int(np.sum(c[:mu]))
            # forward neighbour
            cf = c.copy()
            cf[mu] = (c[mu] + 1) % L[mu]
            sf = _lex(cf, L)
            sgn_f = -1.0 if (antiperiodic_t and mutation != "periodic_t" and mu == 3 and c[3] == L[3] - 1) else 1.0
            Uf = U[s, mu].T if mutation == "transpose_link" else U[s, mu]
            D[3 * s:3 * s + 3, 3 * sf:3 * sf + 3] += half * eta * sgn_f * Uf
            # backward neighbour
            cb = c.copy()
            cb[mu] = (c[mu] - 1) % L[mu]
            sb = _lex(cb, L)
            sgn_b = -1.0 if (antiperiodic_t and mutation != "periodic_t" and mu == 3 and c[3] == 0) else 1.0
            if mutation == "wrong_backward_link":
                Ub = U[s, mu].conj().T
            elif mutation == "no_dagger":
                Ub = U[sb, mu]
            else:
                Ub = U[sb, mu].conj().T
            bsign = +1.0 if mutation == "backward_sign" else -1.0
            D[3 * s:3 * s + 3, 3 * sb:3 * sb + 3] += bsign * half * eta * sgn_b * Ub
    return D


def parity_mask(dims) -> np.ndarray:
    """Boolean [V]: True on odd sites (x+y+z+t odd)."""
    L = np.asarray(dims, dtype=np.int64)
    V = int(np.prod(L))
    par = np.zeros(V, dtype=bool)
    for s in range(V):
        par[s] = bool(np.sum(_coords(s, L)) & 1)
    return par


def dense_normal(D: np.ndarray, m: float) -> np.ndarray:
    """A = m^2 - D^2 as a dense matrix."""
    n = D.shape[0]
    return m * m * np.eye(n, dtype=np.complex128) - D @ D


def lu_solve(dims, U, m, b, antiperiodic_t=True) -> np.ndarray:
    """x = (m^2 - D^2)^{-1} b by LU (numpy.linalg.solve); b, x [V,3]."""
    D = dense_normal(dense_dslash(dims, U, antiperiodic_t), m)
    x = np.linalg.solve(D, np.asarray(b, dtype=np.complex128).reshape(-1))
    return x.reshape(-1, 3)


# ---- Wilson fermions -----------------------------------------------------------------------------
#
# (H psi)(x) = sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu)],
# M = 1 - kappa H, spinor index 12*site + 3*spin + colour.  The gamma matrices of the chiral basis are
# typed here a second time, independently of wilson_oracle.c (a test checks the two agree and obey the
# Clifford algebra).

WILSON_GAMMA = (
    np.array([[0, 0, 0, 1j], [0, 0, 1j, 0], [0, -1j, 0, 0], [-1j, 0, 0, 0]]),
    np.array([[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]], dtype=np.complex128),
    np.array([[0, 0, 1j, 0], [0, 0, 0, -1j], [-1j, 0, 0, 0], [0, 1j, 0, 0]]),
    np.array([[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]], dtype=np.complex128),
)

WILSON_MUTATIONS = (
    "projector_sign",      # (1 + gamma) on the forward hop and (1 - gamma) on the backward one
    "no_dagger",           # U instead of U^dagger on the backward hop
    "periodic_t",          # forget the antiperiodic sign
    "drop_direction",      # leave out the y hops
    "gamma_transpose",     # gamma^T instead of gamma
    "wrong_backward_link", # U_mu(x)^dagger instead of U_mu(x-mu)^dagger
)


def dense_wilson_hop(dims, U, antiperiodic_t=True, mutation=None) -> np.ndarray:
    """The Wilson hopping term H as a dense (12V x 12V) complex matrix."""
    if mutation is not None and mutation not in WILSON_MUTATIONS:
        raise ValueError("unknown mutation %r" % mutation)
    L = np.asarray(dims, dtype=np.int64)
    V = int(np.prod(L))
    U = np.asarray(U).reshape(V, 4, 3, 3)
    H = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    one = np.eye(4)
    for s in range(V):
        c = _coords(s, L)
        for mu in range(4):
            if mutation == "drop_direction" and mu == 1:
                continue
            g = WILSON_GAMMA[mu].T if mutation == "gamma_transpose" else WILSON_GAMMA[mu]
            pf, pb = (one + g, one - g) if mutation == "projector_sign" else (one - g, one + g)
            cf = c.copy()
            cf[mu] = (c[mu] + 1) % L[mu]
            sf = _lex(cf, L)
            sgn_f = -1.0 if (antiperiodic_t and mutation != "periodic_t" and mu == 3 and c[3] == L[3] - 1) else 1.0
            H[12 * s:12 * s + 12, 12 * sf:12 * sf + 12] += sgn_f * np.kron(pf, U[s, mu])
            cb = c.copy()
            cb[mu] = (c[mu] - 1) % L[mu]
            sb = _lex(cb, L)
            sgn_b = -1.0 if (antiperiodic_t and mutation != "periodic_t" and mu == 3 and c[3] == 0) else 1.0
            if mutation == "wrong_backward_link":
                Ub = U[s, mu].conj().T
            elif mutation == "no_dagger":
                Ub = U[sb, mu]
            else:
                Ub = U[sb, mu].conj().T
            H[12 * s:12 * s + 12, 12 * sb:12 * sb + 12] += sgn_b * np.kron(pb, Ub)
    return H


def wilson_parity_of_rows(dims) -> np.ndarray:
    """Parity (0 even, 1 odd) of each row/column index of the dense Wilson matrices."""
    L = np.asarray(dims, dtype=np.int64)
    V = int(np.prod(L))
    par = np.array([int(np.sum(_coords(s, L))) & 1 for s in range(V)])
    return np.repeat(par, 12)
