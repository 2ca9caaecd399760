"""Pins of the Wilson-fermion oracle against facts fixed by the mathematics.

The paper runs an N_f = 2 Wilson-fermion program (Sec. 2, Sec. 6) without writing the
operator out; the oracle takes the textbook M = 1 - kappa H (see
oracle/wilson_oracle.c).  None of these checks re-calls the oracle's own
routine as its reference:
  * the gamma matrices obey the Euclidean Clifford algebra, are Hermitian,
    gamma_5 = diag(1, 1, -1, -1), and the oracle's copy equals the dense
    builder's independently typed copy;
  * free field: a plane wave e^{ipx} chi (antiperiodic momenta in t) is
    mapped to e^{ipx} sum_mu [2 cos p_mu - 2i gamma_mu sin p_mu] chi;
  * the spectrum of M^dagger M on the free 4^4 lattice is the closed form
    (1 - 2 kappa sum cos p)^2 + 4 kappa^2 sum sin^2 p, 12-fold per momentum;
  * gamma_5 H is Hermitian; H is gauge covariant;
  * brute force: an independently written dense builder on three shapes,
    and dense LU for the solve;
  * planted mistakes in the dense builder each fail the comparison.
"""

import itertools

import numpy as np
import pytest

import oracle
from oracle import dense
from paper_1311_2719_amd import inputs


def test_gamma_basis():
    g = [oracle.wilson_gamma(mu) for mu in range(4)]
    for a in range(4):
        assert np.array_equal(g[a], dense.WILSON_GAMMA[a])
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2.0 * (a == b) * np.eye(4))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))


def momenta(dims, antiperiodic_t=True):
    out = []
    for n in itertools.product(*[range(L) for L in dims]):
        p = [2 * np.pi * n[mu] / dims[mu] for mu in range(3)]
        p.append((2 * n[3] + (1 if antiperiodic_t else 0)) * np.pi / dims[3])
        out.append(np.array(p))
    return out


def lex_coords(dims):
    V = int(np.prod(dims))
    s = np.arange(V)
    return np.stack([s % dims[0], (s // dims[0]) % dims[1], (s // (dims[0] * dims[1])) % dims[2],
                     s // (dims[0] * dims[1] * dims[2])], axis=1)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 8)])
def test_free_plane_wave(dims):
    U = inputs.unit_links(dims)
    x = lex_coords(dims)
    rng = np.random.default_rng(3)
    g = dense.WILSON_GAMMA
    for p in momenta(dims)[::7][:12]:
        chi = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
        phase = np.exp(1j * (x @ p))
        psi = phase[:, None, None] * chi[None]
        Hp = sum(2 * np.cos(p[mu]) * np.eye(4) - 2j * np.sin(p[mu]) * g[mu] for mu in range(4))
        want = phase[:, None, None] * (Hp @ chi)[None]
        got = oracle.wilson_hop(dims, U, psi)
        assert np.abs(got - want).max() < 1e-12


def test_free_spectrum_closed_form():
    dims, kappa = (4, 4, 4, 4), 0.11
    U = inputs.unit_links(dims)
    H = dense.dense_wilson_hop(dims, U)
    M = np.eye(H.shape[0]) - kappa * H
    ev = np.sort(np.linalg.eigvalsh(M.conj().T @ M))
    want = []
    for p in momenta(dims):
        a = 1 - 2 * kappa * np.sum(np.cos(p))
        want += [a * a + 4 * kappa * kappa * np.sum(np.sin(p) ** 2)] * 12
    assert np.allclose(ev, np.sort(want), atol=1e-12)


def test_gamma5_hermiticity():
    dims = (4, 4, 2, 6)
    U = inputs.haar_su3(dims, 21)
    rng = np.random.default_rng(4)
    V = int(np.prod(dims))
    phi = rng.normal(size=(V, 4, 3)) + 1j * rng.normal(size=(V, 4, 3))
    psi = rng.normal(size=(V, 4, 3)) + 1j * rng.normal(size=(V, 4, 3))
    g5 = np.array([1, 1, -1, -1])[None, :, None]
    lhs = np.vdot(phi, g5 * oracle.wilson_hop(dims, U, psi))
    rhs = np.conj(np.vdot(psi, g5 * oracle.wilson_hop(dims, U, phi)))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_gauge_covariance():
    dims = (4, 2, 4, 4)
    V = int(np.prod(dims))
    U = inputs.haar_su3(dims, 31)
    g = inputs.random_su3_gauge_transform(dims, 32)
    x = lex_coords(dims)
    Ug = np.empty_like(U)
    for mu in range(4):
        xn = x.copy()
        xn[:, mu] = (xn[:, mu] + 1) % dims[mu]
        sn = xn[:, 0] + dims[0] * (xn[:, 1] + dims[1] * (xn[:, 2] + dims[2] * xn[:, 3]))
        Ug[:, mu] = g @ U[:, mu] @ np.conj(np.transpose(g[sn], (0, 2, 1)))
    rng = np.random.default_rng(5)
    psi = rng.normal(size=(V, 4, 3)) + 1j * rng.normal(size=(V, 4, 3))
    gpsi = np.einsum("sab,sib->sia", g, psi)
    lhs = oracle.wilson_hop(dims, Ug, gpsi)
    rhs = np.einsum("sab,sib->sia", g, oracle.wilson_hop(dims, U, psi))
    assert np.abs(lhs - rhs).max() < 1e-12


@pytest.mark.parametrize("dims,periodic", [((2, 2, 2, 2), False), ((2, 2, 2, 4), False), ((4, 2, 2, 2), True)])
def test_dense_brute_force(dims, periodic):
    V = int(np.prod(dims))
    U = inputs.haar_su3(dims, 41)
    rng = np.random.default_rng(6)
    psi = rng.normal(size=(V, 4, 3)) + 1j * rng.normal(size=(V, 4, 3))
    H = dense.dense_wilson_hop(dims, U, antiperiodic_t=not periodic)
    want = (H @ psi.reshape(-1)).reshape(V, 4, 3)
    assert np.abs(oracle.wilson_hop(dims, U, psi, antiperiodic_t=not periodic) - want).max() < 1e-12
    # one parity only: the other sites of `out` are left as they were
    for par in (0, 1):
        sel = dense.wilson_parity_of_rows(dims).reshape(V, 4, 3)[:, 0, 0] == par
        out = np.full((V, 4, 3), 7.0 + 0j)
        oracle.wilson_hop(dims, U, psi, out_parity=par, antiperiodic_t=not periodic, out=out)
        assert np.abs(out[sel] - want[sel]).max() < 1e-12
        assert np.all(out[~sel] == 7.0)
    kappa = 0.137
    M = np.eye(12 * V) - kappa * H
    got = oracle.wilson_apply(dims, U, kappa, psi, antiperiodic_t=not periodic)
    assert np.abs(got - (M @ psi.reshape(-1)).reshape(V, 4, 3)).max() < 1e-12


@pytest.mark.parametrize("mutation", dense.WILSON_MUTATIONS)
def test_planted_mistakes_fail(mutation):
    dims = (2, 2, 2, 4)
    V = int(np.prod(dims))
    U = inputs.haar_su3(dims, 51)
    rng = np.random.default_rng(7)
    psi = rng.normal(size=(V, 4, 3)) + 1j * rng.normal(size=(V, 4, 3))
    Hm = dense.dense_wilson_hop(dims, U, mutation=mutation)
    assert np.abs((Hm @ psi.reshape(-1)).reshape(V, 4, 3) - oracle.wilson_hop(dims, U, psi)).max() > 1e-3


@pytest.mark.parametrize("dims,kappa", [((2, 2, 2, 4), 0.12), ((4, 2, 2, 2), 0.15)])
def test_even_odd_cg_against_dense_lu(dims, kappa):
    V = int(np.prod(dims))
    U = inputs.haar_su3(dims, 61)
    rng = np.random.default_rng(8)
    b = rng.normal(size=(V, 4, 3)) + 1j * rng.normal(size=(V, 4, 3))
    x, info = oracle.wilson_cg(dims, U, kappa, b, tol=1e-12)
    assert info["status"] == 0 and info["true_rel"] < 1e-10
    M = np.eye(12 * V) - kappa * dense.dense_wilson_hop(dims, U)
    xs = np.linalg.solve(M, b.reshape(-1)).reshape(V, 4, 3)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-10


def test_even_odd_cg_free_field_closed_form():
    # free field: M is diagonal in momentum space, so x = sum_p M(p)^{-1} b(p) e^{ipx}
    dims, kappa = (4, 4, 4, 4), 0.12
    V = int(np.prod(dims))
    U = inputs.unit_links(dims)
    x = lex_coords(dims)
    rng = np.random.default_rng(9)
    g = dense.WILSON_GAMMA
    ps = momenta(dims)[::11][:5]
    b = np.zeros((V, 4, 3), np.complex128)
    xs = np.zeros_like(b)
    for p in ps:
        chi = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
        phase = np.exp(1j * (x @ p))[:, None, None]
        Mp = np.eye(4) - kappa * sum(2 * np.cos(p[mu]) * np.eye(4) - 2j * np.sin(p[mu]) * g[mu] for mu in range(4))
        b += phase * chi[None]
        xs += phase * np.linalg.solve(Mp, chi)[None]
    xo, info = oracle.wilson_cg(dims, U, kappa, b, tol=1e-12)
    assert info["status"] == 0
    assert np.linalg.norm(xo - xs) / np.linalg.norm(xs) < 1e-10


def test_cg_edge_cases():
    dims = (2, 2, 2, 2)
    U = inputs.haar_su3(dims, 71)
    x, info = oracle.wilson_cg(dims, U, 0.1, np.zeros((16, 4, 3), np.complex128))
    assert info["status"] == 0 and info["iters"] == 0 and not np.any(x)
    rng = np.random.default_rng(10)
    b = rng.normal(size=(16, 4, 3)) + 0j
    x, info = oracle.wilson_cg(dims, U, 0.1, b, tol=1e-12, maxiter=2)
    assert info["status"] == -6 and info["iters"] == 2
