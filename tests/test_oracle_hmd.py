"""Pins of the fermion-force oracle (oracle/hmd.py) against facts fixed
outside its code: central finite differences of the pseudofermion action
S_F = phi^dagger (m^2 - D_eo D_oe)^{-1} phi (each value from a tight CG solve
of the oracle, itself pinned in test_oracle_cg.py), gauge covariance of the
force and gauge invariance of the action, and planted mistakes that the
finite-difference pin catches."""

import numpy as np
import pytest

from oracle import hmd
from paper_1311_2719_amd import inputs

T = hmd.su3_generators()


def pseudofermion(dims, seed):
    phi = inputs.gaussian_source(dims, seed)
    phi[hmd.parity(dims) == 1] = 0
    return phi


def fd_derivative(dims, U, m, phi, z, mu, a, w=1e-4):
    Up, Um = U.copy(), U.copy()
    Up[z, mu] = hmd.expi(w, T[a]) @ U[z, mu]
    Um[z, mu] = hmd.expi(-w, T[a]) @ U[z, mu]
    return (hmd.fermion_action(dims, Up, m, phi) - hmd.fermion_action(dims, Um, m, phi)) / (2 * w)


def links_to_check(dims, rng, n):
    """Random (site, mu, generator) triples plus the t-boundary links and one
    link of each parity in every direction."""
    V = int(np.prod(dims))
    par = hmd.parity(dims)
    t = np.arange(V) // (dims[0] * dims[1] * dims[2])
    out = [(int(rng.integers(V)), int(rng.integers(4)), int(rng.integers(8))) for _ in range(n)]
    edge = np.flatnonzero(t == dims[3] - 1)
    out += [(int(edge[0]), 3, 2), (int(edge[-1]), 3, 7)]
    for mu in range(4):
        for p in (0, 1):
            out.append((int(np.flatnonzero(par == p)[mu]), mu, (mu + p) % 8))
    return out


def check_against_fd(dims, U, m, phi, F, cases):
    worst = 0.0
    for z, mu, a in cases:
        fd = fd_derivative(dims, U, m, phi, z, mu, a)
        an = hmd.derivative_from_force(F[z, mu], T[a])
        worst = max(worst, abs(fd - an) / max(1.0, abs(an)))
    return worst


@pytest.mark.parametrize("dims,kind,m", [((4, 4, 4, 4), "haar", 0.3), ((4, 4, 4, 4), "smooth", 0.1),
                                         ((2, 4, 6, 8), "haar", 0.2)])
def test_force_matches_finite_differences(dims, kind, m):
    U = inputs.haar_su3(dims, 511) if kind == "haar" else inputs.smooth_su3(dims, 0.5, 512)
    phi = pseudofermion(dims, 513)
    F = hmd.fermion_force(dims, U, m, phi, tol=1e-13)
    # traceless anti-Hermitian
    assert np.max(np.abs(F + np.conj(np.swapaxes(F, -1, -2)))) < 1e-14
    assert np.max(np.abs(np.trace(F, axis1=-2, axis2=-1))) < 1e-13
    assert check_against_fd(dims, U, m, phi, F, links_to_check(dims, np.random.default_rng(514), 8)) < 1e-6


@pytest.mark.parametrize("mutation", ["no_parity_sign", "no_eta", "periodic_t", "swapped_outer",
                                      "right_multiplied"])
def test_planted_mistakes_fail_the_pin(mutation):
    dims, m = (4, 4, 4, 4), 0.3
    U = inputs.haar_su3(dims, 521)
    phi = pseudofermion(dims, 522)
    F = hmd.fermion_force(dims, U, m, phi, tol=1e-13, mutation=mutation)
    assert check_against_fd(dims, U, m, phi, F, links_to_check(dims, np.random.default_rng(523), 8)) > 1e-3


def test_gauge_covariance():
    # U_mu(z) -> g(z) U_mu(z) g(z+mu)^dagger, phi -> g phi: S_F is unchanged and
    # F_mu(z) -> g(z) F_mu(z) g(z)^dagger
    dims, m = (4, 4, 4, 6), 0.2
    U = inputs.smooth_su3(dims, 0.5, 531)
    phi = pseudofermion(dims, 532)
    g = inputs.random_su3_gauge_transform(dims, 533)
    Ug = np.empty_like(U)
    for mu in range(4):
        fwd = hmd.forward_site(dims, mu)
        Ug[:, mu] = g @ U[:, mu] @ np.conj(np.swapaxes(g[fwd], -1, -2))
    phig = np.einsum("sab,sb->sa", g, phi)
    assert abs(hmd.fermion_action(dims, Ug, m, phig) / hmd.fermion_action(dims, U, m, phi) - 1) < 1e-11
    F = hmd.fermion_force(dims, U, m, phi, tol=1e-13)
    Fg = hmd.fermion_force(dims, Ug, m, phig, tol=1e-13)
    want = g[:, None] @ F @ np.conj(np.swapaxes(g, -1, -2))[:, None]
    assert np.max(np.abs(Fg - want)) < 1e-9 * np.max(np.abs(F))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 8)])
def test_gauge_force_matches_finite_differences(dims):
    beta = 5.6
    U = inputs.haar_su3(dims, 551)
    F = hmd.gauge_force(dims, U, beta)
    worst = 0.0
    for z, mu, a in links_to_check(dims, np.random.default_rng(552), 8):
        # S_G ~ 6 beta V: the rounding of the difference quotient is ~1e-16 S_G / w
        w = 1e-4
        Up, Um = U.copy(), U.copy()
        Up[z, mu] = hmd.expi(w, T[a]) @ U[z, mu]
        Um[z, mu] = hmd.expi(-w, T[a]) @ U[z, mu]
        fd = (hmd.gauge_action(dims, Up, beta) - hmd.gauge_action(dims, Um, beta)) / (2 * w)
        an = hmd.derivative_from_force(F[z, mu], T[a])
        worst = max(worst, abs(fd - an) / max(1.0, abs(an)))
    assert worst < 1e-6


def test_gauge_action_closed_forms():
    dims = (4, 4, 4, 6)
    V = int(np.prod(dims))
    # unit links: every plaquette is the identity
    assert abs(hmd.gauge_action(dims, inputs.unit_links(dims), 6.0)) < 1e-12
    # a constant abelian field U_x = diag(e^{i a}, e^{-i a}, 1), others 1: every
    # plaquette is the identity again (the field is a pure gauge on a torus
    # only up to holonomy, but plaquettes of a constant field close)
    U = inputs.unit_links(dims)
    U[:, 0] = np.diag([np.exp(0.3j), np.exp(-0.3j), 1.0])
    assert abs(hmd.gauge_action(dims, U, 6.0)) < 1e-12
    # gauge invariance on a Haar field
    U = inputs.haar_su3(dims, 553)
    g = inputs.random_su3_gauge_transform(dims, 554)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[:, mu] = g @ U[:, mu] @ np.conj(np.swapaxes(g[hmd.forward_site(dims, mu)], -1, -2))
    s, sg = hmd.gauge_action(dims, U, 5.0), hmd.gauge_action(dims, Ug, 5.0)
    assert abs(sg / s - 1) < 1e-12
    # a Haar field has <Re tr P> = 0: S_G / (beta * 6 V) = 1 within a few percent
    assert abs(s / (5.0 * 6 * V) - 1) < 0.05


def test_leapfrog_second_order_and_reversible():
    dims, beta, m = (4, 4, 4, 4), 5.6, 0.3
    V = int(np.prod(dims))
    U = inputs.smooth_su3(dims, 0.3, 561)
    Q = hmd.momenta_from_gaussian(np.random.default_rng(562).standard_normal((V, 4, 8)))
    phi = hmd.pseudofermion_from_gaussian(dims, U, m, inputs.gaussian_source(dims, 563))
    H0 = hmd.hamiltonian(dims, U, Q, beta, m, phi)[0]
    dH = []
    for eps, n in ((0.05, 4), (0.025, 8), (0.0125, 16)):
        U1, Q1 = hmd.leapfrog(dims, U, Q, beta, m, phi, eps, n)
        dH.append(hmd.hamiltonian(dims, U1, Q1, beta, m, phi)[0] - H0)
        # still special unitary, momenta still traceless anti-Hermitian
        assert np.max(np.abs(U1 @ np.conj(np.swapaxes(U1, -1, -2)) - np.eye(3))) < 1e-13
        assert np.max(np.abs(Q1 + np.conj(np.swapaxes(Q1, -1, -2)))) < 1e-12
    # |dH| falls as eps^2 at fixed trajectory length
    assert 3.5 < dH[0] / dH[1] < 4.5 and 3.5 < dH[1] / dH[2] < 4.5
    # reversibility: flip the momenta and integrate back
    U1, Q1 = hmd.leapfrog(dims, U, Q, beta, m, phi, 0.05, 4)
    U2, Q2 = hmd.leapfrog(dims, U1, -Q1, beta, m, phi, 0.05, 4)
    assert np.max(np.abs(U2 - U)) < 1e-12 and np.max(np.abs(Q2 + Q)) < 1e-11


def test_heatbath_moments():
    # momenta: -tr Q^2 = (1/2) sum_a g_a^2, mean 4 per link; pseudofermions:
    # <phi phi^dagger> = 2 (m^2 - D_eo D_oe) for Re, Im ~ N(0,1), so
    # <S_F> = 2 x (number of even-site colour components)
    dims, m = (4, 4, 4, 4), 0.3
    V = int(np.prod(dims))
    Q = hmd.momenta_from_gaussian(np.random.default_rng(571).standard_normal((V, 4, 8)))
    assert abs(hmd.kinetic_energy(Q) / (4 * V * 4) - 1) < 0.05
    U = inputs.haar_su3(dims, 572)
    sf = [hmd.fermion_action(dims, U, m, hmd.pseudofermion_from_gaussian(dims, U, m, inputs.gaussian_source(dims, s)))
          for s in range(573, 581)]
    assert abs(np.mean(sf) / (2 * 3 * V // 2) - 1) < 0.05
