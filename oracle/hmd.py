"""Oracle for the molecular-dynamics force of the staggered pseudofermion
action (TEST INFRASTRUCTURE ONLY; the library never loads it).

The paper's application (Sec. 2 and Sec. 6) is an N_f = 2 staggered-fermion
Hybrid Molecular Dynamics program whose CG (Sec. 4) returns the solution x on
one half of the lattice and y = D x on the other.  It does not write the
action or the force out; the reading taken here is the textbook one for the
even-site normal operator the CG solves:

  S_F(U) = phi^dagger A^{-1} phi,  A = m^2 - D_eo D_oe  (phi on even sites),

so with X = A^{-1} phi (even) and Y = D_oe X (odd), the full-lattice field
W = X + Y is what the CG returns.  Varying one link U_mu(z) (D as in
stag_oracle.c, with the staggered phase eta_mu and the t-boundary sign b_mu
of the hop from z to z + mu):

  dS_F = sum_{z,mu} 2 Re tr[ dU_mu(z) M_mu(z) ],
  M_mu(z) = eps(z) c_mu(z) W(z + mu) W(z)^dagger,
  c_mu(z) = eta_mu(z) b_mu(z) / 2,  eps(z) = +1 on even, -1 on odd sites.

(From dS_F = -X^dagger dA X = X^dagger dD_eo Y - Y^dagger dD_oe X, using
D_eo = -D_oe^dagger; a link from an even z enters through X(z) and
Y(z + mu), a link from an odd z through Y(z) and X(z + mu) with the opposite
sign.)  For the left-multiplied variation U -> exp(i w T) U with T Hermitian
and traceless, dS_F / dw = 2 Re tr[ i T F ] with F the traceless
anti-Hermitian part of U_mu(z) M_mu(z):

  F_mu(z) = TA[ U_mu(z) M_mu(z) ],  TA(Z) = (Z - Z^dagger)/2 - tr(Z - Z^dagger)/6.

Pinned in tests/test_oracle_hmd.py by central finite differences of S_F
computed from tight CG solves, on Haar and smooth 4^4 fields and on a
2 x 4 x 6 x 8 lattice, by gauge covariance, and by planted mistakes.
"""

from __future__ import annotations

import numpy as np

import oracle


def _coords(dims):
    """x, y, z, t coordinates of every lexicographic site, each [V]."""
    Lx, Ly, Lz, Lt = dims
    s = np.arange(Lx * Ly * Lz * Lt)
    return s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)


def parity(dims):
    x, y, z, t = _coords(dims)
    return (x + y + z + t) & 1


def forward_site(dims, mu):
    """Lexicographic index of z + mu (periodic) for every site z."""
    Lx, Ly, Lz, Lt = dims
    c = list(_coords(dims))
    L = (Lx, Ly, Lz, Lt)
    c[mu] = (c[mu] + 1) % L[mu]
    return c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3]))


def hop_coefficient(dims, mu, antiperiodic_t=True):
    """c_mu(z) = eta_mu(z) b_mu(z) / 2 for every site z: eta_mu(z) =
    (-1)^(x_0 + ... + x_{mu-1}); b_mu(z) = -1 for the hop from the last t
    slice forward across the boundary of an antiperiodic field."""
    x = _coords(dims)
    esum = np.zeros_like(x[0])
    for nu in range(mu):
        esum = esum + x[nu]
    c = np.where(esum % 2 == 0, 0.5, -0.5)
    if mu == 3 and antiperiodic_t:
        c = np.where(x[3] == dims[3] - 1, -c, c)
    return c


def traceless_antihermitian(Z):
    """TA(Z) = (Z - Z^dagger)/2 - tr(Z - Z^dagger)/6 * 1 over the last two axes."""
    A = 0.5 * (Z - np.conj(np.swapaxes(Z, -1, -2)))
    tr = np.trace(A, axis1=-2, axis2=-1)
    return A - (tr / 3.0)[..., None, None] * np.eye(3)


def force_from_field(dims, U, W, antiperiodic_t=True, mutation=None):
    """F_mu(z) = TA[U_mu(z) eps(z) c_mu(z) W(z + mu) W(z)^dagger], complex128
    [V, 4, 3, 3]: the derivative of S_F for the full-lattice field W (the
    solution on the even sites and D_oe of it on the odd sites).
    `mutation` plants a mistake for the tests that show the pins catch it."""
    V = int(np.prod(dims))
    U = np.asarray(U, dtype=np.complex128).reshape(V, 4, 3, 3)
    W = np.asarray(W, dtype=np.complex128).reshape(V, 3)
    eps = np.where(parity(dims) == 0, 1.0, -1.0)
    if mutation == "no_parity_sign":
        eps = np.ones(V)
    F = np.zeros((V, 4, 3, 3), np.complex128)
    for mu in range(4):
        fwd = forward_site(dims, mu)
        coef = eps * hop_coefficient(dims, mu, antiperiodic_t and mutation != "periodic_t")
        if mutation == "no_eta":
            coef = eps * 0.5
        a, b = (W, W[fwd]) if mutation == "swapped_outer" else (W[fwd], W)
        M = coef[:, None, None] * (a[:, :, None] * np.conj(b)[:, None, :])  # W(z+mu) W(z)^dagger
        Z = M @ U[:, mu] if mutation == "right_multiplied" else U[:, mu] @ M
        F[:, mu] = traceless_antihermitian(Z)
    return F


def solve_field(dims, U, m, phi, tol=1e-12, antiperiodic_t=True):
    """W = X + D_oe X with X = A^{-1} phi on the even sites (phi zero on odd
    sites), by the oracle's CG of the Sec. 4 loop; also returns X."""
    X, Y, info = oracle.cg_solve(dims, U, m, phi, tol=tol, parity=oracle.EVEN, want_y=True,
                                 antiperiodic_t=antiperiodic_t)
    if info["status"] != 0:
        raise RuntimeError("oracle CG did not converge: %s" % info)
    odd = parity(dims) == 1
    W = np.where(odd[:, None], Y, X)
    return W, X


def fermion_action(dims, U, m, phi, tol=1e-13, antiperiodic_t=True):
    """S_F = phi^dagger A^{-1} phi (real) for phi on the even sites."""
    _, X = solve_field(dims, U, m, phi, tol=tol, antiperiodic_t=antiperiodic_t)
    even = parity(dims) == 0
    return float(np.real(np.vdot(phi[even], X[even])))


def fermion_force(dims, U, m, phi, tol=1e-12, antiperiodic_t=True, mutation=None):
    """The force of S_F at U for the pseudofermion phi (even sites)."""
    W, _ = solve_field(dims, U, m, phi, tol=tol, antiperiodic_t=antiperiodic_t)
    return force_from_field(dims, U, W, antiperiodic_t, mutation)


def su3_generators():
    """T^a = lambda^a / 2 (Gell-Mann matrices): Hermitian, traceless,
    tr(T^a T^b) = delta^ab / 2.  [8, 3, 3]."""
    l = np.zeros((8, 3, 3), np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l / 2


def expi(w, T):
    """exp(i w T) for Hermitian T, by eigendecomposition."""
    ev, Q = np.linalg.eigh(T)
    return (Q * np.exp(1j * w * ev)) @ np.conj(Q.T)


def derivative_from_force(F, T):
    """dS/dw = 2 Re tr[i T F] for the variation U -> exp(i w T) U."""
    return 2.0 * np.real(np.trace(1j * T @ F))


# ---- the gauge action, momenta and the molecular-dynamics trajectory -----------------
#
# Readings (the paper names the Wilson gauge action and Hybrid Molecular
# Dynamics but gives neither the normalisation nor the integrator):
#   S_G = beta sum_{x, mu < nu} (1 - Re tr P_munu(x) / 3),
#   P_munu(x) = U_mu(x) U_nu(x + mu) U_mu(x + nu)^dagger U_nu(x)^dagger,
#   periodic in every direction (the antiperiodic t is a fermion boundary);
#   momenta Q_mu(x) anti-Hermitian and traceless, H = -sum tr(Q^2) + S_G + S_F;
#   equations of motion dU/dt = Q U, dQ/dt = F_G + F_F with the forces in the
#   convention above (dS/dw = 2 Re tr[i T F] for U -> exp(i w T) U), so H is
#   conserved;
#   leapfrog: Q += eps/2 F; then n times { U = exp(eps Q) U (each new link
#   projected back onto SU(3)); Q += eps F } with the last momentum step eps/2;
#   pseudofermion phi = m chi_e - (D chi)_e on the even sites from a Gaussian
#   chi on every site, so <phi phi^dagger> = m^2 - D_eo D_oe.


def _dagger(A):
    return np.conj(np.swapaxes(A, -1, -2))


def plaquette_field(dims, U, mu, nu):
    """P_munu(x) for every site, [V, 3, 3]."""
    fm, fn = forward_site(dims, mu), forward_site(dims, nu)
    return U[:, mu] @ U[fm, nu] @ _dagger(U[fn, mu]) @ _dagger(U[:, nu])


def gauge_action(dims, U, beta):
    """S_G = beta sum_{x, mu<nu} (1 - Re tr P_munu(x) / 3)."""
    U = np.asarray(U, dtype=np.complex128)
    s = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            s += np.sum(1.0 - np.real(np.trace(plaquette_field(dims, U, mu, nu), axis1=-2, axis2=-1)) / 3.0)
    return float(beta * s)


def backward_site(dims, mu):
    """Lexicographic index of z - mu (periodic) for every site z."""
    Lx, Ly, Lz, Lt = dims
    c = list(_coords(dims))
    L = (Lx, Ly, Lz, Lt)
    c[mu] = (c[mu] - 1) % L[mu]
    return c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3]))


def staple_sum(dims, U, mu):
    """Sigma_mu(x) = sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^dagger U_nu(x)^dagger
    + U_nu(x+mu-nu)^dagger U_mu(x-nu)^dagger U_nu(x-nu)], so that the plaquettes
    holding U_mu(x) sum to Re tr[U_mu(x) Sigma_mu(x)]."""
    fm = forward_site(dims, mu)
    S = np.zeros((U.shape[0], 3, 3), np.complex128)
    for nu in range(4):
        if nu == mu:
            continue
        fn, bn = forward_site(dims, nu), backward_site(dims, nu)
        fm_bn = backward_site(dims, nu)[fm]  # x + mu - nu
        S += U[fm, nu] @ _dagger(U[fn, mu]) @ _dagger(U[:, nu])
        S += _dagger(U[fm_bn, nu]) @ _dagger(U[bn, mu]) @ U[bn, nu]
    return S


def gauge_force(dims, U, beta):
    """F_G = -(beta / 6) TA[U_mu(x) Sigma_mu(x)], [V, 4, 3, 3]."""
    U = np.asarray(U, dtype=np.complex128)
    F = np.zeros_like(U)
    for mu in range(4):
        F[:, mu] = -(beta / 6.0) * traceless_antihermitian(U[:, mu] @ staple_sum(dims, U, mu))
    return F


def kinetic_energy(Q):
    """-sum tr(Q^2) over all links (real, >= 0 for anti-Hermitian Q)."""
    return float(-np.real(np.sum(np.einsum("...ab,...ba->...", Q, Q))))


def expm_antihermitian(A):
    """exp(A) for anti-Hermitian A (...x3x3), through the eigenvectors of -iA."""
    lam, Vv = np.linalg.eigh(-1j * A)
    return (Vv * np.exp(1j * lam)[..., None, :]) @ _dagger(Vv)


def reunitarize(U):
    """Project onto SU(3): Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1)."""
    r0 = U[..., 0, :] / np.linalg.norm(U[..., 0, :], axis=-1, keepdims=True)
    r1 = U[..., 1, :] - np.sum(np.conj(r0) * U[..., 1, :], axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    return np.stack([r0, r1, np.conj(np.cross(r0, r1))], axis=-2)


def momenta_from_gaussian(g):
    """Q = sum_a i g^a T^a from real Gaussians g [..., 8]: the momentum
    heatbath, <-tr Q^2> = 4 per link."""
    T = su3_generators()
    return 1j * np.einsum("...a,aij->...ij", g, T)


def pseudofermion_from_gaussian(dims, U, m, chi, antiperiodic_t=True):
    """phi = m chi - D chi on the even sites, zero on the odd sites."""
    Dchi = oracle.dslash(dims, U, chi, antiperiodic_t=antiperiodic_t)
    phi = m * np.asarray(chi) - Dchi
    phi[parity(dims) == 1] = 0
    return phi


def hamiltonian(dims, U, Q, beta, m, phi, tol=1e-12, antiperiodic_t=True):
    """(H, kinetic, S_G, S_F)."""
    k = kinetic_energy(Q)
    sg = gauge_action(dims, U, beta)
    sf = fermion_action(dims, U, m, phi, tol=tol, antiperiodic_t=antiperiodic_t)
    return k + sg + sf, k, sg, sf


def total_force(dims, U, beta, m, phi, tol=1e-12, antiperiodic_t=True):
    return gauge_force(dims, U, beta) + fermion_force(dims, U, m, phi, tol=tol, antiperiodic_t=antiperiodic_t)


def leapfrog(dims, U, Q, beta, m, phi, eps, nsteps, tol=1e-12, antiperiodic_t=True):
    """The leapfrog trajectory of the reading above; returns (U, Q)."""
    U = np.array(U, dtype=np.complex128)
    Q = np.array(Q, dtype=np.complex128)
    Q = Q + 0.5 * eps * total_force(dims, U, beta, m, phi, tol, antiperiodic_t)
    for k in range(nsteps):
        U = reunitarize(expm_antihermitian(eps * Q) @ U)
        w = eps if k < nsteps - 1 else 0.5 * eps
        Q = Q + w * total_force(dims, U, beta, m, phi, tol, antiperiodic_t)
    return U, Q
