"""The FP64 CG parity contract, per parity system.

The oracle (O3) runs the paper's even-odd loop (Sec. 4) with the same
stopping rule from x = 0.  For each parity system:
  * the iteration counts of the GPU and the oracle agree within 1, and then
    the solutions agree to 1e-10 relative over that parity's sites;
  * otherwise both sides' k-th iterates, k the smaller count, are compared at
    1e-10 (the GPU's through a rerun of the same path with maxiter = k, the
    oracle's from one pass with tol = 0 and maxiter = k).
In floating point, CG's iteration count depends on the rounding order of its
inner products (the GPU's block and lane trees against the oracle's
sequential sums), so on an ill-conditioned system the counts may differ by
more than one; every comparison is printed as a COUNTS line so that the
observed differences can be collected.
"""

import numpy as np

import oracle
from oracle import dense

TOL_X = 1e-10


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def parity_sites(dims, par):
    odd = dense.parity_mask(dims)
    return odd if par == 1 else ~odd


def fp64_contract(dims, U, m, b, x_gpu, iters_parity, rerun=None, tol=1e-10, parities=(0, 1), label="",
                  oracle_runs=None):
    """Check x_gpu (lexicographic [V,3]) against O3 per parity system.
    iters_parity[p]: the GPU's iteration count of parity system p.  rerun(p,
    k) returns the GPU path's k-th iterate of system p (lexicographic).
    oracle_runs[p] = (x, iters), if given, is O3's solve of parity p (run by
    the caller); otherwise it is run here.  Returns [(p, k_gpu, k_oracle,
    rel)] for the record."""
    out = []
    for p in parities:
        sel = parity_sites(dims, p)
        if oracle_runs is not None:
            xo, ko = oracle_runs[p]
        else:
            xo, _, oi = oracle.cg_solve(dims, U, m, b, tol=tol, parity=p)
            ko = oi["iters"]
        kg, ko = int(iters_parity[p]), int(ko)
        if abs(kg - ko) <= 1:
            r = rel(x_gpu[sel], xo[sel])
            how = "final"
        else:
            assert rerun is not None, "%s parity %d: counts %d (GPU) and %d (oracle) differ by more than 1" % (
                label, p, kg, ko)
            k = min(kg, ko)
            xk = rerun(p, k)
            xok, _ = oracle.cg_pass(dims, U, m, b, tol=0.0, maxiter=k, parity=p)
            r = rel(xk[sel], xok[sel])
            how = "equal k=%d" % k
        print("COUNTS %s parity %d: GPU %d oracle %d (%s) rel %.2e" % (label, p, kg, ko, how, r), flush=True)
        assert r <= TOL_X, (label, p, kg, ko, how, r)
        out.append((p, kg, ko, r))
    return out


def oracle_o3(dims, U, m, b, tol=1e-10):
    """O3 per parity system: one pass of the paper's loop to tol with its CG
    coefficients (if the pass's FP64 true residual misses tol, the restarted
    solve is used instead), and the condition estimate from the extreme Ritz
    values over both parities.  Returns (runs {p: (x, iters)}, kappa, x) with
    x the two parities' solutions on the whole lattice."""
    runs, lmax, lmin = {}, 0.0, np.inf
    x3 = np.zeros_like(np.asarray(b, dtype=np.complex128))
    for p in (0, 1):
        xp, al, be, info = oracle.cg_coefficients(dims, U, m, b, tol=tol, parity=p)
        if oracle.true_residual(dims, U, m, b, xp, parity=p) > tol:
            xp, _, oi = oracle.cg_solve(dims, U, m, b, tol=tol, parity=p)
            info = oi
        th = oracle.ritz_values(al, be)
        lmax, lmin = max(lmax, th[-1]), min(lmin, th[0])
        runs[p] = (xp, info["iters"])
        sel = parity_sites(dims, p)
        x3[sel] = xp[sel]
    return runs, lmax / lmin, x3


def oracle_tight(dims, U, m, b, x0, tight=1e-13):
    """O4: textbook CG on the whole lattice to relative residual `tight`,
    with true-residual restarts, started from x0 (an oracle solution)."""
    xt, _ = oracle.cg_full(dims, U, m, b, tol=tight, x0=x0)
    return xt


def wilson_contract(kg, ko, x_gpu, x_oracle, rerun, oracle_k, label=""):
    """The same contract for the Wilson even-odd CG (one system, the even
    sites): rerun(k) / oracle_k(k) give the two sides' solutions after k
    iterations."""
    if abs(kg - ko) <= 1:
        r = rel(x_gpu, x_oracle)
        how = "final"
    else:
        k = min(kg, ko)
        r = rel(rerun(k), oracle_k(k))
        how = "equal k=%d" % k
    print("COUNTS %s: GPU %d oracle %d (%s) rel %.2e" % (label, kg, ko, how, r), flush=True)
    assert r <= TOL_X, (label, kg, ko, how, r)
    return r
