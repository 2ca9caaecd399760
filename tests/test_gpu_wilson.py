"""GPU parity of the Wilson-fermion path against the CPU oracle.

Bars: the hop H per site <= 1e-13 relative (as for the staggered D_slash);
the even-odd CG runs the oracle's loop: iteration counts agree within 1 and
x agrees to 1e-10 relative, or else the two sides' k-th iterates agree at
1e-10 (cg_counts.wilson_contract); every solve's FP64 true residual
||b - M x|| / ||b|| is recomputed by the oracle from the returned x."""

import os

import numpy as np
import pytest
import torch

import oracle
from paper_1311_2719_amd import binding, inputs
from cg_counts import wilson_contract

pytestmark = pytest.mark.gpu

TOL = 1e-13


def site_err(got, ref):
    g = got.reshape(len(got), -1)
    r = ref.reshape(len(ref), -1)
    n = np.linalg.norm(r, axis=1)
    floor = 1e-3 * np.sqrt(np.mean(n ** 2))
    return np.max(np.linalg.norm(g - r, axis=1) / np.maximum(n, floor))


def hop(ctx, f, psi, out_parity=binding.ALL, base=None):
    b = ctx.pack_spinor(f, psi)
    out = ctx.pack_spinor(f, base) if base is not None else ctx.new_spinor(f)
    ctx.wilson_dslash(f, b, out, out_parity=out_parity)
    return ctx.unpack_spinor(f, out).cpu().numpy()


def parity_mask(dims):
    V = int(np.prod(dims))
    s = np.arange(V)
    return ((s % dims[0]) + (s // dims[0]) % dims[1] + (s // (dims[0] * dims[1])) % dims[2]
            + s // (dims[0] * dims[1] * dims[2])) & 1


def test_pack_roundtrip(gpu_ctx):
    dims = (4, 2, 6, 4)
    psi = inputs.gaussian_spinor(dims, 1)
    f = gpu_ctx.set_gauge_wilson(dims, inputs.unit_links(dims))
    try:
        eo = gpu_ctx.pack_spinor(f, psi)
        assert np.array_equal(gpu_ctx.unpack_spinor(f, eo).cpu().numpy(), psi)
    finally:
        gpu_ctx.free_gauge(f)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 6, 8), (6, 4, 2, 10), (8, 8, 8, 8)])
@pytest.mark.parametrize("kind", ["haar", "smooth"])
def test_hop_matches_oracle(gpu_ctx, dims, kind):
    U = inputs.haar_su3(dims, 11) if kind == "haar" else inputs.smooth_su3(dims, 0.5, 12)
    psi = inputs.gaussian_spinor(dims, 13)
    f = gpu_ctx.set_gauge_wilson(dims, U)
    try:
        assert gpu_ctx.link_rows(f) == 2
        assert site_err(hop(gpu_ctx, f, psi), oracle.wilson_hop(dims, U, psi)) <= TOL
    finally:
        gpu_ctx.free_gauge(f)


@pytest.mark.parametrize("case", ["three_rows", "not_special_unitary", "periodic_t"])
def test_hop_formats_and_boundary(gpu_ctx, case):
    dims = (4, 6, 4, 8)
    U = inputs.haar_su3(dims, 21)
    if case == "not_special_unitary":
        U = 0.9 * U
    tap = case != "periodic_t"
    psi = inputs.gaussian_spinor(dims, 22)
    if case == "three_rows":
        os.environ["STAG_LINK_ROWS"] = "3"
    try:
        f = gpu_ctx.set_gauge_wilson(dims, U, antiperiodic_t=tap)
    finally:
        os.environ.pop("STAG_LINK_ROWS", None)
    try:
        assert gpu_ctx.link_rows(f) == (2 if case == "periodic_t" else 3)
        assert site_err(hop(gpu_ctx, f, psi), oracle.wilson_hop(dims, U, psi, antiperiodic_t=tap)) <= TOL
    finally:
        gpu_ctx.free_gauge(f)


@pytest.mark.parametrize("par", [binding.EVEN, binding.ODD])
def test_hop_one_parity(gpu_ctx, par):
    dims = (4, 4, 2, 6)
    U = inputs.haar_su3(dims, 31)
    psi = inputs.gaussian_spinor(dims, 32)
    base = inputs.gaussian_spinor(dims, 33)
    f = gpu_ctx.set_gauge_wilson(dims, U)
    try:
        got = hop(gpu_ctx, f, psi, out_parity=par, base=base)
        sel = parity_mask(dims) == par
        ref = oracle.wilson_hop(dims, U, psi)
        assert site_err(got[sel], ref[sel]) <= TOL
        assert np.array_equal(got[~sel], base[~sel])
    finally:
        gpu_ctx.free_gauge(f)


def test_hop_full_size_16(gpu_ctx):
    dims = (16, 16, 16, 16)
    U = inputs.smooth_su3(dims, 0.3, 102)
    psi = inputs.gaussian_spinor(dims, 202)
    f = gpu_ctx.set_gauge_wilson(dims, U)
    try:
        assert site_err(hop(gpu_ctx, f, psi), oracle.wilson_hop(dims, U, psi)) <= TOL
    finally:
        gpu_ctx.free_gauge(f)


def solve(ctx, f, b_lex, kappa, **kw):
    b = ctx.pack_spinor(f, b_lex)
    x = ctx.new_spinor(f)
    info = ctx.wilson_solve(f, b, x, kappa, check=False, **kw)
    torch.cuda.synchronize()
    return ctx.unpack_spinor(f, x).cpu().numpy(), info


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dims,kappa,kind", [((4, 4, 4, 4), 0.12, "haar"), ((8, 8, 8, 8), 0.12, "smooth"),
                                             ((4, 6, 2, 8), 0.1, "haar")])
def test_solve_matches_oracle(gpu_ctx, dims, kappa, kind):
    U = inputs.haar_su3(dims, 41) if kind == "haar" else inputs.smooth_su3(dims, 0.5, 42)
    b = inputs.gaussian_spinor(dims, 43)
    f = gpu_ctx.set_gauge_wilson(dims, U)
    try:
        x, info = solve(gpu_ctx, f, b, kappa, tol=1e-10)
        xr, oi = oracle.wilson_cg(dims, U, kappa, b, tol=1e-10)
        assert info["status"] == 0 and oi["status"] == 0
        wilson_contract(info["iters"], oi["iters"], x, xr,
                        lambda k: solve(gpu_ctx, f, b, kappa, tol=1e-10, maxiter=k)[0],
                        lambda k: oracle.wilson_cg(dims, U, kappa, b, tol=1e-10, maxiter=k)[0],
                        label="Wilson %s %s" % (dims, kind))
        tr = np.linalg.norm(b - oracle.wilson_apply(dims, U, kappa, x)) / np.linalg.norm(b)
        assert abs(info["true_rel_resid"] - tr) <= 1e-3 * tr + 1e-15
        assert tr <= 1e-8
    finally:
        gpu_ctx.free_gauge(f)


def test_solve_three_rows_and_full_size(gpu_ctx):
    # the benchmark's Wilson workload (16^4, eps = 0.3, kappa = 0.12) and the
    # same field with three stored rows
    dims, kappa = (16, 16, 16, 16), 0.12
    U = inputs.smooth_su3(dims, 0.3, 102)
    b = inputs.gaussian_spinor(dims, 202)
    xr, oi = oracle.wilson_cg(dims, U, kappa, b, tol=1e-10)
    for rows in (2, 3):
        if rows == 3:
            os.environ["STAG_LINK_ROWS"] = "3"
        try:
            f = gpu_ctx.set_gauge_wilson(dims, U)
        finally:
            os.environ.pop("STAG_LINK_ROWS", None)
        try:
            assert gpu_ctx.link_rows(f) == rows
            x, info = solve(gpu_ctx, f, b, kappa, tol=1e-10)
            assert info["status"] == 0
            wilson_contract(info["iters"], oi["iters"], x, xr,
                            lambda k: solve(gpu_ctx, f, b, kappa, tol=1e-10, maxiter=k)[0],
                            lambda k: oracle.wilson_cg(dims, U, kappa, b, tol=1e-10, maxiter=k)[0],
                            label="Wilson 16^4 rows %d" % rows)
        finally:
            gpu_ctx.free_gauge(f)


def test_solve_edge_cases_and_errors(gpu_ctx):
    dims = (4, 4, 4, 4)
    U = inputs.haar_su3(dims, 51)
    f = gpu_ctx.set_gauge_wilson(dims, U)
    fs = gpu_ctx.set_gauge(dims, U)
    try:
        x, info = solve(gpu_ctx, f, np.zeros((256, 4, 3), np.complex128), 0.12)
        assert info["status"] == 0 and info["iters"] == 0 and not np.any(x)
        b = inputs.gaussian_spinor(dims, 52)
        x, info = solve(gpu_ctx, f, b, 0.12, maxiter=3)
        assert info["status"] == binding.ENOCONV and info["iters"] == 3
        bd = gpu_ctx.pack_spinor(f, b)
        xd = gpu_ctx.new_spinor(f)
        for kw in ({"kappa": 0.0}, {"kappa": 0.12, "tol": 0.0}, {"kappa": 0.12, "maxiter": -1}):
            with pytest.raises(binding.StagError) as e:
                gpu_ctx.wilson_solve(f, bd, xd, **kw)
            assert e.value.code == binding.EINVAL
        # ids of the other operator are refused
        with pytest.raises(binding.StagError) as e:
            gpu_ctx.wilson_solve(fs, bd, xd, 0.12)
        assert e.value.code == binding.EINVAL
        with pytest.raises(binding.StagError) as e:
            gpu_ctx.cg_solve(f, gpu_ctx.new_fermion(f), gpu_ctx.new_fermion(f), mass=0.1)
        assert e.value.code == binding.EINVAL
        with pytest.raises(binding.StagError) as e:
            gpu_ctx.wilson_dslash(f, bd, bd)
        assert e.value.code == binding.EINVAL
    finally:
        gpu_ctx.free_gauge(f)
        gpu_ctx.free_gauge(fs)


@pytest.mark.parametrize("lps", ["1", "2", "4", "8"])
def test_every_lanes_per_site(lps):
    # the tuner may pick 1, 2, 4 or 8 lanes per site for the Wilson kernels: each
    # must give the same hop and the same solve
    dims = (6, 4, 2, 10)
    U = inputs.haar_su3(dims, 61)
    psi = inputs.gaussian_spinor(dims, 62)
    os.environ["STAG_WILSON_LPS"] = lps
    try:
        with binding.Context(device=0, arena_bytes=64 << 20) as ctx:
            f = ctx.set_gauge_wilson(dims, U)
            assert site_err(hop(ctx, f, psi), oracle.wilson_hop(dims, U, psi)) <= TOL
            x, info = solve(ctx, f, psi, 0.11, tol=1e-10)
            xr, oi = oracle.wilson_cg(dims, U, 0.11, psi, tol=1e-10)
            assert info["status"] == 0
            wilson_contract(info["iters"], oi["iters"], x, xr,
                            lambda k: solve(ctx, f, psi, 0.11, tol=1e-10, maxiter=k)[0],
                            lambda k: oracle.wilson_cg(dims, U, 0.11, psi, tol=1e-10, maxiter=k)[0],
                            label="Wilson lanes per site %s" % lps)
    finally:
        del os.environ["STAG_WILSON_LPS"]


@pytest.mark.parametrize("lps", ["1", "4"])
def test_nontemporal_link_loads_give_the_same_bits(monkeypatch, lps):
    # fields whose links exceed the Infinity Cache read them with non-temporal
    # loads (STAG_NT_LINKS forces either kind): the hop and every CG iterate
    # are the same to the bit
    dims = (6, 4, 2, 10)
    U = inputs.haar_su3(dims, 71)
    psi = inputs.gaussian_spinor(dims, 72)
    monkeypatch.setenv("STAG_WILSON_LPS", lps)
    res = {}
    for nt in ("0", "1"):
        monkeypatch.setenv("STAG_NT_LINKS", nt)
        with binding.Context(device=0, arena_bytes=64 << 20) as ctx:
            f = ctx.set_gauge_wilson(dims, U)
            x, info = solve(ctx, f, psi, 0.11, tol=1e-10)
            res[nt] = (hop(ctx, f, psi), x, info["iters"])
    assert np.array_equal(res["0"][0], res["1"][0])
    assert np.array_equal(res["0"][1], res["1"][1]) and res["0"][2] == res["1"][2]
    assert site_err(res["1"][0], oracle.wilson_hop(dims, U, psi)) <= TOL
