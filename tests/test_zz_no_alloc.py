"""GPU: the allocation-free solve (stag_cg_solve_noalloc) against the
existing entry point (stag_cg_solve), through the C ABI.

Two calls in a row on one GPU share the fixed workspace, the second with a
smaller lattice, each checked against stag_cg_solve on the same system:
solutions agree to 1e-10 relative (the FP64 parity bar; the same kernels in
the same shape give the same bits), and the oracle's FP64 true residual of
each is <= 1e-10.  A solve whose workspace exceeds the fixed buffer is
rejected with EINVAL and a message naming both sizes."""

import numpy as np
import pytest
import torch

import oracle
from paper_1311_2719_amd import binding, inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("prec", [binding.FP64, binding.FP32_RU])
def test_noalloc_matches_cg_solve(gpu_ctx, prec):
    cases = [((16, 16, 16, 16), 0.05, 401), ((8, 8, 8, 8), 0.02, 402)]  # second call smaller
    for dims, m, seed in cases:
        U = inputs.smooth_su3(dims, 0.5, seed)
        b_lex = inputs.gaussian_source(dims, seed + 1000)
        f = gpu_ctx.set_gauge(dims, U)
        try:
            bd = gpu_ctx.pack(f, b_lex)
            xa = gpu_ctx.new_fermion(f)
            ya = gpu_ctx.new_fermion(f)
            ia = gpu_ctx.cg_solve(f, bd, xa, y=ya, mass=m, tol=1e-10, precision=prec)
            xn = gpu_ctx.new_fermion(f)
            yn = gpu_ctx.new_fermion(f)
            used0 = gpu_ctx.arena_usage()[0]
            inn = gpu_ctx.cg_solve_noalloc(f, bd, xn, y=yn, mass=m, tol=1e-10, precision=prec)
            assert gpu_ctx.arena_usage()[0] == used0  # nothing taken from the arena
            torch.cuda.synchronize()
            xa_l = gpu_ctx.unpack(f, xa).cpu().numpy()
            xn_l = gpu_ctx.unpack(f, xn).cpu().numpy()
            same = np.array_equal(xa_l, xn_l)
            tr = oracle.true_residual(dims, U, m, b_lex, xn_l)
            print("noalloc %s prec %d: iters %s vs %s, bitwise %s, rel %.2e, true residual %.2e"
                  % (dims, prec, inn["iters_parity"], ia["iters_parity"], same, rel(xn_l, xa_l), tr))
            assert inn["status"] == 0 and ia["status"] == 0
            assert rel(xn_l, xa_l) <= 1e-10
            assert rel(gpu_ctx.unpack(f, yn).cpu().numpy(), gpu_ctx.unpack(f, ya).cpu().numpy()) <= 1e-10
            assert tr <= 1e-10 and inn["true_rel_resid"] <= 1e-10
        finally:
            gpu_ctx.free_gauge(f)


def test_noalloc_rejects_oversized(gpu_ctx):
    dims = (24, 24, 24, 48)  # 331 776 sites per parity: an FP64 workspace of ~160 MB
    f = gpu_ctx.set_gauge(dims, inputs.unit_links(dims))
    try:
        b = gpu_ctx.new_fermion(f)
        x = gpu_ctx.new_fermion(f)
        with pytest.raises(binding.StagError) as e:
            gpu_ctx.cg_solve_noalloc(f, b, x, mass=0.1)
        assert e.value.code == binding.EINVAL and "fixed workspace" in str(e.value)
    finally:
        gpu_ctx.free_gauge(f)
