"""Block-defined lattice operators on the GPU (caller-given blocks of up to 128
bases per element, here seeded synthetic blocks; the RWG elements of the largest
single-GPU shape have their own tests in test_gpu_rwg.py): the per-bin products of large blocks (LDS-staged MFMA), the matvec
and preconditioned solves against the dense oracle on small lattices, and at
the full 64 x 64 x 96 shape sampled entries of Z x and of the residual
V - Z I computed entry by entry by the oracle."""
import sys

import numpy as np
import pytest

from oracle import blocks as ob
from oracle import mom
from paper_2608_17844_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2608_17844_amd import mbt
    h = mbt.mbt_ctx_create(0)
    yield h
    mbt.mbt_ctx_destroy(h)


CASES = [(3, 2, 48), (4, 4, 96), (2, 3, 128), (5, 1, 33)]



def _pow2(n):
    """The lattice transform length along an axis: the power of two >= n, at least 8."""
    return max(8, 1 << (int(n) - 1).bit_length())

@pytest.mark.parametrize("case", CASES, ids=["%dx%d_m%d" % c for c in CASES])
def test_block_matvec_matches_dense(ctx, case):
    from paper_2608_17844_amd import mbt
    nx, ny, M = case
    T = W.synthetic_blocks(nx, ny, M, seed=M)
    a = mbt.mbt_array_create_blocks(ctx, T)
    try:
        Tg = mbt.mbt_dbg_fill_blocks(ctx, a, 1.0, W.Lattice(nx, ny, 0.5, 0.5), M)
        assert np.array_equal(Tg, T)
        Z = ob.dense_from_blocks(T, nx, ny)
        x = W.random_vectors(Z.shape[0], 19, seed=1)
        # element by element against |Z| |x|: two lattice transforms and a sum over M bases
        c = 16 * (np.log2(4 * _pow2(nx) * _pow2(ny)) + M)
        aZ, ax = np.abs(Z), np.abs(x)
        for prec, tol, u in ((0, 1e-13, 2.0 ** -53), (1, 3e-6, 2.0 ** -24)):
            for op in (0, 1, 2):
                y = mbt.mbt_dbg_matvec(ctx, a, 1.0, x, op=op, prec=prec)
                ref = Z @ x if op == 0 else (Z.conj().T @ x if op == 1 else Z.conj().T @ (Z @ x))
                mag = aZ @ ax if op == 0 else (aZ.T @ ax if op == 1 else aZ.T @ (aZ @ ax))
                err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
                comp = np.max(np.abs(y - ref) / mag)
                _say("%dx%d M=%d prec=%d op=%d err=%.2e componentwise %.2e" % (nx, ny, M, prec, op, err, comp))
                assert err <= tol
                assert comp <= c * u * (2 if op == 2 else 1)
    finally:
        mbt.mbt_array_destroy(a)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_block_operator_solve_matches_lu(ctx, prec):
    from paper_2608_17844_amd import mbt
    nx, ny, M = 4, 4, 96
    T = W.synthetic_blocks(nx, ny, M, seed=7)
    a = mbt.mbt_array_create_blocks(ctx, T)
    try:
        Z = ob.dense_from_blocks(T, nx, ny)
        ports = [0, 5, 10, 15, 3]
        from types import SimpleNamespace as NS
        V = mom.excitation(NS(nx=nx, ny=ny), NS(nbases=M), ports)
        I = mom.solve_lu(Z, V)
        opts = mbt.mbt_default_opts(prec=prec, pc=mbt.MBT_PC_ELEMENT_BLOCK, restart=32, tol=1e-11,
                                    refine_tol=1e-10)
        Y, iters, st = mbt.mbt_port_admittance(ctx, a, 1.0, ports, opts)
        ref = I.reshape(nx * ny, M, len(ports))[:, (M - 1) // 2, :]
        err = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
        _say("prec=%d err=%.2e iters %s" % (prec, err, list(iters)))
        assert err <= 1e-9
    finally:
        mbt.mbt_array_destroy(a)


@pytest.mark.parametrize("M", [48, 96, 128])
def test_normal_eq_preconditioner_for_large_blocks(ctx, M):
    """P_A for more than 32 bases (blocks factorised in global memory): its
    blocks equal the diagonal blocks of Z^H Z, its apply equals the Cholesky
    solves, and GMRES on P_A^{-1} Z^H Z (FP64, and FP32 with refinement) reaches
    the LU solution."""
    from paper_2608_17844_amd import mbt
    from oracle import gmres as og
    from types import SimpleNamespace as NS
    nx, ny = 3, 2
    T = W.synthetic_blocks(nx, ny, M, seed=M + 1)
    a = mbt.mbt_array_create_blocks(ctx, T)
    try:
        Z = ob.dense_from_blocks(T, nx, ny)
        lat, dip = NS(nx=nx, ny=ny), NS(nbases=M)
        P = nx * ny
        ref_blocks = og.pa_blocks(Z, lat, dip)
        Pb = mbt.mbt_dbg_precond_blocks(ctx, a, 1.0, mbt.MBT_PC_NORMAL_EQ, P, M)
        sc = max(np.abs(b).max() for b in ref_blocks)
        assert max(np.abs(Pb[e] - ref_blocks[e]).max() for e in range(P)) <= 1e-13 * sc
        x = W.random_vectors(Z.shape[0], 3, seed=5)
        y = mbt.mbt_dbg_precond_apply(ctx, a, 1.0, x, mbt.MBT_PC_NORMAL_EQ)
        f = og.pa_factors(ref_blocks)
        ref = np.stack([og.pa_apply(f, x[:, j], M) for j in range(3)], axis=1)
        e_apply = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        ports = [0, 2, 5]
        V = mom.excitation(lat, dip, ports)
        I = mom.solve_lu(Z, V)
        Iref = I.reshape(P, M, len(ports))[:, (M - 1) // 2, :]
        errs = []
        for prec in (mbt.MBT_FP64, mbt.MBT_FP32):
            opts = mbt.mbt_default_opts(prec=prec, pc=mbt.MBT_PC_NORMAL_EQ, restart=40, tol=1e-12,
                                        refine_tol=1e-11, refine_max=6)
            Y, iters, st = mbt.mbt_port_admittance(ctx, a, 1.0, ports, opts)
            errs.append(np.linalg.norm(Y - Iref) / np.linalg.norm(Iref))
        _say("M=%d: P_A apply err %.2e; admittance fp64 %.2e fp32 %.2e" % (M, e_apply, errs[0], errs[1]))
        assert e_apply <= 1e-11 and errs[0] <= 1e-9 and errs[1] <= 1e-9
    finally:
        mbt.mbt_array_destroy(a)


def test_block_operator_limits(ctx):
    from paper_2608_17844_amd import mbt
    T = W.synthetic_blocks(2, 2, 40, seed=3)
    a = mbt.mbt_array_create_blocks(ctx, T)
    try:
        for kw in (dict(prec=mbt.MBT_BF16),):
            with pytest.raises(mbt.MbtError) as ei:
                mbt.mbt_port_admittance(ctx, a, 1.0, [0], mbt.mbt_default_opts(**kw))
            assert ei.value.status == mbt.MBT_EINVAL
        with pytest.raises(mbt.MbtError) as ei:
            mbt.mbt_solve(ctx, a, 1.0, mbt.mbt_default_opts(), [0.1], [0.2])
        assert ei.value.status == mbt.MBT_EINVAL
    finally:
        mbt.mbt_array_destroy(a)
    with pytest.raises(mbt.MbtError) as ei:
        mbt.mbt_array_create_blocks(ctx, np.zeros((3, 3, 129, 129), dtype=np.complex128))
    assert ei.value.status == mbt.MBT_EINVAL


def test_largest_shape_sampled_matvec_and_residual(ctx):
    """64 x 64 elements of 96 bases (N = 393,216), FFT grid 128 x 128."""
    from paper_2608_17844_amd import mbt
    nx, ny, M, seeds, ports = W.blocks_64x64_m96_shape()
    _say("generating 64x64x96 blocks")
    T = W.synthetic_blocks(nx, ny, M, seed=seeds[0])
    a = mbt.mbt_array_create_blocks(ctx, T)
    try:
        N = nx * ny * M
        rng = np.random.default_rng(11)
        rows = np.sort(rng.choice(N, size=24, replace=False))
        x = W.random_vectors(N, 2, seed=3)
        for prec, tol in ((0, 1e-12), (1, 3e-6)):
            y = mbt.mbt_dbg_matvec(ctx, a, 1.0, x, op=0, prec=prec)
            ref = ob.matvec_entries(T, nx, ny, x, rows)
            err = np.max(np.abs(y[rows] - ref)) / np.max(np.abs(ref))
            _say("matvec prec=%d sampled err %.2e" % (prec, err))
            assert err <= tol
        # mixed-precision solve of four port excitations; residual sampled by the oracle
        V = np.zeros((N, 4), dtype=np.complex128)
        for j, p in enumerate(ports[:4]):
            V[int(p) * M + (M - 1) // 2, j] = 1.0
        opts = mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK, restart=32, refine_tol=1e-10)
        I, iters, st = mbt.mbt_dbg_solve(ctx, a, 1.0, opts, V)
        rrows = np.concatenate([rows, [int(p) * M + (M - 1) // 2 for p in ports[:4]]])
        res = ob.matvec_entries(T, nx, ny, I, rrows) - V[rrows]
        _say("solve: iters %s outer %d relres %.2e sampled residual %.2e" % (
            list(iters), st["outer_steps"], st["true_relres_max"], np.max(np.abs(res))))
        assert st["true_relres_max"] <= 1e-10
        assert np.max(np.abs(res)) <= 1e-9
    finally:
        mbt.mbt_array_destroy(a)
