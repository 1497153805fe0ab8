"""Batch shapes on the GPU: ragged and odd right-hand-side counts (one and two
RHS per lane in the Arnoldi sweeps), repeated ports, the empty port list, and
long restart cycles (the FP32 dot sweep split into 32-vector launches), on a
16x16 array checked against the dense oracle."""
import sys

import numpy as np
import pytest

from oracle import mom
from paper_2608_17844_amd import workloads as W

pytestmark = pytest.mark.gpu

LAT = W.Lattice(16, 16, 0.5, 0.5)
DIP = W.Dipole(0.5, 0.005, 15)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    from paper_2608_17844_amd import mbt
    ctx = mbt.mbt_ctx_create(0)
    arr = mbt.mbt_array_create_dipole(ctx, DIP, LAT)
    ref = mom.solve_array(LAT, DIP, 1.0)
    yield mbt, ctx, arr, ref
    mbt.mbt_array_destroy(arr)
    mbt.mbt_ctx_destroy(ctx)


@pytest.mark.parametrize("nports", [1, 33, 34, 65, 256])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_port_subsets_of_any_size(setup, nports, prec):
    mbt, ctx, arr, ref = setup
    rng = np.random.default_rng(nports)
    ports = sorted(rng.choice(256, size=nports, replace=False).tolist()) if nports < 256 else list(range(256))
    opts = mbt.mbt_default_opts(prec=prec, pc=mbt.MBT_PC_ELEMENT_BLOCK, tol=1e-11, refine_tol=1e-10, refine_max=4)
    Y, iters, st = mbt.mbt_port_admittance(ctx, arr, 1.0, ports, opts)
    err = np.linalg.norm(Y - ref.Yp[:, ports]) / np.linalg.norm(ref.Yp[:, ports])
    _say("prec=%d nports=%d err=%.2e iters %d..%d cycles %d" % (prec, nports, err, iters.min(), iters.max(),
                                                               st["cycles"]))
    assert err <= (1e-9 if prec == 0 else 1e-8)
    assert st["nconverged"] == nports


def test_long_cycles_reach_the_split_dot_sweeps(setup):
    """With restart 60 a cycle runs past 32 basis vectors, where the FP32 dot
    sweep is split into two launches; results must not change with the batch."""
    mbt, ctx, arr, ref = setup
    opts = mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK, restart=60, inner_tol=1e-6,
                                refine_tol=1e-10, refine_max=4)
    Y, iters, st = mbt.mbt_port_admittance(ctx, arr, 1.0, None, opts)
    _say("restart 60: iters %d..%d, outer %d" % (iters.min(), iters.max(), st["outer_steps"]))
    assert iters.max() > 40
    assert np.linalg.norm(Y - ref.Yp) / np.linalg.norm(ref.Yp) <= 1e-8
    # the same columns solved in a smaller, odd batch are identical
    sub = [3, 77, 200]
    Ys, _, _ = mbt.mbt_port_admittance(ctx, arr, 1.0, sub, opts)
    assert np.array_equal(Ys, Y[:, sub])


def test_repeated_and_empty_port_lists(setup):
    mbt, ctx, arr, ref = setup
    opts = mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK)
    Y, _, _ = mbt.mbt_port_admittance(ctx, arr, 1.0, [5, 5, 130, 5], opts)
    assert np.array_equal(Y[:, 0], Y[:, 1]) and np.array_equal(Y[:, 0], Y[:, 3])
    assert np.linalg.norm(Y[:, 2] - ref.Yp[:, 130]) <= 1e-9 * np.linalg.norm(ref.Yp[:, 130])
    with pytest.raises(mbt.MbtError) as ei:
        mbt.mbt_port_admittance(ctx, arr, 1.0, [], opts)
    assert ei.value.status == mbt.MBT_EINVAL


def test_packed_basis_against_fp32_basis(setup):
    """The reduced-precision inner solves keep their Krylov basis packed (FP32
    components rounded to 24 bits) unless told otherwise; both forms reach the
    same refined accuracy with about the same work, and an odd port count
    (solved with one port repeated) reports every port exactly once."""
    mbt, ctx, arr, ref = setup
    res = {}
    for name, flags in (("packed", 0), ("fp32", mbt.MBT_FLAG_FP32_BASIS)):
        opts = mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK, restart=32, tol=1e-11,
                                    refine_tol=1e-10, refine_max=4, flags=flags)
        Y, iters, st = mbt.mbt_port_admittance(ctx, arr, 1.0, None, opts)
        err = np.linalg.norm(Y - ref.Yp) / np.linalg.norm(ref.Yp)
        _say("%s basis: iters %d..%d (total %d), outer %d, err %.2e" % (name, iters.min(), iters.max(), iters.sum(),
                                                                         st["outer_steps"], err))
        assert err <= 1e-8
        assert st["nconverged"] == 256
        res[name] = (iters, st)
    ip, ifp = res["packed"][0], res["fp32"][0]
    assert abs(int(ip.sum()) - int(ifp.sum())) <= 0.1 * ifp.sum()
    opts = mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK, tol=1e-11, refine_tol=1e-10,
                                refine_max=4)
    odd = [0, 17, 255]
    Y3, it3, st3 = mbt.mbt_port_admittance(ctx, arr, 1.0, odd, opts)
    assert Y3.shape == (256, 3) and it3.shape == (3,)
    assert st3["nrhs"] == 3 and st3["nconverged"] == 3
    assert np.linalg.norm(Y3 - ref.Yp[:, odd]) <= 1e-8 * np.linalg.norm(ref.Yp[:, odd])


@pytest.mark.parametrize("case", ["fp32_basis", "cgs2"])
def test_mixed_path_without_packed_basis(setup, case):
    """The plain FP32 basis layout is taken where the packed one does not apply
    (asked for, or classical CGS2): both reach the refined accuracy, and an odd
    port count is solved as it is (no padding)."""
    mbt, ctx, arr, ref = setup
    kw = dict(flags=mbt.MBT_FLAG_FP32_BASIS if case == "fp32_basis" else mbt.MBT_FLAG_CGS2)
    opts = mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK, tol=1e-11, refine_tol=1e-10,
                                refine_max=5, **kw)
    ports = [1, 100, 255]
    Y, it, st = mbt.mbt_port_admittance(ctx, arr, 1.0, ports, opts)
    err = np.linalg.norm(Y - ref.Yp[:, ports]) / np.linalg.norm(ref.Yp[:, ports])
    _say("%s: iters %d..%d outer %d err %.2e" % (case, it.min(), it.max(), st["outer_steps"], err))
    assert err <= 1e-8 and st["nconverged"] == 3 and st["nrhs"] == 3
