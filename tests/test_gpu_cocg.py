"""Batched COCG (conjugate orthogonal CG on the complex symmetric Z with the
symmetric element-block preconditioner P_K; not part of the paper) on the GPU:
per-RHS iteration counts against the oracle's COCG, the admittance and port
quantities against the dense LU oracle, FP32 inner solves with FP64
refinement, and option checking."""
import sys

import numpy as np
import pytest

from oracle import gmres as og
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


def _opts(mbt, prec, **kw):
    return mbt.mbt_default_opts(prec=prec, pc=mbt.MBT_PC_ELEMENT_BLOCK, flags=mbt.MBT_FLAG_COCG, **kw)


def test_cocg_iteration_parity_and_admittance_cfg_5x5(ctx, cfg1, cfg1_oracle):
    """COCG minimises nothing: on these systems its residual falls to a plateau
    about a decade above tol 1e-10 for two to four steps before dropping by two
    decades, and rounding order (the oracle applies P_K by LU solves, the GPU by
    its explicit inverse) decides on which plateau step the test first passes.
    Each RHS must therefore stop no later than two steps after the oracle and
    not before the oracle's residual has reached two decades of the tolerance
    (the start of the plateau)."""
    from paper_2608_17844_amd import mbt
    lat, dip = cfg1.lattice, cfg1.dipole
    a = mbt.mbt_array_create_dipole(ctx, dip, lat)
    try:
        Y, iters, st = mbt.mbt_port_admittance(ctx, a, 1.0, None, _opts(mbt, mbt.MBT_FP64, tol=1e-10))
    finally:
        mbt.mbt_array_destroy(a)
    _, res = og.cocg_all(cfg1_oracle.Z, lat, dip, mom.excitation(lat, dip), tol=1e-10)
    ref_it = np.array([r.iters for r in res])
    _say("cocg iterations gpu %s" % iters.tolist())
    _say("cocg iterations oracle %s" % ref_it.tolist())
    bad = []
    for j, r in enumerate(res):
        first = next(i + 1 for i, v in enumerate(r.relres) if v <= 1e-8)
        if not (first <= int(iters[j]) <= r.iters + 2):
            bad.append((j, int(iters[j]), first, r.iters))
    assert not bad, bad
    err = np.linalg.norm(Y - cfg1_oracle.Yp) / np.linalg.norm(cfg1_oracle.Yp)
    _say("cocg fp64 |dY|/|Y| %.2e" % err)
    assert err <= 1e-8
    assert st["nconverged"] == 25 and st["cycles"] == 1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cocg_port_quantities(ctx, cfg1, cfg1_oracle, prec):
    from paper_2608_17844_amd import mbt
    p = mbt.MBT_FP64 if prec == "fp64" else mbt.MBT_FP32
    a = mbt.mbt_array_create_dipole(ctx, cfg1.dipole, cfg1.lattice)
    try:
        out = mbt.mbt_solve(ctx, a, 1.0, _opts(mbt, p, tol=1e-10), cfg1.theta, cfg1.phi, cfg1.z0)
    finally:
        mbt.mbt_array_destroy(a)
    ref = cfg1_oracle
    err = np.linalg.norm(out["Zp"] - ref.Zp) / np.linalg.norm(ref.Zp)
    _say("cocg %s |dZp|/|Zp| %.2e, outer %d, iters %d" % (prec, err, out["stats"]["outer_steps"],
                                                          out["stats"]["iters_max"]))
    bound = 1e-9 if prec == "fp64" else 1e-6
    assert err <= bound
    assert np.max(np.abs(out["Gamma"] - ref.Gamma)) <= bound
    assert np.max(np.abs(out["Gamma_wave"] - ref.Gamma_wave)) <= bound


def test_cocg_agrees_with_gmres_16x16(ctx):
    """Both solvers reach the same admittance on a 16x16 array of 15-basis dipoles."""
    from paper_2608_17844_amd import mbt
    lat, dip = W.Lattice(16, 16, 0.5, 0.5), W.Dipole(0.5, 0.005, 15)
    a = mbt.mbt_array_create_dipole(ctx, dip, lat)
    try:
        Yc, itc, _ = mbt.mbt_port_admittance(ctx, a, 1.0, None, _opts(mbt, mbt.MBT_FP64, tol=1e-11))
        Yg, itg, _ = mbt.mbt_port_admittance(ctx, a, 1.0, None,
                                             mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK,
                                                                  tol=1e-11))
    finally:
        mbt.mbt_array_destroy(a)
    _say("16x16: cocg iterations %d..%d, gmres %d..%d" % (itc.min(), itc.max(), itg.min(), itg.max()))
    assert np.linalg.norm(Yc - Yg) / np.linalg.norm(Yg) <= 1e-8


def test_cocg_option_checks(ctx, cfg1):
    from paper_2608_17844_amd import mbt
    a = mbt.mbt_array_create_dipole(ctx, cfg1.dipole, cfg1.lattice)
    try:
        bad = mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_NORMAL_EQ, flags=mbt.MBT_FLAG_COCG)
        with pytest.raises(mbt.MbtError) as e:
            mbt.mbt_port_admittance(ctx, a, 1.0, None, bad)
        assert e.value.status == mbt.MBT_EINVAL
        both = mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK,
                                    flags=mbt.MBT_FLAG_COCG | mbt.MBT_FLAG_PCG)
        with pytest.raises(mbt.MbtError) as e:
            mbt.mbt_port_admittance(ctx, a, 1.0, None, both)
        assert e.value.status == mbt.MBT_EINVAL
        # at most restart * max_cycles iterations, then MBT_ENOCONV
        short = _opts(mbt, mbt.MBT_FP64, restart=2, max_cycles=1)
        with pytest.raises(mbt.MbtError) as e:
            mbt.mbt_port_admittance(ctx, a, 1.0, None, short)
        assert e.value.status == mbt.MBT_ENOCONV
    finally:
        mbt.mbt_array_destroy(a)
