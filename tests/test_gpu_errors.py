"""Failure paths of the C ABI (a context needs a device, so these run on the
GPU; no kernel is made to fault): a non-finite excitation is reported as
MBT_EBREAKDOWN for its own column while the other columns still solve to the
tolerance; invalid geometry, options, frequencies, ports and scan angles are
MBT_EINVAL with a message."""
import sys

import numpy as np
import pytest

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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nonfinite_excitation_is_breakdown_for_its_column(ctx, cfg1, cfg1_dense, prec):
    from paper_2608_17844_amd import mbt
    a = mbt.mbt_array_create_dipole(ctx, cfg1.dipole, cfg1.lattice)
    try:
        N = cfg1_dense.shape[0]
        V = W.random_vectors(N, 4, seed=9)
        V[7, 2] = np.nan
        if prec == "fp64":
            opts = mbt.mbt_default_opts(prec=mbt.MBT_FP64, tol=1e-12)
            bar = 1e-9
        else:
            opts = mbt.mbt_default_opts(prec=mbt.MBT_FP32, refine_tol=1e-10, refine_max=5)
            bar = 1e-8
        with pytest.raises(mbt.MbtError) as e:
            mbt.mbt_dbg_solve(ctx, a, 1.0, opts, V)
        assert e.value.status == mbt.MBT_EBREAKDOWN and "non-finite" in str(e.value)
        I, it, st = mbt.mbt_dbg_solve(ctx, a, 1.0, opts, V, allow_breakdown=True)
        assert st["status"] == mbt.MBT_EBREAKDOWN and st["nconverged"] == 3
        good = [0, 1, 3]
        ref = mom.solve_lu(cfg1_dense, V[:, good])
        err = np.linalg.norm(I[:, good] - ref) / np.linalg.norm(ref)
        _say("%s: finite columns error %.2e, iterations %s" % (prec, err, list(it)))
        assert err < bar
    finally:
        mbt.mbt_array_destroy(a)


def test_invalid_geometry_is_einval(ctx):
    from paper_2608_17844_amd import mbt
    lat = W.Lattice(3, 3, 0.5, 0.5)
    for dip, lt, what in ((W.Dipole(0.5, 0.005, 14), lat, "even nbases"),
                          (W.Dipole(0.5, 0.005, 0), lat, "no bases"),
                          (W.Dipole(0.5, 0.0, 15), lat, "zero radius"),
                          (W.Dipole(-0.5, 0.005, 15), lat, "negative length"),
                          (W.Dipole(0.5, 0.005, 15), W.Lattice(0, 3, 0.5, 0.5), "empty lattice"),
                          (W.Dipole(0.5, 0.005, 15), W.Lattice(65, 3, 0.5, 0.5), "lattice too large"),
                          (W.Dipole(0.5, 0.005, 15), W.Lattice(3, 3, 0.0, 0.5), "zero spacing")):
        with pytest.raises(mbt.MbtError) as e:
            mbt.mbt_array_create_dipole(ctx, dip, lt)
        assert e.value.status == mbt.MBT_EINVAL, what
        _say("%s: %s" % (what, e.value))


def test_invalid_solve_arguments_are_einval(ctx, cfg1):
    from paper_2608_17844_amd import mbt
    a = mbt.mbt_array_create_dipole(ctx, cfg1.dipole, cfg1.lattice)
    T = W.synthetic_blocks(2, 2, 3, seed=1)
    b = mbt.mbt_array_create_blocks(ctx, T)
    try:
        ok = mbt.mbt_default_opts(prec=mbt.MBT_FP64)

        def einval(fn, what):
            with pytest.raises(mbt.MbtError) as e:
                fn()
            assert e.value.status == mbt.MBT_EINVAL, what
            _say("%s: %s" % (what, e.value))

        einval(lambda: mbt.mbt_port_admittance(ctx, a, 1.0, [0], mbt.mbt_default_opts(restart=0)), "restart 0")
        einval(lambda: mbt.mbt_port_admittance(ctx, a, 1.0, [0], mbt.mbt_default_opts(tol=0.0)), "tol 0")
        einval(lambda: mbt.mbt_port_admittance(ctx, a, 1.0, [0], mbt.mbt_default_opts(prec=7)), "unknown precision")
        einval(lambda: mbt.mbt_port_admittance(ctx, a, 1.0, [0], mbt.mbt_default_opts(pc=5)), "unknown pc")
        einval(lambda: mbt.mbt_port_admittance(ctx, a, 1.0, [0],
                                               mbt.mbt_default_opts(pc=mbt.MBT_PC_ELEMENT_BLOCK,
                                                                    flags=mbt.MBT_FLAG_PCG)), "PCG with P_K")
        einval(lambda: mbt.mbt_port_admittance(ctx, a, 0.0, [0], ok), "zero frequency")
        einval(lambda: mbt.mbt_port_admittance(ctx, a, float("nan"), [0], ok), "NaN frequency")
        einval(lambda: mbt.mbt_port_admittance(ctx, a, 1.0, [25], ok), "port out of range")
        einval(lambda: mbt.mbt_port_admittance(ctx, a, 1.0, [-1], ok), "negative port")
        th, ph = np.array([0.1, np.nan]), np.array([0.0, 0.0])
        einval(lambda: mbt.mbt_scan_solve(ctx, a, 1.0, ok, th, ph), "NaN scan angle")
        einval(lambda: mbt.mbt_scan_solve(ctx, a, 1.0, ok, [0.1], [0.0], z0=0.0), "z0 = 0")
        einval(lambda: mbt.mbt_scan_solve(ctx, a, 1.0, ok, [0.1], [0.0], center=25), "center out of range")
        einval(lambda: mbt.mbt_scan_solve(ctx, b, 1.0, ok, [0.1], [0.0]), "scan on a block array")
        einval(lambda: mbt.mbt_solve(ctx, b, 1.0, ok, [0.1], [0.0]), "scans on a block array")
        einval(lambda: mbt.mbt_port_admittance(ctx, a, 1.0, [0], mbt.mbt_default_opts(prec=mbt.MBT_FP32,
                                                                                    refine_max=0)), "no refinement")
        # the array and context stay usable after the errors
        Y, it, st = mbt.mbt_port_admittance(ctx, a, 1.0, [0, 12], ok)
        assert np.isfinite(Y).all() and st["nconverged"] == 2
    finally:
        mbt.mbt_array_destroy(a)
        mbt.mbt_array_destroy(b)
