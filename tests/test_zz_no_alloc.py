"""The allocation-free entry point (mbt_active_dev_noalloc) against the
allocating one it mirrors (mbt_active): two calls in a row on device buffers,
the second on a smaller array, both bit-identical to mbt_active; and the size
limit of its scratch array."""
import sys

import numpy as np
import pytest

from paper_2608_17844_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _zp(P, seed):
    """A seeded symmetric port impedance matrix with a dominant diagonal (the
    call is pure post-processing of Z_p; any invertible Z_p + z0 will do)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((P, P)) + 1j * rng.standard_normal((P, P))
    return (A + A.T) * 2.0 + np.eye(P) * (80.0 + 40.0j)


def _noalloc(mbt, torch, ctx, arr, s, Zp, th, ph, wave=True):
    dev = torch.device("cuda:0")
    Zt = torch.from_numpy(np.asfortranarray(Zp).ravel(order="F").copy()).to(dev)
    tt = torch.from_numpy(np.ascontiguousarray(th, dtype=np.float64)).to(dev)
    pt = torch.from_numpy(np.ascontiguousarray(ph, dtype=np.float64)).to(dev)
    ns = th.size
    za = torch.zeros(ns, dtype=torch.complex128, device=dev)
    g = torch.zeros(ns, dtype=torch.complex128, device=dev)
    gw = torch.zeros(ns, dtype=torch.complex128, device=dev) if wave else None
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    mbt.mbt_active_dev_noalloc(ctx, arr, s, Zt.data_ptr(), tt.data_ptr(), pt.data_ptr(), ns, 50.0, za.data_ptr(),
                               g.data_ptr(), gw.data_ptr() if wave else None, stream.cuda_stream)
    torch.cuda.synchronize()
    return za.cpu().numpy(), g.cpu().numpy(), (gw.cpu().numpy() if wave else None)


def test_noalloc_active_matches_allocating_entry_point_two_calls():
    import torch
    from paper_2608_17844_amd import mbt
    ctx = mbt.mbt_ctx_create(0)
    try:
        for (nx, ny, ns, s, seed) in ((32, 32, 64, 1.0, 1), (5, 4, 7, 1.2, 2)):
            lat = W.Lattice(nx, ny, 0.5, 0.55)
            arr = mbt.mbt_array_create_dipole(ctx, W.Dipole(0.5, 0.005, 3), lat)
            try:
                Zp = _zp(nx * ny, seed)
                th, ph = W.scan_angles(ns, seed=seed)
                _say("no-alloc active: %dx%d, %d scans" % (nx, ny, ns))
                za0, g0, gw0 = mbt.mbt_active(ctx, arr, s, Zp, th, ph, 50.0)
                za1, g1, gw1 = _noalloc(mbt, torch, ctx, arr, s, Zp, th, ph)
                assert np.array_equal(za0, za1) and np.array_equal(g0, g1) and np.array_equal(gw0, gw1), (
                    np.max(np.abs(za0 - za1)), np.max(np.abs(gw0 - gw1)))
            finally:
                mbt.mbt_array_destroy(arr)
    finally:
        mbt.mbt_ctx_destroy(ctx)


def test_noalloc_scratch_limit():
    """Above 1024 ports the wave-excited ARC does not fit the scratch array: a
    clear MBT_EINVAL before any work; without Gamma_wave no scratch is used."""
    import torch
    from paper_2608_17844_amd import mbt
    ctx = mbt.mbt_ctx_create(0)
    try:
        lat = W.Lattice(33, 32, 0.5, 0.5)
        arr = mbt.mbt_array_create_dipole(ctx, W.Dipole(0.5, 0.005, 3), lat)
        try:
            Zp = _zp(33 * 32, 3)
            th, ph = W.scan_angles(4, seed=4)
            with pytest.raises(mbt.MbtError) as e:
                _noalloc(mbt, torch, ctx, arr, 1.0, Zp, th, ph, wave=True)
            assert e.value.status == mbt.MBT_EINVAL and "scratch" in str(e.value)
            za0, g0, _ = mbt.mbt_active(ctx, arr, 1.0, Zp, th, ph, 50.0)
            za1, g1, _ = _noalloc(mbt, torch, ctx, arr, 1.0, Zp, th, ph, wave=False)
            assert np.array_equal(za0, za1) and np.array_equal(g0, g1)
        finally:
            mbt.mbt_array_destroy(arr)
    finally:
        mbt.mbt_ctx_destroy(ctx)
