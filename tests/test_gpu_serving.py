"""Serving loop on the GPU: results of served requests against the CPU oracle,
the same request alone and inside a mix of concurrent requests, admission by
device-memory footprint, and request validation."""
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


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _mix():
    """A few heterogeneous requests (sizes, bases, frequencies, scans; seeded)."""
    th, ph = W.scan_angles(12, seed=3)
    return [
        (W.Dipole(0.5, 0.005, 15), W.Lattice(8, 8, 0.5, 0.5), [1.2], th[:5], ph[:5]),
        (W.Dipole(0.5, 0.005, 31), W.Lattice(6, 9, 0.5, 0.5), [0.7, 1.1], th, ph),
        (W.Dipole(0.5, 0.005, 15), W.Lattice(12, 10, 0.5, 0.5), [0.9], th[:1], ph[:1]),
        (W.Dipole(0.5, 0.005, 15), W.Lattice(3, 7, 0.5, 0.5), [1.4, 0.6, 1.0], th[:8], ph[:8]),
    ]


def _submit(mbt, srv, dip, lat, freqs, th, ph, opts):
    return mbt.mbt_server_submit(srv, (dip.length, dip.radius, dip.nbases), (lat.nx, lat.ny, lat.dx, lat.dy),
                                 freqs, th, ph, opts)


def test_served_request_matches_oracle_alone_and_in_mix(ctx, cfg1):
    from paper_2608_17844_amd import mbt
    opts = mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK)
    freqs = [0.8, 1.0]
    srv = mbt.mbt_server_create(ctx, 4)
    try:
        _say("serving: cfg1 alone")
        alone = mbt.mbt_server_wait(srv, _submit(mbt, srv, cfg1.dipole, cfg1.lattice, freqs, cfg1.theta, cfg1.phi,
                                                 opts))
        assert alone["status"] == mbt.MBT_OK
        _say("serving: cfg1 inside a mix of", len(_mix()), "requests")
        tickets = []
        mix = _mix()
        for i, (dip, lat, fr, th, ph) in enumerate(mix):
            tickets.append(_submit(mbt, srv, dip, lat, fr, th, ph, opts))
            if i == 1:
                tA = _submit(mbt, srv, cfg1.dipole, cfg1.lattice, freqs, cfg1.theta, cfg1.phi, opts)
        inmix = mbt.mbt_server_wait(srv, tA)
        others = [mbt.mbt_server_wait(srv, t) for t in tickets]
    finally:
        mbt.mbt_server_destroy(srv)
    # the same request gives bit-identical results alone and in the mix (every
    # reduction runs in a fixed order that does not depend on what else runs)
    assert inmix["status"] == mbt.MBT_OK
    for key in ("Zp", "Za", "Gamma", "Gamma_wave"):
        assert np.array_equal(inmix[key], alone[key]), (key, np.max(np.abs(inmix[key] - alone[key])))
    # and both match the oracle at every frequency (the ARC sums a row of Z_p
    # with unit-modulus phases: 1e-8 relative to max(1, |Gamma|) at this size)
    for fi, s in enumerate(freqs):
        ref = mom.solve_array(cfg1.lattice, cfg1.dipole, s, cfg1.theta, cfg1.phi)
        assert _rel(alone["Zp"][fi], ref.Zp) <= 1e-9
        assert np.max(np.abs(alone["Gamma"][fi] - ref.Gamma) / np.maximum(1.0, np.abs(ref.Gamma))) <= 1e-8
        assert np.max(np.abs(alone["Gamma_wave"][fi] - ref.Gamma_wave)) <= 1e-8
    # every other request of the mix matches its own oracle
    for (dip, lat, fr, th, ph), res in zip(mix, others):
        assert res["status"] == mbt.MBT_OK
        for fi, s in enumerate(fr):
            ref = mom.solve_array(lat, dip, s, th, ph)
            e = _rel(res["Zp"][fi], ref.Zp)
            _say("  %dx%d m%d s=%.2f |dZp|=%.2e" % (lat.nx, lat.ny, dip.nbases, s, e))
            assert e <= 1e-9
            assert np.max(np.abs(res["Gamma"][fi] - ref.Gamma) / np.maximum(1.0, np.abs(ref.Gamma))) <= 1e-8
    # requests submitted together ran concurrently
    spans = sorted((r["t_start"], r["t_done"]) for r in others + [inmix])
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    for r in others + [inmix]:
        assert r["t_submit"] <= r["t_start"] <= r["t_done"]


def test_served_mixed_precision_meets_refined_tolerance(ctx, cfg1):
    from paper_2608_17844_amd import mbt
    opts = mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK)
    freqs = [0.6, 1.3]
    srv = mbt.mbt_server_create(ctx, 2)
    try:
        res = mbt.mbt_server_wait(srv, _submit(mbt, srv, cfg1.dipole, cfg1.lattice, freqs, cfg1.theta, cfg1.phi,
                                               opts))
    finally:
        mbt.mbt_server_destroy(srv)
    assert res["status"] == mbt.MBT_OK
    for fi, s in enumerate(freqs):
        ref = mom.solve_array(cfg1.lattice, cfg1.dipole, s, cfg1.theta, cfg1.phi)
        assert _rel(res["Zp"][fi], ref.Zp) <= 1e-6
        assert np.max(np.abs(res["Gamma"][fi] - ref.Gamma)) <= 1e-6


def test_admission_by_memory_footprint_serialises_jobs(ctx, cfg1):
    from paper_2608_17844_amd import mbt
    P = cfg1.lattice.nx * cfg1.lattice.ny
    opts = mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK, rhs_chunk=P)
    arr = mbt.mbt_array_create_dipole(ctx, cfg1.dipole, cfg1.lattice)
    need = mbt.mbt_footprint(arr, P, opts)
    mbt.mbt_array_destroy(arr)
    # room for one job's buffers but not two
    srv = mbt.mbt_server_create(ctx, 3, int(1.3 * need))
    freqs = [0.7, 0.9, 1.1]
    try:
        tickets = [_submit(mbt, srv, cfg1.dipole, cfg1.lattice, [s], cfg1.theta, cfg1.phi, opts) for s in freqs]
        res = [mbt.mbt_server_wait(srv, t) for t in tickets]
    finally:
        mbt.mbt_server_destroy(srv)
    spans = sorted((r["t_start"], r["t_done"]) for r in res)
    for i in range(len(spans) - 1):
        assert spans[i + 1][0] >= spans[i][1] - 1e-6, spans
    srv = mbt.mbt_server_create(ctx, 3)
    try:
        free = mbt.mbt_server_wait(srv, _submit(mbt, srv, cfg1.dipole, cfg1.lattice, freqs, cfg1.theta, cfg1.phi,
                                                opts))
    finally:
        mbt.mbt_server_destroy(srv)
    for fi in range(3):
        assert res[fi]["status"] == mbt.MBT_OK
        assert np.max(np.abs(res[fi]["Zp"][0] - free["Zp"][fi])) <= 1e-12 * np.max(np.abs(free["Zp"][fi]))


def test_request_validation(ctx, cfg1):
    from paper_2608_17844_amd import mbt
    opts = mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK)
    srv = mbt.mbt_server_create(ctx, 1, 64 << 20)
    try:
        d = cfg1.dipole
        with pytest.raises(mbt.MbtError) as e:
            _submit(mbt, srv, d, W.Lattice(0, 5, 0.5, 0.5), [1.0], [], [], opts)
        assert e.value.status == mbt.MBT_EINVAL
        with pytest.raises(mbt.MbtError) as e:
            _submit(mbt, srv, d, cfg1.lattice, [-1.0], [], [], opts)
        assert e.value.status == mbt.MBT_EINVAL
        with pytest.raises(mbt.MbtError) as e:   # 48x48 elements of 31 bases cannot fit 64 MiB
            _submit(mbt, srv, W.Dipole(0.5, 0.005, 31), W.Lattice(48, 48, 0.5, 0.5), [1.0], [], [], opts)
        assert e.value.status == mbt.MBT_ENOMEM
        with pytest.raises(mbt.MbtError) as e:
            mbt.mbt_server_wait(srv, 12345)
        assert e.value.status == mbt.MBT_EINVAL
        # a request without scans still returns Z_p
        r = mbt.mbt_server_wait(srv, _submit(mbt, srv, d, W.Lattice(2, 3, 0.5, 0.5), [1.0], [], [], opts))
        assert r["status"] == mbt.MBT_OK and r["nscan"] == 0 and r["Zp"].shape == (1, 6, 6)
    finally:
        mbt.mbt_server_destroy(srv)


def test_unconverged_request_returns_its_last_iterate(ctx, cfg1, cfg1_oracle):
    """A request that cannot meet its tolerance within its cycle limit ends
    MBT_ENOCONV with finite outputs, and the server goes on serving."""
    from paper_2608_17844_amd import mbt
    srv = mbt.mbt_server_create(ctx, 2)
    try:
        tight = mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK, restart=2, max_cycles=1)
        _say("serving: request limited to one GMRES(2) cycle")
        r = mbt.mbt_server_wait(srv, _submit(mbt, srv, cfg1.dipole, cfg1.lattice, [1.0], cfg1.theta, cfg1.phi,
                                             tight))
        assert r["status"] == mbt.MBT_ENOCONV
        assert np.all(np.isfinite(r["Zp"])) and np.all(np.isfinite(r["Gamma"]))
        assert int(np.max(r["iters_max"])) == 2
        ok = mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK)
        r2 = mbt.mbt_server_wait(srv, _submit(mbt, srv, cfg1.dipole, cfg1.lattice, [1.0], cfg1.theta, cfg1.phi, ok))
        assert r2["status"] == mbt.MBT_OK
        assert _rel(r2["Zp"][0], cfg1_oracle.Zp) <= 1e-9
    finally:
        mbt.mbt_server_destroy(srv)


def test_concurrent_requests_extending_one_cached_operator(ctx):
    """Requests for the same array and frequency with different operator
    needs (FP32 with P_K, FP32 with P_A, FP64 with P_A, FP16 products) in flight at once:
    each extends the shared cached operator with the pieces it lacks while the
    others run kernels on the pieces that exist; every result matches the
    oracle."""
    from paper_2608_17844_amd import mbt
    lat, dip = W.Lattice(6, 5, 0.5, 0.5), W.Dipole(0.5, 0.005, 15)
    s = 1.07
    th, ph = W.scan_angles(5, seed=3)
    ref = mom.solve_array(lat, dip, s, th, ph)
    variants = [
        ("fp32 P_K", mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK, refine_tol=1e-11,
                                           refine_max=6), 1e-9),
        ("fp32 P_A", mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_NORMAL_EQ, refine_tol=1e-11,
                                           refine_max=6), 1e-9),
        ("fp64 P_A", mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_NORMAL_EQ, tol=1e-12), 1e-9),
        ("fp16 P_K", mbt.mbt_default_opts(prec=mbt.MBT_FP16, pc=mbt.MBT_PC_ELEMENT_BLOCK, refine_tol=1e-11,
                                           refine_max=8), 1e-9),
    ]
    srv = mbt.mbt_server_create(ctx, 4)
    try:
        tickets = [_submit(mbt, srv, dip, lat, [s], th, ph, o) for _, o, _ in variants]
        results = [mbt.mbt_server_wait(srv, t) for t in tickets]
    finally:
        mbt.mbt_server_destroy(srv)
    for (name, _, bound), res in zip(variants, results):
        e = _rel(res["Zp"][0], ref.Zp)
        _say("  %s: status %d |dZp|/|Zp| %.2e" % (name, res["status"], e))
        assert e <= bound, (name, e)
