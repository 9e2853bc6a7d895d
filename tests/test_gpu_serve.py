"""Served form: volumes streamed slab by slab must give exactly the outputs
of one plain fused call on the assembled volume (and so of the oracle), for
any slab sizes, interleaved volumes and host or device sources, under both
quantiser flows, and at the detector's slab shape (2048 x 2048 x 32 uint16
planes); and the request state machine must refuse what it should
(out-of-order, repeated or missing slabs, a full pool) without disturbing the
other volumes."""
import numpy as np
import pytest

import synth
from roixtest import compare_fused, criterion, default_caps, log, oracle_fused

pytestmark = pytest.mark.gpu


def _equal(a, b):
    for k in ("rows", "stream", "outliers", "comps"):
        assert a[k].tobytes() == b[k].tobytes(), k
    for k in ("qinfo", "sinfo", "einfo"):
        assert bytes(a[k]) == bytes(b[k]), k


@pytest.fixture(scope="module", params=["default", "onepass"])
def env(request):
    # "onepass": every float32 volume with an absolute bound that a server
    # reduces whole at close (and every plain reference) takes the one-pass
    # 16-bit-proxy flow, whatever its size
    import torch

    from paper_2602_15917_amd import roix
    ctx = roix.Context(0, 2 << 30)
    if request.param == "onepass":
        ctx.set_param("fused16_min_voxels", 0)
    yield ctx, roix, torch
    ctx.close()


def plain(env, vol, eb_mode, eb_value, crit):
    ctx, roix, torch = env
    caps = default_caps(roix, vol, crit)
    out = roix.Outputs("cuda:0", *caps)
    ctx.fused(torch.from_numpy(vol).to("cuda:0"), eb_mode, eb_value, crit, out)
    torch.cuda.synchronize()
    return out.collect(), caps


def slab_cuts(nz, sizes):
    """z0 positions cutting nz planes into slabs of the given sizes (cycled)."""
    cuts, z, k = [], 0, 0
    while z < nz:
        n = min(sizes[k % len(sizes)], nz - z)
        cuts.append((z, n))
        z += n
        k += 1
    return cuts


def server(roix, ctx, budget):
    """A server whose volumes get run arrays for the worst case, so that
    noise volumes never run out (the plain calls here have ample scratch)."""
    srv = roix.Server(ctx, budget)
    srv.set_param("runs_per_row", 1 << 30)
    return srv


def stream_volume(env, srv, vol, eb_mode, eb_value, crit, sizes, source="device"):
    ctx, roix, torch = env
    caps = default_caps(roix, vol, crit)
    out = roix.Outputs("cuda:0", *caps)
    dt = roix.F32 if vol.dtype == np.float32 else roix.U16
    vid = srv.open(vol.shape, dt, eb_mode, eb_value, crit, out)
    keep = []
    reqs = []
    for z0, n in slab_cuts(vol.shape[0], sizes):
        t = torch.from_numpy(np.ascontiguousarray(vol[z0:z0 + n]))
        t = t.to("cuda:0") if source == "device" else t.pin_memory()
        keep.append(t)
        reqs.append(srv.submit(vid, z0, t))
    for r in reqs:
        res = srv.wait(r)
        assert res.status == 0 and res.kind == roix.REQ_SLAB and res.latency_ms >= 0.0
    res = srv.wait(srv.close(vid))
    assert res.status == 0 and res.kind == roix.REQ_CLOSE
    torch.cuda.synchronize()
    return out.collect()


CASES = [
    # (name, volume factory, eb, criterion)
    ("cylinder f32 fixed 26", lambda: synth.cylinder1024(n=96).volume, ("abs", 1e-4),
     synth.Criterion("fixed", 0.3, 26, "largest", 1)),
    ("rings u16 fixed 6", lambda: synth.rings2048(nxy=160, nz=23).volume, ("abs", 3.0),
     synth.Criterion("fixed", 6400.0, 6, "min_size", 5)),
    ("noise f32 fixed 26", lambda: synth.normal((17, 41, 70), 7100, 0.5, 0.1), ("abs", 1e-3),
     synth.Criterion("fixed", 0.55, 26, "min_size", 1)),
    ("noise f32 fixed 6", lambda: synth.normal((13, 33, 129), 7101, 0.5, 0.1), ("abs", 1e-3),
     synth.Criterion("fixed", 0.5, 6, "largest", 1)),
    # a bound too fine for 2^15 code classes: kept whole, not as row extents
    ("rings u16 fixed 26 fine", lambda: synth.rings2048(nxy=128, nz=20).volume, ("abs", 0.4),
     synth.Criterion("fixed", 6400.0, 26, "largest", 1)),
]


@pytest.mark.parametrize("k", range(len(CASES)))
@pytest.mark.parametrize("sizes", [(1,), (7, 1, 3), (64,)])
def test_streamed_equals_plain(env, k, sizes):
    ctx, roix, torch = env
    name, make, (ebm, ebv), c = CASES[k]
    vol = make()
    crit = criterion(roix, c)
    log(f"[case] served {name} slabs={sizes} shape={vol.shape}")
    ref, _ = plain(env, vol, ebm, ebv, crit)
    srv = server(roix, ctx, 2 << 30)
    try:
        got = stream_volume(env, srv, vol, ebm, ebv, crit, sizes)
        _equal(got, ref)
        st = srv.stats()
        assert st.closes_done == 1 and st.volumes_open == 0 and st.bytes_in == vol.nbytes
    finally:
        srv.close_server()


def test_streamed_equals_oracle(env):
    ctx, roix, torch = env
    name, make, (ebm, ebv), c = CASES[2]
    vol = make()
    crit = criterion(roix, c)
    log(f"[case] served vs oracle {name}")
    srv = server(roix, ctx, 1 << 30)
    try:
        got = stream_volume(env, srv, vol, ebm, ebv, crit, (2, 5))
    finally:
        srv.close_server()
    compare_fused(got, oracle_fused(vol, ebm, ebv, c))


def test_host_pinned_source(env):
    ctx, roix, torch = env
    name, make, (ebm, ebv), c = CASES[0]
    vol = make()
    crit = criterion(roix, c)
    log("[case] served from pinned host memory")
    ref, _ = plain(env, vol, ebm, ebv, crit)
    srv = server(roix, ctx, 1 << 30)
    try:
        _equal(stream_volume(env, srv, vol, ebm, ebv, crit, (10, 3), source="host"), ref)
    finally:
        srv.close_server()


@pytest.mark.parametrize("thr,ebm", [("otsu", "abs"), ("fixed", "rel"), ("otsu", "rel")])
def test_deferred_volumes_equal_plain(env, thr, ebm):
    # an Otsu threshold or a relative bound needs the whole volume: reduced at close
    ctx, roix, torch = env
    w = synth.ellipsoids128()
    c = synth.Criterion(thr, 0.5, 6, "min_size", 64)
    ebv = w.eb_value if ebm == "abs" else 1e-3
    crit = criterion(roix, c)
    log(f"[case] served deferred thr={thr} eb={ebm}")
    ref, _ = plain(env, w.volume, ebm, ebv, crit)
    srv = server(roix, ctx, 1 << 30)
    try:
        _equal(stream_volume(env, srv, w.volume, ebm, ebv, crit, (16, 40)), ref)
    finally:
        srv.close_server()


def test_interleaved_volumes(env):
    ctx, roix, torch = env
    log("[case] served interleaved volumes")
    vols = [(CASES[0], CASES[0][1]()), (CASES[2], CASES[2][1]()), (CASES[1], CASES[1][1]())]
    refs, outs, ids, plans, keep = [], [], [], [], []
    srv = server(roix, ctx, 3 << 30)
    try:
        for (name, make, (ebm, ebv), c), vol in vols:
            crit = criterion(roix, c)
            refs.append(plain(env, vol, ebm, ebv, crit)[0])
            out = roix.Outputs("cuda:0", *default_caps(roix, vol, crit))
            dt = roix.F32 if vol.dtype == np.float32 else roix.U16
            ids.append(srv.open(vol.shape, dt, ebm, ebv, crit, out))
            outs.append(out)
            plans.append(slab_cuts(vol.shape[0], (5, 2)))
        reqs = []
        step = 0
        while any(plans):
            for i, ((case, vol), plan) in enumerate(zip(vols, plans)):
                if step < len(plan):
                    z0, n = plan[step]
                    t = torch.from_numpy(np.ascontiguousarray(vol[z0:z0 + n])).to("cuda:0")
                    keep.append(t)
                    reqs.append(srv.submit(ids[i], z0, t))
            step += 1
            if all(step >= len(p) for p in plans):
                break
        closes = [srv.close(v) for v in ids]
        for r in reqs + closes:
            assert srv.wait(r).status == 0
        torch.cuda.synchronize()
        for out, ref in zip(outs, refs):
            _equal(out.collect(), ref)
        assert srv.stats().closes_done == 3
    finally:
        srv.close_server()


def test_nonfinite_voxel_statuses_equal_plain(env):
    ctx, roix, torch = env
    name, make, (ebm, ebv), c = CASES[2]
    vol = make()
    vol[9, 3, 5] = np.nan
    crit = criterion(roix, c)
    log("[case] served NaN voxel")
    ref, _ = plain(env, vol, ebm, ebv, crit)
    srv = server(roix, ctx, 1 << 30)
    try:
        got = stream_volume(env, srv, vol, ebm, ebv, crit, (4,))
    finally:
        srv.close_server()
    for k in ("qinfo", "sinfo", "einfo"):
        assert bytes(got[k]) == bytes(ref[k]), k
    assert got["qinfo"].status == roix.EINVAL


def test_sequence_errors_and_admission(env):
    ctx, roix, torch = env
    log("[case] served request errors and admission")
    vol = synth.normal((8, 16, 40), 7200, 0.5, 0.1)
    c = synth.Criterion("fixed", 0.5, 6, "min_size", 1)
    crit = criterion(roix, c)
    probe = roix.Server(ctx, 1 << 20)
    need = probe.volume_bytes(vol.shape, roix.F32, "abs", 1e-3, crit)
    whole = probe.volume_bytes(vol.shape, roix.F32, "abs", 1e-3, criterion(roix, synth.Criterion()))
    assert need > vol.nbytes and whole - need >= vol.size  # only the deferred path holds the proxy
    assert probe.volume_bytes((0, 4, 4), roix.F32, "abs", 1e-3, crit) == 0
    probe.close_server()
    srv = roix.Server(ctx, need + need // 2)  # room for one such volume, not two
    try:
        out = roix.Outputs("cuda:0", *default_caps(roix, vol, crit))
        vid = srv.open(vol.shape, roix.F32, "abs", 1e-3, crit, out)
        with pytest.raises(roix.RoixError) as e:
            srv.open(vol.shape, roix.F32, "abs", 1e-3, crit, roix.Outputs("cuda:0", *default_caps(roix, vol, crit)))
        assert e.value.status == roix.EBUSY
        d = torch.from_numpy(vol).to("cuda:0")
        with pytest.raises(roix.RoixError) as e:       # first slab must start at 0
            srv.submit(vid, 2, d[2:4])
        assert e.value.status == roix.ESEQ
        with pytest.raises(roix.RoixError) as e:       # beyond the volume
            srv.submit(vid, 0, torch.zeros((9, 16, 40), dtype=torch.float32, device="cuda:0"))
        assert e.value.status == roix.EINVAL
        r1 = srv.submit(vid, 0, d[0:3])
        with pytest.raises(roix.RoixError) as e:       # repeated slab
            srv.submit(vid, 0, d[0:3])
        assert e.value.status == roix.ESEQ
        with pytest.raises(roix.RoixError) as e:       # slabs missing
            srv.close(vid)
        assert e.value.status == roix.ESEQ
        with pytest.raises(roix.RoixError) as e:       # unknown volume
            srv.submit(vid + 100, 3, d[3:4])
        assert e.value.status == roix.EINVAL
        r2 = srv.submit(vid, 3, d[3:8])
        rc = srv.close(vid)
        with pytest.raises(roix.RoixError) as e:       # already closed
            srv.close(vid)
        assert e.value.status == roix.ESEQ
        for r in (r1, r2, rc):
            assert srv.wait(r).status == 0
        with pytest.raises(roix.RoixError):            # a request is forgotten once waited for
            srv.wait(r1)
        torch.cuda.synchronize()
        ref, _ = plain(env, vol, "abs", 1e-3, crit)
        _equal(out.collect(), ref)
        # the pool is free again: admitted, then aborted, then admitted again
        vid2 = srv.open(vol.shape, roix.F32, "abs", 1e-3, crit, roix.Outputs("cuda:0", *default_caps(roix, vol, crit)))
        srv.submit(vid2, 0, d[0:2])
        srv.abort(vid2)
        with pytest.raises(roix.RoixError) as e:
            srv.submit(vid2, 2, d[2:4])
        assert e.value.status in (roix.ESEQ, roix.EINVAL)
        torch.cuda.synchronize()
        vid3 = srv.open(vol.shape, roix.F32, "abs", 1e-3, crit, roix.Outputs("cuda:0", *default_caps(roix, vol, crit)))
        srv.abort(vid3)
        st = srv.stats()
        assert st.volumes_admitted == 3 and st.volumes_refused == 1 and st.closes_done == 1
        assert st.slab_p50_ms > 0.0 and st.slab_p99_ms >= st.slab_p50_ms
    finally:
        srv.close_server()


def test_run_capacity_error_is_isolated(env):
    # a volume with more runs than its arrays hold reports ENOMEM at close;
    # the next volume on the same server is unaffected
    ctx, roix, torch = env
    log("[case] served run capacity")
    noisy = synth.normal((6, 20, 200), 7300, 0.5, 0.1)
    c = criterion(roix, synth.Criterion("fixed", 0.5, 6, "min_size", 1))
    srv = roix.Server(ctx, 1 << 30)
    try:
        srv.set_param("runs_per_row", 2)
        got = stream_volume(env, srv, noisy, "abs", 1e-3, c, (2,))
        assert got["sinfo"].status == roix.ENOMEM and got["einfo"].status == roix.ENOMEM
        assert got["qinfo"].status == 0
        srv.set_param("runs_per_row", 1 << 30)
        name, make, (ebm, ebv), cc = CASES[0]
        vol = make()
        crit = criterion(roix, cc)
        ref, _ = plain(env, vol, ebm, ebv, crit)
        _equal(stream_volume(env, srv, vol, ebm, ebv, crit, (9,)), ref)
    finally:
        srv.close_server()


def test_detector_slab_shape_equals_plain(env):
    """uint16 2048 x 2048 planes in 32-plane slabs from pinned host memory
    (ring-artefact cylinder; ABS bound = 1e-4 x a calibration volume's range;
    FIXED threshold 6400; 26-connectivity; largest component), interleaved
    with a float32 cube sent whole, each equal to its plain call."""
    ctx, roix, torch = env
    calib = synth.served_calibration(nz=4)
    eb = 1e-4 * (float(calib.max()) - float(calib.min()))
    crit = roix.Criterion("fixed", 6400.0, 26, "largest", 1)
    vol = synth.served_stream(0, nz=96)
    cube = synth.served_cube(1, side=(128, 160))
    ccrit = criterion(roix, cube.criterion)
    log(f"[case] served detector slabs {vol.shape} eb={eb:.4g} + cube {cube.volume.shape}")
    ref, caps = plain(env, vol, "abs", eb, crit)
    cref, ccaps = plain(env, cube.volume, cube.eb_mode, cube.eb_value, ccrit)
    srv = roix.Server(ctx, 8 << 30)
    try:
        out = roix.Outputs("cuda:0", *caps)
        cout = roix.Outputs("cuda:0", *ccaps)
        vid = srv.open(vol.shape, roix.U16, "abs", eb, crit, out)
        reqs, keep = [], []
        for k, z0 in enumerate(range(0, vol.shape[0], 32)):
            t = torch.from_numpy(np.ascontiguousarray(vol[z0:z0 + 32])).pin_memory()
            keep.append(t)
            reqs.append(srv.submit(vid, z0, t))
            if k == 1:  # the cube arrives between two slabs
                cid = srv.open(cube.volume.shape, roix.F32, cube.eb_mode, cube.eb_value, ccrit, cout)
                ct = torch.from_numpy(cube.volume).pin_memory()
                keep.append(ct)
                reqs.append(srv.submit(cid, 0, ct))
                reqs.append(srv.close(cid))
        reqs.append(srv.close(vid))
        for r in reqs:
            assert srv.wait(r).status == 0
        torch.cuda.synchronize()
        got = out.collect()
        assert got["einfo"].status == 0 and got["einfo"].n_codes > 0 and got["sinfo"].n_components >= 1
        _equal(got, ref)
        _equal(cout.collect(), cref)
        st = srv.stats()
        assert st.slabs_done == 3 + 1 and st.closes_done == 2
    finally:
        srv.close_server()


@pytest.mark.parametrize("planes", [1, 3, 32])
def test_row_extent_store_staged_in_chunks(env, planes):
    """A uint16 stream kept as row extents, staged a few planes at a time
    (slabs larger than the stage go in turn), equals plain."""
    ctx, roix, torch = env
    name, make, (ebm, ebv), c = CASES[1]
    vol = make()
    crit = criterion(roix, c)
    log(f"[case] served row extents, {planes} planes staged")
    ref, _ = plain(env, vol, ebm, ebv, crit)
    srv = server(roix, ctx, 2 << 30)
    try:
        srv.set_param("slab_planes", planes)
        for sizes in ((7, 1, 3), (23,)):
            _equal(stream_volume(env, srv, vol, ebm, ebv, crit, sizes, source="host"), ref)
    finally:
        srv.close_server()


def test_row_extent_store_bytes_and_overflow(env):
    ctx, roix, torch = env
    log("[case] served row-extent store: size and overflow")
    srv = roix.Server(ctx, 1 << 30)
    try:
        crit = roix.Criterion("fixed", 6400.0, 26, "largest", 1)
        shape = (1024, 2048, 2048)
        srv.set_param("runs_per_row", 4)
        compact = srv.volume_bytes(shape, roix.U16, "abs", 1.24, crit)
        whole = srv.volume_bytes(shape, roix.U16, "abs", 0.4, crit)
        assert 0 < compact * 1.8 < whole, (compact, whole)  # default store: half the voxels
        # a store of 32 % of the voxels: the cylinder's share of the field of view (30 %) and a margin
        srv.set_param("store_permille", 320)
        assert srv.volume_bytes(shape, roix.U16, "abs", 1.24, crit) * 2.6 < whole
        srv.set_param("runs_per_row", 32)
        # a store too small for the extents fails that volume only
        name, make, (ebm, ebv), c = CASES[1]
        vol = make()
        cr = criterion(roix, c)
        srv.set_param("store_permille", 1)
        got = stream_volume(env, srv, vol, ebm, ebv, cr, (5,))
        assert got["sinfo"].status == roix.ENOMEM and got["einfo"].status == roix.ENOMEM
        assert got["qinfo"].status == 0
        srv.set_param("store_permille", 500)
        ref, _ = plain(env, vol, ebm, ebv, cr)
        _equal(stream_volume(env, srv, vol, ebm, ebv, cr, (5,)), ref)
    finally:
        srv.close_server()
