"""Device tests of the serving path (sccg_server_*): every job's per-pair
counts and set sums equal the oracle's; a job gives the same result alone
and in a mix; arenas that are too small for the offered load make jobs wait
and wrap, without changing any result; error paths report per job.  All
calls go through the C ABI."""

import time

import numpy as np
import pytest

import oracle
import paper_1208_0277_amd as sccg
import sccg_gen

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)


@pytest.fixture(scope="module")
def corpus():
    """Uniform-mix pairs (A_i, B_i); a job is the window [s, s + n)."""
    wl = sccg_gen.pairs(2, 20000, seed=sccg_gen.BASE_SEED + 50)
    assert np.array_equal(wl.pa, np.arange(wl.n_pairs)) and np.array_equal(wl.pb, np.arange(wl.n_pairs))
    I, U = oracle.area_pairs(wl.A, wl.B, wl.pa, wl.pb, form=oracle.ROWS)
    return wl, I, U


def window(wl, s, n, pinned=None):
    """Host job arrays for pairs [s, s+n): offsets slices of the corpus CSR
    (not starting at 0) over the whole vertex arrays."""
    a_xy, b_xy = (pinned if pinned is not None else (wl.A.xy, wl.B.xy))
    a_off = np.ascontiguousarray(wl.A.off[s:s + n + 1])
    b_off = np.ascontiguousarray(wl.B.off[s:s + n + 1])
    pa = np.arange(n, dtype=np.int32)
    pb = np.arange(n, dtype=np.int32)
    return a_off, a_xy.reshape(-1), b_off, b_xy.reshape(-1), pa, pb


def expected_sets(I, U, flags=sccg.SCCG_J_NONZERO_ONLY):
    si, su, nn, j, jp = oracle.jaccard_sets(np.array([0, len(I)], np.int64), I, U,
                                            include_zero=(flags == sccg.SCCG_J_INCLUDE_ZERO))
    return int(si[0]), int(su[0]), int(nn[0]), float(j[0]), float(jp[0])


def collect(srv, n, deadline_s=120.0):
    out = {}
    t_end = time.time() + deadline_s
    while len(out) < n:
        got = srv.poll(256, timeout=5.0)
        for r in got:
            out[r["job_id"]] = r
        assert time.time() < t_end, f"only {len(out)} of {n} jobs finished in {deadline_s} s"
    return out


def check_job(r, outs, wl_res, s, n, flags=sccg.SCCG_J_NONZERO_ONLY):
    I, U = wl_res
    gi, gu = outs
    assert r["status"] == sccg.SCCG_OK
    assert r["n_pairs"] == n
    assert np.array_equal(gi, I[s:s + n]) and np.array_equal(gu, U[s:s + n]), f"job window {s}+{n} counts differ"
    si, su, nn, j, jp = expected_sets(I[s:s + n], U[s:s + n], flags)
    assert (r["sum_i"], r["sum_u"], r["n_contrib"]) == (si, su, nn)
    assert r["j"] == j and r["jprime"] == jp
    assert r["t_submit"] <= r["t_admit"] <= r["t_launch"] <= r["t_done"]


def submit_windows(srv, wl, windows, pinned=None):
    jobs = {}
    for (s, n) in windows:
        oi = np.zeros(n, np.int64)
        ou = np.zeros(n, np.int64)
        jid = srv.submit(*window(wl, s, n, pinned), out_inter=oi, out_union=ou)
        jobs[jid] = (s, n, oi, ou)
    return jobs


def test_jobs_exact_and_merged(corpus):
    wl, I, U = corpus
    rng = np.random.default_rng(11)
    windows = []
    for _ in range(60):
        n = int(np.exp(rng.uniform(np.log(1), np.log(3000))))
        s = int(rng.integers(0, wl.n_pairs - n))
        windows.append((s, n))
    srv = sccg.Server(0)
    try:
        jobs = submit_windows(srv, wl, windows)
        res = collect(srv, len(jobs))
        for jid, (s, n, oi, ou) in jobs.items():
            check_job(res[jid], (oi, ou), (I, U), s, n)
        st = srv.stats()
        assert st["jobs_done"] == len(jobs) and st["pairs_done"] == sum(n for _, n in windows)
        assert st["launches"] < len(jobs), "jobs submitted together were not merged into shared launches"
        assert st["max_jobs_per_launch"] > 1
    finally:
        srv.close()


def test_small_arenas_wait_and_wrap(corpus):
    """Arenas hold only a few jobs: jobs wait for admission, ranges wrap, and
    launches are bounded by max_step_pairs; results do not change."""
    wl, I, U = corpus
    rng = np.random.default_rng(12)
    windows = [(int(rng.integers(0, wl.n_pairs - 800)), int(rng.integers(1, 800))) for _ in range(80)]
    vmax = max(int(wl.A.off[s + n] - wl.A.off[s] + wl.B.off[s + n] - wl.B.off[s]) for s, n in windows)
    srv = sccg.Server(0, vertex_cap=int(vmax * 2.5), slot_cap=4000, pair_cap=2000, max_step_pairs=700,
                      max_inflight=2)
    try:
        jobs = submit_windows(srv, wl, windows)
        res = collect(srv, len(jobs))
        for jid, (s, n, oi, ou) in jobs.items():
            check_job(res[jid], (oi, ou), (I, U), s, n)
        st = srv.stats()
        assert st["admission_waits"] > 0
        assert st["peak_resident_pairs"] <= 2000 and st["peak_resident_vertices"] <= int(vmax * 2.5)
    finally:
        srv.close()


def test_alone_equals_in_mix(corpus):
    wl, I, U = corpus
    probe = (1234, 2500)
    srv = sccg.Server(0)
    try:
        alone = submit_windows(srv, wl, [probe])
        r_alone = collect(srv, 1)
        rng = np.random.default_rng(13)
        mix = [(int(rng.integers(0, wl.n_pairs - 2000)), int(rng.integers(1, 2000))) for _ in range(30)]
        mix.insert(15, probe)
        jobs = submit_windows(srv, wl, mix)
        res = collect(srv, len(jobs))
    finally:
        srv.close()
    (ja, (s, n, oi_a, ou_a)), = alone.items()
    check_job(r_alone[ja], (oi_a, ou_a), (I, U), s, n)
    probes = [(jid, v) for jid, v in jobs.items() if (v[0], v[1]) == probe]
    assert probes
    for jid, (s, n, oi, ou) in probes:
        assert np.array_equal(oi, oi_a) and np.array_equal(ou, ou_a)
        for k in ("sum_i", "sum_u", "n_contrib", "j", "jprime"):
            assert res[jid][k] == r_alone[ja][k]
    assert any(res[jid]["jobs_in_launch"] > 1 for jid, _ in probes) or len(jobs) > 1


def bad_window(wl, s, n, k):
    """Job arrays for pairs [s, s + n) whose k-th A polygon lies beyond the
    2^30 coordinate limit: that polygon counts as empty and the job reports
    SCCG_E_RANGE."""
    a_off, a_xy, b_off, b_xy, pa, pb = window(wl, s, n)
    xy = a_xy.reshape(-1, 2).copy()
    xy[int(a_off[k]):int(a_off[k + 1]), 0] += (1 << 30) + 5
    return a_off, xy.reshape(-1), b_off, b_xy, pa, pb


def test_status_alone_equals_in_mix(corpus):
    """A job whose pairs latch a range error reports SCCG_E_RANGE, and the
    same counts, alone and in a launch shared with good jobs, which report
    SCCG_OK and exact counts."""
    wl, I, U = corpus
    arrs = bad_window(wl, 4000, 300, 7)
    srv = sccg.Server(0, max_inflight=1)
    try:
        oi_a, ou_a = np.zeros(300, np.int64), np.zeros(300, np.int64)
        ja = srv.submit(*arrs, out_inter=oi_a, out_union=ou_a)
        r_alone = collect(srv, 1)[ja]
        # a large job keeps the device busy while the rest queue and merge
        jobs = submit_windows(srv, wl, [(0, 15000)])
        jobs.update(submit_windows(srv, wl, [(15000 + 100 * k, 90) for k in range(8)]))
        oi_m, ou_m = np.zeros(300, np.int64), np.zeros(300, np.int64)
        jm = srv.submit(*arrs, out_inter=oi_m, out_union=ou_m)
        jobs.update(submit_windows(srv, wl, [(16000 + 100 * k, 90) for k in range(8)]))
        res = collect(srv, len(jobs) + 1)
    finally:
        srv.close()
    assert r_alone["status"] == sccg.SCCG_E_RANGE
    assert res[jm]["status"] == sccg.SCCG_E_RANGE
    assert res[jm]["jobs_in_launch"] > 1, "the bad job ran alone: the mix was not exercised"
    assert np.array_equal(oi_m, oi_a) and np.array_equal(ou_m, ou_a)
    # the out-of-range polygon counts as empty: I = 0, U = |B|
    rb = wl.B.ring(4007).astype(np.int64)
    area_b = abs(int(np.sum(rb[:, 0] * np.roll(rb[:, 1], -1) - np.roll(rb[:, 0], -1) * rb[:, 1]))) // 2
    assert oi_a[7] == 0 and ou_a[7] == area_b
    keep = np.arange(300) != 7
    assert np.array_equal(oi_a[keep], I[4000:4300][keep]) and np.array_equal(ou_a[keep], U[4000:4300][keep])
    for k in ("sum_i", "sum_u", "n_contrib", "j", "jprime"):
        assert res[jm][k] == r_alone[k]
    for jid, (s, n, oi, ou) in jobs.items():
        check_job(res[jid], (oi, ou), (I, U), s, n)


def test_pinned_corpus(corpus):
    import torch
    wl, I, U = corpus
    pa_xy = torch.empty(wl.A.xy.shape, dtype=torch.int32, pin_memory=True).numpy()
    pb_xy = torch.empty(wl.B.xy.shape, dtype=torch.int32, pin_memory=True).numpy()
    pa_xy[...] = wl.A.xy
    pb_xy[...] = wl.B.xy
    windows = [(0, 5000), (7000, 3000), (15000, 4999)]
    srv = sccg.Server(0)
    try:
        jobs = submit_windows(srv, wl, windows, pinned=(pa_xy, pb_xy))
        res = collect(srv, len(jobs))
        for jid, (s, n, oi, ou) in jobs.items():
            check_job(res[jid], (oi, ou), (I, U), s, n)
    finally:
        srv.close()


def test_empty_job_and_argument_errors(corpus):
    wl, I, U = corpus
    srv = sccg.Server(0, vertex_cap=100000, slot_cap=1000, pair_cap=1000)
    try:
        a_off, a_xy, b_off, b_xy, pa, pb = window(wl, 10, 5)
        jid = srv.submit(a_off, a_xy, b_off, b_xy, pa[:0], pb[:0])
        r = collect(srv, 1)[jid]
        assert r["status"] == sccg.SCCG_OK and r["n_pairs"] == 0 and r["sum_u"] == 0 and r["j"] == 0.0
        bad = pa.copy()
        bad[2] = 5  # A of this job has 5 polygons: index 5 is out of range
        with pytest.raises(sccg.SccgError) as e:
            srv.submit(a_off, a_xy, b_off, b_xy, bad, pb)
        assert e.value.code == sccg.SCCG_E_ARG
        dec = a_off.copy()
        dec[3] = dec[2] - 1
        with pytest.raises(sccg.SccgError) as e:
            srv.submit(dec, a_xy, b_off, b_xy, pa, pb)
        assert e.value.code == sccg.SCCG_E_ARG
        big = window(wl, 0, 1500)
        with pytest.raises(sccg.SccgError) as e:
            srv.submit(*big)
        assert e.value.code == sccg.SCCG_E_NOMEM
        # the server still serves after rejected submissions
        jobs = submit_windows(srv, wl, [(100, 50)])
        res = collect(srv, 1)
        for jid, (s, n, oi, ou) in jobs.items():
            check_job(res[jid], (oi, ou), (I, U), s, n)
        assert srv.stats()["jobs_rejected"] == 1
    finally:
        srv.close()


def test_range_error_is_reported_per_launch(corpus):
    wl, I, U = corpus
    # a job whose polygons reach beyond 2^30: its launch latches SCCG_E_RANGE
    far = np.array([[0, 0], [10, 0], [10, 10], [0, 10]], np.int32) + np.int32((1 << 30) + 5)
    ring = np.array([[0, 0], [4, 0], [4, 4], [0, 4]], np.int32) + np.int32((1 << 30) + 5)
    off = np.array([0, 4], np.int64)
    srv = sccg.Server(0)
    try:
        jid = srv.submit(off, far.reshape(-1), off, ring.reshape(-1), np.zeros(1, np.int32), np.zeros(1, np.int32))
        r = collect(srv, 1)[jid]
        assert r["status"] == sccg.SCCG_E_RANGE
        # the error word is cleared for the next launch
        jobs = submit_windows(srv, wl, [(500, 300)])
        res = collect(srv, 1)
        for j2, (s, n, oi, ou) in jobs.items():
            check_job(res[j2], (oi, ou), (I, U), s, n)
    finally:
        srv.close()


@pytest.mark.parametrize("flags", [sccg.SCCG_J_NONZERO_ONLY, sccg.SCCG_J_INCLUDE_ZERO])
def test_migration_to_host_threads(corpus, flags):
    """Arenas too small for the offered load: jobs wait for admission, and the
    smallest waiting ones (at most cpu_max_pairs) run on host threads.  Every
    job, migrated or not, equals the oracle bit for bit, J' included."""
    wl, I, U = corpus
    rng = np.random.default_rng(21)
    windows = [(int(rng.integers(0, wl.n_pairs - 800)), int(rng.integers(1, 800))) for _ in range(80)]
    vmax = max(int(wl.A.off[s + n] - wl.A.off[s] + wl.B.off[s + n] - wl.B.off[s]) for s, n in windows)
    srv = sccg.Server(0, vertex_cap=int(vmax * 2.5), slot_cap=4000, pair_cap=2000, max_step_pairs=700,
                      max_inflight=2, jaccard_flags=flags, cpu_threads=4, cpu_trigger=1, cpu_max_pairs=400)
    try:
        jobs = submit_windows(srv, wl, windows)
        res = collect(srv, len(jobs))
        for jid, (s, n, oi, ou) in jobs.items():
            check_job(res[jid], (oi, ou), (I, U), s, n, flags)
        st = srv.stats()
    finally:
        srv.close()
    moved = [jid for jid, r in res.items() if r["jobs_in_launch"] == 0]
    assert st["admission_waits"] > 0
    assert st["jobs_migrated"] == len(moved) > 0
    assert st["pairs_migrated"] == sum(jobs[jid][1] for jid in moved)
    assert all(jobs[jid][1] <= 400 for jid in moved)
    assert st["jobs_done"] == len(windows) and st["pairs_done"] == sum(n for _, n in windows)


def test_migration_off_by_default(corpus):
    wl, I, U = corpus
    srv = sccg.Server(0, vertex_cap=200000, slot_cap=4000, pair_cap=2000, max_step_pairs=700)
    try:
        rng = np.random.default_rng(22)
        jobs = submit_windows(srv, wl, [(int(rng.integers(0, 19000)), int(rng.integers(1, 800))) for _ in range(30)])
        res = collect(srv, len(jobs))
        for jid, (s, n, oi, ou) in jobs.items():
            check_job(res[jid], (oi, ou), (I, U), s, n)
        st = srv.stats()
    finally:
        srv.close()
    assert st["jobs_migrated"] == 0 and all(r["jobs_in_launch"] >= 1 for r in res.values())
