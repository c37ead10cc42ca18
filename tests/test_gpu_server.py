"""Serving runtime through the C ABI: every job's records and final spins
are bit for bit those of a plain sim run alone, whatever else shares the
GPU, including jobs admitted mid-run and jobs that wait for memory."""
import math

import numpy as np
import pytest

import oracle
import paper_2302_14720_amd as sw

pytestmark = pytest.mark.gpu

BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0
FIELDS = ("sweep", "e_sum", "energy", "m_sum", "n_clusters", "max_cluster", "sum_sq_sizes")


def _same_records(a, b, where):
    assert len(a) == len(b), where
    for f in FIELDS:
        bad = np.nonzero(a[f] != b[f])[0]
        assert bad.size == 0, f"{where} field {f}: first mismatch at record {bad[0]}"
    assert np.array_equal(a["hist_log2"], b["hist_log2"]), f"{where} hist_log2"


def _solo(L, beta, seed, n, cold=False):
    with sw.Sim(L, beta, 1.0, seed, init=sw.SW_INIT_COLD if cold else sw.SW_INIT_HOT) as s:
        s.sweep(n)
        return s.series(0, n), s.spins()


def _drain(srv, n=5, limit=10000, collect=None):
    """Steps until no job is queued or active; finished jobs are handed to
    collect(job_id) (which may read and release them) as they finish."""
    done = []
    for _ in range(limit):
        st = srv.status()
        if st["queued"] == 0 and st["active"] == 0:
            return done
        fin = srv.step(n)
        done += fin
        if collect:
            for j in fin:
                collect(j)
    raise AssertionError("server did not drain")


JOBS = [  # L, beta, seed, sweeps, cold
    (64, BETA_C, 31, 17, False),
    (96, 0.35, 32, 9, False),
    (128, 0.60, 33, 23, True),
    (160, BETA_C, 34, 12, False),
    (256, 0.44, 35, 30, False),
    (64, 0.0, 36, 4, False),
    (192, 5.0, 37, 8, False),
]


def test_mixed_jobs_match_solo_runs():
    # a pool that holds only some jobs at once, so later ones wait for memory
    need = [sw.Server.job_bytes(L, n) for (L, _, _, n, _) in JOBS]
    pool = sum(sorted(need)[-3:]) + 4096
    print(f"\n[case] server pool={pool} jobs={len(JOBS)}", flush=True)
    with sw.Server(pool, max_jobs=4) as srv:
        ids = [srv.submit(L, b, 1.0, s, n, sw.SW_INIT_COLD if c else sw.SW_INIT_HOT) for (L, b, s, n, c) in JOBS]
        results = {}

        def collect(jid):
            info = srv.info(jid)
            assert info["state"] == sw.SW_JOB_DONE
            results[jid] = (info, srv.series(jid, 0, info["sweeps_done"]), srv.spins(jid))
            srv.release(jid)

        done = _drain(srv, 5, collect=collect)
        assert sorted(done) == sorted(ids)
        assert srv.status()["bytes_used"] == 0
    for jid, (L, b, s, n, c) in zip(ids, JOBS):
        info, got, spins = results[jid]
        assert info["sweeps_done"] == n and info["L"] == L
        ref, sp = _solo(L, b, s, n, c)
        _same_records(got, ref, f"job L={L} seed={s}")
        assert np.array_equal(spins, sp)
        if L <= 96:
            osp = oracle.init(L, s, cold=c)
            orec = oracle.run(L, 1.0, oracle.threshold(b, 1.0), s, 0, n, osp)
            _same_records(got, orec, f"job L={L} vs oracle")
            assert np.array_equal(spins, osp)


def test_job_admitted_mid_run():
    print("\n[case] server mid-run admission", flush=True)
    with sw.Server(1 << 28, max_jobs=8) as srv:
        a = srv.submit(128, BETA_C, 1.0, 41, 40)
        srv.step(13)
        assert srv.info(a)["sweeps_done"] == 13
        b = srv.submit(96, 0.5, 1.0, 42, 21)
        c = srv.submit(256, 0.42, 1.0, 43, 5)
        _drain(srv, 7)
        for jid, (L, beta, seed, n) in ((a, (128, BETA_C, 41, 40)), (b, (96, 0.5, 42, 21)),
                                        (c, (256, 0.42, 43, 5))):
            ref, sp = _solo(L, beta, seed, n)
            _same_records(srv.series(jid, 0, n), ref, f"job {jid}")
            assert np.array_equal(srv.spins(jid), sp)


def test_server_errors():
    print("\n[case] server errors", flush=True)
    with sw.Server(1 << 24, max_jobs=2) as srv:
        with pytest.raises(sw.SwError) as e:
            srv.submit(4096, 0.4, 1.0, 1, 10)  # larger than the whole pool
        assert e.value.code == sw.SW_ENOMEM
        with pytest.raises(sw.SwError) as e:
            srv.submit(100, 0.4, 1.0, 1, 10)
        assert e.value.code == sw.SW_EINVAL
        with pytest.raises(sw.SwError) as e:
            srv.info(12345)
        assert e.value.code == sw.SW_ERANGE
        j = srv.submit(64, 0.4, 1.0, 1, 10)
        srv.step(3)
        with pytest.raises(sw.SwError) as e:
            srv.release(j)
        assert e.value.code == sw.SW_ESTATE
        with pytest.raises(sw.SwError) as e:
            srv.spins(j)
        assert e.value.code == sw.SW_ESTATE
        with pytest.raises(sw.SwError) as e:
            srv.series(j, 0, 4)
        assert e.value.code == sw.SW_ERANGE
        with pytest.raises(sw.SwError) as e:  # the active job's last record is not complete yet
            srv.series(j, 2, 1)
        assert e.value.code == sw.SW_ERANGE
        assert len(srv.series(j, 0, 2)) == 2
        for bad_q in (1, 9, -3):  # Potts q outside [2, 8]
            with pytest.raises(sw.SwError) as e:
                srv.submit(64, 1.0, 1.0, 1, 10, q=bad_q)
            assert e.value.code == sw.SW_EINVAL and "q" in str(e.value)
        with pytest.raises(sw.SwError) as e:
            srv.submit(100, 1.0, 1.0, 1, 10, q=5)  # not a multiple of 32
        assert e.value.code == sw.SW_EINVAL
        with pytest.raises(sw.SwError) as e:
            srv.submit(4096, 1.0, 1.0, 1, 10, q=3)  # larger than the whole pool
        assert e.value.code == sw.SW_ENOMEM
        with pytest.raises(sw.SwError) as e:
            srv.submit(64, 1.0, 1.0, 1, 0, q=3)
        assert e.value.code == sw.SW_EINVAL
        q = srv.submit(64, 0.4, 1.0, 2, 10)
        srv.release(q)  # a queued job can be withdrawn
        _drain(srv)
        srv.release(j)


def test_ising_and_potts_jobs_share_the_server():
    """Ising jobs and q-state Potts jobs (64-wide tiles for q <= 4, 32-wide
    above) in one pool: every job's records and spins are those of a plain
    sim run alone, and for small lattices of the oracle."""
    jobs = [  # L, beta, seed, sweeps, q
        (64, BETA_C, 51, 11, 0),
        (128, math.log(1.0 + math.sqrt(3.0)), 52, 14, 3),
        (96, 0.9, 53, 9, 5),
        (192, 1.2, 54, 7, 2),
        (64, 1.5, 55, 13, 8),
        (160, 0.4, 56, 6, 0),
    ]
    need = [sw.Server.job_bytes(L, n, q) for (L, _, _, n, q) in jobs]
    assert all(x > 0 for x in need)
    print(f"\n[case] server Ising + Potts jobs, pool={sum(need)}", flush=True)
    with sw.Server(sum(sorted(need)[-4:]) + 4096, max_jobs=4) as srv:
        ids = [srv.submit(L, b, 1.0, s, n, q=q) for (L, b, s, n, q) in jobs]
        results = {}

        def collect(jid):
            info = srv.info(jid)
            results[jid] = (srv.series(jid, 0, info["sweeps_done"]), srv.spins(jid))
            srv.release(jid)

        done = _drain(srv, 4, collect=collect)
        assert sorted(done) == sorted(ids)
    for jid, (L, b, s, n, q) in zip(ids, jobs):
        got, spins = results[jid]
        with sw.Sim(L, b, 1.0, s, q=q) as solo:
            solo.sweep(n)
            ref, sp = solo.series(0, n), solo.spins()
        _same_records(got, ref, f"job L={L} q={q}")
        assert np.array_equal(spins, sp)
        if q and L <= 96:
            osp = oracle.potts_init(L, s, q)
            orec = oracle.potts_run(L, 1.0, oracle.potts_threshold(b, 1.0), q, s, 0, n, osp)
            _same_records(got, orec, f"job L={L} q={q} vs oracle")
            assert np.array_equal(spins, osp)


def test_active_job_series_mid_run():
    """Records of a job that is still running: 0 .. done-2 are complete and
    equal the solo run's; record done-1 is refused until the next sweep."""
    print("\n[case] server series of an active job", flush=True)
    L, beta, seed, n = 128, BETA_C, 61, 30
    ref, sp = _solo(L, beta, seed, n)
    with sw.Server(1 << 26, max_jobs=4) as srv:
        j = srv.submit(L, beta, 1.0, seed, n)
        done = 0
        for k in (1, 6, 9):
            srv.step(k)
            done += k
            assert srv.info(j)["sweeps_done"] == done
            with pytest.raises(sw.SwError) as e:
                srv.series(j, 0, done)
            assert e.value.code == sw.SW_ERANGE
            if done >= 2:
                _same_records(srv.series(j, 0, done - 1), ref[: done - 1], f"active job after {done} sweeps")
        _drain(srv, 8)
        assert srv.info(j)["state"] == sw.SW_JOB_DONE
        _same_records(srv.series(j, 0, n), ref, "finished job")
        assert np.array_equal(srv.spins(j), sp)


def test_serving_workload_shaped_jobs_match_solo_runs():
    """Jobs shaped like the serving workload: L log-uniform in [128, 4096]
    rounded to a multiple of 32 (one of them 4096), beta uniform in
    [0.35, 0.55], hot starts, a few hundred sweeps each; half are queued at
    the start and half arrive while the first ones run, into a pool that
    holds only some of them at once.  Every job's records and final spins
    equal a plain sim run alone."""
    rng = np.random.default_rng(2024)
    njobs = 10
    Ls = [int(round(math.exp(rng.uniform(math.log(128), math.log(4096))) / 32.0)) * 32 for _ in range(njobs)]
    Ls[3] = 4096
    betas = rng.uniform(0.35, 0.55, njobs)
    sweeps = rng.integers(100, 401, njobs)
    seeds = 7000 + np.arange(njobs)
    need = [sw.Server.job_bytes(L, int(n)) for L, n in zip(Ls, sweeps)]
    pool = max(need) + sum(sorted(need)[:3]) + 4096
    print(f"\n[case] serving-shaped jobs L={Ls} sweeps={sweeps.tolist()} pool={pool}", flush=True)
    results = {}
    with sw.Server(pool, max_jobs=6) as srv:

        def collect(jid):
            info = srv.info(jid)
            results[jid] = (srv.series(jid, 0, info["sweeps_done"]), srv.spins(jid))
            srv.release(jid)

        ids = {}
        for i in range(njobs // 2):
            ids[i] = srv.submit(Ls[i], float(betas[i]), 1.0, int(seeds[i]), int(sweeps[i]))
        for _ in range(6):  # the first jobs run; the rest arrive mid-run
            for jid in srv.step(37):
                collect(jid)
        for i in range(njobs // 2, njobs):
            ids[i] = srv.submit(Ls[i], float(betas[i]), 1.0, int(seeds[i]), int(sweeps[i]))
        _drain(srv, 37, collect=collect)
        assert srv.status()["bytes_used"] == 0
    for i in range(njobs):
        got, spins = results[ids[i]]
        ref, sp = _solo(Ls[i], float(betas[i]), int(seeds[i]), int(sweeps[i]))
        _same_records(got, ref, f"job {i} L={Ls[i]} sweeps={int(sweeps[i])}")
        assert np.array_equal(spins, sp), f"job {i} spins"
