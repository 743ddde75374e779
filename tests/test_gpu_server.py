"""Serving engine on the GPU: continuous batching of independent systems.

Each result is checked against the FP64 residual of its own system (tolerance
1e-8 relative, computed here on the CPU with scipy) and against its exact x*
(error bound kappa * tol with kappa ~ 3 for m = 4n, checked at 1e-7).  The
same system solved alone and inside a mix agrees within twice that bound.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import paper_1401_4780_amd as P
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-8


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _systems(ids, sizes):
    return [synth.serving_system(rid, m, m // 4) for rid, m in zip(ids, sizes)]


def _rel_res(s, x):
    A = sp.csr_matrix((s.val64, s.col, s.row_ptr), shape=(s.m, s.n))
    return np.linalg.norm(s.b - A @ x) / np.linalg.norm(s.b)


def _run_all(srv, systems, seeds=None, max_rounds=400):
    ids = [srv.submit(s.row_ptr, s.col, s.val, s.b, n=s.n, tol=TOL,
                      seed=(seeds[k] if seeds else k)) for k, s in enumerate(systems)]
    out = {}
    for _ in range(max_rounds):
        srv.progress()
        for k, rid in enumerate(ids):
            if k in out:
                continue
            r = srv.poll(rid, n=systems[k].n)
            if r is not None:
                out[k] = r
        if len(out) == len(ids):
            break
    assert len(out) == len(ids), "server did not drain"
    return [out[k] for k in range(len(ids))]


def _check(s, res):
    status, st, x = res
    assert status == "OK", st
    assert st["rel_residual"] <= TOL
    assert _rel_res(s, x) <= 1.05 * TOL  # the FP64 residual of the returned x
    assert np.linalg.norm(x - s.x_star) <= 1e-7 * np.linalg.norm(s.x_star)
    assert st["t_submit"] <= st["t_admit"] <= st["t_done"]


@pytest.mark.parametrize("use_graph,pinned", [(True, 1 << 30), (False, 0), (True, 8 << 20)])
def test_server_solves_a_mixed_stream(use_graph, pinned):
    """pinned = 8 MiB holds only the small requests: both upload paths in one
    run (every request is submitted before the first round, from the thread
    that drives the rounds, so submits do not wait for staging)."""
    _say(f"server mixed stream graph={use_graph} pinned={pinned}")
    sizes = [1000, 1500, 4000, 12000, 30000, 2000, 800, 60000, 5000, 1000]
    systems = _systems(range(100, 110), sizes)
    with P.Server(budget_bytes=1 << 30, use_graph=use_graph, pinned_bytes=pinned, pinned_wait_ms=0) as srv:
        res = _run_all(srv, systems)
        for s, r in zip(systems, res):
            _check(s, r)
        st = srv.stats()
        assert st["completed"] == len(systems) and st["active"] == 0 and st["arena_used"] == 0
        if pinned == 8 << 20:
            assert 0 < st["pageable_uploads"] < len(systems)
        else:
            assert st["pageable_uploads"] == (len(systems) if pinned == 0 else 0)


def test_submit_waits_for_pinned_staging_while_the_loop_runs():
    """A pinned staging of 12 MiB holds one of these requests (6-9 MiB packed)
    at a time: with the round loop running, submits wait for uploads to
    release staging instead of packing into pageable memory, and every
    request is still solved; with pinned_wait_ms = 0 some go pageable."""
    import threading
    _say("server submit waits for pinned staging")
    systems = _systems(range(720, 732), [16000 + 1000 * k for k in range(12)])
    for wait_ms, expect_pageable in ((10000, False), (0, True)):
        ids = [None] * len(systems)
        with P.Server(budget_bytes=1 << 30, pinned_bytes=12 << 20, pinned_wait_ms=wait_ms) as srv:
            srv.start()

            def worker(lo):
                for k in range(lo, len(systems), 2):
                    s = systems[k]
                    ids[k] = srv.submit(s.row_ptr, s.col, s.val, s.b, n=s.n, tol=TOL, seed=k)
            threads = [threading.Thread(target=worker, args=(t,)) for t in range(2)]
            for t in threads:
                t.start()
            for t in threads:
                t.join()
            out = {}
            import time
            t_end = time.monotonic() + 60.0
            while len(out) < len(systems) and time.monotonic() < t_end:
                for rid in srv.take_completed():
                    k = ids.index(rid)
                    out[k] = srv.poll(rid, n=systems[k].n)
                time.sleep(0.001)
            srv.stop()
            assert len(out) == len(systems)
            for k, s in enumerate(systems):
                _check(s, out[k])
            st = srv.stats()
            assert (st["pageable_uploads"] > 0) == expect_pageable, (wait_ms, st["pageable_uploads"])


def test_busy_rounds_without_replacement_take_fewer_sweeps():
    """pipe_workers = 0: every round is a busy (plain) one, so order decides
    the row order of every sweep: slices without replacement (order = 1) or
    rows drawn with replacement (order = 0).  Both reach the tolerance; the
    slices need fewer sweeps (about 13 against 16-17 on this stream)."""
    _say("server busy rounds: slices vs sampled rows")
    sizes = [1000, 1500, 4000, 12000, 30000, 2000, 800, 60000, 5000, 1000]
    systems = _systems(range(300, 310), sizes)
    sweeps = {}
    for order in (1, 0):
        with P.Server(budget_bytes=1 << 30, pipe_workers=0, order=order) as srv:
            res = _run_all(srv, systems)
            for s, r in zip(systems, res):
                _check(s, r)
            sweeps[order] = sum(r[1]["sweeps"] for r in res)
            assert srv.stats()["pipelined_rounds"] == 0
    assert sweeps[1] < sweeps[0], sweeps


def test_result_alone_equals_result_in_mix():
    _say("server alone vs mix")
    target = synth.serving_system(7, 20000, 5000)
    others = _systems(range(200, 215), [3000 + 1000 * k for k in range(15)])
    with P.Server(budget_bytes=1 << 30) as srv:
        alone = _run_all(srv, [target], seeds=[42])[0]
    with P.Server(budget_bytes=1 << 30) as srv:
        mixed = _run_all(srv, others[:7] + [target] + others[7:],
                         seeds=list(range(7)) + [42] + list(range(7, 15)))
    _check(target, alone)
    for s, r in zip(others[:7] + [target] + others[7:], mixed):
        _check(s, r)
    xa, xm = alone[2], mixed[7][2]
    assert np.linalg.norm(xa - xm) <= 2e-7 * np.linalg.norm(target.x_star)


def test_budget_admission_and_continuous_batching():
    """A budget that holds about two systems: the rest wait in the queue and
    are admitted as memory frees up, while new requests keep arriving."""
    _say("server budget admission")
    systems = _systems(range(300, 310), [20000] * 10)
    one = 20000 * (16 + 36 * 8) + 20000 * 16 + 5000 * 12  # about one system's footprint
    with P.Server(budget_bytes=int(2.5 * one) + (1 << 20)) as srv:
        ids = [srv.submit(s.row_ptr, s.col, s.val, s.b, n=s.n, tol=TOL, seed=k)
               for k, s in enumerate(systems[:5])]
        active, queued = srv.progress()
        assert active <= 2 and queued >= 3
        assert srv.poll(ids[-1], n=systems[4].n) is None  # still queued: pending
        ids += [srv.submit(s.row_ptr, s.col, s.val, s.b, n=s.n, tol=TOL, seed=5 + k)
                for k, s in enumerate(systems[5:])]
        out = {}
        for _ in range(2000):
            srv.progress()
            for k, rid in enumerate(ids):
                if k not in out:
                    r = srv.poll(rid, n=systems[k].n)
                    if r is not None:
                        out[k] = r
            if len(out) == len(ids):
                break
        assert len(out) == len(ids)
        for k, s in enumerate(systems):
            _check(s, out[k])
        assert srv.stats()["arena_used"] == 0
        with pytest.raises(P.AsyrkError):
            srv.poll(ids[0])  # already collected
        big = synth.serving_system(1, 200000, 50000)
        with pytest.raises(P.AsyrkError) as ei:
            srv.submit(big.row_ptr, big.col, big.val, big.b, n=big.n)
        assert ei.value.name == "OOM"


@pytest.mark.parametrize("pipe_workers", [8192, 0])
def test_concurrent_submitters_while_rounds_run(pipe_workers):
    """submit() from several threads while one thread drives progress().
    pipe_workers = 0 makes every round with active systems a busy one, so
    requests arriving meanwhile upload during it and join the next round."""
    import threading
    _say(f"server concurrent submitters pipe_workers={pipe_workers}")
    systems = _systems(range(400, 424), [1000 + 700 * k for k in range(24)])
    ids = [None] * len(systems)
    with P.Server(budget_bytes=1 << 30, pipe_workers=pipe_workers) as srv:
        def worker(lo):
            for k in range(lo, len(systems), 4):
                s = systems[k]
                ids[k] = srv.submit(s.row_ptr, s.col, s.val, s.b, n=s.n, tol=TOL, seed=k)
        threads = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
        for t in threads:
            t.start()
        out = {}
        for _ in range(3000):
            srv.progress()
            for k in range(len(systems)):
                if k not in out and ids[k] is not None:
                    r = srv.poll(ids[k], n=systems[k].n)
                    if r is not None:
                        out[k] = r
            if len(out) == len(systems):
                break
        for t in threads:
            t.join()
        assert len(out) == len(systems)
        for k, s in enumerate(systems):
            _check(s, out[k])
        assert len(set(ids)) == len(ids)
        st = srv.stats()
        assert st["completed"] == len(systems) and st["active"] == 0 and st["arena_used"] == 0


@pytest.mark.parametrize("pipe_workers,pipe_lanes", [(0, 8), (1 << 24, 4), (1 << 24, 8), (1 << 24, 16),
                                                     (1 << 24, 32)])
@pytest.mark.parametrize("lanes", [4, 8])
def test_lane_widths_and_completion_list(lanes, pipe_workers, pipe_lanes):
    """Every lane width and worker loop (plain: pipe_workers = 0; pipelined:
    every round) of the packed sweep drains a mixed stream to tolerance;
    take_completed reports each finished id exactly once."""
    _say(f"server lanes={lanes} pipe_workers={pipe_workers} pipe_lanes={pipe_lanes} take_completed")
    sizes = [900, 3000, 17000, 1200, 40000, 2500]
    systems = _systems(range(500, 506), sizes)
    with P.Server(budget_bytes=1 << 30, lanes=lanes, pipe_workers=pipe_workers, pipe_lanes=pipe_lanes) as srv:
        ids = [srv.submit(s.row_ptr, s.col, s.val, s.b, n=s.n, tol=TOL, seed=k)
               for k, s in enumerate(systems)]
        index = {rid: k for k, rid in enumerate(ids)}
        seen, out = [], {}
        for _ in range(400):
            srv.progress()
            for rid in srv.take_completed(cap=2):
                seen.append(rid)
                k = index[rid]
                out[k] = srv.poll(rid, n=systems[k].n)
            if len(out) == len(ids):
                break
        assert sorted(seen) == sorted(ids) and len(seen) == len(set(seen))
        assert srv.take_completed() == []
        for k, s in enumerate(systems):
            _check(s, out[k])


def test_native_round_loop_with_concurrent_submitters():
    """start() runs the library's round loop (asyrk_server_run) on its own
    thread: requests submitted from several threads while it runs all finish
    to tolerance, an idle loop wakes for a late submit, and stop() ends it."""
    import threading
    import time
    _say("server native round loop")
    systems = _systems(range(700, 716), [1000 + 900 * k for k in range(16)])
    ids = [None] * len(systems)
    with P.Server(budget_bytes=1 << 30) as srv:
        srv.start()
        with pytest.raises(RuntimeError):
            srv.start()
        with pytest.raises(RuntimeError):
            srv.progress()  # one thread runs rounds at a time

        def worker(lo):
            for k in range(lo, len(systems) - 1, 3):
                s = systems[k]
                ids[k] = srv.submit(s.row_ptr, s.col, s.val, s.b, n=s.n, tol=TOL, seed=k)
        threads = [threading.Thread(target=worker, args=(t,)) for t in range(3)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        out = {}

        def collect(want):
            t_end = time.monotonic() + 60.0
            while len(out) < want and time.monotonic() < t_end:
                got = srv.take_completed()
                if not got:
                    time.sleep(0.001)
                for rid in got:
                    k = ids.index(rid)
                    out[k] = srv.poll(rid, n=systems[k].n)

        collect(len(systems) - 1)
        assert len(out) == len(systems) - 1
        # the loop is idle now; a late request wakes it
        time.sleep(0.01)
        s = systems[-1]
        ids[-1] = srv.submit(s.row_ptr, s.col, s.val, s.b, n=s.n, tol=TOL, seed=99)
        collect(len(systems))
        srv.stop()
        srv.stop()  # a second stop is a no-op
        assert len(out) == len(systems)
        for k, s in enumerate(systems):
            _check(s, out[k])
        st = srv.stats()
        assert st["completed"] == len(systems) and st["active"] == 0 and st["arena_used"] == 0
        srv.start()  # close() ends a running loop before destroying the server


def test_sized_later_rounds_vs_fixed_rounds():
    """By default a request's later rounds run only the sweeps its measured
    contraction predicts (at most inner_sweeps); fixed_rounds = 1 runs
    inner_sweeps every round.  At tol = 1e-6 the first 8 sweeps leave a few
    more to do, so sized requests end between multiples of 8; both modes reach
    the tolerance (the FP64 residual of the returned x is checked here), and
    the sized total is at most about one sweep per request above the fixed
    one (asynchronous rounds make the measured contraction vary from run to
    run; the saving is measured by the serving benchmark)."""
    _say("server sized vs fixed rounds")
    tol = 1e-6
    systems = _systems(range(800, 808), [2000, 9000, 30000, 1500, 60000, 4000, 12000, 25000])
    sweeps = {}
    for fixed in (0, 1):
        with P.Server(budget_bytes=1 << 30, fixed_rounds=fixed) as srv:
            assert srv.config["fixed_rounds"] == fixed
            ids = [srv.submit(s.row_ptr, s.col, s.val, s.b, n=s.n, tol=tol, seed=k) for k, s in enumerate(systems)]
            out = {}
            for _ in range(400):
                srv.progress()
                for k, rid in enumerate(ids):
                    if k not in out:
                        r = srv.poll(rid, n=systems[k].n)
                        if r is not None:
                            out[k] = r
                if len(out) == len(ids):
                    break
            assert len(out) == len(ids)
            for k, s in enumerate(systems):
                status, st, x = out[k]
                assert status == "OK" and st["rel_residual"] <= tol
                assert _rel_res(s, x) <= 1.05 * tol
            sweeps[fixed] = [out[k][1]["sweeps"] for k in range(len(ids))]
    assert all(v % 8 == 0 for v in sweeps[1])
    assert any(v % 8 for v in sweeps[0])
    assert sum(sweeps[0]) <= sum(sweeps[1]) + len(systems)

def test_invalid_submissions_are_rejected_and_the_server_goes_on():
    """Submit validates on the caller's thread: a zero row is ZERO_ROW;
    unsorted or out-of-range columns, a non-finite value or b, a nonpositive
    tolerance are INVALID_ARG.  Rejected requests leave no trace (no id, no
    staging memory), and a valid request afterwards is served normally."""
    _say("server invalid submissions")
    s = _systems([900], [3000])[0]
    with P.Server(budget_bytes=1 << 30) as srv:
        def bad(name, expect, **edit):
            rp, col, val, b = s.row_ptr.copy(), s.col.copy(), s.val.copy(), s.b.copy()
            tol = edit.pop("tol", TOL)
            if "fn" in edit:
                rp, col, val, b = edit["fn"](rp, col, val, b)
            with pytest.raises(P.AsyrkError) as ei:
                srv.submit(rp, col, val, b, n=s.n, tol=tol)
            assert ei.value.name == expect, name

        def empty_row(rp, col, val, b):  # row 5's stored values all zero: ||a_5|| = 0
            val = val.copy()
            val[int(rp[5]):int(rp[6])] = 0.0
            return rp, col, val, b

        def swap_cols(rp, col, val, b):
            col = col.copy()
            a = int(rp[7])
            col[a], col[a + 1] = col[a + 1], col[a]
            return rp, col, val, b

        def col_oob(rp, col, val, b):
            col = col.copy()
            col[int(rp[9 + 1]) - 1] = s.n
            return rp, col, val, b

        def nan_val(rp, col, val, b):
            val = val.copy()
            val[11] = np.nan
            return rp, col, val, b

        def inf_b(rp, col, val, b):
            b = b.copy()
            b[3] = np.inf
            return rp, col, val, b

        bad("empty row", "ZERO_ROW", fn=empty_row)
        bad("unsorted columns", "INVALID_ARG", fn=swap_cols)
        bad("column out of range", "INVALID_ARG", fn=col_oob)
        bad("NaN value", "INVALID_ARG", fn=nan_val)
        bad("infinite b", "INVALID_ARG", fn=inf_b)
        bad("zero tolerance", "INVALID_ARG", tol=0.0)
        with pytest.raises(ValueError):  # arrays shorter than row_ptr says: caught before the ABI
            srv.submit(s.row_ptr, s.col[:-1], s.val, s.b, n=s.n)
        with pytest.raises(ValueError):
            srv.submit(s.row_ptr, s.col, s.val, s.b[:-1], n=s.n)
        st = srv.stats()
        assert st["submitted"] == 0 and st["queued"] == 0 and st["arena_used"] == 0
        res = _run_all(srv, [s])
        _check(s, res[0])
        rid = srv.submit(s.row_ptr, s.col, s.val, s.b, n=s.n, tol=TOL)
        with pytest.raises(ValueError):  # poll writes the request's own n values
            srv.poll(rid, n=s.n - 1)


@pytest.mark.parametrize("use_graph", [True, False])
def test_online_lane_tuning(use_graph):
    """lanes = 0 / pipe_lanes = 0: the first rounds of each kind and load
    bucket sweep their systems once per candidate width, timed, and keep the
    fastest; results are unaffected (every candidate sweeps from d = 0 on the
    same tickets, the round's own sweep last), and tuned buckets run the
    chosen width (its captured graph)."""
    _say(f"server online lane tuning use_graph={use_graph}")
    with P.Server(budget_bytes=1 << 30, lanes=0, pipe_lanes=0, pipe_workers=256, inner_sweeps=2,
                  use_graph=use_graph) as srv:
        assert srv.stats()["buckets_untuned"] == 8
        big = _systems(range(900, 903), [40000] * 3)       # about 2400 workers: plain rounds
        for s, r in zip(big, _run_all(srv, big)):
            _check(s, r)
        small = _systems(range(903, 906), [2000] * 3)      # about 120 workers: pipelined rounds
        for s, r in zip(small, _run_all(srv, small)):
            _check(s, r)
        st = srv.stats()
        # the systems split over the two round groups, so rounds fall in one
        # or more load buckets; at least one has finished tuning
        assert st["buckets_untuned"] <= 7, st
        assert st["lanes"] in (4, 8) and st["pipe_lanes"] in (4, 8, 16, 32)
        more = _systems(range(906, 908), [30000, 1500])
        for s, r in zip(more, _run_all(srv, more)):
            _check(s, r)
