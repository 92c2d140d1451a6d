"""Continuous-batching server: admission by device footprint, requests joining while others run,
and every result the same alone and in the mix (bitwise: a request's arithmetic never depends on what
else is resident), checked against the FP64 oracle as well."""
import numpy as np
import pytest

import oracle
from oracle import models as om
import workloads
import paper_2504_21440_amd as qt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] creating context", flush=True)
    c = qt.Context(0)
    yield c
    c.close()


def _request(ctx, p, prec=qt.MIXED, nt=21):
    if p["kind"] == "kerr":
        H, c = qt.model_kerr(p["N"], p["delta"], p["U"], p["F"], p["kappa"])
        L = qt.Liouvillian(ctx, H, c, qt.FORM_DENSE, prec)
        return (L, om.fock_dm(p["N"], 0), workloads.tlist(p["t_end"], nt), [om.number(p["N"])]), (H, c)
    H, cs = qt.model_ising(p["L"], p["J"], p["h"], p["gamma"])
    L = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, prec)
    Lc = p["L"]
    return (L, om.all_up_ket(Lc), workloads.tlist(p["t_end"], nt), [om.site_op(Lc, 0, om.sigmaz())]), (H, cs)


def _trace(n, seed):
    tr = workloads.serving_trace(n=n, seed=seed)
    for p in tr:  # smaller sizes keep the oracle check quick
        if p["kind"] == "kerr":
            p["N"] = min(p["N"], 30)
            p["U"] = min(p["U"], 0.3)
        else:
            p["L"] = min(p["L"], 6)
    return tr


def test_server_results_equal_alone_and_in_mix(ctx):
    print("[gpu] server mix vs alone", flush=True)
    trace = _trace(10, 3)
    reqs = [_request(ctx, p) for p in trace]
    o = qt.opts(abstol=1e-7, reltol=1e-5, precision=qt.MIXED)
    srv = qt.Server(ctx, pool_bytes=1 << 30, max_slots=64, steps_per_epoch=8, options=o)
    tickets = {}
    pending = list(range(len(reqs)))
    results = {}
    epochs = 0
    # requests arrive two per epoch while earlier ones are still running
    while pending or tickets:
        for _ in range(2):
            if pending:
                i = pending.pop(0)
                t = srv.submit(*reqs[i][0])
                assert t is not None
                tickets[t] = i
        srv.step()
        epochs += 1
        for t in list(tickets):
            r = srv.poll(t)
            if r is not None:
                results[tickets.pop(t)] = r
        assert epochs < 100000
    assert len(results) == len(reqs)
    for i, (pr, ops) in enumerate(reqs):
        plan = qt.MePlan(ctx, [pr], o)
        plan.set_shape(8, 1, 0, 2)  # the server's CSR launch shape
        plan.run()
        alone = plan.result(0)
        plan.close()
        np.testing.assert_array_equal(results[i][0], alone[0])
        assert results[i][1]["n_accept"] == alone[1]["n_accept"]
        H, cs = ops
        ref, _, _, _ = oracle.mesolve(H, cs, pr[1], pr[2], pr[3])
        assert np.abs(results[i][0] - ref).max() < 1e-4
    srv.close()


def test_server_large_and_small_lanes_match_alone(ctx):
    """A large chain (L = 8: 65,536 Liouville rows, the large lane) served together with small CSR
    cavities and chains (the small lane, which replays its epochs while the large one runs): every
    result bitwise equal to the same problem solved alone in a plan, and the small ones within 1e-4
    of the FP64 oracle."""
    print("[gpu] server lanes vs alone", flush=True)
    o = qt.opts(abstol=1e-7, reltol=1e-5, precision=qt.MIXED)
    probs = []
    H, cs = qt.model_ising(8, 1.0, 0.7, 0.2)
    L8 = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, qt.MIXED)
    probs.append(((L8, om.all_up_ket(8), workloads.tlist(1.0, 6), [om.site_op(8, 0, om.sigmaz())]), None))
    for N, U in [(12, 0.3), (20, 0.5), (30, 0.2)]:
        Hk, ck = qt.model_kerr(N, 1.0, U, 0.8, 1.0)
        Lk = qt.Liouvillian(ctx, Hk, ck, qt.FORM_CSR, qt.MIXED)
        probs.append(((Lk, om.fock_dm(N, 0), workloads.tlist(5.0, 11), [om.number(N)]), (Hk, ck)))
    for Lc in (4, 5):
        Hi, ci = qt.model_ising(Lc, 1.0, 0.9, 0.3)
        Li = qt.Liouvillian(ctx, Hi, ci, qt.FORM_CSR, qt.MIXED)
        probs.append(((Li, om.all_up_ket(Lc), workloads.tlist(3.0, 7), [om.site_op(Lc, 0, om.sigmaz())]),
                      (Hi, ci)))
    srv = qt.Server(ctx, pool_bytes=1 << 30, max_slots=16, steps_per_epoch=8, options=o)
    tickets = {srv.submit(*pr): i for i, (pr, _) in enumerate(probs)}
    assert None not in tickets
    results, epochs = {}, 0
    while tickets:
        srv.step()
        epochs += 1
        for t in list(tickets):
            r = srv.poll(t)
            if r is not None:
                results[tickets.pop(t)] = r
        assert epochs < 100000
    for i, (pr, ops) in enumerate(probs):
        plan = qt.MePlan(ctx, [pr], o)
        plan.set_shape(8, 1, 0, 2)  # the server's CSR launch shape
        plan.run()
        alone = plan.result(0)
        plan.close()
        np.testing.assert_array_equal(results[i][0], alone[0])
        assert results[i][1]["n_accept"] == alone[1]["n_accept"]
        if ops is not None:
            ref, _, _, _ = oracle.mesolve(ops[0], ops[1], pr[1], pr[2], pr[3])
            assert np.abs(results[i][0] - ref).max() < 1e-4
    srv.close()


def test_server_admission_by_footprint(ctx):
    print("[gpu] server admission", flush=True)
    o = qt.opts(precision=qt.MIXED)
    p_big = {"kind": "ising", "L": 6, "J": 1.0, "h": 0.7, "gamma": 0.2, "t_end": 2.0, "nt": 5}
    big, _ = _request(ctx, p_big, nt=5)
    probe = qt.Server(ctx, pool_bytes=1 << 30, max_slots=4, steps_per_epoch=16, options=o)
    fp = probe.footprint(*big)
    probe.close()
    # pool for exactly one request of this size: the second must wait until the first retires
    srv = qt.Server(ctx, pool_bytes=int(fp * 1.5), max_slots=8, steps_per_epoch=16, options=o)
    t1 = srv.submit(*big)
    assert t1 is not None
    big2, _ = _request(ctx, dict(p_big, h=0.9), nt=5)
    assert srv.submit(*big2) is None  # QT_EBUSY: does not fit now
    done = None
    while done is None:
        srv.step()
        done = srv.poll(t1)
    t2 = srv.submit(*big2)
    assert t2 is not None
    while srv.poll(t2) is None:
        srv.step()
    # a request larger than the whole pool can never be admitted
    huge, _ = _request(ctx, dict(p_big, L=8), nt=5)
    with pytest.raises(qt.QtError) as e:
        srv.submit(*huge)
    assert e.value.code == qt.QT_ENOMEM
    srv.close()


def test_server_slot_limit_and_errors(ctx):
    o = qt.opts(precision=qt.MIXED, max_steps=5)
    srv = qt.Server(ctx, pool_bytes=1 << 28, max_slots=2, steps_per_epoch=4, options=o)
    p = {"kind": "kerr", "N": 12, "delta": 1.0, "U": 0.5, "F": 0.8, "kappa": 1.0, "t_end": 20.0, "nt": 5}
    r1, _ = _request(ctx, p, nt=5)
    r2, _ = _request(ctx, dict(p, N=14), nt=5)
    r3, _ = _request(ctx, dict(p, N=16), nt=5)
    t1, t2 = srv.submit(*r1), srv.submit(*r2)
    assert t1 is not None and t2 is not None
    assert srv.submit(*r3) is None  # no free slot
    for _ in range(10):
        srv.step()
    # max_steps = 5 cannot reach t = 20: both requests end with QT_EMAXSTEPS and free their slots
    for t in (t1, t2):
        with pytest.raises(qt.QtError) as e:
            srv.poll(t)
        assert e.value.code == qt.QT_EMAXSTEPS
    assert srv.submit(*r3) is not None
    srv.close()


SERVED_RTOL = 1e-4  # the served mixed tolerance the bench calibrates (loosest ladder rung meeting 1e-4)


def test_served_stream_at_benched_size_matches_oracle_and_alone(ctx):
    """Requests of the served stream exactly as benchmarked: Kerr cavities (up to N = 80) and chains
    (up to L = 9) in the CSR form, 100 saves, mixed precision at the served tolerance, all submitted
    together to a server configured as the bench's.  The stiffest cavities (largest U N^2), the first
    L = 9 chains and a spread of smaller requests are each within 1e-4 of the stored oracle solution
    (abstol 1e-10, reltol 1e-8) and bitwise equal to the same request solved alone."""
    import json
    import os
    print("[gpu] served stream at benched size", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "serving_trace240.json")) as f:
        refs = {r["id"]: np.array(r["expect_re"][0]) + 1j * np.array(r["expect_im"][0]) for r in json.load(f)["requests"]}
    trace = workloads.serving_trace(n=240)
    kerr = sorted((p for p in trace if p["kind"] == "kerr"), key=lambda p: -p["U"] * p["N"] ** 2)
    chains = [p for p in trace if p["kind"] == "ising"]
    pick = kerr[:4] + [p for p in chains if p["L"] == 9][:2] + [kerr[len(kerr) // 2], kerr[-1]]
    pick += [next(p for p in chains if p["L"] == L) for L in (4, 6, 8)]
    o = qt.opts(abstol=SERVED_RTOL / 100, reltol=SERVED_RTOL, precision=qt.MIXED)
    reqs = []
    for p in pick:
        tl = workloads.tlist(p["t_end"], p["nt"])
        if p["kind"] == "kerr":
            H, c = qt.model_kerr(p["N"], p["delta"], p["U"], p["F"], p["kappa"])
            reqs.append((qt.Liouvillian(ctx, H, c, qt.FORM_CSR, qt.MIXED), om.fock_dm(p["N"], 0), tl, [om.number(p["N"])]))
        else:
            H, cs = qt.model_ising(p["L"], p["J"], p["h"], p["gamma"])
            reqs.append((qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, qt.MIXED), om.all_up_ket(p["L"]), tl,
                         [om.site_op(p["L"], 0, om.sigmaz())]))
    srv = qt.Server(ctx, pool_bytes=16 << 30, max_slots=1024, steps_per_epoch=32, options=o)
    tickets = {srv.submit(*pr): i for i, pr in enumerate(reqs)}
    assert None not in tickets
    results, epochs = {}, 0
    while tickets:
        srv.step()
        epochs += 1
        for t in list(tickets):
            r = srv.poll(t)
            if r is not None:
                results[tickets.pop(t)] = r
        assert epochs < 200000
    srv.close()
    for i, (p, pr) in enumerate(zip(pick, reqs)):
        err = np.abs(results[i][0][0] - refs[p["id"]]).max()
        print(f"[gpu]   request {p['id']} {p['kind']} {p.get('N', p.get('L'))}: max |d<O>| = {err:.2e}", flush=True)
        assert err <= 1e-4
        plan = qt.MePlan(ctx, [pr], o)
        plan.set_shape(8, 1, 0, 2)  # the server's CSR launch shape: 16-byte matrix loads through the caches
        plan.run()
        alone = plan.result(0)
        plan.close()
        np.testing.assert_array_equal(results[i][0], alone[0])
        pr[0].close()
