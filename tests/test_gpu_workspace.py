"""Caller-owned device workspace: plans, one-shot solves and a server laid out in device memory the
caller allocated (here through the HIP runtime the library links), with results bitwise those of the
library-allocated calls and within the oracle bars, and the size and alignment errors."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import models as om
import workloads
import paper_2504_21440_amd as qt

pytestmark = pytest.mark.gpu


class DeviceBuffer:
    """Raw device memory from the system HIP runtime (the library's), as a caller would own it."""

    def __init__(self, nbytes):
        from hipmem import rt
        self.nbytes = int(nbytes)
        self.ptr = ctypes.c_void_p()
        assert rt().hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(max(1, self.nbytes))) == 0
        assert self.ptr.value % 256 == 0

    def ws(self, offset=0, nbytes=None):
        return (self.ptr.value + offset, self.nbytes - offset if nbytes is None else nbytes)

    def free(self):
        from hipmem import rt
        if self.ptr:
            rt().hipFree(self.ptr)
            self.ptr = ctypes.c_void_p()


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] workspace: creating context", flush=True)
    c = qt.Context(0)
    yield c
    c.close()


def test_me_plan_in_caller_workspace_matches_allocating_plan(ctx):
    print("[gpu] workspace: ME plan (CSR + dense, mixed)", flush=True)
    tl = np.linspace(0.0, 3.0, 16)
    Hi, ci = qt.model_ising(6, 1.0, 0.7, 0.2)
    Hk, ck = qt.model_kerr(16, 1.0, 0.5, 0.8, 1.0)
    Li = qt.Liouvillian(ctx, Hi, ci, qt.FORM_CSR, qt.MIXED)
    Lk = qt.Liouvillian(ctx, Hk, ck, qt.FORM_DENSE, qt.MIXED)
    assert Li.footprint() == Li.info()[2] > 0 and Lk.footprint() == Lk.info()[2] > 0
    ei = [om.site_op(6, k, om.sigmaz()) for k in (0, 2)]
    ek = [om.number(16)]
    probs = [(Li, om.all_up_ket(6), tl, ei), (Lk, om.fock_dm(16, 0), tl, ek)]
    o = qt.opts(precision=qt.MIXED, abstol=1e-7, reltol=1e-5)
    need = qt.me_plan_workspace(ctx, probs, o)
    n = 64 * 64  # Liouville rows of the L = 6 chain
    assert need >= 11 * n * 8
    buf = DeviceBuffer(need + 512)
    with pytest.raises(qt.QtError) as e:
        qt.MePlan(ctx, probs, o, workspace=buf.ws(0, need - 1))
    assert e.value.code == qt.QT_ENOMEM
    with pytest.raises(qt.QtError) as e:
        qt.MePlan(ctx, probs, o, workspace=buf.ws(128, need))
    assert e.value.code == qt.QT_EINVAL
    ref_plan = qt.MePlan(ctx, probs, o)
    ref_plan.run()
    refs = [ref_plan.result(i) for i in range(2)]
    ref_plan.close()
    P = qt.MePlan(ctx, probs, o, workspace=buf.ws(256, need))
    for rep in range(2):  # a plan in caller memory runs again from its resident inputs
        P.run()
        for i in range(2):
            got = P.result(i)
            np.testing.assert_array_equal(got[0], refs[i][0])
            assert got[1]["n_accept"] == refs[i][1]["n_accept"]
    P.close()
    exact_i = oracle.mesolve(Hi, ci, om.all_up_ket(6), tl, ei)[0]
    exact_k = oracle.mesolve(Hk, ck, om.fock_dm(16, 0), tl, ek)[0]
    assert np.abs(refs[0][0] - exact_i).max() < 1e-4
    assert np.abs(refs[1][0] - exact_k).max() < 1e-4
    buf.free()
    Li.close()
    Lk.close()


def test_mesolve_ws_fp64_kerr_matches_mesolve(ctx):
    print("[gpu] workspace: qt_mesolve_ws FP64 Kerr N=20", flush=True)
    H, c = qt.model_kerr(20, 1.0, 0.5, 0.8, 1.0)
    L = qt.Liouvillian(ctx, H, c, qt.FORM_CSR, qt.F64)
    tl = workloads.tlist(20.0, 41)
    prob = [(L, om.fock_dm(20, 0), tl, [om.number(20)])]
    need = qt.me_plan_workspace(ctx, prob)
    buf = DeviceBuffer(need)
    a = qt.mesolve(ctx, L, om.fock_dm(20, 0), tl, [om.number(20)], want_final=True)
    b = qt.mesolve(ctx, L, om.fock_dm(20, 0), tl, [om.number(20)], want_final=True, workspace=buf.ws())
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[2], b[2])
    ref = oracle.mesolve(H, c, om.fock_dm(20, 0), tl, [om.number(20)])[0]
    assert np.abs(b[0] - ref).max() < 1e-6
    buf.free()
    L.close()


def test_mcsolve_ws_matches_mcsolve_per_trajectory(ctx):
    print("[gpu] workspace: qt_mcsolve_ws Ising L=4, 64 trajectories", flush=True)
    H, cs = qt.model_ising(4, 1.0, 1.0, 0.3)
    tl = workloads.tlist(4.0, 21)
    e = [om.site_op(4, 0, om.sigmaz())]
    o = qt.opts(precision=qt.F64)
    args = (H, cs, om.all_up_ket(4), tl, e, 64, 99)
    need = qt.mc_plan_workspace(ctx, *args, options=o, max_jump_record=8)
    buf = DeviceBuffer(need)
    a = qt.mcsolve(ctx, *args, options=o, want_traj=True, max_jump_record=8)
    b = qt.mcsolve_ws(ctx, buf.ws(), *args, options=o, want_traj=True, max_jump_record=8)
    for k in ("mean", "se", "njumps", "expect_tr"):
        np.testing.assert_array_equal(a[k], b[k])
    rec = np.arange(8)[None, :] < np.minimum(a["njumps"], 8)[:, None]  # slots past njumps are unspecified
    np.testing.assert_array_equal(a["jump_times"][rec], b["jump_times"][rec])
    np.testing.assert_array_equal(a["jump_channels"][rec], b["jump_channels"][rec])
    assert b["njumps"].sum() > 0
    buf.free()


def test_server_in_caller_workspace_matches_allocating_server(ctx):
    print("[gpu] workspace: server in caller memory", flush=True)
    o = qt.opts(abstol=1e-7, reltol=1e-5, precision=qt.MIXED)
    reqs = []
    for N, U in [(12, 0.3), (24, 0.5)]:
        Hk, ck = qt.model_kerr(N, 1.0, U, 0.8, 1.0)
        reqs.append(((qt.Liouvillian(ctx, Hk, ck, qt.FORM_DENSE, qt.MIXED), om.fock_dm(N, 0),
                      workloads.tlist(4.0, 9), [om.number(N)]), (Hk, ck)))
    for Lc in (5, 7):
        Hi, ci = qt.model_ising(Lc, 1.0, 0.9, 0.3)
        reqs.append(((qt.Liouvillian(ctx, Hi, ci, qt.FORM_CSR, qt.MIXED), om.all_up_ket(Lc),
                      workloads.tlist(2.0, 9), [om.site_op(Lc, 0, om.sigmaz())]), (Hi, ci)))
    pool = 256 << 20
    need = qt.server_workspace(pool, 16, 8, o)
    assert need > pool
    buf = DeviceBuffer(need)

    def serve(srv):
        tickets = {srv.submit(*pr): i for i, (pr, _) in enumerate(reqs)}
        assert None not in tickets
        out, epochs = {}, 0
        while tickets:
            srv.step()
            epochs += 1
            for t in list(tickets):
                r = srv.poll(t)
                if r is not None:
                    out[tickets.pop(t)] = r
            assert epochs < 100000
        srv.close()
        return out

    a = serve(qt.Server(ctx, pool_bytes=pool, max_slots=16, steps_per_epoch=8, options=o))
    b = serve(qt.Server(ctx, pool_bytes=pool, max_slots=16, steps_per_epoch=8, options=o, workspace=buf.ws()))
    for i, (pr, (H, cs)) in enumerate(reqs):
        np.testing.assert_array_equal(a[i][0], b[i][0])
        ref = oracle.mesolve(H, cs, pr[1], pr[2], pr[3])[0]
        assert np.abs(b[i][0] - ref).max() < 1e-4
        pr[0].close()
    buf.free()
