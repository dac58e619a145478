"""GPU tests of the request loop (ssrpa_server_*).

Each request's E_c must be the same alone and in the mix: solves run on
their own streams and systems, and every kernel configuration and reduction
order depends only on the request's own sizes, so equality is bitwise.
Memory admission: the footprint model must bound the measured high-water
mark of a solve, and a request larger than the budget is refused.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _systems():
    from synth import systems as sy
    out = []
    shapes = [(4, 28, 5, 8.0, 16), (6, 40, 6, 9.0, 18), (3, 21, 4, 7.0, 16),
              (8, 56, 9, 10.0, 18), (5, 37, 6, 9.0, 18), (2, 30, 3, 8.0, 16)]
    for i, (nv, nc, nsq, a, fft) in enumerate(shapes):
        spec = sy.small_spec(a=a, fft=fft, n_v=nv, n_c=nc, nsq_chi=nsq,
                             e_psi=4.0, name=f"serve{i}")
        s = sy.make_system(spec, 900 + i)
        n_eig = 10 + 3 * i
        prec = "fp64" if i % 2 == 0 else "bf16x3"
        out.append((s, n_eig, prec))
    return out


def test_alone_equals_mixed():
    import torch  # noqa: F401  (initializes the runtime like other GPU tests)
    from paper_2405_20258_amd import ssrpa
    from synth import systems as sy
    # 48 frequencies: each solve then lasts longer than the host needs to
    # submit the next request, so the mix can overlap on the device
    om, wt = sy.frequency_grid(48)
    reqs = _systems()
    ctx = ssrpa.Context(0)
    # alone: one request at a time
    alone = []
    srv = ssrpa.Server(ctx, max_running=1, max_bypass_s=0.0)
    for s, n_eig, prec in reqs:
        rid = srv.submit(s, n_eig, om, wt, prec)
        srv.drain()
        r = srv.poll(rid)
        assert r["state"] == ssrpa.REQ_DONE, r
        alone.append(r["ec"])
    srv.close()
    _log(f"alone: {alone}")
    # mixed: everything submitted at once, up to 4 on the device together
    srv = ssrpa.Server(ctx, max_running=4, max_bypass_s=1.0)
    ids = [srv.submit(s, n_eig, om, wt, prec) for s, n_eig, prec in reqs]
    srv.drain()
    res = [srv.poll(i) for i in ids]
    dev = [srv.device_times(i) for i in ids]
    srv.close()
    _log(f"mixed: {[r['ec'] for r in res]}")
    assert all(r["state"] == ssrpa.REQ_DONE for r in res)
    for a, r in zip(alone, res):
        assert r["ec"] == a          # bitwise: independent of the mix
        assert r["ec"] < 0.0
    # the loop really overlapped requests on the device: the device-clock
    # intervals (events on each request's stream) of some two requests
    # intersect
    _log(f"device intervals (ms): {dev}")
    assert all(0.0 <= a <= b for a, b in dev)
    assert any(dev[i][0] < dev[j][1] and dev[j][0] < dev[i][1]
               for i in range(len(dev)) for j in range(i + 1, len(dev)))
    ctx.close()


def test_footprint_bounds_high_water_and_admission():
    import torch  # noqa: F401
    from paper_2405_20258_amd import ssrpa
    from synth import systems as sy
    om, wt = sy.frequency_grid(16)
    s, n_eig, prec = _systems()[3]
    keep = []
    d = ssrpa.make_desc(s.a, s.fft, s.miller, s.coeff, s.energy, s.n_v,
                        s.ecut_chi, keep)
    import ctypes
    fp = ctypes.c_size_t()
    assert ssrpa.ssrpa_footprint(ctypes.byref(d), n_eig, 16, 0, 0,
                                 ctypes.byref(fp)) == ssrpa.OK
    ctx = ssrpa.Context(0)
    g = ssrpa.System.from_synthetic(ctx, s)
    g.chi0_static("fp64")
    g.subspace(n_eig)
    g.correlation_energy(n_eig, om, wt, "fp64")
    g.close()
    _, high = ctx.memory()
    _log(f"footprint {fp.value} high water {high}")
    assert high <= fp.value
    ctx.close()
    # a budget below the request's footprint: refused at submission
    small = ssrpa.Context(0, hbm_budget=fp.value // 4)
    srv = ssrpa.Server(small, max_running=2)
    with pytest.raises(ssrpa.SsrpaError) as e:
        srv.submit(s, n_eig, om, wt, "fp64")
    assert e.value.status == ssrpa.ERR_NOMEM
    srv.close()
    small.close()
