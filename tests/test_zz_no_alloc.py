"""GPU test of the allocation-free log-determinant entry point.

ssrpa_trace_log_noalloc runs the kernels of ssrpa_trace_log on a fixed
per-device work array instead of allocated memory.  Through the C ABI, its
F_j must equal those of ssrpa_trace_log (same kernels, same order: bitwise)
and the eigenvalue form sum log1p(-l mu) + l mu of numpy, on two calls in a
row with the second smaller than the first (the array keeps the first
call's contents); a batch beyond the array is refused before any launch;
a matrix with I - X not positive definite gives NaN and a raised flag.
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _batch(rng, n, nm):
    xs = []
    for _ in range(nm):
        a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        xs.append(-(a @ a.conj().T) / (n * 2.0))   # negative semidefinite
    return np.stack(xs)


def test_noalloc_matches_allocating_entry_point():
    import torch
    from paper_2405_20258_amd import ssrpa
    ctx = ssrpa.Context(0)
    rng = np.random.default_rng(77)
    stream = torch.cuda.current_stream().cuda_stream
    # first call larger than the second: the second must not see the first's
    # leftovers
    for n, nm, c in ((200, 12, 1.0), (75, 3, 0.5)):
        _log(f"noalloc trace_log n={n} batch={nm} coupling={c}")
        x = _batch(rng, n, nm)
        xd = torch.from_numpy(x).to("cuda")
        f_ref = np.empty(nm)
        assert ssrpa.ssrpa_trace_log(ctx.handle, xd.data_ptr(), n, nm, c,
                                     f_ref.ctypes.data_as(ssrpa._dp),
                                     stream) == ssrpa.OK
        f_dev = torch.full((nm,), -1.0, dtype=torch.float64, device="cuda")
        flag = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        st = ssrpa.ssrpa_trace_log_noalloc(ctx.handle, xd.data_ptr(), n, nm, c,
                                           f_dev.data_ptr(), flag.data_ptr(),
                                           stream)
        assert st == ssrpa.OK, ssrpa.ssrpa_last_error(ctx.handle)
        torch.cuda.synchronize()
        f = f_dev.cpu().numpy()
        assert int(flag.cpu()[0]) == 0
        assert np.array_equal(f, f_ref), (f, f_ref)
        for j in range(nm):
            mu = np.linalg.eigvalsh(x[j])
            ref = float(np.sum(np.log1p(-c * mu) + c * mu))
            assert abs(f[j] - ref) <= 1e-11 * max(1.0, abs(ref)), (n, j)
    ctx.close()


def test_noalloc_limits_and_failure_flag():
    import torch
    from paper_2405_20258_amd import ssrpa
    ctx = ssrpa.Context(0)
    stream = torch.cuda.current_stream().cuda_stream
    f_dev = torch.zeros((2,), dtype=torch.float64, device="cuda")
    flag = torch.zeros((1,), dtype=torch.int32, device="cuda")
    # beyond the 64 MiB array (2 x 1500^2 complex = 72 MB): refused on the
    # host, nothing launched (x is never read, so a small buffer suffices)
    xsmall = torch.zeros((4,), dtype=torch.complex128, device="cuda")
    st = ssrpa.ssrpa_trace_log_noalloc(ctx.handle, xsmall.data_ptr(), 1500, 2,
                                       1.0, f_dev.data_ptr(), flag.data_ptr(),
                                       stream)
    assert st == ssrpa.ERR_ARG
    assert b"64" in ssrpa.ssrpa_last_error(ctx.handle) or \
        b"beyond" in ssrpa.ssrpa_last_error(ctx.handle)
    # matrix 1 has a negative pivot: NaN there, flag raised, matrix 0 exact
    x = np.zeros((2, 4, 4), dtype=np.complex128)
    x[0] = -0.25 * np.eye(4)
    x[1, 2, 2] = 2.0
    xd = torch.from_numpy(x).to("cuda")
    st = ssrpa.ssrpa_trace_log_noalloc(ctx.handle, xd.data_ptr(), 4, 2, 1.0,
                                       f_dev.data_ptr(), flag.data_ptr(),
                                       stream)
    assert st == ssrpa.OK
    torch.cuda.synchronize()
    f = f_dev.cpu().numpy()
    assert int(flag.cpu()[0]) != 0
    assert np.isnan(f[1])
    assert abs(f[0] - 4 * (np.log1p(0.25) - 0.25)) < 1e-15
    # the flag is cleared by the next good call
    x1 = np.zeros((1, 3, 3), dtype=np.complex128)
    xd1 = torch.from_numpy(x1).to("cuda")
    st = ssrpa.ssrpa_trace_log_noalloc(ctx.handle, xd1.data_ptr(), 3, 1, 1.0,
                                       f_dev.data_ptr(), flag.data_ptr(),
                                       stream)
    assert st == ssrpa.OK
    torch.cuda.synchronize()
    assert int(flag.cpu()[0]) == 0 and float(f_dev.cpu()[0]) == 0.0
    ctx.close()
