"""qsv_expect_z_dev, the allocation-free entry point (its scratch is a fixed
per-GPU array), called through the C ABI against qsv_expect_z on the same
state: values bit-identical, nothing written past nterms, twice in a row
with the second call smaller, in both precisions; and against the FP64
oracle to 1e-12."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2303_00123_amd as qq
    return qq


def test_expect_z_dev_matches_expect_z(q):
    import torch
    ctx = q.Context()
    L = q.lib()
    # the second call is smaller (fewer qubits, fewer terms, fewer blocks)
    for n, nt, seed in [(15, 37, 1), (11, 5, 2)]:
        rng = np.random.default_rng(900 + seed)
        phi = W.random_state(n, 910 + seed)
        masks = [0] + [int(rng.integers(1, 2 ** n)) for _ in range(nt - 1)]
        obs = [(tuple(qq for qq in range(n) if (m >> qq) & 1), 1.0) for m in masks]
        ref = np.array([O.expect_z(phi, qs) for qs, _ in obs])
        for dtype in (q.QSV_C128, q.QSV_C64):
            st = q.State(ctx, n, dtype)
            st.from_numpy(phi.astype(np.complex128 if dtype == q.QSV_C128 else np.complex64))
            terms, _ = st.expect_z(obs)
            out = torch.full((nt + 8,), float("nan"), dtype=torch.float64, device="cuda")
            m = np.ascontiguousarray(masks, dtype=np.uint64)
            rc = L.qsv_expect_z_dev(st.handle, nt, m.ctypes.data_as(ctypes.c_void_p),
                                    ctypes.c_void_p(out.data_ptr()))
            assert rc == 0, L.qsv_last_error(ctx.handle)
            ctx.sync()
            got = out.cpu().numpy()
            assert np.array_equal(got[:nt], terms)
            assert np.all(np.isnan(got[nt:]))
            if dtype == q.QSV_C128:
                assert np.max(np.abs(got[:nt] - ref)) <= 1e-12
            else:
                assert np.max(np.abs(got[:nt] - ref)) <= 1e-5
            st.free()
    # argument errors leave the output untouched
    st = q.State(ctx, 4, q.QSV_C128)
    st.init_basis(0)
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    bad = np.array([1 << 4], dtype=np.uint64)
    code = {v: k for k, v in q.qsv.STATUS.items()}
    assert L.qsv_expect_z_dev(st.handle, 1, bad.ctypes.data_as(ctypes.c_void_p),
                              ctypes.c_void_p(out.data_ptr())) == code["QSV_ERR_QUBIT"]
    assert L.qsv_expect_z_dev(st.handle, 0, bad.ctypes.data_as(ctypes.c_void_p),
                              ctypes.c_void_p(out.data_ptr())) != 0
    assert L.qsv_expect_z_dev(st.handle, 1, bad.ctypes.data_as(ctypes.c_void_p), None) != 0
    ctx.sync()
    assert np.all(np.isnan(out.cpu().numpy()))
    st.free()
    ctx.close()
