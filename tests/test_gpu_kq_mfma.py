"""Dense k-qubit gates (Sec. 2.4) on the matrix cores (qsv_set_matrix_cores):
FP64 MFMA for complex128, FP32 MFMA for complex64, against the FP64 oracle's
k-qubit gate on the same seeded inputs (complex128 max |d amp| <= 1e-12,
complex64 infidelity <= 1e-6), for k = 3, 4, 5 on contiguous, scattered,
descending and lowest-bit qubit sets (mode 2: matrix cores for every k),
the default mode's choice of kernel (matrix cores for k = 3 and 5), the
vector kernel agreeing with them, the sizes where the matrix-core form does
not apply (n - k < 6) and a 20-qubit state."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL128 = 1e-12


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2303_00123_amd as qq
    return qq


def infidelity(a64, b128):
    ov = np.vdot(a64.astype(np.complex128), b128)
    return 1.0 - abs(ov) ** 2


def run(q, ctx, n, dtype, phi, qs, u):
    st = q.State(ctx, n, dtype)
    st.from_numpy(phi.astype(np.complex128 if dtype == q.QSV_C128 else np.complex64))
    st.applyKq(qs, u)
    out = st.to_numpy()
    st.free()
    return out


QUBIT_SETS = {
    3: [[0, 1, 2], [11, 4, 7], [12, 13, 0], [2, 1, 0]],
    4: [[0, 1, 2, 3], [13, 2, 9, 5], [3, 2, 1, 0], [12, 0, 7, 13]],
    5: [[0, 1, 2, 3, 4], [13, 1, 8, 4, 11], [4, 3, 2, 1, 0], [9, 13, 0, 12, 6]],
}


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [3, 4, 5])
def test_matrix_core_kq_vs_oracle(q, dtype, k):
    dt = q.QSV_C128 if dtype == "c128" else q.QSV_C64
    rng = np.random.default_rng(5100 + k)
    n = 14
    ctx = q.Context()
    ctx.set_matrix_cores(2)
    for i, qs in enumerate(QUBIT_SETS[k]):
        u = W.haar_unitary(2 ** k, rng)
        phi = W.random_state(n, 5110 + 10 * k + i)
        ref = O.apply_kq(phi, qs, u)
        got = run(q, ctx, n, dt, phi, qs, u)
        if dt == q.QSV_C128:
            assert np.max(np.abs(got - ref)) <= TOL128, qs
        else:
            assert infidelity(got, ref) <= 1e-6, qs
    ctx.close()


@pytest.mark.parametrize("k", [3, 4, 5])
def test_matrix_cores_and_vector_units_agree(q, k):
    """Same gate both ways: the two kernels differ only in summation order."""
    rng = np.random.default_rng(5200 + k)
    n = 16
    qs = [int(x) for x in rng.choice(n, size=k, replace=False)]
    u = W.haar_unitary(2 ** k, rng)
    phi = W.random_state(n, 5210 + k)
    outs = []
    for mode in (2, 0):
        ctx = q.Context()
        ctx.set_matrix_cores(mode)
        outs.append(run(q, ctx, n, q.QSV_C128, phi, qs, u))
        ctx.close()
    assert np.max(np.abs(outs[0] - outs[1])) <= 1e-13


def test_small_states_use_the_vector_kernel(q):
    """n - k < 6: the matrix-core form does not apply; the call is still exact."""
    rng = np.random.default_rng(5300)
    ctx = q.Context()
    ctx.set_matrix_cores(1)
    for n, k in ((8, 3), (9, 4), (10, 5), (5, 5)):
        qs = [int(x) for x in rng.choice(n, size=k, replace=False)]
        u = W.haar_unitary(2 ** k, rng)
        phi = W.random_state(n, 5310 + n)
        got = run(q, ctx, n, q.QSV_C128, phi, qs, u)
        assert np.max(np.abs(got - O.apply_kq(phi, qs, u))) <= TOL128, (n, k)
    ctx.close()


def test_matrix_core_kq_20_qubits(q):
    rng = np.random.default_rng(5400)
    n, qs = 20, [19, 0, 7, 12, 3]
    u = W.haar_unitary(32, rng)
    phi = W.random_state(n, 5401)
    ref = O.apply_kq(phi, qs, u)
    ctx = q.Context()
    ctx.set_matrix_cores(2)
    got = run(q, ctx, n, q.QSV_C128, phi, qs, u)
    assert np.max(np.abs(got - ref)) <= TOL128
    got64 = run(q, ctx, n, q.QSV_C64, phi, qs, u)
    assert infidelity(got64, ref) <= 1e-6
    ctx.close()


def test_default_mode_picks_matrix_cores_for_k3_and_k5(q):
    rng = np.random.default_rng(5500)
    ctx = q.Context()
    st = q.State(ctx, 12, q.QSV_C128)
    st.init_basis(0)
    for k, want in ((3, "kq_mfma_c128"), (4, "kq_c128"), (5, "kq_mfma_c128")):
        ctx.profile_begin()
        st.applyKq(list(range(k)), W.haar_unitary(2 ** k, rng))
        prof = ctx.profile_end()
        assert list(prof) == [want], (k, prof)
    st.free()
    ctx.close()


def test_matrix_core_mode_is_checked(q):
    ctx = q.Context()
    for bad in (-1, 3):
        with pytest.raises(q.QsvError):
            ctx.set_matrix_cores(bad)
    ctx.close()
