"""Degenerate and edge inputs on the GPU path, against the oracle:

  * an empty circuit leaves any state bit for bit as it was (fused and one
    kernel per gate, from 1 qubit up to several tiles);
  * circuits made only of permutation gates (X, CNOT, SWAP) and the
    sign-only CZ: the fused pass folds trailing permutations into its write
    and store offsets, so every path must reproduce the oracle exactly;
  * the adjoint sweep of a circuit without rotation angles (value only);
  * a batch holding an empty circuit, a one-gate circuit and a circuit
    without observable terms (whose value is 0);
  * a context rebound to another stream, and the state query;
  * the from-|0...0> flag of the circuit call.
"""
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


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context()
    yield c
    c.close()


@pytest.mark.parametrize("n", [1, 5, 14])
def test_empty_circuit_is_identity(q, ctx, n):
    for dtype in (q.QSV_C128, q.QSV_C64):
        a = W.random_state(n, seed=40 + n).astype(np.complex128 if dtype == q.QSV_C128 else np.complex64)
        st = q.State(ctx, n, dtype)
        for flags in (0, q.FLAG_NO_FUSE):
            st.from_numpy(a)
            st.apply_circuit([], flags=flags)
            assert np.array_equal(st.to_numpy(), a)
        st.free()


def permutation_circuit(n, ngates, seed):
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(ngates):
        k = int(rng.integers(4))
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        if k == 0:
            gates.append(W.g1(a, W.X))
        elif k == 1:
            gates.append(W.cnot(a, b))
        elif k == 2:
            gates.append(W.g2(a, b, W.SWAP))
        else:
            gates.append(W.cz(a, b))
    return W.Circuit(n, gates)


@pytest.mark.parametrize("n,ngates,seed", [(3, 12, 1), (12, 40, 2), (15, 80, 3)])
def test_permutation_circuits_are_exact(q, ctx, n, ngates, seed):
    c = permutation_circuit(n, ngates, seed)
    start = W.random_state(n, seed=seed)
    ref = O.run(c, state=start)
    for dtype in (q.QSV_C128, q.QSV_C64):
        cdt = np.complex128 if dtype == q.QSV_C128 else np.complex64
        st = q.State(ctx, n, dtype)
        for flags in (0, q.FLAG_NO_FUSE):
            st.from_numpy(start.astype(cdt))
            st.apply_circuit(c.gates, flags=flags)
            # the oracle moves FP64 values; in FP32 the same moves of the
            # rounded start values are exact too
            want = ref if dtype == q.QSV_C128 else O.run(c, state=start.astype(np.complex64).astype(np.complex128))
            assert np.array_equal(st.to_numpy().astype(np.complex128), want.astype(cdt).astype(np.complex128)), flags
        st.free()


def test_adjoint_without_angles(q, ctx):
    c = W.random_mix(11, 50, seed=9)
    c.observable = [((0, 10), 0.7), ((3,), -1.2)]
    f_ref = O.expect_obs(O.run(c), c.observable)
    psi, lam = q.State(ctx, c.n), q.State(ctx, c.n)
    for flags in (q.FLAG_FORWARD, q.FLAG_FORWARD | q.FLAG_NO_FUSE):
        f, g = q.adjoint(psi, lam, c.gates, None, c.observable, flags=flags)
        assert abs(f - f_ref) <= 1e-12 * 1.9
        assert g.size == 0
    psi.free()
    lam.free()


@pytest.mark.parametrize("dtype", [2, 1])
def test_batch_with_empty_and_termless_circuits(q, ctx, dtype):
    rng = np.random.default_rng(77)
    empty = W.Circuit(6, [], np.zeros(0), [((0,), 1.0), ((5,), 0.5)])
    one = W.Circuit(4, [W.g1(2, W.haar_unitary(2, rng))], np.zeros(0), [((2,), 1.0)])
    termless = W.random_mix(9, 30, seed=5)
    termless.observable = []
    full = W.ry_rz_cnot_ladder(13, 2, rng)
    circs = [empty, one, termless, full]
    got = ctx.batch_run(circs, dtype)
    ref = np.array([O.expect_obs(O.run(c), c.observable) if c.observable else 0.0 for c in circs])
    assert got[0] == pytest.approx(1.5, abs=1e-15)
    assert got[2] == 0.0
    assert np.max(np.abs(got - ref)) <= (1e-12 if dtype == 2 else 2e-5) * 2


def test_context_on_a_torch_stream_and_state_info(q):
    """A context rebound to a torch stream runs there (results by the oracle);
    qsv_state_info reports the wrapped buffer."""
    import ctypes
    import torch
    lib = q.qsv.lib()
    s = torch.cuda.Stream()
    ctx = q.Context()
    ctx.set_stream(s.cuda_stream)
    c = W.random_mix(12, 60, seed=21)
    for dtype in (q.QSV_C128, q.QSV_C64):
        st = q.State(ctx, 12, dtype)
        n, dt, ptr = ctypes.c_int(), ctypes.c_int(), ctypes.c_void_p()
        assert lib.qsv_state_info(st.handle, ctypes.byref(n), ctypes.byref(dt), ctypes.byref(ptr)) == 0
        assert (n.value, dt.value, ptr.value) == (12, dtype, st.tensor.data_ptr())
        st.init_basis(0)
        st.apply_circuit(c.gates)
        s.synchronize()
        got = st.tensor.cpu().numpy().astype(np.complex128)
        ref = O.run(c)
        if dtype == q.QSV_C128:
            assert np.max(np.abs(got - ref)) < 1e-12
        else:
            assert 1.0 - abs(np.vdot(got, ref)) ** 2 < 1e-6
        st.free()
    ctx.close()


@pytest.mark.parametrize("n", [9, 12, 16])
def test_from_zero_flag(q, ctx, n):
    """QSV_FLAG_FROM_ZERO: the result is the circuit applied to |0...0>
    whatever the state held before (the first fused pass makes |0...0> in
    registers); also with one kernel per gate, a circuit whose first pass is
    a single gate, and an empty circuit."""
    rng = np.random.default_rng(500 + n)
    c = W.random_mix(n, 40, seed=60 + n)
    one = [W.g1(n - 1, W.haar_unitary(2, rng))]
    ref = O.run(c)
    ref_one = O.run(W.Circuit(n, one))
    zero = O.basis(n)
    junk = W.random_state(n, seed=7)
    for dtype in (q.QSV_C128, q.QSV_C64):
        cdt = np.complex128 if dtype == q.QSV_C128 else np.complex64
        st = q.State(ctx, n, dtype)
        for gates, want in ((c.gates, ref), (one, ref_one), ([], zero)):
            for flags in (q.FLAG_FROM_ZERO, q.FLAG_FROM_ZERO | q.FLAG_NO_FUSE):
                st.from_numpy(junk.astype(cdt))
                st.apply_circuit(gates, flags=flags)
                got = st.to_numpy().astype(np.complex128)
                if dtype == q.QSV_C128:
                    assert np.max(np.abs(got - want)) < 1e-12, (len(gates), flags)
                else:
                    assert 1.0 - abs(np.vdot(got, want)) ** 2 < 1e-6, (len(gates), flags)
        st.free()
