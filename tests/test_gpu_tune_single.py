"""Single-state tile-shape tuning (QSV_FLAG_TUNE on qsv_apply_circuit): the
state after the tuning call, and after a later call that reuses the chosen
shape, equals the FP64 oracle's |0...0> run; the flag is refused without
QSV_FLAG_FROM_ZERO; the context's own tile shape is left as it was."""
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


def zero_ref(c):
    phi = np.zeros(1 << c.n, dtype=np.complex128)
    phi[0] = 1.0
    return O.run(c, phi)


@pytest.mark.parametrize("jit", [0, 1])
def test_tuned_apply_matches_oracle(q, jit):
    ctx = q.Context()
    ctx.set_jit(jit)
    flags = q.FLAG_FROM_ZERO | q.FLAG_TUNE
    cases = [W.layered_cnot_brick(17, 3, seed=1701), W.random_multicontrol(15, 80, seed=1703)]
    if not jit:   # with specialised kernels every candidate shape compiles its own
        cases.append(W.random_mix(16, 200, seed=1702))
    for c in cases:
        ref = zero_ref(c)
        st = q.State(ctx, c.n, q.QSV_C128)
        st.init_basis(5)          # overwritten: the flag starts from |0...0>
        st.apply_circuit(c.gates, params=c.params, flags=flags)
        assert np.max(np.abs(st.to_numpy() - ref)) <= TOL128, (c.name, "tuning call")
        st.init_basis(3)
        st.apply_circuit(c.gates, params=c.params, flags=flags)
        assert np.max(np.abs(st.to_numpy() - ref)) <= TOL128, (c.name, "tuned call")
        # the context's shape still serves calls without the flag
        st.init_basis(0)
        st.apply_circuit(c.gates, params=c.params)
        assert np.max(np.abs(st.to_numpy() - ref)) <= TOL128, (c.name, "untuned call")
        st.free()
    ctx.close()


def test_tuned_apply_c64_and_small(q):
    ctx = q.Context()
    for n in (10, 11, 12, 14):
        c = W.random_mix(n, 60, seed=1710 + n)
        ref = zero_ref(c)
        st = q.State(ctx, n, q.QSV_C64)
        st.apply_circuit(c.gates, params=c.params, flags=q.FLAG_FROM_ZERO | q.FLAG_TUNE)
        got = st.to_numpy().astype(np.complex128)
        assert 1.0 - abs(np.vdot(got, ref)) ** 2 <= 1e-6, n
        st.free()
    ctx.close()


def test_tune_needs_from_zero(q):
    ctx = q.Context()
    c = W.random_mix(12, 20, seed=1720)
    st = q.State(ctx, 12, q.QSV_C128)
    with pytest.raises(q.QsvError, match="FROM_ZERO"):
        st.apply_circuit(c.gates, params=c.params, flags=q.FLAG_TUNE)
    st.free()
    ctx.close()
