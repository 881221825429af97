"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.  complex128 amplitudes must agree to 1e-12 (max abs);
complex64 results are checked by infidelity 1 - |<psi64|psi128>|^2 <= 1e-6."""
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


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context()
    yield c
    c.close()


def make_state(q, ctx, n, dtype=None, init=None):
    dtype = q.QSV_C128 if dtype is None else dtype
    st = q.State(ctx, n, dtype)
    if init is None:
        st.init_basis(0)
    else:
        st.from_numpy(init)
    return st


def infidelity(a64, b128):
    ov = np.vdot(a64.astype(np.complex128), b128)
    return 1.0 - abs(ov) ** 2


# ---------------------------------------------------------------- init
@pytest.mark.parametrize("n", [1, 2, 5, 11, 16])
def test_init_basis(q, ctx, n):
    rng = np.random.default_rng(n)
    for dtype in (q.QSV_C128, q.QSV_C64):
        st = q.State(ctx, n, dtype)
        for b in {0, 2 ** n - 1, int(rng.integers(2 ** n))}:
            st.init_basis(b)
            v = st.to_numpy()
            ref = np.zeros(2 ** n)
            ref[b] = 1
            assert np.array_equal(v, ref.astype(v.dtype))


# ------------------------------------------------------- single gates
@pytest.mark.parametrize("n", [1, 2, 3, 5, 9, 14])
def test_apply1q_every_qubit(q, ctx, n):
    rng = np.random.default_rng(100 + n)
    phi = W.random_state(n, 1000 + n)
    for qb in range(n):
        u = W.haar_unitary(2, rng)
        st = make_state(q, ctx, n, init=phi)
        st.apply1q(qb, u)
        assert np.max(np.abs(st.to_numpy() - O.apply_1q(phi, qb, u))) <= TOL128, qb


@pytest.mark.parametrize("n", [2, 3, 6, 13])
def test_applyc1q_pairs_and_states(q, ctx, n):
    rng = np.random.default_rng(200 + n)
    phi = W.random_state(n, 2000 + n)
    pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
    if len(pairs) > 24:
        pairs = [pairs[i] for i in rng.choice(len(pairs), 24, replace=False)]
    for qc, qt in pairs:
        for cs in (0, 1):
            u = W.haar_unitary(2, rng)
            st = make_state(q, ctx, n, init=phi)
            st.applyC1q(qc, qt, u, cs)
            ref = O.apply_c1q(phi, qc, qt, u, cs)
            assert np.max(np.abs(st.to_numpy() - ref)) <= TOL128, (qc, qt, cs)


@pytest.mark.parametrize("n", [2, 3, 6, 13])
def test_apply2q_any_pair(q, ctx, n):
    rng = np.random.default_rng(300 + n)
    phi = W.random_state(n, 3000 + n)
    pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
    if len(pairs) > 24:
        pairs = [pairs[i] for i in rng.choice(len(pairs), 24, replace=False)]
    for qa, qb in pairs:
        u = W.haar_unitary(4, rng)
        st = make_state(q, ctx, n, init=phi)
        st.apply2q(qa, qb, u)
        assert np.max(np.abs(st.to_numpy() - O.apply_2q(phi, qa, qb, u))) <= TOL128, (qa, qb)


def test_pairings_match_paper_index_maps(q, ctx):
    """Apply X / CNOT / SWAP to the state phi[x] = x: the result reveals which
    index each amplitude was paired with; it must match the index maps of
    Algs. 1-3 (exact integers)."""
    from oracle import indices as IX
    n = 7
    enc = np.arange(2 ** n, dtype=np.complex128)
    for qb in range(n):
        st = make_state(q, ctx, n, init=enc)
        st.apply1q(qb, W.X)
        v = st.to_numpy().real.astype(np.int64)
        for a, b in IX.pairs_1q(n, qb):
            assert v[a] == b and v[b] == a
    for qc in range(n):
        for qt in range(n):
            if qc == qt:
                continue
            for cs in (0, 1):
                st = make_state(q, ctx, n, init=enc)
                st.applyC1q(qc, qt, W.X, cs)
                v = st.to_numpy().real.astype(np.int64)
                moved = set()
                for a, b in IX.pairs_c1q(n, qc, qt, cs):
                    assert v[a] == b and v[b] == a
                    moved |= {a, b}
                rest = [x for x in range(2 ** n) if x not in moved]
                assert np.array_equal(v[rest], np.array(rest))
            st = make_state(q, ctx, n, init=enc)
            st.apply2q(qc, qt, W.SWAP)
            v = st.to_numpy().real.astype(np.int64)
            for a, b, c, d in IX.quads_2q(n, qc, qt):
                assert v[a] == a and v[d] == d and v[b] == c and v[c] == b


# ------------------------------------------------------------- circuits
@pytest.mark.parametrize("flags", [0, 1])
def test_mix10_state_and_z(q, ctx, flags):
    c = W.mix_n10_g200()
    st = make_state(q, ctx, c.n)
    st.apply_circuit(c.gates, flags=flags)
    ref = O.run(c)
    assert np.max(np.abs(st.to_numpy() - ref)) <= TOL128
    terms, _ = st.expect_z(c.observable)
    ref_terms = np.array([O.expect_z(ref, qs) for qs, _ in c.observable])
    assert np.max(np.abs(terms - ref_terms)) <= TOL128


@pytest.mark.parametrize("n,seed", [(13, 1), (15, 2), (17, 3)])
def test_fused_multi_tile_vs_oracle(q, ctx, n, seed):
    """States larger than one tile: many tiles per pass, many passes."""
    c = W.random_mix(n, 120, seed=seed)
    phi = W.random_state(n, seed + 50)
    st = make_state(q, ctx, n, init=phi)
    st.apply_circuit(c.gates)
    ref = O.run(c, phi)
    assert np.max(np.abs(st.to_numpy() - ref)) <= TOL128


@pytest.mark.parametrize("lr", [1, 2])
@pytest.mark.parametrize("tb,lb", [(10, 1), (10, 8), (11, 3), (12, 3), (12, 8), (12, 10), (13, 3)])
def test_tile_shapes_agree(q, ctx, tb, lb, lr):
    """Every tile size, low-bit count and both LDS exchanges (whole tile,
    or two half-tile rounds) against the oracle."""
    n = 14
    c = W.random_mix(n, 80, seed=tb * 10 + lb)
    ref = O.run(c)
    c2 = q.Context()
    c2.set_tile(q.QSV_C128, tb, lb, 0, lr)
    c2.set_tile(q.QSV_C64, min(tb + 1, 13), lb, 0, lr)
    st = make_state(q, c2, n)
    st.apply_circuit(c.gates)
    assert np.max(np.abs(st.to_numpy() - ref)) <= TOL128
    s64 = make_state(q, c2, n, q.QSV_C64)
    s64.apply_circuit(c.gates)
    assert infidelity(s64.to_numpy(), ref) <= 1e-6
    st.free()
    s64.free()
    c2.close()


def permutation_mix(n, ngates, seed):
    """Random circuit rich in permutation gates (X, CNOT on either control
    state, SWAP) between Haar gates, so that many register stages end in
    permutation gates (which the kernels fold into their write offsets)."""
    rng = np.random.default_rng(seed)
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    SWAP = np.eye(4)[[0, 2, 1, 3]].astype(complex)
    gates = []
    for _ in range(ngates):
        r = rng.random()
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        if r < 0.2:
            gates.append(W.g1(a, X))
        elif r < 0.45:
            gates.append(W.gc(a, b, X, cs=int(rng.integers(2))))
        elif r < 0.6:
            gates.append(W.g2(a, b, SWAP))
        elif r < 0.8:
            gates.append(W.g1(a, W.haar_unitary(2, rng)))
        else:
            gates.append(W.g2(a, b, W.haar_unitary(4, rng)))
    return W.Circuit(n, gates, name="permutation_mix")


@pytest.mark.parametrize("lr", [1, 2])
@pytest.mark.parametrize("tb,lb,rb", [(12, 3, 4), (11, 3, 3), (10, 3, 2), (12, 3, 3), (13, 3, 5), (13, 3, 4)])
def test_permutation_gates_at_stage_ends(q, tb, lb, rb, lr):
    n = 14
    c = permutation_mix(n, 160, seed=tb * 100 + rb)
    phi = W.random_state(n, 77)
    ref = O.run(c, phi)
    c2 = q.Context()
    c2.set_tile(q.QSV_C128, tb, lb, rb, lr)
    c2.set_tile(q.QSV_C64, tb, lb + 1 if lb < 4 else lb, rb, lr)
    st = make_state(q, c2, n, init=phi)
    st.apply_circuit(c.gates)
    assert np.max(np.abs(st.to_numpy() - ref)) <= TOL128
    s64 = make_state(q, c2, n, q.QSV_C64, init=phi.astype(np.complex64))
    s64.apply_circuit(c.gates)
    assert infidelity(s64.to_numpy(), ref) <= 1e-6
    st.free()
    s64.free()
    c2.close()


def test_set_tile_rejects_bad_shapes(q):
    c2 = q.Context()
    for args in [(14, 3, 0, 0), (9, 3, 0, 0), (12, 11, 0, 0), (12, 3, 6, 0), (13, 3, 3, 0), (12, 3, 4, 3)]:
        with pytest.raises(q.QsvError):
            c2.set_tile(q.QSV_C128, *args)
    c2.set_tile(q.QSV_C128, 13, 3, 5, 2)    # the defaults, spelled out
    c2.close()


def test_layered_brick_and_qft(q, ctx):
    c = W.layered_cnot_brick(16, 4, seed=11)
    st = make_state(q, ctx, 16)
    st.apply_circuit(c.gates)
    ref = O.run(c)
    assert np.max(np.abs(st.to_numpy() - ref)) <= TOL128
    for n in (3, 8, 14):
        phi = W.random_state(n, n)
        st = make_state(q, ctx, n, init=phi)
        st.apply_circuit(W.qft(n).gates)
        assert np.max(np.abs(st.to_numpy() - np.fft.fft(phi) / np.sqrt(2 ** n))) <= TOL128


def test_rotations_in_circuit(q, ctx):
    c = W.hea_cz_ring(9, 3, seed=4)
    st = make_state(q, ctx, c.n)
    st.apply_circuit(c.gates, c.params)
    assert np.max(np.abs(st.to_numpy() - O.run(c))) <= TOL128


# ------------------------------------------------------------- complex64
@pytest.mark.parametrize("n,ng", [(10, 200), (15, 150)])
def test_c64_infidelity(q, ctx, n, ng):
    c = W.random_mix(n, ng, seed=n)
    st = make_state(q, ctx, n, q.QSV_C64)
    st.apply_circuit(c.gates)
    ref = O.run(c)
    v = st.to_numpy()
    assert infidelity(v, ref) <= 1e-6
    assert abs(st.norm2() - 1.0) <= 1e-5
    st128 = make_state(q, ctx, n)
    st128.from_numpy(ref)
    ov = st.inner(st128)
    assert abs(1 - abs(ov) ** 2 - infidelity(v, ref)) < 1e-9


# ------------------------------------------------------------- reductions
def test_reductions_vs_oracle(q, ctx):
    n = 16
    rng = np.random.default_rng(9)
    a, b = W.random_state(n, 91), W.random_state(n, 92)
    sa, sb = make_state(q, ctx, n, init=a), make_state(q, ctx, n, init=b)
    assert abs(sa.norm2() - O.norm2(a)) <= 1e-13
    obs = [(tuple(sorted(rng.choice(n, size=k, replace=False).tolist())), float(rng.standard_normal()))
           for k in (1, 2, 3, 5, 1, 2) for _ in range(5)]
    terms, tot = sa.expect_z(obs)
    ref = np.array([O.expect_z(a, qs) for qs, _ in obs])
    assert np.max(np.abs(terms - ref)) <= 1e-13
    assert abs(tot - O.expect_obs(a, obs)) <= 1e-12
    assert abs(sa.inner(sb) - O.inner(a, b)) <= 1e-13
    for qb in range(n):
        assert abs(sa.prob1(qb) - O.prob1(a, qb)) <= 1e-13
    s64 = make_state(q, ctx, n, q.QSV_C64, init=b.astype(np.complex64))
    ref = O.inner(a, b.astype(np.complex64).astype(np.complex128))
    assert abs(sa.inner(s64) - ref) <= 1e-12


def test_reductions_repeatable(q, ctx):
    n = 20
    st = make_state(q, ctx, n)
    st.apply_circuit(W.random_mix(n, 40, seed=3).gates)
    vals = {st.norm2() for _ in range(3)}
    assert len(vals) == 1


def test_measure_collapse(q, ctx):
    n = 12
    phi = W.random_state(n, 33)
    for qb in (0, 5, 11):
        p1 = O.prob1(phi, qb)
        for r in (0.5 * (1 - p1), 1 - 0.5 * p1):
            st = make_state(q, ctx, n, init=phi)
            k = st.measure1(qb, r)
            kr, post = O.measure1(phi, qb, r)
            assert k == kr
            assert np.max(np.abs(st.to_numpy() - post)) <= TOL128


# ------------------------------------------------------------- gradients
@pytest.mark.parametrize("n,layers", [(4, 2), (7, 3), (13, 2)])
def test_adjoint_vs_oracle(q, ctx, n, layers):
    c = W.hea_cz_ring(n, layers, seed=n)
    f_ref, g_ref = O.adjoint(c)
    psi, lam = q.State(ctx, n), q.State(ctx, n)
    f, g = q.adjoint(psi, lam, c.gates, c.params, c.observable)
    wsum = max(1.0, sum(abs(w) for _, w in c.observable))
    assert abs(f - f_ref) <= 1e-12 * wsum
    assert np.max(np.abs(g - g_ref)) <= 1e-10 * wsum
    ps = O.param_shift(c, sel=range(0, len(c.params), 5))
    assert np.max(np.abs(g[::5] - ps)) <= 1e-10 * wsum
    p64, l64 = q.State(ctx, n, q.QSV_C64), q.State(ctx, n, q.QSV_C64)
    f64, g64 = q.adjoint(p64, l64, c.gates, c.params, c.observable)
    assert abs(f64 - f_ref) <= 1e-4 * wsum
    assert np.max(np.abs(g64 - g_ref)) <= 1e-4 * wsum


def test_adjoint_ry_ladder(q, ctx):
    rng = np.random.default_rng(5)
    c = W.ry_rz_cnot_ladder(8, 3, rng)
    f_ref, g_ref = O.adjoint(c)
    psi, lam = q.State(ctx, c.n), q.State(ctx, c.n)
    f, g = q.adjoint(psi, lam, c.gates, c.params, c.observable, flags=q.FLAG_FORWARD | q.FLAG_NO_FUSE)
    assert abs(f - f_ref) <= 1e-12 * c.n
    assert np.max(np.abs(g - g_ref)) <= 1e-10 * c.n


# ------------------------------------------------------------- errors
def test_invalid_arguments_leave_state_untouched(q, ctx):
    n = 6
    phi = W.random_state(n, 44)
    st = make_state(q, ctx, n, init=phi)
    bad = [
        lambda: st.apply1q(n, W.H),
        lambda: st.apply1q(-1, W.H),
        lambda: st.applyC1q(2, 2, W.X),
        lambda: st.applyC1q(1, 2, W.X, 2),
        lambda: st.apply2q(3, 3, W.SWAP),
        lambda: st.apply2q(0, n, W.SWAP),
        lambda: st.apply_circuit([W.g1(0, W.H), W.g1(n + 3, W.H)]),
        lambda: st.prob1(n),
        lambda: st.measure1(0, 1.5),
        lambda: st.init_basis(2 ** n),
    ]
    for f in bad:
        with pytest.raises(q.QsvError):
            f()
    assert np.array_equal(st.to_numpy(), phi)


def test_wrap_rejects_bad_buffers(q, ctx):
    import ctypes
    import torch
    t = torch.empty(2 ** 5 + 1, dtype=torch.complex128, device="cuda")
    h = ctypes.c_void_p()
    L = q.lib()
    assert L.qsv_state_wrap(ctx.handle, ctypes.c_void_p(t.data_ptr() + 8), 2 ** 5 * 16, 5,
                            q.QSV_C128, ctypes.byref(h)) == 6     # misaligned
    assert L.qsv_state_wrap(ctx.handle, ctypes.c_void_p(t.data_ptr()), 2 ** 5 * 16 - 1, 5,
                            q.QSV_C128, ctypes.byref(h)) == 7     # too small
    assert L.qsv_state_wrap(ctx.handle, ctypes.c_void_p(t.data_ptr()), 2 ** 5 * 16, 5, 3,
                            ctypes.byref(h)) == 5                 # dtype
    assert L.qsv_state_wrap(ctx.handle, ctypes.c_void_p(t.data_ptr()), 2 ** 5 * 16, 0,
                            q.QSV_C128, ctypes.byref(h)) == 7     # n
    hh = ctypes.c_void_p()
    assert L.qsv_state_alloc(ctx.handle, 36, q.QSV_C128, ctypes.byref(hh)) == 3   # 1 TiB: no memory
