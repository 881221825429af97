"""Adjoint-gradient sweep: fused two-vector tile passes vs one kernel per
gate vs the FP64 oracle (adjoint and parameter shift), and the 24-qubit
configuration against parameter shift evaluated with the GPU forward pass."""
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


def wsum(c):
    return max(1.0, sum(abs(w) for _, w in c.observable))


@pytest.mark.parametrize("maker", [
    lambda: W.hea_cz_ring(12, 3, seed=12),
    lambda: W.hea_cz_ring(14, 4, seed=14, ring_obs=True),
    lambda: W.ry_rz_cnot_ladder(15, 3, np.random.default_rng(15)),
])
def test_fused_adjoint_vs_unfused_and_oracle(q, ctx, maker):
    c = maker()
    f_ref, g_ref = O.adjoint(c)
    psi, lam = q.State(ctx, c.n), q.State(ctx, c.n)
    f1, g1 = q.adjoint(psi, lam, c.gates, c.params, c.observable)                     # fused
    f2, g2 = q.adjoint(psi, lam, c.gates, c.params, c.observable,
                       flags=q.FLAG_FORWARD | q.FLAG_NO_FUSE)                         # unfused
    tol = 1e-10 * wsum(c)
    assert abs(f1 - f_ref) <= 1e-12 * wsum(c) and abs(f2 - f_ref) <= 1e-12 * wsum(c)
    assert np.max(np.abs(g1 - g_ref)) <= tol
    assert np.max(np.abs(g2 - g_ref)) <= tol
    sel = list(range(0, len(c.params), 7))
    assert np.max(np.abs(g1[sel] - O.param_shift(c, sel))) <= tol
    # the oracle's central finite differences (h = 1e-6): truncation ~h^2,
    # rounding ~1e-16 |f| / h
    assert np.max(np.abs(g1[sel[:5]] - O.finite_diff(c, sel[:5]))) <= 1e-7 * wsum(c)
    # psi is rewound to |0...0>
    v = psi.to_numpy()
    assert abs(v[0] - 1.0) <= 1e-10 and abs(np.linalg.norm(v) - 1.0) <= 1e-10
    p64, l64 = q.State(ctx, c.n, q.QSV_C64), q.State(ctx, c.n, q.QSV_C64)
    f3, g3 = q.adjoint(p64, l64, c.gates, c.params, c.observable)
    assert np.max(np.abs(g3 - g_ref)) <= 1e-4 * wsum(c)


def test_hea24_adjoint_vs_gpu_parameter_shift(q, ctx):
    """24 qubits, 10 layers RY,RZ + CZ ring, 480 parameters: the fused adjoint
    gradient against parameter shift on 24 sampled parameters, each shifted
    energy evaluated with the (oracle-validated) GPU forward pass."""
    c = W.hea_n24()
    psi, lam = q.State(ctx, c.n), q.State(ctx, c.n)
    f, g = q.adjoint(psi, lam, c.gates, c.params, c.observable)
    g_unf = q.adjoint(psi, lam, c.gates, c.params, c.observable,
                      flags=q.FLAG_FORWARD | q.FLAG_NO_FUSE)[1]
    marsh = q.marshal_gates(c.gates)

    def energy(params):
        psi.init_basis(0)
        psi.apply_circuit(None, params, marshalled=marsh)
        return psi.expect_z(c.observable)[1]

    assert abs(energy(c.params) - f) <= 1e-11 * wsum(c)
    rng = np.random.default_rng(55)
    sel = rng.choice(len(c.params), size=24, replace=False)
    for j in sel:
        p = c.params.copy()
        p[j] += np.pi / 2
        fp = energy(p)
        p[j] -= np.pi
        fm = energy(p)
        assert abs(g[j] - 0.5 * (fp - fm)) <= 1e-10 * wsum(c), j
    assert np.max(np.abs(g - g_unf)) <= 1e-11 * wsum(c)
    # central finite differences, h = 1e-6, FP64 forward passes
    h = 1e-6
    for j in sel[:8]:
        p = c.params.copy()
        p[j] += h
        fp = energy(p)
        p[j] -= 2 * h
        fm = energy(p)
        assert abs(g[j] - (fp - fm) / (2 * h)) <= 1e-6 * wsum(c), j
    p64, l64 = q.State(ctx, c.n, q.QSV_C64), q.State(ctx, c.n, q.QSV_C64)
    g64 = q.adjoint(p64, l64, c.gates, c.params, c.observable)[1]
    assert np.max(np.abs(g64 - g)) <= 1e-4 * wsum(c)


@pytest.mark.parametrize("n,layers,seed", [(12, 3, 41), (14, 3, 42), (15, 4, 43)])
def test_adjoint_through_general_fixed_gates(q, ctx, n, layers, seed):
    """Rotations interleaved with Haar 1q, Haar 2q (both qubit orders) and
    controlled Haar gates (control state 0 and 1), none of them its own
    inverse: the sweep rewinds each with its conjugate transpose.  Fused and
    one kernel per gate, complex128 and complex64, against the oracle's
    adjoint sweep (pinned by dense-matrix derivatives) and its parameter
    shift."""
    c = W.mixed_param_circuit(n, layers, seed)
    f_ref, g_ref = O.adjoint(c)
    tol = 1e-10 * wsum(c)
    psi, lam = q.State(ctx, c.n), q.State(ctx, c.n)
    for flags in (q.FLAG_FORWARD, q.FLAG_FORWARD | q.FLAG_NO_FUSE):
        f, g = q.adjoint(psi, lam, c.gates, c.params, c.observable, flags=flags)
        assert abs(f - f_ref) <= 1e-12 * wsum(c), flags
        assert np.max(np.abs(g - g_ref)) <= tol, flags
        v = psi.to_numpy()   # rewound through every gate: back to |0...0>
        assert abs(v[0] - 1.0) <= 1e-10 and np.max(np.abs(v[1:])) <= 1e-10, flags
    sel = list(range(0, len(c.params), 5))
    assert np.max(np.abs(g[sel] - O.param_shift(c, sel))) <= tol
    p64, l64 = q.State(ctx, c.n, q.QSV_C64), q.State(ctx, c.n, q.QSV_C64)
    for flags in (q.FLAG_FORWARD, q.FLAG_FORWARD | q.FLAG_NO_FUSE):
        f3, g3 = q.adjoint(p64, l64, c.gates, c.params, c.observable, flags=flags)
        assert abs(f3 - f_ref) <= 1e-5 * wsum(c), flags
        assert np.max(np.abs(g3 - g_ref)) <= 1e-4 * wsum(c), flags
    for s in (psi, lam, p64, l64):
        s.free()


@pytest.mark.parametrize("dt_name", ["c128", "c64"])
def test_hea_ansatz_20_qubits_vs_oracle_adjoint(q, ctx, dt_name):
    """The configuration's ansatz (10 layers of RY, RZ on every qubit + CZ
    ring, open-chain ZZ observable with N(0,1) weights) at 20 qubits, 400
    parameters: every gradient component of the fused sweep against one
    FP64 oracle adjoint sweep (the 24-qubit sweep takes minutes on the host),
    and a sample against the oracle's parameter shift."""
    c = W.hea_cz_ring(20, 10, seed=1005)
    f_ref, g_ref = O.adjoint(c)
    dt = q.QSV_C128 if dt_name == "c128" else q.QSV_C64
    psi, lam = q.State(ctx, c.n, dt), q.State(ctx, c.n, dt)
    f, g = q.adjoint(psi, lam, c.gates, c.params, c.observable)
    tv, tg = (1e-12, 1e-10) if dt == q.QSV_C128 else (1e-5, 1e-4)
    assert abs(f - f_ref) <= tv * wsum(c)
    assert np.max(np.abs(g - g_ref)) <= tg * wsum(c)
    if dt == q.QSV_C128:
        sel = [0, 1, 57, 199, 398, 399]
        assert np.max(np.abs(g[sel] - O.param_shift(c, sel))) <= tg * wsum(c)
    print(f"20-qubit ansatz {dt_name}: max |d grad| = {np.max(np.abs(g - g_ref)):.3e}", flush=True)
    psi.free()
    lam.free()
