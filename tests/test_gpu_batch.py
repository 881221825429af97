"""Batched persistent launch (qsv_batch_run) against the FP64 oracle and the
single-state path: every circuit's <O> must match, eager, tuned and
graph-replayed (with new angles between replays)."""
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


def mixed_batch(seed):
    """Circuits of many widths: below the tile (padded), exactly one tile,
    and several tiles with several passes; fixed gates and rotations."""
    rng = np.random.default_rng(seed)
    out = []
    for k, n in enumerate([1, 2, 3, 7, 10, 12, 13, 14, 15, 16, 11, 9]):
        if n == 1:
            c = W.Circuit(1, [W.g1(0, W.haar_unitary(2, rng)), W.grot(0, "Y", 0)],
                          np.array([rng.uniform(0, 6.28)]), [((0,), 0.7)])
        elif k % 2:
            c = W.random_mix(n, 60, seed=seed * 100 + k)
            c.observable = [((q,), float(rng.standard_normal())) for q in range(n)]
        else:
            c = W.ry_rz_cnot_ladder(n, 3, rng)
        out.append(c)
    return out


def oracle_values(circs):
    return np.array([O.expect_obs(O.run(c), c.observable) for c in circs])


def tol(c, dtype):
    wsum = max(1.0, sum(abs(w) for _, w in c.observable))
    return (1e-12 if dtype == 2 else 2e-5) * wsum


@pytest.mark.parametrize("dtype", [2, 1])
def test_batch_matches_oracle(q, ctx, dtype):
    circs = mixed_batch(1)
    got = ctx.batch_run(circs, dtype)
    ref = oracle_values(circs)
    for b, c in enumerate(circs):
        assert abs(got[b] - ref[b]) <= tol(c, dtype), (b, c.n, got[b], ref[b])


def test_batch_graph_replays_with_new_angles(q, ctx):
    circs = mixed_batch(2)
    rng = np.random.default_rng(7)
    for rep in range(3):
        for c in circs:
            if c.params.size:
                c.params = rng.uniform(0, 2 * np.pi, size=c.params.size)
        got = ctx.batch_run(circs, q.QSV_C128, flags=q.FLAG_CAPTURE_GRAPH)
        ref = oracle_values(circs)
        for b, c in enumerate(circs):
            assert abs(got[b] - ref[b]) <= tol(c, 2), (rep, b)
        # eager work and synchronisation between replays
        eager = ctx.batch_run(circs, q.QSV_C128)
        assert np.max(np.abs(eager - got)) <= 1e-12


def test_two_part_batch_graph_and_eager(q, ctx):
    """37 circuits (an odd count above the split size: two launches of 18
    and 19): graph replays with new angles and the eager path against the
    oracle, in both precisions."""
    circs = (mixed_batch(4) * 4)[:37]
    circs = [W.Circuit(c.n, list(c.gates), np.array(c.params, dtype=float), list(c.observable)) for c in circs]
    rng = np.random.default_rng(11)
    for rep in range(3):
        for c in circs:
            if c.params.size:
                c.params = rng.uniform(0, 2 * np.pi, size=c.params.size)
        ref = oracle_values(circs)
        for dtype in (2, 1):
            got = ctx.batch_run(circs, dtype, flags=q.FLAG_CAPTURE_GRAPH)
            eager = ctx.batch_run(circs, dtype)
            for b, c in enumerate(circs):
                assert abs(got[b] - ref[b]) <= tol(c, dtype), (rep, dtype, b)
                assert abs(eager[b] - ref[b]) <= tol(c, dtype), (rep, dtype, b)


def test_batch_tuned_shape_is_correct_and_cached(q, ctx):
    circs = mixed_batch(3)
    ref = oracle_values(circs)
    for _ in range(2):
        got = ctx.batch_run(circs, q.QSV_C128, flags=q.FLAG_TUNE)
        for b, c in enumerate(circs):
            assert abs(got[b] - ref[b]) <= tol(c, 2)


@pytest.mark.parametrize("dtype", [2, 1])
def test_ladder_batch_vs_single_state_path(q, ctx, dtype):
    """256 circuits, 12..20 qubits, 6 layers RY RZ + CNOT ladder: each batch
    result against the same circuit run alone through qsv_apply_circuit."""
    circs = W.ladder_batch_256()
    got = ctx.batch_run(circs, dtype)
    for b, c in enumerate(circs):
        st = q.State(ctx, c.n, dtype)
        st.init_basis(0)
        st.apply_circuit(c.gates, c.params)
        ref = st.expect_z(c.observable)[1]
        st.free()
        assert abs(got[b] - ref) <= (1e-11 if dtype == 2 else 1e-5 * c.n), (b, c.n)


@pytest.fixture(scope="module")
def ladder_batch_oracle():
    """<sum_i Z_i> of every circuit of the 256-circuit ladder batch (256 circuits, 12..20 qubits)
    from the FP64 oracle: about a minute on the host, shared by both dtypes."""
    circs = W.ladder_batch_256()
    vals = []
    for b, c in enumerate(circs):
        vals.append(O.expect_obs(O.run(c), c.observable))
        if b % 64 == 63:
            print(f"ladder batch oracle: {b + 1}/{len(circs)} circuits", flush=True)
    return circs, np.array(vals)


@pytest.mark.parametrize("dtype", [2, 1])
def test_ladder_batch_every_circuit_vs_oracle(q, ctx, ladder_batch_oracle, dtype):
    """All 256 ladder-batch circuits (12..20 qubits, every width present) in one
    batch launch against the FP64 oracle's final state and observable:
    complex128 to 1e-11, complex64 to 1e-5 per qubit of the observable."""
    circs, ref = ladder_batch_oracle
    assert {c.n for c in circs} == set(range(12, 21))
    got = ctx.batch_run(circs, dtype)
    for b, c in enumerate(circs):
        assert abs(got[b] - ref[b]) <= (1e-11 if dtype == 2 else 1e-5 * c.n), (b, c.n, got[b], ref[b])
    err = np.max(np.abs(got - ref))
    print(f"ladder batch, dtype {dtype}: max |d <sum Z>| = {err:.3e}", flush=True)


def test_batch_rejects_bad_input(q, ctx):
    c = W.random_mix(5, 10, seed=1)
    bad = W.Circuit(5, [W.g1(7, W.H)], np.zeros(0), [((0,), 1.0)])
    with pytest.raises(q.QsvError):
        ctx.batch_run([c, bad], q.QSV_C128)
    big = W.Circuit(25, [W.g1(0, W.H)], np.zeros(0), [((0,), 1.0)])
    with pytest.raises(q.QsvError):
        ctx.batch_run([big], q.QSV_C128)


def test_batch_wait_failure_is_reported(q, ctx, monkeypatch):
    """Failure path, forced from the host: with the dependency-wait bound set
    to zero, every item that has to wait for the previous pass of its circuit
    gives up at once, raises the batch's error flag and the rest of the
    launch drains (no workgroup hangs).  The call reports the error; the next
    normal call on the same context is correct."""
    circs = mixed_batch(3) * 4
    monkeypatch.setenv("QSV_BATCH_SPIN_LIMIT", "0")
    with pytest.raises(q.QsvError, match="spin limit"):
        ctx.batch_run(circs, q.QSV_C128)
    monkeypatch.delenv("QSV_BATCH_SPIN_LIMIT")
    got = ctx.batch_run(circs, q.QSV_C128)
    ref = oracle_values(circs)
    for b, c in enumerate(circs):
        assert abs(got[b] - ref[b]) <= tol(c, 2), b


def test_tune_cache_file_reloads_in_a_fresh_context(q, tmp_path, monkeypatch):
    """QSV_TUNE_CACHE: a tuned choice written by one context is read back by
    a fresh one, which then does not tune again (no new line in the file).
    The stored line is rewritten to 2^13-amplitude tiles, the complex64
    default shape, to check that the reader accepts the largest tile."""
    import json
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("QSV_TUNE_CACHE", str(path))
    circs = mixed_batch(4)
    ref = oracle_values(circs)
    c1 = q.Context()
    got = c1.batch_run(circs, q.QSV_C64, flags=q.FLAG_TUNE)
    c1.close()
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert rec["dtype"] == q.QSV_C64
    rec["tile_bits"], rec["low_bits"] = 13, 4
    path.write_text(json.dumps(rec) + "\n")
    c2 = q.Context()
    got2 = c2.batch_run(circs, q.QSV_C64, flags=q.FLAG_TUNE)
    c2.close()
    assert len(path.read_text().splitlines()) == 1   # loaded, not tuned again
    for b, c in enumerate(circs):
        assert abs(got[b] - ref[b]) <= tol(c, 1) and abs(got2[b] - ref[b]) <= tol(c, 1), b
