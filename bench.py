"""Benchmark: gate throughput of the HIP state-vector engine on one MI355X.

Primary workload (the `value`): a 30-qubit complex128 layered circuit --
20 layers, each a Haar-random 1-qubit gate on every qubit followed by CNOTs
on the even then the odd nearest-neighbour pairs (1180 gates), seeded and
synthetic.  One step = init |0...0> + the whole circuit (fused tile passes)
+ norm + <Z_0 Z_29>.  value = gates / second over the timed steps.

Also reported (same JSON line):
  roofline      the dominant kernel (fused tile pass) from HIP events on the
                library's stream over the timed steps: algorithmic flops
                (FP64 for complex128) and bytes per launch over the average
                launch time, against MI355X peaks; `bound` is the resource
                whose time at peak is longer; `traffic` from the committed
                HBM counter summary while the kernel sources match it
  cpu_baseline  the FP64 CPU oracle on the same 30-qubit circuit, first gates
                only (time-bounded sample), on all of this host's cores
  extras        the pass kernels used (specialised per pass structure, with
                their compile time, unless --no-jit or no device compiler);
                complex64 throughput of the same circuit; the 1000-gate
                random mix at 30 qubits and random Haar pairs at 32 qubits
                (64 GiB / 32 GiB) in both precisions, with the flops the fused
                kernels execute; unfused per-gate kernel bandwidth (c128 and
                c64 at 30 qubits, c128 at 32); adjoint-gradient / forward time
                ratio on a 24-qubit ansatz (10 layers RY,RZ + CZ ring, 480
                parameters) in both precisions; the structured one-pass
                kernels (diagonal and permutation gates) with their bytes;
                gates with extra controls and k-qubit gates (one pass each);
                QFT and Trotter at 30 qubits with the specialised kernels; a 256-circuit batch (12..20
                qubits) in one persistent launch; QFT and a Trotter TFXY chain
                from 16 to 32 qubits; the CPU oracle on one thread and the
                host CPU model
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}   # MI355X dense vector FP64 / FP32
METRIC = "gates/s + HBM GB/s (% peak) at 30 qubits; adjoint-grad time / forward time"


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_circuit(q, c, dtype: int, steps: int, warmup: int, jit: bool = False, obs=None):
    """Time `steps` runs of circuit c from |0...0> (after `warmup` untimed
    runs, which also plan and, with jit, compile the pass kernels); each step
    ends with the norm and the observable's Z strings in one reduction."""
    import torch
    n = c.n
    g = q.marshal_gates(c.gates)
    ctx = q.Context()
    if jit:
        ctx.set_jit(1)
    st = q.State(ctx, n, dtype)
    # the norm is the Z string over no qubits: one reduction pass gives
    # both it and the observable's terms
    obs = [((), 1.0)] + list(c.observable if obs is None else obs)

    def step():
        # |0...0>, then the circuit: the first tile pass makes |0...0> itself
        st.apply_circuit(None, c.params, marshalled=g, flags=q.FLAG_FROM_ZERO)
        return st.expect_z(obs)

    t0 = time.perf_counter()
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    ctx.profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        terms, _ = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_end()
    norm = st.norm2()
    jk, js = ctx.jit_stats()
    st.free()
    del st
    ctx.close()
    torch.cuda.empty_cache()
    flops = sum(gate_flops_per_amp(x) for x in c.gates) * float(2 ** n)
    exec_flops = executed_flops_per_amp(q, c, dtype) * float(2 ** n)
    _, pas = q.plan_fused(n, c.gates, c.params, dtype)
    return {"gates": len(c.gates), "seconds": t1 - t0, "prof": prof, "norm": norm,
            "norm_in_step": float(terms[0]), "terms": [float(x) for x in terms[1:]],
            "flops_per_step": min(flops, exec_flops), "gate_by_gate_flops_per_step": flops,
            "warmup_s": t_warm, "jit_kernels": jk, "jit_compile_s": js,
            "passes": int(pas.max()) + 1 if len(pas) else 0}


def primary(q, W, n: int, dtype: int, steps: int, warmup: int, layers: int = 20, seed: int = 3002,
            jit: bool = False):
    c = W.layered_cnot_brick(n, layers, seed)
    r = run_circuit(q, c, dtype, steps, warmup, jit)
    r["zz"] = r["terms"][0]
    return r


def circuit_extra(q, c, dtype: int, steps: int, warmup: int, jit: bool, label: str):
    """gates/s and the tile-pass roofline of one circuit (an `extras` entry)."""
    c64 = dtype == q.QSV_C64
    r = run_circuit(q, c, dtype, steps, warmup, jit)
    out = {"workload": label, "gates": r["gates"], "passes": r["passes"],
           "gates_per_s": round(r["gates"] * steps / r["seconds"], 2),
           "ms_per_circuit": round(r["seconds"] / steps * 1e3, 3),
           "norm": r["norm"], "jit": jit}
    if jit:
        out["jit_kernels"] = r["jit_kernels"]
        out["jit_compile_s"] = round(r["jit_compile_s"], 2)
    roof = kernel_roofline(r["prof"], "tile_pass_c64" if c64 else "tile_pass_c128", steps,
                           r["flops_per_step"], "f32" if c64 else "f64")
    if roof is not None:
        # flops the fused kernels execute; gate by gate (Algs. 1-3) the same
        # circuit would take this many per launch
        roof["gate_by_gate_flops_per_launch"] = r["gate_by_gate_flops_per_step"] * steps / roof["launches"]
        out["roofline"] = roof
    return out


def gate_flops_per_amp(gate) -> float:
    """Algorithmic real flops per amplitude of one gate, as Algs. 1-3 apply
    it: a dense 2x2 costs 2 complex multiplies + 1 complex add per output
    (14 per amplitude), a controlled 2x2 touches half the amplitudes (7), a
    dense 4x4 costs 4 multiplies + 3 adds per output (30); a diagonal 2x2
    is one complex multiply per amplitude (6, half that when controlled);
    permutation matrices (X, CNOT, SWAP) move data and do no arithmetic."""
    import numpy as np
    if gate.kind == "rot":
        return 6.0 if str(gate.axis).lower() == "z" else 14.0
    m = np.asarray(gate.matrix)
    if np.all((m == 0) | (m == 1)) and np.all(m.sum(axis=0) == 1):
        return 0.0
    diag = np.count_nonzero(m - np.diag(np.diag(m))) == 0
    if gate.kind == "1q":
        return 6.0 if diag else 14.0
    if gate.kind == "c1q":
        return 3.0 if diag else 7.0
    return 6.0 if diag else 30.0


def executed_flops_per_amp(q, c, dtype: int) -> float:
    """Real flops per amplitude that the tile kernels execute for circuit c:
    the fused gate sequence (1-qubit products folded into neighbouring
    2-qubit gates where that adds no arithmetic), each gate at the cost of
    the register body that runs it: dense 2x2 14, real 2x2 (RY) 6, diagonal
    6, controlled dense 7, controlled diagonal 3, dense 4x4 30 (also a
    controlled gate on control state 0), permutations 0."""
    import numpy as np
    recs, _ = q.plan_fused(c.n, c.gates, c.params, dtype)
    tot = 0.0
    for r in recs:
        m = r["m"][0::2] + 1j * r["m"][1::2]
        d = 4 if r["kind"] == q.qsv.G2Q or (r["kind"] == q.qsv.GC1Q and r["ctrl_state"] == 0) else 2
        u = m[: d * d].reshape(d, d)
        perm = np.all((u == 0) | (u == 1)) and np.all(u.sum(axis=0) == 1)
        diag = np.count_nonzero(u - np.diag(np.diag(u))) == 0
        if perm:
            continue
        if r["kind"] == q.qsv.G1Q:
            tot += 6.0 if (diag or np.all(u.imag == 0)) else 14.0
        elif d == 2:
            tot += 3.0 if diag else 7.0
        elif r["kind"] == q.qsv.GC1Q:
            tot += 30.0
        else:
            tot += 6.0 if diag else 30.0
    return tot


def kernel_roofline(prof: dict, name: str, steps: int, flops_per_step: float, dtype: str):
    """Roofline of the dominant kernel from its average launch duration:
    algorithmic bytes (one read + one write of the state) and algorithmic
    flops (the circuit's gates, spread over the step's launches) per launch.
    `bound` is whichever takes longer at its peak; the other is reported
    alongside."""
    k = prof.get(name)
    if not k or k["launches"] == 0 or k["ms"] <= 0:
        return None
    per_launch_bytes = k["bytes"] / k["launches"]
    per_launch_flops = flops_per_step / (k["launches"] / steps)
    avg_s = k["ms"] / k["launches"] / 1e3
    gbs = per_launch_bytes / avg_s / 1e9
    tfl = per_launch_flops / avg_s / 1e12
    peak_tf = PEAK_TFLOPS[dtype]
    hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(gbs / PEAK_HBM_GBS, 4)}
    alu = {"bound": "alu", "achieved": round(tfl, 2), "peak": peak_tf, "unit": "TFLOP/s",
           "frac": round(tfl / peak_tf, 4)}
    alu_time = per_launch_flops / (peak_tf * 1e12)
    hbm_time = per_launch_bytes / (PEAK_HBM_GBS * 1e9)
    main, other = (alu, hbm) if alu_time >= hbm_time else (hbm, alu)
    out = dict(main)
    out.update({"traffic": None, "kernel": name, "launches": k["launches"],
                "avg_ms": round(k["ms"] / k["launches"], 4), "bytes_per_launch": per_launch_bytes,
                "flops_per_launch": per_launch_flops,
                "time_at_peak_ms": {"alu": round(alu_time * 1e3, 3), "hbm": round(hbm_time * 1e3, 3)},
                "other": other})
    return out


def measured_traffic(n: int, jit: bool = False):
    """HBM bytes per tile-pass launch from the committed FETCH_SIZE/WRITE_SIZE
    summary, if it was measured on the current kernel sources and workload."""
    path = os.path.join(ROOT, "profiles", f"traffic_tile_pass_c128_n{n}{'_jit' if jit else ''}.json")
    if not os.path.exists(path):
        return None
    from paper_2303_00123_amd import profsum
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != profsum.source_hash():
        return None
    return rec.get("traffic_bytes_per_launch")


def structured_sweep(q, W, n: int):
    """One-pass kernels of structured gates at n qubits (c128): diagonal gates
    touch only the amplitudes they change (Z, S, T, P: half the state when the
    qubit's index bit is at or above the 128-byte line; CZ and CP a quarter),
    permutation gates (X, CNOT, SWAP) only move data.  Bandwidth against the
    bytes each kernel must move."""
    import numpy as np
    import torch
    Z = np.diag([1.0, -1.0]).astype(complex)
    T = np.diag([1.0, np.exp(0.25j * np.pi)])
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    SW = np.eye(4, dtype=complex)[[0, 2, 1, 3]]
    cases = {"diag_z_T": [W.g1(qb, Z if qb % 2 else T) for qb in range(0, n - 3, 3)],
             "diag_cz": [W.gc(qb, qb + 2, Z) for qb in range(0, n - 6, 4)],
             "perm_x": [W.g1(qb, X) for qb in range(0, n, 4)],
             "perm_cnot": [W.cnot(qb, qb + 1) for qb in range(0, n - 4, 4)],
             "perm_swap": [W.g2(qb, n - 1 - qb, SW) for qb in range(0, n // 2 - 1, 3)]}
    ctx = q.Context()
    st = q.State(ctx, n, q.QSV_C128)
    st.init_basis(0)
    out = {}
    for name, gl in cases.items():
        g = q.marshal_gates(gl)
        st.apply_circuit(None, marshalled=g, flags=q.FLAG_NO_FUSE)
        torch.cuda.synchronize()
        ctx.profile_begin()
        st.apply_circuit(None, marshalled=g, flags=q.FLAG_NO_FUSE)
        prof = ctx.profile_end()
        for k, v in prof.items():
            out[f"{name}:{k}"] = {"launches": v["launches"], "avg_ms": round(v["ms"] / v["launches"], 4),
                                  "bytes_per_launch": v["bytes"] / v["launches"],
                                  "GB/s": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1)}
    st.free()
    del st
    ctx.close()
    torch.cuda.empty_cache()
    return out


def general_gate_sweep(q, W, n: int):
    """One-pass kernels of the general gates at n qubits: gates with extra
    controls (c128; each control halves the amplitudes moved; Toffoli only
    swaps) and dense gates on k = 3, 4, 5 qubits (8 * 2^k flops per
    amplitude) on the matrix cores and on the vector units, both
    precisions.  Bandwidth against the bytes each kernel must move; for the
    k-qubit kernels also their flop rate."""
    import numpy as np
    import torch
    rng = np.random.default_rng(3007)
    ctx = q.Context()
    st = q.State(ctx, n, q.QSV_C128)
    st.init_basis(0)
    out = {}
    mc = {"toffoli": [W.toffoli(0, n - 1, 5), W.toffoli(3, 7, n - 2), W.toffoli(n - 5, 1, 9)],
          "mc3_haar": [W.with_controls(W.g1(4, W.haar_unitary(2, rng)), (0, 10, n - 3)),
                       W.with_controls(W.g1(n - 6, W.haar_unitary(2, rng)), (2, 12, 20), (1, 0, 1))],
          "mc1_haar2q": [W.with_controls(W.g2(6, n - 8, W.haar_unitary(4, rng)), (1,))]}
    for name, gl in mc.items():
        g = q.marshal_gates(gl)
        st.apply_circuit(None, marshalled=g, flags=q.FLAG_NO_FUSE)
        torch.cuda.synchronize()
        ctx.profile_begin()
        st.apply_circuit(None, marshalled=g, flags=q.FLAG_NO_FUSE)
        prof = ctx.profile_end()
        for kname, v in prof.items():
            out[f"{name}:{kname}"] = {"launches": v["launches"], "avg_ms": round(v["ms"] / v["launches"], 4),
                                      "bytes_per_launch": v["bytes"] / v["launches"],
                                      "GB/s": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1)}
    st.free()
    del st
    ctx.close()
    torch.cuda.empty_cache()
    # dense k-qubit gates: matrix cores (FP64 MFMA for complex128, FP32 for
    # complex64; mode 2, so also k = 4, which the default leaves on the
    # vector units) against the vector-unit kernel, same qubits and matrix
    for k in (3, 4, 5):
        qs = [int(x) for x in rng.choice(n, size=k, replace=False)]
        u = W.haar_unitary(2 ** k, rng)
        for dtype, tag in ((q.QSV_C128, "c128"), (q.QSV_C64, "c64")):
            for mode, kname in ((2, "kq_mfma"), (0, "kq")):
                ctx = q.Context()
                ctx.set_matrix_cores(mode)
                st = q.State(ctx, n, dtype)
                st.init_basis(0)
                st.applyKq(qs, u)
                torch.cuda.synchronize()
                ctx.profile_begin()
                for _ in range(2):
                    st.applyKq(qs, u)
                prof = ctx.profile_end()
                v = prof[f"{kname}_{tag}"]
                sec = v["ms"] / v["launches"] / 1e3
                label = f"kq{k}_{tag}" + ("_matrix_cores" if mode else "_vector")
                out[label] = {"qubits": qs, "avg_ms": round(sec * 1e3, 4),
                              "GB/s": round(v["bytes"] / v["launches"] / sec / 1e9, 1),
                              ("TFLOP/s (FP64)" if tag == "c128" else "TFLOP/s (FP32)"):
                                  round(8 * 2 ** k * 2 ** n / sec / 1e12, 2)}
                st.free()
                del st
                ctx.close()
                torch.cuda.empty_cache()
    return out


def jit_usable(q) -> bool:
    """True if this host has the device compiler the specialised pass kernels need."""
    ctx = q.Context()
    try:
        ctx.set_jit(1)
        return True
    except q.QsvError:
        return False
    finally:
        ctx.close()


def size_sweep(q, W, sizes=(16, 20, 24, 28, 30, 32)):
    """Time per circuit against the qubit count for the paper's two benchmark
    circuits (QFT and a Trotter TFXY chain, 5 steps), both precisions; the
    interpreting tile kernel (no compile step per size)."""
    out = {}
    for name, make in (("qft", lambda n: W.qft(n)), ("trotter_tfxy_5", lambda n: W.trotter_tfxy(n, 5, 4000 + n))):
        rows = []
        for n in sizes:
            c = make(n)
            for dt, tag in ((q.QSV_C128, "c128"), (q.QSV_C64, "c64")):
                r = run_circuit(q, c, dt, 2, 1, False, obs=[])
                rows.append({"n": n, "dtype": tag, "gates": r["gates"], "passes": r["passes"],
                             "ms": round(r["seconds"] / 2 * 1e3, 3),
                             "gates_per_s": round(r["gates"] * 2 / r["seconds"], 1)})
            log(f"sweep {name} n={n}")
        out[name] = rows
    return out


def unfused_sweep(q, W, n: int, every: int = 1, dtype=None):
    """Average bandwidth of the one-pass-per-gate kernels (Algs. 1-3).

    A controlled gate moves half the state (2^n * 16 bytes, its algorithmic
    bytes) when its control is an index bit at or above 3; below that the
    amplitudes it skips share 128-byte lines with the ones it moves, so HBM
    carries the whole state.  The sweep keeps controls at bits >= 3 and times
    the low-control case on its own, reported against both byte counts.
    every = k uses every k-th qubit position (a shorter sweep)."""
    import numpy as np
    import torch
    rng = np.random.default_rng(3003)
    gates = []
    for qb in range(0, n, every):
        gates.append(W.g1(qb, W.haar_unitary(2, rng)))
    for qb in range(0, n - 4, 3 * every):      # control qubit qb: index bit n-1-qb >= 3
        gates.append(W.gc(qb, qb + 1, W.haar_unitary(2, rng)))
    for qb in range(0, n - 1, 3 * every):
        gates.append(W.g2(qb, n - 1 - qb if n - 1 - qb != qb else qb + 1, W.haar_unitary(4, rng)))
    low = [W.gc(n - 1, 0, W.haar_unitary(2, rng)) for _ in range(4 if every == 1 else 2)]   # control at index bit 0
    ctx = q.Context()
    st = q.State(ctx, n, q.QSV_C128 if dtype is None else dtype)
    st.init_basis(0)
    out = {}
    for gl, tag in ((gates, ""), (low, "_ctrl_bit0")):
        g = q.marshal_gates(gl)
        st.apply_circuit(None, marshalled=g, flags=q.FLAG_NO_FUSE)
        torch.cuda.synchronize()
        ctx.profile_begin()
        st.apply_circuit(None, marshalled=g, flags=q.FLAG_NO_FUSE)
        prof = ctx.profile_end()
        for k, v in prof.items():
            out[k + tag] = {"launches": v["launches"], "avg_ms": round(v["ms"] / v["launches"], 4),
                            "GB/s": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1)}
            if tag:
                out[k + tag]["GB/s_hbm"] = round(2 * v["bytes"] / (v["ms"] / 1e3) / 1e9, 1)
    st.free()
    del st
    ctx.close()
    torch.cuda.empty_cache()
    return out


def adjoint_ratio(q, W, n: int = 24, layers: int = 10, dtype=None, reps: int = 3):
    import torch
    dtype = q.QSV_C128 if dtype is None else dtype
    c = W.hea_cz_ring(n, layers, seed=1005)
    g = q.marshal_gates(c.gates)
    ctx = q.Context()
    psi, lam = q.State(ctx, n, dtype), q.State(ctx, n, dtype)

    def forward():
        psi.init_basis(0)
        psi.apply_circuit(None, c.params, marshalled=g)
        return psi.expect_z(c.observable)[1]

    def backward():
        return q.adjoint(psi, lam, None, c.params, c.observable, flags=0, marshalled=g)

    forward()
    backward()
    tf, tb = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        forward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tf.append(t1 - t0)
        tb.append(t2 - t1)
    psi.free()
    lam.free()
    ctx.close()
    tf, tb = min(tf), min(tb)
    return {"workload": f"hea_cz_ring n={n} layers={layers} params={len(c.params)}",
            "forward_ms": round(tf * 1e3, 3), "adjoint_ms": round(tb * 1e3, 3),
            "adjoint_over_forward": round(tb / tf, 3)}


def batch_bench(q, W, dtype, reps: int = 5):
    """256 parametrised circuits (12..20 qubits, 6 layers RY RZ + CNOT ladder)
    in two persistent launches of 128 circuits (the second staged on the host
    while the first runs): wall time per call (host planning included) and
    the GPU time of the replayed hipGraphs."""
    import torch
    import numpy as np
    circs = W.ladder_batch_256()
    spec = q.BatchSpec(circs)
    ctx = q.Context()
    ctx.batch_run(spec, dtype, flags=q.FLAG_TUNE)
    ctx.batch_run(spec, dtype, flags=q.FLAG_CAPTURE_GRAPH)
    rng = np.random.default_rng(4999)
    angle_sets = [rng.uniform(0, 2 * np.pi, size=spec.params.size) for _ in range(reps)]
    torch.cuda.synchronize()
    ctx.profile_begin()
    t0 = time.perf_counter()
    for a in angle_sets:   # new angles every call, same circuit structure
        ctx.batch_run(spec, dtype, flags=q.FLAG_CAPTURE_GRAPH, params=a)
    t1 = time.perf_counter()
    prof = ctx.profile_end()
    ctx.close()
    name = "batch_graph_c128" if dtype == q.QSV_C128 else "batch_graph_c64"
    k = prof.get(name, {"launches": 1, "ms": float("nan")})
    gpu_ms = k["ms"] / reps   # one or two launches per call
    wall_ms = (t1 - t0) / reps * 1e3
    return {"workload": "256 circuits, 12..20 qubits, 6 layers RY RZ + CNOT ladder, <sum Z_i>",
            "circuits": len(circs), "wall_ms_per_batch": round(wall_ms, 3),
            "graph_ms_per_batch": round(gpu_ms, 3),
            "circuits_per_s_wall": round(len(circs) / (wall_ms / 1e3), 1),
            "circuits_per_s_gpu": round(len(circs) / (gpu_ms / 1e3), 1)}


def host_cpu():
    """CPU model, physical cores and hardware threads of this host (lscpu)."""
    import subprocess
    info = {"model": None, "physical_cores": None, "threads": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        info["model"] = kv.get("Model name")
        cps, sockets = kv.get("Core(s) per socket"), kv.get("Socket(s)")
        if cps and sockets:
            info["physical_cores"] = int(cps) * int(sockets)
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    try:   # the kernel's own description (lscpu may print only the family)
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["model_cpuinfo"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        info["threads_available"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    return info


def cpu_baseline(W, n: int, budget_s: float = 15.0, threads: int = 0):
    import numpy as np
    import oracle as O
    if threads:
        O.set_num_threads(threads)
    c = W.layered_cnot_brick(n, 20, 3002)
    s = np.zeros(2 ** n, dtype=np.complex128)
    s[0] = 1.0
    work = np.zeros_like(s)
    L = O.lib()
    gates = O.marshal(c)
    p = np.zeros(1)
    done = 0
    t_total = 0.0
    ptr = lambda a: a.ctypes.data_as(O.ctypes.c_void_p)  # noqa: E731
    # warm the pages of both buffers with one untimed gate
    L.orc_run(n, ptr(s), ptr(work), 1, ptr(gates[0:1]), ptr(p))
    k = 1
    while t_total < budget_s and k < len(gates):
        t0 = time.perf_counter()
        L.orc_run(n, ptr(s), ptr(work), 1, ptr(gates[k:k + 1]), ptr(p))
        t_total += time.perf_counter() - t0
        done += 1
        k += 1
        log(f"cpu oracle gate {k}/{len(gates)}: {t_total:.1f} s")
    used = O.num_threads()
    return {"value": round(done / t_total, 4), "unit": "gates/s", "cores": used,
            "kind": "oracle",
            "sample": f"gates 2..{k} of the same {n}-qubit 1180-gate circuit, FP64 oracle "
                      f"(out-of-place Kronecker-definition loops, OpenMP, {used} threads), "
                      f"{t_total:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-jit", action="store_true",
                    help="run the fused passes with the interpreting tile kernel only")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--dtype", choices=["c128", "c64"], default="c128",
                    help="precision of the primary workload (profiling aid; the reported "
                         "metric is defined on complex128)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a device copy of 2^k complex128 amplitudes (counter calibration)")
    ap.add_argument("--general-only", action="store_true",
                    help="only run the sweep of multi-controlled and dense k-qubit gates (matrix cores "
                         "and vector units) at 30 qubits and print it (profiling aid)")
    ap.add_argument("--unfused-only", action="store_true",
                    help="only run the one-kernel-per-gate sweeps (30 qubits in both precisions, "
                         "32 qubits complex128) and print their bandwidths (profiling aid)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the path runs on one MI355X per process; --gpus must be 1 "
                                   "(the multi-GPU layout is a design, not a measured path)"}))
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device"}))
        sys.exit(1)
    import paper_2303_00123_amd as q
    import workloads as W

    if args.copy_probe:
        a = torch.empty(2 ** args.copy_probe, dtype=torch.complex128, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 16, "copies": 3}))
        return

    if args.general_only:
        print(json.dumps({"general_gates": general_gate_sweep(q, W, 30)}), flush=True)
        return

    if args.unfused_only:
        out = {"unfused_c128": unfused_sweep(q, W, 30),
               "unfused_c64": unfused_sweep(q, W, 30, dtype=q.QSV_C64),
               "unfused_c128_n32": unfused_sweep(q, W, 32, every=4)}
        print(json.dumps(out), flush=True)
        return

    jit = not args.no_jit and jit_usable(q)
    log(f"primary: n={args.n} {args.dtype} steps={args.steps} warmup={args.warmup} jit={jit}")
    c64 = args.dtype == "c64"
    r = primary(q, W, args.n, q.QSV_C64 if c64 else q.QSV_C128, args.steps, args.warmup, jit=jit)
    value = r["gates"] * args.steps / r["seconds"]
    roof = kernel_roofline(r["prof"], "tile_pass_c64" if c64 else "tile_pass_c128", args.steps,
                           r["flops_per_step"], "f32" if c64 else "f64")
    if roof is not None:
        roof["traffic"] = None if c64 else measured_traffic(args.n, jit)
    log(f"primary: {value:.1f} gates/s, roofline {roof}")
    extras = {"norm_after": r["norm"], "zz_0_last": r["zz"], "passes": r["passes"],
              "pass_kernels": "specialised per pass structure" if jit else "interpreting",
              "kernels_c128": {k: {"launches": v["launches"], "avg_ms": round(v["ms"] / v["launches"], 4)}
                               for k, v in r["prof"].items()}}
    if jit:
        extras["jit"] = {"kernels": r["jit_kernels"], "compile_s": round(r["jit_compile_s"], 2),
                         "warmup_s": round(r["warmup_s"], 2)}
    if not args.no_extras:
        log("extras: complex64")
        s64 = max(2, args.steps // 2)
        r64 = primary(q, W, args.n, q.QSV_C64, s64, 1, jit=jit)
        extras["c64"] = {"gates_per_s": round(r64["gates"] * s64 / r64["seconds"], 2),
                         "passes": r64["passes"],
                         "roofline": kernel_roofline(r64["prof"], "tile_pass_c64", s64,
                                                     r64["flops_per_step"], "f32")}
        log("extras: 1000-gate random mix at 30 qubits")
        mix = W.random_mix(30, 1000, 3001, "random_mix")
        extras["random_mix_n30"] = {
            "c128": circuit_extra(q, mix, q.QSV_C128, 3, 1, jit, "50/25/25 Haar 1q / controlled Haar / "
                                  "Haar 2q, 1000 gates, 30 qubits, complex128, seed 3001"),
            "c64": circuit_extra(q, mix, q.QSV_C64, 3, 1, jit, "the same circuit, complex64")}
        log("extras: random Haar pairs at 32 qubits")
        hp = W.layered_haar_pairs(32, 10, 1003)
        extras["haar_pairs_n32"] = {
            "c128": circuit_extra(q, hp, q.QSV_C128, 2, 1, jit, "10 layers of Haar 1q on every qubit + "
                                  "Haar 2q on a random matching, 32 qubits (64 GiB), complex128, seed 1003"),
            "c64": circuit_extra(q, hp, q.QSV_C64, 2, 1, jit, "the same circuit, complex64 (32 GiB)")}
        log("extras: unfused sweep")
        extras["unfused_c128"] = unfused_sweep(q, W, args.n)
        extras["unfused_c64"] = unfused_sweep(q, W, args.n, dtype=q.QSV_C64)
        log("extras: structured one-pass kernels")
        extras["structured_c128"] = structured_sweep(q, W, args.n)
        log("extras: multi-controlled and k-qubit gates")
        extras["general_gates_c128"] = general_gate_sweep(q, W, args.n)
        if jit:
            log("extras: QFT and Trotter at 30 qubits, specialised kernels")
            extras["paper_circuits_specialised"] = {
                "qft": circuit_extra(q, W.qft(args.n), q.QSV_C128, 2, 1, True,
                                     f"QFT (Fig. 1), {args.n} qubits, complex128"),
                "trotter_tfxy_5": circuit_extra(q, W.trotter_tfxy(args.n, 5, 4000 + args.n), q.QSV_C128, 2,
                                                1, True, f"Trotter TFXY chain, 5 steps, {args.n} qubits, "
                                                         "complex128")}
        if args.n == 30:
            log("extras: unfused sweep at 32 qubits")
            extras["unfused_c128_n32"] = unfused_sweep(q, W, 32, every=4)
        log("extras: adjoint ratio")
        extras["adjoint"] = adjoint_ratio(q, W)
        extras["adjoint_c64"] = adjoint_ratio(q, W, dtype=q.QSV_C64)
        log("extras: batch")
        extras["batch_c128"] = batch_bench(q, W, q.QSV_C128)
        extras["batch_c64"] = batch_bench(q, W, q.QSV_C64)
        if not args.no_sweep:
            log("extras: QFT and Trotter time vs qubits")
            extras["sweep"] = size_sweep(q, W)
    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(W, args.n)
        extras["host_cpu"] = host_cpu()
        log("cpu baseline, one thread")
        extras["cpu_1thread"] = cpu_baseline(W, args.n, budget_s=10.0, threads=1)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["seconds"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if c64 else "f64",
        "data": "synthetic",
        "config": {"workload": f"layered CNOT-brick circuit, {args.n} qubits, 20 layers "
                               f"({r['gates']} gates: Haar 1q on every qubit + CNOT even/odd "
                               f"pairs), {'complex64' if c64 else 'complex128'}, seed 3002; step = init + circuit + norm "
                               f"+ <Z0 Z{args.n - 1}>",
                   "n_qubits": args.n, "gates": r["gates"], "state_bytes": 16 * 2 ** args.n},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
