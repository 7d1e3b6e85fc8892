"""Benchmark of the ACE exchange hot path on one MI355X.

A step is one pass of the whole path over the workload: ACE build (all unique pair Poisson
solves, W, M, Cholesky, xi, E_x) followed by ACE application to the test vectors.  The
headline runs with FP32 storage (FP64 kernel spectrum, Gram sums, Cholesky and E_x); the
same step with FP64 storage is timed beside it.

Workload (default): 48^3 box, h = 0.25 bohr, padded 96^3, 8 complex orbitals (36 unique pair
solves), K applied to 32 complex test vectors; seeded synthetic Gaussian orbitals.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair Poisson solves/s and ACE K*psi/s, mixed vs FP64 GPU at 1e-6 Ha"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def xy_pass_flops(n):
    """Algorithmic FLOPs of the XY pass per pair: per plane 2(N+P) length-P complex transforms
    at 5 P log2 P each (standard FFT count) plus the real kernel multiply (2 per element)."""
    p = 2 * n
    per_plane = 2 * (n + p) * 5.0 * p * math.log2(p) + 2.0 * p * p
    return p * per_plane


def xy_pass_bytes(n, elem):
    """Algorithmic HBM bytes of the XY pass per pair: read and write N*N*P complex values."""
    return 2.0 * n * n * 2 * n * elem


def run_gpu(mol, dtype, steps, warmup, trace, graph=True):
    import torch
    import paper_2405_01522_amd as ace
    import synth

    single = dtype == torch.complex64
    dev = torch.device("cuda", 0)
    phi = torch.from_numpy(synth.to_precision(mol.phi, single)).to(dev)
    psi = torch.from_numpy(synth.to_precision(mol.psi, single)).to(dev)
    ctx = ace.AceContext(mol.n, mol.h, dtype, dev)
    n = phi.shape[0]
    xi = torch.empty_like(phi)
    mm = torch.empty((n, n), dtype=torch.complex128, device=dev)
    ex = torch.empty((), dtype=torch.float64, device=dev)
    kpsi = torch.empty_like(psi)

    def step():
        ctx.ace_build(phi, xi, mm, ex)
        ctx.ace_apply(xi, psi, kpsi)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    st, info = ctx.status()
    if st != 0:
        raise RuntimeError("device status %d (info %d)" % (st, info))
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    if trace:
        ctx.trace_reset()
        ctx.trace(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for _ in range(steps):
        step()
    ev[1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if trace:
        ctx.trace(False)
        kt = ctx.trace_read()
    else:
        kt = {}
    total_ms = ev[0].elapsed_time(ev[1])
    eager_ms = total_ms / steps
    graph_ms = None
    if graph:
        # the same step captured once into a HIP graph and replayed (no per-kernel launch cost);
        # replays must reproduce the eager results bit for bit
        ref = (xi.clone(), ex.clone(), kpsi.clone())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        g.replay()
        torch.cuda.synchronize()
        same = torch.equal(ref[0], xi) and torch.equal(ref[1], ex) and torch.equal(ref[2], kpsi)
        if not same:
            raise RuntimeError("graph replay differs from the eager step")
        ev[0].record(stream)
        for _ in range(steps):
            g.replay()
        ev[1].record(stream)
        torch.cuda.synchronize()
        graph_ms = ev[0].elapsed_time(ev[1]) / steps
        total_ms = graph_ms * steps
        del g
    # apply alone, for the K psi rate
    ev[0].record(stream)
    for _ in range(steps):
        ctx.ace_apply(xi, psi, kpsi)
    ev[2].record(stream)
    torch.cuda.synchronize()
    apply_ms = ev[0].elapsed_time(ev[2]) / steps
    res = dict(ms_per_step=total_ms / steps, eager_ms_per_step=eager_ms, graph_ms_per_step=graph_ms,
               wall_ms_per_step=1e3 * wall / steps,
               apply_ms=apply_ms, ex=float(ex.cpu()), kernels=kt,
               kpsi=kpsi.cpu().numpy(), xi_dtype=str(dtype))
    ctx.close()
    return res


def run_batched(mols, dtype, steps, warmup):
    """Uneven batch (one call builds ACE for every system), graph-captured and replayed."""
    import torch
    import paper_2405_01522_amd as ace
    import synth

    single = dtype == torch.complex64
    dev = torch.device("cuda", 0)
    systems = [{"h": m.h, "phi": torch.from_numpy(synth.to_precision(m.phi, single)).to(dev)}
               for m in mols]
    b = ace.AceBatch(dtype, dev)
    for _ in range(max(1, warmup)):
        b.build(systems)
    torch.cuda.synchronize()
    st, mol, info = b.status()
    if st != 0:
        raise RuntimeError("batched build: device status %d (system %d, info %d)" % (st, mol, info))
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        b.build(systems)
    e1.record(stream)
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / steps
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.build(systems)
    g.replay()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / steps
    del g
    b.close()
    npairs = sum(m.phi.shape[0] * (m.phi.shape[0] + 1) // 2 for m in mols)
    return dict(ms_per_build=graph_ms, eager_ms_per_build=eager_ms, pair_solves=npairs,
                pair_solves_per_s=npairs / (graph_ms * 1e-3), systems=len(mols))


def run_tda(mol, steps, warmup):
    """TDA coupling block (real FP32 orbitals): ov + oo pair solves and the MFMA contractions,
    graph-captured and replayed; the contraction time comes from the library's event tracer."""
    import torch
    import paper_2405_01522_amd as ace
    import synth

    dev = torch.device("cuda", 0)
    occ = torch.from_numpy(synth.to_precision(mol.phi, True)).to(dev)
    virt = torch.from_numpy(synth.to_precision(mol.phi_virt, True)).to(dev)
    no, nv = occ.shape[0], virt.shape[0]
    ctx = ace.AceContext(mol.n, mol.h, torch.float32, dev)
    c = torch.empty((no * nv, no * nv), dtype=torch.float64, device=dev)
    for _ in range(max(1, warmup)):
        ctx.tda_coupling(occ, virt, 2, c)
    torch.cuda.synchronize()
    ctx.trace_reset()
    ctx.trace(True)
    ctx.tda_coupling(occ, virt, 2, c)
    ctx.trace(False)
    kt = ctx.trace_read()
    stream = torch.cuda.current_stream(dev)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.tda_coupling(occ, virt, 2, c)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del g
    ctx.close()
    nov, noo = no * nv, no * (no + 1) // 2
    t = (nov + 127) // 128
    # contraction FLOPs as launched: upper 128-tiles of the symmetric ov block + the oo x vv block
    flops = 2.0 * mol.n ** 3 * (t * (t + 1) // 2 * 128 * 128 + noo * nv * nv)
    gemm_ms = kt.get("tda_gemm", (float("nan"), 1))[0]
    return dict(ms_per_block=ms, pair_solves=nov + noo,
                pair_solves_per_s=(nov + noo) / (ms * 1e-3),
                gemm_ms=gemm_ms, gemm_tflops=flops / (gemm_ms * 1e-3) / 1e12,
                gemm_frac_fp32_mfma=flops / (gemm_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
                kernel_ms={k: v[0] for k, v in kt.items()})


def cpu_baseline(mol, budget_s=20.0):
    """The FP64 oracle, timed on the host cores on a bounded sample of the same workload:
    whole ACE builds (36 pair solves each) plus applications to the 32 vectors, repeated
    until about budget_s seconds have passed."""
    from oracle import exchange, poisson

    khat = poisson.kernel_hat(mol.n, mol.h)
    reps, t_build = 0, 0.0
    t_apply = 0.0
    t_end = time.perf_counter() + budget_s
    xi = ex = kp = None
    while reps < 1 or time.perf_counter() < t_end:
        t0 = time.perf_counter()
        xi, _, _, ex = exchange.ace_build(mol.phi, mol.h, khat)
        t1 = time.perf_counter()
        kp = exchange.ace_apply(xi, mol.psi, mol.h)
        t2 = time.perf_counter()
        t_build += t1 - t0
        t_apply += t2 - t1
        reps += 1
        if reps >= 20:
            break
    n = mol.phi.shape[0]
    npairs = n * (n + 1) // 2
    return dict(value=npairs * reps / (t_build + t_apply), reps=reps, ex=ex, kpsi=kp,
                kpsi_per_s=mol.psi.shape[0] * reps / t_apply, seconds=t_build + t_apply)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-trace", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-tda", action="store_true")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        return 2

    import torch
    import synth

    mol = synth.config2()
    n = mol.phi.shape[0]
    npairs = n * (n + 1) // 2
    nvec = mol.psi.shape[0]
    mixed = run_gpu(mol, torch.complex64, a.steps, a.warmup, not a.no_trace, not a.no_graph)
    fp64 = run_gpu(mol, torch.complex128, a.steps, a.warmup, not a.no_trace, not a.no_graph)

    value = npairs / (mixed["ms_per_step"] * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "eager_ms_per_step": mixed["eager_ms_per_step"],
        "timing": "HIP-graph replay of the captured step" if mixed["graph_ms_per_step"] else "eager",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "48^3 box h=0.25 bohr padded to 96^3; 8 complex orbitals "
                               "(36 unique pair Poisson solves) ACE build + K psi on 32 vectors",
                   "grid": 48, "padded": 96, "orbitals": n, "pair_solves_per_step": npairs,
                   "vectors": nvec, "seed": 102},
        "kpsi_per_s": nvec / (mixed["apply_ms"] * 1e-3),
        "fp64": {"pair_solves_per_s": npairs / (fp64["ms_per_step"] * 1e-3),
                 "kpsi_per_s": nvec / (fp64["apply_ms"] * 1e-3),
                 "ms_per_step": fp64["ms_per_step"],
                 "eager_ms_per_step": fp64["eager_ms_per_step"]},
    }
    out["speedup_vs_fp64"] = out["value"] / out["fp64"]["pair_solves_per_s"]

    # roofline of the dominant kernel class (the XY pass of the pair Poisson solves)
    kt = mixed["kernels"]
    if kt:
        xy_ms, xy_cnt = kt.get("poisson_xy", (0.0, 0))
        launches = xy_cnt
        avg_ms = xy_ms / max(1, launches)
        pairs_per_launch = npairs  # one launch covers every pair of a build
        flops = xy_pass_flops(mol.n) * pairs_per_launch
        achieved = flops / (avg_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "alu", "kernel": "k_xy<float,48>", "achieved": achieved,
                           "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                           "avg_launch_ms": avg_ms,
                           "hbm_model_gbs": xy_pass_bytes(mol.n, 8) * pairs_per_launch / (avg_ms * 1e-3) / 1e9}
        out["kernel_ms_per_step"] = {k: v[0] / a.steps for k, v in kt.items()}
        out["fp64"]["kernel_ms_per_step"] = {k: v[0] / a.steps for k, v in fp64["kernels"].items()}

    if not a.no_batched:
        bt = run_batched(synth.config4(), torch.complex64, min(a.steps, 10), 2)
        out["batched_uneven"] = {"workload": "64 systems, edges {32..64} step 8, h=0.25, 2-16 complex "
                                             "orbitals (seed 104), one graph-captured call",
                                 "dtype": "f32", **bt}

    if not a.no_tda:
        td = run_tda(synth.config3(), min(a.steps, 10), 2)
        out["tda_block"] = {"workload": "64^3 box h=0.2 padded 128^3; 16 occupied + 32 virtual real "
                                        "orbitals (seed 103); 512 ov + 136 oo pair solves, 512x512 "
                                        "singlet coupling block; one graph-captured call",
                            "dtype": "f32 (FP64 split-K sums)", **td}

    if not a.no_cpu_baseline:
        cb = cpu_baseline(mol)
        out["cpu_baseline"] = {"value": cb["value"], "unit": "pair solves/s",
                               "cores": os.cpu_count(), "kind": "oracle",
                               "sample": "%d full FP64 ACE builds + applies of the same workload "
                                         "(%.1f s)" % (cb["reps"], cb["seconds"]),
                               "kpsi_per_s": cb["kpsi_per_s"]}
        out["ex_error_ha"] = {"mixed": abs(mixed["ex"] - cb["ex"]), "fp64": abs(fp64["ex"] - cb["ex"])}
        ref = cb["kpsi"]
        scale = float(np.max(np.abs(ref)))
        out["kpsi_rel_error"] = {"mixed": float(np.max(np.abs(mixed["kpsi"] - ref)) / scale),
                                 "fp64": float(np.max(np.abs(fp64["kpsi"] - ref)) / scale)}
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
