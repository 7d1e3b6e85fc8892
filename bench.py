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
FP32_PEAK_TFLOPS = 157.3          # published vector FP32 (two packed FMAs per lane per cycle)
FP32_NONPACKED_TFLOPS = 78.6      # 256 CUs x 4 SIMDs x 16 lanes x 1 FMA x 2.4 GHz
FP64_PEAK_TFLOPS = 78.6
BF16_DENSE_PEAK_TFLOPS = 2500.0   # dense BF16 matrix cores
FP64_MFMA_PEAK_TFLOPS = 78.6
HA_TO_EV = 27.211386
# HBM bytes per launch of k_xy<float, 48, 1, 1024> (32 transforms) from rocprofv3 FETCH_SIZE /
# WRITE_SIZE, each scaled by its reading on a plain 256 MiB copy (factors 2.00 and 1.00);
# valid for the kernel and launch as they stand (profiles/k_xy_c2_hbm_traffic.md)
XY48_F32_TRAFFIC_BYTES = 2.00 * 29431 * 1024 + 1.00 * 55296 * 1024
# HBM bytes of one whole C2 FP32 step (ace_build_apply over 32 vectors, seven kernels), from
# the same counters and scaling (profiles/ace_c2_step_hbm_traffic.md)
C2_F32_STEP_TRAFFIC_BYTES = 423.4e6


def xy_pass_flops(n):
    """Algorithmic FLOPs of the XY pass per pair: per plane 2(N+P) length-P complex transforms
    at 5 P log2 P each (standard FFT count) plus the real kernel multiply (2 per element)."""
    p = 2 * n
    per_plane = 2 * (n + p) * 5.0 * p * math.log2(p) + 2.0 * p * p
    return p * per_plane


def xy_pass_bytes(n, elem):
    """Algorithmic HBM bytes of the XY pass per pair: read and write N*N*P complex values."""
    return 2.0 * n * n * 2 * n * elem


def pair_solve_model_bytes(n, s_work, s_orb):
    """Minimum-pass HBM model of one pair solve: the N*N*P = 2 N^3 intermediate is written by
    the z-forward pass, read and written by the XY pass and read by the z-inverse pass, i.e.
    8 N^3 working elements, plus 3 N^3 orbital / potential elements (two orbitals in, one
    potential out)."""
    return 8.0 * n ** 3 * s_work + 3.0 * n ** 3 * s_orb


def measure_copy_gbs(reps=10):
    """Device-to-device copy bandwidth (256 MiB, read + write bytes) on this GPU."""
    import torch
    src = torch.empty(64 * 2 ** 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return 2.0 * src.numel() * 4 / (ms * 1e-3) / 1e9


def run_gpu(mol, dtype, steps, warmup, trace, graph=True):
    import torch
    import paper_2405_01522_amd as ace
    import synth

    single = dtype == torch.complex64
    dev = torch.device("cuda", 0)
    phi = torch.from_numpy(synth.to_precision(mol.phi, single)).to(dev)
    psi = torch.from_numpy(synth.to_precision(mol.psi, single)).to(dev)
    ace.AceContext(mol.n, mol.h, dtype, dev).close()  # first use: module load, allocator
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    ctx = ace.AceContext(mol.n, mol.h, dtype, dev)  # includes the kernel spectrum setup (a1)
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t_setup)
    n = phi.shape[0]
    xi = torch.empty_like(phi)
    mm = torch.empty((n, n), dtype=torch.complex128, device=dev)
    ex = torch.empty((), dtype=torch.float64, device=dev)
    kpsi = torch.empty_like(psi)

    def step():
        # ACE build + K psi in one call (xi^H psi as L^{-1} W^H psi: its Gram and reduction
        # share launches with the reduction of M and the Cholesky step)
        ctx.ace_build_apply(phi, psi, xi, mm, ex, kpsi)

    def split_step():
        ctx.ace_build(phi, xi, mm, ex)
        ctx.ace_apply(xi, psi, kpsi)

    split_step()
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
    graph_ms = split_graph_ms = None
    if graph:
        # the K timed steps captured into one HIP graph (no per-kernel or per-step launch
        # cost); the first, untimed replay must reproduce the eager results bit for bit
        ref = (xi.clone(), ex.clone(), kpsi.clone())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(steps):
                step()
        g.replay()
        torch.cuda.synchronize()
        same = torch.equal(ref[0], xi) and torch.equal(ref[1], ex) and torch.equal(ref[2], kpsi)
        if not same:
            raise RuntimeError("graph replay differs from the eager step")
        # two more untimed replays: the GPU idles while the graph is captured and instantiated,
        # and the replay right after that runs a few per cent slow
        for _ in range(2):
            g.replay()
        ev[0].record(stream)
        g.replay()
        ev[1].record(stream)
        torch.cuda.synchronize()
        graph_ms = ev[0].elapsed_time(ev[1]) / steps
        total_ms = graph_ms * steps
        del g
        # the same K steps as two calls each (ace_build, then ace_apply)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(steps):
                split_step()
        for _ in range(3):
            g.replay()
        ev[0].record(stream)
        g.replay()
        ev[1].record(stream)
        torch.cuda.synchronize()
        split_graph_ms = ev[0].elapsed_time(ev[1]) / steps
        del g
    # apply alone, for the K psi rate
    ev[0].record(stream)
    for _ in range(steps):
        ctx.ace_apply(xi, psi, kpsi)
    ev[2].record(stream)
    torch.cuda.synchronize()
    apply_ms = ev[0].elapsed_time(ev[2]) / steps
    res = dict(ms_per_step=total_ms / steps, eager_ms_per_step=eager_ms, graph_ms_per_step=graph_ms,
               split_graph_ms_per_step=split_graph_ms,
               setup_ms=setup_ms,
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
    tuning = b.tuning()
    ex = [float(x["ex"].cpu()) for x in systems]
    b.close()
    npairs = sum(m.phi.shape[0] * (m.phi.shape[0] + 1) // 2 for m in mols)
    return dict(ms_per_build=graph_ms, eager_ms_per_build=eager_ms, pair_solves=npairs,
                pair_solves_per_s=npairs / (graph_ms * 1e-3), systems=len(mols), tuning=tuning,
                ex=ex)


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
    nov, noo, nvv = no * nv, no * (no + 1) // 2, nv * (nv + 1) // 2
    ng = mol.n ** 3
    t = (nov + 127) // 128
    # entries of the two contractions: the method's (the upper triangle of the symmetric ov
    # block, and oo pairs x vv pairs a <= b) and the launched 128 x 128 tiles
    method_entries = nov * (nov + 1) // 2 + noo * nvv
    launched_entries = (t * (t + 1) // 2 + ((noo + 127) // 128) * ((nvv + 127) // 128)) * 128 * 128
    gemm_ms = kt.get("tda_gemm", (float("nan"), 1))[0]
    sec = gemm_ms * 1e-3
    # each FP32 product is three BF16 products on the matrix cores (hi*hi + hi*lo + lo*hi)
    method_mfma = 3 * 2.0 * ng * method_entries
    launched_mfma = 3 * 2.0 * ng * launched_entries
    return dict(ms_per_block=ms, pair_solves=nov + noo,
                pair_solves_per_s=(nov + noo) / (ms * 1e-3),
                gemm_ms=gemm_ms,
                gemm={"bound": "mfma", "dtype": "bf16x3 (FP32 operands split hi + lo)",
                      "peak_tflops": BF16_DENSE_PEAK_TFLOPS,
                      "method_fp32_gflop": 2.0 * ng * method_entries / 1e9,
                      "method_bf16_tflops": method_mfma / sec / 1e12,
                      "frac_method": method_mfma / sec / 1e12 / BF16_DENSE_PEAK_TFLOPS,
                      "launched_bf16_tflops": launched_mfma / sec / 1e12,
                      "frac_launched": launched_mfma / sec / 1e12 / BF16_DENSE_PEAK_TFLOPS},
                kernel_ms={k: v[0] for k, v in kt.items()}, c_block=c.cpu().numpy())


def _golden_json(name):
    """Values the oracle wrote (tests/golden/, by scripts that call only the oracle)."""
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def _golden_npy(name):
    path = os.path.join(ROOT, "tests", "golden", name)
    return np.load(path, allow_pickle=False) if os.path.exists(path) else None


def _scf_start(s, k, seed):
    """Seeded random starting vectors (Gaussian envelope), orthonormalised in FP64."""
    import synth
    rng = np.random.default_rng(seed)
    x = synth.coords(s.n, s.h)
    r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
    raw = rng.normal(size=(k, s.n, s.n, s.n)) * np.exp(-0.08 * r2)
    return synth.mgs(raw, s.h ** 3)


def run_scf(train_seeds=(1051, 1052, 1053, 1054, 1055), eval_seed=105, pairs=10000,
            train_steps=2000, batch=8, lr=2e-3, oracle_check=True):
    """C5: closed-shell HF SCF (64^3, h 0.2, 16 doubly occupied orbitals, ACE rebuilt every
    iteration, states mixing 0.3, 3 LOBPCG steps per iteration) with the plain kinetic
    preconditioner and with the learned network beside it, after training the network on
    (residual, correction) pairs recorded from plain runs on other seeded systems."""
    import torch
    import paper_2405_01522_amd as ace
    import synth

    dev = torch.device("cuda", 0)
    dt = torch.float32
    k = 16
    ctx = ace.AceContext(64, 0.2, dt, dev)
    tensor = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)
    eig_kin = ace.eig_opts(max_steps=3, tol=1e-4)
    scf_kw = dict(alpha=0.3, tol=1e-6, max_iter=300)

    def core(s, seed):
        phi = tensor(_scf_start(s, k, seed))
        ctx.fock_lowest_states(tensor(s.v_ext[None]), phi, opts=ace.eig_opts(max_steps=300, tol=1e-3))
        return phi

    # 1. training pairs from plain runs
    per = pairs // len(train_seeds)
    rin = torch.empty((per * len(train_seeds), 64, 64, 64), dtype=dt, device=dev)
    rtg = torch.empty_like(rin)
    count, runs = 0, []
    t0 = time.perf_counter()
    for seed in train_seeds:
        s = synth.config5(seed)
        phi = core(s, seed)
        r = ctx.scf_run(tensor(s.v_ext[None]), phi, ace.scf_opts(eig=eig_kin, **scf_kw),
                        record=(rin[count:count + per], rtg[count:count + per]), record_stride=4)
        ctx.precond_targets(phi, rtg[count:count + r["rec_count"]], r["rec_count"])
        count += r["rec_count"]
        runs.append(dict(seed=seed, iterations=r["iterations"], converged=r["converged"],
                         recorded=r["rec_count"]))
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    # 2. training (random minibatches with sign flips)
    rng = np.random.default_rng(7)
    init = np.concatenate([np.concatenate([rng.normal(scale=0.3 / np.sqrt(27 * ci), size=co * ci * 27),
                                           np.zeros(co)]) for ci, co in ((1, 8), (8, 8), (8, 1))])
    net = ace.ConvNet(init.astype(np.float32), dev)
    t0 = time.perf_counter()
    hist = net.train(rin[:count].contiguous() if count < rin.shape[0] else rin,
                     rtg[:count].contiguous() if count < rtg.shape[0] else rtg,
                     steps=train_steps, batch=batch, lr=lr, seed=11)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    y = net.forward(rin[:64].contiguous())
    fit = float(((y - rtg[:64]) ** 2).sum() / (rtg[:64] ** 2).sum())
    del rin, rtg
    # 3. held-out system: SCF with each preconditioner from the same start
    s = synth.config5(eval_seed)
    v = tensor(s.v_ext[None])
    start = core(s, eval_seed)
    out = {}
    finals = {}
    for name, eo in (("kinetic", eig_kin),
                     ("learned", ace.eig_opts(max_steps=3, tol=1e-4, precond="net", net=net))):
        phi = start.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.scf_run(v, phi, ace.scf_opts(eig=eo, **scf_kw))
        torch.cuda.synchronize()
        out[name] = dict(seconds=time.perf_counter() - t0, iterations=r["iterations"],
                         eig_steps=r["eig_steps"], converged=r["converged"],
                         energy=r["total"], terms={t: r[t] for t in ace.ENERGY_TERMS[1:]},
                         density_error=r["density_error"],
                         eigenvalues=[float(x) for x in r["eigenvalues"]])
        finals[name] = phi
    # 4. eigensolver alone on the converged Hamiltonian (non-self-consistent run): steps from
    # the core guess to residuals below 1e-4 with each preconditioner
    phi_c = finals["kinetic"]
    vloc = v + ctx.hartree_potential(ctx.scf_density(phi_c))
    xi, _, _ = ctx.ace_build(phi_c)
    eig_only = {}
    for name, eo in (("kinetic", ace.eig_opts(max_steps=500, tol=1e-4)),
                     ("learned", ace.eig_opts(max_steps=500, tol=1e-4, precond="net", net=net))):
        phi = start.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, rn, st = ctx.fock_lowest_states(vloc, phi, xi=xi, opts=eo)
        torch.cuda.synchronize()
        eig_only[name] = dict(steps=st, seconds=time.perf_counter() - t0, max_residual=float(rn.max()))
    # 5. excited states on top: unoccupied orbitals (ACE over occupied + unoccupied), the
    # singlet TDA and full TDHF blocks, Davidson, oscillator strengths and the spectrum
    pipe = {}
    nvirt, nbuf = 16, 4  # 16 unoccupied orbitals kept, 4 buffer states above them
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    psi_all = tensor(_scf_start(s, nvirt + nbuf, eval_seed + 7))
    ev_u, rn_u, outer_u, steps_u = ctx.unocc_states(vloc, phi_c, psi_all,
                                                    opts=ace.eig_opts(max_steps=10, tol=1e-4),
                                                    max_outer=80, nconv=nvirt)
    torch.cuda.synchronize()
    psi = psi_all[:nvirt].contiguous()
    ev_u = ev_u[:nvirt]
    pipe["unoccupied"] = dict(states=nvirt, buffer_states=nbuf, seconds=time.perf_counter() - t0,
                              outer=outer_u, steps=steps_u, max_residual=float(rn_u[:nvirt].max()),
                              lowest=float(ev_u[0]), highest=float(ev_u[-1]))
    eps_occ = np.asarray(out["kinetic"].get("eigenvalues", []), dtype=np.float64)
    t0 = time.perf_counter()
    c_s, b_s = ctx.tdhf_coupling(phi_c, psi, 2)
    torch.cuda.synchronize()
    pipe["coupling_seconds"] = time.perf_counter() - t0
    de = (ev_u[None, :] - eps_occ[:, None]).reshape(-1)
    t0 = time.perf_counter()
    om_t, x_t, it_t = ctx.tda_excitations_diag(c_s, de, 8, tol=1e-7)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    om_r, xpy_r, it_r = ctx.tdhf_excitations(c_s, b_s, de, 8, tol=1e-7)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    f_t, _ = ctx.tda_oscillator_strengths(phi_c, psi, x_t, om_t)
    f_r, _ = ctx.tda_oscillator_strengths(phi_c, psi, xpy_r, om_r)
    torch.cuda.synchronize()
    pipe.update(tda=dict(omega_ha=om_t.cpu().tolist(), f=f_t.cpu().tolist(), iterations=it_t,
                         seconds=t1 - t0),
                full_tdhf=dict(omega_ha=om_r.cpu().tolist(), f=f_r.cpu().tolist(), iterations=it_r,
                               seconds=t2 - t1),
                transitions=int(de.size))
    res = dict(workload="C5: 64^3 box h=0.2 bohr, 16 doubly occupied orbitals, 8 soft nuclei "
                        "(seed %d); ACE rebuilt each SCF iteration; states mixing 0.3; "
                        "stop at density error 1e-6 and residuals 1e-4" % eval_seed,
               dtype="f32 grid (FP64 Gram / Rayleigh-Ritz / Cholesky)",
               training=dict(systems=runs, pairs=count, collect_s=t_collect, steps=train_steps,
                             batch=batch, lr=lr, seconds=t_train, loss_first=float(hist[:10].mean()),
                             loss_last=float(hist[-50:].mean()), rel_mse_first64=fit),
               scf=out, eig_only_converged_hamiltonian=eig_only, excited_states=pipe,
               energy_diff_learned_vs_kinetic=abs(out["learned"]["energy"] - out["kinetic"]["energy"]))
    if oracle_check:
        # where the FP32 SCF's energy differs from the FP64 oracle's, term by term: the same
        # (FP32) orbitals evaluated by the FP32 GPU path, by the GPU path in FP64 storage, by the
        # oracle, and by the oracle after an FP64 Loewdin re-orthonormalisation
        from oracle import poisson, scf as oscf
        phi32 = finals["kinetic"]
        p = phi32.cpu().numpy().astype(np.float64)
        khat = poisson.kernel_hat(s.n, s.h)
        t0 = time.perf_counter()
        eo = oscf.energies(p, s.v_ext, s.h, khat)
        t_oracle = time.perf_counter() - t0
        eo_orth = oscf.energies(oscf.loewdin(p, s.h), s.v_ext, s.h, khat)
        e32 = ctx.scf_energies(tensor(s.v_ext[None]), phi32)
        ctx64 = ace.AceContext(64, 0.2, torch.float64, dev)
        e64 = ctx64.scf_energies(torch.from_numpy(np.ascontiguousarray(s.v_ext[None])).to(dev),
                                 phi32.to(torch.float64).contiguous())
        ctx64.close()
        terms = ("kinetic", "external", "hartree", "exchange", "total")
        res["oracle_energy_of_gpu_orbitals"] = dict(
            total=eo["total"], abs_diff=abs(eo["total"] - out["kinetic"]["energy"]),
            seconds=t_oracle,
            gpu_fp32_minus_oracle={t: e32[t] - eo[t] for t in terms},
            gpu_fp64_minus_oracle={t: e64[t] - eo[t] for t in terms},
            orthonormalised_minus_oracle={t: eo_orth[t] - eo[t] for t in terms})
    net.close()
    ctx.close()
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _done(what, t0):
    """One progress line per finished block on stderr (stdout carries only the JSON line)."""
    print("[bench] %s done after %.1f s" % (what, time.perf_counter() - t0), file=sys.stderr,
          flush=True)


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
    # the rate in the GPU's unit (unique pairs per build, build + apply time), and the oracle's
    # own Poisson-solve rate (it solves all n^2 ordered pairs of a build)
    return dict(value=npairs * reps / (t_build + t_apply), reps=reps, ex=ex, kpsi=kp,
                kpsi_per_s=mol.psi.shape[0] * reps / t_apply, seconds=t_build + t_apply,
                oracle_solves_per_s=n * n * reps / t_build)


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
    ap.add_argument("--no-scf", action="store_true")
    ap.add_argument("--no-scf-oracle", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with one plain 256 MiB device-to-device copy (hardware-counter "
                         "calibration under rocprofv3 --pmc)")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import torch
    import synth

    mol = synth.config2()
    n = mol.phi.shape[0]
    npairs = n * (n + 1) // 2
    nvec = mol.psi.shape[0]
    t_start = time.perf_counter()
    mixed = run_gpu(mol, torch.complex64, a.steps, a.warmup, not a.no_trace, not a.no_graph)
    _done("C2 FP32 storage", t_start)
    fp64 = run_gpu(mol, torch.complex128, a.steps, a.warmup, not a.no_trace, not a.no_graph)
    _done("C2 FP64 storage", t_start)

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
        "timing": "one HIP graph of the K steps: three untimed replays (the first checked bit for bit "
                  "against the eager steps), then one timed replay" if mixed["graph_ms_per_step"] else "eager",
        "step": "ace_build_apply (one call: ACE build + K psi, 7 launches after the pair solves "
                "instead of 9)",
        "two_call_ms_per_step": mixed["split_graph_ms_per_step"],
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
        "fp64": {"path": "plain FP64 GPU path: the same kernels with FP64 storage and arithmetic, "
                         "one launch sequence per build",
                 "pair_solves_per_s": npairs / (fp64["ms_per_step"] * 1e-3),
                 "kpsi_per_s": nvec / (fp64["apply_ms"] * 1e-3),
                 "ms_per_step": fp64["ms_per_step"],
                 "eager_ms_per_step": fp64["eager_ms_per_step"],
                 "two_call_ms_per_step": fp64["split_graph_ms_per_step"]},
    }
    out["speedup_vs_fp64"] = out["value"] / out["fp64"]["pair_solves_per_s"]
    # context creation with the sampled Coulomb kernel spectrum (once per geometry; not in a step)
    out["kernel_setup_ms"] = {"mixed": mixed["setup_ms"], "fp64": fp64["setup_ms"]}

    # roofline of the dominant kernel class (the XY pass of the pair Poisson solves)
    kt = mixed["kernels"]
    if kt:
        xy_ms, xy_cnt = kt.get("poisson_xy", (0.0, 0))
        launches = xy_cnt
        avg_ms = xy_ms / max(1, launches)
        # one launch covers every transform of a build: the n(n-1)/2 off-diagonal pair
        # densities, and the n real diagonal densities two per complex transform
        norb = int(mol.phi.shape[0])
        per_launch = norb * (norb - 1) // 2 + (norb + 1) // 2
        flops = xy_pass_flops(mol.n) * per_launch
        achieved = flops / (avg_ms * 1e-3) / 1e12
        tb = XY48_F32_TRAFFIC_BYTES
        out["roofline"] = {"bound": "alu", "kernel": "k_xy<float,48,1,1024>", "achieved": achieved,
                           "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": achieved / FP32_PEAK_TFLOPS, "traffic": tb,
                           "traffic_unit": "bytes per launch (HBM, rocprofv3 counters)",
                           "traffic_gbs": tb / (avg_ms * 1e-3) / 1e9 if tb else None,
                           "transforms_per_launch": per_launch,
                           "avg_launch_ms": avg_ms,
                           "flops_convention": "5 P log2 P per length-P transform + 2 per kernel multiply",
                           "nonpacked_fp32_peak": FP32_NONPACKED_TFLOPS,
                           "frac_nonpacked": achieved / FP32_NONPACKED_TFLOPS,
                           "hbm_model_gbs": xy_pass_bytes(mol.n, 8) * per_launch / (avg_ms * 1e-3) / 1e9}
        out["kernel_ms_per_step"] = {k: v[0] / a.steps for k, v in kt.items()}
    # whole pair-solve path: HBM bytes of the step from the counters over the step time, and
    # the minimum-pass model per pair solve (context beside the kernel roofline)
    copy_gbs = measure_copy_gbs()
    step_gbs = C2_F32_STEP_TRAFFIC_BYTES / (mixed["ms_per_step"] * 1e-3) / 1e9
    out["path_hbm"] = {"counter_bytes_per_step": C2_F32_STEP_TRAFFIC_BYTES,
                       "counter_gbs": step_gbs, "frac_hbm_peak": step_gbs / HBM_PEAK_GBS,
                       "frac_copy": step_gbs / copy_gbs, "copy_gbs": copy_gbs,
                       "model": "8 N^3 s_w + 3 N^3 s_o bytes per pair solve (minimum passes)"}
    for key, sw, val in (("mixed", 8, out["value"]), ("fp64", 16, out["fp64"]["pair_solves_per_s"])):
        b = pair_solve_model_bytes(mol.n, sw, sw)
        gbs = b * val / 1e9
        out["path_hbm"][key + "_model"] = {"bytes_per_pair": b, "achieved_gbs": gbs,
                                           "frac_hbm_peak": gbs / HBM_PEAK_GBS}
    out["fp64"]["kernel_ms_per_step"] = {k: v[0] / a.steps for k, v in fp64["kernels"].items()}

    if not a.no_batched:
        c4 = synth.config4()
        bt = run_batched(c4, torch.complex64, min(a.steps, 10), 2)
        _done("C4 batch FP32", t_start)
        ex_gpu = bt.pop("ex")
        golden = _golden_json("c4_ace.json")
        if golden is not None:
            err = [abs(e - g["ex"]) for e, g in zip(ex_gpu, golden["systems"])]
            bt["ex_error_ha_vs_oracle"] = {"max": max(err), "mean": sum(err) / len(err),
                                           "systems_above_1e-6": sum(e > 1e-6 for e in err)}
        out["batched_uneven"] = {"workload": "64 systems, edges {32..64} step 8, h=0.25, 2-16 complex "
                                             "orbitals (seed 104), one graph-captured call",
                                 "dtype": "f32", **bt}
        # the same batch with FP64 storage (the plain FP64 path of the batch)
        bt64 = run_batched(c4, torch.complex128, min(a.steps, 10), 2)
        _done("C4 batch FP64", t_start)
        ex64 = bt64.pop("ex")
        if golden is not None:
            rel = [abs(e - g["ex"]) / abs(g["ex"]) for e, g in zip(ex64, golden["systems"])]
            bt64["ex_rel_error_vs_oracle_max"] = max(rel)
        out["batched_uneven_fp64"] = {"workload": "the same 64 systems, FP64 storage", **bt64,
                                      "speedup_f32_vs_f64": bt["pair_solves_per_s"] /
                                                            bt64["pair_solves_per_s"]}

    if not a.no_tda:
        c3 = synth.config3()
        td = run_tda(c3, min(a.steps, 10), 2)
        _done("C3 TDA block", t_start)
        cblk = td.pop("c_block")
        golden = _golden_json("c3_eigen.json")
        gold_c = _golden_npy("c3_coupling_singlet.npy")
        if golden is not None and gold_c is not None:
            w = np.linalg.eigvalsh(np.diag(np.repeat(-c3.eps_occ, c3.phi_virt.shape[0])
                                           + np.tile(c3.eps_virt, c3.phi.shape[0])) + cblk)
            td["vs_oracle"] = {"c_max_rel_error": float(np.max(np.abs(cblk - gold_c)) /
                                                       np.max(np.abs(gold_c))),
                               "eigenvalue_max_error_ev":
                                   float(np.max(np.abs(w - np.asarray(golden["eigenvalues_ha"])))) * HA_TO_EV}
        out["tda_block"] = {"workload": "64^3 box h=0.2 padded 128^3; 16 occupied + 32 virtual real "
                                        "orbitals (seed 103); 512 ov + 136 oo pair solves, 512x512 "
                                        "singlet coupling block; one graph-captured call",
                            "dtype": "f32 (FP64 split-K sums)", **td}

    if not a.no_scf:
        out["scf_learned_preconditioner"] = run_scf(oracle_check=not a.no_scf_oracle)
        _done("C5 SCF", t_start)

    if not a.no_cpu_baseline:
        cb = cpu_baseline(mol)
        _done("oracle on the host", t_start)
        out["cpu_baseline"] = {"value": cb["value"], "unit": "pair solves/s",
                               "cores": os.cpu_count(), "cpu_model": _cpu_model(), "kind": "oracle",
                               "sample": "%d full FP64 ACE builds + applies of the same workload "
                                         "(%.1f s)" % (cb["reps"], cb["seconds"]),
                               "kpsi_per_s": cb["kpsi_per_s"],
                               "oracle_own_solves_per_s": cb["oracle_solves_per_s"],
                               "note": "value counts the 36 unique pairs of a build; the oracle "
                                       "solves all 64 ordered pairs (oracle_own_solves_per_s)"}
        out["ex_error_ha"] = {"mixed": abs(mixed["ex"] - cb["ex"]), "fp64": abs(fp64["ex"] - cb["ex"])}
        ref = cb["kpsi"]
        scale = float(np.max(np.abs(ref)))
        out["kpsi_rel_error"] = {"mixed": float(np.max(np.abs(mixed["kpsi"] - ref)) / scale),
                                 "fp64": float(np.max(np.abs(fp64["kpsi"] - ref)) / scale)}
    if a.calibrate_copy:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = 2 * src.numel() * 4
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
